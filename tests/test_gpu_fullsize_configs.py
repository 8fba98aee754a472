"""The 1 kHz precision-stress band and the 512-run injection campaign at their full
sizes, in the launch configurations the benchmark times, against the oracle's
evaluation of every template:

* 2 detectors x 5000 SFTs, 1000-1000.1 Hz, 180 f0 x 5 f1 x 2e4 sky points
  (1.8e7 templates, 1.8e11 template-SFT pairs; x ~ 1.8e6 bins, where FP32 bins
  flip): every FP32 statistic within the certified blocked-summation bound of
  its FP64 sum, both sub-bands' toplists bit for bit, with the autotuned tile;
  every tile shape on a reduced sky gives the same bits;
* 512 uneven runs (N ~ U{500..5000} SFTs, 1e3-1e5 templates, one injection
  each, K = 10) evaluated in one graph-captured batch with autotuned tiles:
  every run's toplist equals the oracle's on tables the oracle generates itself.

The oracle's sums run on all host threads (a few tens of seconds)."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def rel_bound(n_sft):
    return 40 * 2.0 ** -24 + 4 * n_sft * 2.0 ** -53


def _grid_eval(ft, w, tile, dev):
    import torch
    stats = torch.empty(w.n_templates, dtype=torch.float32, device=dev)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
                   torch.from_numpy(w.power).to(dev))
        c.set_velocities(torch.from_numpy(w.v).to(dev))
        c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges, tile=tile, stats=stats)
        tops = [c.toplist(j, w.k) for j in range(len(w.sub_edges) - 1)]
        info = c.info()
    return stats.cpu().numpy(), tops, info


def _check(w, s32, tops, s64):
    rel = np.abs(s32.astype(np.float64) - s64) / s64
    assert rel.max() <= rel_bound(w.n_sft) and rel.max() < 1e-5, rel.max()
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    want = oracle.toplist(s64, oracle.subband(f0t, w.sub_edges), len(w.sub_edges) - 1, w.k)
    for got, exp in zip(tops, want):
        assert [t.index for t in got] == list(exp)
        assert [t.s64 for t in got] == s64[exp].tolist()


def test_precision_stress_full_size(ft):
    import torch
    dev = torch.device("cuda:0")
    w = synth.precision_stress(seed=2)
    s32, tops, info = _grid_eval(ft, w, ft.FT_TILE_TUNE, dev)
    print("tile", ft.ft_tile_name(info.tile), "eval ms", info.eval_ms, flush=True)
    assert info.tile > 0 and info.n_evals == w.evals
    s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0,
                                w.f1, w.sky)
    assert bad == -1
    _check(w, s32, tops, s64)


def test_precision_stress_every_tile(ft):
    import torch
    dev = torch.device("cuda:0")
    w = synth.precision_stress(seed=2, n_sky=37)
    s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0,
                                w.f1, w.sky)
    assert bad == -1
    ref = None
    for tile in range(1, ft.ft_tile_count() + 1):
        s32, tops, info = _grid_eval(ft, w, tile, dev)
        assert info.tile == tile, ft.ft_tile_name(tile)
        _check(w, s32, tops, s64)
        if ref is None:
            ref = s32
        assert np.array_equal(ref, s32), ft.ft_tile_name(tile)


def _oracle_run(cp, R):
    sl = slice(R["sft_begin"], R["sft_begin"] + R["n_sft"])
    table = inject.generate_table(R["seed"], R["run_id"], cp.t_mid[sl], R["t_ref"], cp.t_sft,
                                  cp.v[sl], cp.arms[sl], R["first_bin"], R["n_bins"], R["inj"])
    f0 = cp.f0[R["f0_begin"]:R["f0_begin"] + R["n_f0"]]
    f1 = cp.f1[R["f1_begin"]:R["f1_begin"] + R["n_f1"]]
    sky = cp.sky[R["sky_begin"]:R["sky_begin"] + R["n_sky"]]
    s64, bad = oracle.eval_grid(cp.t_mid[sl], R["t_ref"], cp.t_sft, R["first_bin"], table, None,
                                cp.v[sl], f0, f1, sky)
    assert bad == -1
    order = np.argsort(-s64, kind="stable")[:cp.k]  # (S desc, index asc)
    return order.tolist(), s64[order].tolist()


def test_campaign_full_size(ft):
    import torch
    cp = synth.campaign(512, seed=4)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_campaign(cp, use_graph=1, tile=ft.FT_TILE_TUNE)
        got = [c.batch_toplist(r, cp.k) for r in range(len(cp.runs))]
    threads = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(threads) as ex:
        want = list(ex.map(lambda R: _oracle_run(cp, R), cp.runs))
    for r, (idx, s64) in enumerate(want):
        assert [t.index for t in got[r]] == idx, r
        assert [t.s64 for t in got[r]] == s64, r
