"""Batched form: one persistent (optionally graph-captured) launch over many
uneven runs must give, run by run, exactly the toplists of separate plain
calls, and agree with the oracle evaluating its own generated tables."""
import numpy as np
import pytest

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _small_campaign(seed=41, n_runs=12):
    return synth.campaign(n_runs, seed=seed, n_pool=700, n_sft_range=(80, 600),
                          width_range=(0.005, 0.06), nt_range=(200, 6000), k=5)


def _plain_run(ft, c, cp, r):
    R = cp.runs[r]
    sl = slice(R["sft_begin"], R["sft_begin"] + R["n_sft"])
    c.gen_sfts([R["n_sft"]], cp.t_mid[sl], cp.t_sft, R["first_bin"], R["n_bins"], cp.v[sl],
               cp.arms[sl], R["seed"], R["run_id"], R["t_ref"], R["inj"])
    f0 = cp.f0[R["f0_begin"]:R["f0_begin"] + R["n_f0"]]
    f1 = cp.f1[R["f1_begin"]:R["f1_begin"] + R["n_f1"]]
    sky = cp.sky[R["sky_begin"]:R["sky_begin"] + R["n_sky"]]
    edges = np.array([f0[0] - 1.0, f0[-1] + 1.0])
    c.eval_templates(f0, f1, sky, R["t_ref"], cp.k, edges)
    return c.toplist(0, cp.k), (f0, f1, sky)


def _key(top):
    return [(t.index, t.s64, t.s32) for t in top]


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_equals_plain_calls(ft, use_graph):
    import torch
    cp = _small_campaign()
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_campaign(cp, use_graph=use_graph)
        batched = [c.batch_toplist(r, cp.k) for r in range(len(cp.runs))]
        labels, max_z = c.batch_labels(8.0, len(cp.runs))
        plain = [_plain_run(ft, c, cp, r)[0] for r in range(len(cp.runs))]
    for r in range(len(cp.runs)):
        assert _key(batched[r]) == _key(plain[r]), r
        assert max_z[r] == batched[r][0].z
        assert labels[r] == (batched[r][0].z > 8.0)


def test_batch_graph_replay_is_identical(ft):
    import torch
    cp = _small_campaign(seed=42, n_runs=9)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_campaign(cp, use_graph=1)
        first = [_key(c.batch_toplist(r, cp.k)) for r in range(len(cp.runs))]
        for _ in range(3):
            c.batch_replay()
            again = [_key(c.batch_toplist(r, cp.k)) for r in range(len(cp.runs))]
            assert again == first
        assert c.batch_time() > 0


def test_batch_matches_oracle_on_its_own_tables(ft):
    import torch
    cp = _small_campaign(seed=43, n_runs=6)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_campaign(cp, use_graph=1)
        batched = [c.batch_toplist(r, cp.k) for r in range(len(cp.runs))]
    for r, R in enumerate(cp.runs):
        sl = slice(R["sft_begin"], R["sft_begin"] + R["n_sft"])
        table = inject.generate_table(R["seed"], R["run_id"], cp.t_mid[sl], R["t_ref"], cp.t_sft,
                                      cp.v[sl], cp.arms[sl], R["first_bin"], R["n_bins"],
                                      R["inj"])
        f0 = cp.f0[R["f0_begin"]:R["f0_begin"] + R["n_f0"]]
        f1 = cp.f1[R["f1_begin"]:R["f1_begin"] + R["n_f1"]]
        sky = cp.sky[R["sky_begin"]:R["sky_begin"] + R["n_sky"]]
        s64, bad = oracle.eval_grid(cp.t_mid[sl], R["t_ref"], cp.t_sft, R["first_bin"], table,
                                    None, cp.v[sl], f0, f1, sky)
        assert bad == -1
        order = sorted(range(s64.size), key=lambda t: (-s64[t], t))[:cp.k]
        # tables agree to the last bit except for rare transcendental ulps, so
        # compare values within 1e-9 and the order where the gaps are larger
        for got, want in zip(batched[r], order):
            assert abs(got.s64 - s64[want]) <= 1e-9 * s64[want]
        gaps = np.diff(-np.sort(-s64)[:cp.k + 1])
        if np.all(np.abs(gaps) > 1e-6 * s64.max()):
            assert [t.index for t in batched[r]] == order


def test_batch_given_tables_and_errors(ft):
    """Batches also take caller tables; bad slices are rejected on the host."""
    import torch
    cp = _small_campaign(seed=44, n_runs=4)
    tables, runs = [], []
    off = 0
    for R in cp.runs:
        sl = slice(R["sft_begin"], R["sft_begin"] + R["n_sft"])
        t = inject.generate_table(R["seed"], R["run_id"], cp.t_mid[sl], R["t_ref"], cp.t_sft,
                                  cp.v[sl], cp.arms[sl], R["first_bin"], R["n_bins"], R["inj"])
        tables.append(t.ravel())
        runs.append(dict(R, table_offset=off))
        off += t.size
    power = np.concatenate(tables)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_batch(runs, cp.t_mid, cp.v, cp.t_sft, cp.f0, cp.f1, cp.sky, cp.k, power=power)
        tops = [c.batch_toplist(r, cp.k) for r in range(len(runs))]
        assert all(len(t) == min(cp.k, R["n_f0"] * R["n_f1"] * R["n_sky"])
                   for t, R in zip(tops, runs))
        bad = [dict(runs[0], sft_begin=len(cp.t_mid))]
        with pytest.raises(ft.FtError) as e:
            c.eval_batch(bad, cp.t_mid, cp.v, cp.t_sft, cp.f0, cp.f1, cp.sky, cp.k, power=power)
        assert e.value.status == ft.FT_E_INVALID
        bad = [dict(runs[0], table_offset=power.size)]
        with pytest.raises(ft.FtError) as e:
            c.eval_batch(bad, cp.t_mid, cp.v, cp.t_sft, cp.f0, cp.f1, cp.sky, cp.k, power=power)
        assert e.value.status == ft.FT_E_INVALID
