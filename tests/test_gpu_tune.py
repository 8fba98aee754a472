"""Tile autotuner: a tuning call times candidate tiles on its own data, caches
the fastest per shape class, and changes no result (every tile computes the
canonical FP64 bins, so toplists are bit-identical whatever the tile)."""
import numpy as np
import pytest

import oracle
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _key(top):
    return [(t.index, t.s64, t.s32) for t in top]


def _eval(c, w, tile, stats=None):
    c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges, tile=tile, stats=stats)
    return [c.toplist(j, w.k) for j in range(len(w.sub_edges) - 1)]


def test_tuned_plain_call_is_exact_and_cached(ft):
    import torch
    w = synth.plain_small(seed=1)
    s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, w.weight,
                                w.v, w.f0, w.f1, w.sky)
    assert bad == -1
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    want = oracle.toplist(s64, oracle.subband(f0t, w.sub_edges), len(w.sub_edges) - 1, w.k)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.load_workload(w)
        tuned = _eval(c, w, ft.FT_TILE_TUNE)
        rep, ms = c.tune_report()
        assert rep and ms > 0
        assert sum(e["chosen"] for e in rep) == 1
        assert all(e["klass"] == 0 and e["evals_per_s"] > 0 for e in rep)
        chosen = next(e for e in rep if e["chosen"])
        assert chosen["evals_per_s"] == max(e["evals_per_s"] for e in rep)
        assert c.info().tile == chosen["tile"]
        # the class is cached: the library choice is now the tuned tile
        again = _eval(c, w, 0)
        assert c.info().tile == chosen["tile"]
        c.tune_clear()
        model = _eval(c, w, 0)
        with pytest.raises(ft.FtError):
            _eval(c, w, -2)
    for tops in (tuned, again, model):
        for got, idx in zip(tops, want):
            assert [t.index for t in got] == list(idx)
            assert all(t.s64 == s64[t.index] for t in got)


def test_tuned_batch_equals_untuned(ft):
    import torch
    cp = synth.campaign(10, seed=45, n_pool=700, n_sft_range=(80, 600), width_range=(0.02, 0.1),
                        nt_range=(2000, 20000), k=5)
    assert any(R["n_f0"] >= 32 for R in cp.runs)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.eval_campaign(cp, tile=0)
        base = [_key(c.batch_toplist(r, cp.k)) for r in range(cp.n_runs)]
        c.eval_campaign(cp, tile=ft.FT_TILE_TUNE, use_graph=1)
        tuned = [_key(c.batch_toplist(r, cp.k)) for r in range(cp.n_runs)]
        rep, ms = c.tune_report()
        c.eval_campaign(cp, tile=0)
        cached = [_key(c.batch_toplist(r, cp.k)) for r in range(cp.n_runs)]
    assert tuned == base and cached == base
    assert rep and ms > 0
    classes = {e["klass"] for e in rep}
    assert all(k >= 1 for k in classes)
    for k in classes:
        rows = [e for e in rep if e["klass"] == k]
        assert sum(e["chosen"] for e in rows) == 1
        best = max(e["evals_per_s"] for e in rows)
        assert next(e for e in rows if e["chosen"])["evals_per_s"] == best


def test_lds_gather_probe(ft):
    """The gather-accumulate probe runs for every tile shape and rejects bad
    arguments on the host."""
    import torch
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        rates = [c.probe_lds_gather(t) for t in range(1, ft.ft_tile_count() + 1)]
        assert all(r > 1e11 for r in rates), rates
        for bad in ((0, 0), (ft.ft_tile_count() + 1, 0), (1, 65), (1, 64)):
            with pytest.raises(ft.FtError):
                c.probe_lds_gather(*bad)
