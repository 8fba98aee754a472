"""The no-allocation entry point (ft_count_index_mismatches_noalloc) against
the entry point it mirrors (ft_count_index_mismatches): equal mismatch and
FP64-fallback counts on two calls in a row through the C ABI, the second
smaller (fewer SFTs and templates) than the first, so stale scratch contents
would show; host-memory banks and SFT counts beyond the scratch are rejected."""
import numpy as np
import pytest

from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _count_both(ft, c, f0, f1, sky, t_ref, mode, kind):
    import torch
    dev = torch.device("cuda:0")
    want = c.count_index_mismatches(f0, f1, sky, t_ref, mode, kind=kind, fallback=True)
    got = c.count_index_mismatches_noalloc(torch.from_numpy(f0).to(dev), torch.from_numpy(f1).to(dev),
                                           torch.from_numpy(sky).to(dev), t_ref, mode, kind=kind)
    return got, want


def test_noalloc_matches_allocating_entry_point(ft):
    import torch
    big = synth.precision_stress(seed=11, n_sky=40, n_per_det=300)
    small = synth.precision_stress(seed=12, n_sky=7, n_per_det=90)
    rng = np.random.default_rng(13)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        for w in (big, small):
            c.load_workload(w)
            n = 257
            lf0 = rng.uniform(w.f0[0], w.f0[-1], n)
            lf1 = rng.uniform(-1e-9, 0.0, n)
            lsky = synth.isotropic_sky(n, rng)
            for mode in (ft.FT_INDEX_FP32, ft.FT_INDEX_DF64, ft.FT_INDEX_GUARDED, ft.FT_INDEX_GUARDED_FP32,
                         ft.FT_INDEX_FP64):
                got, want = _count_both(ft, c, w.f0, w.f1, w.sky, w.t_ref, mode, ft.FT_BANK_GRID)
                assert got == want, (w.name, mode, got, want)
                got, want = _count_both(ft, c, lf0, lf1, lsky, w.t_ref, mode, ft.FT_BANK_LIST)
                assert got == want, (w.name, mode, got, want)
                if mode == ft.FT_INDEX_FP32:
                    assert got[0] > 0  # a count that can differ between the calls


def test_noalloc_rejects_host_memory_and_oversized_sft_sets(ft):
    import torch
    w = synth.precision_stress(seed=14, n_sky=3, n_per_det=40)
    dev = torch.device("cuda:0")
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        with pytest.raises(ft.FtError, match="FT_E_STATE"):
            c.count_index_mismatches_noalloc(torch.from_numpy(w.f0).to(dev), torch.from_numpy(w.f1).to(dev),
                                             torch.from_numpy(w.sky).to(dev), w.t_ref, ft.FT_INDEX_FP32)
        c.load_workload(w)
        with pytest.raises(ft.FtError, match="FT_E_INVALID"):
            c.count_index_mismatches_noalloc(w.f0, w.f1, w.sky, w.t_ref, ft.FT_INDEX_FP32)
        n_big = 131073  # one SFT more than the scratch holds
        t_mid = 1.2e9 + 1800.0 * (np.arange(n_big) + 0.5)
        c.set_sfts([n_big], t_mid, 1800.0, w.first_bin, np.ones((n_big, 4), np.float32))
        c.set_velocities(np.zeros((n_big, 3)))
        with pytest.raises(ft.FtError, match="FT_E_UNSUPPORTED"):
            c.count_index_mismatches_noalloc(torch.from_numpy(w.f0).to(dev), torch.from_numpy(w.f1).to(dev),
                                             torch.from_numpy(w.sky).to(dev), w.t_ref, ft.FT_INDEX_FP32)
