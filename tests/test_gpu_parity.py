"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bins and toplists must match bit for bit; FP32 statistics must lie within the
certified blocked-summation bound e = 40*2^-24 + 4*N*2^-53 of the FP64 sum
(and so within the 1e-5 relative target).
"""
import numpy as np
import pytest

import oracle
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def rel_bound(n_sft):
    return 40 * 2.0 ** -24 + 4 * n_sft * 2.0 ** -53


def _dev_tensors(w):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(w.t_mid)).to(dev),
            torch.from_numpy(np.ascontiguousarray(w.power)).to(dev),
            torch.from_numpy(np.ascontiguousarray(w.v)).to(dev),
            None if w.weight is None else torch.from_numpy(w.weight).to(dev))


def run_gpu(ft, w, tile=0, sum_mode=0, kind=0, f0=None, f1=None, sky=None, k=None,
            edges=None, host_inputs=False):
    import torch
    f0 = w.f0 if f0 is None else f0
    f1 = w.f1 if f1 is None else f1
    sky = w.sky if sky is None else sky
    k = w.k if k is None else k
    edges = w.sub_edges if edges is None else edges
    n_t = len(f0) * len(f1) * len(sky) if kind == 0 else len(f0)
    stats = torch.empty(n_t, dtype=torch.float32, device="cuda:0")
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        if host_inputs:
            c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power, w.weight)
            c.set_velocities(w.v)
        else:
            tm, p, v, wt = _dev_tensors(w)
            c.set_sfts(w.n_sft_per_det, tm, w.t_sft, w.first_bin, p, wt)
            c.set_velocities(v)
        c.eval_templates(f0, f1, sky, w.t_ref, k, edges, kind=kind, tile=tile,
                         sum_mode=sum_mode, stats=stats)
        tops = [c.toplist(j, k) for j in range(len(edges) - 1)]
        info = c.info()
    return stats.cpu().numpy(), tops, info


def oracle_grid(w):
    s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, w.weight,
                                w.v, w.f0, w.f1, w.sky)
    assert bad == -1
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    sub = oracle.subband(f0t, w.sub_edges)
    tops = oracle.toplist(s64, sub, len(w.sub_edges) - 1, w.k)
    return s64, tops


def assert_stats(s32, s64, n_sft):
    rel = np.abs(s32.astype(np.float64) - s64) / np.maximum(s64, 1e-300)
    assert rel.max() <= rel_bound(n_sft), rel.max()
    assert rel.max() < 1e-5


def assert_toplists(gpu_tops, want_tops, s64, n_sft, weight=None):
    mu, sig = oracle.noise_moments(n_sft, weight)
    for got, want in zip(gpu_tops, want_tops):
        assert [c.index for c in got] == list(want)
        for c in got:
            assert c.s64 == s64[c.index]
            assert abs(c.z - (s64[c.index] - mu) / sig) <= 1e-12 * max(1.0, abs(c.z))


def test_plain_small_bitexact_toplist(ft):
    w = synth.plain_small(seed=1)
    s32, tops, info = run_gpu(ft, w)
    s64, want = oracle_grid(w)
    assert_stats(s32, s64, w.n_sft)
    assert_toplists(tops, want, s64, w.n_sft)
    assert info.n_evals == w.evals


def test_allsky_ragged_tiles_all_tiles_identical(ft):
    """Reduced all-sky band: several tiles per dimension with ragged tails in
    f0 (900), f1 (11) and sky (23); every tile shape gives the same bits."""
    w = synth.allsky_band(seed=3, n_sky=23, n_per_det=300)
    s64, want = oracle_grid(w)
    ref = None
    for tile in range(1, ft.ft_tile_count() + 1):
        s32, tops, info = run_gpu(ft, w, tile=tile)
        assert info.tile == tile
        assert_stats(s32, s64, w.n_sft)
        assert_toplists(tops, want, s64, w.n_sft)
        if ref is None:
            ref = s32
        else:
            assert np.array_equal(ref, s32), ft.ft_tile_name(tile)


@pytest.mark.parametrize("n_f0,n_f1,n_sky,n_per_det", [
    (1, 1, 1, 1),     # one template, two SFTs: a single short stage
    (1, 3, 2, 4),     # eight SFTs: one full K8 stage, half a K16 stage
    (2, 1, 5, 5),     # ten SFTs: a full stage and two SFTs, prepared in one pass
    (7, 2, 3, 12),    # three K8 stages: the second pass prepares one stage
    (65, 4, 1, 20),   # one f0 value past a 64-wide L1 tile
    (321, 5, 4, 17),  # one f0 value past a full L5 tile; 34 SFTs cross a summation block
])
def test_smallest_banks_every_tile(ft, n_f0, n_f1, n_sky, n_per_det):
    """Degenerate and short banks through every tile shape: the statistics
    within the bound and the toplists bit for bit against the oracle, and
    every shape giving the same bits."""
    w = synth.tiny_bank(n_f0, n_f1, n_sky, n_per_det)
    s64, want = oracle_grid(w)
    ref = None
    for tile in range(1, ft.ft_tile_count() + 1):
        s32, tops, info = run_gpu(ft, w, tile=tile)
        assert info.n_evals == w.evals, ft.ft_tile_name(tile)
        assert_stats(s32, s64, w.n_sft)
        assert_toplists(tops, want, s64, w.n_sft)
        if ref is None:
            ref = s32
        else:
            assert np.array_equal(ref, s32), ft.ft_tile_name(tile)


def test_list_bank_parity(ft):
    w = synth.allsky_band(seed=4, n_sky=8, n_per_det=250)
    rng = np.random.default_rng(40)
    n = 3000
    f0 = rng.uniform(w.f0[0], w.f0[-1], n)
    f1 = rng.uniform(w.f1.min(), w.f1.max(), n)
    sky = synth.isotropic_sky(n, rng)
    s32, tops, info = run_gpu(ft, w, kind=1, f0=f0, f1=f1, sky=sky, k=25)
    s64, bad = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v,
                                f0, f1, sky)
    assert bad == -1
    assert_stats(s32, s64, w.n_sft)
    want = oracle.toplist(s64, oracle.subband(f0, w.sub_edges), len(w.sub_edges) - 1, 25)
    assert_toplists(tops, want, s64, w.n_sft)


def test_bins_fp64_bitexact(ft):
    import torch
    w = synth.precision_stress(seed=5, n_sky=4, n_per_det=200)
    rng = np.random.default_rng(50)
    n = 400
    f0 = rng.uniform(w.f0[0], w.f0[-1], n)
    f1 = rng.uniform(-1e-9, 0, n)
    sky = synth.isotropic_sky(n, rng)
    want = oracle.bins_list(w.t_mid, w.t_ref, w.t_sft, w.v, f0, f1, sky)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.load_workload(w)
        got = c.bins(f0, f1, sky, w.t_ref, ft.FT_INDEX_FP64)
        guarded = c.bins(f0, f1, sky, w.t_ref, ft.FT_INDEX_GUARDED)
        guarded32 = c.bins(f0, f1, sky, w.t_ref, ft.FT_INDEX_GUARDED_FP32)
        fp32 = c.bins(f0, f1, sky, w.t_ref, ft.FT_INDEX_FP32)
        df64 = c.bins(f0, f1, sky, w.t_ref, ft.FT_INDEX_DF64)
        counts = {m: c.count_index_mismatches(f0, f1, sky, w.t_ref, m, kind=ft.FT_BANK_LIST, fallback=True)
                  for m in (0, 1, 2, 3, 4)}
    assert np.array_equal(got, want)
    assert np.array_equal(guarded, want)
    assert np.array_equal(guarded32, want)
    assert counts[0] == (0, 0) and counts[3][0] == 0 and counts[4][0] == 0
    assert counts[1][0] == int(np.sum(fp32 != want)) and counts[1][0] > 0 and counts[1][1] == 0
    assert counts[2][0] == int(np.sum(df64 != want)) and counts[2][1] == 0
    # at 1 kHz the df64 margin (4.7e-7 bins) accepts nearly every estimate, the
    # FP32 margin (1.7 bins) none
    assert counts[3][1] <= 1e-4 * want.size
    assert counts[4][1] == want.size
    # FP32 at 1 kHz is off by at most a bin or two; df64 only near half-bins
    assert np.abs(fp32 - want).max() <= 2
    assert np.abs(df64 - want).max() <= 1


def test_guard_fallback_on_half_bin_grid(ft):
    """f0 grid centred on half-bins with a near-zero Doppler: every run's first
    template sits within rounding of a bin edge, so the guarded runs fall back
    to FP64 for whole waves; columns alternate 0/100 so a one-bin slip shows."""
    rng = np.random.default_rng(6)
    n_sft, t_sft, b0 = 96, 1800.0, 360_000
    t_mid = 1.2e9 + t_sft * (np.arange(n_sft) + 0.5)
    v = np.zeros((n_sft, 3))
    v[:, 0] = rng.uniform(-1e-15, 1e-15, n_sft)
    f0 = (b0 + np.arange(700) + 0.5) / t_sft
    first_bin, n_bins = b0 - 4, 712
    cols = np.arange(n_bins) + first_bin
    power = (100.0 * (cols % 2)[None, :] + rng.uniform(0, 1, (n_sft, n_bins))).astype(np.float32)
    w = synth.Workload("half-bin", t_sft, [n_sft], t_mid, v, 1.2e9, first_bin, n_bins, power,
                       None, f0, np.array([0.0, 1e-13]), synth.isotropic_sky(5, rng), 7,
                       np.array([f0[0] - 1e-6, f0[-1] + 1e-6]))
    s64, want = oracle_grid(w)
    for tile in range(1, ft.ft_tile_count() + 1):
        s32, tops, _ = run_gpu(ft, w, tile=tile)
        assert_stats(s32, s64, n_sft)
        assert_toplists(tops, want, s64, n_sft)


def test_guarded_index_modes_on_half_bins(ft):
    """Tracks placed on half-bins at 1 kHz (zero Doppler, f1 = 0) and a hair to
    either side: the guarded modes must recompute every such evaluation in FP64
    and return the canonical bin; the unguarded df64 estimate is not held to it."""
    import torch
    n_sft, t_sft, b0 = 64, 1800.0, 1_800_000
    t_mid = 1.2e9 + t_sft * (np.arange(n_sft) + 0.5)
    v = np.zeros((n_sft, 3))
    x = b0 + np.arange(50) + 0.5
    f0 = np.concatenate([x, np.nextafter(x, 0), np.nextafter(x, np.inf)]) / t_sft
    f1 = np.zeros_like(f0)
    sky = np.tile([[0.0, 0.0, 1.0]], (f0.size, 1))
    first_bin, n_bins = b0 - 4, 64
    power = np.ones((n_sft, n_bins), np.float32)
    w = synth.Workload("half-bin-1kHz", t_sft, [n_sft], t_mid, v, 1.2e9, first_bin, n_bins, power,
                       None, f0[:1], f1[:1], sky[:1], 1, np.array([0.0, 2e3]))
    want = oracle.bins_list(w.t_mid, w.t_ref, w.t_sft, w.v, f0, f1, sky)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.load_workload(w)
        for mode in (ft.FT_INDEX_GUARDED, ft.FT_INDEX_GUARDED_FP32):
            got = c.bins(f0, f1, sky, w.t_ref, mode)
            n, fb = c.count_index_mismatches(f0, f1, sky, w.t_ref, mode, kind=ft.FT_BANK_LIST,
                                             fallback=True)
            assert np.array_equal(got, want) and n == 0
            assert fb == want.size  # every one of them within the margin of an edge


def test_weights_and_host_inputs(ft):
    w = synth.allsky_band(seed=7, n_sky=6, n_per_det=200)
    w.weight = np.random.default_rng(70).uniform(0.2, 1.8, w.n_sft).astype(np.float32)
    s32, tops, _ = run_gpu(ft, w, host_inputs=True)
    s64, want = oracle_grid(w)
    assert_stats(s32, s64, w.n_sft)
    assert_toplists(tops, want, s64, w.n_sft, weight=w.weight)


def test_plain_fp32_sums_keep_exact_toplists(ft):
    w = synth.allsky_band(seed=8, n_sky=6, n_per_det=400)
    s32, tops, info = run_gpu(ft, w, sum_mode=1)
    s64, want = oracle_grid(w)
    rel = np.abs(s32 - s64) / s64
    assert rel.max() <= (w.n_sft + 8) * 2.0 ** -24
    assert_toplists(tops, want, s64, w.n_sft)


def test_out_of_table_track_is_reported(ft):
    import torch
    w = synth.plain_small(seed=9, n_sky=3)
    v = w.v.copy()
    v[50] *= 40.0  # |v| ~ 4e-3: the track leaves the table at SFT 50
    for kind in (0, 1):
        with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
            c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
            c.set_velocities(v)
            if kind == 0:
                c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, 5, w.sub_edges)
            else:
                f0t, f1t, st = oracle.grid_params(w.f0, w.f1, 3)
                c.eval_templates(f0t, f1t, w.sky[st], w.t_ref, 5, w.sub_edges, kind=1)
            with pytest.raises(ft.FtError) as e:
                c.toplist(0, 5)
            assert e.value.status == ft.FT_E_RANGE


def test_argument_and_state_errors(ft):
    import torch
    w = synth.plain_small(seed=10, n_sky=2)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        with pytest.raises(ft.FtError) as e:
            c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, 5, w.sub_edges)
        assert e.value.status == ft.FT_E_STATE
        with pytest.raises(ft.FtError) as e:
            c.set_velocities(w.v)
        assert e.value.status == ft.FT_E_STATE
        bad = w.power.copy()
        bad[3, 7] = np.nan
        with pytest.raises(ft.FtError) as e:
            c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, bad)
        assert e.value.status == ft.FT_E_INVALID
        neg = w.power.copy()
        neg[0, 0] = -1.0
        with pytest.raises(ft.FtError) as e:
            c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, neg)
        assert e.value.status == ft.FT_E_INVALID
        c.load_workload(w)
        vbad = w.v.copy()
        vbad[1] = [1.0, 0, 0]
        with pytest.raises(ft.FtError) as e:
            c.set_velocities(vbad)
        assert e.value.status == ft.FT_E_INVALID
        cases = [
            dict(sky=w.sky * 1.001),                       # not unit vectors
            dict(f0=w.f0[::-1].copy()),                    # grid not increasing
            dict(k=0),
            dict(edges=np.array([101.0, 100.0])),          # edges not increasing
            dict(f0=np.array([np.nan])),
            dict(f0=np.zeros(0)),                          # an empty bank
            dict(sky=np.zeros((0, 3))),
        ]
        for case in cases:
            kw = dict(f0=w.f0, f1=w.f1, sky=w.sky, k=5, edges=w.sub_edges)
            kw.update(case)
            with pytest.raises(ft.FtError) as e:
                c.eval_templates(kw["f0"], kw["f1"], kw["sky"], w.t_ref, kw["k"], kw["edges"])
            assert e.value.status == ft.FT_E_INVALID, case
        with pytest.raises(ft.FtError) as e:
            c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, 5, w.sub_edges,
                             precision=ft.FT_INDEX_FP32)
        assert e.value.status == ft.FT_E_UNSUPPORTED
        # the context still works after errors
        c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, 5, w.sub_edges)
        assert len(c.toplist(0, 5)) == 5


def test_short_subbands_and_empty_subband(ft):
    """K larger than a sub-band's population, and a sub-band with no template."""
    w = synth.plain_small(seed=11, n_sky=2)
    edges = np.array([w.f0[0] - 1e-6, w.f0[3] + 1e-7, w.f0[-1] + 1.0, w.f0[-1] + 2.0])
    s32, tops, _ = run_gpu(ft, w, k=50, edges=edges)
    s64, _ = oracle_grid(w)
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, 2)
    want = oracle.toplist(s64, oracle.subband(f0t, edges), 3, 50)
    assert len(tops[0]) == 4 * 3 * 2 and len(tops[2]) == 0
    assert_toplists(tops, want, s64, w.n_sft)


def test_repeat_is_deterministic(ft):
    w = synth.allsky_band(seed=12, n_sky=8, n_per_det=200)
    a, ta, _ = run_gpu(ft, w)
    b, tb, _ = run_gpu(ft, w)
    assert np.array_equal(a, b)
    assert [[c.index for c in t] for t in ta] == [[c.index for c in t] for t in tb]


def test_alternating_banks_in_one_context(ft):
    """One context evaluating bank A, then B (another sky), then A again, then A
    with one sky coordinate changed by an ulp: each result equals a fresh
    context's (the cached sky order is reused only for the identical sky)."""
    import torch
    w = synth.allsky_band(seed=13, n_sky=40, n_per_det=150)
    sky_b = synth.isotropic_sky(40, np.random.default_rng(99))
    sky_c = w.sky.copy()
    sky_c[7, 0] = np.nextafter(sky_c[7, 0], 2.0)
    fresh = {name: run_gpu(ft, w, sky=sk)[0] for name, sk in (("a", w.sky), ("b", sky_b), ("c", sky_c))}
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.load_workload(w)
        for name, sk in (("a", w.sky), ("b", sky_b), ("a", w.sky), ("c", sky_c), ("a", w.sky)):
            stats = torch.empty(w.f0.size * w.f1.size * sk.shape[0], dtype=torch.float32, device="cuda:0")
            c.eval_templates(w.f0, w.f1, sk, w.t_ref, w.k, w.sub_edges, stats=stats)
            c.sync()
            assert np.array_equal(stats.cpu().numpy(), fresh[name]), name


@pytest.mark.parametrize("n_f0,n_sub", [(1024, 6), (1025, 6), (2048, 6), (2049, 6), (1500, 40)])
@pytest.mark.parametrize("noise", [True, False])
def test_grid_row_lengths_selection(ft, n_f0, n_sub, noise):
    """f0 rows at both sides of the 1024 and 2048 column limits of the selection's
    grid form, more sub-bands than fit its LDS histogram, f0 columns outside every
    sub-band at both ends, and a table of zeros where every template ties."""
    w = synth.wide_band(n_f0, seed=20 + n_f0, with_noise=noise)
    cuts = np.linspace(3, n_f0 - 2, n_sub + 1).round().astype(np.int64)
    edges = w.f0[0] + (cuts - 0.5) / w.t_sft
    s32, tops, _ = run_gpu(ft, w, edges=edges)
    s64, _ = oracle_grid(w)
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    sub = oracle.subband(f0t, edges)
    assert (sub < 0).sum() == 5 * w.f1.size * w.sky.shape[0]
    want = oracle.toplist(s64, sub, n_sub, w.k)
    assert_stats(s32, s64, w.n_sft)
    assert_toplists(tops, want, s64, w.n_sft)
    assert all(len(t) == w.k for t in tops)


def test_max_subbands_and_max_k(ft):
    """The documented maxima: 4096 sub-bands (two f0 columns each, K = 5) on an
    8192-column row, then K = 65536 in one sub-band over 81,920 templates (and
    K above the bank size over a smaller sky)."""
    w = synth.wide_band(8192, seed=31, n_sky=5)
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    s64, _ = oracle_grid(w)
    edges = w.f0[0] + (np.arange(0, 8193, 2) - 0.5) / w.t_sft
    assert edges.size == 4097
    s32, tops, _ = run_gpu(ft, w, k=5, edges=edges)
    want = oracle.toplist(s64, oracle.subband(f0t, edges), 4096, 5)
    assert_stats(s32, s64, w.n_sft)
    assert_toplists(tops, want, s64, w.n_sft)
    one = np.array([w.f0[0] - 0.5 / w.t_sft, w.f0[-1] + 0.5 / w.t_sft])
    _, tops, _ = run_gpu(ft, w, k=65536, edges=one)
    want = oracle.toplist(s64, oracle.subband(f0t, one), 1, 65536)
    assert len(tops[0]) == 65536
    assert_toplists(tops, want, s64, w.n_sft)
    sky3 = w.sky[:3]
    s64_3 = s64[:8192 * w.f1.size * 3]
    _, tops, _ = run_gpu(ft, w, k=65536, edges=one, sky=sky3)
    assert len(tops[0]) == s64_3.size
    assert_toplists(tops, [oracle.toplist(s64_3, np.zeros(s64_3.size, np.int32), 1, 65536)[0]], s64_3, w.n_sft)


def test_joint_maxima_and_candidate_regrowth(ft):
    """K = 65536 with 4096 sub-bands in one call: every sub-band returns all of
    its 20 templates, and the candidate buffer is sized by the bank, not by
    K x sub-bands.  Then a table of zeros over 81,920 templates with K = 25 in
    one sub-band: every template ties at the threshold, more than the first
    candidate buffer (65,536) holds, so the selection grows it to the exact
    count and runs again."""
    w = synth.wide_band(8192, seed=31, n_sky=5)
    f0t, _, _ = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    s64, _ = oracle_grid(w)
    edges = w.f0[0] + (np.arange(0, 8193, 2) - 0.5) / w.t_sft
    s32, tops, _ = run_gpu(ft, w, k=65536, edges=edges)
    want = oracle.toplist(s64, oracle.subband(f0t, edges), 4096, 65536)
    assert all(len(t) == 20 for t in tops)
    assert_stats(s32, s64, w.n_sft)
    assert_toplists(tops, want, s64, w.n_sft)
    z = synth.wide_band(8192, seed=32, n_sky=5, with_noise=False)
    one = np.array([z.f0[0] - 0.5 / z.t_sft, z.f0[-1] + 0.5 / z.t_sft])
    s32, tops, info = run_gpu(ft, z, k=25, edges=one)
    assert info.n_candidates == s32.size == 81920
    s64z, _ = oracle_grid(z)
    f0z, _, _ = oracle.grid_params(z.f0, z.f1, z.sky.shape[0])
    assert_toplists(tops, oracle.toplist(s64z, oracle.subband(f0z, one), 1, 25), s64z, z.n_sft)
