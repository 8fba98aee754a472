"""Sources in circular binary systems on the GPU (Eq. track with a_p > 0, the
paper's benchmark and search workload): the library cosine, the bins and the
random template bank bit for bit against the oracle, the exact toplists of
explicit and generated banks, range and argument errors, and a sampled check
at the benchmark's size (10^6 templates x 10^4 SFTs)."""
import numpy as np
import pytest

import oracle
from oracle import bank as obank
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _ctx(ft, w):
    import torch
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
    c.set_velocities(w.v)
    return c


def rel_bound(n_sft):
    return 40 * 2.0 ** -24 + 4 * n_sft * 2.0 ** -53


def test_library_cosine_is_bitexact(ft):
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([np.linspace(-100.0, 100.0, 200_001), rng.uniform(-1.4e6, 1.4e6, 200_000),
                        [0.0, -0.0, 1e-300, np.pi / 2]])
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        gc, gs = c.lib_sincos(x)
        with pytest.raises(ft.FtError):
            c.lib_sincos(np.array([2e6]))
    oc, os_ = oracle.pcos(x)
    assert np.array_equal(gc.view(np.uint64), oc.view(np.uint64))
    assert np.array_equal(gs.view(np.uint64), os_.view(np.uint64))


def test_binary_bins_are_bitexact(ft):
    w = synth.binary_band(seed=21, n_tmpl=3000, n_per_det=400)
    with _ctx(ft, w) as c:
        got = c.bins_binary(w.f0, w.sky, w.ap, w.omega, w.phib, w.t_ref)
    want = oracle.bins_binary(w.t_mid, w.t_ref, w.t_sft, w.v, w.f0, w.sky, w.ap, w.omega, w.phib)
    assert np.array_equal(got.astype(np.int64), want)


def _check_toplists(ft, c, w, s64, k, f0, stats=None):
    mu, sig = oracle.noise_moments(w.n_sft)
    sub = oracle.subband(f0, w.sub_edges)
    want = oracle.toplist(s64, sub, len(w.sub_edges) - 1, k)
    for j, idx in enumerate(want):
        top = c.toplist(j, k)
        assert [t.index for t in top] == list(idx), j
        for t in top:
            assert t.s64 == s64[t.index]
            assert t.sub == j and t.f0 == f0[t.index]
            assert abs(t.z - (t.s64 - mu) / sig) <= 1e-12 * abs(t.z)
            assert abs(t.s32 - t.s64) <= rel_bound(w.n_sft) * t.s64
    if stats is not None:
        rel = np.abs(stats.astype(np.float64) - s64) / s64
        assert rel.max() <= rel_bound(w.n_sft)


@pytest.mark.parametrize("cos_mode", [0, 1])
@pytest.mark.parametrize("n_tmpl,n_per_det,trim", [(5000, 300, 0), (777, 61, 1), (300, 7, 1)])
def test_binary_bank_toplists_match_oracle(ft, n_tmpl, n_per_det, trim, cos_mode):
    """Ragged template counts and SFT counts (odd, and below one 32-SFT sum block),
    with the hardware-cosine and the polynomial track estimates."""
    import torch
    w = synth.binary_band(seed=22, n_tmpl=n_tmpl, n_per_det=n_per_det)
    if trim:
        w.t_mid, w.v, w.power = w.t_mid[:-trim], w.v[:-trim], np.ascontiguousarray(w.power[:-trim])
        w.n_sft_per_det = [n_per_det, n_per_det - trim]
    s64, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0,
                                  w.sky, w.ap, w.omega, w.phib)
    assert bad == -1
    k = 25
    stats = torch.empty(n_tmpl, dtype=torch.float32, device="cuda")
    with _ctx(ft, w) as c:
        c.binary_cos_mode(cos_mode)
        c.eval_binary(w.f0, w.sky, w.ap, w.omega, w.phib, w.t_ref, k, w.sub_edges, stats=stats)
        c.sync()  # the library may run on its own stream
        _check_toplists(ft, c, w, s64, k, w.f0, stats.cpu().numpy())
        # plain FP32 sums (study mode): the same toplists here, looser statistics
        c.eval_binary(w.f0, w.sky, w.ap, w.omega, w.phib, w.t_ref, k, w.sub_edges,
                      sum_mode=ft.FT_SUM_PLAIN_FP32)
        assert [t.index for t in c.toplist(0, k)] == \
            list(oracle.toplist(s64, oracle.subband(w.f0, w.sub_edges), len(w.sub_edges) - 1, k)[0])


@pytest.mark.parametrize("cos_mode", [0, 1])
def test_random_bank_is_bitexact_and_evaluates_like_the_explicit_bank(ft, cos_mode):
    w = synth.binary_band(seed=23, n_tmpl=1, n_per_det=250)
    n, seed, k = 6000, 12345, 20
    f0, sky, ap, om, pb = obank.random_binary_bank(seed, 0, n, **w.region)
    s64, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, f0, sky,
                                  ap, om, pb)
    assert bad == -1
    with _ctx(ft, w) as c:
        got = c.gen_binary_bank(w.region, seed, 0, n)
        for a, b in zip(got, (f0, sky, ap, om, pb)):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        part = c.gen_binary_bank(w.region, seed, 4000, 7)
        assert all(np.array_equal(a, b[4000:4007]) for a, b in zip(part, (f0, sky, ap, om, pb)))
        # a local box (sky and phase limits)
        box = dict(w.region, alpha_lo=1.0, alpha_hi=1.3, sdec_lo=-0.2, sdec_hi=0.05, phib_lo=-2.0,
                   phib_hi=3.5)
        gb = c.gen_binary_bank(box, seed, 17, 3000)
        ob = obank.random_binary_bank(seed, 17, 3000, **box)
        for a, b in zip(gb, ob):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert np.all((gb[1][:, 2] >= -0.2) & (gb[1][:, 2] <= 0.05))
        assert np.all((gb[4] >= -2.0) & (gb[4] <= 3.5))
        c.binary_cos_mode(cos_mode)
        c.eval_binary_random(w.region, seed, n, w.t_ref, k, w.sub_edges)
        _check_toplists(ft, c, w, s64, k, f0)
        c.eval_binary(f0, sky, ap, om, pb, w.t_ref, k, w.sub_edges)
        _check_toplists(ft, c, w, s64, k, f0)


def test_hardware_cosine_bound(ft):
    """The error of v_cos_f32 over every float in [0, 1] is measured once per
    context; it is small enough for the estimate, and mode 1 switches to the
    polynomial (the bins are canonical either way)."""
    w = synth.binary_band(seed=25, n_tmpl=50, n_per_det=20)
    with _ctx(ft, w) as c:
        err = c.binary_cos_mode(0)
        print("hardware cosine max error over [0, 1]:", err, flush=True)
        assert 0.0 < err < 1e-4
        assert c.binary_cos_mode(1) == err
        with pytest.raises(ft.FtError):
            c.binary_cos_mode(2)


def test_binary_range_and_argument_errors(ft):
    w = synth.binary_band(seed=24, n_tmpl=200, n_per_det=100)
    with _ctx(ft, w) as c:
        args = (w.f0, w.sky, w.ap, w.omega, w.phib)
        # a table starting above the lowest tracks: reported, never clamped
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin + 40, np.ascontiguousarray(w.power[:, 40:]))
        c.set_velocities(w.v)
        c.eval_binary(*args, w.t_ref, 5, w.sub_edges)
        with pytest.raises(ft.FtError) as e:
            c.toplist(0, 5)
        assert e.value.status == ft.FT_E_RANGE
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
        c.set_velocities(w.v)
        c.eval_binary(*args, w.t_ref, 5, w.sub_edges)
        assert len(c.toplist(0, 5)) == 5
        for bad in (dict(ap=-w.ap), dict(omega=w.omega * 1e4), dict(phib=w.phib + 2e6),
                    dict(f0=-w.f0)):
            a = dict(zip(("f0", "sky", "ap", "omega", "phib"), args))
            a.update(bad)
            with pytest.raises(ft.FtError):
                c.eval_binary(a["f0"], a["sky"], a["ap"], a["omega"], a["phib"], w.t_ref, 5, w.sub_edges)
        with pytest.raises(ft.FtError) as e:
            c.gen_binary_bank(dict(w.region, ap_lo=0.0), 1, 0, 10)
        assert e.value.status == ft.FT_E_INVALID
        with pytest.raises(ft.FtError) as e:
            c.count_index_mismatches(w.f0, w.f0, w.sky, w.t_ref, ft.FT_INDEX_FP32, kind=ft.FT_BANK_BINARY)
        assert e.value.status in (ft.FT_E_UNSUPPORTED, ft.FT_E_INVALID)


def test_binary_random_bank_at_benchmark_size(ft):
    """10^6 generated templates x 2 x 5000 SFTs (the bench configuration): sampled
    templates and every toplist member against the oracle; nothing outside a
    toplist beats its K-th member beyond the FP32 bound."""
    import torch
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    n, seed, k = 1_000_000, 2024, 10
    stats = torch.empty(n, dtype=torch.float32, device="cuda")
    with _ctx(ft, w) as c:
        c.eval_binary_random(w.region, seed, n, w.t_ref, k, w.sub_edges, stats=stats)
        tops = [c.toplist(j, k) for j in range(len(w.sub_edges) - 1)]  # synchronises
        print("eval ms", c.info().eval_ms, flush=True)
    rng = np.random.default_rng(9)
    sample = np.sort(rng.choice(n, 1500, replace=False))
    members = np.array([t.index for top in tops for t in top])
    idx = np.concatenate([sample, members])
    bank = obank.random_binary_bank(seed, 0, n, **w.region)
    f0, sky, ap, om, pb = (a[idx] for a in bank)
    s64, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, f0, sky, ap,
                                  om, pb)
    assert bad == -1
    exact = dict(zip(idx.tolist(), s64.tolist()))
    s32 = stats[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(s32 - s64) / s64) <= rel_bound(w.n_sft)
    sub_all = oracle.subband(bank[0], w.sub_edges)
    S = stats.cpu().numpy()
    for j, top in enumerate(tops):
        assert len(top) == k
        for t in top:
            assert t.s64 == exact[t.index] and t.sub == j
        keys = [(-t.s64, t.index) for t in top]
        assert keys == sorted(keys)
        rest = S[(sub_all == j)].astype(np.float64)
        thr = top[-1].s64
        assert np.sort(rest)[-k - 1] <= thr * (1 + rel_bound(w.n_sft))


def test_binary_random_bank_sky_weights_at_benchmark_size(ft):
    """The bench's 10^6-template random bank with the all-sky weights (normalised
    per template): sampled templates and every toplist member against the
    oracle's per-template weights (S64 and z bit for bit); nothing outside a
    toplist beats its K-th member beyond the FP32 bound."""
    import torch
    from oracle import weighting as ow
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    n, seed, k = 1_000_000, 2025, 10
    stats = torch.empty(n, dtype=torch.float32, device="cuda")
    with _ctx(ft, w) as c:
        c.set_arms(w.arms)
        c.eval_binary_random(w.region, seed, n, w.t_ref, k, w.sub_edges, stats=stats,
                             weights=ft.FT_WEIGHTS_SKY)
        tops = [c.toplist(j, k) for j in range(len(w.sub_edges) - 1)]
        print("eval ms", c.info().eval_ms, flush=True)
    rng = np.random.default_rng(10)
    sample = np.sort(rng.choice(n, 800, replace=False))
    members = np.array([t.index for top in tops for t in top])
    idx = np.concatenate([sample, members])
    bank = obank.random_binary_bank(seed, 0, n, **w.region)
    f0, sky, ap, om, pb = (a[idx] for a in bank)
    bins = oracle.bins_binary(w.t_mid, w.t_ref, w.t_sft, w.v, f0, sky, ap, om, pb)
    W = ow.sky_weights(w.arms, None, sky)
    S = ow.weighted_sums_at(w.first_bin, w.power, W, bins)
    bound = 44 * 2.0 ** -24 + 4 * w.n_sft * 2.0 ** -53
    s32 = stats[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(s32 - S) / S) <= bound
    exact = dict(zip(idx.tolist(), S.tolist()))
    row = dict(zip(idx.tolist(), range(idx.size)))
    sub_all = oracle.subband(bank[0], w.sub_edges)
    St = stats.cpu().numpy()
    for j, top in enumerate(tops):
        assert len(top) == k
        for t in top:
            assert t.s64 == exact[t.index] and t.sub == j
            mu, sig = ow.power_moments(W[row[t.index]])
            assert t.z == (exact[t.index] - mu) / sig
        rest = St[(sub_all == j)].astype(np.float64)
        assert np.sort(rest)[-k - 1] <= top[-1].s64 * (1 + bound)


@pytest.mark.parametrize("cos_mode", [0, 1])
@pytest.mark.parametrize("n_small", [1000, 100_000])
def test_split_small_bank_equals_unsplit_bits(ft, n_small, cos_mode):
    """Banks below 2^19 templates split their 32-SFT blocks over workgroup rows
    and add the block sums afterwards; the same templates as the head of a bank
    of 2^19 + 123 (evaluated one lane per template over every SFT) give the same
    statistics bit for bit.  302 SFTs: 10 blocks, the last one of 14."""
    import torch
    w = synth.binary_band(seed=41, n_tmpl=n_small, n_per_det=151)
    n_big = 2 ** 19 + 123
    reps = -(-n_big // n_small)
    big = [np.concatenate([a] * reps)[:n_big] for a in (w.f0, w.sky, w.ap, w.omega, w.phib)]
    s_small = torch.empty(n_small, dtype=torch.float32, device="cuda")
    s_big = torch.empty(n_big, dtype=torch.float32, device="cuda")
    with _ctx(ft, w) as c:
        c.binary_cos_mode(cos_mode)
        c.eval_binary(w.f0, w.sky, w.ap, w.omega, w.phib, w.t_ref, 5, w.sub_edges, stats=s_small)
        c.sync()
        c.eval_binary(*big, w.t_ref, 5, w.sub_edges, stats=s_big)
        c.sync()
    a, b = s_small.cpu().numpy(), s_big.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b[:n_small].view(np.uint32))
    assert np.array_equal(a.view(np.uint32), b[n_small:2 * n_small].view(np.uint32))
