"""Pins of the oracle's injection-campaign generator (signal hypothesis, Sec. II.B.2).

Philox is pinned to its published known-answer vectors, the Gaussian noise to
N(0, 1), the bin-offset factor to the paper's printed 0.7737, the antenna
patterns to textbook sky averages and a closed-form geometry, and the complete
generator to the non-central chi-squared mean and variance of the statistic.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([[int(x, 16) for x in v["ctr"]]], np.uint64)
        key = np.array([[int(x, 16) for x in v["key"]]], np.uint64)
        out = inject.philox4x32_10(ctr, key)[0]
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_noise_is_standard_normal_and_decorrelated():
    re, im = inject.noise_normals(seed=0x1234_5678_9ABC, run=3, n_sft=200, n_bins=300)
    for x in (re.ravel(), im.ravel()):
        assert stats.kstest(x, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(re.ravel(), im.ravel())[0, 1]) < 0.01
    re2, _ = inject.noise_normals(seed=0x1234_5678_9ABC, run=4, n_sft=200, n_bins=300)
    assert abs(np.corrcoef(re.ravel(), re2.ravel())[0, 1]) < 0.01
    p = re * re + im * im
    assert stats.kstest(p.ravel(), stats.chi2(2).cdf).pvalue > 1e-3


def test_sinc2_bin_average_is_papers_factor():
    """Mean of sinc^2(pi delta) over delta uniform in [-1/2, 1/2): the paper's 0.7737."""
    want = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["sinc2_bin_average"]["value"]
    delta = (np.arange(200_000) + 0.5) / 200_000 - 0.5
    got = float(np.mean(inject.sinc(np.pi * delta) ** 2))
    assert abs(got - want) < 5e-5
    # the three modelled bins keep at least 85% of the power (the sum over all m is 1)
    tot = sum(inject.sinc(np.pi * (delta - m)) ** 2 for m in (-1, 0, 1))
    assert 0.85 < tot.min() and tot.max() <= 1.0 + 1e-12


def test_antenna_pattern_sky_averages():
    """Isotropic sky and uniform psi: <F+^2> = <Fx^2> = 1/5 for a 90-degree
    interferometer; orientation averages <A+^2> = 7/15, <Ax^2> = 1/3."""
    rng = np.random.default_rng(1)
    t = synth.EPOCH + 1800.0 * np.arange(24)
    arms = synth.detector_arms(t, synth.DETECTORS[0])
    fp2, fx2 = [], []
    for n in synth.isotropic_sky(4000, rng):
        psi = rng.uniform(-np.pi / 4, np.pi / 4)
        fp, fx = inject.antenna_patterns(arms, n, psi)
        fp2.append(np.mean(fp ** 2))
        fx2.append(np.mean(fx ** 2))
        assert np.all(fp ** 2 + fx ** 2 <= 1.0 + 1e-12)
    assert abs(np.mean(fp2) - 0.2) < 0.01 and abs(np.mean(fx2) - 0.2) < 0.01
    ci = rng.uniform(-1, 1, 400_000)
    assert abs(np.mean((0.5 * (1 + ci ** 2)) ** 2) - 7 / 15) < 2e-3
    assert abs(np.mean(ci ** 2) - 1 / 3) < 2e-3


def test_antenna_pattern_zenith_closed_form():
    """Source at the detector's zenith, polarisation axes along the arms:
    F+ = +-1, Fx = 0; rotated by 45 degrees: |F+| = 0, |Fx| = 1."""
    u = np.array([1.0, 0.0, 0.0])
    w = np.array([0.0, 1.0, 0.0])
    arms = np.concatenate([u, w])[None, :]
    n = np.array([0.0, 0.0, 1.0])  # zenith of an equatorial-plane detector at the pole
    p, q = inject.wave_frame(n, 0.0)
    psi0 = np.arctan2(p @ w, p @ u)  # rotate the frame so p lies along u
    fp, fx = inject.antenna_patterns(arms, n, -psi0)
    assert abs(abs(fp[0]) - 1.0) < 1e-12 and abs(fx[0]) < 1e-12
    fp, fx = inject.antenna_patterns(arms, n, -psi0 + np.pi / 4)
    assert abs(fp[0]) < 1e-12 and abs(abs(fx[0]) - 1.0) < 1e-12


def test_injected_statistic_is_noncentral_chi2():
    """At the injection's own template, S over N SFTs is non-central chi^2_{2N}
    with non-centrality sum_k rho_k^2 sinc^2(pi delta_k): mean 2N + lambda,
    variance 4N + 4 lambda (Sec. II.B.2 with the textbook variance)."""
    w = synth.plain_small(seed=21, n_sky=1)
    rng = np.random.default_rng(22)
    inj = synth.injection_params(rng, 100.02, 100.08, 0.05, 0.05, -1e-10, 1e-10)
    B, A = inject.signal_amplitudes(w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, inj)
    lam = float(np.sum(A[:, 1] ** 2))
    assert 20 < lam < 2000
    s = []
    for seed in range(300):
        p = inject.generate_table(1000 + seed, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms,
                                  w.first_bin, w.n_bins, inj)
        v, _ = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, p, None, w.v,
                                [inj["f0"]], [inj["f1"]], [inj["sky"]])
        s.append(v[0])
    s = np.array(s)
    n = w.n_sft
    assert abs(s.mean() - (2 * n + lam)) < 5 * np.sqrt((4 * n + 4 * lam) / len(s))
    assert abs(s.var() / (4 * n + 4 * lam) - 1) < 0.25
    assert stats.kstest(s, stats.ncx2(2 * n, lam).cdf).pvalue > 1e-3


def test_injected_bins_light_the_track():
    """A loud injection lights only bins B_k - 1, B_k, B_k + 1 of each SFT, and
    every one of them that carries a large share of the power."""
    w = synth.plain_small(seed=23, n_sky=1)
    rng = np.random.default_rng(24)
    inj = synth.injection_params(rng, 100.02, 100.08, 50.0, 50.0)
    p = inject.generate_table(7, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                              w.n_bins, inj)
    B, A = inject.signal_amplitudes(w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, inj)
    loud = p > 200.0  # a noise-only bin exceeds 200 with probability e^-100
    assert (A[:, 1] ** 2 > 1000.0).mean() > 0.9
    for k in range(w.n_sft):
        cols = set(np.nonzero(loud[k])[0] + w.first_bin)
        allowed = {int(B[k]) + m for m in (-1, 0, 1)}
        must = {int(B[k]) + m for m in (-1, 0, 1) if A[k, m + 1] ** 2 > 1000.0}
        assert must <= cols <= allowed, k


def test_signals_superpose_linearly_in_amplitude():
    """Strain is linear in h0, so two equal signals of amplitude a give the table
    of one signal of amplitude 2a; a signal of amplitude 0 changes nothing."""
    w = synth.plain_small(seed=25, n_sky=1)
    rng = np.random.default_rng(26)
    a = synth.injection_params(rng, 100.02, 100.08, 3.0, 3.0)
    args = (11, 2, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin, w.n_bins)
    two = inject.generate_table(*args, [a, a])
    double = inject.generate_table(*args, dict(a, amp=6.0))
    assert np.allclose(two, double, rtol=1e-6, atol=1e-6)
    assert np.sum(two != inject.generate_table(*args, a)) > w.n_sft
    zero = dict(a, amp=0.0)
    assert np.array_equal(inject.generate_table(*args, [a, zero]), inject.generate_table(*args, a))
    assert np.array_equal(inject.generate_table(*args, [zero]), inject.generate_table(*args))


def _ulp_err(got, want):
    return np.abs(got - want) / np.spacing(np.abs(want))


def test_plog_against_libm():
    """The project logarithm (a fixed sequence of IEEE operations) against the
    C library's log: within 2 ulp over the Box-Muller range [2^-54, 1), exact
    at 1, and e ln 2 at powers of two within an ulp."""
    rng = np.random.default_rng(31)
    x = np.concatenate([
        2.0 ** rng.uniform(-54, 0, 400_000),            # log-uniform over the uniforms' range
        (np.arange(200_000) + 0.5) * 2.0 ** -53,         # the smallest uniforms, exactly as drawn
        1.0 - (np.arange(1, 200_001)) * 2.0 ** -53,      # next to 1 (ln x ~ x - 1)
        rng.uniform(0.5, 2.0, 200_000),                  # the reduction's seam at sqrt(1/2)
        2.0 ** rng.uniform(-1000, 1000, 100_000),
    ])
    got = oracle.core.plog(x)
    want = np.log(x)
    nz = want != 0
    assert _ulp_err(got[nz], want[nz]).max() <= 2.0
    assert oracle.core.plog(np.array([1.0]))[0] == 0.0
    e = np.arange(-60, 61).astype(np.float64)
    e = e[e != 0]
    assert _ulp_err(oracle.core.plog(2.0 ** e), e * np.log(2.0)).max() <= 1.0


def test_c_philox_known_answers_and_numpy_agree():
    """The C Philox-4x32-10 behind the fast table generator gives the published
    known answers and the same words as the numpy implementation."""
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([int(x, 16) for x in v["ctr"]], np.uint32)
        key = [int(x, 16) for x in v["key"]]
        assert [int(x) for x in oracle.core.philox(ctr, key)] == [int(x, 16) for x in v["out"]]
    rng = np.random.default_rng(32)
    ctr = rng.integers(0, 2 ** 32, size=(5000, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
    a = oracle.core.philox(ctr.astype(np.uint32), key).astype(np.uint64)
    b = inject.philox4x32_10(ctr, np.broadcast_to(key, (5000, 2)))
    assert np.array_equal(a, b)


def test_two_table_generators_agree_bit_for_bit():
    """generate_table (C) and generate_table_numpy (Philox and the signal adds
    in numpy) are two implementations of one specification: equal bits, with
    and without signals, at an SFT offset."""
    w = synth.plain_small(seed=33, n_sky=1)
    rng = np.random.default_rng(34)
    injs = [synth.injection_params(rng, 100.02, 100.08, 3.0, 3.0, -1e-10, 1e-10) for _ in range(2)]
    for inj, off in ((None, 0), (injs[0], 0), (injs, 17)):
        args = (0xDEADBEEF12, 5, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin, w.n_bins, inj, off)
        assert np.array_equal(inject.generate_table(*args), inject.generate_table_numpy(*args))


def _zenith_detector(n_sft):
    """Arms along x and y for every SFT, source at the zenith z, no detector motion."""
    arms = np.tile(np.array([1.0, 0.0, 0.0, 0.0, 1.0, 0.0]), (n_sft, 1))
    return arms, np.array([0.0, 0.0, 1.0]), np.zeros((n_sft, 3))


def test_rho2_absolute_scale_at_the_zenith():
    """Source at the zenith of a detector with perpendicular arms, face on
    (cos iota = 1): F+^2 + Fx^2 = 1 at any psi and A+ = Ax = 1, so the
    non-centrality 4|h~|^2/(T S_n) with |h~| = (T/2) h0 is exactly T amp^2
    (amp = h0/sqrt(S_n)).  A factor T/2, or amp in place of amp^2, fails."""
    arms, n, _ = _zenith_detector(4)
    t_sft = 1800.0
    for amp in (0.25, 0.5, 2.0):
        got = inject.rho2(arms, n, 0.0, 1.0, amp, t_sft)
        assert np.all(got == t_sft * amp * amp), (amp, got)
    for psi in np.linspace(-np.pi / 4, np.pi / 4, 9):
        got = inject.rho2(arms, n, psi, 1.0, 0.25, t_sft)
        assert np.allclose(got, 112.5, rtol=1e-14, atol=0), (psi, got)
    # edge on (cos iota = 0): only the plus polarisation, A+ = 1/2
    got = inject.rho2(arms, n, 0.0, 0.0, 0.25, t_sft)
    assert np.allclose(got, 112.5 / 4, rtol=4e-16, atol=0)


def test_mean_power_at_a_bin_centred_track():
    """At a track centred on a bin (delta = 0) the generator adds sqrt(rho^2) to
    Re there and nothing to the neighbours, so the mean power at that bin is
    2 + T amp^2 (non-central chi^2_2) and 2 next to it; 300 seeds x 50 SFTs."""
    n_sft, t_sft, amp = 50, 1800.0, 0.25
    arms, n, v = _zenith_detector(n_sft)
    t_mid = 1e9 + t_sft * (np.arange(n_sft) + 0.5)
    B = 180_010
    inj = dict(f0=B / t_sft, f1=0.0, sky=n, psi=0.0, cos_iota=1.0, amp=amp)
    _, A = inject.signal_amplitudes(t_mid, t_mid[0], t_sft, v, arms, inj)
    assert np.allclose(A[:, 1], np.sqrt(t_sft) * amp, rtol=1e-15) and np.all(A[:, [0, 2]] < 1e-12)
    first = B - 4
    at, side = [], []
    for seed in range(300):
        p = inject.generate_table(500 + seed, 1, t_mid, t_mid[0], t_sft, v, arms, first, 9, inj)
        at.append(p[:, 4])
        side.append(p[:, [3, 5]].ravel())
    at = np.concatenate(at).astype(np.float64)
    side = np.concatenate(side).astype(np.float64)
    lam = t_sft * amp * amp
    assert abs(at.mean() - (2 + lam)) < 5 * np.sqrt((4 + 4 * lam) / at.size)
    assert abs(side.mean() - 2.0) < 5 * np.sqrt(4.0 / side.size)
