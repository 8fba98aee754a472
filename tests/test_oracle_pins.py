"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula: tracks are *constructed* so that
the bin each SFT must hit is an integer known in advance, noise sums are
checked against the chi-squared closed forms of Sec. II.B.1, and toplists
against a brute-force sort.  A dropped term, a flipped Doppler sign, a
transposed velocity component or a wrong time origin each fails one of them.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

T_SFT = 1800.0


def _zero_v(n):
    return np.zeros((n, 3))


def _planted_table(bins_abs, n_sft, first_bin, n_bins, rng):
    """Table that is zero except for one distinct value per SFT at the given bin."""
    p = np.zeros((n_sft, n_bins), np.float32)
    vals = rng.uniform(1.0, 2.0, n_sft).astype(np.float32)
    p[np.arange(n_sft), np.asarray(bins_abs) - first_bin] = vals
    return p, vals


def _seq_sum(vals):
    # np.cumsum is sequential, so its last element is the left-to-right FP64 sum
    return float(np.cumsum(np.asarray(vals, np.float64))[-1])


def test_column_sum_special_case():
    """v = 0 and f1 = 0: every SFT hits the same bin, S is the column sum."""
    rng = np.random.default_rng(10)
    n_sft, first_bin, n_bins = 57, 179_990, 40
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    p = rng.uniform(0, 5, (n_sft, n_bins)).astype(np.float32)
    for b0 in (179_990, 180_001, 180_029):
        f0 = (b0 + 0.25) / T_SFT
        s, bad = oracle.eval_list(t_mid, 1.2e9, T_SFT, first_bin, p, None, _zero_v(n_sft),
                                  [f0], [0.0], [[0.0, 0.0, 1.0]])
        assert bad == -1
        assert s[0] == _seq_sum(p[:, b0 - first_bin])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_doppler_track_hits_constructed_bins(axis):
    """n along one axis, v along the same axis with v.n = m_k/B0: the track
    (1 + v.n) f0 T with f0 = B0/T must land on B0 + m_k (Eq. track sign)."""
    rng = np.random.default_rng(11 + axis)
    n_sft, b0 = 80, 180_000
    m = rng.integers(-15, 16, n_sft)
    v = np.zeros((n_sft, 3))
    v[:, axis] = m / b0
    # the other components carry different offsets so a transposed index misses
    v[:, (axis + 1) % 3] = rng.integers(-15, 16, n_sft) / b0 + 3.0 / b0
    v[:, (axis + 2) % 3] = -rng.integers(1, 9, n_sft) / b0
    n = np.zeros(3)
    n[axis] = 1.0
    first_bin, n_bins = b0 - 40, 81
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    p, vals = _planted_table(b0 + m, n_sft, first_bin, n_bins, rng)
    s, bad = oracle.eval_list(t_mid, 1.2e9, T_SFT, first_bin, p, None, v, [b0 / T_SFT], [0.0],
                              [n])
    assert bad == -1
    assert s[0] == _seq_sum(vals)
    bins = oracle.bins_list(t_mid, 1.2e9, T_SFT, v, [b0 / T_SFT], [0.0], [n])
    assert np.array_equal(bins[0], b0 + m)


def test_oblique_sky_projection():
    """v = d_k * n for an oblique unit n: v.n = d_k (Eq. track projection)."""
    rng = np.random.default_rng(5)
    n_sft, b0 = 64, 360_000
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    m = rng.integers(-30, 31, n_sft)
    v = (m / b0)[:, None] * n[None, :]
    first_bin, n_bins = b0 - 40, 81
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    bins = oracle.bins_list(t_mid, 1.2e9, T_SFT, v, [b0 / T_SFT], [0.0], [n])
    assert np.array_equal(bins[0], b0 + m)


def test_spindown_and_doppler_compose_multiplicatively():
    """f_k = (f0 + f1 dt_k)(1 + v.n): with f1 dt_k T = r k' and v.n = m_k/(B0 + r k')
    the bin is B0 + r k' + m_k, k' = k - k_ref (negative before t_ref).  An
    additive Doppler f0(1+v.n) + f1 dt, a dropped f1 term or a wrong time origin
    all miss (the cross term r k' m_k/(B0 + r k') reaches several bins here)."""
    rng = np.random.default_rng(7)
    n_sft, b0, r, k_ref = 120, 1000, 7, 40
    dt_slot = T_SFT
    t_ref = 1.2e9
    t_mid = t_ref + dt_slot * (np.arange(n_sft) - k_ref)      # dt = k' * dt_slot
    f1 = r / (T_SFT * dt_slot)
    kp = np.arange(n_sft) - k_ref
    m = rng.integers(-12, 13, n_sft)
    v = np.zeros((n_sft, 3))
    v[:, 2] = m / (b0 + r * kp)
    expected = b0 + r * kp + m
    bins = oracle.bins_list(t_mid, t_ref, T_SFT, v, [b0 / T_SFT], [f1], [[0, 0, 1.0]])
    assert np.array_equal(bins[0], expected)
    cross = np.abs(r * kp * m / (b0 + r * kp))
    assert cross.max() > 3  # the test discriminates the composition
    first_bin = int(expected.min()) - 2
    n_bins = int(expected.max()) - first_bin + 3
    p, vals = _planted_table(expected, n_sft, first_bin, n_bins, rng)
    s, bad = oracle.eval_list(t_mid, t_ref, T_SFT, first_bin, p, None, v, [b0 / T_SFT], [f1],
                              [[0, 0, 1.0]])
    assert bad == -1 and s[0] == _seq_sum(vals)


def test_weights_multiply_power():
    """Weighted statistic sum_k w_k P[k][b] with w = 2^j exact (Eq. short_coh_general)."""
    rng = np.random.default_rng(8)
    n_sft, b0 = 30, 180_003
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    p = rng.uniform(0, 4, (n_sft, 8)).astype(np.float32)
    w = (2.0 ** rng.integers(-3, 4, n_sft)).astype(np.float32)
    s, _ = oracle.eval_list(t_mid, 1.2e9, T_SFT, b0 - 3, p, w, _zero_v(n_sft),
                            [(b0 + 0.1) / T_SFT], [0.0], [[1.0, 0, 0]])
    assert s[0] == _seq_sum(w.astype(np.float64) * p[:, 3])


def _noise_columns(n_sft, n_cols, seed, weight=None):
    from paper_2411_18370_amd import synth
    rng = np.random.default_rng(seed)
    p = synth.noise_power(n_sft, n_cols, rng)
    first_bin = 200_000
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    f0 = (first_bin + np.arange(n_cols) + 0.3) / T_SFT
    s, bad = oracle.eval_list(t_mid, 1.2e9, T_SFT, first_bin, p, weight, _zero_v(n_sft), f0,
                              np.zeros(n_cols), np.tile([0, 0, 1.0], (n_cols, 1)))
    assert bad == -1
    return s


def test_noise_sum_is_chi2_2n():
    """Unweighted noise-only S over N independent bins is exactly chi^2_{2N}
    (Eq. s_chi2 summed); mean 2N and variance 4N (mu_G, sigma_G^2)."""
    n_sft, n_cols = 50, 4000
    s = _noise_columns(n_sft, n_cols, 21)
    ks = stats.kstest(s, stats.chi2(2 * n_sft).cdf)
    assert ks.pvalue > 1e-3
    assert abs(s.mean() - 2 * n_sft) < 5 * np.sqrt(4 * n_sft / n_cols)
    assert abs(s.var() / (4 * n_sft) - 1) < 0.1


def test_weighted_noise_moments_and_z():
    """mu_G = 2 sum w, sigma_G^2 = 4 sum w^2 (Sec. II.B.1); z ~ (0, 1)."""
    rng = np.random.default_rng(3)
    n_sft, n_cols = 400, 3000
    w = rng.uniform(0.2, 1.8, n_sft).astype(np.float32)
    s = _noise_columns(n_sft, n_cols, 22, weight=w)
    mu, sig = oracle.noise_moments(n_sft, w)
    wd = w.astype(np.float64)
    assert np.isclose(mu, 2 * wd.sum(), rtol=1e-12)
    assert np.isclose(sig, np.sqrt(4 * (wd ** 2).sum()), rtol=1e-12)
    assert abs(s.mean() - mu) < 5 * sig / np.sqrt(n_cols)
    assert abs(s.std() / sig - 1) < 0.06
    z = oracle.critical_ratio(s, n_sft, w)
    assert abs(z.mean()) < 0.1 and abs(z.std() - 1) < 0.06
    # z is scale-free: doubling every weight (exact in binary) leaves it unchanged
    z2 = oracle.critical_ratio(2.0 * s, n_sft, 2.0 * w)
    assert np.array_equal(z, z2)


def test_toplist_matches_brute_force_sort_with_ties():
    rng = np.random.default_rng(4)
    n, n_sub, k = 5000, 4, 17
    s = rng.integers(0, 300, n).astype(np.float64)     # many exact ties
    sub = rng.integers(-1, n_sub, n).astype(np.int32)  # -1: outside every sub-band
    got = oracle.toplist(s, sub, n_sub, k)
    for j in range(n_sub):
        members = [t for t in range(n) if sub[t] == j]
        want = sorted(members, key=lambda t: (-s[t], t))[:k]
        assert list(got[j]) == want


def test_toplist_short_subband():
    s = np.array([1.0, 3.0, 3.0, 2.0])
    got = oracle.toplist(s, np.array([0, 0, 1, 0], np.int32), 2, 5)
    assert list(got[0]) == [1, 3, 0] and list(got[1]) == [2]


def test_subband_half_open():
    edges = np.array([1.0, 2.0, 3.0])
    sub = oracle.subband(np.array([0.5, 1.0, 1.999, 2.0, 2.5, 3.0]), edges)
    assert list(sub) == [-1, 0, 0, 1, 1, -1]


def test_out_of_table_track_is_an_error():
    n_sft = 10
    t_mid = 1.2e9 + T_SFT * (np.arange(n_sft) + 0.5)
    p = np.ones((n_sft, 5), np.float32)
    v = np.zeros((n_sft, 3))
    v[7, 0] = 3.0 / 100_000  # pushes SFT 7 three bins up, past the table
    s, bad = oracle.eval_list(t_mid, 1.2e9, T_SFT, 99_998, p, None, v,
                              [100_000.1 / T_SFT, 100_000.1 / T_SFT], [0.0, 0.0],
                              [[0, 0, 1.0], [1.0, 0, 0]])
    assert bad == 1 and np.isfinite(s[0]) and np.isnan(s[1])


def test_grid_equals_list_on_workload():
    """Grid and list entry points agree bit for bit on the 1-detector workload."""
    from paper_2411_18370_amd import synth
    w = synth.plain_small(n_sky=4)
    sg, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v,
                               w.f0, w.f1, w.sky)
    f0t, f1t, st = oracle.grid_params(w.f0, w.f1, w.sky.shape[0])
    sl, bad2 = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v,
                                f0t, f1t, w.sky[st])
    assert bad == bad2 == -1
    assert np.array_equal(sg, sl)


def test_degenerate_spindown_triplets_tie_exactly():
    """With |f1| = 1e-10 Hz/s over 100 SFTs the spindown moves tracks by at most
    ~0.03 bin, so many f1 triplets share every bin and tie exactly; the toplist
    must then break the tie by template index."""
    from paper_2411_18370_amd import synth
    w = synth.plain_small(n_sky=3)
    s, _ = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v,
                            w.f0, w.f1, w.sky)
    s = s.reshape(3, 3, 180)
    ties = np.mean((s[:, 0] == s[:, 1]) & (s[:, 1] == s[:, 2]))
    assert ties > 0.3
