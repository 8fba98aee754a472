"""FP64 reference of the weighted number count and of the all-sky weights
(Sec. II.B) -- TEST INFRASTRUCTURE ONLY.

Number count (Eq. number_count): nc[t; f] = 1 when the normalised power exceeds
3.2, else 0; the weighted number count of a template is the sum over SFTs of
w_k nc_k at the template's bins, the same form as Eq. short_coh_general.  In
Gaussian noise P is chi^2 with 2 degrees of freedom, so nc_k is Bernoulli with
p = P(P > 3.2) = exp(-3.2 / 2): noise mean p sum w and variance p (1 - p) sum w^2.

All-sky weights: w_k(n) proportional to (a_k^2(n) + b_k^2(n)) / S_n,k and
normalised to sum 1 over the SFTs, a and b the detector response functions
(F+ = a cos 2psi + b sin 2psi, Fx = b cos 2psi - a sin 2psi, so a^2 + b^2 is
F+^2 + Fx^2 at any psi); 1/S_n,k is the caller's per-SFT weight u_k.

Canonical FP64 form (both sides evaluate exactly this sequence, so the
weighted statistics agree bit for bit):
  x = (u0 n0 + u1 n1) + u2 n2, y = (w0 n0 + w1 n1) + w2 n2,
  c = (u0 w0 + u1 w1) + u2 w2 (arm unit vectors u, w);
  ab = ((1 - c c) - ((x x + y y) - (2 (c x)) y)) + 0.25 ((x x - y y)(x x - y y)),
which is F+^2 + Fx^2 of the detector tensor D = (u u^T - w w^T)/2 written out
(twice the squared norm of D's transverse-traceless part with respect to n;
tests check it against the antenna patterns of the injector);
  W = sum_k u_k ab_k, sequential in SFT order; inv = 1/W;
  w_k = u_k (ab_k inv).
"""
from __future__ import annotations

import math

import numpy as np

from . import core
from .inject import antenna_patterns

NC_THRESHOLD = 3.2


def number_count_table(power):
    """1[P > 3.2] of every table cell (float32 0/1), P compared as a real number."""
    return (np.asarray(power, np.float32).astype(np.float64) > NC_THRESHOLD).astype(np.float32)


def nc_probability():
    """P(P > 3.2) for P ~ chi^2_2: the survival function exp(-x/2) at x = 3.2."""
    return math.exp(-NC_THRESHOLD / 2.0)


def nc_moments(weights):
    """Noise-only (mean, sigma) of the weighted number count for weights w_k (FP64)."""
    w = np.asarray(weights, np.float64)
    p = nc_probability()
    w1 = 0.0
    w2 = 0.0
    for x in w:
        w1 = w1 + x
        w2 = w2 + x * x
    return p * w1, math.sqrt(p * (1.0 - p) * w2)


def power_moments(weights):
    """Noise-only (mean, sigma) of S = sum w P: 2 sum w and 2 sqrt(sum w^2) (Sec. II.B.1)."""
    w = np.asarray(weights, np.float64)
    w1 = 0.0
    w2 = 0.0
    for x in w:
        w1 = w1 + x
        w2 = w2 + x * x
    return 2.0 * w1, 2.0 * math.sqrt(w2)


def response_ab(arms, n):
    """a^2 + b^2 [N] of every SFT's detector for a source in direction n, in
    the canonical closed form."""
    a = np.asarray(arms, np.float64)
    n = np.asarray(n, np.float64)
    x = (a[:, 0] * n[0] + a[:, 1] * n[1]) + a[:, 2] * n[2]
    y = (a[:, 3] * n[0] + a[:, 4] * n[1]) + a[:, 5] * n[2]
    c = (a[:, 0] * a[:, 3] + a[:, 1] * a[:, 4]) + a[:, 2] * a[:, 5]
    x2 = x * x
    y2 = y * y
    dxy = x2 - y2
    return ((1.0 - c * c) - ((x2 + y2) - (2.0 * (c * x)) * y)) + 0.25 * (dxy * dxy)


def response_ab_patterns(arms, n):
    """a^2 + b^2 as F+^2 + Fx^2 from the injector's antenna patterns at psi = 0
    (the tensor contraction; used to check the closed form)."""
    fp, fx = antenna_patterns(np.asarray(arms, np.float64), np.asarray(n, np.float64), 0.0)
    return fp * fp + fx * fx


def sky_weights(arms, u, sky):
    """[n_sky, N] all-sky weights w_k(n) = u_k (a^2 + b^2)_k / sum_k' u_k' (a^2 + b^2)_k'
    (u: per-SFT weights, float32 or None for 1)."""
    arms = np.asarray(arms, np.float64)
    sky = np.atleast_2d(np.asarray(sky, np.float64))
    n_sft = arms.shape[0]
    uu = np.ones(n_sft) if u is None else np.asarray(u, np.float32).astype(np.float64)
    out = np.empty((sky.shape[0], n_sft))
    for s in range(sky.shape[0]):
        ab = response_ab(arms, sky[s])
        c = uu * ab
        total = np.cumsum(c)[-1]  # sequential in SFT order
        inv = 1.0 / total
        out[s] = uu * (ab * inv)
    return out


def weighted_sums(t_mid, t_ref, t_sft, first_bin, table, weights, v, f0, f1, sky):
    """S[t] = sum_k weights[t, k] table[k, B_tk] for templates t of a list bank
    (canonical bins of the oracle), sums sequential in SFT order in FP64."""
    bins = core.bins_list(t_mid, t_ref, t_sft, v, f0, f1, sky)
    return weighted_sums_at(first_bin, table, weights, bins)


def weighted_sums_at(first_bin, table, weights, bins):
    """S[t] = sum_k weights[t, k] table[k, bins[t, k] - first_bin], sequential in
    SFT order in FP64 (bins from any of the oracle's track models)."""
    bins = np.asarray(bins, np.int64)
    tab = np.asarray(table, np.float32).astype(np.float64)
    cols = bins - int(first_bin)
    assert cols.min() >= 0 and cols.max() < tab.shape[1], "track leaves the table"
    w = np.asarray(weights, np.float64)
    acc = np.zeros(bins.shape[0])
    rows = np.arange(bins.shape[1])
    for k in rows:
        acc = acc + w[:, k] * tab[k, cols[:, k]]
    return acc


def grid_as_list(f0, f1, sky):
    """The templates of a grid bank in template order t = (s n_f1 + j) n_f0 + i:
    (f0[t], f1[t], sky[t], sky index[t])."""
    f0 = np.asarray(f0, np.float64)
    f1 = np.asarray(f1, np.float64)
    sky = np.asarray(sky, np.float64)
    s_idx, j_idx, i_idx = np.meshgrid(np.arange(sky.shape[0]), np.arange(f1.size), np.arange(f0.size),
                                      indexing="ij")
    s_idx, j_idx, i_idx = s_idx.ravel(), j_idx.ravel(), i_idx.ravel()
    return f0[i_idx], f1[j_idx], sky[s_idx], s_idx


def eval_grid_sky_weighted(t_mid, t_ref, t_sft, first_bin, table, arms, u, v, f0, f1, sky):
    """Statistic of every template of a grid bank with the all-sky weights:
    (S [n_templates], W [n_sky, N])."""
    W = sky_weights(arms, u, sky)
    lf0, lf1, lsky, s_idx = grid_as_list(f0, f1, sky)
    return weighted_sums(t_mid, t_ref, t_sft, first_bin, table, W[s_idx], v, lf0, lf1, lsky), W
