"""Semi-analytic sensitivity estimate (Sec. V): the detection probability
p_det(D, o) of a search at depth D = sqrt(S_n)/h0 and oversampling o, by Monte
Carlo over
  * the signal-response quantities q = (mu_G, sigma_G, rho1, rho2) of population
    samples (isotropic sky and orientation), computed by the library
    (ft_q_sample) on the search's SFTs,
  * mismatches m drawn from p(m|o) (mismatch.sample),
  * the Gaussian limit of the statistic (Eq. s_gauss): with
    lambda = (1 - m) eta / D^2,
      mu_S = mu_G + lambda rho1,  sigma_S^2 = sigma_G^2 + 4 lambda rho2,
    z = (s - mu_G) / sigma_G and the detection rule 1[z > tau] (Sec. V.B).
eta = <sinc^2> over a uniform bin offset (0.7737, the paper's factor read as a
power factor) is the power the canonical bin keeps on average; the factor 4 of
sigma_S^2 is the variance 4 + 4 rho^2 of a non-central chi^2_2 (the printed
variance lacks it).  injection_p_det is the comparison the paper makes: plain
injections into Gaussian noise, the loudest template of a random bank around
each, and the same detection rule.

The estimate models the search's loudest template as one template at the
bank's smallest mismatch.  The loudest of a bank is at least as loud as that
template, and near threshold it also collects the noise of its neighbours.
p_det_bounds brackets this gain: the one-template estimate is a lower bound,
and the maximum over the k best templates of each bank (joint mismatches from
one trial) with independent noise draws is an upper bound, since the noise of
nearby templates is positively correlated (Slepian's inequality) and the
templates beyond the k-th add only their chance of a noise excursion past tau.
"""
from __future__ import annotations

import numpy as np

from . import fasttracks as ft
from . import mismatch
from .synth import isotropic_sky

# mean of sinc^2(pi d) over d uniform in [-1/2, 1/2] (integral evaluated to 16 digits)
BIN_OFFSET_POWER = 0.7736950099028163


def population(rng, n):
    """Isotropic sky and orientation: sky [n,3], cos iota U[-1,1], psi U[-pi/4, pi/4]."""
    return isotropic_sky(n, rng), rng.uniform(-1.0, 1.0, n), rng.uniform(-np.pi / 4, np.pi / 4, n)


def q_samples(ctx: ft.Context, arms, n, seed):
    rng = np.random.default_rng(seed)
    sky, ci, psi = population(rng, n)
    return ctx.q_sample(arms, sky, ci, psi)


def z_samples(q, m, eps, depth, eta=BIN_OFFSET_POWER):
    """Critical ratios of the Gaussian model (Eq. s_gauss) for population samples
    q [n, 4], mismatches m [n] and standard normal draws eps [n] at one depth:
    s = mu_G + lambda rho1 + eps sqrt(sigma_G^2 + 4 lambda rho2), lambda = (1 - m) eta / D^2."""
    lam = (1.0 - m) * eta / (depth * depth)
    sd_s = np.sqrt(q[:, 1] ** 2 + 4.0 * lam * q[:, 3])
    return (lam * q[:, 2] + eps * sd_s) / q[:, 1]


def p_det(q, m_samples, depths, tau, seed=0, eta=BIN_OFFSET_POWER):
    """Semi-analytic p_det at each depth (Monte Carlo over the rows of q); tau is
    the detection threshold on z, one value or one per sample."""
    rng = np.random.default_rng(seed)
    q = np.asarray(q, np.float64)
    out = []
    for d in depths:
        m = rng.choice(np.asarray(m_samples, np.float64), q.shape[0])
        eps = rng.standard_normal(q.shape[0])
        out.append(float(np.mean(z_samples(q, m, eps, d, eta) > tau)))
    return np.array(out)


def p_det_bounds(q, m_k, depths, tau, seed=0, eta=BIN_OFFSET_POWER):
    """(lower, upper) p_det at each depth: lower is the one-template estimate at
    the smallest mismatch of each bank; upper detects when any of the k best
    templates of a bank (rows of m_k, drawn jointly) crosses tau with
    independent noise draws.  The same draws serve both bounds and every depth
    (so both fall with depth)."""
    rng = np.random.default_rng(seed)
    q = np.asarray(q, np.float64)
    m_k = np.asarray(m_k, np.float64)
    n, k = q.shape[0], m_k.shape[1]
    rows = m_k[rng.integers(0, m_k.shape[0], n)]
    eps = rng.standard_normal((n, k))
    lo, hi = [], []
    for d in depths:
        z = np.stack([z_samples(q, rows[:, j], eps[:, j], d, eta) for j in range(k)], axis=1)
        lo.append(float(np.mean(z[:, 0] > tau)))
        hi.append(float(np.mean(z.max(axis=1) > tau)))
    return np.array(lo), np.array(hi)


def depth_at(q, m_samples, p, tau, seed=0, eta=BIN_OFFSET_POWER, d_lo=1.0, d_hi=1e4, iters=60):
    """Sensitivity depth D^p (Eq. solve_this): the depth at which the
    semi-analytic p_det equals p, by bisection in log D with the same mismatch
    and normal draws at every depth (so p_det is monotone in D)."""
    rng = np.random.default_rng(seed)
    q = np.asarray(q, np.float64)
    m = rng.choice(np.asarray(m_samples, np.float64), q.shape[0])
    eps = rng.standard_normal(q.shape[0])

    def pd(d):
        return float(np.mean(z_samples(q, m, eps, d, eta) > tau))

    if pd(d_lo) < p:
        return d_lo
    if pd(d_hi) >= p:
        return d_hi
    lo, hi = np.log(d_lo), np.log(d_hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if pd(np.exp(mid)) >= p:
            lo = mid
        else:
            hi = mid
    return float(np.exp(lo))


def injection_p_det(ctx: ft.Context, w, depths, n_inj, o, tau, seed=0):
    """Detected fraction of plain injections at each depth: the loudest template
    of a random bank at oversampling o around each signal, rule z > tau.  The
    trials run on unit weights, so z = (s - 2N) / (2 sqrt(N))."""
    mu, sig = 2.0 * w.n_sft, 2.0 * np.sqrt(w.n_sft)
    out = []
    for i, d in enumerate(depths):
        r = mismatch.sample(ctx, w, o=o, n_trials=n_inj, seed=seed + 7919 * i, amp=1.0 / d)
        z = (np.array([t["s_best"] for t in r["trials"]]) - mu) / sig
        out.append(float(np.mean(z > tau)))
    return np.array(out)
