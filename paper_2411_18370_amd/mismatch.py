"""Mismatch distribution p(m|o) of random template banks (Sec. IV.A).

For each trial a source in a circular binary orbit is injected into Gaussian
noise by the library's generator; the statistic is evaluated at the signal's
own parameters and over a random bank of o N(box) templates drawn uniformly in
the uniform-density coordinates (Eq. unif_transform) in a box of the parameter
space around the signal, and the mismatch of the bank's loudest template is
(Eq. mismatch)
    m = (s(signal) - max_bank s) / (s(signal) - mu_G).
A random bank's density is uniform in xi, so the loudest template near the
signal has the same statistics in a box of a few resolution cells as in the
whole search region; the box keeps a trial to ~10^4 templates instead of the
region's ~10^10.

Resolutions (Eq. example and the binary appendix): delta f0 = 1/T_sft, a sky
cell of solid angle (T_sft f0 v/c)^-2 (split equally between alpha and
sin delta), delta a_p = 1/(T_sft f0 Omega), delta phi_b = 1/(T_sft f0 a_p Omega),
delta Omega = 1/(T_sft T_obs f0 a_p Omega).  The number of templates of a box
at o = 1 is Eq. N_binary: k * (f0^6/6) * alpha * sin delta * (a_p^3/3) *
(Omega^4/4) * phi_b differences, k = T_sft^6 T_obs (v/c)^2.

Every statistic comes from the library (exact FP64 toplists); this module draws
the trials' inputs and forms m from the two statistics.
"""
from __future__ import annotations

import math

import numpy as np

from . import fasttracks as ft
from .synth import BinaryWorkload, isotropic_sky

TWO_PI = 2.0 * math.pi


def resolutions(f0, ap, omega, t_sft, t_obs, vmax):
    """Parameter-space resolutions (delta f0, delta alpha, delta sin delta, delta a_p,
    delta Omega, delta phi_b) at one point."""
    d_sky = 1.0 / (t_sft * f0 * vmax)
    return (1.0 / t_sft, d_sky, d_sky, 1.0 / (t_sft * f0 * omega),
            1.0 / (t_sft * t_obs * f0 * ap * omega), 1.0 / (t_sft * f0 * ap * omega))


def n_templates(region, t_sft, t_obs, vmax):
    """Eq. N_binary over a box region (o = 1)."""
    r = region
    k = t_sft ** 6 * t_obs * vmax ** 2
    return (k * (r["f0_hi"] ** 6 - r["f0_lo"] ** 6) / 6.0 * (r["alpha_hi"] - r["alpha_lo"])
            * (r["sdec_hi"] - r["sdec_lo"]) * (r["ap_hi"] ** 3 - r["ap_lo"] ** 3) / 3.0
            * (r["omega_hi"] ** 4 - r["omega_lo"] ** 4) / 4.0 * (r["phib_hi"] - r["phib_lo"]))


def box_around(lam, half_cells, w: BinaryWorkload, t_obs, vmax):
    """Region of +-half_cells resolutions around lam = (f0, alpha, sdec, ap, omega,
    phib), clipped to the search region (f0, a_p, Omega) and the sky."""
    f0, alpha, sdec, ap, om, pb = lam
    d = resolutions(f0, ap, om, w.t_sft, t_obs, vmax)
    R = w.region
    h = half_cells
    return dict(f0_lo=max(f0 - h * d[0], R["f0_lo"]), f0_hi=min(f0 + h * d[0], R["f0_hi"]),
                alpha_lo=alpha - h * d[1], alpha_hi=alpha + h * d[1],
                sdec_lo=max(sdec - h * d[2], -1.0), sdec_hi=min(sdec + h * d[2], 1.0),
                ap_lo=max(ap - h * d[3], R["ap_lo"]), ap_hi=min(ap + h * d[3], R["ap_hi"]),
                omega_lo=max(om - h * d[4], R["omega_lo"]), omega_hi=min(om + h * d[4], R["omega_hi"]),
                phib_lo=pb - h * d[5], phib_hi=pb + h * d[5])


def draw_signal(rng, region):
    """A signal uniform in the xi coordinates of the search region (inputs only)."""
    u = rng.uniform(0.0, 1.0, 6)
    r = region
    f0 = (r["f0_lo"] ** 6 + u[0] * (r["f0_hi"] ** 6 - r["f0_lo"] ** 6)) ** (1 / 6)
    alpha = TWO_PI * u[1]
    sdec = 2.0 * u[2] - 1.0
    ap = (r["ap_lo"] ** 3 + u[3] * (r["ap_hi"] ** 3 - r["ap_lo"] ** 3)) ** (1 / 3)
    om = (r["omega_lo"] ** 4 + u[4] * (r["omega_hi"] ** 4 - r["omega_lo"] ** 4)) ** 0.25
    pb = TWO_PI * u[5]
    return f0, alpha, sdec, ap, om, pb


def sample(ctx: ft.Context, w: BinaryWorkload, o: float, n_trials: int, seed: int, amp: float = 1.0,
           half_cells: float = 2.0, f_margin: float = 0.01, k_best: int = 1):
    """n_trials mismatches of random banks at oversampling o.  Returns a dict with
    the mismatches and every trial's inputs (signal, injection, seeds, box, n).
    With k_best > 1, "m_k" [n_trials, k_best] also holds the mismatches of the
    k_best loudest templates of each bank in decreasing order of s (1.0 where
    the bank has fewer templates); at a high signal amplitude these are the
    bank's k_best smallest mismatches."""
    rng = np.random.default_rng(seed)
    t_obs = float(w.t_mid.max() - w.t_mid.min() + w.t_sft)
    vmax = float(np.max(np.linalg.norm(w.v, axis=1)))
    mu_g = 2.0 * w.n_sft
    inner = dict(w.region, f0_lo=w.region["f0_lo"] + f_margin, f0_hi=w.region["f0_hi"] - f_margin)
    ms, mks, trials = [], [], []
    for trial in range(n_trials):
        lam = draw_signal(rng, inner)
        f0, alpha, sdec, ap, om, pb = lam
        cd = math.sqrt(1.0 - sdec * sdec)
        n = np.array([cd * math.cos(alpha), cd * math.sin(alpha), sdec])
        n /= np.linalg.norm(n)
        inj = dict(amp=amp, cos_iota=float(rng.uniform(-1, 1)), psi=float(rng.uniform(-np.pi / 4, np.pi / 4)),
                   sky=n, f0=f0, f1=0.0, ap=ap, omega=om, phib=pb)
        noise_seed = int(rng.integers(1, 2 ** 62))
        bank_seed = int(rng.integers(1, 2 ** 62))
        ctx.gen_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.n_bins, w.v, w.arms, noise_seed,
                     trial, w.t_ref, inj)
        edges = np.array([w.region["f0_lo"] - 1.0, w.region["f0_hi"] + 1.0])
        one = lambda x: np.array([x], np.float64)
        ctx.eval_binary(one(f0), n[None, :], one(ap), one(om), one(pb), w.t_ref, 1, edges)
        s_sig = ctx.toplist(0, 1)[0].s64
        box = box_around(lam, half_cells, w, t_obs, vmax)
        n_bank = max(1, int(round(o * n_templates(box, w.t_sft, t_obs, vmax))))
        ctx.eval_binary_random(box, bank_seed, n_bank, w.t_ref, k_best, edges)
        top = ctx.toplist(0, k_best)
        best = top[0]
        m = (s_sig - best.s64) / (s_sig - mu_g)
        ms.append(m)
        mk = np.ones(k_best)
        mk[:len(top)] = [(s_sig - t.s64) / (s_sig - mu_g) for t in top]
        mks.append(mk)
        trials.append(dict(inj=inj, noise_seed=noise_seed, run=trial, bank_seed=bank_seed, box=box,
                           n_bank=n_bank, s_signal=s_sig, s_best=best.s64, best_index=best.index))
    return dict(o=o, m=np.array(ms), m_k=np.array(mks), trials=trials, t_obs=t_obs, vmax=vmax)


def summary(m):
    """Mean, median, standard deviation and quantiles of mismatches."""
    m = np.asarray(m, np.float64)
    q = np.quantile(m, [0.05, 0.25, 0.5, 0.75, 0.95])
    return dict(n=int(m.size), mean=float(m.mean()), std=float(m.std()), q05=float(q[0]), q25=float(q[1]),
                median=float(q[2]), q75=float(q[3]), q95=float(q[4]))
