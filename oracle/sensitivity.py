"""FP64 reference of the signal-response quantities of the semi-analytic
sensitivity estimate (Sec. V.A) -- TEST INFRASTRUCTURE ONLY.

For a population sample (sky n, cos iota, psi) and SFTs with arm unit vectors
arms [N, 6] and weights u_k (1 when absent):
  q = (mu_G, sigma_G, rho1, rho2) = (2 sum u, 2 sqrt(sum u^2), sum u rho_k, sum u^2 rho_k),
  rho_k = T_sft (F+^2 A+^2 + Fx^2 Ax^2), A+ = (1 + cos^2 iota)/2, Ax = cos iota,
with the antenna patterns of the injector (inject.antenna_patterns); sums in
SFT order.
"""
from __future__ import annotations

import numpy as np

from .inject import antenna_patterns


def q_sample(t_sft, arms, weight, sky, cos_iota, psi):
    arms = np.asarray(arms, np.float64)
    sky = np.asarray(sky, np.float64)
    n_sft = arms.shape[0]
    u = np.ones(n_sft) if weight is None else np.asarray(weight, np.float32).astype(np.float64)
    out = np.empty((len(cos_iota), 4))
    for i in range(len(cos_iota)):
        fp, fx = antenna_patterns(arms, sky[i], psi[i])
        ap = 0.5 * (1.0 + cos_iota[i] * cos_iota[i])
        ax = cos_iota[i]
        rk = t_sft * (fp * fp * ap * ap + fx * fx * ax * ax)
        out[i, 0] = 2.0 * np.cumsum(u)[-1]
        out[i, 1] = 2.0 * np.sqrt(np.cumsum(u * u)[-1])
        out[i, 2] = np.cumsum(u * rk)[-1]
        out[i, 3] = np.cumsum((u * u) * rk)[-1]
    return out
