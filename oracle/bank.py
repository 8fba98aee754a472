"""FP64 reference of the random template bank for sources in circular binary
systems -- TEST INFRASTRUCTURE ONLY.

Templates are drawn uniformly in the uniform-density coordinates of the
binary appendix (Eq. unif_transform): xi is, up to constants, (f0^6, alpha,
sin delta, a_p^3, Omega^4, phi_b), so a uniform draw in xi is
  f0 = root6(lo^6 + u0 (hi^6 - lo^6)), alpha = lo + u1 (hi - lo),
  sin delta = lo + u2 (hi - lo), a_p = root3(lo^3 + u3 (hi^3 - lo^3)),
  Omega = root4(lo^4 + u4 (hi^4 - lo^4)), phi_b = lo + u5 (hi - lo)
(the whole sky and phase range: alpha and phi_b in [0, 2 pi], sin delta in [-1, 1]),
with n = (cos delta cos alpha, cos delta sin alpha, sin delta), cos delta =
sqrt(1 - sin^2 delta) and the library cosine/sine for alpha.

Uniforms: template i uses three Philox-4x32-10 calls (Salmon et al., SC'11)
with counter (i_lo, i_hi, 0, 1 + j), j = 0, 1, 2, and key (seed_lo, seed_hi);
each call gives two 53-bit uniforms (m + 1/2) 2^-53 from its two 64-bit halves:
(u0, u1), (u2, u3), (u4, u5).  (The noise generator uses counter word 3 = 0,
so the streams never meet.)

Roots: a fixed sequence of IEEE operations, so that any implementation of it
returns the same bits -- 12 Newton steps z <- z - (z^p - y) / (p z^(p-1))
from the linear interpolation lo + u (hi - lo), with powers formed as
z^3 = (z z) z, z^4 = (z z)(z z), z^5 = ((z z)(z z)) z, z^6 = ((z z) z)((z z) z).
"""
from __future__ import annotations

import numpy as np

from .core import pcos
from .inject import MASK32, philox4x32_10, uniform_pair

TWO_PI = float.fromhex("0x1.921fb54442d18p+2")
NEWTON_STEPS = 12


def _pow(z, p):
    z2 = z * z
    if p == 2:
        return z2
    if p == 3:
        return z2 * z
    if p == 4:
        return z2 * z2
    if p == 5:
        return (z2 * z2) * z
    if p == 6:
        z3 = z2 * z
        return z3 * z3
    raise ValueError(p)


def root(lo, hi, u, p):
    """The p-th root of lo^p + u (hi^p - lo^p) by the fixed Newton sequence."""
    lo = np.float64(lo)
    hi = np.float64(hi)
    y = _pow(lo, p) + u * (_pow(hi, p) - _pow(lo, p))
    z = lo + u * (hi - lo)
    for _ in range(NEWTON_STEPS):
        z = z - (_pow(z, p) - y) / (np.float64(p) * _pow(z, p - 1))
    return z


def uniforms(seed, first, n):
    """u [n, 6] of templates first .. first + n - 1."""
    i = np.arange(first, first + n, dtype=np.uint64)
    key = np.empty((n, 2), np.uint64)
    key[:, 0] = np.uint64(seed & MASK32)
    key[:, 1] = np.uint64((seed >> 32) & MASK32)
    u = np.empty((n, 6))
    for j in range(3):
        ctr = np.empty((n, 4), np.uint64)
        ctr[:, 0] = i & np.uint64(MASK32)
        ctr[:, 1] = i >> np.uint64(32)
        ctr[:, 2] = 0
        ctr[:, 3] = 1 + j
        a, b = uniform_pair(philox4x32_10(ctr, key))
        u[:, 2 * j] = a
        u[:, 2 * j + 1] = b
    return u


def random_binary_bank(seed, first, n, f0_lo, f0_hi, ap_lo, ap_hi, omega_lo, omega_hi, alpha_lo=0.0,
                       alpha_hi=TWO_PI, sdec_lo=-1.0, sdec_hi=1.0, phib_lo=0.0, phib_hi=TWO_PI):
    """(f0, sky [n,3], ap, omega, phib) of templates first .. first + n - 1 of the
    region (right ascension, sin(declination) and phase limits default to the
    whole range)."""
    u = uniforms(seed, first, n)
    f0 = root(f0_lo, f0_hi, u[:, 0], 6)
    alpha = alpha_lo + u[:, 1] * (alpha_hi - alpha_lo)
    sd = sdec_lo + u[:, 2] * (sdec_hi - sdec_lo)
    cd = np.sqrt(1.0 - sd * sd)
    ca, sa = pcos(alpha)
    sky = np.stack([cd * ca, cd * sa, sd], axis=1)
    ap = root(ap_lo, ap_hi, u[:, 3], 3)
    omega = root(omega_lo, omega_hi, u[:, 4], 4)
    phib = phib_lo + u[:, 5] * (phib_hi - phib_lo)
    return f0, sky, ap, omega, phib


def boxes(seed, first, n, n_div):
    """Hyperbox of templates first .. first + n - 1 for a regular partition of the
    uniform-density coordinates into n_div[d] intervals per coordinate (Sec. IV.B):
    b_d = min(floor(n_div[d] u_d), n_div[d] - 1) from the uniform u_d each
    coordinate was drawn from, row-major with f0 slowest."""
    u = uniforms(seed, first, n)
    b = np.zeros(n, np.int64)
    for d in range(6):
        nd = int(n_div[d])
        bd = np.minimum(np.floor(np.float64(nd) * u[:, d]).astype(np.int64), nd - 1)
        b = b * nd + bd
    return b


def loudest_per_box(s, box, n_boxes):
    """(index, count, max) per box: the template with the largest s, ties to the
    lower index; index -1 and max 0 for an empty box."""
    s = np.asarray(s, np.float64)
    box = np.asarray(box, np.int64)
    order = np.lexsort((np.arange(s.size), -s, box))
    idx = np.full(n_boxes, -1, np.int64)
    best = np.zeros(n_boxes)
    count = np.bincount(box, minlength=n_boxes)
    first = np.ones(order.size, bool)
    first[1:] = box[order[1:]] != box[order[:-1]]
    winners = order[first]
    idx[box[winners]] = winners
    best[box[winners]] = s[winners]
    return idx, count, best
