"""FP64 reference of the injection-campaign data generator -- TEST INFRASTRUCTURE ONLY.

Generates the normalised power of one run's SFT table: circular complex Gaussian
noise plus, optionally, one continuous-wave signal, following the signal
hypothesis of Sec. II.B.2:

* noise: Re, Im ~ N(0, 1) per (SFT k, bin b) (so P ~ chi^2_2, Eq. s_chi2), drawn
  from the counter-based generator Philox-4x32-10 (Salmon, Moraes, Dror and Shaw,
  SC'11) with counter (b, k, run, 0) and key (seed_lo, seed_hi); two 53-bit
  uniforms per call feed the Box-Muller transform (Box and Muller 1958);
* signal: in SFT k the track sits at x_k = (f0 + f1 dt_k)(1 + v_k.n) T_sft bins
  (Eq. track with a_p = 0), or for a source in a circular binary orbit at
  x_k = (f0 + f1 dt_k)(1 + v_k.n - a_p Omega cos(Omega dt_k - phi_b)) T_sft
  (Eq. track), B_k = floor(x_k + 1/2), delta_k = x_k - B_k.  Its
  power non-centrality is rho_k^2 = T_sft (h0^2/S_n) (F+^2 A+^2 + Fx^2 Ax^2),
  A+ = (1 + cos^2 iota)/2, Ax = cos iota -- rho^2 = 4|h~|^2/(T S_n) with
  |h~| = (T/2) h0 |F+ A+ + i Fx Ax| (the two polarisations in quadrature); the
  bin-offset loss of the paper's 0.7737 factor is modelled explicitly: bin
  B_k + m, m in {-1, 0, 1}, receives amplitude sqrt(rho_k^2) |sinc(pi(delta_k - m))|
  added to Re;
* antenna patterns F+ = D:e+, Fx = D:ex with detector tensor D = (u u^T - w w^T)/2
  (arm unit vectors u, w at the SFT mid-time) and polarisation tensors
  e+ = p p^T - q q^T, ex = p q^T + q p^T, (p, q) = (e_alpha, e_delta) rotated by
  psi: p = cos psi e_alpha + sin psi e_delta, q = -sin psi e_alpha + cos psi e_delta.

Every transcendental function is one of the project's fixed sequences of IEEE
operations (the logarithm core.plog, the cosine and sine core.pcos; square roots
and divisions are correctly rounded), and every dot product is summed in the
order (x0 y0 + x1 y1) + x2 y2, so any implementation of this specification
produces the same bits.  The GPU generator implements it independently.

Two implementations of the noise live here: noise_normals (Philox in numpy)
and the C generator behind generate_table (core.gen_table); tests check that
they agree bit for bit.
"""
from __future__ import annotations

import numpy as np

from . import core
from .core import pcos

M0, M1 = 0xD2511F53, 0xCD9E8D57     # Philox-4x32 round multipliers
W0, W1 = 0x9E3779B9, 0xBB67AE85     # Weyl key increments
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox-4x32 with 10 rounds.  ctr: uint64 array [..., 4] of 32-bit words,
    key: [..., 2].  Returns uint64 array [..., 4] of 32-bit words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK32 for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK32
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK32)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK32)
    return np.stack(c, axis=-1)


def uniform_pair(words):
    """Two uniforms in (0, 1) from four 32-bit words: the top 53 bits of each
    64-bit half, centred: (m + 1/2) 2^-53."""
    w = np.asarray(words, dtype=np.uint64)
    m1 = ((w[..., 0] << np.uint64(32)) | w[..., 1]) >> np.uint64(11)
    m2 = ((w[..., 2] << np.uint64(32)) | w[..., 3]) >> np.uint64(11)
    u1 = (m1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (m2.astype(np.float64) + 0.5) * 2.0 ** -53
    return u1, u2


def box_muller(u1, u2):
    u1 = np.asarray(u1, np.float64)
    r = np.sqrt(-2.0 * core.plog(u1).reshape(u1.shape))
    th = 2.0 * np.pi * np.asarray(u2, np.float64)
    c, s = pcos(th)
    return r * c.reshape(th.shape), r * s.reshape(th.shape)


def noise_normals(seed, run, n_sft, n_bins, sft_offset=0):
    """(Re, Im) [n_sft, n_bins] of run `run`; SFT k uses counter word k + sft_offset."""
    b = np.arange(n_bins, dtype=np.uint64)[None, :]
    k = (np.arange(n_sft, dtype=np.uint64) + np.uint64(sft_offset))[:, None]
    ctr = np.empty((n_sft, n_bins, 4), np.uint64)
    ctr[..., 0] = b
    ctr[..., 1] = k
    ctr[..., 2] = np.uint64(run & MASK32)
    ctr[..., 3] = 0
    key = np.empty((n_sft, n_bins, 2), np.uint64)
    key[..., 0] = np.uint64(seed & MASK32)
    key[..., 1] = np.uint64((seed >> 32) & MASK32)
    u1, u2 = uniform_pair(philox4x32_10(ctr, key))
    return box_muller(u1, u2)


def wave_frame(n, psi):
    """Polarisation basis (p, q) of a source in direction n rotated by psi."""
    n = np.asarray(n, np.float64)
    rho = np.sqrt(n[0] * n[0] + n[1] * n[1])
    if rho > 0:
        ea = np.array([-n[1] / rho, n[0] / rho, 0.0])
        ed = np.array([-n[2] * n[0] / rho, -n[2] * n[1] / rho, rho])
    else:  # at a pole: right ascension 0
        ea = np.array([0.0, 1.0, 0.0])
        ed = np.array([-n[2], 0.0, 0.0])
    c, s = pcos(np.array([psi], np.float64))
    cp, sp = float(c[0]), float(s[0])
    return cp * ea + sp * ed, -sp * ea + cp * ed


def dot3(a, b):
    """(a0 b0 + a1 b1) + a2 b2 along the last axis (the canonical order)."""
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def antenna_patterns(arms, n, psi):
    """F+, Fx [N] for arm unit vectors arms [N, 6] = (u, w) and source n, psi."""
    p, q = wave_frame(n, psi)
    u, w = arms[:, :3], arms[:, 3:]
    up, uq, wp, wq = dot3(u, p), dot3(u, q), dot3(w, p), dot3(w, q)
    fp = 0.5 * ((up * up - uq * uq) - (wp * wp - wq * wq))
    fx = up * uq - wp * wq
    return fp, fx


def track_bins(t_mid, t_ref, t_sft, v, n, f0, f1, ap=0.0, omega=0.0, phib=0.0):
    """(x_k, B_k): exact FP64 track position in bins and its nearest bin.  With
    ap > 0 the source is in a circular binary orbit (Eq. track): the Doppler
    factor g becomes g - (ap omega) cos(omega dt - phib), cos the library cosine
    of the oracle (core.pcos)."""
    d = (v[:, 0] * n[0] + v[:, 1] * n[1]) + v[:, 2] * n[2]
    g = 1.0 + d
    dt = t_mid - t_ref
    h = g
    if ap > 0.0:
        ph = omega * dt
        ph = ph - phib
        cb, _ = pcos(ph)
        h = g - (ap * omega) * cb
    x = ((f0 + f1 * dt) * h) * t_sft
    return x, np.floor(x + 0.5)


def rho2(arms, n, psi, cos_iota, amp, t_sft):
    """Per-SFT power non-centrality T_sft amp^2 (F+^2 A+^2 + Fx^2 Ax^2), amp = h0/sqrt(S_n)."""
    fp, fx = antenna_patterns(arms, n, psi)
    ap = 0.5 * (1.0 + cos_iota * cos_iota)
    ax = cos_iota
    return t_sft * amp * amp * (fp * fp * ap * ap + fx * fx * ax * ax)


def sinc(y):
    """sin(y)/y (1 at 0) with the project sine."""
    y = np.asarray(y, np.float64)
    out = np.ones_like(y)
    nz = y != 0
    _, s = pcos(y[nz])
    out[nz] = s / y[nz]
    return out


def signal_amplitudes(t_mid, t_ref, t_sft, v, arms, inj):
    """(B_k, A [N, 3]) -- amplitude added to Re at bins B_k - 1, B_k, B_k + 1."""
    n = np.asarray(inj["sky"], np.float64)
    x, B = track_bins(t_mid, t_ref, t_sft, v, n, inj["f0"], inj.get("f1", 0.0), inj.get("ap", 0.0),
                      inj.get("omega", 0.0), inj.get("phib", 0.0))
    delta = x - B
    r2 = rho2(arms, n, inj["psi"], inj["cos_iota"], inj["amp"], t_sft)
    A = np.stack([np.sqrt(r2) * np.abs(sinc(np.pi * (delta - m))) for m in (-1, 0, 1)], axis=1)
    return B.astype(np.int64), A


def generate_table(seed, run, t_mid, t_ref, t_sft, v, arms, first_bin, n_bins, inj=None,
                   sft_offset=0):
    """FP32 power table [N, n_bins] of one run: noise plus the signals of `inj`
    (None, one dict or a list of dicts).  Signals superpose linearly in the SFT
    amplitude (the strain is a sum of the sources' strains), so each adds its
    leakage amplitudes to Re, in the order given."""
    n_sft = len(t_mid)
    injs = [] if inj is None else [inj] if isinstance(inj, dict) else list(inj)
    bins, amps = [], []
    for one in injs:
        if one.get("amp", 0.0) == 0.0:
            continue
        B, A = signal_amplitudes(np.asarray(t_mid, np.float64), t_ref, t_sft,
                                 np.asarray(v, np.float64), np.asarray(arms, np.float64), one)
        bins.append(B)
        amps.append(A)
    bins = np.array(bins, np.int64).reshape(-1, n_sft)
    amps = np.array(amps, np.float64).reshape(-1, n_sft, 3)
    return core.gen_table(seed, run, n_sft, n_bins, sft_offset, first_bin, bins, amps)


def generate_table_numpy(seed, run, t_mid, t_ref, t_sft, v, arms, first_bin, n_bins, inj=None,
                         sft_offset=0):
    """generate_table through noise_normals (Philox in numpy): the second implementation."""
    n_sft = len(t_mid)
    re, im = noise_normals(seed, run, n_sft, n_bins, sft_offset)
    injs = [] if inj is None else [inj] if isinstance(inj, dict) else list(inj)
    for one in injs:
        if one.get("amp", 0.0) == 0.0:
            continue
        B, A = signal_amplitudes(np.asarray(t_mid, np.float64), t_ref, t_sft,
                                 np.asarray(v, np.float64), np.asarray(arms, np.float64), one)
        for k in range(n_sft):
            for j, m in enumerate((-1, 0, 1)):
                col = B[k] + m - first_bin
                if 0 <= col < n_bins:
                    re[k, col] = re[k, col] + A[k, j]
    return (re * re + im * im).astype(np.float32)
