"""The grid kernel's whole-tile certificate against the oracle's canonical bins.

Per (sky point, SFT, f1 value) and f0 tile of n_in templates the stage
preparation forms, in FP64 and in this order,
    g = 1 + ((vx nx + vy ny) + vz nz),  G = g T_sft,  c = f1 (t - t_ref),
    e = dT g - 1,  x0 = (c G + 1/2) + f0min G,  B0 = floor(x0),  u0 = x0 - B0,
and certifies the step when u0 + min(0, (n_in - 1) e) >= eta and
u0 + max(0, (n_in - 1) e) < 1 - eta, eta being the host's bound
    eta = 2 (2 rho + 2 tau (1 + vmax) T + 2^-40),  rho = 6 2^-53 x_max,
with tau the grid's deviation from uniform spacing.  It then reads template m
of the tile at bin B0 + m.  Here that arithmetic is replayed over every SFT,
f1 value and f0 tile of a few sky points, and wherever the certificate holds
every template's bin from the oracle must be B0 + m.  A certificate that drops
the drift term (checks the first template only) must fail the same test, so
the comparison can tell."""
import numpy as np
import pytest

import oracle
from paper_2411_18370_amd import synth

TILE = 64 * 5  # f0 values of an L5 tile


def host_eta(w):
    T = w.t_sft
    f0 = w.f0
    n0 = f0.size
    dT = (f0[-1] - f0[0]) / (n0 - 1) * T
    tau = np.max(np.abs(f0 - f0[0] - np.arange(n0) * (dT / T))) + 8.0 * 2.0 ** -52 * f0[-1]
    vmax = np.max(np.sqrt(np.sum(w.v * w.v, axis=1)))
    dt = w.t_mid - w.t_ref
    cs = [w.f1.min() * dt.min(), w.f1.min() * dt.max(), w.f1.max() * dt.min(), w.f1.max() * dt.max()]
    x_max = (f0[-1] + max(cs)) * (1.0 + vmax) * T
    rho = 6.0 * 2.0 ** -53 * x_max
    return dT, 2.0 * (2.0 * rho + 2.0 * tau * (1.0 + vmax) * T + 2.0 ** -40)


def check(w, sky_idx, drift_term=True):
    """(certified steps, steps, certified steps with a wrong bin)."""
    T = w.t_sft
    dT, eta = host_eta(w)
    dt = w.t_mid - w.t_ref
    n_cert = n_all = n_wrong = 0
    for s in sky_idx:
        n = w.sky[s]
        g = 1.0 + ((w.v[:, 0] * n[0] + w.v[:, 1] * n[1]) + w.v[:, 2] * n[2])
        G = g * T
        e = dT * g - 1.0
        for i0 in range(0, w.f0.size, TILE):
            f0 = w.f0[i0:i0 + TILE]
            n_in = f0.size
            span = (n_in - 1) * e if drift_term else 0.0 * e
            for f1 in w.f1:
                c = f1 * dt
                x0 = (c * G + 0.5) + f0[0] * G
                b0 = np.floor(x0)
                u0 = x0 - b0
                ok = (u0 + np.minimum(0.0, span) >= eta) & (u0 + np.maximum(0.0, span) < 1.0 - eta)
                bins = oracle.bins_list(w.t_mid, w.t_ref, T, w.v, f0, np.full(n_in, f1),
                                        np.repeat(n[None, :], n_in, axis=0))  # [n_in, n_sft]
                want = b0[None, :].astype(np.int64) + np.arange(n_in)[:, None]
                wrong = np.any(bins != want, axis=0)
                n_cert += int(ok.sum())
                n_all += ok.size
                n_wrong += int((ok & wrong).sum())
    return n_cert, n_all, n_wrong


@pytest.mark.parametrize("band", ["allsky_200Hz", "precision_1kHz"])
def test_certified_steps_have_the_canonical_bins(band):
    if band == "allsky_200Hz":
        w = synth.allsky_band(seed=2, n_sky=64, n_per_det=1500)
    else:
        w = synth.precision_stress(seed=2, n_sky=64, n_per_det=1500)
    n_cert, n_all, n_wrong = check(w, [0, 21, 42, 63])
    print(band, "certified %d of %d steps, %d with a wrong bin" % (n_cert, n_all, n_wrong))
    assert n_wrong == 0
    # the certificate is not vacuous: most steps are whole-wave
    assert n_cert > 0.8 * n_all


def test_certificate_without_the_drift_term_fails():
    w = synth.allsky_band(seed=2, n_sky=64, n_per_det=1500)
    _, _, n_wrong = check(w, [0, 21], drift_term=False)
    assert n_wrong > 0
