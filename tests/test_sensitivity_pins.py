"""Pins of the semi-analytic sensitivity estimate's ingredients (Sec. V): the
oracle's signal-response quantities against their closed forms, and the
bin-offset power factor against its integral."""
import numpy as np
from scipy.integrate import quad

from oracle import sensitivity as osens
from paper_2411_18370_amd import sensitivity, synth


def test_bin_offset_power_is_the_mean_of_sinc2():
    v, _ = quad(lambda x: np.sinc(x) ** 2, -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)
    assert abs(sensitivity.BIN_OFFSET_POWER - v) < 1e-12
    # the paper's 0.7737 is this number
    assert abs(v - 0.7737) < 1e-4


def test_q_closed_forms():
    """Isotropic sky, cos iota U[-1,1], psi uniform: <F+^2> = <Fx^2> = 1/5,
    <A+^2> = 7/15, <Ax^2> = 1/3, so <rho_k> = T (7/75 + 5/75) = 4 T/25 for any
    SFT; mu_G = 2 N and sigma_G = 2 sqrt(N) without weights, and the weighted
    sums follow the weights."""
    w = synth.binary_band(seed=51, n_tmpl=1, n_per_det=5)
    rng = np.random.default_rng(3)
    n = 40_000
    sky, ci, psi = sensitivity.population(rng, n)
    q = osens.q_sample(w.t_sft, w.arms, None, sky, ci, psi)
    N = w.n_sft
    assert np.all(q[:, 0] == 2.0 * N) and np.allclose(q[:, 1], 2.0 * np.sqrt(N), rtol=0, atol=1e-12)
    mean_rho = q[:, 2].mean() / (N * w.t_sft)
    se = q[:, 2].std() / (N * w.t_sft) / np.sqrt(n)
    assert abs(mean_rho - 4.0 / 25.0) < 4 * se
    # rho2 = rho1 without weights; with weights u the sums follow u and u^2
    assert np.allclose(q[:, 3], q[:, 2], rtol=1e-14)
    u = np.linspace(0.5, 1.5, N).astype(np.float32)
    qw = osens.q_sample(w.t_sft, w.arms, u, sky[:50], ci[:50], psi[:50])
    uu = u.astype(np.float64)
    assert np.allclose(qw[:, 0], 2 * uu.sum()) and np.allclose(qw[:, 1], 2 * np.sqrt((uu * uu).sum()))
    # one SFT: rho1 = u rho_k and rho2 = u^2 rho_k, so rho2 / rho1 = u
    u1 = np.array([0.7], np.float32)
    q1 = osens.q_sample(w.t_sft, w.arms[:1], u1, sky[:20], ci[:20], psi[:20])
    q0 = osens.q_sample(w.t_sft, w.arms[:1], None, sky[:20], ci[:20], psi[:20])
    assert np.allclose(q1[:, 2], float(u1[0]) * q0[:, 2], rtol=1e-15)
    assert np.allclose(q1[:, 3], float(u1[0]) ** 2 * q0[:, 2], rtol=1e-15)
