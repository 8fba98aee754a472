"""Semi-analytic sensitivity estimate on the GPU (Sec. V): the signal-response
quantities against the oracle, and the estimated p_det against plain
injections with the same detection rule (the comparison of Sec. VI)."""
import numpy as np
import pytest

from oracle import sensitivity as osens
from paper_2411_18370_amd import mismatch, sensitivity, synth

pytestmark = pytest.mark.gpu


def test_q_samples_match_oracle(ft):
    import torch
    w = synth.binary_band(seed=52, n_tmpl=1, n_per_det=300)
    rng = np.random.default_rng(4)
    sky, ci, psi = sensitivity.population(rng, 500)
    u = rng.uniform(0.2, 2.0, w.n_sft).astype(np.float32)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
        got = c.q_sample(w.arms, sky, ci, psi)
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power, u)
        got_w = c.q_sample(w.arms, sky, ci, psi)
        with pytest.raises(ft.FtError):
            c.q_sample(w.arms, sky * 2.0, ci, psi)
    want = osens.q_sample(w.t_sft, w.arms, None, sky, ci, psi)
    want_w = osens.q_sample(w.t_sft, w.arms, u, sky, ci, psi)
    # one fixed sequence of IEEE operations on both sides (the project's cosine
    # and sine for the polarisation angle, dot products in one order)
    assert np.array_equal(got, want)
    assert np.array_equal(got_w, want_w)


def test_semi_analytic_p_det_brackets_injections(ft):
    """p_det at four depths from the estimate (10^4 population samples, the 16
    smallest mismatches of each of 60 high-SNR random banks) against 500 plain
    injections per depth, both at oversampling 3.44 with the rule z > 6.  The
    injections' detected fraction lies within three standard errors (binomial
    at 500 injections, combined with the estimate's Monte Carlo error) of the
    band from the one-template lower bound to the independent-noise upper
    bound of the loudest of the bank."""
    import torch
    w = synth.binary_band(seed=53, n_tmpl=1, n_per_det=400)
    o, tau, n_inj, n_q = 3.44, 6.0, 500, 10_000
    depths = np.array([7.0, 13.0, 17.0, 26.0])
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        m_k = mismatch.sample(c, w, o=o, n_trials=60, seed=8, amp=1.5, k_best=16)["m_k"]
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
        q = sensitivity.q_samples(c, w.arms, n_q, seed=9)
        p_lo, p_hi = sensitivity.p_det_bounds(q, m_k, depths, tau, seed=10)
        p_inj = sensitivity.injection_p_det(c, w, depths, n_inj, o, tau, seed=11)
    print("lower", p_lo, "upper", p_hi, "injections", p_inj, flush=True)
    assert np.all(np.diff(m_k, axis=1) >= 0)
    assert p_lo[0] > 0.9 and p_hi[-1] < 0.3
    assert np.all(p_lo <= p_hi)
    assert np.all(np.diff(p_lo) <= 0) and np.all(np.diff(p_hi) <= 0)
    for a, b, x in zip(p_lo, p_hi, p_inj):
        se_a = np.sqrt(max(a * (1 - a), 1.0 / n_inj) * (1.0 / n_inj + 1.0 / n_q))
        se_b = np.sqrt(max(b * (1 - b), 1.0 / n_inj) * (1.0 / n_inj + 1.0 / n_q))
        assert a - 3 * se_a <= x <= b + 3 * se_b, (p_lo, p_hi, p_inj)
