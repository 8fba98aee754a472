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


def test_semi_analytic_p_det_matches_injections(ft):
    """p_det at four depths from the estimate (10^4 population samples, p(m|o)
    from 60 high-SNR trials) against 120 plain injections per depth, both at
    oversampling 3.44 with the rule z > 6: agreement within four binomial
    standard errors plus 0.03."""
    import torch
    w = synth.binary_band(seed=53, n_tmpl=1, n_per_det=400)
    o, tau = 3.44, 6.0
    depths = np.array([7.0, 13.0, 17.0, 26.0])
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        m = mismatch.sample(c, w, o=o, n_trials=60, seed=8, amp=1.5)["m"]
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
        q = sensitivity.q_samples(c, w.arms, 10_000, seed=9)
        p_sa = sensitivity.p_det(q, m, depths, tau, seed=10)
        p_inj = sensitivity.injection_p_det(c, w, depths, 120, o, tau, seed=11)
    print("semi-analytic", p_sa, "injections", p_inj, flush=True)
    assert p_sa[0] > 0.9 and p_sa[-1] < 0.3
    assert np.all(np.diff(p_sa) <= 0) and np.all(np.diff(p_inj) <= 0.05)
    # the estimate treats the loudest of ~10^4 bank templates as one template at
    # mismatch m; near threshold the loudest also collects positive noise, so
    # injections may be detected somewhat more often (a known approximation)
    for a, b in zip(p_sa, p_inj):
        se = np.sqrt(max(a * (1 - a), 0.02) / 120)
        assert abs(a - b) <= 4 * se + 0.03, (p_sa, p_inj)
