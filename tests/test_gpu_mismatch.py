"""Mismatch distribution of random banks (Sec. IV.A, Eq. mismatch): every
trial's m recomputed by the oracle from the trial's recorded inputs (noise
seed, injection, box, bank seed, size), and the distribution's basic shape
(m concentrated in [0, 1], smaller at higher oversampling)."""
import numpy as np
import pytest

import oracle
from oracle import bank as obank
from oracle import inject
from paper_2411_18370_amd import mismatch, synth

pytestmark = pytest.mark.gpu


def test_mismatch_trials_match_oracle(ft):
    import torch
    w = synth.binary_band(seed=41, n_tmpl=1, n_per_det=150)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        res = mismatch.sample(c, w, o=2.0, n_trials=3, seed=5, amp=1.5)
    mu = 2.0 * w.n_sft
    for m, tr in zip(res["m"], res["trials"]):
        table = inject.generate_table(tr["noise_seed"], tr["run"], w.t_mid, w.t_ref, w.t_sft, w.v, w.arms,
                                      w.first_bin, w.n_bins, tr["inj"])
        inj = tr["inj"]
        one = lambda x: np.array([x], np.float64)
        s_sig, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v, one(inj["f0"]),
                                        np.asarray(inj["sky"])[None, :], one(inj["ap"]), one(inj["omega"]),
                                        one(inj["phib"]))
        assert bad == -1
        f0, sky, ap, om, pb = obank.random_binary_bank(tr["bank_seed"], 0, tr["n_bank"], **tr["box"])
        s_bank, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v, f0, sky, ap,
                                         om, pb)
        assert bad == -1
        best = int(np.argmax(s_bank))
        m_or = (s_sig[0] - s_bank[best]) / (s_sig[0] - mu)
        # the tables agree except for rare last-ulp differences of log/sin/cos
        assert abs(m - m_or) < 1e-6, (m, m_or)
        assert tr["best_index"] == best


def test_mismatch_distribution_shape(ft):
    import torch
    w = synth.binary_band(seed=42, n_tmpl=1, n_per_det=400)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        lo = mismatch.sample(c, w, o=0.5, n_trials=40, seed=6, amp=1.5)
        hi = mismatch.sample(c, w, o=8.0, n_trials=40, seed=7, amp=1.5)
    for r in (lo, hi):
        m = r["m"]
        assert np.all(m < 1.0) and np.mean((m >= -0.05) & (m <= 1.0)) > 0.95
    assert np.median(hi["m"]) < np.median(lo["m"])
    s = mismatch.summary(hi["m"])
    assert s["q05"] <= s["median"] <= s["q95"]
