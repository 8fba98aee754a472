"""Host logic of the hyperbox search (Sec. IV.B, VI.A) and of the semi-analytic
estimate it uses (Sec. V): the box assignment of the oracle against its
definition, the estimate against its closed form, the selection rule and the
N_reject optimisation on constructed box maxima."""
import math

import numpy as np
from scipy import stats as sps

from oracle import bank as obank
from paper_2411_18370_amd import hyperbox, mismatch, sensitivity, synth


def test_oracle_boxes_follow_the_uniforms():
    n_div = (5, 3, 2, 4, 1, 3)
    u = obank.uniforms(17, 100, 4000)
    b = obank.boxes(17, 100, 4000, n_div)
    # decode the row-major index and compare with floor(n u) per coordinate
    rest = b.copy()
    for d in reversed(range(6)):
        bd = rest % n_div[d]
        rest //= n_div[d]
        assert np.array_equal(bd, np.minimum(np.floor(n_div[d] * u[:, d]), n_div[d] - 1).astype(np.int64))
    assert np.all(rest == 0)
    # equal coordinate volumes: counts are multinomial with equal cells
    counts = np.bincount(b, minlength=int(np.prod(n_div)))
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert sps.chi2.sf(chi2, counts.size - 1) > 1e-4
    # the f0 box is monotone in f0 (f0 is the slowest index)
    f0 = obank.random_binary_bank(17, 100, 4000, 100.0, 100.1, 5.0, 15.0, 4e-6, 1e-5)[0]
    b0 = b // int(np.prod(n_div[1:]))
    assert np.all(np.diff(b0[np.argsort(f0)]) >= 0)


def test_loudest_per_box_brute_force():
    rng = np.random.default_rng(3)
    s = rng.integers(0, 5, 300).astype(float)  # many ties
    box = rng.integers(0, 40, 300)
    idx, count, best = obank.loudest_per_box(s, box, 45)
    for b in range(45):
        members = np.flatnonzero(box == b)
        assert count[b] == members.size
        if members.size == 0:
            assert idx[b] == -1 and best[b] == 0
        else:
            top = s[members].max()
            assert best[b] == top and idx[b] == members[s[members] == top].min()


def test_p_det_matches_its_closed_form():
    """One q and one mismatch: p_det = P(N(mu, sd) > tau) in closed form."""
    n = 400_000
    q = np.tile([2000.0, 2.0 * math.sqrt(1000.0), 640.0, 640.0], (n, 1))
    m, tau = 0.1, 5.0
    for d in (10.0, 14.0, 20.0):
        lam = (1 - m) * sensitivity.BIN_OFFSET_POWER / d ** 2
        mu = lam * q[0, 2] / q[0, 1]
        sd = math.sqrt(q[0, 1] ** 2 + 4 * lam * q[0, 3]) / q[0, 1]
        want = sps.norm.sf(tau, mu, sd)
        got = sensitivity.p_det(q, [m], [d], tau, seed=5)[0]
        assert abs(got - want) < 5 * math.sqrt(want * (1 - want) / n) + 1e-4
    # D^p inverts p_det
    d95 = sensitivity.depth_at(q, [m], 0.95, tau, seed=6)
    lam = lambda d: (1 - m) * sensitivity.BIN_OFFSET_POWER / d ** 2
    p_at = sps.norm.sf(tau, lam(d95) * q[0, 2] / q[0, 1],
                       math.sqrt(q[0, 1] ** 2 + 4 * lam(d95) * q[0, 3]) / q[0, 1])
    assert abs(p_at - 0.95) < 0.003


def test_p_det_bounds_closed_forms():
    """Fixed q and each bank's k mismatches fixed: the lower bound is the
    one-template p_1 = P(N(mu_1, sd_1) > tau) and the upper bound is
    1 - prod_j (1 - p_j) for k independent templates; with k = 1 they agree."""
    n = 400_000
    q = np.tile([2000.0, 2.0 * math.sqrt(1000.0), 640.0, 640.0], (n, 1))
    tau = 5.0
    mk = np.array([[0.05, 0.2, 0.4, 0.9]])
    lam = lambda d, m: (1 - m) * sensitivity.BIN_OFFSET_POWER / d ** 2
    for d in (10.0, 14.0, 20.0):
        p = [sps.norm.sf(tau, lam(d, m) * q[0, 2] / q[0, 1],
                         math.sqrt(q[0, 1] ** 2 + 4 * lam(d, m) * q[0, 3]) / q[0, 1]) for m in mk[0]]
        want_hi = 1 - np.prod([1 - x for x in p])
        lo, hi = sensitivity.p_det_bounds(q, mk, [d], tau, seed=7)
        se = lambda x: 5 * math.sqrt(x * (1 - x) / n) + 1e-4
        assert abs(lo[0] - p[0]) < se(p[0]) and abs(hi[0] - want_hi) < se(want_hi)
        lo1, hi1 = sensitivity.p_det_bounds(q, mk[:, :1], [d], tau, seed=7)
        assert lo1[0] == hi1[0]
    # monotone in depth on common draws
    lo, hi = sensitivity.p_det_bounds(q[:20000], mk, [8.0, 12.0, 16.0, 24.0], tau, seed=8)
    assert np.all(np.diff(lo) <= 0) and np.all(np.diff(hi) <= 0) and np.all(lo <= hi)


def test_thresholds_rule():
    z = np.array([3.0, 9.0, np.nan, 5.0, 9.0, 1.0])
    thr = hyperbox.thresholds(z, n_cand=2, n_reject=1)
    # order: box 1 (9), box 4 (9, later index), box 3 (5), box 0, box 5, box 2 (empty)
    assert thr[1] == np.inf                       # rejected
    assert thr[4] == 9.0 and thr[3] == 5.0        # selected: their own z
    assert thr[0] == 5.0 and thr[5] == 5.0 and thr[2] == 5.0  # the last selected z
    assert np.all(hyperbox.thresholds(z, 0, 0) == np.inf)
    assert np.array_equal(hyperbox.thresholds(z, 10, 0)[[0, 1, 3, 4, 5]], z[[0, 1, 3, 4, 5]])


def test_box_z_marks_empty_boxes():
    res = np.zeros(4, dtype=[("index", np.int64), ("z", np.float64)])
    res["index"] = [3, -1, 7, -1]
    res["z"] = [1.5, 0.0, -0.5, 0.0]
    z = hyperbox.box_z(res)
    assert z[0] == 1.5 and z[2] == -0.5 and np.isnan(z[1]) and np.isnan(z[3])


def test_optimizer_rejects_the_outlier_boxes():
    """30 boxes on an artifact outnumber the 20 candidates: without rejection they
    set every threshold; rejecting them restores the sensitivity, and rejecting
    15% of the boxes cannot reach 95% detection at all."""
    rng = np.random.default_rng(8)
    n_boxes = 2000
    # maxima of ~1e4 Gaussian templates per box, plus 30 boxes on an artifact
    z = sps.norm.isf(rng.uniform(0, 1, n_boxes) / 1e4)
    z[rng.choice(n_boxes, 30, replace=False)] = 60.0
    # 1000 SFTs of 1800 s: rho1 = rho2 ~ N T <F^2 A^2> at unit amplitude
    q = np.tile([2000.0, 2.0 * math.sqrt(1000.0), 2.9e5, 2.9e5], (20_000, 1))
    best, table = hyperbox.optimize_reject(q, [0.05], z, n_cand=20, rejects=[0, 10, 30, 45, 300], seed=1)
    d = dict(table)
    assert best >= 30
    assert d[best] > 1.5 * d[0]
    assert d[300] == 1.0 and d[best] > 10


def test_partition_sizes():
    w = synth.binary_band(seed=3, n_tmpl=10, n_per_det=200)
    t_obs = float(w.t_mid.max() - w.t_mid.min() + w.t_sft)
    vmax = float(np.max(np.linalg.norm(w.v, axis=1)))
    region = dict(w.region)
    region.update(alpha_lo=0.0, alpha_hi=2 * math.pi, sdec_lo=-1.0, sdec_hi=1.0, phib_lo=0.0,
                  phib_hi=2 * math.pi)
    n_bank = 3.44 * mismatch.n_templates(region, w.t_sft, t_obs, vmax)
    for per_box in (1e4, 1e6):
        n_div = hyperbox.partition(region, w.t_sft, t_obs, vmax, 3.44, per_box)
        boxes = int(np.prod(n_div))
        assert all(d >= 1 for d in n_div)
        assert 0.5 * n_bank / per_box <= boxes <= 2.5 * n_bank / per_box
    n_div = hyperbox.partition(region, w.t_sft, t_obs, vmax, 3.44, n_bank, min_boxes=10_000)
    assert int(np.prod(n_div)) >= 10_000
