"""Loudest template per hyperbox of a random binary bank (Sec. IV.B) on the GPU
against the oracle: box assignment from the generator's uniforms, counts, the
exact FP64 box maxima and their indices (ties to the lower index), for the
power and the number-count statistic, with empty boxes and a candidate pass
that has to grow; argument errors."""
import numpy as np
import pytest

import oracle
from oracle import bank as obank
from oracle import weighting as ow
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _setup(ft, b):
    import torch
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    c.set_sfts(b.n_sft_per_det, b.t_mid, b.t_sft, b.first_bin, b.power)
    c.set_velocities(b.v)
    return c


def _region(b):
    return dict(b.region, alpha_lo=0.0, alpha_hi=2 * np.pi, sdec_lo=-1.0, sdec_hi=1.0, phib_lo=0.0,
                phib_hi=2 * np.pi)


@pytest.mark.parametrize("n_div,statistic", [((4, 3, 2, 2, 2, 3), 0), ((4, 3, 2, 2, 2, 3), 1),
                                             ((10, 8, 5, 4, 4, 4), 0), ((1, 1, 1, 1, 1, 1), 0),
                                             ((7, 1, 1, 1, 1, 1), 1)])
def test_loudest_per_box_matches_oracle(ft, n_div, statistic):
    import torch
    b = synth.binary_band(seed=21, n_tmpl=1, n_per_det=150)
    reg = _region(b)
    n, seed = 20_000, 77
    f0, sky, ap, om, pb = obank.random_binary_bank(seed, 0, n, **reg)
    table = b.power if statistic == 0 else ow.number_count_table(b.power)
    s64, bad = oracle.eval_binary(b.t_mid, b.t_ref, b.t_sft, b.first_bin, table, None, b.v, f0, sky, ap, om, pb)
    assert bad == -1
    n_boxes = int(np.prod(n_div))
    box = obank.boxes(seed, 0, n, n_div)
    idx, count, best = obank.loudest_per_box(s64, box, n_boxes)
    N = b.t_mid.size
    mu, sig = ((2.0 * N, 2.0 * np.sqrt(N)) if statistic == 0 else ow.nc_moments(np.ones(N)))
    c = _setup(ft, b)
    try:
        stats = torch.empty(n, dtype=torch.float32, device="cuda:0")
        res = c.eval_binary_boxes(reg, seed, n, b.t_ref, n_div, statistic=statistic, stats=stats)
        s32 = stats.cpu().numpy().astype(np.float64)
    finally:
        c.close()
    assert res.shape == (n_boxes,)
    assert np.array_equal(res["count"], count)
    assert np.array_equal(res["index"], idx)
    full = count > 0
    assert np.array_equal(res["s64"][full], best[full])
    assert np.all(res["s64"][~full] == 0) and np.all(res["index"][~full] == -1)
    assert np.array_equal(res["s32"][full], s32[idx[full]].astype(np.float32))
    assert np.allclose(res["z"][full], (best[full] - mu) / sig, rtol=1e-12, atol=1e-12)
    bound = 40 * 2.0 ** -24 + 4 * N * 2.0 ** -53
    assert np.all(np.abs(s32 - s64) <= bound * s64)
    if n_boxes > n:
        assert (~full).sum() > 0


def test_many_candidates_grow_the_buffer(ft):
    """An all-zero table ties every template of the one box at S = 0: all of
    them are candidates (beyond the first buffer) and the lowest index wins."""
    import torch
    b = synth.binary_band(seed=22, n_tmpl=1, n_per_det=20)
    reg = _region(b)
    n, seed = 150_000, 5
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    try:
        c.set_sfts(b.n_sft_per_det, b.t_mid, b.t_sft, b.first_bin, np.zeros_like(b.power))
        c.set_velocities(b.v)
        res = c.eval_binary_boxes(reg, seed, n, b.t_ref, (1, 1, 1, 1, 1, 1))
    finally:
        c.close()
    assert res["index"][0] == 0 and res["s64"][0] == 0.0 and res["count"][0] == n


def test_box_errors(ft):
    b = synth.binary_band(seed=23, n_tmpl=1, n_per_det=20)
    reg = _region(b)
    c = _setup(ft, b)
    try:
        for bad in ((0, 1, 1, 1, 1, 1), (1 << 21, 1, 1, 1, 1, 1), (1024, 1024, 128, 1, 1, 1)):
            with pytest.raises(ft.FtError, match="FT_E_INVALID"):
                c.eval_binary_boxes(reg, 1, 100, b.t_ref, bad)
        with pytest.raises(ft.FtError, match="FT_E_INVALID"):
            c.eval_binary_boxes(reg, 1, 100, b.t_ref, (2, 1, 1, 1, 1, 1), statistic=5)
    finally:
        c.close()


def test_box_search_at_benchmark_size(ft):
    """The bench's box search: 10^8 templates (o = 3.44, full sky and phase) in at
    least 10^4 boxes, 2 x 5000 SFTs.  The oracle cannot enumerate every box at this
    size, so it checks sampled boxes and templates one by one: each winner lies in
    its box and its S64 is the oracle's bit for bit; every sampled template's S64 is
    at most its box's maximum (and not a lower-index tie); counts add up to n."""
    from paper_2411_18370_amd import hyperbox, mismatch
    b = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    t_obs = float(b.t_mid.max() - b.t_mid.min() + b.t_sft)
    vmax = float(np.max(np.linalg.norm(b.v, axis=1)))
    reg = _region(b)
    per_f06 = mismatch.n_templates(reg, b.t_sft, t_obs, vmax) / (reg["f0_hi"] ** 6 - reg["f0_lo"] ** 6)
    n, o, seed = 10 ** 8, 3.44, 7
    reg["f0_hi"] = (reg["f0_lo"] ** 6 + n / (o * per_f06)) ** (1.0 / 6.0)
    n_div = hyperbox.partition(reg, b.t_sft, t_obs, vmax, o, n / 10_000, min_boxes=10_000)
    n_boxes = int(np.prod(n_div))
    c = _setup(ft, b)
    try:
        res = c.eval_binary_boxes(reg, seed, n, b.t_ref, n_div)
    finally:
        c.close()
    assert n_boxes >= 10_000 and int(res["count"].sum()) == n
    rng = np.random.default_rng(4)
    boxes = rng.choice(np.flatnonzero(res["index"] >= 0), 600, replace=False)
    winners = res["index"][boxes]
    samples = rng.choice(n, 1500, replace=False)
    idx = np.concatenate([winners, samples])
    par = [np.concatenate(x) for x in zip(*[obank.random_binary_bank(seed, int(i), 1, **reg) for i in idx])]
    s64, bad = oracle.eval_binary(b.t_mid, b.t_ref, b.t_sft, b.first_bin, b.power, None, b.v, par[0],
                                  par[1].reshape(-1, 3), par[2], par[3], par[4])
    assert bad == -1
    box_of = np.array([obank.boxes(seed, int(i), 1, n_div)[0] for i in idx])
    assert np.array_equal(box_of[:len(boxes)], boxes)
    assert np.array_equal(s64[:len(boxes)], res["s64"][boxes])
    N = b.t_mid.size
    assert np.allclose(res["z"][boxes], (res["s64"][boxes] - 2.0 * N) / (2.0 * np.sqrt(N)), rtol=1e-12, atol=1e-12)
    for q in range(len(boxes), idx.size):
        bx, t = box_of[q], idx[q]
        top, win = res["s64"][bx], res["index"][bx]
        assert s64[q] < top or (s64[q] == top and t >= win)
