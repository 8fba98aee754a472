"""The surrogate's GPU kernels (BF16 matrix cores, FP32 accumulation) against
the FP64 oracle network: forward outputs, loss and the full gradient."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu

SHIFT = np.array([-3.5, 0.0, 0.0, 0.0, np.pi, 200.0])
SCALE = np.array([1.0, 0.58, 0.45, 0.58, 1.8, 58.0])


def _raw(rng, n):
    return np.stack([np.exp(rng.uniform(np.log(0.005), np.log(0.1), n)), rng.uniform(-1, 1, n),
                     rng.uniform(-np.pi / 4, np.pi / 4, n), rng.uniform(-1, 1, n),
                     rng.uniform(0, 2 * np.pi, n), rng.uniform(100, 300, n)], axis=1)


def test_forward_and_gradient_match_fp64(ft):
    import torch
    rng = np.random.default_rng(1)
    theta = ref.init_params(2).astype(np.float32)
    raw = _raw(rng, 200).astype(np.float32)
    y = (rng.uniform(size=200) < 0.4).astype(np.float32)
    x = ref.features(raw.astype(np.float64), SHIFT, SCALE)
    t64 = theta.astype(np.float64)
    logit, _ = ref.forward(t64, x)
    loss64, g64 = ref.loss_and_grad(t64, x, y.astype(np.float64))
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        net = ft.Mlp(c, SHIFT, SCALE, max_batch=256, params=theta)
        p = net.predict(raw)
        loss, g = net.loss_grad(raw, y)
        assert np.array_equal(net.params(), theta)
        net.close()
    assert np.max(np.abs(p - ref.sigmoid(logit))) < 0.02
    assert abs(loss - loss64) < 2e-2 * loss64
    rel = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    cos = float(np.dot(g, g64) / (np.linalg.norm(g) * np.linalg.norm(g64)))
    assert rel <= 2e-2 and cos >= 0.999, (rel, cos)
    # every layer's block individually
    off = 0
    for o, i in ref.SIZES:
        for n in (o * i, o):
            a, b = g[off:off + n], g64[off:off + n]
            if np.linalg.norm(b) > 0:
                assert np.linalg.norm(a - b) <= 5e-2 * np.linalg.norm(b), (off, n)
            off += n


def _check_grad(g, g64):
    rel = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    cos = float(np.dot(g, g64) / (np.linalg.norm(g) * np.linalg.norm(g64)))
    assert rel <= 2e-2 and cos >= 0.999, (rel, cos)
    off = 0
    for o, i in ref.SIZES:
        for n in (o * i, o):
            a, b = g[off:off + n], g64[off:off + n]
            if np.linalg.norm(b) > 0:
                assert np.linalg.norm(a - b) <= 5e-2 * np.linalg.norm(b), (off, n)
            off += n


@pytest.mark.parametrize("n", [2048, 1000, 64, 1])
def test_gradient_over_slices_and_chunks(ft, n):
    """Batches that split the weight-gradient products into 8 or 3 slices and
    the column sums into 32 or 16 chunks (ragged last chunk), one padded tile,
    and a single sample; two calls in a row reuse every scratch buffer."""
    import torch
    rng = np.random.default_rng(10 + n)
    theta = ref.init_params(4).astype(np.float32)
    raw = _raw(rng, n).astype(np.float32)
    y = (rng.uniform(size=n) < 0.4).astype(np.float32)
    x = ref.features(raw.astype(np.float64), SHIFT, SCALE)
    loss64, g64 = ref.loss_and_grad(theta.astype(np.float64), x, y.astype(np.float64))
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        net = ft.Mlp(c, SHIFT, SCALE, max_batch=2048, params=theta)
        loss_a, g_a = net.loss_grad(raw, y)
        loss_b, g_b = net.loss_grad(raw, y)
        net.close()
    assert np.array_equal(g_a, g_b) and loss_a == loss_b  # deterministic reductions
    assert abs(loss_a - loss64) < 2e-2 * loss64
    _check_grad(g_a, g64)


def test_one_adam_step_matches_oracle(ft):
    """One training step on one full batch (the epoch's permutation only
    reorders the batch): theta moves by the oracle's Adam update of the FP64
    gradient wherever that gradient is clearly resolved by the BF16 products."""
    import torch
    rng = np.random.default_rng(21)
    n, lr = 2048, 1e-3
    theta = ref.init_params(6).astype(np.float32)
    raw = _raw(rng, n).astype(np.float32)
    y = (rng.uniform(size=n) < 0.4).astype(np.float32)
    x = ref.features(raw.astype(np.float64), SHIFT, SCALE)
    t64 = theta.astype(np.float64)
    _, g64 = ref.loss_and_grad(t64, x, y.astype(np.float64))
    want, _, _ = ref.adam_step(t64, g64, np.zeros_like(t64), np.zeros_like(t64), 1, lr)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        net = ft.Mlp(c, SHIFT, SCALE, max_batch=n, params=theta)
        net.train(raw, y, batch=n, epochs=1, lr=lr, seed=3)
        got = net.params()
        net.close()
    # at t = 1 the update is lr g/(|g| + eps): every entry moves by at most lr
    assert np.all(np.abs(got.astype(np.float64) - t64) <= lr * (1 + 1e-5) + 1e-7)
    # resolved: at least a quarter of the rms of its own parameter block
    big = np.zeros(len(g64), bool)
    off = 0
    for o, i in ref.SIZES:
        for m in (o * i, o):
            b = g64[off:off + m]
            big[off:off + m] = np.abs(b) > 0.25 * np.sqrt(np.mean(b ** 2))
            off += m
    assert big.sum() > 0.3 * len(g64)
    err = np.abs(got.astype(np.float64) - want)[big]
    assert np.max(err) <= 1e-6 + 1e-6 * np.max(np.abs(t64)), np.max(err)


def test_training_learns_a_threshold_rule(ft):
    """Labels 1[log amp + 2 sin(delta) > -3.5]: GPU Adam training must reach
    well below the initial loss and classify held-out samples."""
    import torch
    rng = np.random.default_rng(3)
    raw = _raw(rng, 20000).astype(np.float32)
    rule = lambda r: (np.log(r[:, 0]) + 2.0 * r[:, 3] > -3.5).astype(np.float32)
    y = rule(raw)
    test = _raw(rng, 4000).astype(np.float32)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        net = ft.Mlp(c, SHIFT, SCALE, max_batch=1024, seed=5)
        hist = net.train(raw, y, batch=1024, epochs=12, lr=2e-3, seed=7)
        p = net.predict(test)
        net.close()
    assert hist[-1] < 0.5 * hist[0]
    acc = np.mean((p > 0.5) == (rule(test) > 0.5))
    assert acc > 0.95, acc


def test_invalid_inputs_rejected(ft):
    import torch
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        net = ft.Mlp(c, SHIFT, SCALE, max_batch=64, seed=1)
        bad = np.ones((4, 6), np.float32)
        bad[2, 0] = -1.0  # amplitude must be > 0
        with pytest.raises(ft.FtError) as e:
            net.predict(bad)
        assert e.value.status == ft.FT_E_INVALID
        with pytest.raises(ft.FtError):
            net.loss_grad(np.ones((4, 6), np.float32), np.array([0, 1, 2, 0], np.float32))
        net.close()
