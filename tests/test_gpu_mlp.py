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
