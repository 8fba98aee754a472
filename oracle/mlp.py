"""FP64 reference of the detection-probability surrogate -- TEST INFRASTRUCTURE ONLY.

A multilayer perceptron 6 -> 256 -> 256 -> 256 -> 1 with GELU hidden activations
and a sigmoid output estimates p_det (Sec. V: the detection probability of
Eqs. pdet_abstract and sampling, as a function of the injection parameters),
trained with binary cross-entropy on detection labels and Adam.

Parameter vector (flat, this order): W1 [256, 6], b1 [256], W2 [256, 256], b2,
W3 [256, 256], b3, W4 [1, 256], b4 [1] -- 133,633 values.  Layer l computes
Z_l = A_{l-1} W_l^T + b_l.  GELU(x) = x Phi(x) with the normal CDF
Phi(x) = (1 + erf(x / sqrt 2)) / 2.  Inputs are the features
(log amp, cos iota, psi, sin delta, alpha, f) standardised by a fixed
(shift, scale) per feature.
"""
from __future__ import annotations

import math

import numpy as np

SIZES = [(256, 6), (256, 256), (256, 256), (1, 256)]
N_PARAMS = sum(o * i + o for o, i in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, off = [], 0
    for o, i in SIZES:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    assert off == N_PARAMS
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed):
    """He-style initialisation (normal, std sqrt(2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    return pack([(rng.standard_normal((o, i)) * math.sqrt(2.0 / i), np.zeros(o)) for o, i in SIZES])


_erf = np.vectorize(math.erf)


def gelu(x):
    return x * 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def features(raw, shift, scale):
    """raw [n, 6] = (amp, cos iota, psi, sin delta, alpha, f) -> standardised features."""
    raw = np.asarray(raw, np.float64)
    f = raw.copy()
    f[:, 0] = np.log(raw[:, 0])
    return (f - np.asarray(shift)) / np.asarray(scale)


def forward(theta, x):
    """Logits [n] and the cache for backward."""
    layers = unpack(theta)
    a = np.asarray(x, np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a[:, 0], cache


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def bce_loss(logit, y):
    """Mean binary cross-entropy of sigmoid(logit) against labels y in {0, 1}."""
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit)))))


def loss_and_grad(theta, x, y):
    logit, cache = forward(theta, x)
    n = logit.shape[0]
    y = np.asarray(y, np.float64)
    loss = bce_loss(logit, y)
    layers = unpack(theta)
    dz = ((sigmoid(logit) - y) / n)[:, None]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        a_prev, z = cache[li]
        W, _ = layers[li]
        if li < len(layers) - 1:
            dz = dz * gelu_grad(z)
        grads[li] = (dz.T @ a_prev, dz.sum(axis=0))
        dz = dz @ W
    return loss, pack(grads)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction, step t >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
