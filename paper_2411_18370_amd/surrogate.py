"""Injection campaigns and the learned p_det surrogate, driven through the C ABI.

The detection probability of a population (Sec. V, Eqs. pdet_abstract and
sampling) is estimated by injecting signals into synthetic data, searching them
with the brute-force statistic and applying the detection rule
R(z; tau) = 1[z > tau] (Sec. V.B) to the loudest critical ratio of each run.
Those labels train a small network p_det(h0/sqrt(S_n), cos iota, psi, sin delta,
alpha, f) on the GPU; plain injection campaigns remain the check on it.

All arithmetic runs in the HIP library (table generation, evaluation, exact
toplists, labels, network training and inference); this module only chunks the
campaign and summarises results.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fasttracks as ft
from . import synth

AMP_RANGE = (0.005, 0.1)
# feature standardisation of (log amp, cos iota, psi, sin delta, alpha, f):
# mean and standard deviation of the uniform sampling distributions
FEAT_SHIFT = np.array([0.5 * (math.log(AMP_RANGE[0]) + math.log(AMP_RANGE[1])), 0.0, 0.0, 0.0,
                       math.pi, 200.0])
FEAT_SCALE = np.array([(math.log(AMP_RANGE[1]) - math.log(AMP_RANGE[0])) / math.sqrt(12.0),
                       1.0 / math.sqrt(3.0), (math.pi / 2.0) / math.sqrt(12.0),
                       1.0 / math.sqrt(3.0), 2.0 * math.pi / math.sqrt(12.0),
                       200.0 / math.sqrt(12.0)])


def noise_threshold(ctx: ft.Context, w: synth.Workload, rank: int = 100) -> float:
    """Detection threshold tau: mean over the sub-bands of the rank-th largest
    critical ratio of a noise-only search of workload w (its K must be >= rank)."""
    ctx.load_workload(w)
    ctx.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges)
    zs = []
    for j in range(len(w.sub_edges) - 1):
        top = ctx.toplist(j, w.k)
        zs.append(top[min(rank, len(top)) - 1].z)
    return float(np.mean(zs))


def make_labels(ctx: ft.Context, base: synth.Workload, n: int, seed: int, tau: float,
                chunk: int = 4096, amp_range=AMP_RANGE):
    """n injection-recovery labels on the SFTs of `base`.  Returns
    (raw [n, 6], labels [n] in {0, 1}, max_z [n], GPU seconds of the batches)."""
    raws, labels, zs = [], [], []
    gpu_s = 0.0
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        cp, raw = synth.label_campaign(m, seed * 1_000_003 + c0, base, amp_range=amp_range)
        ctx.eval_campaign(cp)
        lab, mz = ctx.batch_labels(tau, m)
        gpu_s += ctx.batch_time() * 1e-3
        raws.append(raw)
        labels.append(lab)
        zs.append(mz)
    return np.concatenate(raws), np.concatenate(labels), np.concatenate(zs), gpu_s


SCHEDULE = ((8, 2e-3), (6, 6e-4), (6, 2e-4))


def train(ctx: ft.Context, raw, y, schedule=SCHEDULE, batch: int = 2048, seed: int = 0):
    """Train the surrogate with Adam in phases of (epochs, learning rate) (the
    moments and step count carry over between phases); returns (Mlp, per-epoch
    loss, seconds)."""
    net = ft.Mlp(ctx, FEAT_SHIFT, FEAT_SCALE, max_batch=max(batch, 8192), seed=seed)
    raw = np.asarray(raw, np.float32)
    y = np.asarray(y, np.float32)
    hist = []
    t0 = time.perf_counter()
    for i, (epochs, lr) in enumerate(schedule):
        hist.extend(net.train(raw, y, batch=batch, epochs=epochs, lr=lr, seed=seed + 1 + i))
    return net, np.asarray(hist), time.perf_counter() - t0


def calibration(p_hat, y, raw, n_amp_bins: int = 20, n_p_bins: int = 10):
    """Surrogate against plain injections: largest |mean predicted p - detected
    fraction| over log-amplitude bins and over deciles of the predicted p, with
    the binomial standard error of the worst bin."""
    p_hat = np.asarray(p_hat, np.float64)
    y = np.asarray(y, np.float64)
    la = np.log(np.asarray(raw)[:, 0])
    edges = np.linspace(la.min(), la.max() + 1e-12, n_amp_bins + 1)
    idx = np.clip(np.digitize(la, edges) - 1, 0, n_amp_bins - 1)

    def worst(groups):
        err, se, rows = 0.0, 0.0, []
        for g in groups:
            if g.sum() < 10:
                continue
            d = abs(p_hat[g].mean() - y[g].mean())
            s = math.sqrt(max(y[g].mean() * (1 - y[g].mean()), 1e-12) / g.sum())
            rows.append((float(p_hat[g].mean()), float(y[g].mean()), int(g.sum())))
            if d > err:
                err, se = d, s
        return err, se, rows

    amp_err, amp_se, amp_rows = worst([idx == b for b in range(n_amp_bins)])
    q = np.quantile(p_hat, np.linspace(0, 1, n_p_bins + 1))
    pidx = np.clip(np.searchsorted(q, p_hat, side="right") - 1, 0, n_p_bins - 1)
    p_err, p_se, _ = worst([pidx == b for b in range(n_p_bins)])
    return {"max_abs_err_amp_bins": amp_err, "se_worst_amp_bin": amp_se,
            "max_abs_err_p_deciles": p_err, "se_worst_p_decile": p_se,
            "amp_bins": amp_rows}
