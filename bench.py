#!/usr/bin/env python3
"""Throughput of the brute-force short-coherence statistic on one MI355X.

Workload: the all-sky band -- 2 detectors x 5000 SFTs (T_sft = 1800 s, 10% gaps),
200-200.5 Hz, bank 900 f0 x 11 f1 x 1e5 isotropic sky points (9.9e8 templates,
9.9e12 template-SFT evaluations), K = 100 per 0.05 Hz sub-band; seeded synthetic
unit-variance complex-Gaussian noise.

One step = upload the SFT table and velocities (device-resident inputs, device
to device), evaluate every template, select + FP64-re-sum + rank the toplists
of all 10 sub-bands, copy them to the host.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.32e12 VALU
# lane-operations per second (the FP64 vector peak of 78.6 TFLOP/s counts an
# FMA as two).
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def valu_ops_per_eval(tile_name):
    """VALU lane-operations the grid kernel issues per template-SFT evaluation.

    A lane's run of L templates costs 10 operations for the first bin
    (4 FP64 arithmetic, 2 conversions, 1 subtraction, 2 guard compares, 1 LDS
    address) plus one FP32 accumulate per template."""
    L = int(tile_name.split("_")[0][1:]) if tile_name else 1
    return (10.0 + L) / L if L > 1 else 7.0


def cpu_baseline(w, target_s):
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    n_sky = max(1, threads)
    sky = w.sky[:n_sky]
    t0 = time.perf_counter()
    oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0, w.f1, sky)
    dt = time.perf_counter() - t0
    if dt < target_s / 3:
        n_sky = int(min(w.sky.shape[0], max(n_sky, n_sky * target_s / max(dt, 1e-3))))
        n_sky = max(threads, (n_sky // threads) * threads)
        sky = w.sky[:n_sky]
        t0 = time.perf_counter()
        oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0, w.f1,
                         sky)
        dt = time.perf_counter() - t0
    evals = w.f0.size * w.f1.size * n_sky * w.n_sft
    del np
    return {"value": evals / dt, "unit": "template*SFT evals/s", "cores": threads,
            "kind": "oracle",
            "sample": "same band, SFTs and f0 x f1 grid; first %d of the 1e5 sky points "
                      "(%.3g evals, %.1f s)" % (n_sky, evals, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-sky", type=int, default=100_000)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the statistic shards by sub-band or sky point "
              "with no exchange, and multi-GPU runs are not part of this build "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_18370_amd import fasttracks as ft
    from paper_2411_18370_amd import synth

    ft.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating the all-sky workload (n_sky=%d)" % args.n_sky)
    w = synth.allsky_band(seed=2, n_sky=args.n_sky)
    t_mid = torch.from_numpy(w.t_mid).to(dev)
    power = torch.from_numpy(w.power).to(dev)
    vel = torch.from_numpy(w.v).to(dev)
    f0 = torch.from_numpy(w.f0).to(dev)
    f1 = torch.from_numpy(w.f1).to(dev)
    sky = torch.from_numpy(np.ascontiguousarray(w.sky)).to(dev)
    edges = torch.from_numpy(w.sub_edges).to(dev)
    n_sub = len(w.sub_edges) - 1
    stream = torch.cuda.current_stream()
    c = ft.Context(0, stream.cuda_stream)

    def step():
        c.set_sfts(w.n_sft_per_det, t_mid, w.t_sft, w.first_bin, power)
        c.set_velocities(vel)
        c.eval_templates(f0, f1, sky, w.t_ref, w.k, edges, tile=args.tile)
        return [c.toplist(j, w.k) for j in range(n_sub)]

    for i in range(args.warmup):
        step()
        log("warmup step %d done: eval %.1f ms" % (i, c.info().eval_ms))
    torch.cuda.synchronize()
    eval_ms, sel_ms = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        tops = step()
        info = c.info()
        eval_ms.append(info.eval_ms)
        sel_ms.append(info.select_ms)
        log("step %d: eval %.1f ms, select %.2f ms, %d candidates" %
            (i, info.eval_ms, info.select_ms, info.n_candidates))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    evals = w.evals
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = evals * args.steps / (t1 - t0)
    tile_name = ft.ft_tile_name(info.tile)
    k_ms = float(np.mean(eval_ms))
    ops = valu_ops_per_eval(tile_name)
    achieved = evals * ops / (k_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    top1 = max((t[0] for t in tops if t), key=lambda c_: c_.z)
    line = {
        "metric": "template*SFT evals/s on 1 GPU (plain)",
        "value": value,
        "unit": "template*SFT evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 index, f32 sums (f64 re-summed toplists)",
        "data": "synthetic: seeded unit-variance complex Gaussian SFT bins, analytic Earth "
                "orbit+rotation velocities, isotropic sky",
        "config": {"workload": "all-sky band 200-200.5 Hz, 2 det x 5000 SFTs (10%% gaps), "
                               "900 f0 x 11 f1 x %d sky, K=100 per 0.05 Hz" % args.n_sky,
                   "n_templates": w.n_templates, "n_sft": w.n_sft, "evals_per_step": evals,
                   "tile": tile_name, "lds_window_bins": info.window},
        "kernel_ms": k_ms,
        "select_ms": float(np.mean(sel_ms)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak, "traffic": None,
                     "ops_per_eval": ops,
                     "note": "VALU lane-ops of the grid kernel per evaluation x evals / kernel "
                             "time (HIP events on the library stream)"},
        "loudest_z": top1.z,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a CPU sample")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    c.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
