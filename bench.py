#!/usr/bin/env python3
"""Throughput of the brute-force short-coherence statistic on one MI355X.

Workload: the all-sky band -- 2 detectors x 5000 SFTs (T_sft = 1800 s, 10% gaps),
200-200.5 Hz, bank 900 f0 x 11 f1 x 1e5 isotropic sky points (9.9e8 templates,
9.9e12 template-SFT evaluations), K = 100 per 0.05 Hz sub-band; seeded synthetic
unit-variance complex-Gaussian noise with 3 injected signals (h0/sqrt(S_n) in
[0.05, 0.2]), generated on the GPU before timing.

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
    """VALU lane-operations the grid kernel needs per template-SFT evaluation.

    A lane's run of L consecutive f0 costs 6 operations for the first bin (one
    FP64 fused multiply-add, fraction, conversion, 2 guard compares, 1 LDS
    address) plus one FP32 accumulate per template; with L = 1 the canonical bin
    costs 3 FP64 arithmetic, 1 add, 1 conversion, 1 address, 1 accumulate."""
    L = int(tile_name.split("_")[0][1:]) if tile_name else 1
    return (6.0 + L) / L if L > 1 else 7.0


def kernel_source_hash():
    """SHA-256 of the grid kernel's source (the traffic figure below is only
    valid for the kernel it was measured on)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2411_18370_amd", "csrc", "eval_grid.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(tile_name):
    """HBM bytes per launch of the grid kernel at the all-sky band, from the
    committed rocprofv3 counter summary, or None when that summary was taken on
    another kernel source or tile."""
    path = os.path.join(ROOT, "profiles", "eval_grid_allsky_band_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.split()[0] if v.split() else ""
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("tile") != tile_name:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model string (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


ONE_THREAD_CHILD = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2411_18370_amd import synth
n_sky = int(sys.argv[2])
w = synth.allsky_band(seed=2, n_sky=n_sky)
t0 = time.perf_counter()
oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, w.power, None, w.v, w.f0, w.f1, w.sky)
dt = time.perf_counter() - t0
print(json.dumps({"evals": w.evals, "seconds": dt}))
"""


def cpu_baseline_one_thread(n_sky=4):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1),
    on the first n_sky sky points of the same band."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", ONE_THREAD_CHILD, ROOT, str(n_sky)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["evals"] / d["seconds"], "unit": "template*SFT evals/s", "cores": 1,
            "sample": "first %d sky points of the same band (%.3g evals, %.1f s)"
                      % (n_sky, d["evals"], d["seconds"])}


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
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "same band, SFTs and f0 x f1 grid; first %d of the 1e5 sky points "
                      "(%.3g evals, %.1f s)" % (n_sky, evals, dt),
            "one_thread": cpu_baseline_one_thread()}


def bench_batched(ft, synth, n_runs, log):
    """Uneven injection campaign: plain (one call per run) against batched (one
    persistent graph-captured launch)."""
    import numpy as np
    import torch
    cp = synth.campaign(n_runs, seed=4)
    evals = cp.evals
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    # plain: table generation + evaluation + toplist, run by run
    def plain():
        for R in cp.runs:
            sl = slice(R["sft_begin"], R["sft_begin"] + R["n_sft"])
            c.gen_sfts([R["n_sft"]], cp.t_mid[sl], cp.t_sft, R["first_bin"], R["n_bins"],
                       cp.v[sl], cp.arms[sl], R["seed"], R["run_id"], R["t_ref"], R["inj"])
            f0 = cp.f0[R["f0_begin"]:R["f0_begin"] + R["n_f0"]]
            f1 = cp.f1[R["f1_begin"]:R["f1_begin"] + R["n_f1"]]
            sky = cp.sky[R["sky_begin"]:R["sky_begin"] + R["n_sky"]]
            c.eval_templates(f0, f1, sky, R["t_ref"], cp.k, np.array([f0[0] - 1.0, f0[-1] + 1.0]))
            c.toplist(0, cp.k)
    plain()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log("batched campaign: plain %.3f s for %d runs" % (t_plain, n_runs))
    # batched: capture once (includes host planning and uploads), then replay
    t0 = time.perf_counter()
    c.eval_campaign(cp, use_graph=1, tile=ft.FT_TILE_TUNE)
    c.batch_toplist(0, cp.k)
    t_first = time.perf_counter() - t0
    rep, tune_ms = c.tune_report()
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpu = []
    for _ in range(reps):
        c.batch_replay()
        c.batch_toplist(n_runs - 1, cp.k)
        gpu.append(c.batch_time())
    t_replay = (time.perf_counter() - t0) / reps
    log("batched campaign: first call %.3f s, graph replay %.4f s (GPU %.4f s)"
        % (t_first, t_replay, np.mean(gpu) * 1e-3))
    c.close()
    return {"workload": "%d uneven injection runs, 2 det, N ~ U{500..5000}, band 100-300 Hz, "
                        "width U[0.01,0.2] Hz, 1e3-1e5 templates each, K=%d" % (n_runs, cp.k),
            "evals": evals, "plain_evals_per_s": evals / t_plain,
            "batched_evals_per_s": evals / t_replay,
            "batched_first_call_evals_per_s": evals / t_first,
            "batched_gpu_ms": float(np.mean(gpu)), "speedup_vs_plain": t_plain / t_replay,
            "autotune": {"tune_ms": tune_ms,
                         "chosen": {str(e["klass"]): e["name"] for e in rep if e["chosen"]},
                         "n_timed": len(rep)}}


def bench_precision(ft, synth, log):
    """Index precision at 1 kHz (mismatches against the FP64 bin) and the error of
    plain against blocked FP32 sums (against the FP64 re-summed toplist)."""
    import numpy as np
    import torch
    w = synth.precision_stress(seed=2)
    dev = torch.device("cuda:0")
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
               torch.from_numpy(w.power).to(dev))
    c.set_velocities(torch.from_numpy(w.v).to(dev))
    out = {"workload": "2 det x 5000 SFTs, 1000-1000.1 Hz, 180 f0 x 5 f1 x 2e4 sky "
                       "(%.3g evals)" % w.evals}
    for name, mode in (("fp32", ft.FT_INDEX_FP32), ("df64", ft.FT_INDEX_DF64),
                       ("guarded_df64", ft.FT_INDEX_GUARDED), ("guarded_fp32", ft.FT_INDEX_GUARDED_FP32),
                       ("fp64", ft.FT_INDEX_FP64)):
        t0 = time.perf_counter()
        n, fb = c.count_index_mismatches(w.f0, w.f1, w.sky, w.t_ref, mode, fallback=True)
        out["mismatch_" + name] = n
        if mode in (ft.FT_INDEX_GUARDED, ft.FT_INDEX_GUARDED_FP32):
            out["fallback_frac_" + name] = fb / w.evals
        log("precision: %s index mismatches %d, FP64 fallbacks %d (%.2f s)"
            % (name, n, fb, time.perf_counter() - t0))
    out["evals"] = w.evals
    stats = torch.empty(w.n_templates, dtype=torch.float32, device=dev)
    for name, mode in (("blocked", ft.FT_SUM_BLOCKED), ("plain", ft.FT_SUM_PLAIN_FP32)):
        c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges, sum_mode=mode, stats=stats)
        tops = [c.toplist(j, w.k) for j in range(len(w.sub_edges) - 1)]
        info = c.info()
        s = stats.cpu().numpy()
        rel = np.array([abs(float(s[t.index]) - t.s64) / t.s64 for top in tops for t in top])
        out["sum_%s_max_rel_err" % name] = float(rel.max())
        out["sum_%s_rms_rel_err" % name] = float(np.sqrt(np.mean(rel ** 2)))
        if name == "blocked":
            out["fp64_index_evals_per_s"] = w.evals / (info.eval_ms * 1e-3)
    c.close()
    return out


def paper_cost_per_template(n, n_sft):
    """The paper's fit of the GPU cost per template (Sec. III, seconds assumed):
    log10 c = -(5/3) log10 n + log10 N_SFT / (1 + (10^6/n)^(5/6))."""
    import math
    return 10.0 ** (-(5.0 / 3.0) * math.log10(n) + math.log10(n_sft) / (1.0 + (1e6 / n) ** (5.0 / 6.0)))


def bench_binary(ft, synth, log, sizes=(10 ** 5, 10 ** 6, 10 ** 7), reps=3):
    """The paper's benchmark workload (Sec. III): random banks of sources in
    circular binary systems, generated on the device and evaluated over 10^4
    SFTs (T = 1024 s, half-overlapping, 2 detectors; 110.5 Hz, 0.125 Hz band,
    periods 7-15 d, a_p 5-15 lt-s), per batch size n, next to the paper's cost
    model (its fit for one H100; context, not a target)."""
    import torch
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    dev = torch.device("cuda:0")
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
               torch.from_numpy(w.power).to(dev))
    c.set_velocities(torch.from_numpy(w.v).to(dev))
    out = {"workload": "random binary-system banks uniform in the xi coordinates, generated on "
                       "the GPU; 2 det x 5000 SFTs of 1024 s (half-overlapping, 10%% gaps), "
                       "110.5-110.625 Hz, periods 7-15 d, a_p 5-15 lt-s, K=10 per 0.025 Hz",
           "n_sft": w.n_sft, "batches": []}
    for n in sizes:
        c.eval_binary_random(w.region, 99, n, w.t_ref, w.k, w.sub_edges)
        c.toplist(0, w.k)
        eval_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            c.eval_binary_random(w.region, 100 + r, n, w.t_ref, w.k, w.sub_edges)
            c.toplist(0, w.k)  # synchronises
            eval_ms.append(c.info().eval_ms)
        t1 = time.perf_counter()
        evals = n * w.n_sft
        call_s = (t1 - t0) / reps
        model = paper_cost_per_template(n, w.n_sft)
        e = {"n_templates": n, "evals": evals,
             "evals_per_s_kernel": evals / (sum(eval_ms) / reps * 1e-3),
             "evals_per_s_call": evals / call_s,
             "s_per_template_call": call_s / n,
             "paper_model_s_per_template": model,
             "paper_model_evals_per_s": w.n_sft / model}
        out["batches"].append(e)
        log("binary bank n=%d: kernel %.3g evals/s, whole call %.3g evals/s (%.3g s/template; "
            "paper's H100 fit %.3g)" % (n, e["evals_per_s_kernel"], e["evals_per_s_call"],
                                         e["s_per_template_call"], model))
    # the all-sky weights of Sec. II.B on the largest batch (normalised per template)
    n = sizes[-1]
    c.set_arms(torch.from_numpy(w.arms).to(dev))
    c.eval_binary_random(w.region, 99, n, w.t_ref, w.k, w.sub_edges, weights=ft.FT_WEIGHTS_SKY)
    c.toplist(0, w.k)
    ms = []
    for r in range(reps):
        c.eval_binary_random(w.region, 100 + r, n, w.t_ref, w.k, w.sub_edges, weights=ft.FT_WEIGHTS_SKY)
        c.toplist(0, w.k)
        ms.append(c.info().eval_ms)
    out["sky_weights"] = {"n_templates": n, "evals_per_s_kernel": n * w.n_sft / (sum(ms) / reps * 1e-3)}
    log("binary bank n=%d with all-sky weights: kernel %.3g evals/s" % (n, out["sky_weights"]["evals_per_s_kernel"]))
    c.close()
    return out


def bench_mismatch(ft, synth, log, oversampling=(1.0, 3.44, 10.0), n_trials=100):
    """Mismatch distribution p(m|o) of random binary-system banks (Sec. IV.A) at
    the paper's oversampling 3.44 and around it: per trial a binary signal in
    noise (h0/sqrt(Sn) = 1), a random bank of o N(box) templates in a +-2
    resolution-cell box around it, m of the loudest template (Eq. mismatch)."""
    import numpy as np
    import torch
    from paper_2411_18370_amd import mismatch
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    out = {"workload": "2 det x 5000 SFTs of 1024 s (half-overlapping), 110.5-110.625 Hz, periods 7-15 d, "
                       "a_p 5-15 lt-s; %d trials per oversampling" % n_trials, "p_m_given_o": []}
    for o in oversampling:
        t0 = time.perf_counter()
        r = mismatch.sample(c, w, o=o, n_trials=n_trials, seed=int(o * 1000), amp=1.0)
        s = mismatch.summary(r["m"])
        s["o"] = o
        s["mean_bank_templates"] = float(np.mean([t["n_bank"] for t in r["trials"]]))
        s["seconds"] = time.perf_counter() - t0
        out["p_m_given_o"].append(s)
        log("mismatch o=%.2f: mean %.3f, median %.3f, 90%% in [%.3f, %.3f], %.0f templates per bank (%.1f s)"
            % (o, s["mean"], s["median"], s["q05"], s["q95"], s["mean_bank_templates"], s["seconds"]))
    c.close()
    return out


def bench_sensitivity(ft, synth, log, o=3.44, tau=8.0, depths=(15.0, 22.0, 27.0, 33.0, 45.0), n_inj=500,
                      n_q=100_000, k_best=16):
    """Semi-analytic sensitivity estimate (Sec. V) against plain injections (the
    comparison of Sec. VI) for the random-bank binary search at oversampling o:
    p_det at each depth from q samples of 10^5 population draws and p(m|o), and
    from n_inj injections per depth (loudest template of a random bank around
    each), rule z > tau; with the cost of each.  The loudest-of-bank noise gain
    is bracketed by the one-template lower bound and the independent-noise
    maximum over the k_best smallest mismatches of each bank."""
    import numpy as np
    import torch
    from paper_2411_18370_amd import mismatch, sensitivity
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    ms = mismatch.sample(c, w, o=o, n_trials=100, seed=12, amp=1.0, k_best=k_best)
    m = ms["m"]
    c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
    t0 = time.perf_counter()
    q = sensitivity.q_samples(c, w.arms, n_q, seed=13)
    p_sa = sensitivity.p_det(q, m, depths, tau, seed=14)
    t_sa = time.perf_counter() - t0
    p_lo, p_hi = sensitivity.p_det_bounds(q, ms["m_k"], depths, tau, seed=16)
    t0 = time.perf_counter()
    p_inj = sensitivity.injection_p_det(c, w, depths, n_inj, o, tau, seed=15)
    t_inj = time.perf_counter() - t0
    c.close()
    se = np.sqrt(np.maximum(p_inj * (1 - p_inj), 1.0 / n_inj) / n_inj)
    # distance of the injections' fraction outside the [lower, upper] band, in binomial se
    outside = np.maximum(np.maximum(p_lo - p_inj, p_inj - p_hi), 0.0) / se
    out = {"workload": "random-bank binary search, 2 det x 5000 SFTs of 1024 s, 110.5 Hz; oversampling %g, "
                       "rule z > %g; %d q samples, %d injections per depth" % (o, tau, n_q, n_inj),
           "depths": list(depths), "p_det_semi_analytic": p_sa.tolist(), "p_det_injections": p_inj.tolist(),
           "binomial_se": se.tolist(), "max_abs_diff": float(np.max(np.abs(p_sa - p_inj))),
           "loudest_of_bank_bounds": {"k_best": k_best, "lower": p_lo.tolist(), "upper": p_hi.tolist(),
                                      "injections_outside_band_in_se": outside.tolist()},
           "seconds_semi_analytic": t_sa, "seconds_injections": t_inj}
    log("sensitivity: depths %s, semi-analytic %s (%.2f s), band [%s, %s], injections %s (%.1f s)"
        % (list(depths), np.round(p_sa, 3).tolist(), t_sa, np.round(p_lo, 3).tolist(),
           np.round(p_hi, 3).tolist(), np.round(p_inj, 3).tolist(), t_inj))
    return out


def bench_hyperbox(ft, synth, log, n_bank=10 ** 8, min_boxes=10_000, o=3.44, n_q=100_000,
                   n_cands=(1, 10, 100, 1000), rejects=(0, 1, 3, 10, 30, 100, 300, 500)):
    """Search step of Sec. IV.B / VI.A on the paper's binary workload: a random
    bank of n_bank templates (o = 3.44, full sky and orbital phase, a_p 5-15
    lt-s, periods 7-15 d, f0 from 110.5 Hz up to the width that holds them)
    partitioned into at least 10^4 equal-volume hyperboxes, the exact loudest
    template of each (whole call timed: generation, evaluation, per-box
    selection); then D^95% for N_cand candidates with the optimal number of
    rejected boxes (semi-analytic estimate with p(m|o) and 10^5 q samples), on
    Gaussian noise and with a synthetic transient instrumental line (+4 in the
    bin 6 bins above the band, over the middle 30% of the SFTs)."""
    import numpy as np
    import torch
    from paper_2411_18370_amd import hyperbox, mismatch, sensitivity
    w = synth.binary_band(seed=3, n_tmpl=1, n_per_det=5000)
    t_obs = float(w.t_mid.max() - w.t_mid.min() + w.t_sft)
    vmax = float(np.max(np.linalg.norm(w.v, axis=1)))
    region = dict(w.region, alpha_lo=0.0, alpha_hi=2 * np.pi, sdec_lo=-1.0, sdec_hi=1.0, phib_lo=0.0,
                  phib_hi=2 * np.pi)
    per_f06 = mismatch.n_templates(region, w.t_sft, t_obs, vmax) / (region["f0_hi"] ** 6 - region["f0_lo"] ** 6)
    region["f0_hi"] = (region["f0_lo"] ** 6 + n_bank / (o * per_f06)) ** (1.0 / 6.0)
    n_div = hyperbox.partition(region, w.t_sft, t_obs, vmax, o, n_bank / min_boxes, min_boxes=min_boxes)
    n_boxes = int(np.prod(n_div))
    dev = torch.device("cuda:0")
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    power = torch.from_numpy(w.power).to(dev)
    c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin, power)
    c.set_velocities(torch.from_numpy(w.v).to(dev))
    c.eval_binary_boxes(region, 1, 10 ** 6, w.t_ref, n_div)  # warm-up
    runs = {}
    # the line sits 6 bins above the band: only tracks with a large orbital
    # Doppler amplitude a_p Omega f0 T (up to ~8 bins here) reach it
    line_col = int(round(region["f0_lo"] * w.t_sft)) + 6 - w.first_bin
    k0, k1 = int(0.35 * w.n_sft), int(0.65 * w.n_sft)
    for case in ("gaussian", "line"):
        if case == "line":
            tab = w.power.copy()
            tab[k0:k1, line_col] += 4.0
            c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
                       torch.from_numpy(tab).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = c.eval_binary_boxes(region, 7, n_bank, w.t_ref, n_div)
        secs = time.perf_counter() - t0
        runs[case] = (res, secs)
        z = res["z"][res["index"] >= 0]
        log("hyperbox %s: %d templates in %d boxes (n_div %s) in %.2f s (%.3g evals/s); box z max %.1f, "
            "median %.2f" % (case, n_bank, n_boxes, n_div, secs, n_bank * w.n_sft / secs, z.max(), np.median(z)))
    m = mismatch.sample(c, w, o=o, n_trials=100, seed=12, amp=1.0)["m"]
    c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power)
    q = sensitivity.q_samples(c, w.arms, n_q, seed=13)
    c.close()
    out = {"workload": "random binary bank of %d templates (o = %g) over f0 %.6f-%.6f Hz, full sky and phase, "
                       "a_p 5-15 lt-s, periods 7-15 d; 2 det x 5000 SFTs of 1024 s"
                       % (n_bank, o, region["f0_lo"], region["f0_hi"]),
           "n_div": n_div, "n_boxes": n_boxes, "cases": {}}
    for case, (res, secs) in runs.items():
        z_box = hyperbox.box_z(res)
        t0 = time.perf_counter()
        rows = []
        for n_cand in n_cands:
            best, table = hyperbox.optimize_reject(q, m, z_box, n_cand, rejects, p=0.95, seed=21)
            d = dict(table)
            rows.append({"n_cand": n_cand, "d95_no_reject": d[0], "best_n_reject": best, "d95_best": d[best],
                         "table": table})
            log("hyperbox %s N_cand=%d: D95 %.2f without rejection, %.2f rejecting %d boxes"
                % (case, n_cand, d[0], d[best], best))
        out["cases"][case] = {"seconds": secs, "evals_per_s_call": n_bank * w.n_sft / secs,
                              "empty_boxes": int((res["index"] < 0).sum()),
                              "templates_per_box_mean": float(res["count"].mean()),
                              "box_z_max": float(np.nanmax(z_box)), "selection": rows,
                              "optimisation_s": time.perf_counter() - t0}
    out["line"] = {"column_hz": (w.first_bin + line_col) / w.t_sft, "sfts": [k0, k1], "excess_power": 4.0}
    return out


def bench_weighted(ft, c, w, f0, f1, sky, edges, arms, log, reps=2):
    """The all-sky band (table already loaded in c) with the other statistics and
    weights of Sec. II.B: the power with the all-sky weights (a^2 + b^2)/S_n, the
    weighted number count with per-SFT and with all-sky weights; kernel rates
    (HIP events) and the whole call; then the persistence-checked candidate of
    Sec. VI.B (loudest power with number-count z >= 3) of each injected sub-band."""
    import numpy as np
    import torch
    from paper_2411_18370_amd import persistence
    c.set_arms(arms)
    out = {}
    n_sub = len(w.sub_edges) - 1
    for name, stat, wts in (("power_sky_weights", ft.FT_STAT_POWER, ft.FT_WEIGHTS_SKY),
                            ("number_count", ft.FT_STAT_NUMBER_COUNT, ft.FT_WEIGHTS_SFT),
                            ("number_count_sky_weights", ft.FT_STAT_NUMBER_COUNT, ft.FT_WEIGHTS_SKY)):
        ms, wall = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.eval_templates(f0, f1, sky, w.t_ref, w.k, edges, statistic=stat, weights=wts)
            tops = [c.toplist(j, w.k) for j in range(n_sub)]
            wall.append(time.perf_counter() - t0)
            ms.append(c.info().eval_ms)
        info = c.info()
        inj_z = []
        for inj in w.injections:
            j = int(np.searchsorted(w.sub_edges, inj["f0"], side="right")) - 1
            inj_z.append(tops[j][0].z)
        out[name] = {"kernel_evals_per_s": w.evals / (min(ms) * 1e-3), "kernel_ms": min(ms),
                     "call_evals_per_s": w.evals / min(wall), "tile": ft.ft_tile_name(info.tile),
                     "top_z_injected_subbands": inj_z}
        log("weighted %s: kernel %.3g evals/s (%.0f ms, %s), call %.3g evals/s, top z at injections %s"
            % (name, out[name]["kernel_evals_per_s"], min(ms), out[name]["tile"],
               out[name]["call_evals_per_s"], np.round(inj_z, 1).tolist()))
    # persistence-checked candidates (power toplists with their exact number counts)
    c.eval_templates(f0, f1, sky, w.t_ref, w.k, edges)
    t0 = time.perf_counter()
    cands = []
    for inj in w.injections:
        j = int(np.searchsorted(w.sub_edges, inj["f0"], side="right")) - 1
        got = persistence.loudest_persistent(c, j, w.k, 3.0)
        cands.append(None if got is None else {"sub_band": j, "z": got[0].z, "nc": got[1], "z_nc": got[2],
                                               "df0_bins": (got[0].f0 - inj["f0"]) * w.t_sft})
    out["persistent_candidates"] = cands
    out["persistence_check_s"] = time.perf_counter() - t0
    log("persistent candidates at the injections: %s" % cands)
    return out


def bench_surrogate(ft, synth, tau, n_train, n_test, log):
    """Labels from GPU injection campaigns, GPU training, calibration on held-out
    injections, and the cost of a surrogate query against a plain label."""
    import numpy as np
    import torch
    from paper_2411_18370_amd import surrogate
    base = synth.allsky_band(seed=2, n_sky=1)
    c = ft.Context(0, torch.cuda.current_stream().cuda_stream)
    t0 = time.perf_counter()
    raw, y, _, gpu_tr = surrogate.make_labels(c, base, n_train, 11, tau)
    rt, yt, _, gpu_te = surrogate.make_labels(c, base, n_test, 12, tau)
    t_labels = time.perf_counter() - t0
    log("surrogate: %d + %d labels in %.1f s (GPU %.1f s), detected fraction %.3f"
        % (n_train, n_test, t_labels, gpu_tr + gpu_te, y.mean()))
    torch.cuda.synchronize()
    net, hist, t_train = surrogate.train(c, raw, y, seed=13)
    t0 = time.perf_counter()
    p = net.predict(rt.astype(np.float32))
    t_pred = time.perf_counter() - t0
    cal = surrogate.calibration(p, yt, rt)
    log("surrogate: trained in %.1f s, calibration max err %.4f (amp bins), %.4f (p deciles)"
        % (t_train, cal["max_abs_err_amp_bins"], cal["max_abs_err_p_deciles"]))
    net.close()
    c.close()
    per_label = (gpu_tr + gpu_te) / (n_train + n_test)
    # matrix-core work of training: per step of m rows (padded to 64) the two
    # 256 x 256 layers take 2 m 256^2 flops in each of the forward, input-
    # gradient and weight-gradient products
    batch = 2048
    epochs = sum(e for e, _ in surrogate.SCHEDULE)
    rows = epochs * (n_train // batch * batch + ((n_train % batch + 63) // 64 * 64))
    flops = rows * 2 * 3 * 2 * 256 * 256
    mfma = {"flops": flops, "steps": epochs * -(-n_train // batch), "TFLOPs": flops / t_train / 1e12,
            "frac_of_bf16_dense_peak": flops / t_train / 2.5e15,
            "note": "whole training call (host validation, 10 launches per step) over the "
                    "bf16 dense peak of 2.5 PFLOP/s; batch 2048 leaves each product at 0.27 "
                    "GFLOP, so a step is bound by launch and reduction latency"}
    per_query = t_pred / n_test
    return {"workload": "labels on the all-sky SFT set (2 det x 5000 SFTs), local bank 5 f0 x "
                        "11 f1 x 16 sky, f ~ U[100,300] Hz, h0/sqrt(Sn) log-uniform [0.005, 0.1]; "
                        "MLP 6-256-256-256-1 GELU/sigmoid, BF16 MFMA; Adam, batch 2048, "
                        "epochs x lr = %s" % (surrogate.SCHEDULE,),
            "tau_z": tau, "n_train": n_train, "n_test": n_test,
            "p_det_abs_err": cal["max_abs_err_amp_bins"],
            "p_det_abs_err_p_deciles": cal["max_abs_err_p_deciles"],
            "binomial_se_worst_bin": cal["se_worst_amp_bin"],
            "train_s": t_train, "final_loss": float(hist[-1]),
            "train_mfma": mfma,
            "s_per_plain_label": per_label, "s_per_surrogate_query": per_query,
            "speedup": per_label / per_query}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-sky", type=int, default=100_000)
    ap.add_argument("--tile", type=int, default=-1,
                    help="-1: autotune during warm-up (default), 0: cost model, else a tile id")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-runs", type=int, default=512)
    ap.add_argument("--surrogate-train", type=int, default=1_000_000)
    ap.add_argument("--surrogate-test", type=int, default=100_000)
    ap.add_argument("--skip-extras", action="store_true",
                    help="plain workload only (no batched, precision or surrogate sections)")
    ap.add_argument("--sections", default="weighted,batched,precision,surrogate,binary,mismatch,sensitivity,hyperbox",
                    help="comma-separated extra sections to run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the statistic shards by sub-band or sky point "
              "with no exchange, and multi-GPU runs are not implemented "
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
    vel = torch.from_numpy(w.v).to(dev)
    arms = torch.from_numpy(w.arms).to(dev)
    f0 = torch.from_numpy(w.f0).to(dev)
    f1 = torch.from_numpy(w.f1).to(dev)
    sky = torch.from_numpy(np.ascontiguousarray(w.sky)).to(dev)
    edges = torch.from_numpy(w.sub_edges).to(dev)
    n_sub = len(w.sub_edges) - 1
    stream = torch.cuda.current_stream()
    c = ft.Context(0, stream.cuda_stream)
    # the SFT table: Philox noise plus the band's 3 injected signals, generated
    # on the GPU once; every step then loads it from HBM
    power = torch.empty((w.n_sft, w.n_bins), dtype=torch.float32, device=dev)
    c.gen_sfts(w.n_sft_per_det, t_mid, w.t_sft, w.first_bin, w.n_bins, vel, arms, 2, 0, w.t_ref,
               w.injections, power_out=power)

    def step():
        c.set_sfts(w.n_sft_per_det, t_mid, w.t_sft, w.first_bin, power)
        c.set_velocities(vel)
        c.eval_templates(f0, f1, sky, w.t_ref, w.k, edges, tile=args.tile)
        return [c.toplist(j, w.k) for j in range(n_sub)]

    for i in range(args.warmup):
        step()
        log("warmup step %d done: eval %.1f ms" % (i, c.info().eval_ms))
    tune_rep, tune_ms = c.tune_report()
    if tune_rep:
        log("autotune (%.0f ms): %s" % (tune_ms, ", ".join(
            "%s%s %.3g" % (e["name"], "*" if e["chosen"] else "", e["evals_per_s"])
            for e in tune_rep)))
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
    # detection threshold of the learned part: median over the sub-bands of the
    # 100th-largest critical ratio (the median ignores the few injected sub-bands)
    tau = float(np.median([t[min(100, len(t)) - 1].z for t in tops if t]))
    recovered = []
    for inj in w.injections:
        j = int(np.searchsorted(w.sub_edges, inj["f0"], side="right")) - 1
        top = tops[j][0]
        recovered.append({"inj_f0": inj["f0"], "inj_amp": inj["amp"], "sub_band": j,
                          "top_z": top.z, "df0_bins": (top.f0 - inj["f0"]) * w.t_sft,
                          "sky_sep_rad": float(np.arccos(np.clip(np.dot(np.array(top.n[:]), inj["sky"]),
                                                                 -1, 1)))})
    line = {
        "metric": "template*SFT evals/s on 1 GPU, plain vs batched; surrogate p_det abs error",
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
        "data": "synthetic: seeded unit-variance complex Gaussian SFT bins (Philox) with 3 "
                "injected signals, analytic Earth orbit+rotation velocities, isotropic sky",
        "config": {"workload": "all-sky band 200-200.5 Hz, 2 det x 5000 SFTs (10%% gaps), "
                               "3 injections h0/sqrt(Sn) 0.05-0.2, 900 f0 x 11 f1 x %d sky, "
                               "K=100 per 0.05 Hz" % args.n_sky,
                   "n_templates": w.n_templates, "n_sft": w.n_sft, "evals_per_step": evals,
                   "tile": tile_name, "lds_window_bins": info.window},
        "kernel_ms": k_ms,
        "select_ms": float(np.mean(sel_ms)),
        "roofline": None,  # filled in below, from the ceilings measured on this device
        "autotune": {"tune_ms": tune_ms,
                     "timed": {e["name"]: e["evals_per_s"] for e in tune_rep},
                     "sample_evals": tune_rep[0]["sample_evals"] if tune_rep else 0},
        "loudest_z": top1.z,
        "injections": recovered,
        "tau_z": tau,
    }
    # Roofline of the dominant kernel (the grid kernel, >= 98% of a step): it is
    # bound by LDS, 4 B gathered per evaluation (the table is 40 MB and stays in
    # the last-level cache; HBM traffic is reported beside it).  The peak is the
    # fastest LDS read form measured on this device with one FP32 add per dword
    # read (what a gather-sum must do), not a vendor figure.
    wtp = (info.window + 63) // 64 * 64
    probe = c.probe_lds_gather(info.tile, wtp)
    achieved_evals = evals / (k_ms * 1e-3)
    lds_forms = {name: c.probe_lds_read(form, True) for name, form in ft.LDS_FORMS.items()}
    lds_forms_one = {name: c.probe_lds_read(form, False) for name, form in ft.LDS_FORMS.items()}
    best_form = max(lds_forms, key=lds_forms.get)
    lds_peak = lds_forms[best_form]
    hbm_read = c.probe_hbm_read(4 << 30)
    lds_nominal = 256 * 128 * 2.4e9  # bytes/s: 128 B per clock per CU
    achieved_Bps = 4.0 * achieved_evals
    traffic = measured_traffic(tile_name) if args.n_sky == 100_000 else None
    line["roofline"] = {
        "bound": "lds", "achieved": achieved_Bps / 1e9, "peak": lds_peak / 1e9, "unit": "GB/s",
        "frac": achieved_Bps / lds_peak, "traffic": traffic,
        "bytes_per_eval": 4.0, "evals_per_launch_step": evals, "kernel_ms": k_ms,
        "peak_source": "ft_probe_lds_read, %s with one add per dword read, measured in this run"
                       % best_form,
        "lds_read_TBps_add_per_dword": {k: v / 1e12 for k, v in lds_forms.items()},
        "lds_read_TBps_add_per_instruction": {k: v / 1e12 for k, v in lds_forms_one.items()},
        "frac_of_tile_pattern_probe": achieved_evals / probe,
        "tile_pattern_probe_evals_per_s": probe,
        "frac_of_nominal_128B_per_clk": achieved_Bps / lds_nominal,
        "hbm": {"measured_read_TBps": hbm_read / 1e12,
                "traffic_TBps": traffic / (k_ms * 1e-3) / 1e12 if traffic else None},
        "valu": {"model_ops_per_eval": ops, "achieved_Tops": achieved, "peak_Tops": peak,
                 "frac": achieved / peak},
        "note": "achieved = 4 B x template-SFT evaluations per step / grid-kernel time per step "
                "(HIP events on the library stream); traffic = HBM bytes per step from rocprofv3 "
                "FETCH_SIZE + WRITE_SIZE, copy-calibrated"}
    log("LDS roofline: kernel %.3g TB/s of %.3g TB/s (%s), %.0f%%; tile-pattern probe %.3g evals/s"
        % (achieved_Bps / 1e12, lds_peak / 1e12, best_form, 100 * achieved_Bps / lds_peak, probe))
    sections = set() if args.skip_extras else set(args.sections.split(","))
    if "weighted" in sections:
        line["weighted"] = bench_weighted(ft, c, w, f0, f1, sky, edges, arms, log)
    c.close()
    if "batched" in sections:
        line["batched"] = bench_batched(ft, synth, args.batched_runs, log)
    if "precision" in sections:
        line["precision"] = bench_precision(ft, synth, log)
    if "surrogate" in sections and args.surrogate_train > 0:
        line["surrogate"] = bench_surrogate(ft, synth, tau, args.surrogate_train,
                                            args.surrogate_test, log)
    if "binary" in sections:
        line["binary"] = bench_binary(ft, synth, log)
    if "mismatch" in sections:
        line["mismatch"] = bench_mismatch(ft, synth, log)
    if "sensitivity" in sections:
        line["sensitivity"] = bench_sensitivity(ft, synth, log)
    if "hyperbox" in sections:
        line["hyperbox"] = bench_hyperbox(ft, synth, log)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a CPU sample")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def report_children():
    """Print to stderr any child process of this one that is still alive."""
    try:
        import psutil
        kids = psutil.Process().children(recursive=True)
    except Exception as e:  # psutil missing or /proc unreadable
        log("child processes at exit: unknown (%s)" % e)
        return
    desc = []
    for k in kids:
        try:
            desc.append("%d %s" % (k.pid, " ".join(k.cmdline()[:4])))
        except Exception:  # gone meanwhile, or not readable
            desc.append("%d ?" % k.pid)
    if desc:
        log("child processes at exit: %s" % ", ".join(desc))


if __name__ == "__main__":
    main()
    report_children()
