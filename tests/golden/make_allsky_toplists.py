"""Write the exact FP64 toplists of the all-sky band at its full size.

Workload: 2 detectors x 5000 SFTs of 1800 s (10% gaps), 200-200.5 Hz,
900 f0 x 11 f1 x 1e5 isotropic sky points (9.9e8 templates, 9.9e12
template-SFT pairs), K = 100 in each of 10 sub-bands of 0.05 Hz, the table
being seeded Philox noise plus the band's 3 injected signals (seed 2, run 0).

Only the oracle computes here: the table comes from the oracle's generator
(Sec. II.B.2 signal model), every statistic from its plain FP64 sum in SFT
order (Eq. of the short-coherence statistic, Sec. II.B), and each toplist is
the first K templates under (S desc, template index asc).  The sky is walked
in chunks; each chunk's per-sub-band toplist is merged into the running one
under the same total order, so the result equals the toplist of the whole
bank.  Output: tests/golden/allsky_toplists.json with every member's template
index and the bits of its S64 (as a hex string), 10 x 100 entries.

Run from the repository root:  python tests/golden/make_allsky_toplists.py
(about 30-60 min on 8 host threads).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import inject  # noqa: E402
from paper_2411_18370_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "allsky_toplists.json")


def merge(best, idx, s, k):
    """Merge candidate (index, S) pairs into a per-sub-band list, keeping the
    first k under (S desc, index asc)."""
    pairs = best + list(zip(idx.tolist(), s.tolist()))
    pairs.sort(key=lambda p: (-p[1], p[0]))
    return pairs[:k]


def main(chunk=1000, n_sky=100_000):
    w = synth.allsky_band(seed=2, n_sky=n_sky)
    table = inject.generate_table(2, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                  w.n_bins, w.injections)
    n0, n1 = w.f0.size, w.f1.size
    n_sub = len(w.sub_edges) - 1
    per_sky = n0 * n1
    # the sub-band of a template depends on its f0 only
    sub_f0 = oracle.subband(w.f0, w.sub_edges)
    sub_chunk = np.tile(sub_f0, n1 * chunk)
    best = [[] for _ in range(n_sub)]
    t0 = time.time()
    for a in range(0, n_sky, chunk):
        b = min(a + chunk, n_sky)
        s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v,
                                    w.f0, w.f1, w.sky[a:b])
        if bad != -1:
            raise RuntimeError("track out of the table at chunk %d" % a)
        sub = sub_chunk[:s64.size]
        tops = oracle.toplist(s64, sub, n_sub, w.k)
        for j in range(n_sub):
            loc = tops[j]
            best[j] = merge(best[j], loc + a * per_sky, s64[loc], w.k)
        el = time.time() - t0
        print("sky %d/%d  %.0f s  (%.3g evals/s)" % (b, n_sky, el, b * per_sky * w.n_sft / el),
              flush=True)
    doc = {
        "workload": "all-sky band 200-200.5 Hz, 2 det x 5000 SFTs (10%% gaps), 900 f0 x 11 f1 x "
                    "%d sky, 3 injections, K = %d per 0.05 Hz sub-band" % (n_sky, w.k),
        "generator": "synth.allsky_band(seed=2); oracle inject.generate_table(seed 2, run 0)",
        "n_sky": n_sky, "k": w.k, "n_sub": n_sub,
        "toplists": [[[int(i), float(s).hex()] for i, s in best[j]] for j in range(n_sub)],
    }
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        # one line per sub-band: [[index, S64 hex], ...]
        head = {k_: v_ for k_, v_ in doc.items() if k_ != "toplists"}
        f.write(json.dumps(head)[:-1] + ', "toplists": [\n')
        f.write(",\n".join(json.dumps(t) for t in doc["toplists"]) + "\n]}\n")
    os.replace(tmp, OUT)
    print("wrote", OUT, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
