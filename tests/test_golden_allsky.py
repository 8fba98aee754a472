"""The stored full-size toplists of the all-sky band (tests/golden/allsky_toplists.json,
written by tests/golden/make_allsky_toplists.py from the oracle alone) are what the
oracle computes: their shape and order follow the toplist rule (S desc, index asc,
every member in its sub-band), and the first and last member of every sub-band are
re-evaluated here, one template at a time, to the same FP64 bits."""
import json
import os

import numpy as np

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "allsky_toplists.json")


def test_golden_allsky_toplists_are_the_oracles():
    with open(GOLDEN) as fh:
        doc = json.load(fh)
    assert doc["n_sky"] == 100_000 and doc["k"] == 100 and doc["n_sub"] == 10
    w = synth.allsky_band(seed=2)
    n0, n1 = w.f0.size, w.f1.size
    tops = [[(int(i), float.fromhex(h)) for i, h in top] for top in doc["toplists"]]
    assert len(tops) == 10 and all(len(t) == 100 for t in tops)
    idx = []
    for j, top in enumerate(tops):
        keys = [(-s, i) for i, s in top]
        assert keys == sorted(keys) and len(set(i for i, _ in top)) == 100
        for i, _ in top:
            assert 0 <= i < n0 * n1 * 100_000
            assert w.sub_edges[j] <= w.f0[i % n0] < w.sub_edges[j + 1]
        idx += [top[0][0], top[-1][0]]
    table = inject.generate_table(2, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                  w.n_bins, w.injections)
    idx = np.array(idx, dtype=np.int64)
    s64, bad = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v,
                                w.f0[idx % n0], w.f1[(idx // n0) % n1], w.sky[idx // (n0 * n1)])
    assert bad == -1
    want = [s for top in tops for s in (top[0][1], top[-1][1])]
    assert s64.tolist() == want
    # the three loudest sub-bands are the injected ones
    mu, sig = oracle.noise_moments(w.n_sft)
    z1 = np.array([(top[0][1] - mu) / sig for top in tops])
    inj = {int(np.searchsorted(w.sub_edges, x["f0"], side="right")) - 1 for x in w.injections}
    assert set(np.argsort(z1)[-3:].tolist()) == inj and z1.min() > 4
