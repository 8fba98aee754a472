"""The all-sky band at its full size -- 2 detectors x 5000 SFTs, 900 f0 x 11 f1 x
1e5 sky points (9.9e8 templates), K = 100 in each of 10 sub-bands, 3 injected
signals -- in the launch configuration the benchmark times (autotuned tile).
The plain statistic's toplists are compared bit for bit with the oracle's
evaluation of all 9.9e12 template-SFT pairs (stored under tests/golden/, about
an hour of host time); sampled templates and every toplist member are checked
one by one, and properties that hold at any size cover the rest (no statistic
outside a toplist beats its K-th member beyond the FP32 bound; the injections
are the loudest candidates near them)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "allsky_toplists.json")


def golden_toplists():
    """The oracle's exact toplists of the full band (tests/golden/make_allsky_toplists.py):
    per sub-band, (template index, S64) of its K members in order."""
    with open(GOLDEN) as fh:
        doc = json.load(fh)
    return [[(int(i), float.fromhex(h)) for i, h in top] for top in doc["toplists"]]


def rel_bound(n_sft):
    return 40 * 2.0 ** -24 + 4 * n_sft * 2.0 ** -53


def test_allsky_full_size(ft):
    import torch
    dev = torch.device("cuda:0")
    w = synth.allsky_band(seed=2)
    table = inject.generate_table(2, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                  w.n_bins, w.injections)
    n0, n1, ns = w.f0.size, w.f1.size, w.sky.shape[0]
    n_sub = len(w.sub_edges) - 1
    stats = torch.empty(n0 * n1 * ns, dtype=torch.float32, device=dev)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
                   torch.from_numpy(table).to(dev))
        c.set_velocities(torch.from_numpy(w.v).to(dev))
        c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges, tile=ft.FT_TILE_TUNE,
                         stats=stats)
        tops = [c.toplist(j, w.k) for j in range(n_sub)]
        info = c.info()
    print("tile", ft.ft_tile_name(info.tile), "eval ms", info.eval_ms, flush=True)
    assert info.tile > 0 and info.n_templates == n0 * n1 * ns
    e = rel_bound(w.n_sft)

    # every toplist of the whole bank, bit for bit: the oracle's full FP64
    # evaluation of all 9.9e12 template-SFT pairs, written once on the CPU
    gold = golden_toplists()
    assert len(gold) == n_sub
    for jsub, top in enumerate(tops):
        assert [(t.index, t.s64) for t in top] == gold[jsub], jsub

    # sampled templates and every toplist member against the oracle
    rng = np.random.default_rng(5)
    sample = rng.choice(n0 * n1 * ns, 4000, replace=False)
    members = np.array([t.index for top in tops for t in top], dtype=np.int64)
    idx = np.concatenate([sample, members])
    i, j, s = idx % n0, (idx // n0) % n1, idx // (n0 * n1)
    s64, bad = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v,
                                w.f0[i], w.f1[j], w.sky[s])
    assert bad == -1
    s32 = stats[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    rel = np.abs(s32 - s64) / s64
    assert rel.max() <= e and rel.max() < 1e-5, rel.max()
    mu, sig = oracle.noise_moments(w.n_sft)
    exact = dict(zip(idx.tolist(), s64.tolist()))
    thr = []
    for jsub, top in enumerate(tops):
        assert len(top) == w.k
        for t in top:
            assert t.sub == jsub
            assert w.sub_edges[jsub] <= t.f0 < w.sub_edges[jsub + 1]
            assert t.s64 == exact[t.index]
            assert abs(t.z - (t.s64 - mu) / sig) <= 1e-12 * abs(t.z)
            assert t.f0 == w.f0[t.index % n0] and t.f1 == w.f1[(t.index // n0) % n1]
        keys = [(-t.s64, t.index) for t in top]
        assert keys == sorted(keys)
        thr.append((top[-1].s64, top[-1].index))

    # sampled non-members never beat their sub-band's K-th member
    member_set = set(members.tolist())
    sub_of = np.searchsorted(w.sub_edges, w.f0[i[:len(sample)]], side="right") - 1
    for q, t in enumerate(sample.tolist()):
        jsub = int(sub_of[q])
        if t in member_set or not 0 <= jsub < n_sub:
            continue
        assert (-exact[t], t) > (-thr[jsub][0], thr[jsub][1])

    # every statistic: nothing outside a toplist exceeds its K-th member by
    # more than the FP32 bound
    S = stats.view(ns * n1, n0)
    for jsub, top in enumerate(tops):
        lo = int(np.searchsorted(w.f0, w.sub_edges[jsub], side="left"))
        hi = int(np.searchsorted(w.f0, w.sub_edges[jsub + 1], side="left"))
        block = S[:, lo:hi].clone()
        rows = torch.tensor([t.index // n0 for t in top], device=dev)
        cols = torch.tensor([t.index % n0 - lo for t in top], device=dev)
        block[rows, cols] = -float("inf")
        assert block.max().item() <= thr[jsub][0] * (1 + e)
        del block

    # the injections: each is the loudest candidate of its sub-band, close to it
    f0i = np.array([x["f0"] for x in w.injections])
    f1i = np.array([x["f1"] for x in w.injections])
    skyi = np.array([x["sky"] for x in w.injections])
    s_inj, bad = oracle.eval_list(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v,
                                  f0i, f1i, skyi)
    z_inj = (s_inj - mu) / sig
    for q, x in enumerate(w.injections):
        jsub = int(np.searchsorted(w.sub_edges, x["f0"], side="right")) - 1
        top = tops[jsub][0]
        print("injection", q, "z at injection", z_inj[q], "top z", top.z,
              "df0 bins", (top.f0 - x["f0"]) * w.t_sft, flush=True)
        assert z_inj[q] > 20
        assert top.z >= 0.25 * z_inj[q]
        assert abs(top.f0 - x["f0"]) * w.t_sft <= 3.0


def test_allsky_full_size_number_count_sky_weights(ft):
    """The same band with the weighted number count and the all-sky weights
    (Sec. II.B): sampled templates and every toplist member against the oracle's
    sky weights and indicator table; nothing outside a toplist beats its K-th
    member beyond the FP32 bound."""
    import torch
    from oracle import weighting as ow
    dev = torch.device("cuda:0")
    w = synth.allsky_band(seed=2)
    table = inject.generate_table(2, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                  w.n_bins, w.injections)
    n0, n1, ns = w.f0.size, w.f1.size, w.sky.shape[0]
    n_sub = len(w.sub_edges) - 1
    stats = torch.empty(n0 * n1 * ns, dtype=torch.float32, device=dev)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.set_sfts(w.n_sft_per_det, torch.from_numpy(w.t_mid).to(dev), w.t_sft, w.first_bin,
                   torch.from_numpy(table).to(dev))
        c.set_velocities(torch.from_numpy(w.v).to(dev))
        c.set_arms(torch.from_numpy(w.arms).to(dev))
        c.eval_templates(w.f0, w.f1, w.sky, w.t_ref, w.k, w.sub_edges, stats=stats,
                         statistic=ft.FT_STAT_NUMBER_COUNT, weights=ft.FT_WEIGHTS_SKY)
        tops = [c.toplist(j, w.k) for j in range(n_sub)]
        info = c.info()
    print("tile", ft.ft_tile_name(info.tile), "eval ms", info.eval_ms, flush=True)
    rng = np.random.default_rng(6)
    sample = rng.choice(n0 * n1 * ns, 3000, replace=False)
    members = np.array([t.index for top in tops for t in top], dtype=np.int64)
    idx = np.concatenate([sample, members])
    i, j, s = idx % n0, (idx // n0) % n1, idx // (n0 * n1)
    W = ow.sky_weights(w.arms, None, w.sky[s])
    ind = ow.number_count_table(table)
    S = ow.weighted_sums(w.t_mid, w.t_ref, w.t_sft, w.first_bin, ind, W, w.v, w.f0[i], w.f1[j], w.sky[s])
    s32 = stats[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    e = 44 * 2.0 ** -24 + 4 * w.n_sft * 2.0 ** -53
    assert np.all(np.abs(s32 - S) <= e * S + 1e-13)
    exact = dict(zip(idx.tolist(), S.tolist()))
    wrow = dict(zip(idx.tolist(), range(idx.size)))
    thr = []
    for jsub, top in enumerate(tops):
        assert len(top) == w.k
        for t in top:
            assert t.s64 == exact[t.index]
            mu, sig = ow.nc_moments(W[wrow[t.index]])
            assert t.z == (exact[t.index] - mu) / sig
        keys = [(-t.s64, t.index) for t in top]
        assert keys == sorted(keys)
        thr.append((top[-1].s64, top[-1].index))
    member_set = set(members.tolist())
    sub_of = np.searchsorted(w.sub_edges, w.f0[i[:len(sample)]], side="right") - 1
    for q, t in enumerate(sample.tolist()):
        jsub = int(sub_of[q])
        if t in member_set or not 0 <= jsub < n_sub:
            continue
        assert (-exact[t], t) > (-thr[jsub][0], thr[jsub][1])
    Sg = stats.view(ns * n1, n0)
    for jsub, top in enumerate(tops):
        lo = int(np.searchsorted(w.f0, w.sub_edges[jsub], side="left"))
        hi = int(np.searchsorted(w.f0, w.sub_edges[jsub + 1], side="left"))
        block = Sg[:, lo:hi].clone()
        rows = torch.tensor([t.index // n0 for t in top], device=dev)
        cols = torch.tensor([t.index % n0 - lo for t in top], device=dev)
        block[rows, cols] = -float("inf")
        assert block.max().item() <= thr[jsub][0] * (1 + e)
        del block
