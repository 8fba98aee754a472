"""Parity of the GPU campaign generator with the oracle's FP64 twin.

Both sides draw the same Philox-4x32-10 words (integer arithmetic, exact) and
evaluate the same fixed sequence of IEEE operations: the project's logarithm,
cosine and sine (each side its own implementation of the one published
sequence), dot products in one order, correctly rounded square roots and
divisions.  So the FP32 tables agree bit for bit, and injection bins come from
the canonical FP64 track on both sides.
"""
import numpy as np
import pytest

import oracle
from oracle import inject
from paper_2411_18370_amd import synth

pytestmark = pytest.mark.gpu


def _gen_gpu(ft, w, seed, run, inj):
    import torch
    out = np.empty((w.n_sft, w.n_bins), np.float32)
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.gen_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.n_bins, w.v, w.arms, seed,
                   run, w.t_ref, inj, power_out=out)
    return out


def _assert_tables_equal(got, want):
    assert got.shape == want.shape
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), int(np.sum(got != want))


@pytest.mark.parametrize("amp", [0.0, 0.1, 3.0])
def test_generated_table_matches_oracle(ft, amp):
    w = synth.allsky_band(seed=31, n_sky=1, n_per_det=150)
    rng = np.random.default_rng(32)
    inj = synth.injection_params(rng, 200.1, 200.4, amp, amp, -1e-9, 0.0)
    seed, run = 0xDEADBEEF12345, 77
    got = _gen_gpu(ft, w, seed, run, inj)
    want = inject.generate_table(seed, run, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                 w.n_bins, inj)
    _assert_tables_equal(got, want)


def test_several_injections_superpose_like_the_oracle(ft):
    """Three signals, one with amp 0 and two sharing SFT bins (equal f0 and sky):
    the GPU adds them in the given order like the oracle."""
    w = synth.allsky_band(seed=33, n_sky=1, n_per_det=120)
    rng = np.random.default_rng(34)
    a = synth.injection_params(rng, 200.1, 200.4, 2.0, 2.0, -1e-9, 0.0)
    b = dict(synth.injection_params(rng, 200.1, 200.4, 1.5, 1.5, -1e-9, 0.0),
             f0=a["f0"], sky=a["sky"])
    z = synth.injection_params(rng, 200.1, 200.4, 0.0, 0.0)
    seed, run = 99, 3
    got = _gen_gpu(ft, w, seed, run, [a, z, b])
    want = inject.generate_table(seed, run, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                 w.n_bins, [a, z, b])
    _assert_tables_equal(got, want)
    one = inject.generate_table(seed, run, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                w.n_bins, a)
    assert np.sum(want != one) > w.n_sft  # the second signal changed the table


def test_generated_campaign_toplist_recovers_injection(ft):
    """Generate with a loud injection, evaluate a local bank around it: the
    loudest template's FP64 statistic matches the oracle on its own table."""
    import torch
    w = synth.allsky_band(seed=33, n_sky=1, n_per_det=300)
    rng = np.random.default_rng(34)
    inj = synth.injection_params(rng, 200.2, 200.3, 0.3, 0.3, -1e-9, 0.0)
    i0 = int(round((inj["f0"] - w.f0[0]) * w.t_sft))
    f0 = w.f0[max(0, i0 - 3):i0 + 4]
    f1 = np.linspace(-1e-9, 0.0, 11)
    sky = np.vstack([inj["sky"], synth.isotropic_sky(7, rng)])
    edges = np.array([f0[0] - 1e-6, f0[-1] + 1e-6])
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.gen_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.n_bins, w.v, w.arms, 5, 0,
                   w.t_ref, inj)
        c.eval_templates(f0, f1, sky, w.t_ref, 5, edges)
        top = c.toplist(0, 5)
    table = inject.generate_table(5, 0, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                  w.n_bins, inj)
    s64, bad = oracle.eval_grid(w.t_mid, w.t_ref, w.t_sft, w.first_bin, table, None, w.v, f0, f1,
                                sky)
    assert bad == -1
    order = sorted(range(s64.size), key=lambda t: (-s64[t], t))
    assert top[0].index == order[0]
    assert [c_.index for c_ in top] == order[:len(top)]
    for c_ in top:
        assert c_.s64 == s64[c_.index]
    # the injection is loud: the loudest template sits at the injected sky point
    assert top[0].index // (len(f0) * len(f1)) == 0 and top[0].z > 20


def test_binary_injection_matches_oracle(ft):
    """A source in a circular binary orbit (Eq. track with a_p > 0): the table
    matches the oracle's, and the BINARY template at the signal's parameters
    collects the signal (its statistic equals the oracle's, far above noise)."""
    import torch
    w = synth.binary_band(seed=35, n_tmpl=1, n_per_det=200)
    rng = np.random.default_rng(36)
    inj = synth.injection_params(rng, w.region["f0_lo"] + 0.03, w.region["f0_hi"] - 0.03, 2.0, 2.0)
    inj = dict(inj, f1=0.0, ap=11.3, omega=2 * np.pi / (9.7 * 86400.0), phib=1.234)
    seed, run = 4242, 5
    got = _gen_gpu(ft, w, seed, run, inj)
    want = inject.generate_table(seed, run, w.t_mid, w.t_ref, w.t_sft, w.v, w.arms, w.first_bin,
                                 w.n_bins, inj)
    _assert_tables_equal(got, want)
    one = lambda x: np.array([x], np.float64)
    s64, bad = oracle.eval_binary(w.t_mid, w.t_ref, w.t_sft, w.first_bin, want, None, w.v, one(inj["f0"]),
                                  np.asarray(inj["sky"])[None, :], one(inj["ap"]), one(inj["omega"]),
                                  one(inj["phib"]))
    mu, sig = oracle.noise_moments(w.n_sft)
    assert bad == -1 and (s64[0] - mu) / sig > 20
    with ft.Context(0, torch.cuda.current_stream().cuda_stream) as c:
        c.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, got)
        c.set_velocities(w.v)
        c.eval_binary(one(inj["f0"]), np.asarray(inj["sky"])[None, :], one(inj["ap"]), one(inj["omega"]),
                      one(inj["phib"]), w.t_ref, 1, np.array([w.region["f0_lo"], w.region["f0_hi"]]))
        top = c.toplist(0, 1)
    assert top[0].s64 == s64[0]
