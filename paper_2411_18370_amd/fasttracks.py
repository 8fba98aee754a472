"""Thin ctypes binding of libfasttracks (C ABI in include/fasttracks.h).

Argument marshalling only: every function forwards to the C entry point of the
same name; arrays may be numpy arrays (host) or torch tensors (host or device),
passed as raw pointers.  All computation happens in the HIP library, which must
be built (``paper_2411_18370_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfasttracks.so")

FT_OK, FT_E_INVALID, FT_E_STATE, FT_E_RANGE, FT_E_NOMEM, FT_E_DEVICE, FT_E_UNSUPPORTED, \
    FT_E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
FT_BANK_GRID, FT_BANK_LIST, FT_BANK_BINARY = 0, 1, 2
FT_INDEX_FP64, FT_INDEX_FP32, FT_INDEX_DF64, FT_INDEX_GUARDED, FT_INDEX_GUARDED_FP32 = 0, 1, 2, 3, 4
FT_SUM_BLOCKED, FT_SUM_PLAIN_FP32 = 0, 1
FT_STAT_POWER, FT_STAT_NUMBER_COUNT = 0, 1
FT_WEIGHTS_SFT, FT_WEIGHTS_SKY = 0, 1
FT_TILE_TUNE = -1
FT_LDS_B32, FT_LDS_READ2ST64, FT_LDS_READ2_ADJ, FT_LDS_B64, FT_LDS_B128, FT_LDS_READ2ST64_B64 = range(6)
LDS_FORMS = {"b32": FT_LDS_B32, "read2st64_b32": FT_LDS_READ2ST64, "read2_b32_adjacent": FT_LDS_READ2_ADJ,
             "b64": FT_LDS_B64, "b128": FT_LDS_B128, "read2st64_b64": FT_LDS_READ2ST64_B64}


class FtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


class ft_bank(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("n_f0", C.c_int64),
                ("n_f1", C.c_int64), ("n_sky", C.c_int64), ("n_list", C.c_int64),
                ("f0", C.c_void_p), ("f1", C.c_void_p), ("sky_xyz", C.c_void_p),
                ("ap", C.c_void_p), ("omega", C.c_void_p), ("phib", C.c_void_p)]


class ft_binary_region(C.Structure):
    _fields_ = [("f0_lo", C.c_double), ("f0_hi", C.c_double), ("ap_lo", C.c_double),
                ("ap_hi", C.c_double), ("omega_lo", C.c_double), ("omega_hi", C.c_double),
                ("alpha_lo", C.c_double), ("alpha_hi", C.c_double), ("sdec_lo", C.c_double),
                ("sdec_hi", C.c_double), ("phib_lo", C.c_double), ("phib_hi", C.c_double)]


FULL_SKY_AND_PHASE = dict(alpha_lo=0.0, alpha_hi=2.0 * np.pi, sdec_lo=-1.0, sdec_hi=1.0, phib_lo=0.0,
                          phib_hi=2.0 * np.pi)


def make_region(d):
    """ft_binary_region from a dict (sky and phase limits default to the whole range)."""
    r = ft_binary_region()
    full = dict(FULL_SKY_AND_PHASE, **d)
    for name, _ in ft_binary_region._fields_:
        setattr(r, name, float(full[name]))
    return r


class ft_eval_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("k", C.c_int32), ("n_sub", C.c_int32),
                ("sum_mode", C.c_int32), ("sub_edges", C.c_void_p), ("tile", C.c_int32),
                ("statistic", C.c_int32), ("weights", C.c_int32), ("reserved", C.c_int32)]


class ft_box_partition(C.Structure):
    _fields_ = [("n_div", C.c_int32 * 6), ("reserved", C.c_int32 * 2)]


class ft_box_result(C.Structure):
    _fields_ = [("index", C.c_int64), ("count", C.c_int32), ("s32", C.c_float), ("s64", C.c_double),
                ("z", C.c_double)]


BOX_DTYPE = np.dtype([("index", np.int64), ("count", np.int32), ("s32", np.float32), ("s64", np.float64),
                      ("z", np.float64)])


class ft_candidate(C.Structure):
    _fields_ = [("index", C.c_int64), ("sub", C.c_int32), ("s32", C.c_float),
                ("f0", C.c_double), ("f1", C.c_double), ("n", C.c_double * 3),
                ("s64", C.c_double), ("z", C.c_double)]


class ft_injection(C.Structure):
    _fields_ = [("amp", C.c_double), ("cos_iota", C.c_double), ("psi", C.c_double),
                ("sky", C.c_double * 3), ("f0", C.c_double), ("f1", C.c_double),
                ("ap", C.c_double), ("omega", C.c_double), ("phib", C.c_double)]


class ft_run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("run_id", C.c_uint32), ("sft_begin", C.c_int32),
                ("n_sft", C.c_int32), ("n_bins", C.c_int32), ("first_bin", C.c_int64),
                ("table_offset", C.c_int64), ("f0_begin", C.c_int32), ("n_f0", C.c_int32),
                ("f1_begin", C.c_int32), ("n_f1", C.c_int32), ("sky_begin", C.c_int32),
                ("n_sky", C.c_int32), ("t_ref", C.c_double), ("inj", ft_injection)]


class ft_batch(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("k", C.c_int32), ("runs", C.c_void_p),
                ("n_sft_total", C.c_int32), ("generate", C.c_int32), ("t_mid", C.c_void_p),
                ("v_over_c", C.c_void_p), ("arms", C.c_void_p), ("t_sft", C.c_double),
                ("n_f0_total", C.c_int64), ("n_f1_total", C.c_int64), ("n_sky_total", C.c_int64),
                ("f0", C.c_void_p), ("f1", C.c_void_p), ("sky_xyz", C.c_void_p),
                ("power_len", C.c_int64), ("power", C.c_void_p), ("tile", C.c_int32),
                ("reserved", C.c_int32)]


class ft_eval_info(C.Structure):
    _fields_ = [("eval_ms", C.c_double), ("select_ms", C.c_double),
                ("n_templates", C.c_int64), ("n_evals", C.c_int64),
                ("n_candidates", C.c_int64), ("tile", C.c_int32), ("window", C.c_int32),
                ("slow_groups", C.c_int64)]


class ft_tune_entry(C.Structure):
    _fields_ = [("klass", C.c_int32), ("tile", C.c_int32), ("chosen", C.c_int32),
                ("reserved", C.c_int32), ("evals_per_s", C.c_double), ("sample_evals", C.c_double)]


_lib = None
EXPORTS = ("ft_create", "ft_destroy", "ft_last_error", "ft_status_string", "ft_set_sfts",
           "ft_set_velocities", "ft_eval_templates", "ft_toplist", "ft_sync",
           "ft_last_eval_info", "ft_bins", "ft_count_index_mismatches",
           "ft_count_index_mismatches_noalloc", "ft_lib_sincos",
           "ft_gen_binary_bank", "ft_eval_binary_random", "ft_q_sample", "ft_tile_count",
           "ft_tile_name", "ft_gen_sfts", "ft_eval_batch", "ft_batch_toplist", "ft_batch_labels",
           "ft_batch_replay", "ft_batch_time", "ft_mlp_create", "ft_mlp_destroy",
           "ft_mlp_get_params", "ft_mlp_predict", "ft_mlp_loss_grad", "ft_mlp_train",
           "ft_tune_report", "ft_tune_clear", "ft_probe_lds_gather", "ft_set_arms",
           "ft_toplist_number_count", "ft_eval_binary_boxes", "ft_binary_cos_mode",
           "ft_probe_lds_read", "ft_probe_hbm_read")


def load(path: str = LIB_PATH):
    """Load libfasttracks.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            "libfasttracks.so is not built (%s); run paper_2411_18370_amd.build.build()" % path)
    lib = C.CDLL(path)
    P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ft_create": (C.c_int, [C.POINTER(P), C.c_int, P]),
        "ft_destroy": (None, [P]),
        "ft_last_error": (C.c_char_p, [P]),
        "ft_status_string": (C.c_char_p, [C.c_int]),
        "ft_set_sfts": (C.c_int, [P, i32, P, P, f64, i64, i32, P, P]),
        "ft_set_velocities": (C.c_int, [P, P]),
        "ft_eval_templates": (C.c_int, [P, C.POINTER(ft_bank), f64, C.POINTER(ft_eval_opts), P]),
        "ft_toplist": (C.c_int, [P, i32, C.POINTER(ft_candidate), C.POINTER(i32)]),
        "ft_sync": (C.c_int, [P]),
        "ft_last_eval_info": (C.c_int, [P, C.POINTER(ft_eval_info)]),
        "ft_bins": (C.c_int, [P, C.POINTER(ft_bank), f64, i32, P]),
        "ft_lib_sincos": (C.c_int, [P, P, i64, P, P]),
        "ft_q_sample": (C.c_int, [P, P, i64, P, P, P, P]),
        "ft_gen_binary_bank": (C.c_int, [P, C.POINTER(ft_binary_region), C.c_uint64, i64, i64, P, P, P,
                                         P, P]),
        "ft_eval_binary_random": (C.c_int, [P, C.POINTER(ft_binary_region), C.c_uint64, i64, f64,
                                            C.POINTER(ft_eval_opts), P]),
        "ft_count_index_mismatches": (C.c_int, [P, C.POINTER(ft_bank), f64, i32,
                                                C.POINTER(i64), C.POINTER(i64)]),
        "ft_count_index_mismatches_noalloc": (C.c_int, [P, C.POINTER(ft_bank), f64, i32,
                                                        C.POINTER(i64), C.POINTER(i64)]),
        "ft_tile_count": (i32, []),
        "ft_gen_sfts": (C.c_int, [P, i32, P, P, f64, i64, i32, P, P, C.c_uint64, C.c_uint32, f64,
                                  C.POINTER(ft_injection), i32, P]),
        "ft_tile_name": (C.c_char_p, [i32]),
        "ft_eval_batch": (C.c_int, [P, C.POINTER(ft_batch), i32]),
        "ft_batch_toplist": (C.c_int, [P, i32, C.POINTER(ft_candidate), C.POINTER(i32)]),
        "ft_batch_labels": (C.c_int, [P, f64, P, P]),
        "ft_batch_replay": (C.c_int, [P]),
        "ft_batch_time": (C.c_int, [P, C.POINTER(f64)]),
        "ft_mlp_create": (C.c_int, [P, P, C.c_uint64, P, P, i32, C.POINTER(P)]),
        "ft_mlp_destroy": (None, [P]),
        "ft_mlp_get_params": (C.c_int, [P, P]),
        "ft_mlp_predict": (C.c_int, [P, P, i64, P]),
        "ft_mlp_loss_grad": (C.c_int, [P, P, P, i32, C.POINTER(C.c_float), P]),
        "ft_mlp_train": (C.c_int, [P, P, P, i64, i32, i32, C.c_float, C.c_uint64, P]),
        "ft_tune_report": (C.c_int, [P, C.POINTER(ft_tune_entry), i32, C.POINTER(i32),
                                     C.POINTER(f64)]),
        "ft_tune_clear": (C.c_int, [P]),
        "ft_probe_lds_gather": (C.c_int, [P, i32, i32, C.POINTER(f64)]),
        "ft_probe_lds_read": (C.c_int, [P, i32, i32, C.POINTER(f64)]),
        "ft_probe_hbm_read": (C.c_int, [P, i64, C.POINTER(f64)]),
        "ft_set_arms": (C.c_int, [P, P]),
        "ft_binary_cos_mode": (C.c_int, [P, i32, C.POINTER(f64)]),
        "ft_eval_binary_boxes": (C.c_int, [P, C.POINTER(ft_binary_region), C.c_uint64, i64, f64,
                                           C.POINTER(ft_box_partition), C.POINTER(ft_eval_opts), P, P]),
        "ft_toplist_number_count": (C.c_int, [P, i32, P, P, C.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_name(st):
    try:
        return load().ft_status_string(st).decode()
    except Exception:
        return str(st)


def _check(ctx, st):
    if st != FT_OK:
        msg = load().ft_last_error(ctx).decode() if ctx else ""
        raise FtError(st, msg)


class _Arr:
    """Pointer to a contiguous numpy array or torch tensor of a required dtype."""

    def __init__(self, a, dtype):
        self.keep = None
        if a is None:
            self.ptr = None
            return
        try:
            import torch
            if isinstance(a, torch.Tensor):
                tdt = {np.float64: torch.float64, np.float32: torch.float32,
                       np.int32: torch.int32, np.int64: torch.int64}[dtype]
                if a.dtype != tdt:
                    raise TypeError("expected %s, got %s" % (tdt, a.dtype))
                a = a.contiguous()
                self.keep = a
                self.ptr = a.data_ptr()
                return
        except ImportError:
            pass
        a = np.ascontiguousarray(a, dtype=dtype)
        self.keep = a
        self.ptr = a.ctypes.data


def ft_create(device: int = 0, stream=None):
    """Create a context; `stream` is a hipStream_t handle (int) or None."""
    lib = load()
    ctx = C.c_void_p()
    st = lib.ft_create(C.byref(ctx), device, C.c_void_p(stream) if stream else None)
    if st != FT_OK:
        raise FtError(st, "ft_create failed")
    return ctx


def ft_destroy(ctx):
    load().ft_destroy(ctx)


def ft_set_sfts(ctx, n_sft_per_det, t_mid, t_sft, first_bin, power, weight=None):
    n = _Arr(np.asarray(n_sft_per_det, np.int32), np.int32)
    tm = _Arr(t_mid, np.float64)
    p = _Arr(power, np.float32)
    w = _Arr(weight, np.float32)
    n_bins = int(power.shape[1])
    _check(ctx, load().ft_set_sfts(ctx, len(n_sft_per_det), n.ptr, tm.ptr, float(t_sft),
                                   int(first_bin), n_bins, p.ptr, w.ptr))


def make_injection(inj):
    """ft_injection from a dict with amp, cos_iota, psi, sky, f0, f1 and, for a
    binary orbit, ap, omega, phib (or None)."""
    if inj is None:
        return None
    r = ft_injection()
    r.amp, r.cos_iota, r.psi = inj["amp"], inj["cos_iota"], inj["psi"]
    for d in range(3):
        r.sky[d] = float(inj["sky"][d])
    r.f0, r.f1 = inj["f0"], inj.get("f1", 0.0)
    r.ap, r.omega, r.phib = inj.get("ap", 0.0), inj.get("omega", 0.0), inj.get("phib", 0.0)
    return r


def ft_gen_sfts(ctx, n_sft_per_det, t_mid, t_sft, first_bin, n_bins, v_over_c, arms, seed, run,
                t_ref, inj=None, power_out=None):
    n = _Arr(np.asarray(n_sft_per_det, np.int32), np.int32)
    tm, v, a = _Arr(t_mid, np.float64), _Arr(v_over_c, np.float64), _Arr(arms, np.float64)
    out = _Arr(power_out, np.float32)
    injs = [] if inj is None else [inj] if isinstance(inj, dict) else list(inj)
    arr = (ft_injection * max(1, len(injs)))(*[make_injection(x) for x in injs])
    _check(ctx, load().ft_gen_sfts(ctx, len(n_sft_per_det), n.ptr, tm.ptr, float(t_sft),
                                   int(first_bin), int(n_bins), v.ptr, a.ptr, int(seed), int(run),
                                   float(t_ref), arr if injs else None, len(injs), out.ptr))


def ft_set_velocities(ctx, v_over_c):
    v = _Arr(v_over_c, np.float64)
    _check(ctx, load().ft_set_velocities(ctx, v.ptr))


def _bank(f0, f1, sky, kind):
    a0, a1, a2 = _Arr(f0, np.float64), _Arr(f1, np.float64), _Arr(sky, np.float64)
    b = ft_bank()
    b.kind = kind
    if kind == FT_BANK_GRID:
        b.n_f0, b.n_f1, b.n_sky = len(f0), len(f1), int(sky.shape[0])
    else:
        b.n_list = len(f0)
    b.f0, b.f1, b.sky_xyz = a0.ptr, a1.ptr, a2.ptr
    return b, (a0, a1, a2)


def _binary_bank(f0, sky, ap, omega, phib):
    arrs = [_Arr(x, np.float64) for x in (f0, sky, ap, omega, phib)]
    b = ft_bank()
    b.kind = FT_BANK_BINARY
    b.n_list = len(f0)
    b.f0, b.sky_xyz, b.ap, b.omega, b.phib = (a.ptr for a in arrs)
    return b, arrs


def ft_eval_binary(ctx, f0, sky, ap, omega, phib, t_ref, k, sub_edges, sum_mode=FT_SUM_BLOCKED,
                   stats=None, statistic=FT_STAT_POWER, weights=FT_WEIGHTS_SFT):
    """Evaluate a BINARY bank (f0, sky[n,3], a_p, Omega, phi_b, each [n]); optional
    `stats` output (float32 [n], host or device)."""
    bank, keep = _binary_bank(f0, sky, ap, omega, phib)
    edges = _Arr(sub_edges, np.float64)
    o = ft_eval_opts()
    o.precision, o.k, o.n_sub, o.sum_mode, o.tile = FT_INDEX_FP64, k, len(sub_edges) - 1, sum_mode, 0
    o.statistic, o.weights = statistic, weights
    o.sub_edges = edges.ptr
    s = _Arr(stats, np.float32)
    _check(ctx, load().ft_eval_templates(ctx, C.byref(bank), float(t_ref), C.byref(o), s.ptr))


def ft_bins_binary(ctx, f0, sky, ap, omega, phib, t_ref):
    """Absolute bins [n, N] (int32) of a BINARY bank."""
    bank, keep = _binary_bank(f0, sky, ap, omega, phib)
    out = np.empty((len(f0), _n_sft_of(ctx)), np.int32)
    _check(ctx, load().ft_bins(ctx, C.byref(bank), float(t_ref), FT_INDEX_FP64,
                               out.ctypes.data_as(C.c_void_p)))
    return out


def ft_gen_binary_bank(ctx, region, seed, first, n):
    """Templates first .. first+n-1 of the random binary bank: (f0, sky [n,3], ap, omega, phib)."""
    reg = make_region(region)
    out = [np.empty(n), np.empty((n, 3)), np.empty(n), np.empty(n), np.empty(n)]
    _check(ctx, load().ft_gen_binary_bank(ctx, C.byref(reg), int(seed), int(first), int(n),
                                          *[a.ctypes.data_as(C.c_void_p) for a in out]))
    return tuple(out)


def ft_eval_binary_random(ctx, region, seed, n, t_ref, k, sub_edges, sum_mode=FT_SUM_BLOCKED,
                          stats=None, statistic=FT_STAT_POWER, weights=FT_WEIGHTS_SFT):
    """Generate templates 0..n-1 of the random binary bank on the device and evaluate them."""
    reg = make_region(region)
    edges = _Arr(sub_edges, np.float64)
    o = ft_eval_opts()
    o.precision, o.k, o.n_sub, o.sum_mode, o.tile = FT_INDEX_FP64, k, len(sub_edges) - 1, sum_mode, 0
    o.statistic, o.weights = statistic, weights
    o.sub_edges = edges.ptr
    s = _Arr(stats, np.float32)
    _check(ctx, load().ft_eval_binary_random(ctx, C.byref(reg), int(seed), int(n), float(t_ref),
                                             C.byref(o), s.ptr))


def ft_eval_binary_boxes(ctx, region, seed, n, t_ref, n_div, statistic=FT_STAT_POWER,
                         sum_mode=FT_SUM_BLOCKED, stats=None):
    """Loudest template of every hyperbox of the random binary bank: numpy array of
    BOX_DTYPE records (index, count, s32, s64, z), one per box in box order."""
    reg = make_region(region)
    part = ft_box_partition()
    for d in range(6):
        part.n_div[d] = int(n_div[d])
    o = ft_eval_opts()
    o.precision, o.sum_mode, o.statistic = FT_INDEX_FP64, sum_mode, statistic
    n_boxes = int(np.prod([int(x) for x in n_div]))
    out = np.zeros(max(1, n_boxes), BOX_DTYPE)
    assert BOX_DTYPE.itemsize == C.sizeof(ft_box_result)
    st = _Arr(stats, np.float32)
    _check(ctx, load().ft_eval_binary_boxes(ctx, C.byref(reg), int(seed), int(n), float(t_ref), C.byref(part),
                                            C.byref(o), out.ctypes.data_as(C.c_void_p), st.ptr))
    return out[:n_boxes]


def ft_q_sample(ctx, arms, sky, cos_iota, psi):
    """q [n, 4] = (mu_G, sigma_G, rho1, rho2) of population samples on the context's SFTs."""
    a = np.ascontiguousarray(arms, np.float64)
    sk = np.ascontiguousarray(sky, np.float64)
    ci = np.ascontiguousarray(cos_iota, np.float64)
    ps = np.ascontiguousarray(psi, np.float64)
    q = np.empty((ci.size, 4))
    _check(ctx, load().ft_q_sample(ctx, a.ctypes.data_as(C.c_void_p), ci.size, sk.ctypes.data_as(C.c_void_p),
                                   ci.ctypes.data_as(C.c_void_p), ps.ctypes.data_as(C.c_void_p),
                                   q.ctypes.data_as(C.c_void_p)))
    return q


def ft_lib_sincos(ctx, x):
    """(cos x, sin x) with the library's FP64 cosine/sine (numpy float64 arrays)."""
    x = np.ascontiguousarray(x, np.float64)
    c = np.empty_like(x)
    s = np.empty_like(x)
    _check(ctx, load().ft_lib_sincos(ctx, x.ctypes.data_as(C.c_void_p), x.size,
                                     c.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p)))
    return c, s


def ft_eval_templates(ctx, f0, f1, sky, t_ref, k, sub_edges, kind=FT_BANK_GRID,
                      precision=FT_INDEX_FP64, sum_mode=FT_SUM_BLOCKED, tile=0, stats=None,
                      statistic=FT_STAT_POWER, weights=FT_WEIGHTS_SFT):
    """Evaluate a GRID (f0[n_f0], f1[n_f1], sky[n_sky,3]) or LIST bank; optional
    `stats` output (float32, n_templates, host or device)."""
    bank, keep = _bank(f0, f1, sky, kind)
    edges = _Arr(sub_edges, np.float64)
    o = ft_eval_opts()
    o.precision, o.k, o.n_sub, o.sum_mode, o.tile = precision, k, len(sub_edges) - 1, \
        sum_mode, tile
    o.statistic, o.weights = statistic, weights
    o.sub_edges = edges.ptr
    s = _Arr(stats, np.float32)
    _check(ctx, load().ft_eval_templates(ctx, C.byref(bank), float(t_ref), C.byref(o), s.ptr))


def ft_toplist(ctx, sub, k):
    """List of ft_candidate records of sub-band `sub` (at most k)."""
    out = (ft_candidate * k)()
    n = C.c_int32()
    _check(ctx, load().ft_toplist(ctx, sub, out, C.byref(n)))
    return [out[i] for i in range(n.value)]


def ft_toplist_number_count(ctx, sub, k):
    """(nc, z_nc): exact weighted number counts (float64) of the entries of sub-band
    `sub`'s toplist and their critical ratios."""
    out = np.empty(max(1, k), np.float64)
    z = np.empty(max(1, k), np.float64)
    n = C.c_int32()
    _check(ctx, load().ft_toplist_number_count(ctx, sub, out.ctypes.data_as(C.c_void_p),
                                               z.ctypes.data_as(C.c_void_p), C.byref(n)))
    return out[:n.value].copy(), z[:n.value].copy()


def ft_binary_cos_mode(ctx, mode):
    """Set the binary-track cosine estimate (0 auto/hardware, 1 polynomial);
    returns the measured error of the hardware cosine."""
    err = C.c_double()
    _check(ctx, load().ft_binary_cos_mode(ctx, int(mode), C.byref(err)))
    return err.value


def ft_set_arms(ctx, arms):
    """Detector arm unit vectors [N, 6] = (u, w) at the SFT mid-times (host or device)."""
    a = _Arr(arms, np.float64)
    _check(ctx, load().ft_set_arms(ctx, a.ptr))


def ft_sync(ctx):
    _check(ctx, load().ft_sync(ctx))


def ft_last_eval_info(ctx):
    info = ft_eval_info()
    _check(ctx, load().ft_last_eval_info(ctx, C.byref(info)))
    return info


def ft_bins(ctx, f0, f1, sky, t_ref, precision=FT_INDEX_FP64):
    """Absolute bins [n_list, N] (int32) of a LIST bank."""
    bank, keep = _bank(f0, f1, sky, FT_BANK_LIST)
    n_sft = _n_sft_of(ctx)
    out = np.empty((len(f0), n_sft), np.int32)
    _check(ctx, load().ft_bins(ctx, C.byref(bank), float(t_ref), precision,
                               out.ctypes.data_as(C.c_void_p)))
    return out


def ft_count_index_mismatches(ctx, f0, f1, sky, t_ref, precision, kind=FT_BANK_GRID, fallback=False):
    """Bins of `precision` that differ from the canonical FP64 bin; with
    fallback=True, (mismatches, evaluations a guarded mode recomputed in FP64)."""
    bank, keep = _bank(f0, f1, sky, kind)
    n = C.c_int64()
    fb = C.c_int64()
    _check(ctx, load().ft_count_index_mismatches(ctx, C.byref(bank), float(t_ref), precision,
                                                 C.byref(n), C.byref(fb)))
    return (int(n.value), int(fb.value)) if fallback else int(n.value)


def ft_count_index_mismatches_noalloc(ctx, f0, f1, sky, t_ref, precision, kind=FT_BANK_GRID):
    """(mismatches, FP64 fallbacks) as ft_count_index_mismatches, with no device
    allocation: f0, f1, sky must be device tensors (read in place)."""
    bank, keep = _bank(f0, f1, sky, kind)
    n = C.c_int64()
    fb = C.c_int64()
    _check(ctx, load().ft_count_index_mismatches_noalloc(ctx, C.byref(bank), float(t_ref), precision,
                                                         C.byref(n), C.byref(fb)))
    return int(n.value), int(fb.value)


def ft_tile_count():
    return int(load().ft_tile_count())


def ft_tune_report(ctx):
    """(entries, tune_ms) of the context's most recent tile tuning; entries are
    dicts with klass, tile, name, chosen, evals_per_s, sample_evals."""
    lib = load()
    n = C.c_int32()
    ms = C.c_double()
    _check(ctx, lib.ft_tune_report(ctx, None, 0, C.byref(n), C.byref(ms)))
    buf = (ft_tune_entry * max(1, n.value))()
    _check(ctx, lib.ft_tune_report(ctx, buf, n.value, C.byref(n), C.byref(ms)))
    out = [{"klass": e.klass, "tile": e.tile, "name": ft_tile_name(e.tile), "chosen": bool(e.chosen),
            "evals_per_s": e.evals_per_s, "sample_evals": e.sample_evals} for e in buf[:n.value]]
    return out, ms.value


def ft_tune_clear(ctx):
    _check(ctx, load().ft_tune_clear(ctx))


def ft_probe_lds_gather(ctx, tile, wtp=0):
    r = C.c_double()
    _check(ctx, load().ft_probe_lds_gather(ctx, int(tile), int(wtp), C.byref(r)))
    return r.value


def ft_probe_lds_read(ctx, form, consume_all=True):
    r = C.c_double()
    _check(ctx, load().ft_probe_lds_read(ctx, int(form), int(bool(consume_all)), C.byref(r)))
    return r.value


def ft_probe_hbm_read(ctx, n_bytes=4 << 30):
    r = C.c_double()
    _check(ctx, load().ft_probe_hbm_read(ctx, int(n_bytes), C.byref(r)))
    return r.value


def ft_tile_name(tile):
    return load().ft_tile_name(tile).decode()


RUN_DTYPE = np.dtype([("seed", "<u8"), ("run_id", "<u4"), ("sft_begin", "<i4"),
                      ("n_sft", "<i4"), ("n_bins", "<i4"), ("first_bin", "<i8"),
                      ("table_offset", "<i8"), ("f0_begin", "<i4"), ("n_f0", "<i4"),
                      ("f1_begin", "<i4"), ("n_f1", "<i4"), ("sky_begin", "<i4"),
                      ("n_sky", "<i4"), ("t_ref", "<f8"), ("amp", "<f8"), ("cos_iota", "<f8"),
                      ("psi", "<f8"), ("inj_sky", "<f8", (3,)), ("inj_f0", "<f8"),
                      ("inj_f1", "<f8"), ("inj_ap", "<f8"), ("inj_omega", "<f8"),
                      ("inj_phib", "<f8")], align=True)


def make_runs(runs):
    """ft_run array from a list of dicts (keys as the C fields; 'inj' a dict or
    None) or from a dict of columns (injection columns amp, cos_iota, psi,
    inj_sky, inj_f0, inj_f1)."""
    if isinstance(runs, dict):
        n = len(runs["seed"])
        arr = np.zeros(n, RUN_DTYPE)
        for name in RUN_DTYPE.names:
            if name in runs:
                arr[name] = runs[name]
        assert arr.itemsize == C.sizeof(ft_run)
        return arr
    arr = (ft_run * len(runs))()
    for i, d in enumerate(runs):
        r = arr[i]
        r.seed, r.run_id = int(d.get("seed", 0)), int(d.get("run_id", i))
        r.sft_begin, r.n_sft = int(d["sft_begin"]), int(d["n_sft"])
        r.n_bins, r.first_bin = int(d["n_bins"]), int(d["first_bin"])
        r.table_offset = int(d.get("table_offset", 0))
        r.f0_begin, r.n_f0 = int(d["f0_begin"]), int(d["n_f0"])
        r.f1_begin, r.n_f1 = int(d["f1_begin"]), int(d["n_f1"])
        r.sky_begin, r.n_sky = int(d["sky_begin"]), int(d["n_sky"])
        r.t_ref = float(d["t_ref"])
        if d.get("inj") is not None:
            r.inj = make_injection(d["inj"])
    return arr


def ft_eval_batch(ctx, runs, t_mid, v_over_c, t_sft, f0, f1, sky, k, arms=None, power=None,
                  tile=0, use_graph=0):
    """Evaluate a batch; runs is a list of dicts (see make_runs).  Tables are
    generated on the GPU when `power` is None (arms required)."""
    keep = [_Arr(t_mid, np.float64), _Arr(v_over_c, np.float64), _Arr(arms, np.float64),
            _Arr(f0, np.float64), _Arr(f1, np.float64), _Arr(sky, np.float64),
            _Arr(power, np.float32)]
    rr = make_runs(runs)
    b = ft_batch()
    n_runs = len(rr)
    b.n_runs, b.k = n_runs, int(k)
    b.runs = rr.ctypes.data if isinstance(rr, np.ndarray) else C.cast(rr, C.c_void_p)
    b.n_sft_total = len(t_mid)
    b.generate = 1 if power is None else 0
    b.t_mid, b.v_over_c, b.arms = keep[0].ptr, keep[1].ptr, keep[2].ptr
    b.t_sft = float(t_sft)
    b.n_f0_total, b.n_f1_total, b.n_sky_total = len(f0), len(f1), int(sky.shape[0])
    b.f0, b.f1, b.sky_xyz = keep[3].ptr, keep[4].ptr, keep[5].ptr
    b.power_len = 0 if power is None else int(np.prod(power.shape))
    b.power = keep[6].ptr
    b.tile = tile
    _check(ctx, load().ft_eval_batch(ctx, C.byref(b), int(use_graph)))


def ft_batch_toplist(ctx, run, k):
    out = (ft_candidate * k)()
    n = C.c_int32()
    _check(ctx, load().ft_batch_toplist(ctx, run, out, C.byref(n)))
    return [out[i] for i in range(n.value)]


def ft_batch_labels(ctx, tau, n_runs):
    labels = np.empty(n_runs, np.uint8)
    max_z = np.empty(n_runs, np.float64)
    _check(ctx, load().ft_batch_labels(ctx, float(tau), labels.ctypes.data_as(C.c_void_p),
                                       max_z.ctypes.data_as(C.c_void_p)))
    return labels, max_z


def ft_batch_replay(ctx):
    _check(ctx, load().ft_batch_replay(ctx))


def ft_batch_time(ctx):
    ms = C.c_double()
    _check(ctx, load().ft_batch_time(ctx, C.byref(ms)))
    return ms.value


MLP_N_PARAMS = 133_633


class Mlp:
    """The p_det surrogate network (ft_mlp_*)."""

    def __init__(self, ctx, feat_shift, feat_scale, max_batch=8192, params=None, seed=0):
        self.ctx = ctx.ctx if isinstance(ctx, Context) else ctx
        self._p = None
        sh = _Arr(np.asarray(feat_shift, np.float32), np.float32)
        sc = _Arr(np.asarray(feat_scale, np.float32), np.float32)
        pr = _Arr(params, np.float32)
        h = C.c_void_p()
        _check(self.ctx, load().ft_mlp_create(self.ctx, pr.ptr, int(seed), sh.ptr, sc.ptr,
                                              int(max_batch), C.byref(h)))
        self._p = h

    def close(self):
        if self._p:
            load().ft_mlp_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.empty(MLP_N_PARAMS, np.float32)
        _check(self.ctx, load().ft_mlp_get_params(self._p, out.ctypes.data_as(C.c_void_p)))
        return out

    def predict(self, raw):
        raw = np.ascontiguousarray(raw, np.float32)
        out = np.empty(raw.shape[0], np.float32)
        _check(self.ctx, load().ft_mlp_predict(self._p, raw.ctypes.data_as(C.c_void_p),
                                               raw.shape[0], out.ctypes.data_as(C.c_void_p)))
        return out

    def loss_grad(self, raw, y):
        raw = np.ascontiguousarray(raw, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        loss = C.c_float()
        g = np.empty(MLP_N_PARAMS, np.float32)
        _check(self.ctx, load().ft_mlp_loss_grad(self._p, raw.ctypes.data_as(C.c_void_p),
                                                 y.ctypes.data_as(C.c_void_p), raw.shape[0],
                                                 C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def train(self, raw, y, batch, epochs, lr, seed=0):
        raw = _Arr(raw, np.float32)
        yy = _Arr(y, np.float32)
        n = int(raw.keep.shape[0])
        hist = np.empty(max(epochs, 1), np.float32)
        _check(self.ctx, load().ft_mlp_train(self._p, raw.ptr, yy.ptr, n, int(batch), int(epochs),
                                             float(lr), int(seed),
                                             hist.ctypes.data_as(C.c_void_p)))
        return hist[:epochs]


_n_sft_cache = {}


def _n_sft_of(ctx):
    return _n_sft_cache[ctx.value]


# ---------------------------------------------------------------------------
# Convenience wrapper holding a context and the SFT count.
# ---------------------------------------------------------------------------
class Context:
    def __init__(self, device=0, stream=None):
        self.ctx = ft_create(device, stream)

    def close(self):
        if self.ctx:
            _n_sft_cache.pop(self.ctx.value, None)
            ft_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_sfts(self, n_sft_per_det, t_mid, t_sft, first_bin, power, weight=None):
        ft_set_sfts(self.ctx, n_sft_per_det, t_mid, t_sft, first_bin, power, weight)
        _n_sft_cache[self.ctx.value] = int(sum(n_sft_per_det))

    def set_velocities(self, v):
        ft_set_velocities(self.ctx, v)

    def set_arms(self, arms):
        ft_set_arms(self.ctx, arms)

    def binary_cos_mode(self, mode):
        return ft_binary_cos_mode(self.ctx, mode)

    def toplist_number_count(self, sub, k):
        return ft_toplist_number_count(self.ctx, sub, k)

    def gen_sfts(self, n_sft_per_det, t_mid, t_sft, first_bin, n_bins, v, arms, seed, run, t_ref,
                 inj=None, power_out=None):
        ft_gen_sfts(self.ctx, n_sft_per_det, t_mid, t_sft, first_bin, n_bins, v, arms, seed, run,
                    t_ref, inj, power_out)
        _n_sft_cache[self.ctx.value] = int(sum(n_sft_per_det))

    def eval_templates(self, *a, **kw):
        ft_eval_templates(self.ctx, *a, **kw)

    def toplist(self, sub, k):
        return ft_toplist(self.ctx, sub, k)

    def sync(self):
        ft_sync(self.ctx)

    def info(self):
        return ft_last_eval_info(self.ctx)

    def bins(self, *a, **kw):
        return ft_bins(self.ctx, *a, **kw)

    def eval_binary(self, *a, **kw):
        ft_eval_binary(self.ctx, *a, **kw)

    def bins_binary(self, *a, **kw):
        return ft_bins_binary(self.ctx, *a, **kw)

    def lib_sincos(self, x):
        return ft_lib_sincos(self.ctx, x)

    def q_sample(self, *a, **kw):
        return ft_q_sample(self.ctx, *a, **kw)

    def gen_binary_bank(self, *a, **kw):
        return ft_gen_binary_bank(self.ctx, *a, **kw)

    def eval_binary_random(self, *a, **kw):
        ft_eval_binary_random(self.ctx, *a, **kw)

    def eval_binary_boxes(self, *a, **kw):
        return ft_eval_binary_boxes(self.ctx, *a, **kw)

    def count_index_mismatches(self, *a, **kw):
        return ft_count_index_mismatches(self.ctx, *a, **kw)

    def count_index_mismatches_noalloc(self, *a, **kw):
        return ft_count_index_mismatches_noalloc(self.ctx, *a, **kw)

    def eval_batch(self, *a, **kw):
        ft_eval_batch(self.ctx, *a, **kw)

    def batch_toplist(self, run, k):
        return ft_batch_toplist(self.ctx, run, k)

    def batch_labels(self, tau, n_runs):
        return ft_batch_labels(self.ctx, tau, n_runs)

    def batch_replay(self):
        ft_batch_replay(self.ctx)

    def batch_time(self):
        return ft_batch_time(self.ctx)

    def tune_report(self):
        return ft_tune_report(self.ctx)

    def tune_clear(self):
        ft_tune_clear(self.ctx)

    def probe_lds_gather(self, tile, wtp=0):
        return ft_probe_lds_gather(self.ctx, tile, wtp)

    def probe_lds_read(self, form, consume_all=True):
        return ft_probe_lds_read(self.ctx, form, consume_all)

    def probe_hbm_read(self, n_bytes=4 << 30):
        return ft_probe_hbm_read(self.ctx, n_bytes)

    def eval_campaign(self, cp, use_graph=0, tile=0, power=None):
        """Evaluate a synth.Campaign (tables generated on the GPU unless given)."""
        ft_eval_batch(self.ctx, cp.runs, cp.t_mid, cp.v, cp.t_sft, cp.f0, cp.f1, cp.sky, cp.k,
                      arms=cp.arms, power=power, tile=tile, use_graph=use_graph)

    def load_workload(self, w):
        """Upload a synth.Workload's SFTs and velocities."""
        self.set_sfts(w.n_sft_per_det, w.t_mid, w.t_sft, w.first_bin, w.power, w.weight)
        self.set_velocities(w.v)
