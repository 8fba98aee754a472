"""ctypes wrapper around the FP64 oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ft_oracle.c")
_LIB = os.path.join(_HERE, "libft_oracle.so")
_lock = threading.Lock()
_lib = None

# -O2 with FMA contraction and fast-math explicitly off: the oracle's operation
# order is the canonical one and must not be fused or reassociated.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fno-unsafe-math-optimizations"]


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile ft_oracle.c with gcc into oracle/libft_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = C.CDLL(_LIB)
            P = C.c_void_p
            i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
            lib.ftor_bins_list.argtypes = [i32, P, f64, f64, P, i64, P, P, P, P]
            lib.ftor_eval_list.argtypes = [i32, P, f64, f64, i64, i32, P, P, P, i64, P, P, P, P, P]
            lib.ftor_eval_grid.argtypes = [i32, P, f64, f64, i64, i32, P, P, P, i64, P, i64, P,
                                           i64, P, P, P]
            lib.ftor_pcos.argtypes = [i64, P, P, P]
            lib.ftor_pcos.restype = None
            lib.ftor_plog.argtypes = [i64, P, P]
            lib.ftor_plog.restype = None
            u32, u64 = C.c_uint32, C.c_uint64
            lib.ftor_philox.argtypes = [i64, P, u32, u32, P]
            lib.ftor_philox.restype = None
            lib.ftor_noise_normals.argtypes = [u64, u32, i32, i32, i64, P, P]
            lib.ftor_noise_normals.restype = None
            lib.ftor_gen_table.argtypes = [u64, u32, i32, i32, i64, i64, i32, P, P, P]
            lib.ftor_gen_table.restype = None
            lib.ftor_bins_binary.argtypes = [i32, P, f64, f64, P, i64, P, P, P, P, P, P]
            lib.ftor_eval_binary.argtypes = [i32, P, f64, f64, i64, i32, P, P, P, i64, P, P, P, P, P,
                                             P, P]
            lib.ftor_bins_binary.restype = C.c_int
            lib.ftor_eval_binary.restype = C.c_int
            lib.ftor_noise_moments.argtypes = [i32, P, P, P]
            lib.ftor_critical_ratio.argtypes = [i64, P, i32, P, P]
            lib.ftor_subband.argtypes = [i64, P, i32, P, P]
            lib.ftor_toplist.argtypes = [i64, P, P, i32, i32, P, P]
            for name in ("ftor_bins_list", "ftor_eval_list", "ftor_eval_grid", "ftor_toplist"):
                getattr(lib, name).restype = C.c_int
            lib.ftor_noise_moments.restype = None
            lib.ftor_critical_ratio.restype = None
            lib.ftor_subband.restype = None
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def bins_list(t_mid, t_ref, t_sft, v, f0, f1, sky):
    """Absolute bin indices [n_tmpl, n_sft] (int64) of a template list."""
    lib = _load()
    t_mid, v, f0, f1, sky = map(_f64, (t_mid, v, f0, f1, sky))
    n = f0.size
    out = np.empty((n, t_mid.size), np.int64)
    rc = lib.ftor_bins_list(t_mid.size, _p(t_mid), t_ref, t_sft, _p(v), n, _p(f0), _p(f1),
                            _p(sky), _p(out))
    if rc != 0:
        raise ValueError("ftor_bins_list failed: %d" % rc)
    return out


def eval_list(t_mid, t_ref, t_sft, first_bin, power, weight, v, f0, f1, sky):
    """(S64 [n_tmpl], first_bad) for a template list."""
    lib = _load()
    t_mid, v, f0, f1, sky = map(_f64, (t_mid, v, f0, f1, sky))
    power = _f32(power)
    weight = _f32(weight)
    n = f0.size
    out = np.empty(n, np.float64)
    bad = C.c_int64(-1)
    rc = lib.ftor_eval_list(t_mid.size, _p(t_mid), t_ref, t_sft, first_bin, power.shape[1],
                            _p(power), _p(weight), _p(v), n, _p(f0), _p(f1), _p(sky), _p(out),
                            C.byref(bad))
    if rc not in (0, -3):
        raise ValueError("ftor_eval_list failed: %d" % rc)
    return out, int(bad.value)


def eval_grid(t_mid, t_ref, t_sft, first_bin, power, weight, v, f0, f1, sky):
    """(S64 [n_sky*n_f1*n_f0], first_bad) for a grid bank, index (s*n_f1+j)*n_f0+i."""
    lib = _load()
    t_mid, v, f0, f1, sky = map(_f64, (t_mid, v, f0, f1, sky))
    power = _f32(power)
    weight = _f32(weight)
    out = np.empty(f0.size * f1.size * sky.shape[0], np.float64)
    bad = C.c_int64(-1)
    rc = lib.ftor_eval_grid(t_mid.size, _p(t_mid), t_ref, t_sft, first_bin, power.shape[1],
                            _p(power), _p(weight), _p(v), f0.size, _p(f0), f1.size, _p(f1),
                            sky.shape[0], _p(sky), _p(out), C.byref(bad))
    if rc not in (0, -3):
        raise ValueError("ftor_eval_grid failed: %d" % rc)
    return out, int(bad.value)


def noise_moments(n_sft, weight=None):
    lib = _load()
    weight = _f32(weight)
    mu, sig = C.c_double(), C.c_double()
    lib.ftor_noise_moments(n_sft, _p(weight), C.byref(mu), C.byref(sig))
    return mu.value, sig.value


def critical_ratio(s, n_sft, weight=None):
    lib = _load()
    s = _f64(s)
    weight = _f32(weight)
    z = np.empty_like(s)
    lib.ftor_critical_ratio(s.size, _p(s), n_sft, _p(weight), _p(z))
    return z


def subband(f, edges):
    lib = _load()
    f, edges = _f64(f), _f64(edges)
    out = np.empty(f.size, np.int32)
    lib.ftor_subband(f.size, _p(f), edges.size - 1, _p(edges), _p(out))
    return out


def toplist(s, sub, n_sub, k):
    """Per sub-band list of template indices under (S desc, index asc)."""
    lib = _load()
    s = _f64(s)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    idx = np.empty(n_sub * k, np.int64)
    cnt = np.empty(n_sub, np.int32)
    rc = lib.ftor_toplist(s.size, _p(s), _p(sub), n_sub, k, _p(idx), _p(cnt))
    if rc != 0:
        raise ValueError("ftor_toplist failed: %d" % rc)
    idx = idx.reshape(n_sub, k)
    return [idx[j, :cnt[j]].copy() for j in range(n_sub)]


def grid_params(f0, f1, n_sky):
    """Per-template (f0, f1, sky index) arrays of a grid bank in template order."""
    f0 = np.asarray(f0, np.float64)
    f1 = np.asarray(f1, np.float64)
    i = np.tile(np.arange(f0.size), f1.size * n_sky)
    j = np.tile(np.repeat(np.arange(f1.size), f0.size), n_sky)
    s = np.repeat(np.arange(n_sky), f0.size * f1.size)
    return f0[i], f1[j], s


def pcos(x):
    """(cos x, sin x) with the project's FP64 cosine/sine (|x| < 1.6e6)."""
    lib = _load()
    x = _f64(x)
    c = np.empty_like(x)
    s = np.empty_like(x)
    lib.ftor_pcos(x.size, _p(x), _p(c), _p(s))
    return c, s


def plog(x):
    """The project's FP64 natural logarithm (finite normal x > 0)."""
    lib = _load()
    x = _f64(x)
    out = np.empty_like(x)
    lib.ftor_plog(x.size, _p(x), _p(out))
    return out


def philox(ctr, key):
    """Philox-4x32-10 words [..., 4] (uint32) of counters ctr [..., 4] under key (k0, k1)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.empty_like(c)
    lib.ftor_philox(c.size // 4, _p(c), int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF, _p(out))
    return out


def noise_normals(seed, run, n_sft, n_bins, sft_offset=0):
    """(Re, Im) [n_sft, n_bins] of one run's campaign noise (the C generator)."""
    lib = _load()
    re = np.empty((n_sft, n_bins))
    im = np.empty((n_sft, n_bins))
    lib.ftor_noise_normals(int(seed) & (2**64 - 1), int(run) & 0xFFFFFFFF, n_sft, n_bins, sft_offset,
                           _p(re), _p(im))
    return re, im


def gen_table(seed, run, n_sft, n_bins, sft_offset, first_bin, bins, amps):
    """FP32 power table [n_sft, n_bins]: noise plus signals with absolute bins
    bins [n_inj, n_sft] (int64, INT64_MIN for none) and Re amplitudes amps
    [n_inj, n_sft, 3] at bins - 1, bins, bins + 1."""
    lib = _load()
    bins = np.ascontiguousarray(bins, dtype=np.int64).reshape(-1, n_sft)
    amps = np.ascontiguousarray(amps, dtype=np.float64).reshape(-1, n_sft, 3)
    out = np.empty((n_sft, n_bins), np.float32)
    lib.ftor_gen_table(int(seed) & (2**64 - 1), int(run) & 0xFFFFFFFF, n_sft, n_bins, sft_offset,
                       int(first_bin), bins.shape[0], _p(bins), _p(amps), _p(out))
    return out


def bins_binary(t_mid, t_ref, t_sft, v, f0, sky, ap, omega, phib):
    """Absolute bins [n_tmpl, n_sft] (int64) of binary-system templates."""
    lib = _load()
    t_mid, v, f0, sky, ap, omega, phib = map(_f64, (t_mid, v, f0, sky, ap, omega, phib))
    n = f0.size
    out = np.empty((n, t_mid.size), np.int64)
    rc = lib.ftor_bins_binary(t_mid.size, _p(t_mid), t_ref, t_sft, _p(v), n, _p(f0), _p(sky), _p(ap),
                              _p(omega), _p(phib), _p(out))
    if rc != 0:
        raise ValueError("ftor_bins_binary failed: %d" % rc)
    return out


def eval_binary(t_mid, t_ref, t_sft, first_bin, power, weight, v, f0, sky, ap, omega, phib):
    """(S64 [n_tmpl], first_bad) for binary-system templates."""
    lib = _load()
    t_mid, v, f0, sky, ap, omega, phib = map(_f64, (t_mid, v, f0, sky, ap, omega, phib))
    power = _f32(power)
    weight = _f32(weight)
    n = f0.size
    out = np.empty(n, np.float64)
    bad = C.c_int64(-1)
    rc = lib.ftor_eval_binary(t_mid.size, _p(t_mid), t_ref, t_sft, first_bin, power.shape[1], _p(power),
                              _p(weight), _p(v), n, _p(f0), _p(sky), _p(ap), _p(omega), _p(phib), _p(out),
                              C.byref(bad))
    if rc not in (0, -3):
        raise ValueError("ftor_eval_binary failed: %d" % rc)
    return out, bad.value
