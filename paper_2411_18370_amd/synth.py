"""Seeded synthetic inputs shaped like the paper's all-sky short-coherence search.

This module produces *inputs only*: SFT mid-times with gaps, detector velocities
from an analytic Earth orbit plus rotation, isotropic sky points, template-bank
grids and unit-variance complex-Gaussian noise power.  It holds none of the
method's arithmetic (no track, no bin index, no statistic, no signal model), so
both the FP64 oracle and the GPU library can consume what it produces.

Physical model of the inputs (Sec. II of the paper uses real LVK SFTs; these
stand in for them):

* SFTs have duration ``t_sft``; a detector observes on a grid of consecutive
  slots, of which a seeded uniform random subset is present (gaps are allowed,
  Sec. II.B footnote on timestamps).  Timestamps are slot *mid-times*.
* Detector velocity ``v/c`` in equatorial Cartesian coordinates: circular
  heliocentric orbit (1 AU, sidereal year, obliquity 23.4393 deg) plus the
  detector's rotation with the Earth (sidereal day, equatorial radius).
* Isotropic sky: right ascension uniform in [0, 2 pi), sin(declination)
  uniform in [-1, 1] (App. A parametrisation of the sky).
* Noise power: Re, Im ~ N(0, 1) i.i.d. per bin, power = Re^2 + Im^2, so each
  bin is chi^2 with 2 degrees of freedom (Eq. s_chi2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0
AU = 1.495978707e11
SIDEREAL_YEAR = 365.256363004 * 86400.0
SIDEREAL_DAY = 86164.0905
R_EARTH = 6.378137e6
OBLIQUITY = math.radians(23.4393)
EPOCH = 1.2e9  # GPS-like start of observation [s]


@dataclass(frozen=True)
class Detector:
    """A synthetic ground-based interferometer (geometry loosely LIGO-like)."""
    name: str
    lat_deg: float
    lon_deg: float
    arm_azimuths_deg: tuple  # azimuths of the two arms, from North towards East


DETECTORS = (
    Detector("H1-like", 46.455, -119.408, (125.9994, 215.9994)),
    Detector("L1-like", 30.563, -90.774, (197.7165, 287.7165)),
)


def sidereal_angle(t: np.ndarray, lon_deg: float) -> np.ndarray:
    """Local sidereal angle of a detector at time t (zero at EPOCH for lon 0)."""
    return 2.0 * np.pi * (t - EPOCH) / SIDEREAL_DAY + math.radians(lon_deg)


def detector_velocity(t_mid: np.ndarray, det: Detector) -> np.ndarray:
    """v/c [N,3] (equatorial) at the SFT mid-times: orbit + rotation."""
    t = np.asarray(t_mid, dtype=np.float64)
    v_orb = 2.0 * np.pi * AU / SIDEREAL_YEAR
    lam = 2.0 * np.pi * (t - EPOCH) / SIDEREAL_YEAR + 0.3  # ecliptic longitude
    vx_e = -v_orb * np.sin(lam)
    vy_e = v_orb * np.cos(lam)
    # ecliptic -> equatorial: rotation about x by the obliquity
    vx = vx_e
    vy = vy_e * math.cos(OBLIQUITY)
    vz = vy_e * math.sin(OBLIQUITY)
    th = sidereal_angle(t, det.lon_deg)
    w = 2.0 * np.pi / SIDEREAL_DAY
    rc = R_EARTH * math.cos(math.radians(det.lat_deg))
    vx = vx - w * rc * np.sin(th)
    vy = vy + w * rc * np.cos(th)
    return np.stack([vx, vy, vz], axis=1) / C_LIGHT


def detector_arms(t_mid: np.ndarray, det: Detector) -> np.ndarray:
    """Arm unit vectors [N, 6] = (u, w) in equatorial coordinates at the mid-times:
    local North/East frame of the detector rotated with the Earth."""
    th = sidereal_angle(np.asarray(t_mid, dtype=np.float64), det.lon_deg)
    lat = math.radians(det.lat_deg)
    east = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], axis=1)
    north = np.stack([-math.sin(lat) * np.cos(th), -math.sin(lat) * np.sin(th),
                      np.full_like(th, math.cos(lat))], axis=1)
    arms = []
    for az in det.arm_azimuths_deg:
        a = math.radians(az)
        arms.append(math.cos(a) * north + math.sin(a) * east)
    return np.concatenate(arms, axis=1)


def sft_mid_times(n_present: int, t_sft: float, gap_frac: float, rng: np.random.Generator,
                  t0: float = EPOCH) -> np.ndarray:
    """Mid-times of ``n_present`` SFTs drawn from ceil(n/(1-gap)) consecutive slots."""
    if gap_frac <= 0.0:
        slots = np.arange(n_present)
    else:
        n_slots = int(math.ceil(n_present / (1.0 - gap_frac)))
        slots = np.sort(rng.choice(n_slots, size=n_present, replace=False))
    return t0 + slots.astype(np.float64) * t_sft + 0.5 * t_sft


def isotropic_sky(n: int, rng: np.random.Generator) -> np.ndarray:
    """Unit vectors [n,3], uniform in (alpha, sin delta)."""
    alpha = rng.uniform(0.0, 2.0 * np.pi, size=n)
    sdec = rng.uniform(-1.0, 1.0, size=n)
    cdec = np.sqrt(np.maximum(0.0, 1.0 - sdec * sdec))
    n_xyz = np.stack([cdec * np.cos(alpha), cdec * np.sin(alpha), sdec], axis=1)
    return n_xyz / np.linalg.norm(n_xyz, axis=1, keepdims=True)


def noise_power(n_sft: int, n_bins: int, rng: np.random.Generator) -> np.ndarray:
    """Normalised power of unit-variance complex Gaussian bins, float32 [n_sft, n_bins]."""
    re = rng.standard_normal((n_sft, n_bins))
    im = rng.standard_normal((n_sft, n_bins))
    return (re * re + im * im).astype(np.float32)


def table_range(f0_min, f0_max, f1_min, f1_max, dt_min, dt_max, v_max, t_sft, margin=2):
    """Conservative [first_bin, n_bins] covering every track of the bank (sizing only)."""
    corners = [f1_min * dt_min, f1_min * dt_max, f1_max * dt_min, f1_max * dt_max]
    lo = math.floor((f0_min + min(corners)) * (1.0 - v_max) * t_sft) - margin
    hi = math.ceil((f0_max + max(corners)) * (1.0 + v_max) * t_sft) + margin
    return int(lo), int(hi - lo + 1)


@dataclass
class Workload:
    """Everything one plain evaluation needs, as host numpy arrays."""
    name: str
    t_sft: float
    n_sft_per_det: list
    t_mid: np.ndarray            # [N] float64, detector-major, time ascending
    v: np.ndarray                # [N,3] float64, v/c
    t_ref: float
    first_bin: int
    n_bins: int
    power: np.ndarray            # [N, n_bins] float32
    weight: np.ndarray | None    # [N] float32 or None (all ones)
    f0: np.ndarray               # [n_f0]
    f1: np.ndarray               # [n_f1]
    sky: np.ndarray              # [n_sky,3]
    k: int
    sub_edges: np.ndarray        # [n_sub+1]
    injections: list = field(default_factory=list)  # dicts of injection parameters
    arms: np.ndarray | None = None  # [N, 6] detector arm unit vectors (u, w) at t_mid

    @property
    def n_sft(self):
        return int(self.t_mid.shape[0])

    @property
    def n_templates(self):
        return int(self.f0.size * self.f1.size * self.sky.shape[0])

    @property
    def evals(self):
        return self.n_templates * self.n_sft


def _build(name, n_det, n_per_det, t_sft, gap, f_start, n_f0, f1, n_sky, k, n_sub, seed,
           with_noise=True, sky=None):
    rng = np.random.default_rng(seed)
    t_parts, v_parts, a_parts = [], [], []
    for d in range(n_det):
        t = sft_mid_times(n_per_det, t_sft, gap, rng)
        t_parts.append(t)
        v_parts.append(detector_velocity(t, DETECTORS[d]))
        a_parts.append(detector_arms(t, DETECTORS[d]))
    t_mid = np.concatenate(t_parts)
    v = np.concatenate(v_parts)
    arms = np.concatenate(a_parts)
    t_ref = EPOCH
    f0 = f_start + np.arange(n_f0, dtype=np.float64) / t_sft
    f1 = np.asarray(f1, dtype=np.float64)
    if sky is None:
        sky = isotropic_sky(n_sky, rng)
    vmax = float(np.max(np.linalg.norm(v, axis=1)))
    dt = t_mid - t_ref
    first_bin, n_bins = table_range(f0.min(), f0.max(), f1.min(), f1.max(), dt.min(), dt.max(),
                                    vmax, t_sft)
    power = noise_power(t_mid.size, n_bins, rng) if with_noise else \
        np.zeros((t_mid.size, n_bins), np.float32)
    per = n_f0 // n_sub
    edges = np.array([f_start + (j * per - 0.5) / t_sft for j in range(n_sub)]
                     + [f_start + (n_f0 - 0.5) / t_sft], dtype=np.float64)
    return Workload(name, t_sft, [n_per_det] * n_det, t_mid, v, t_ref, first_bin, n_bins, power,
                    None, f0, f1, sky, k, edges, arms=arms)


def injection_params(rng: np.random.Generator, f_lo: float, f_hi: float, amp_lo: float,
                     amp_hi: float, f1_lo: float = 0.0, f1_hi: float = 0.0,
                     log_amp: bool = False) -> dict:
    """One injected signal: amplitude h0/sqrt(S_n), isotropic orientation and sky."""
    if log_amp:
        amp = float(np.exp(rng.uniform(np.log(amp_lo), np.log(amp_hi))))
    else:
        amp = float(rng.uniform(amp_lo, amp_hi))
    sky = isotropic_sky(1, rng)[0]
    return {"amp": amp, "cos_iota": float(rng.uniform(-1.0, 1.0)),
            "psi": float(rng.uniform(-np.pi / 4, np.pi / 4)), "sky": sky,
            "f0": float(rng.uniform(f_lo, f_hi)), "f1": float(rng.uniform(f1_lo, f1_hi))}


def plain_small(seed: int = 1, n_sky: int = 20) -> Workload:
    """1 detector, 100 contiguous SFTs, 100.0-100.1 Hz, 180 f0 x 3 f1 x 20 sky, K=10."""
    return _build("plain-1det-100sft-100Hz", 1, 100, 1800.0, 0.0, 100.0, 180,
                  [-1e-10, 0.0, 1e-10], n_sky, 10, 1, seed)


def weighted_small(seed: int = 5, n_sky: int = 24, n_per_det: int = 300) -> Workload:
    """2 detectors x 300 SFTs of 1800 s (10% gaps), 150.0-150.22 Hz, 400 f0 x 2 f1 x 24 sky,
    K = 20 in each of 4 sub-bands: several tiles with a ragged tail, for the weighted
    statistics (arms included)."""
    return _build("weighted-2det-300sft-150Hz", 2, n_per_det, 1800.0, 0.1, 150.0, 400,
                  [-2e-10, 1e-10], n_sky, 20, 4, seed)


def wide_band(n_f0: int, seed: int = 20, n_sky: int = 3, n_per_det: int = 30,
              with_noise: bool = True) -> Workload:
    """1 detector x n_per_det SFTs of 1800 s, n_f0 f0 from 120 Hz x 2 f1 x n_sky, K = 25:
    long f0 rows for the selection over grid banks (with_noise False gives a table
    of zeros, so every template ties)."""
    return _build("wide-1det-%dsft-120Hz-%df0" % (n_per_det, n_f0), 1, n_per_det, 1800.0, 0.0,
                  120.0, n_f0, [-1e-10, 0.0], n_sky, 25, 1, seed, with_noise=with_noise)


def tiny_bank(n_f0: int, n_f1: int, n_sky: int, n_per_det: int, seed: int = 40) -> Workload:
    """2 detectors x n_per_det SFTs of 1800 s (10% gaps), n_f0 f0 from 150 Hz x n_f1 f1 values
    in [-3e-10, 2e-10] x n_sky, K = 5 in one sub-band: the smallest shapes (a single template,
    SFT counts that end inside a stage, one f0 value past a full tile)."""
    f1 = np.linspace(-3e-10, 2e-10, n_f1) if n_f1 > 1 else [1e-10]
    return _build("tiny-2det-%dsft-150Hz-%dx%dx%d" % (2 * n_per_det, n_f0, n_f1, n_sky), 2, n_per_det,
                  1800.0, 0.1, 150.0, n_f0, f1, n_sky, 5, 1, seed)


def allsky_band(seed: int = 2, n_sky: int = 100_000, n_per_det: int = 5000) -> Workload:
    """2 detectors x 5000 SFTs (10% gaps), 200-200.5 Hz, 900 f0 x 11 f1 x n_sky, K=100/0.05 Hz.

    `power` holds noise only; `injections` lists 3 signals for tables generated with
    them: h0/sqrt(S_n) ~ U[0.05, 0.2], f1 ~ U[-1e-9, 0], isotropic sky and orientation,
    f0 ~ U[0.01, 0.04] Hz into three distinct inner 0.05 Hz sub-bands."""
    w = _build("allsky-2det-10ksft-200Hz", 2, n_per_det, 1800.0, 0.1, 200.0, 900,
               np.linspace(-1e-9, 0.0, 11), n_sky, 100, 10, seed)
    rng = np.random.default_rng(seed + 7919)
    subs = rng.choice(np.arange(1, 9), 3, replace=False)
    w.injections = [injection_params(rng, 200.0 + 0.05 * j + 0.01, 200.0 + 0.05 * j + 0.04,
                                     0.05, 0.2, -1e-9, 0.0) for j in subs]
    return w


def precision_stress(seed: int = 2, n_sky: int = 20_000, n_per_det: int = 5000) -> Workload:
    """Same timestamps as the all-sky band; 1000-1000.1 Hz, 180 f0 x 5 f1 x n_sky."""
    return _build("precision-2det-10ksft-1kHz", 2, n_per_det, 1800.0, 0.1, 1000.0, 180,
                  np.linspace(-1e-9, 0.0, 5), n_sky, 100, 2, seed)


@dataclass
class Campaign:
    """Many independent runs sharing one SFT pool and one bank pool (inputs only)."""
    t_sft: float
    t_mid: np.ndarray     # [n_pool] time-interleaved SFTs of the two detectors
    v: np.ndarray         # [n_pool, 3]
    arms: np.ndarray      # [n_pool, 6]
    f0: np.ndarray        # concatenated per-run f0 grids
    f1: np.ndarray        # concatenated per-run f1 sets
    sky: np.ndarray       # concatenated per-run sky sets
    runs: object          # list of dicts (seed, run_id, sft_begin, n_sft, first_bin, n_bins,
                          # f0_begin, n_f0, f1_begin, n_f1, sky_begin, n_sky, t_ref, inj) or
                          # the same as columns (injection: amp, cos_iota, psi, inj_sky,
                          # inj_f0, inj_f1)
    k: int

    @property
    def evals(self):
        if isinstance(self.runs, dict):
            R = self.runs
            return int(np.sum(R["n_f0"].astype(np.int64) * R["n_f1"] * R["n_sky"] * R["n_sft"]))
        return sum(r["n_f0"] * r["n_f1"] * r["n_sky"] * r["n_sft"] for r in self.runs)

    @property
    def n_runs(self):
        return len(self.runs["seed"]) if isinstance(self.runs, dict) else len(self.runs)


def campaign(n_runs: int, seed: int = 4, n_pool: int = 5000, n_sft_range=(500, 5000),
             f_range=(100.0, 300.0), width_range=(0.01, 0.2), nt_range=(1e3, 1e5), n_f1: int = 3,
             amp_range=(0.05, 0.2), k: int = 10, t_sft: float = 1800.0, gap: float = 0.1) -> Campaign:
    """Uneven injection-recovery runs: N ~ U{n_sft_range} SFTs (a contiguous slice of a
    two-detector, time-interleaved pool with gaps), band start ~ U(f_range), width
    ~ U(width_range), template count log-uniform in nt_range as a grid of
    round(width T) f0 x n_f1 f1 x ceil(n_T/(n_f1 n_f0)) isotropic sky points, one
    injected signal inside each band."""
    rng = np.random.default_rng(seed)
    per_det = (n_pool + 1) // 2
    ts, vs, arms = [], [], []
    for d in range(2):
        t = sft_mid_times(per_det, t_sft, gap, rng)
        ts.append(t)
        vs.append(detector_velocity(t, DETECTORS[d]))
        arms.append(detector_arms(t, DETECTORS[d]))
    t_all = np.concatenate(ts)
    order = np.argsort(t_all, kind="stable")[:n_pool]
    t_mid = t_all[order]
    v = np.concatenate(vs)[order]
    arm = np.concatenate(arms)[order]
    vmax = float(np.max(np.linalg.norm(v, axis=1)))
    f0_parts, f1_parts, sky_parts, runs = [], [], [], []
    nf0 = nf1 = nsk = 0
    for r in range(n_runs):
        n_sft = int(rng.integers(n_sft_range[0], n_sft_range[1] + 1))
        n_sft = min(n_sft, n_pool)
        begin = int(rng.integers(0, n_pool - n_sft + 1))
        f_lo = float(rng.uniform(*f_range))
        width = float(rng.uniform(*width_range))
        n_f0 = max(1, int(round(width * t_sft)))
        n_t = float(np.exp(rng.uniform(np.log(nt_range[0]), np.log(nt_range[1]))))
        n_sky = max(1, int(math.ceil(n_t / (n_f1 * n_f0))))
        f0 = f_lo + np.arange(n_f0, dtype=np.float64) / t_sft
        f1 = np.linspace(-1e-9, 0.0, n_f1) if n_f1 > 1 else np.zeros(1)
        sky = isotropic_sky(n_sky, rng)
        t_ref = float(t_mid[begin] - 0.5 * t_sft)
        dt = t_mid[begin:begin + n_sft] - t_ref
        first_bin, n_bins = table_range(f0.min(), f0.max(), f1.min(), f1.max(), dt.min(),
                                        dt.max(), vmax, t_sft)
        inj = injection_params(rng, f0[0], f0[-1], amp_range[0], amp_range[1], f1.min(), f1.max())
        runs.append({"seed": int(rng.integers(1, 2 ** 62)), "run_id": r, "sft_begin": begin,
                     "n_sft": n_sft, "first_bin": first_bin, "n_bins": n_bins, "f0_begin": nf0,
                     "n_f0": n_f0, "f1_begin": nf1, "n_f1": len(f1), "sky_begin": nsk,
                     "n_sky": n_sky, "t_ref": t_ref, "inj": inj})
        f0_parts.append(f0)
        f1_parts.append(f1)
        sky_parts.append(sky)
        nf0 += n_f0
        nf1 += len(f1)
        nsk += n_sky
    return Campaign(t_sft, t_mid, v, arm, np.concatenate(f0_parts), np.concatenate(f1_parts),
                    np.concatenate(sky_parts), runs, k)


def cap_points(center: np.ndarray, n: int, radius: float, rng: np.random.Generator) -> np.ndarray:
    """n unit vectors uniform in the spherical cap of angular radius `radius` around center."""
    c = np.asarray(center, np.float64)
    a = np.array([1.0, 0.0, 0.0]) if abs(c[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(c, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(c, e1)
    cos_t = rng.uniform(math.cos(radius), 1.0, n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    pts = cos_t[:, None] * c + sin_t[:, None] * (np.cos(ph)[:, None] * e1 + np.sin(ph)[:, None] * e2)
    return pts / np.linalg.norm(pts, axis=1, keepdims=True)


def label_campaign(n_runs: int, seed: int, base: "Workload", amp_range=(0.005, 0.1),
                   f_range=(100.0, 300.0), n_f0: int = 5, n_f1: int = 11, n_sky: int = 16,
                   n_sky_bank: int = 100_000, k: int = 1):
    """Injection-recovery runs on the SFTs of `base` (inputs of the p_det labels).

    Each run injects one signal (amplitude log-uniform in amp_range, isotropic
    orientation and sky, f uniform in f_range, f1 uniform in [-1e-9, 0]) and
    searches it with a local bank: the 5 f0 bins of the 1/T_sft grid nearest to
    f, 11 f1 values in [-1e-9, 0] and 16 sky points spread uniformly over the cap
    that holds, on average, the 16 nearest points of an isotropic bank of
    `n_sky_bank` points.  Runs are returned as columns (arrays named like the
    fields of a run).  Returns (Campaign, raw [n_runs, 6]) with
    raw = (amp, cos iota, psi, sin delta, alpha, f)."""
    rng = np.random.default_rng(seed)
    radius = math.acos(1.0 - 2.0 * n_sky / n_sky_bank)
    f1 = np.linspace(-1e-9, 0.0, n_f1)
    vmax = float(np.max(np.linalg.norm(base.v, axis=1)))
    dt = base.t_mid - base.t_ref
    amp = np.exp(rng.uniform(np.log(amp_range[0]), np.log(amp_range[1]), n_runs))
    cos_iota = rng.uniform(-1.0, 1.0, n_runs)
    psi = rng.uniform(-np.pi / 4, np.pi / 4, n_runs)
    inj_sky = isotropic_sky(n_runs, rng)
    f_inj = rng.uniform(f_range[0], f_range[1], n_runs)
    f1_inj = rng.uniform(-1e-9, 0.0, n_runs)
    i0 = np.round((f_inj - f_range[0]) * base.t_sft).astype(np.int64)
    offs = np.arange(-(n_f0 // 2), n_f0 - n_f0 // 2)
    f0 = f_range[0] + (i0[:, None] + offs[None, :]) / base.t_sft          # [n_runs, n_f0]
    # sky caps, vectorised
    a = np.where(np.abs(inj_sky[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    e1 = np.cross(inj_sky, a)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(inj_sky, e1)
    cos_t = rng.uniform(math.cos(radius), 1.0, (n_runs, n_sky))
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    ph = rng.uniform(0.0, 2.0 * np.pi, (n_runs, n_sky))
    sky = (cos_t[..., None] * inj_sky[:, None, :]
           + sin_t[..., None] * (np.cos(ph)[..., None] * e1[:, None, :]
                                 + np.sin(ph)[..., None] * e2[:, None, :]))
    sky /= np.linalg.norm(sky, axis=2, keepdims=True)
    corners = np.array([f1.min() * dt.min(), f1.min() * dt.max(), f1.max() * dt.min(),
                        f1.max() * dt.max()])
    lo = np.floor((f0[:, 0] + corners.min()) * (1.0 - vmax) * base.t_sft).astype(np.int64) - 2
    hi = np.ceil((f0[:, -1] + corners.max()) * (1.0 + vmax) * base.t_sft).astype(np.int64) + 2
    r = np.arange(n_runs)
    runs = {"seed": rng.integers(1, 2 ** 62, n_runs, dtype=np.int64).astype(np.uint64),
            "run_id": r.astype(np.uint32), "sft_begin": np.zeros(n_runs, np.int32),
            "n_sft": np.full(n_runs, base.n_sft, np.int32), "first_bin": lo,
            "n_bins": (hi - lo + 1).astype(np.int32), "f0_begin": (r * n_f0).astype(np.int32),
            "n_f0": np.full(n_runs, n_f0, np.int32), "f1_begin": np.zeros(n_runs, np.int32),
            "n_f1": np.full(n_runs, n_f1, np.int32), "sky_begin": (r * n_sky).astype(np.int32),
            "n_sky": np.full(n_runs, n_sky, np.int32), "t_ref": np.full(n_runs, base.t_ref),
            "amp": amp, "cos_iota": cos_iota, "psi": psi, "inj_sky": inj_sky, "inj_f0": f_inj,
            "inj_f1": f1_inj}
    cp = Campaign(base.t_sft, base.t_mid, base.v, base.arms, f0.ravel(), f1,
                  sky.reshape(-1, 3), runs, k)
    alpha = np.mod(np.arctan2(inj_sky[:, 1], inj_sky[:, 0]), 2.0 * np.pi)
    raw = np.stack([amp, cos_iota, psi, inj_sky[:, 2], alpha, f_inj], axis=1)
    return cp, raw


@dataclass
class BinaryWorkload:
    """SFTs plus a list bank of sources in circular binary systems (inputs only)."""
    name: str
    t_sft: float
    n_sft_per_det: list
    t_mid: np.ndarray            # [N] float64, detector-major, time ascending
    v: np.ndarray                # [N,3] float64, v/c
    arms: np.ndarray             # [N,6]
    t_ref: float
    first_bin: int
    n_bins: int
    power: np.ndarray            # [N, n_bins] float32
    f0: np.ndarray               # [n] Hz
    sky: np.ndarray              # [n,3]
    ap: np.ndarray               # [n] light-seconds
    omega: np.ndarray            # [n] rad/s
    phib: np.ndarray             # [n] rad at t_ref
    region: dict                 # f0_lo, f0_hi, ap_lo, ap_hi, omega_lo, omega_hi
    k: int
    sub_edges: np.ndarray

    @property
    def n_sft(self):
        return int(self.t_mid.shape[0])

    @property
    def n_templates(self):
        return int(self.f0.size)

    @property
    def evals(self):
        return self.n_templates * self.n_sft


DAY = 86400.0


def binary_band(seed: int = 3, n_tmpl: int = 10_000, n_per_det: int = 5000, f_lo: float = 110.5,
                width: float = 0.125, t_sft: float = 1024.0, gap: float = 0.1, period_days=(7.0, 15.0),
                ap_range=(5.0, 15.0), k: int = 10, n_sub: int = 5, with_noise: bool = True) -> BinaryWorkload:
    """The search setup of the real-data section as synthetic input: 2 detectors,
    SFTs of T = 1024 s overlapping by half (a new SFT every 512 s; 10% of the slots
    missing), a 0.125 Hz band at f_lo, orbital periods 7-15 days and projected
    semimajor axes 5-15 light-seconds; `n_tmpl` templates drawn uniformly in each
    parameter (f0, isotropic sky, a_p, period, phi_b in [0, 2 pi)); noise table."""
    rng = np.random.default_rng(seed)
    stride = 0.5 * t_sft
    t_parts, v_parts, a_parts = [], [], []
    for d in range(2):
        n_slots = int(math.ceil(n_per_det / (1.0 - gap)))
        slots = np.sort(rng.choice(n_slots, size=n_per_det, replace=False))
        t = EPOCH + slots.astype(np.float64) * stride + 0.5 * t_sft
        t_parts.append(t)
        v_parts.append(detector_velocity(t, DETECTORS[d]))
        a_parts.append(detector_arms(t, DETECTORS[d]))
    t_mid = np.concatenate(t_parts)
    v = np.concatenate(v_parts)
    arms = np.concatenate(a_parts)
    f_hi = f_lo + width
    om_lo, om_hi = 2.0 * np.pi / (period_days[1] * DAY), 2.0 * np.pi / (period_days[0] * DAY)
    f0 = rng.uniform(f_lo, f_hi, n_tmpl)
    sky = isotropic_sky(n_tmpl, rng)
    ap = rng.uniform(ap_range[0], ap_range[1], n_tmpl)
    omega = 2.0 * np.pi / (rng.uniform(period_days[0], period_days[1], n_tmpl) * DAY)
    phib = rng.uniform(0.0, 2.0 * np.pi, n_tmpl)
    vmax = float(np.max(np.linalg.norm(v, axis=1)))
    awmax = ap_range[1] * om_hi
    first_bin = int(math.floor(f_lo * (1.0 - vmax - awmax) * t_sft)) - 2
    last = int(math.ceil(f_hi * (1.0 + vmax + awmax) * t_sft)) + 2
    n_bins = last - first_bin + 1
    power = noise_power(t_mid.size, n_bins, rng) if with_noise else \
        np.zeros((t_mid.size, n_bins), np.float32)
    edges = f_lo + width * np.arange(n_sub + 1) / n_sub
    region = dict(f0_lo=f_lo, f0_hi=f_hi, ap_lo=ap_range[0], ap_hi=ap_range[1], omega_lo=om_lo, omega_hi=om_hi)
    return BinaryWorkload("binary-2det-%dsft-%gHz" % (2 * n_per_det, f_lo), t_sft, [n_per_det] * 2, t_mid, v,
                          arms, EPOCH, first_bin, n_bins, power, f0, sky, ap, omega, phib, region, k, edges)
