// List-bank evaluation (one lane per template, no assumption on the bank's
// structure -- the batch evaluation of Sec. III), bin dumps and the index
// precision study (FP32 / split double-FP32 / guarded against FP64), plus the
// small helper kernels of the host layer.
#include <mutex>

#include "ft_internal.h"

namespace ft {

namespace {

// ---------------------------------------------------------------------------
// Index precision variants.
// ---------------------------------------------------------------------------

// The canonical expression evaluated in FP32 throughout.
__device__ __forceinline__ int bin_fp32(double f0, double f1, double dt, const double *v,
                                        const double *n, double t_sft)
{
    const float px = (float)v[0] * (float)n[0];
    const float py = (float)v[1] * (float)n[1];
    const float pz = (float)v[2] * (float)n[2];
    float d = px + py;
    d = d + pz;
    const float g = 1.f + d;
    const float c = (float)f1 * (float)dt;
    const float a = (float)f0 + c;
    const float f = a * g;
    const float x = f * (float)t_sft;
    return (int)floorf(x + 0.5f);
}

// Unevaluated sums of two floats ("double-float"): error-free two-sum
// (Knuth, TAOCP vol. 2, 4.2.2) and two-product via a fused multiply-add
// (Dekker 1971), combined as in the double-double arithmetic of Hida, Li and
// Bailey (2001) with float limbs.
struct df {
    float hi, lo;
};
__device__ __forceinline__ df two_sum(float a, float b)
{
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ df fast_two_sum(float a, float b)
{
    const float s = a + b;
    const float e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ df df_split(double x)
{
    const float h = (float)x;
    return {h, (float)(x - (double)h)};
}
__device__ __forceinline__ df df_add(df a, df b)
{
    df s = two_sum(a.hi, b.hi);
    const df t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ df df_mul(df a, df b)
{
    const float p = a.hi * b.hi;
    float e = fmaf(a.hi, b.hi, -p);
    const float cross = a.hi * b.lo + a.lo * b.hi;
    e += cross;
    return fast_two_sum(p, e);
}
// x + 1/2 of the canonical track in double-float arithmetic; c_out is f1 dt.
__device__ __forceinline__ df track_df64(double f0, double f1, double dt, const double *v, const double *n,
                                         double t_sft, df &c_out)
{
    const df px = df_mul(df_split(v[0]), df_split(n[0]));
    const df py = df_mul(df_split(v[1]), df_split(n[1]));
    const df pz = df_mul(df_split(v[2]), df_split(n[2]));
    df d = df_add(px, py);
    d = df_add(d, pz);
    const df g = df_add(df{1.f, 0.f}, d);
    c_out = df_mul(df_split(f1), df_split(dt));
    const df a = df_add(df_split(f0), c_out);
    const df f = df_mul(a, g);
    const df x = df_mul(f, df_split(t_sft));
    return df_add(x, df{0.5f, 0.f});
}

// floor of a double-float value below 2^24 (t.hi integral and t.lo < 0: one less).
__device__ __forceinline__ float df_floor(df t)
{
    float fl = floorf(t.hi);
    if (fl == t.hi && t.lo < 0.f) fl -= 1.f;
    return fl;
}

__device__ __forceinline__ int bin_df64(double f0, double f1, double dt, const double *v,
                                        const double *n, double t_sft)
{
    df c;
    return (int)df_floor(track_df64(f0, f1, dt, v, n, t_sft, c));
}

__device__ __forceinline__ int bin_canonical(double f0, double f1, double dt, const double *v,
                                             const double *n, double t_sft)
{
    const double g = doppler_factor(v[0], v[1], v[2], n[0], n[1], n[2]);
    return bin_fp64(f0, f1 * dt, g, t_sft);
}

// Split double-FP32 estimate verified against FP64: the double-float value t
// of x + 1/2 is accepted when its fraction lies farther than beta from a bin
// edge, otherwise the canonical FP64 bin is computed.  Error bound, with
// u = 2^-24: the operations are the accurate double-word sum (relative error
// <= 3u^2) and the double-word product with an FMA two-product (<= 8u^2: the
// 7u^2 of its FMA form plus the separate rounding of one cross term), after
// Joldes, Muller and Popescu (ACM TOMS 2017); each double input is split with
// error <= u^2 |input|.  Propagated through d = (vx nx + vy ny) + vz nz
// (<= 26u^2 |v|, |n| = 1), g = 1 + d (<= 4u^2), c = f1 dt (<= 10u^2 |c|),
// a = f0 + c (<= u^2 (4|a| + 11|c|)), f = a g, x = f T (T = 1800 exact) and
// t = x + 1/2, |t - (x + 1/2)_real| <= 28u^2 (|x| + |c| T) to first order
// (|v| <= 1e-4).  The canonical FP64 bin's own error is below 8*2^-53 (|x| + 1),
// and the float fraction (t.hi - floor) + t.lo rounds once (<= 2^-25).  So
// beta = 2^-42 (|t.hi| + |c.hi| T) + 2^-24 (2^-42 = 64u^2, over twice the
// derived factor) certifies floor(t) = the canonical bin.  At x = 1.8e6
// (1 kHz) beta is 4.7e-7 bins, so nearly every evaluation is accepted.
// Values of 2^24 bins and above (where floats stop holding every integer) are
// always recomputed.
__device__ __forceinline__ int bin_guarded(double f0, double f1, double dt, const double *v,
                                           const double *n, double t_sft, int *fallback)
{
    df c;
    const df t = track_df64(f0, f1, dt, v, n, t_sft, c);
    const float ta = fabsf(t.hi);
    if (ta < 0x1p24f) {
        const float fl = df_floor(t);
        const float frac = (t.hi - fl) + t.lo;
        const float beta = 0x1p-42f * (ta + fabsf(c.hi) * (float)t_sft) + 0x1p-24f;
        if (frac > beta && frac < 1.f - beta) return (int)fl;
    }
    ++*fallback;
    return bin_canonical(f0, f1, dt, v, n, t_sft);
}

// FP32 estimate accepted only when it is farther from a bin edge than its
// error bound; otherwise the canonical FP64 bin.  The FP32 evaluation has
// relative error below 8*2^-24 (input roundings plus five operations), so a
// margin of 16*2^-24*x + 2^-20 bins certifies the FP32 floor.  The margin
// reaches half a bin at x = 5.2e5 (290 Hz at T = 1800 s): above that every
// evaluation is recomputed in FP64.
__device__ __forceinline__ int bin_guarded_fp32(double f0, double f1, double dt, const double *v,
                                                const double *n, double t_sft, int *fallback)
{
    const float px = (float)v[0] * (float)n[0];
    const float py = (float)v[1] * (float)n[1];
    const float pz = (float)v[2] * (float)n[2];
    float d = px + py;
    d = d + pz;
    const float g = 1.f + d;
    const float c = (float)f1 * (float)dt;
    const float a = (float)f0 + c;
    const float f = a * g;
    const float x = f * (float)t_sft;
    const float t = x + 0.5f;
    const float fl = floorf(t);
    const float u = t - fl;
    const float beta = 16.f * 5.9604645e-8f * fabsf(x) + 9.5367432e-7f;
    if (u > beta && u < 1.f - beta) return (int)fl;
    ++*fallback;
    return bin_canonical(f0, f1, dt, v, n, t_sft);
}

__device__ __forceinline__ int bin_mode(int mode, double f0, double f1, double dt,
                                        const double *v, const double *n, double t_sft,
                                        int *fallback)
{
    switch (mode) {
    case FT_INDEX_FP32: return bin_fp32(f0, f1, dt, v, n, t_sft);
    case FT_INDEX_DF64: return bin_df64(f0, f1, dt, v, n, t_sft);
    case FT_INDEX_GUARDED: return bin_guarded(f0, f1, dt, v, n, t_sft, fallback);
    case FT_INDEX_GUARDED_FP32: return bin_guarded_fp32(f0, f1, dt, v, n, t_sft, fallback);
    default: return bin_canonical(f0, f1, dt, v, n, t_sft);
    }
}

// ---------------------------------------------------------------------------
// Direct evaluation: one lane per template, gathers straight from the (cached)
// table.  Used for LIST banks and for grids whose tile window would not fit
// in LDS.
// ---------------------------------------------------------------------------
template <bool GRID>
__device__ __forceinline__ void eval_direct_one(const EvalRun &r, int64_t t)
{
    double f0, f1;
    const double *n;
    if (GRID) {
        const int64_t i = t % r.n_f0;
        const int64_t rest = t / r.n_f0;
        f0 = r.f0[i];
        f1 = r.f1[rest % r.n_f1];
        n = r.sky + 3 * (rest / r.n_f1);
    } else {
        f0 = r.f0[t];
        f1 = r.f1[t];
        n = r.sky + 3 * t;
    }
    const double nx = n[0], ny = n[1], nz = n[2];
    // sky-dependent weights: w_k = u_k (ab_k(n) / sum_k' u_k' ab_k'(n))
    const double inv = GRID && r.sky_norm ? r.sky_norm[t / ((int64_t)r.n_f0 * r.n_f1)] : 0.0;
    float acc = 0.f;
    double tot = 0.0;
    uint32_t bad = 0;
    for (int k = 0; k < r.n_sft; ++k) {
        const double *vk = r.v + 3 * (int64_t)k;
        const double g = doppler_factor(vk[0], vk[1], vk[2], nx, ny, nz);
        const int B = bin_fp64(f0, f1 * r.dt[k], g, r.t_sft);
        int b = B - r.first_bin;
        if (b < 0 || b >= r.n_bins) {
            bad = ERR_RANGE;
            b = b < 0 ? 0 : r.n_bins - 1;
        }
        float val = r.power[(int64_t)k * r.n_bins + b];
        if (r.weight) val *= r.weight[k];
        if (GRID && r.sky_norm) val *= (float)(sky_ab(r.arms + 6 * (int64_t)k, nx, ny, nz) * inv);
        acc += val;
        if (r.sum_mode == FT_SUM_BLOCKED && ((k + 1) & (SUM_BLOCK - 1)) == 0) {
            tot += (double)acc;
            acc = 0.f;
        }
    }
    if (bad) atomicOr(r.err, bad);
    r.stats[t] = (float)(tot + (double)acc);
}

template <bool GRID>
__global__ __launch_bounds__(256) void eval_direct_kernel(EvalRun r)
{
    const int64_t n_t = GRID ? (int64_t)r.n_f0 * r.n_f1 * r.n_sky : r.n_list;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t;
         t += (int64_t)gridDim.x * blockDim.x)
        eval_direct_one<GRID>(r, t);
}

// Persistent evaluation of batch runs whose grid is too small for the tile
// kernel (or whose window does not fit in LDS).  A wavefront pulls an item
// (run, chunk) from the queue; chunk = f0 chunk * n_js_chunks + js chunk,
// covering up to SF0 consecutive f0 values (SF0 = 5 or 8, chosen per batch)
// and 64 consecutive (f1, sky)
// pairs js = s * n_f1 + j, one pair per lane.  Per SFT a lane forms the
// canonical Doppler factor and f1 * dt once and then the canonical FP64 bin of
// each of its f0 values, gathering from the (cached) table; the gathers of SFT
// k+1 are issued before the values of SFT k are added.  The bin is monotone
// in f0 (f0 strictly increasing, g > 0), so the run's first and last bins
// bound all of them and only those two are range-checked; a wave with an
// out-of-range lane clamps every read into the row and flags the error.
static_assert(SUM_BLOCK % 2 == 0, "blocks are walked in pairs of SFTs");

// Read-only inputs that the kernel reaches through pointers held in the run
// record, read through the constant address space so that wave-uniform reads
// (velocities, time offsets, f0 values) become scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}
typedef const __attribute__((address_space(1))) float global_float;

// Velocity and time offset of one SFT (wave-uniform, loaded a step ahead).
struct SmallSft {
    double vx, vy, vz, dt;
};

__device__ __forceinline__ SmallSft small_sft(const EvalRun &r, int k)
{
    const auto *vk = as_const(r.v + 3 * (int64_t)k);
    return {vk[0], vk[1], vk[2], as_const(r.dt)[k]};
}

// Bins of one SFT step as byte offsets (B - first_bin) * 4 into row k (exact
// in 32 bits: rows hold fewer than 2^28 columns); returns false in every lane
// if some lane of the wave left the table (the offsets are then clamped into
// the row).
template <int SF0>
__device__ __forceinline__ bool small_bins(const EvalRun &r, const SmallSft &q, const double (&f0v)[SF0],
                                           double f1, double nx, double ny, double nz, uint32_t (&off)[SF0],
                                           bool &bad)
{
    const double g = doppler_factor(q.vx, q.vy, q.vz, nx, ny, nz);
    const double c = f1 * q.dt;
    int B[SF0];
#pragma unroll
    for (int l = 0; l < SF0; ++l) B[l] = bin_fp64(f0v[l], c, g, r.t_sft);
    // B[l] is non-decreasing in l (the last f0 repeats past the chunk's end)
    const bool in = B[0] >= r.first_bin && B[SF0 - 1] - r.first_bin < r.n_bins;
    const bool wave_in = __builtin_amdgcn_ballot_w64(!in) == 0;
    if (!wave_in) {
        bad |= !in;
#pragma unroll
        for (int l = 0; l < SF0; ++l) B[l] = min(max(B[l], r.first_bin), r.first_bin + r.n_bins - 1);
    }
    const uint32_t fb4 = (uint32_t)r.first_bin * 4u;
#pragma unroll
    for (int l = 0; l < SF0; ++l) off[l] = (uint32_t)B[l] * 4u - fb4;
    return wave_in;
}

template <int SF0>
__device__ __forceinline__ void small_gather(const EvalRun &r, int k, const uint32_t (&off)[SF0],
                                             float (&v)[SF0])
{
    const char *base = (const char *)(r.power_w + (int64_t)k * r.n_bins);
#pragma unroll
    for (int l = 0; l < SF0; ++l) v[l] = *(global_float *)(base + off[l]);
}

template <int SF0>
__device__ __forceinline__ void small_add(const float (&v)[SF0], float (&acc)[SF0])
{
#pragma unroll
    for (int l = 0; l < SF0; ++l) acc[l] += v[l];
}

template <int SF0>
__global__ __launch_bounds__(64) void eval_batch_small_kernel(const EvalRun *__restrict__ runs,
                                                              const int2 *__restrict__ items, int n_items,
                                                              unsigned *counter)
{
    const int lane = threadIdx.x;
    for (;;) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(counter, 1u);
        const int item = __builtin_amdgcn_readlane((int)got, 0);
        if (item >= n_items) break;
        const int2 it = items[item];
        const EvalRun r = runs[it.x];
        const int n_js = r.n_f1 * r.n_sky;
        const int n_jsc = (n_js + 63) / 64;
        const int i0 = (it.y / n_jsc) * SF0;
        const int n_i = min(SF0, r.n_f0 - i0);
        const int js_raw = (it.y % n_jsc) * 64 + lane;
        const bool live = js_raw < n_js;
        const int js = live ? js_raw : n_js - 1;
        const int j = js % r.n_f1, s = js / r.n_f1;
        const double f1 = r.f1[j];
        const double nx = r.sky[3 * s], ny = r.sky[3 * s + 1], nz = r.sky[3 * s + 2];
        double f0v[SF0];
#pragma unroll
        for (int l = 0; l < SF0; ++l) f0v[l] = as_const(r.f0)[i0 + min(l, n_i - 1)];
        float acc[SF0];
        double tot[SF0];
#pragma unroll
        for (int l = 0; l < SF0; ++l) {
            acc[l] = 0.f;
            tot[l] = 0.0;
        }
        bool bad = false;
        const int n = r.n_sft;
        // Two value buffers in turn: the gathers of SFT k+1 go out before the
        // values of SFT k are added; velocities are read a step ahead.  Reads
        // past the last SFT re-read the last SFT (unused).  Summation blocks
        // of SUM_BLOCK SFTs (even) are walked in pairs, so va holds the next
        // block's first SFT when a block ends.
        uint32_t off[SF0];
        float va[SF0], vb[SF0];
        SmallSft q = small_sft(r, 0);
        small_bins(r, q, f0v, f1, nx, ny, nz, off, bad);
        small_gather(r, 0, off, va);
        q = small_sft(r, min(1, n - 1));
        for (int kb = 0; kb < n; kb += SUM_BLOCK) {
            const int ke = min(kb + SUM_BLOCK, n);
            int k = kb;
            for (; k + 1 < ke; k += 2) {
                small_bins(r, q, f0v, f1, nx, ny, nz, off, bad);
                q = small_sft(r, min(k + 2, n - 1));
                small_gather(r, k + 1, off, vb);
                small_add(va, acc);
                small_bins(r, q, f0v, f1, nx, ny, nz, off, bad);
                q = small_sft(r, min(k + 3, n - 1));
                small_gather(r, min(k + 2, n - 1), off, va);
                small_add(vb, acc);
            }
            if (k < ke) small_add(va, acc);  // odd tail: k = n - 1
            if (r.sum_mode == FT_SUM_BLOCKED) {
#pragma unroll
                for (int l = 0; l < SF0; ++l) {
                    tot[l] += (double)acc[l];
                    acc[l] = 0.f;
                }
            }
        }
        if (bad && live) atomicOr(r.err, ERR_RANGE);
        if (live) {
            float *out = r.stats + (int64_t)js * r.n_f0 + i0;
#pragma unroll
            for (int l = 0; l < SF0; ++l)
                if (l < n_i) out[l] = (float)(tot[l] + (double)acc[l]);
        }
    }
}

// Binary-system list banks: one lane per template (the paper's random
// template banks carry no structure to share between lanes).  Per SFT a lane
// forms an estimate of the track position x (single-precision Doppler factor,
// orbital phase in FP64, single-precision cosine) and keeps
// B = floor(x + 1/2) when x + 1/2 is farther than eps from an integer; else
// (about once per 2*10^4 evaluations) it forms the canonical bin with the
// library cosine and FP64 throughout.  It gathers from the table (scalar row
// base, lane offset); velocities and time offsets are wave-uniform scalar
// loads.  Lanes past the bank's end repeat its last template and store
// nothing, so the SFT loop stays wave-uniform.
//
// Estimate.  y = (Omega/pi) dt - phi_b/pi (the phase in units of pi),
// q = floor(y + 1/2), r = (y - q) pi (y - q is exact), cos ph = (-1)^q cos r
// with |r| <= pi/2; r is rounded to float (< 1e-7) and put through the Taylor
// polynomial of cos to r^12 (truncation < 6.5e-9) in fused single-precision
// Horner steps (seven roundings of values of magnitude <= 1.3: < 6e-7).
// Measured over 4e6 phases the estimate stays within 1.6e-7 of cos; the
// library cosine is within 2^-52 of cos, and the rounding of the phase (a few
// ulps of y) moves cos by < 1e-13.  delta = 1e-6 bounds the cosine error.
// Then w = d - (a_p Omega) c with d = v.n, in float from rounded velocities
// and sky: the roundings of v, n, a_p Omega, the three products and the two
// fused steps are each below 2^-24 (|v| + |w|) with |w| <= |v| + a_p Omega,
// so |w - (d - a_p Omega cos ph)| <= a_p Omega delta + 8 * 2^-24 (2|v| + a_p Omega).
// u = f0 T w + (f0 T + 1/2) is one FP64 fused multiply-add; the canonical
// x + 1/2 differs from u by at most
//   eps = f0 T (a_p Omega delta + 8 * 2^-24 (2 |v|max + a_p Omega)) + 1e-9
// (the last term covers the FP64 roundings, a few ulps of x).
constexpr double BINARY_COS_DELTA = 1e-6;

__device__ __forceinline__ float binary_cos_estimate(double y)
{
    const double q = floor(y + 0.5);
    const float r = (float)((y - q) * 0x1.921fb54442d18p+1);  // pi
    const float r2 = r * r;
    float p = __builtin_fmaf(r2, 2.08767570e-9f, -2.75573192e-7f);  // 1/12!, -1/10!
    p = __builtin_fmaf(p, r2, 2.48015873e-5f);                      // 1/8!
    p = __builtin_fmaf(p, r2, -1.38888889e-3f);                     // -1/6!
    p = __builtin_fmaf(p, r2, 4.16666667e-2f);                      // 1/4!
    p = __builtin_fmaf(p, r2, -0.5f);
    const float c = __builtin_fmaf(p, r2, 1.0f);
    return ((int)q & 1) ? -c : c;
}

// Per-lane constants of one binary template.
struct BinaryLane {
    double f0, f0T, f0T_half, nx, ny, nz, aw, omega, phib, om_pi, phib_pi, eps;
    float nxf, nyf, nzf, awf;
    // hardware-cosine form: phase in revolutions, pre-scaled track terms
    double om_rev, phib_rev;
    float Fx, Fy, Fz, Cw, Af, thr;
    int32_t off_base;  // 4 (Ai - first_bin)
};

// Canonical bin of a binary template (the rare guard fallback).
__device__ __forceinline__ int binary_canonical(const EvalRun &r, const BinaryLane &p, int k, double dt)
{
    const auto *vk = as_const(r.v + 3 * (int64_t)k);
    const double g = doppler_factor(vk[0], vk[1], vk[2], p.nx, p.ny, p.nz);
    return bin_binary(p.f0, g, p.aw, p.omega, p.phib, dt, r.t_sft);
}

// Byte offset of the canonical bin of one binary template in row k (clamped
// into the row and flagged when the track leaves the table).
__device__ __forceinline__ uint32_t binary_offset(const EvalRun &r, const BinaryLane &p, int k, bool &bad)
{
    const auto *v32 = as_const(r.v32 + 3 * (int64_t)k);
    const double dt = as_const(r.dt)[k];
    const float d = __builtin_fmaf(v32[2], p.nzf, __builtin_fmaf(v32[1], p.nyf, v32[0] * p.nxf));
    const float c = binary_cos_estimate(p.om_pi * dt - p.phib_pi);
    const float w = __builtin_fmaf(-p.awf, c, d);
    const double u = fma(p.f0T, (double)w, p.f0T_half);
    const double fr = __builtin_amdgcn_fract(u);
    int B = (int)u;
    if (!(fr > p.eps && fr < 1.0 - p.eps)) B = binary_canonical(r, p, k, dt);
    int b = B - r.first_bin;
    if (b < 0 || b >= r.n_bins) {
        bad = true;
        b = min(max(b, 0), r.n_bins - 1);
    }
    return (uint32_t)b * 4u;
}

// Hardware-cosine form of the estimate.  The phase in revolutions
// x = (Omega/2pi) dt - phi_b/2pi is reduced in FP64 (fract) and rounded to
// float (< 2^-25 rev), and c = v_cos_f32(x) = cos 2 pi x, whose error over every
// float in [0, 1] the library measures on the device (delta_hw); with the
// phase rounding and the canonical phase's own rounding the cosine is within
// delta = delta_hw + 2.1e-7 of the canonical one.  The track, shifted by eps
// and relative to the integer Ai, is four single-precision fused steps:
//   U = Af + Cw c + Fx vx + Fy vy + Fz vz,
// Cw = -f0 T a_p Omega, F = f0 T n, Af = (f0 T + 1/2 - eps) - Ai in [0, 1),
// all rounded to float, v rounded to float.  Against the canonical
// x + 1/2 - eps - Ai the error is below
//   f0 T a_p Omega delta + 2^-24 (5 f0 T a_p Omega + 6 f0 T |v|max + 4) + 2^-25,
// which eps (twice that, plus 1e-7) covers.  So when fract(U) < 1 - 2 eps the
// canonical bin is Ai + floor(U); otherwise (about once per 3*10^4
// evaluations) the canonical bin is formed in FP64.  RANGE: the host has not
// proved that every track stays in the table, so each bin is checked.
template <bool RANGE>
__device__ __forceinline__ uint32_t binary_offset_hw(const EvalRun &r, const BinaryLane &p, int k, bool &bad)
{
    const auto *v32 = as_const(r.v32 + 3 * (int64_t)k);
    const double dt = as_const(r.dt)[k];
    const float x = (float)__builtin_amdgcn_fract(fma(p.om_rev, dt, -p.phib_rev));
    const float c = __builtin_amdgcn_cosf(x);
    float U = __builtin_fmaf(p.Cw, c, p.Af);
    U = __builtin_fmaf(p.Fx, v32[0], U);
    U = __builtin_fmaf(p.Fy, v32[1], U);
    U = __builtin_fmaf(p.Fz, v32[2], U);
    const float fr = __builtin_amdgcn_fractf(U);
    int off;
    if (fr < p.thr) {
        off = (int)(U - fr) * 4 + p.off_base;
    } else {
        off = (binary_canonical(r, p, k, dt) - r.first_bin) * 4;
    }
    if (RANGE && !(off >= 0 && off < r.n_bins * 4)) {
        bad = true;
        off = min(max(off, 0), (r.n_bins - 1) * 4);
    }
    return (uint32_t)off;
}

__device__ __forceinline__ float binary_gather(const EvalRun &r, int k, uint32_t off)
{
    return *(global_float *)((const char *)(r.power_w + (int64_t)k * r.n_bins) + off);
}

// HW: the hardware-cosine estimate (r.cos_delta > 0), else the polynomial one.
// SKYW: sky-dependent weights (Sec. II.B): the staged values u_k P are
// multiplied by ab_k(n) (FP64, rounded to float) and the sum is divided at the
// end by W1 = sum_k u_k ab_k (FP64, sequential in SFT order).
// SPLIT (blocked sums, no sky weights): workgroup row blockIdx.y takes the
// SUM_BLOCK-SFT blocks [y bps, (y + 1) bps) and stores each block's FP32 sum
// in bsum[block][template]; binary_block_sum_kernel then adds them in block
// order in FP64, which is the unsplit kernel's sequence of operations.  Small
// banks use it to fill the GPU.
template <bool HW, bool RANGE, bool SKYW, bool SPLIT = false>
__global__ __launch_bounds__(256) void eval_binary_kernel(EvalRun r, float *bsum, int bps)
{
    static_assert(!(SPLIT && SKYW), "W1 is one sequential sum over every SFT");
    const int64_t n = r.n_list;
    const int n_sft = r.n_sft;
    const int k_begin = SPLIT ? (int)blockIdx.y * bps * SUM_BLOCK : 0;
    const int k_end = SPLIT ? min(k_begin + bps * SUM_BLOCK, n_sft) : n_sft;
    if (k_begin >= k_end) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t t_raw = base + threadIdx.x;
        const bool live = t_raw < n;
        const int64_t t = live ? t_raw : n - 1;
        BinaryLane p;
        p.f0 = r.f0[t];
        p.nx = r.sky[3 * t];
        p.ny = r.sky[3 * t + 1];
        p.nz = r.sky[3 * t + 2];
        p.omega = r.omega[t];
        p.phib = r.phib[t];
        p.aw = r.ap[t] * p.omega;
        p.f0T = p.f0 * r.t_sft;
        if (HW) {
            const double delta = r.cos_delta;
            const double e = 2.0 * (p.f0T * p.aw * delta +
                                    0x1p-24 * (5.0 * p.f0T * p.aw + 6.0 * p.f0T * r.vmax + 4.0) + 0x1p-25) +
                             1e-7;
            const double a = (p.f0T + 0.5) - e;
            const double ai = floor(a);
            p.om_rev = p.omega * 0x1.45f306dc9c883p-3;  // 1/(2 pi)
            p.phib_rev = p.phib * 0x1.45f306dc9c883p-3;
            p.Fx = (float)(p.f0T * p.nx);
            p.Fy = (float)(p.f0T * p.ny);
            p.Fz = (float)(p.f0T * p.nz);
            p.Cw = (float)(-(p.f0T * p.aw));
            p.Af = (float)(a - ai);
            p.thr = (float)(1.0 - 2.0 * e) - 0x1p-23f;
            p.off_base = ((int)ai - r.first_bin) * 4;
        } else {
            p.f0T_half = p.f0T + 0.5;
            p.om_pi = p.omega * 0x1.45f306dc9c883p-2;   // 1/pi
            p.phib_pi = p.phib * 0x1.45f306dc9c883p-2;
            p.nxf = (float)p.nx;
            p.nyf = (float)p.ny;
            p.nzf = (float)p.nz;
            p.awf = (float)p.aw;
            p.eps = p.f0T * (p.aw * BINARY_COS_DELTA + 8.0 * 0x1p-24 * (2.0 * r.vmax + p.aw)) + 1e-9;
        }
        auto offset = [&](int k, bool &bad) {
            return HW ? binary_offset_hw<RANGE>(r, p, k, bad) : binary_offset(r, p, k, bad);
        };
        double w1 = 0.0;
        // acc += value of SFT k (times its sky weight, which also enters W1)
        auto add = [&](float acc_in, float v, int k) {
            if (!SKYW) return acc_in + v;
            const double ab = sky_ab(as_const(r.arms + 6 * (int64_t)k), p.nx, p.ny, p.nz);
            w1 += (r.weight ? (double)as_const(r.weight)[k] : 1.0) * ab;
            return __builtin_fmaf(v, (float)ab, acc_in);
        };
        float acc = 0.f;
        double tot = 0.0;
        bool bad = false;
        // Two value buffers in turn: the gather of SFT k+1 goes out before the
        // value of SFT k is added (reads past the last SFT re-read it, unused);
        // blocks of SUM_BLOCK SFTs (even) are walked in pairs, so va holds the
        // next block's first SFT when a block ends.
        float va = binary_gather(r, k_begin, offset(k_begin, bad));
        for (int kb = k_begin; kb < k_end; kb += SUM_BLOCK) {
            const int ke = min(kb + SUM_BLOCK, n_sft);
            int k = kb;
            for (; k + 1 < ke; k += 2) {
                const float vb = binary_gather(r, k + 1, offset(k + 1, bad));
                acc = add(acc, va, k);
                const int k2 = min(k + 2, n_sft - 1);
                va = binary_gather(r, k2, offset(k2, bad));
                acc = add(acc, vb, k + 1);
            }
            if (k < ke) acc = add(acc, va, k);  // odd tail: k = n_sft - 1
            if (SPLIT) {
                if (live) bsum[(int64_t)(kb / SUM_BLOCK) * n + t] = acc;
                acc = 0.f;
            } else if (r.sum_mode == FT_SUM_BLOCKED) {
                tot += (double)acc;
                acc = 0.f;
            }
        }
        if (bad && live) atomicOr(r.err, ERR_RANGE);
        if (SPLIT) {
        } else if (SKYW) {
            if (!(w1 > 0.0) && live) atomicOr(r.err, ERR_BAD_POWER);
            if (live) r.stats[t] = (float)((tot + (double)acc) / w1);
        } else if (live) {
            r.stats[t] = (float)(tot + (double)acc);
        }
    }
}

// Statistic of the split binary evaluation: the block sums of each template
// added in block order in FP64 (the unsplit kernel's totals).
__global__ __launch_bounds__(256) void binary_block_sum_kernel(const float *bsum, int64_t n, int n_blk, float *stats)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double tot = 0.0;
        int b = 0;
        for (; b + 8 <= n_blk; b += 8) {  // eight loads in flight, then the additions in order
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = bsum[(int64_t)(b + i) * n + t];
#pragma unroll
            for (int i = 0; i < 8; ++i) tot += (double)x[i];
        }
        for (; b < n_blk; ++b) tot += (double)bsum[(int64_t)b * n + t];
        stats[t] = (float)tot;
    }
}

// Largest error of the hardware cosine over every float x in [0, 1]:
// |v_cos_f32(x) - cos 2 pi x|, the reference from the library cosine of the
// FP64 product 2 pi x (within 1e-15).  The maximum of non-negative doubles is
// taken on their bit patterns.
__global__ __launch_bounds__(256) void hw_cos_error_kernel(unsigned long long *max_bits)
{
    double worst = 0.0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= 0x3F800000u; i += gridDim.x * blockDim.x) {
        const float x = __uint_as_float(i);
        double sv, cv;
        lib_sincos((double)x * 0x1.921fb54442d18p+2, sv, cv);  // 2 pi x
        worst = fmax(worst, fabs((double)__builtin_amdgcn_cosf(x) - cv));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(max_bits, (unsigned long long)__double_as_longlong(worst));
}

// The library cosine and sine of an array (exposed for callers that
// reproduce binary-track phases, and for parity checks of the library cosine).
__global__ void lib_sincos_kernel(const double *x, int64_t n, double *c, double *s)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double sv, cv;
        lib_sincos(x[i], sv, cv);
        if (c) c[i] = cv;
        if (s) s[i] = sv;
    }
}

__global__ __launch_bounds__(256) void bins_list_kernel(EvalRun r, int mode, int32_t *bins)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < r.n_list;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double *n = r.sky + 3 * t;
        int fallback = 0;
        if (r.ap) {
            const double aw = r.ap[t] * r.omega[t];
            for (int k = 0; k < r.n_sft; ++k) {
                const double *vk = r.v + 3 * (int64_t)k;
                const double g = doppler_factor(vk[0], vk[1], vk[2], n[0], n[1], n[2]);
                bins[t * r.n_sft + k] = bin_binary(r.f0[t], g, aw, r.omega[t], r.phib[t], r.dt[k], r.t_sft);
            }
            continue;
        }
        for (int k = 0; k < r.n_sft; ++k)
            bins[t * r.n_sft + k] = bin_mode(mode, r.f0[t], r.f1[t], r.dt[k],
                                             r.v + 3 * (int64_t)k, n, r.t_sft, &fallback);
    }
}

// Index mismatches of `mode` against the canonical FP64 bin; one thread per
// template, every SFT.
// count[0] += mismatches, count[1] += evaluations the guarded modes recomputed
// in FP64.
template <bool GRID>
__global__ __launch_bounds__(256) void mismatch_kernel(EvalRun r, int mode,
                                                       unsigned long long *count)
{
    const int64_t n_t = GRID ? (int64_t)r.n_f0 * r.n_f1 * r.n_sky : r.n_list;
    unsigned long long mism = 0, fb = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_t;
         t += (int64_t)gridDim.x * blockDim.x) {
        double f0, f1;
        const double *n;
        if (GRID) {
            const int64_t i = t % r.n_f0;
            const int64_t rest = t / r.n_f0;
            const int64_t j = rest % r.n_f1;
            const int64_t s = rest / r.n_f1;
            f0 = r.f0[i];
            f1 = r.f1[j];
            n = r.sky + 3 * s;
        } else {
            f0 = r.f0[t];
            f1 = r.f1[t];
            n = r.sky + 3 * t;
        }
        int fallback = 0;
        for (int k = 0; k < r.n_sft; ++k) {
            const double *vk = r.v + 3 * (int64_t)k;
            const int ref = bin_canonical(f0, f1, r.dt[k], vk, n, r.t_sft);
            const int got = bin_mode(mode, f0, f1, r.dt[k], vk, n, r.t_sft, &fallback);
            mism += (ref != got);
        }
        fb += (unsigned long long)fallback;
    }
    // wave reduction, one atomic per counter and wave
    for (int off = 32; off > 0; off >>= 1) {
        mism += __shfl_down(mism, off, 64);
        fb += __shfl_down(fb, off, 64);
    }
    if ((threadIdx.x & 63) == 0 && mism) atomicAdd(count, mism);
    if ((threadIdx.x & 63) == 0 && fb) atomicAdd(count + 1, fb);
}

__global__ void check_table_kernel(const float *power, const float *weight, int64_t n_rows,
                                   int64_t n_cols, uint32_t *err)
{
    const int64_t n = n_rows * n_cols;
    bool bad = false;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float p = power[q];
        bad |= !(p >= 0.f && p <= 3.402823466e38f);
    }
    if (weight)
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows;
             q += (int64_t)gridDim.x * blockDim.x) {
            const float w = weight[q];
            bad |= !(w >= 0.f && w <= 3.402823466e38f);
        }
    if (bad) atomicOr(err, ERR_BAD_POWER);
}

__global__ void weight_table_kernel(const float *power, const float *weight, float *out,
                                    int64_t n_rows, int64_t n_cols)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows * n_cols;
         q += (int64_t)gridDim.x * blockDim.x)
        out[q] = power[q] * weight[q / n_cols];
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long value, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = value;
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = value;
}

__global__ void dt_kernel(const double *t_mid, double t_ref, double *dt, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dt[k] = t_mid[k] - t_ref;
}

// dt of every run of a batch: dt[dt_prefix[r] + k] = t_mid[sft_begin[r] + k] - t_ref[r].
__global__ void batch_dt_kernel(const double *t_mid, const int32_t *sft_begin, const double *t_ref,
                                const int64_t *dt_prefix, int n_runs, int64_t total, double *dt)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_runs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (dt_prefix[mid] <= q) lo = mid;
            else hi = mid;
        }
        dt[q] = t_mid[sft_begin[lo] + (q - dt_prefix[lo])] - t_ref[lo];
    }
}

// Moments for per-SFT weights: one wavefront, lane l sums SFTs l, l + 64, ...
// in order, then lane 0 adds the 64 partial sums in lane order (a fixed
// order, so the result does not depend on scheduling).
__global__ void noise_moments_kernel(const float *weight, int n, int stat, double *mu_sigma)
{
    __shared__ double part[2][64];
    const int lane = threadIdx.x;
    if (blockIdx.x != 0 || lane >= 64) return;
    double sw = 0.0, sw2 = 0.0;
    for (int k = lane; k < n; k += 64) {
        const double w = weight ? (double)weight[k] : 1.0;
        sw = sw + w;
        sw2 = sw2 + w * w;
    }
    part[0][lane] = sw;
    part[1][lane] = sw2;
    __syncthreads();
    if (lane == 0) {
        double a = 0.0, b = 0.0;
        for (int l = 0; l < 64; ++l) {
            a = a + part[0][l];
            b = b + part[1][l];
        }
        stat_moments(stat, a, b, mu_sigma);
    }
}

// Number-count tables (Eq. number_count): ind = 1[P > 3.2] and u_k ind.
__global__ void nc_table_kernel(const float *power, const float *weight, float *ind, float *ind_w,
                                int64_t n_rows, int64_t n_cols)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_rows * n_cols;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float b = power[q] >= NC_THRESHOLD_F ? 1.f : 0.f;
        ind[q] = b;
        if (weight) ind_w[q] = b * weight[q / n_cols];
    }
}

// Sky-dependent weights, one wavefront per sky point: norm = 1 / W with
// W = sum_k u_k ab_k(n), then the moments W1 = sum w_k, W2 = sum w_k^2 of
// w_k = u_k (ab_k norm).  All three sums are sequential in SFT order (lanes
// form 256 terms at a time into the wave's LDS slice, lane 0 adds them), the
// canonical order of the oracle, so norm and the moments are bit-exact.
__global__ __launch_bounds__(256) void sky_moments_kernel(const double *arms, const float *weight, int n_sft,
                                                          const double *sky, int64_t n_sky, int stat, double *norm,
                                                          double *ms, uint32_t *err)
{
    __shared__ double sbuf[4][256];
    double *buf = sbuf[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    for (int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); s < n_sky; s += (int64_t)gridDim.x * 4) {
        const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
        const double c1 = sky_norm_sum(arms, weight, n_sft, nx, ny, nz, buf, lane);
        if (!(c1 > 0.0 && c1 < 1e300)) {
            if (lane == 0) {
                atomicOr(err, ERR_BAD_POWER);
                norm[s] = 0.0;
                ms[2 * s] = 0.0;
                ms[2 * s + 1] = 1.0;
            }
            continue;
        }
        const double inv = 1.0 / c1;
        double w1 = 0.0, w2 = 0.0;
        for (int k0 = 0; k0 < n_sft; k0 += 256) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + 64 * j + lane;
                double w = 0.0;
                if (k < n_sft) w = (weight ? (double)weight[k] : 1.0) * (sky_ab(arms + 6 * (int64_t)k, nx, ny, nz) * inv);
                buf[64 * j + lane] = w;
            }
            wave_lds_sync();
            if (lane == 0) {
                const int m = min(256, n_sft - k0);
                for (int q = 0; q < m; ++q) {
                    const double w = buf[q];
                    w1 = w1 + w;
                    w2 = w2 + w * w;
                }
            }
            wave_lds_sync();
        }
        if (lane == 0) {
            norm[s] = inv;
            stat_moments(stat, w1, w2, ms + 2 * s);
        }
    }
}

unsigned grid_for(int64_t n, int block, unsigned cap = 1u << 20)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_eval_list(const EvalRun &run, hipStream_t s)
{
    if (run.n_list <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_direct_kernel<false>, dim3(grid_for(run.n_list, 256, (1u << 22))),
                       dim3(256), 0, s, run);
    return hipGetLastError();
}

hipError_t launch_eval_binary(const EvalRun &run, float *bsum, int n_seg, hipStream_t s)
{
    if (run.n_list <= 0) return hipSuccess;
    const dim3 grid(grid_for(run.n_list, 256, (1u << 16)));
    const bool sky = run.arms != nullptr;
    const int n_blk = (run.n_sft + SUM_BLOCK - 1) / SUM_BLOCK;
    if (bsum && n_seg > 1 && !sky && run.sum_mode == FT_SUM_BLOCKED) {
        const int bps = (n_blk + n_seg - 1) / n_seg;
        const dim3 g2(grid.x, (unsigned)((n_blk + bps - 1) / bps));  // no empty rows
        if (run.cos_delta > 0.0 && run.range_ok)
            hipLaunchKernelGGL((eval_binary_kernel<true, false, false, true>), g2, dim3(256), 0, s, run, bsum, bps);
        else if (run.cos_delta > 0.0)
            hipLaunchKernelGGL((eval_binary_kernel<true, true, false, true>), g2, dim3(256), 0, s, run, bsum, bps);
        else
            hipLaunchKernelGGL((eval_binary_kernel<false, true, false, true>), g2, dim3(256), 0, s, run, bsum, bps);
        hipLaunchKernelGGL(binary_block_sum_kernel, grid, dim3(256), 0, s, (const float *)bsum, run.n_list, n_blk,
                           run.stats);
        return hipGetLastError();
    }
    float *const none = nullptr;
    if (run.cos_delta > 0.0 && run.range_ok) {
        if (sky) hipLaunchKernelGGL((eval_binary_kernel<true, false, true>), grid, dim3(256), 0, s, run, none, 0);
        else hipLaunchKernelGGL((eval_binary_kernel<true, false, false>), grid, dim3(256), 0, s, run, none, 0);
    } else if (run.cos_delta > 0.0) {
        if (sky) hipLaunchKernelGGL((eval_binary_kernel<true, true, true>), grid, dim3(256), 0, s, run, none, 0);
        else hipLaunchKernelGGL((eval_binary_kernel<true, true, false>), grid, dim3(256), 0, s, run, none, 0);
    } else {
        if (sky) hipLaunchKernelGGL((eval_binary_kernel<false, true, true>), grid, dim3(256), 0, s, run, none, 0);
        else hipLaunchKernelGGL((eval_binary_kernel<false, true, false>), grid, dim3(256), 0, s, run, none, 0);
    }
    return hipGetLastError();
}

hipError_t launch_hw_cos_error(unsigned long long *max_bits, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, s, max_bits, 0ull, (int64_t)1);
    hipLaunchKernelGGL(hw_cos_error_kernel, dim3(4096), dim3(256), 0, s, max_bits);
    return hipGetLastError();
}

hipError_t launch_lib_sincos(const double *x, int64_t n, double *c, double *s, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lib_sincos_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, x, n, c, s);
    return hipGetLastError();
}

hipError_t launch_eval_grid_direct(const EvalRun &run, hipStream_t s)
{
    const int64_t n = (int64_t)run.n_f0 * run.n_f1 * run.n_sky;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_direct_kernel<true>, dim3(grid_for(n, 256, (1u << 22))), dim3(256),
                       0, s, run);
    return hipGetLastError();
}

hipError_t launch_eval_batch_small(const EvalRun *runs, const int2 *items, int n_items, int f0_chunk,
                                   unsigned *counter, int grid, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (f0_chunk == 5)
        hipLaunchKernelGGL(eval_batch_small_kernel<5>, dim3((unsigned)grid), dim3(64), 0, s, runs, items, n_items,
                           counter);
    else if (f0_chunk == 8)
        hipLaunchKernelGGL(eval_batch_small_kernel<8>, dim3((unsigned)grid), dim3(64), 0, s, runs, items, n_items,
                           counter);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bins_list(const EvalRun &run, int precision, int32_t *bins, hipStream_t s)
{
    if (run.n_list <= 0) return hipSuccess;
    hipLaunchKernelGGL(bins_list_kernel, dim3(grid_for(run.n_list, 256, (1u << 22))), dim3(256),
                       0, s, run, precision, bins);
    return hipGetLastError();
}

hipError_t launch_count_mismatch(const EvalRun &run, bool grid, int precision,
                                 unsigned long long *count, hipStream_t s)
{
    const int64_t n = grid ? (int64_t)run.n_f0 * run.n_f1 * run.n_sky : run.n_list;
    if (n <= 0) return hipSuccess;
    if (grid)
        hipLaunchKernelGGL(mismatch_kernel<true>, dim3(grid_for(n, 256, (1u << 22))), dim3(256),
                           0, s, run, precision, count);
    else
        hipLaunchKernelGGL(mismatch_kernel<false>, dim3(grid_for(n, 256, (1u << 22))),
                           dim3(256), 0, s, run, precision, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the no-allocation mismatch count.  Each GPU the library runs on
// holds its own copy of this array until the process ends; every call on a
// GPU shares it (calls that overlap on one GPU race).  Host code never names
// the array: it uses the address hipGetSymbolAddress returns on each device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[NOALLOC_HEAD + NOALLOC_MAX_SFT];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// counters[0..1] = 0; dt[k] = t_mid[k] - t_ref (a fill kernel rather than a
// memset, so the sequence may be captured into a graph).
__global__ void noalloc_prep_kernel(const double *t_mid, double t_ref, int n, double *dt,
                                    unsigned long long *counters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) counters[i] = 0ull;
    for (int k = i; k < n; k += gridDim.x * blockDim.x) dt[k] = t_mid[k] - t_ref;
}

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

hipError_t launch_count_mismatch_noalloc(EvalRun run, bool grid, int precision, const double *t_mid, double t_ref,
                                         void *scratch_ptr, hipStream_t s)
{
    if (!scratch_ptr || run.n_sft < 1 || run.n_sft > NOALLOC_MAX_SFT) return hipErrorInvalidValue;
    unsigned long long *counters = (unsigned long long *)scratch_ptr;
    double *dt = (double *)scratch_ptr + NOALLOC_HEAD;
    hipLaunchKernelGGL(noalloc_prep_kernel, dim3(grid_for(run.n_sft, 256, 512)), dim3(256), 0, s, t_mid, t_ref,
                       run.n_sft, dt, counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    run.dt = dt;
    return launch_count_mismatch(run, grid, precision, counters, s);
}

hipError_t launch_check_table(const float *power, const float *weight, int64_t n_rows,
                              int64_t n_cols, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL(check_table_kernel, dim3(grid_for(n_rows * n_cols, 256, 4096)), dim3(256),
                       0, s, power, weight, n_rows, n_cols, err);
    return hipGetLastError();
}

hipError_t launch_weight_table(const float *power, const float *weight, float *out,
                               int64_t n_rows, int64_t n_cols, hipStream_t s)
{
    hipLaunchKernelGGL(weight_table_kernel, dim3(grid_for(n_rows * n_cols, 256, 8192)), dim3(256),
                       0, s, power, weight, out, n_rows, n_cols);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, value,
                       n);
    return hipGetLastError();
}

hipError_t launch_dt(const double *t_mid, double t_ref, double *dt, int n, hipStream_t s)
{
    hipLaunchKernelGGL(dt_kernel, dim3(grid_for(n, 256, (1u << 22))), dim3(256), 0, s, t_mid,
                       t_ref, dt, n);
    return hipGetLastError();
}

hipError_t launch_batch_dt(const double *t_mid, const int32_t *sft_begin, const double *t_ref,
                           const int64_t *dt_prefix, int n_runs, int64_t total, double *dt,
                           hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_dt_kernel, dim3(grid_for(total, 256, 8192)), dim3(256), 0, s, t_mid,
                       sft_begin, t_ref, dt_prefix, n_runs, total, dt);
    return hipGetLastError();
}

hipError_t launch_noise_moments(const float *weight, int n, int stat, double *mu_sigma, hipStream_t s)
{
    hipLaunchKernelGGL(noise_moments_kernel, dim3(1), dim3(64), 0, s, weight, n, stat, mu_sigma);
    return hipGetLastError();
}

hipError_t launch_nc_table(const float *power, const float *weight, float *ind, float *ind_w, int64_t n_rows,
                           int64_t n_cols, hipStream_t s)
{
    hipLaunchKernelGGL(nc_table_kernel, dim3(grid_for(n_rows * n_cols, 256, 8192)), dim3(256), 0, s, power, weight,
                       ind, ind_w, n_rows, n_cols);
    return hipGetLastError();
}

hipError_t launch_sky_moments(const double *arms, const float *weight, int n_sft, const double *sky, int64_t n_sky,
                              int stat, double *norm, double *ms, uint32_t *err, hipStream_t s)
{
    if (n_sky <= 0) return hipSuccess;
    hipLaunchKernelGGL(sky_moments_kernel, dim3(grid_for((n_sky + 3) / 4, 1, 16384)), dim3(256), 0, s, arms, weight,
                       n_sft, sky, n_sky, stat, norm, ms, err);
    return hipGetLastError();
}

}  // namespace ft
