// Internal declarations shared by the HIP translation units of libfasttracks.
// Every file that computes a bin index is compiled with -ffp-contract=off so
// that the FP64 expression below is never fused into an FMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fasttracks.h"

namespace ft {

// Device-side error flags (bit mask in a uint32 owned by the context).
enum : uint32_t {
    ERR_RANGE = 1u,          // a track bin left [first_bin, first_bin + n_bins)
    ERR_WINDOW = 2u,         // a tile needed a wider LDS window than allocated
    ERR_CAND_OVERFLOW = 4u,  // more toplist candidates than the buffer holds
    ERR_BAD_POWER = 8u,      // non-finite or negative power / weight
};

// Blocked-summation length: FP32 partial sums over aligned blocks of this many
// SFTs, accumulated in FP64.
constexpr int SUM_BLOCK = 32;

// ---------------------------------------------------------------------------
// Canonical FP64 track and bin (Eq. track with a_p = 0 plus spindown).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double doppler_factor(double vx, double vy, double vz, double nx,
                                                 double ny, double nz)
{
    double px = vx * nx;
    double py = vy * ny;
    double pz = vz * nz;
    double d = px + py;
    d = d + pz;
    return 1.0 + d;
}

// floor(((f0 + c) * g) * T + 0.5) for positive arguments (truncation == floor).
__device__ __forceinline__ int bin_fp64(double f0, double c, double g, double t_sft)
{
    double a = f0 + c;
    double f = a * g;
    double x = f * t_sft;
    double t = x + 0.5;
    return (int)t;
}

// ---------------------------------------------------------------------------
// Sources in circular binary systems (Eq. track with a_p > 0, no spindown):
// f = f0 (1 + v.n - a_p Omega cos(Omega (t - t_ref) - phi_b)).
// ---------------------------------------------------------------------------
// The library's FP64 cosine and sine: a fixed sequence of IEEE additions and
// multiplications (compiled without contraction), so every implementation of
// the same sequence returns the same bits.  Range reduction after Cody and
// Waite (1980): q = floor(x 2/pi + 1/2), r = ((x - q P1) - q P2) - q P3 with
// pi/2 = P1 + P2 + P3 and P1, P2 of 33 significant bits (exact products for
// |q| < 2^20, i.e. |x| < 1.6e6); Taylor polynomials of sin and cos on
// |r| <= pi/4 (terms to r^17 and r^18, truncation below 1e-19) in Horner form
// with coefficients 1/n! rounded to double; the quadrant q mod 4 picks
// (c, -s, -c, s) for the cosine and (s, c, -s, -c) for the sine.
__device__ __forceinline__ void lib_sincos(double x, double &sin_out, double &cos_out)
{
    const double t = x * 0x1.45f306dc9c883p-1;  // 2/pi
    const double q = floor(t + 0.5);
    double r = x - q * 0x1.921fb54400000p+0;
    r = r - q * 0x1.0b4611a600000p-34;
    r = r - q * 0x1.3198a2e037073p-69;
    const double r2 = r * r;
    double ps = 0x1.952c77030ad4ap-49;                // 1/17!
    ps = ps * r2; ps = ps - 0x1.ae7f3e733b81fp-41;    // 1/15!
    ps = ps * r2; ps = ps + 0x1.6124613a86d09p-33;    // 1/13!
    ps = ps * r2; ps = ps - 0x1.ae64567f544e4p-26;    // 1/11!
    ps = ps * r2; ps = ps + 0x1.71de3a556c734p-19;    // 1/9!
    ps = ps * r2; ps = ps - 0x1.a01a01a01a01ap-13;    // 1/7!
    ps = ps * r2; ps = ps + 0x1.1111111111111p-7;     // 1/5!
    ps = ps * r2; ps = ps - 0x1.5555555555555p-3;     // 1/3!
    const double s = r + (r * r2) * ps;
    double pc = -0x1.6827863b97d97p-53;               // 1/18!
    pc = pc * r2; pc = pc + 0x1.ae7f3e733b81fp-45;    // 1/16!
    pc = pc * r2; pc = pc - 0x1.93974a8c07c9dp-37;    // 1/14!
    pc = pc * r2; pc = pc + 0x1.1eed8eff8d898p-29;    // 1/12!
    pc = pc * r2; pc = pc - 0x1.27e4fb7789f5cp-22;    // 1/10!
    pc = pc * r2; pc = pc + 0x1.a01a01a01a01ap-16;    // 1/8!
    pc = pc * r2; pc = pc - 0x1.6c16c16c16c17p-10;    // 1/6!
    pc = pc * r2; pc = pc + 0x1.5555555555555p-5;     // 1/4!
    const double c = (1.0 - 0.5 * r2) + (r2 * r2) * pc;
    const int n = (int)q & 3;  // |q| < 2^20: the 32-bit conversion is exact
    cos_out = n == 0 ? c : n == 1 ? -s : n == 2 ? -c : s;
    sin_out = n == 0 ? s : n == 1 ? c : n == 2 ? -s : -c;
}

// The library's FP64 natural logarithm for finite normal x > 0, also a fixed
// sequence of IEEE operations: x = m 2^e (frexp, exact), m doubled into
// [sqrt(1/2), sqrt(2)); s = (m - 1)/(m + 1), z = s^2; ln m = 2 atanh(s) =
// 2s + s (z P(z)) with P(z) = sum_{n=1..11} 2/(2n+1) z^(n-1) in Horner form
// (|s| <= 0.1716: the first omitted term is below 2^-57 of ln m); ln x =
// e L_hi + (e L_lo + ln m) with L_hi = ln 2 cut to 42 bits (e L_hi exact for
// |e| < 2^11) and L_lo the rest.  Coefficients are 2/(2n+1) rounded to double.
__device__ __forceinline__ double lib_log(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {  // sqrt(1/2)
        m = m + m;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 2.0 / 23;
    p = p * z; p = p + 2.0 / 21;
    p = p * z; p = p + 2.0 / 19;
    p = p * z; p = p + 2.0 / 17;
    p = p * z; p = p + 2.0 / 15;
    p = p * z; p = p + 2.0 / 13;
    p = p * z; p = p + 2.0 / 11;
    p = p * z; p = p + 2.0 / 9;
    p = p * z; p = p + 2.0 / 7;
    p = p * z; p = p + 2.0 / 5;
    p = p * z; p = p + 2.0 / 3;
    const double lm = (s + s) + s * (z * p);
    const double de = (double)e;
    return de * 0x1.62e42fefa3800p-1 + (de * 0x1.ef35793c76730p-45 + lm);
}

// Canonical bin of a binary-system template at an SFT (offset dt from t_ref,
// Doppler factor g = 1 + v.n in canonical order; aw = a_p * Omega):
// ph = Omega dt - phi_b, e = aw cos(ph), f = f0 (g - e), B = floor(f T + 1/2).
__device__ __forceinline__ int bin_binary(double f0, double g, double aw, double omega, double phib,
                                          double dt, double t_sft)
{
    double ph = omega * dt;
    ph = ph - phib;
    double sb, cb;
    lib_sincos(ph, sb, cb);
    const double e = aw * cb;
    const double h = g - e;
    const double f = f0 * h;
    const double x = f * t_sft;
    const double t = x + 0.5;
    return (int)t;
}

// ---------------------------------------------------------------------------
// All-sky weights (Sec. II.B): a^2 + b^2 = F+^2 + Fx^2 (independent of the
// polarisation angle) of a detector with arm unit vectors u = arm[0..2],
// w = arm[3..5] for a source in direction n.  With D = (u u^T - w w^T)/2 the
// sum is twice the squared norm of D's transverse-traceless part with respect
// to n, which expands to
//   (1 - c^2) - (x^2 + y^2 - 2 c x y) + (x^2 - y^2)^2 / 4,
// x = u.n, y = w.n, c = u.w (1 overhead, 1/4 along an arm, 2/5 on average).
// ---------------------------------------------------------------------------
// (arm: any pointer type to six doubles, e.g. one into the scalar address space)
template <typename ArmPtr>
__device__ __forceinline__ double sky_ab(ArmPtr arm, double nx, double ny, double nz)
{
    const double x = (arm[0] * nx + arm[1] * ny) + arm[2] * nz;
    const double y = (arm[3] * nx + arm[4] * ny) + arm[5] * nz;
    const double c = (arm[0] * arm[3] + arm[1] * arm[4]) + arm[2] * arm[5];
    const double x2 = x * x, y2 = y * y;
    const double dxy = x2 - y2;
    return ((1.0 - c * c) - ((x2 + y2) - 2.0 * (c * x) * y)) + 0.25 * (dxy * dxy);
}

// Orders a wavefront's LDS writes before its own later reads (the lanes of one
// wave run in lock step; this keeps the compiler from reordering across it).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sequential FP64 sum of u_k ab_k(n) over the SFTs k = 0 .. n_sft-1 in SFT order,
// by one wavefront: lanes form 256 terms at a time into buf[256] (the wave's own
// LDS slice) and lane 0 adds them one after another.  Every lane returns the sum.
// This is the normaliser of the all-sky weights w_k = u_k (ab_k / W).
template <typename ArmPtr>
__device__ __forceinline__ double sky_norm_sum(ArmPtr arms, const float *weight, int n_sft, double nx, double ny,
                                               double nz, double *buf, int lane)
{
    double acc = 0.0;
    for (int k0 = 0; k0 < n_sft; k0 += 256) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 64 * j + lane;
            double term = 0.0;
            if (k < n_sft) term = (weight ? (double)weight[k] : 1.0) * sky_ab(arms + 6 * (int64_t)k, nx, ny, nz);
            buf[64 * j + lane] = term;
        }
        wave_lds_sync();
        if (lane == 0) {
            const int m = min(256, n_sft - k0);
            for (int q = 0; q < m; ++q) acc = acc + buf[q];
        }
        wave_lds_sync();
    }
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(acc));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(acc));
    return __hiloint2double(hi, lo);
}

// Number-count threshold (Eq. number_count): P > 3.2 as real numbers, which for
// FP32 P is P >= 3.2f (the float nearest 3.2 lies above it).
constexpr float NC_THRESHOLD_F = 3.2f;

// exp(-1.6): the probability that a chi^2 variable with 2 degrees of freedom
// (the noise-only normalised power) exceeds the number-count threshold 3.2.
constexpr double NC_P = 0x1.9d7bebefb4e15p-3;

// Noise-only (mu, sigma) of statistic `stat` from W1 = sum w, W2 = sum w^2:
// power 2 W1, 2 sqrt(W2) (Sec. II.B.1); number count p W1, sqrt(p (1-p) W2).
__device__ __forceinline__ void stat_moments(int stat, double w1, double w2, double *out)
{
    if (stat == FT_STAT_NUMBER_COUNT) {
        out[0] = NC_P * w1;
        out[1] = sqrt((NC_P * (1.0 - NC_P)) * w2);
    } else {
        out[0] = 2.0 * w1;
        out[1] = 2.0 * sqrt(w2);
    }
}

// The data of one evaluation: an SFT set, its velocities and a grid bank.
struct EvalRun {
    const float *power;   // [n_sft][n_bins]
    const float *power_w; // [n_sft][n_bins], w_k * P[k][b] in FP32 (== power without weights)
    const float *weight;  // [n_sft] or nullptr (all ones)
    const double *dt;     // [n_sft] t_mid - t_ref
    const double *v;      // [n_sft][3]
    const float *v32;     // [n_sft][3] v rounded to float (binary-track estimates)
    const double *f0;     // grid [n_f0] / list [n]
    const double *f1;     // grid [n_f1] / list [n]
    const double *sky;    // grid [n_sky][3] / list [n][3]
    const double *sky_tile;   // grid: sky points in tile (Doppler-coherent) order
    const int32_t *sky_perm;  // grid: tile position -> original sky index
    const double *ap;     // binary list banks: [n] a_p (light-seconds), else nullptr
    const double *omega;  // binary list banks: [n] Omega (rad/s)
    const double *phib;   // binary list banks: [n] phi_b (rad, at t_ref)
    const double *arms;      // [n_sft][6] detector arms (sky-dependent weights), else nullptr
    const double *sky_norm;  // grid: [n_sky] 1 / sum_k u_k (a^2 + b^2)_k(n) per sky point
                             // (original order) -- the sky-dependent weights are on; else nullptr
    const double *sky_ms;    // grid with sky weights: [n_sky][2] (mu, sigma) of the statistic
                             // (binary banks with sky weights: arms set, sky_norm null; the
                             // weights are normalised per template)
    int32_t stat;            // FT_STAT_* of the evaluation (moments of per-template weights)
    float *stats;         // [n_templates]
    uint32_t *err;        // error flags
    int32_t n_sft;
    int32_t n_bins;
    int32_t first_bin;
    int32_t n_f0, n_f1, n_sky;
    int64_t n_list;
    double t_sft;
    double vmax;          // max |v_k| (binary-track estimate bound)
    double cos_delta;     // binary banks: bound of the hardware-cosine estimate (> 0 selects it; else
                          // the polynomial estimate)
    int32_t range_ok;     // binary banks: every track is proved to stay in the table (no per-bin check)
    double dT;            // grid spacing * T_sft (run guard)
    double eta;           // run-guard margin in bins
    int32_t wt;           // LDS window width per SFT (bins, including run padding)
    int32_t wtp;          // wt rounded up to a multiple of 64 (LDS row stride)
    int32_t tiles_f0, tiles_f1, tiles_sky;
    int32_t n_f1_stride;  // grid: f1 count of the output's rows (0: n_f1); a launch over the f1
                          // values [j0, j0 + n_f1) has f1 and stats shifted by j0 (rows) already
    int32_t sum_mode;
    int32_t precision;
};

// Tile configurations of the grid kernel.
struct TileCfg {
    int id;
    const char *name;
    int L;    // consecutive f0 per lane (run length)
    int JT;   // f1 values per workgroup tile
    int NW;   // waves per workgroup = sky points per tile
    int KS;   // SFTs per LDS stage
};
int tile_count();
const TileCfg &tile_cfg(int id);
size_t tile_static_lds(int id);
bool tile_has_sky_weights(int id);  // the tile has a form with sky-dependent weights
// The tile of the same L, NW, KS and register budget with JT = jt, or -1.
int tile_companion(int id, int jt);

// Launchers (stream-ordered, no synchronisation).
hipError_t launch_eval_grid(const EvalRun &run, const TileCfg &cfg, hipStream_t s);
// items[i] = (run, tile within the run); counter must be zero at launch.
hipError_t launch_eval_batch(const EvalRun *runs, const int2 *items, int n_items, int max_wtp,
                             unsigned *counter, int grid, const TileCfg &cfg, hipStream_t s);
// Batch runs outside the tile kernel (one wavefront per item): items[i] =
// (run, chunk), chunk = f0 chunk * ceil(n_f1 n_sky / 64) + (f1, sky) chunk,
// f0 chunks of f0_chunk values (5 or 8; one choice per batch); counter must be
// zero at launch.
hipError_t launch_eval_batch_small(const EvalRun *runs, const int2 *items, int n_items, int f0_chunk,
                                   unsigned *counter, int grid, hipStream_t s);
// Exact per-run toplists of a batch (one workgroup per run, all of a run's
// templates form one segment): out[r*k + rank], n_out[r], max_z[r].
hipError_t launch_select_batch(const EvalRun *runs, int n_runs, int k, int cap_per_run,
                               int64_t *cand, double *cand_s64, ft_candidate *out,
                               int32_t *n_out, double *max_z, uint32_t *err, hipStream_t s);
hipError_t launch_labels(const double *max_z, int n_runs, double tau, uint8_t *labels,
                         hipStream_t s);
hipError_t launch_eval_list(const EvalRun &run, hipStream_t s);
// Binary-system list bank (run.ap/omega/phib set): one lane per template.
// bsum: with n_seg > 1 (blocked sums, no sky weights) the SFT blocks are split
// over n_seg workgroup rows and bsum [ceil(n_sft / SUM_BLOCK)][n_list] holds the
// per-block FP32 sums; else nullptr.
hipError_t launch_eval_binary(const EvalRun &run, float *bsum, int n_seg, hipStream_t s);
// Largest |v_cos_f32(x) - cos 2 pi x| over every float x in [0, 1], as the bit
// pattern of a non-negative double in *max_bits (device memory).
hipError_t launch_hw_cos_error(unsigned long long *max_bits, hipStream_t s);
// The library cosine/sine of x[0..n) into c[], s[] (device arrays).
hipError_t launch_lib_sincos(const double *x, int64_t n, double *c, double *s, hipStream_t st);
hipError_t launch_eval_grid_direct(const EvalRun &run, hipStream_t s);
// LDS gather probe of a tile shape: n_blocks workgroups, n_step SFT steps over
// a staged window of LDS row stride wtp; out [n_blocks * 64 NW] floats.
hipError_t launch_lds_probe(const TileCfg &cfg, int n_blocks, int n_step, int wtp, float *out, hipStream_t s);
// Chip-ceiling microbenchmarks: LDS reads of one FT_LDS_* form (n_blocks
// workgroups of 256 lanes, out [n_blocks * 256]) and a streaming HBM read of
// `bytes` from src (out [n_blocks * 256]).
hipError_t launch_lds_read_probe(int form, bool consume_all, int n_blocks, int n_iter, float *out, hipStream_t s);
hipError_t launch_hbm_read_probe(const void *src, int64_t bytes, int n_blocks, float *out, hipStream_t s);
hipError_t launch_bins_list(const EvalRun &run, int precision, int32_t *bins, hipStream_t s);
hipError_t launch_count_mismatch(const EvalRun &run, bool grid, int precision,
                                 unsigned long long *count, hipStream_t s);
// No-allocation form of the mismatch count (ft_count_index_mismatches_noalloc).
// Its scratch is one fixed device array per GPU: two 64-bit counters in the
// first NOALLOC_HEAD doubles, then dt_k = t_k - t_ref for up to
// NOALLOC_MAX_SFT SFTs (256 B + 1 MiB in all).
constexpr int NOALLOC_HEAD = 32;
constexpr int NOALLOC_MAX_SFT = 131072;
// Resolves the scratch array's address on `device` (which must be current)
// once; later calls return at once.
hipError_t noalloc_scratch_init(int device);
// The scratch address on `device` (nullptr before noalloc_scratch_init).
void *noalloc_scratch_ptr(int device);
// Clears the counters, forms dt into the scratch and counts the mismatches of
// run (whose dt is replaced by the scratch's) into them.
hipError_t launch_count_mismatch_noalloc(EvalRun run, bool grid, int precision, const double *t_mid, double t_ref,
                                         void *scratch_ptr, hipStream_t s);
hipError_t launch_check_table(const float *power, const float *weight, int64_t n_rows,
                              int64_t n_cols, uint32_t *err, hipStream_t s);
hipError_t launch_weight_table(const float *power, const float *weight, float *out,
                               int64_t n_rows, int64_t n_cols, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_dt(const double *t_mid, double t_ref, double *dt, int n, hipStream_t s);
// Noise moments (mu, sigma) of statistic `stat` (FT_STAT_*) for per-SFT weights.
hipError_t launch_noise_moments(const float *weight, int n, int stat, double *mu_sigma, hipStream_t s);
// Number-count tables: ind = 1[P >= 3.2f], ind_w = u_k ind (when weight is non-null).
hipError_t launch_nc_table(const float *power, const float *weight, float *ind, float *ind_w, int64_t n_rows,
                           int64_t n_cols, hipStream_t s);
// Sky-dependent weights of sky points sky[0..n_sky) (original order):
// norm[s] = 1 / sum_k u_k ab_k(n_s) and ms[s] = (mu, sigma) of statistic `stat`
// from W1 = sum w_k, W2 = sum w_k^2, w_k = u_k (ab_k norm[s]).  A sky point
// whose weights sum to zero flags ERR_BAD_POWER.
hipError_t launch_sky_moments(const double *arms, const float *weight, int n_sft, const double *sky, int64_t n_sky,
                              int stat, double *norm, double *ms, uint32_t *err, hipStream_t s);
hipError_t launch_batch_dt(const double *t_mid, const int32_t *sft_begin, const double *t_ref,
                           const int64_t *dt_prefix, int n_runs, int64_t total, double *dt,
                           hipStream_t s);

// One synthetic run of an injection campaign (table generator).
struct GenRun {
    uint64_t seed;
    uint32_t run;
    int32_t sft_offset;   // added to the SFT index in the Philox counter
    int32_t n_sft, n_bins;
    int64_t first_bin;
    const double *t_mid;  // [n_sft]
    const double *v;      // [n_sft][3]
    const float *v32;     // [n_sft][3] v rounded to float (binary-track estimates)
    const double *arms;   // [n_sft][6]
    double t_ref, t_sft;
    double amp, cos_iota, psi, sky[3], f0, f1;
    double ap, omega, phib;  // binary orbit of the signal (ap = 0: isolated)
    float *table;         // [n_sft][n_bins] output
    int32_t *inj_bin;     // [n_inj][n_sft] scratch (a preparation record: [n_sft])
    double *inj_amp;      // [n_inj][n_sft][3] scratch (a preparation record: [n_sft][3])
    int32_t n_inj;        // signals the noise step adds (preparation records: unused)
    // Columns to generate.  band_mode 0: all of them.  band_mode 1 (batch
    // runs): per SFT only [band[2k], band[2k+1]], the columns the run's grid
    // bank (f0 in [bank_f0_lo, bank_f0_hi], f1 in [bank_f1_lo, bank_f1_hi],
    // sky bank_sky[0..n_bank_sky)) can reach; the rest of the table is left
    // as it was (never read by an evaluation of that bank).
    int32_t band_mode;
    int32_t n_bank_sky;
    const double *bank_sky;
    double bank_f0_lo, bank_f0_hi, bank_f1_lo, bank_f1_hi;
    int32_t *band;        // [n_sft][2], written by the preparation step
};
// Generate tables.  prep[0..n_prep) are the per-SFT signal preparations (one
// record per injected signal, each writing its own inj_bin / inj_amp slice,
// and for batch runs the generated column band; prep_prefix: exclusive prefix
// sums of their n_sft, n_prep + 1 entries); runs[0..n_runs) are the tables
// (row_prefix: exclusive prefix sums of their n_sft), each adding its n_inj
// prepared signals to the noise in order.  All arrays on the device.
hipError_t launch_gen_tables(const GenRun *prep, int n_prep, const int64_t *prep_prefix, int64_t total_prep_sft,
                             const GenRun *runs, int n_runs, const int64_t *row_prefix, int64_t total_rows,
                             hipStream_t s);

// Hyperbox partition: divisions of (f0, alpha, sin delta, a_p, Omega, phi_b).
struct BoxDiv {
    int32_t n[6];
};

// Random binary-system bank (uniform in the xi coordinates) of templates
// first .. first + n - 1 into device arrays f0[n], sky[n][3], ap[n],
// omega[n], phib[n]; with a partition, box[n] receives each template's box.
hipError_t launch_gen_binary_bank(const ft_binary_region &reg, uint64_t seed, int64_t first, int64_t n, double *f0,
                                  double *sky, double *ap, double *omega, double *phib, hipStream_t s,
                                  const BoxDiv *div = nullptr, int32_t *box = nullptr);

// Loudest template per hyperbox (templates' FP32 statistics in run.stats, their
// boxes in box[n]): per-box FP32 maximum, candidates within the certified
// bound of it (cand, n_cand = {0, count}; overflow flags ERR_CAND_OVERFLOW),
// FP64 re-summation, per-box FP64 maximum and lowest index, and the results.
struct BoxBufs {
    const int32_t *box;      // [n] box of each template
    uint32_t *max32;         // [n_boxes] FP32 maximum (bits)
    int32_t *count;          // [n_boxes]
    unsigned long long *max64, *idx;  // [n_boxes] FP64 maximum (bits), lowest index attaining it
    int64_t *cand;           // [cap]
    double *cand_s64;        // [cap]
    uint32_t *n_cand;        // [2] = {0, candidates}
    int64_t cap;
};
hipError_t launch_box_max(const EvalRun &run, int64_t n, int64_t n_boxes, const BoxBufs &b, double rel_err,
                          hipStream_t s);
hipError_t launch_box_pick(const EvalRun &run, int64_t n_boxes, const BoxBufs &b, const double *mu_sigma,
                           ft_box_result *out, hipStream_t s);

// Semi-analytic sensitivity: q[i] = (mu_G, sigma_G, rho_hat_1^2, rho_hat_2^2)
// of population samples (sky [n][3], cos_iota [n], psi [n]) for the SFTs'
// arms [n_sft][6] and weights (nullptr: all 1).
hipError_t launch_q_sample(const double *arms, const float *weight, int n_sft, double t_sft, const double *sky,
                           const double *cos_iota, const double *psi, int64_t n, double *q, hipStream_t s);

// Selection: exact toplists per segment (segment = sub-band here).
struct SelectBufs {
    uint32_t *hist;       // [n_seg][256]
    uint32_t *state;      // [n_seg][4]: prefix, mask, k_rem, thr_key
    uint32_t *cnt;        // [n_seg]
    uint32_t *off;        // [n_seg + 1]
    uint32_t *fill;       // [n_seg]
    int64_t *cand;        // [cap]
    double *cand_s64;     // [cap]
    double *cand_mom;     // [cap][2] sums of each candidate's weights and squared weights
    int32_t *seg_of_f0;   // grid [n_f0] or list [n]
    ft_candidate *out;    // [n_seg][k]
    int32_t *n_out;       // [n_seg]
    const double *mu_sigma;
    int64_t cap;
};
hipError_t launch_subband_map(const double *f0, int64_t n, const double *edges, int n_sub,
                              int32_t *seg, hipStream_t s);
hipError_t launch_select(const EvalRun &run, bool grid, int n_seg, int k, double rel_err,
                         const SelectBufs &b, hipStream_t s);
hipError_t launch_rescore_rank(const EvalRun &run, bool grid, int n_seg, int k,
                               const SelectBufs &b, hipStream_t s);
// FP64 re-summation (canonical bins, the run's weights and table) of the
// templates of toplist entries top[0..n_out[0]): out[3i .. 3i+2] = (sum,
// sum w, sum w^2).
hipError_t launch_rescore_entries(const EvalRun &run, bool grid, const ft_candidate *top, const int32_t *n_out,
                                  double *out, hipStream_t s);

// Surrogate MLP (6 -> 256 -> 256 -> 256 -> 1).
constexpr int MLP_H = 256;
constexpr int MLP_OFF_W2 = MLP_H * 6 + MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_W2 + MLP_H * MLP_H + MLP_H;
constexpr int MLP_OFF_W4 = MLP_OFF_W3 + MLP_H * MLP_H + MLP_H;
constexpr int MLP_N_PARAMS = MLP_OFF_W4 + MLP_H + 1;  // 133,633

struct MlpConst {
    float shift[6], scale[6];  // feature standardisation
    int64_t base;              // first sample of the batch (in permuted order)
    int64_t n_total;           // samples in the data set
    uint64_t perm_a, perm_c;   // sample = (perm_a * i + perm_c) mod n_total (perm_a = 0: i)
};

// Gradient reductions: column sums in chunks of MLP_RED_ROWS rows over the
// MLP_RED_VEC entries that are not 256 x 256 weights (W1, b1, b2, b3, W4, b4),
// and the two weight-gradient products in up to MLP_MAX_SLICES batch slices.
constexpr int MLP_RED_ROWS = 64;
constexpr int MLP_RED_VEC = 10 * MLP_H + 1;
constexpr int MLP_MAX_SLICES = 8;

struct MlpBufs {
    float *theta, *m, *v, *grad;
    __bf16 *w2b, *w3b;  // BF16 copies of W2, W3 ([out][in])
    __bf16 *w2t, *w3t;  // and transposed ([in][out])
    float *x, *z1, *z2, *z3, *dz1, *dz2, *dz3, *logit, *dlogit, *loss;
    float *lossv;   // [max_batch] per-sample loss of the current batch
    __bf16 *a1, *a2, *a3, *dz1b, *dz2b, *dz3b;
    float *part;    // [max_batch / MLP_RED_ROWS][MLP_RED_VEC] per-chunk column sums
    float *wpart;   // [2][MLP_MAX_SLICES][MLP_H][MLP_H] per-slice weight gradients
    int max_batch;  // multiple of 64
};
struct MlpAdamStep {
    float lr;
    int t;  // step count, from 1
};
hipError_t mlp_refresh_bf16(const MlpBufs &m, hipStream_t s);
hipError_t mlp_forward(const MlpBufs &m, const float *raw, const float *labels, const MlpConst &c,
                       int bsz, float *prob, hipStream_t s);
hipError_t mlp_backward(const MlpBufs &m, int bsz, const MlpAdamStep *adam, hipStream_t s);

}  // namespace ft
