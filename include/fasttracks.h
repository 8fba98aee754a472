/*
 * fasttracks.h -- C ABI of the MI355X (gfx950) brute-force short-coherence
 * statistic library (arXiv:2411.18370, Secs. II-III).
 *
 * The library evaluates, for every template lambda = (f0, f1, n) of a bank and
 * every SFT k of the data,
 *
 *     f_k(lambda) = (f0 + f1 (t_k - t_ref)) (1 + v_k . n)        (Eq. track,
 *                   isolated source a_p = 0, plus a linear spindown term)
 *     B_k         = floor(f_k T_sft + 1/2)                         (bins of
 *                   width 1/T_sft, Sec. IV.A resolution Eq. resolution)
 *     S(lambda)   = sum_k w_k P[k][B_k - first_bin]               (Eq.
 *                   short_coh_general with the normalised power of Eq. s_tf)
 *
 * and keeps, for every sub-band of f0, the K loudest templates (the list of
 * per-region loudest candidates of Secs. IV.B and VI), each with its critical
 * ratio z = (S - mu_G)/sigma_G, mu_G = 2 sum w, sigma_G = 2 sqrt(sum w^2)
 * (Sec. II.B.1, Eq. critical_ratio).
 *
 * Exactness.  Bin indices are computed in FP64 in the fixed order
 *   d = (vx*nx + vy*ny) + vz*nz ; g = 1 + d ; c = f1*dt ; a = f0 + c ;
 *   f = a*g ; x = f*T_sft ; B = floor(x + 0.5)
 * with no fused multiply-add, so every bin equals the one of a plain FP64
 * evaluation.  Sums run in FP32 over aligned blocks of 32 SFTs, the block sums
 * are accumulated in FP64 (relative error <= 40*2^-24 + 4*N*2^-53 against the
 * FP64 sum).  Toplists are exact: every template whose FP32 statistic could
 * belong to the FP64 top-K is re-summed in FP64 in SFT order and ranked by
 * (S descending, template index ascending).
 *
 * Memory.  Every pointer argument may be host or device memory (HIP unified
 * addressing); every ft_set_* call copies what it is given, so the caller may
 * free or reuse its buffers when the call returns.  Output buffers are owned by
 * the caller.
 *
 * Streams and threads.  A context serialises all its GPU work on one HIP
 * stream (the caller's, or one it owns).  ft_eval_templates is asynchronous;
 * errors detectable on the host are returned synchronously, errors found by
 * the GPU (a track leaving the table) are returned by the next ft_sync /
 * ft_toplist.  A context is not thread-safe: use one per host thread.
 */
#ifndef FASTTRACKS_H
#define FASTTRACKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FT_OK = 0,
    FT_E_INVALID = -1,     /* bad argument: non-finite value, |v| >= 1, |n| != 1, ...     */
    FT_E_STATE = -2,       /* call out of order (eval before set_sfts/set_velocities)     */
    FT_E_RANGE = -3,       /* a track bin lies outside [first_bin, first_bin + n_bins)    */
    FT_E_NOMEM = -4,       /* device allocation failed                                    */
    FT_E_DEVICE = -5,      /* HIP runtime error / no device                               */
    FT_E_UNSUPPORTED = -6, /* valid request outside the library's limits                  */
    FT_E_INTERNAL = -7     /* internal consistency check failed (a bug: please report)    */
} ft_status;

typedef struct ft_ctx_s *ft_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t the
 * context will use (not owned), or NULL for a stream the context owns. */
ft_status ft_create(ft_ctx *out, int device, void *hip_stream);
/* Destroy a context and free its device memory (NULL is a no-op). */
void ft_destroy(ft_ctx ctx);
/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *ft_last_error(ft_ctx ctx);
/* Name of a status code. */
const char *ft_status_string(int status);

/*
 * ft_set_sfts -- the normalised spectrogram (Eq. s_tf) and its timestamps
 * (Sec. II.B: SFTs of duration T_sft labelled by detector X and time index
 * alpha; consecutive timestamps may be further apart than T_sft when there
 * are gaps).
 *   n_det      number of detectors (>= 1)
 *   n_sft      [n_det] SFTs per detector (>= 1 each); N = sum n_sft[d] <= 2^31-1
 *   t_mid      [N] SFT mid-times in seconds, detector-major; the summation order
 *              of the statistic is this order
 *   t_sft      SFT duration in seconds (> 0); bin B has frequency B / t_sft
 *   first_bin  absolute bin index of column 0 of the table (>= 0)
 *   n_bins     columns of the table (>= 1); first_bin + n_bins < 2^31
 *   power      [N][n_bins] row-major normalised power, finite and >= 0
 *   weight     [N] per-SFT weights w_k (finite, >= 0) or NULL for w_k = 1
 * Errors: FT_E_INVALID for any violated condition above.  Invalidates the
 * velocities if N changes.
 */
ft_status ft_set_sfts(ft_ctx ctx, int32_t n_det, const int32_t *n_sft, const double *t_mid,
                      double t_sft, int64_t first_bin, int32_t n_bins, const float *power,
                      const float *weight);

/*
 * ft_set_velocities -- detector velocity at each SFT mid-time, v/c, [N][3] in
 * equatorial Cartesian coordinates (the v(t)/c of Eq. track), same order as
 * t_mid.  Errors: FT_E_STATE before ft_set_sfts; FT_E_INVALID if a value is
 * non-finite or |v| >= 1.
 */
ft_status ft_set_velocities(ft_ctx ctx, const double *v_over_c);

/*
 * ft_set_arms -- unit vectors of the two detector arms at each SFT mid-time,
 * arms[N][6] = (u, w), equatorial Cartesian, same order as t_mid (host or
 * device), for FT_WEIGHTS_SKY.  Errors: FT_E_STATE before ft_set_sfts;
 * FT_E_INVALID if a vector is non-finite or its norm is off 1 by more than
 * 1e-6.  Invalidated when the SFT count changes.
 */
ft_status ft_set_arms(ft_ctx ctx, const double *arms);

enum { FT_BANK_GRID = 0, FT_BANK_LIST = 1, FT_BANK_BINARY = 2 };

/*
 * Template bank (Sec. III: a batch of templates with no assumption on its
 * structure; the grid form is the Cartesian product used by the paper's
 * all-sky setups).
 *   GRID: f0[n_f0] strictly increasing and > 0, f1[n_f1], sky_xyz[n_sky][3]
 *         unit vectors; template index t = (s*n_f1 + j)*n_f0 + i.
 *   LIST: f0[n_list] > 0, f1[n_list], sky_xyz[n_list][3]; template index t.
 *   BINARY: sources in circular binary systems (Eq. track with a_p > 0, no
 *         spindown; the paper's benchmark and search workload):
 *         f0[n_list] > 0, sky_xyz[n_list][3], ap[n_list] (projected semimajor
 *         axis, light-seconds, >= 0), omega[n_list] (orbital angular frequency,
 *         rad/s, >= 0, a_p*Omega < 1/2), phib[n_list] (orbital phase at t_ref,
 *         rad); f1 is ignored.  Track
 *           f_k = f0 (1 + v_k.n - a_p Omega cos(Omega (t_k - t_ref) - phi_b)),
 *         canonical order d = (vx nx + vy ny) + vz nz, g = 1 + d,
 *         ph = Omega dt - phi_b, e = (a_p Omega) lib_cos(ph), f = f0 (g - e),
 *         B = floor(f T + 1/2), lib_cos the library cosine (ft_lib_sincos);
 *         |Omega dt| + |phi_b| < 1.5e6.  Index mode FT_INDEX_FP64 only.
 * Every f0 + f1*(t_k - t_ref) must be > 0.
 */
typedef struct {
    int32_t kind;
    int32_t reserved;
    int64_t n_f0, n_f1, n_sky;
    int64_t n_list;
    const double *f0;
    const double *f1;
    const double *sky_xyz;
    const double *ap, *omega, *phib;  /* BINARY banks only (else ignored) */
} ft_bank;

/*
 * ft_q_sample -- the four signal-response quantities of the semi-analytic
 * sensitivity estimate (Sec. V.A) for population samples i = 0..n-1 (sky
 * unit vectors sky[n][3], cos_iota[n] in [-1, 1], psi[n]) on the context's
 * SFTs (ft_set_sfts: count, T_sft, weights u_k, all 1 when none), with the
 * detectors' arm unit vectors arms[N][6] = (u, w) at the SFT mid-times:
 *   q[i] = (mu_G, sigma_G, rho1, rho2) = (2 sum u, 2 sqrt(sum u^2),
 *           sum u rho_k, sum u^2 rho_k),
 *   rho_k = T_sft (F+^2 A+^2 + Fx^2 Ax^2), A+ = (1 + cos^2 iota)/2,
 *   Ax = cos iota, F+ = D:e+, Fx = D:ex, D = (u u^T - w w^T)/2, (e+, ex) from
 *   the source frame (e_alpha, e_delta) rotated by psi -- rho_hat^2 of
 *   Sec. II.B.2 with the polarisations in quadrature (h0^2/S_n = 1; the bin
 *   offset's power loss is not included).  Sums in FP64, sequential in SFT
 *   order.  q_out[n][4] host or device; synchronous.  Errors: FT_E_STATE
 *   before ft_set_sfts, FT_E_INVALID (inputs).
 */
ft_status ft_q_sample(ft_ctx ctx, const double *arms, int64_t n, const double *sky, const double *cos_iota,
                      const double *psi, double *q_out);

/*
 * ft_lib_sincos -- the library's FP64 cosine and sine (the phase function of
 * BINARY banks): a fixed sequence of IEEE additions and multiplications --
 * Cody-Waite reduction by pi/2 (three-part constant, 33-bit leading parts)
 * and Taylor polynomials to r^17 / r^18 on |r| <= pi/4 in Horner form -- so
 * the same bits come out of any implementation of that sequence.  Within
 * 2^-52 of the exact values.  x[0..n) finite with |x| < 1.5e6 (host or device
 * arrays); cos_out / sin_out [n] (either may be NULL).  Synchronous.
 */
ft_status ft_lib_sincos(ft_ctx ctx, const double *x, int64_t n, double *cos_out, double *sin_out);

enum {
    FT_INDEX_FP64 = 0,         /* exact: canonical FP64 bins (default)                        */
    FT_INDEX_FP32 = 1,         /* study: the same expression in FP32                           */
    FT_INDEX_DF64 = 2,         /* study: unevaluated float-float sums/products, then floor     */
    FT_INDEX_GUARDED = 3,      /* exact: split double-FP32 (df64) estimate verified against
                                  FP64: accepted farther than a derived margin beta =
                                  2^-42 (|x| + |f1 dt| T) + 2^-24 bins from a bin edge,
                                  else the canonical FP64 bin (beta = 4.7e-7 bins at 1 kHz) */
    FT_INDEX_GUARDED_FP32 = 4  /* exact: FP32 estimate with margin 16 2^-24 |x| + 2^-20,
                                  else FP64 (the margin passes half a bin above x = 5.2e5,
                                  i.e. 290 Hz at T = 1800 s: from there on all FP64)        */
};

enum { FT_SUM_BLOCKED = 0, FT_SUM_PLAIN_FP32 = 1 };

/* Detection statistic (Sec. II.B).  POWER: s = sum_k w_k P_k[B_k] (Eq.
 * short_coh_general with the normalised power of Eq. s_tf).  NUMBER_COUNT: the
 * weighted number count nc = sum_k w_k 1[P_k[B_k] > 3.2] (Eq. number_count; P
 * is compared as a real number, i.e. P >= 3.2f for FP32 P). */
enum { FT_STAT_POWER = 0, FT_STAT_NUMBER_COUNT = 1 };

/* SFT weights.  SFT: w_k = u_k, the per-SFT weights of ft_set_sfts (1 when
 * none).  SKY: the all-sky weights of Sec. II.B, w_k(n) = c_k(n) / sum_k' c_k'(n)
 * with c_k(n) = u_k (a_k^2(n) + b_k^2(n)) (u_k in the role of 1/S_n), a, b the
 * detector response functions at the SFT mid-time; a^2 + b^2 = F+^2 + Fx^2 for
 * any polarisation angle, F+ = D:e+, Fx = D:ex, D = (u u^T - w w^T)/2 from the
 * arms of ft_set_arms.  GRID banks (normalised per sky point) and BINARY
 * banks (normalised per template); not LIST banks or the box search. */
enum { FT_WEIGHTS_SFT = 0, FT_WEIGHTS_SKY = 1 };

/* Noise-only moments of the statistics (z = (s - mu)/sigma), with
 * W1 = sum w_k and W2 = sum w_k^2 (sums in FP64):
 *   POWER         mu = 2 W1,     sigma = 2 sqrt(W2)        (Sec. II.B.1)
 *   NUMBER_COUNT  mu = p W1,     sigma = sqrt(p (1-p) W2), p = exp(-1.6), the
 *                 probability that P > 3.2 when P is chi^2 with 2 degrees of
 *                 freedom. */

/*
 * Evaluation options.
 *   precision  FT_INDEX_* (bins of the stored statistic; toplists are always
 *              re-summed with canonical FP64 bins)
 *   k          toplist length per sub-band (1..65536)
 *   n_sub      number of f0 sub-bands (1..4096)
 *   sub_edges  [n_sub+1] strictly increasing; sub-band j is
 *              sub_edges[j] <= f0 < sub_edges[j+1] (templates outside every
 *              sub-band are evaluated but enter no toplist)
 *   sum_mode   FT_SUM_BLOCKED (default) or FT_SUM_PLAIN_FP32 (study only:
 *              toplists are then not guaranteed exact)
 *   tile       0 = library choice (the tile the autotuner cached for this
 *              shape class in this context, else the cost model);
 *              FT_TILE_TUNE = time the eligible tiles first if the class is
 *              not cached (see ft_tune_report); otherwise a tile id in
 *              1..ft_tile_count() (see ft_tile_name); ignored for LIST banks;
 *              with FT_WEIGHTS_SKY the library chooses among the tiles that
 *              have a sky-weighted form (a tile id without one is an error)
 *   statistic  FT_STAT_POWER (default) or FT_STAT_NUMBER_COUNT; stats,
 *              toplists (s32, s64) and z are then of that statistic
 *   weights    FT_WEIGHTS_SFT (default) or FT_WEIGHTS_SKY (GRID and BINARY
 *              banks, after ft_set_arms; the statistic is normalised by
 *              sum w = 1 per sky point and z uses that point's moments)
 */
typedef struct {
    int32_t precision;
    int32_t k;
    int32_t n_sub;
    int32_t sum_mode;
    const double *sub_edges;
    int32_t tile;
    int32_t statistic;  /* FT_STAT_*                                              */
    int32_t weights;    /* FT_WEIGHTS_*                                           */
    int32_t reserved;   /* 0                                                      */
} ft_eval_opts;

/*
 * ft_eval_templates -- evaluate S for every template of `bank` and build the
 * per-sub-band toplists.  `stats` ([n_templates] float, host or device) receives
 * the FP32 statistic of every template in template order, or is NULL.
 * Asynchronous on the context's stream.  Errors: FT_E_STATE (no SFTs or
 * velocities), FT_E_INVALID (bank/options), FT_E_UNSUPPORTED (sizes beyond
 * limits), FT_E_NOMEM; FT_E_RANGE is reported by the next ft_sync/ft_toplist.
 * A BINARY bank of fewer than 2^19 templates with blocked sums and per-SFT
 * weights may keep n_templates * ceil(N / 32) floats (at most 256 MB) of
 * context memory for its per-block sums; the statistics are the same bits
 * either way.
 */
ft_status ft_eval_templates(ft_ctx ctx, const ft_bank *bank, double t_ref,
                            const ft_eval_opts *opts, float *stats);

/*
 * Random template banks of sources in circular binary systems (Sec. IV.A: a
 * random bank drawn uniformly in the uniform-density coordinates, which for
 * this model are, up to constants, (f0^6, alpha, sin delta, a_p^3, Omega^4,
 * phi_b) -- Eq. unif_transform of the binary appendix).  The region is the box
 * [f0_lo, f0_hi] x [alpha_lo, alpha_hi] x [sdec_lo, sdec_hi] x [ap_lo, ap_hi]
 * x [omega_lo, omega_hi] x [phib_lo, phib_hi] (right ascension, sine of the
 * declination; the whole sky and phase range is [0, 2 pi] x [-1, 1] and
 * [0, 2 pi]); lo <= hi everywhere, 0 < lo for f0, a_p and Omega,
 * -1 <= sdec_lo, sdec_hi <= 1, |alpha|, |phi_b| < 1e6, ap_hi * omega_hi < 1/2.
 */
typedef struct {
    double f0_lo, f0_hi;        /* Hz                    */
    double ap_lo, ap_hi;        /* light-seconds         */
    double omega_lo, omega_hi;  /* rad/s                 */
    double alpha_lo, alpha_hi;  /* rad                   */
    double sdec_lo, sdec_hi;    /* sin(declination)      */
    double phib_lo, phib_hi;    /* rad, at t_ref         */
} ft_binary_region;

/*
 * ft_gen_binary_bank -- templates first .. first + n - 1 of the random bank
 * with key `seed`: f0[n], sky_xyz[n][3], ap[n], omega[n], phib[n] (host or
 * device arrays, caller-owned).  Template i depends on (seed, i) only: six
 * 53-bit uniforms (m + 1/2) 2^-53 from Philox-4x32-10 with counter
 * (i_lo, i_hi, 0, 1 + j), j = 0, 1, 2, key (seed_lo, seed_hi); f0, a_p and
 * Omega are p-th roots of lo^p + u (hi^p - lo^p) (p = 6, 3, 4) by 12 Newton
 * steps from lo + u (hi - lo); alpha = alpha_lo + u1 (alpha_hi - alpha_lo),
 * sin delta = sdec_lo + u2 (sdec_hi - sdec_lo), phi_b = phib_lo + u5 (phib_hi
 * - phib_lo), n = (cos delta cos alpha, cos delta sin alpha, sin delta) with
 * cos delta = sqrt(1 - sin^2 delta) and the library cosine/sine -- a fixed
 * sequence of IEEE operations, reproducible bit for bit.  Synchronous.
 * Errors: FT_E_INVALID (region, sizes, null arrays).
 */
ft_status ft_gen_binary_bank(ft_ctx ctx, const ft_binary_region *region, uint64_t seed, int64_t first,
                             int64_t n, double *f0, double *sky_xyz, double *ap, double *omega,
                             double *phib);

/*
 * ft_binary_cos_mode -- how BINARY evaluations estimate the orbital cosine
 * before the guard (the bins are the canonical ones either way).  mode 0
 * (default): the hardware cosine v_cos_f32 when its error, measured on first
 * use over every float in [0, 1] against the library cosine, is at most 1e-4
 * (the guard margin includes it); mode 1: a single-precision Taylor polynomial
 * with a fixed bound.  *hw_err (may be NULL) receives the measured error.
 * Errors: FT_E_INVALID (mode).
 */
ft_status ft_binary_cos_mode(ft_ctx ctx, int32_t mode, double *hw_err);

/*
 * ft_eval_binary_random -- generate templates 0 .. n-1 of the random bank on
 * the device (as ft_gen_binary_bank) and evaluate them as a BINARY bank with
 * `opts` (the paper's timed pipeline: template generation, bins, gathers,
 * sums), building the toplists.  Candidates report f0 and the sky vector;
 * ft_gen_binary_bank(first = index, n = 1) recovers the orbital parameters.
 * Asynchronous; errors as ft_eval_templates.  1 <= n < 2^31.
 */
ft_status ft_eval_binary_random(ft_ctx ctx, const ft_binary_region *region, uint64_t seed, int64_t n,
                                double t_ref, const ft_eval_opts *opts, float *stats);

/*
 * Ahead-of-time hyperbox partition of a random binary bank's region (Sec.
 * IV.B): the uniform-density coordinates xi (f0^6, alpha, sin delta, a_p^3,
 * Omega^4, phi_b) are cut into n_div[d] equal intervals each, so every box
 * holds the same coordinate volume -- the same expected number of templates.
 * Template i lies in box b = (((((b0 n1 + b1) n2 + b2) n3 + b3) n4 + b4) n5 + b5)
 * with b_d = min(floor(n_div[d] * u_d), n_div[d] - 1), u_d the uniform its
 * coordinate d was drawn from (ft_gen_binary_bank: u0 f0, u1 alpha,
 * u2 sin delta, u3 a_p, u4 Omega, u5 phi_b; the product in IEEE FP64).
 * 1 <= n_div[d] <= 2^20, prod n_div <= 2^26.
 */
typedef struct {
    int32_t n_div[6];
    int32_t reserved[2];
} ft_box_partition;

/* The loudest template of one box (index -1 and count 0 for an empty box). */
typedef struct {
    int64_t index;  /* template index in the random bank                          */
    int32_t count;  /* templates of the bank in the box                           */
    float s32;      /* FP32 statistic of the evaluation pass                      */
    double s64;     /* statistic re-summed in FP64 (the box maximum, exactly)      */
    double z;       /* critical ratio (Eq. critical_ratio)                        */
} ft_box_result;

/* One toplist entry. */
typedef struct {
    int64_t index;   /* template index in the bank                              */
    int32_t sub;     /* sub-band                                                */
    float s32;       /* FP32 statistic of the evaluation pass                   */
    double f0, f1;   /* template parameters                                     */
    double n[3];     /* sky unit vector                                         */
    double s64;      /* S re-summed in FP64 in SFT order                        */
    double z;        /* critical ratio (S64 - mu_G)/sigma_G                     */
} ft_candidate;

/*
 * ft_toplist -- copy the toplist of sub-band `sub` of the last evaluation,
 * ordered by (s64 descending, index ascending), into out[0..*n_out-1]
 * (capacity k).  Synchronises the context's stream; returns deferred GPU
 * errors (FT_E_RANGE).
 */
ft_status ft_toplist(ft_ctx ctx, int32_t sub, ft_candidate *out, int32_t *n_out);

/*
 * ft_toplist_number_count -- the exact weighted number count (Eq.
 * number_count, weights as in the evaluation: FP64 sum in SFT order at the
 * canonical bins) of each entry of sub-band `sub`'s toplist of the last
 * evaluation, in toplist order, into nc_out[0..*n_out-1] (capacity k), and
 * its critical ratio (nc - p W1)/sqrt(p (1-p) W2), p = exp(-1.6), W1, W2 the
 * sums of the entry's weights and squared weights, into z_out (may be NULL).  With
 * the POWER statistic this is the persistence check of Sec. VI.B: the loudest
 * template whose number count reaches a minimum is the first entry that
 * reaches it (when none of the k does, it lies deeper than the toplist).
 * Synchronises the context's stream.  Errors as ft_toplist.
 */
ft_status ft_toplist_number_count(ft_ctx ctx, int32_t sub, double *nc_out, double *z_out, int32_t *n_out);

/* Wait for the context's stream and report deferred GPU errors. */
ft_status ft_sync(ft_ctx ctx);

/*
 * ft_eval_binary_boxes -- the search step of Sec. IV.B over a random binary
 * bank: generate templates 0 .. n-1 (as ft_eval_binary_random), evaluate them
 * with opts->statistic and opts->sum_mode (per-SFT weights; k, n_sub,
 * sub_edges and tile are not used) and return the loudest template of every
 * box of `part` in out[0 .. prod n_div - 1] (host or device): the maximum of
 * the FP64 re-summed statistic, ties to the lower index, exact (every
 * template whose FP32 statistic is within the certified bound of its box's
 * FP32 maximum is re-summed).  stats [n] receives the FP32 statistic (or
 * NULL).  Synchronous.  Errors as ft_eval_binary_random; FT_E_INVALID for a
 * partition outside the limits.
 */
ft_status ft_eval_binary_boxes(ft_ctx ctx, const ft_binary_region *region, uint64_t seed, int64_t n,
                               double t_ref, const ft_box_partition *part, const ft_eval_opts *opts,
                               ft_box_result *out, float *stats);

/* Timing and bookkeeping of the last ft_eval_templates (after ft_sync). */
typedef struct {
    double eval_ms;        /* evaluation kernel, HIP events on the context stream     */
    double select_ms;      /* selection + FP64 re-summation + ranking                 */
    int64_t n_templates;
    int64_t n_evals;       /* n_templates * N                                         */
    int64_t n_candidates;  /* templates re-summed in FP64                             */
    int32_t tile;          /* tile id used (1-based; 0 for LIST banks)                */
    int32_t window;        /* LDS window width per SFT (bins)                          */
    int64_t slow_groups;   /* reserved                                                */
} ft_eval_info;
ft_status ft_last_eval_info(ft_ctx ctx, ft_eval_info *info);

/*
 * ft_bins -- study/parity helper: absolute bin B_k of every template of a LIST
 * bank at every SFT, computed with index mode `precision`, into
 * bins[t*N + k] (int32, host or device).  Errors as ft_eval_templates.
 */
ft_status ft_bins(ft_ctx ctx, const ft_bank *bank, double t_ref, int32_t precision,
                  int32_t *bins);

/*
 * ft_count_index_mismatches -- precision study (bins of FT_INDEX_FP32/DF64/
 * GUARDED/GUARDED_FP32 against the canonical FP64 bin; the bins of Sec. IV.A):
 * number of (template, SFT) pairs of `bank` (GRID or LIST) whose bin differs,
 * written to *n_mismatch, and the number of pairs whose estimate a guarded mode
 * did not accept (recomputed in FP64) to *n_fallback (may be NULL; 0 for the
 * unguarded modes).  Synchronous.
 */
ft_status ft_count_index_mismatches(ft_ctx ctx, const ft_bank *bank, double t_ref,
                                    int32_t precision, int64_t *n_mismatch, int64_t *n_fallback);

/*
 * ft_count_index_mismatches_noalloc -- the same count with no device memory
 * allocated, for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Results equal
 * ft_count_index_mismatches's for the same inputs.
 *   bank        GRID or LIST; f0, f1 and sky_xyz are read in place and must be
 *               device memory of the context's GPU holding the sizes the bank
 *               states (n_f0 / n_f1 / n_sky*3, or n_list / n_list / n_list*3);
 *               host pointers are rejected (FT_E_INVALID)
 *   n_mismatch, n_fallback   host pointers (n_fallback may be NULL)
 * Scratch: one fixed device array per GPU held by the library until the
 * process ends (256 B of counters and the N time offsets t_k - t_ref, at most
 * 131072 SFTs, 1 MiB + 256 B); more SFTs give FT_E_UNSUPPORTED.  Every call on
 * a GPU shares that array, so calls that overlap on one GPU (other contexts,
 * other host threads) race; it is cleared by a kernel at the start of each
 * call.  Needs ft_set_sfts and ft_set_velocities first (FT_E_STATE).  Leaves
 * the context's evaluation state untouched.  Synchronous.
 */
ft_status ft_count_index_mismatches_noalloc(ft_ctx ctx, const ft_bank *bank, double t_ref,
                                            int32_t precision, int64_t *n_mismatch, int64_t *n_fallback);

/* One injected continuous-wave signal (Sec. II.B.2).  amp = h0/sqrt(S_n)
 * (the inverse sensitivity depth of Sec. V; 0 = no signal), cos_iota and psi
 * its orientation, sky its unit direction, f0/f1 its frequency and spindown at
 * t_ref.  ap > 0 puts the source in a circular binary orbit (Eq. track):
 * projected semimajor axis ap (light-seconds), orbital angular frequency
 * omega (rad/s), orbital phase phib at t_ref; the track is then
 * x_k = (f0 + f1 dt) (g - (ap omega) lib_cos(omega dt - phib)) T_sft with the
 * library cosine (ft_lib_sincos), the BINARY bank's canonical track for
 * f1 = 0.  ap = 0: an isolated source (omega, phib ignored). */
typedef struct {
    double amp, cos_iota, psi;
    double sky[3];
    double f0, f1;
    double ap, omega, phib;
} ft_injection;

/*
 * ft_gen_sfts -- load a synthetic SFT set whose table the GPU generates
 * (injection campaigns): same SFT arguments as ft_set_sfts (no weights), the
 * velocities of ft_set_velocities, and the detector arm unit vectors
 * arms [N][6] = (u, w) (equatorial) at each mid-time.  Noise: Re, Im ~ N(0, 1)
 * per (bin b, SFT k) from Philox-4x32-10 keyed by `seed` with counter
 * (b, k, run, 0) and Box-Muller; power P = Re^2 + Im^2 (Eq. s_chi2).  Signals
 * (inj[0..n_inj), n_inj <= 64, those with amp > 0; they superpose, each added
 * to Re in the order given): track x_k = (f0 + f1 (t_k - t_ref))(1 + v_k.n)
 * T_sft bins, B_k = floor(x_k + 1/2), delta_k = x_k - B_k; bins B_k + m,
 * m in {-1, 0, 1}, get sqrt(rho_k^2) |sinc(pi (delta_k - m))| added to Re with
 * rho_k^2 = T_sft amp^2 (F+^2 A+^2 + Fx^2 Ax^2), A+ = (1 + cos^2 iota)/2,
 * Ax = cos iota, antenna patterns from D = (u u^T - w w^T)/2 and the source's
 * polarisation frame (e_alpha, e_delta) rotated by psi.  `power_out`
 * ([N][n_bins], host or device) receives a copy of the table, or is NULL.
 * Replaces the SFTs and velocities of the context; errors as ft_set_sfts /
 * ft_set_velocities.
 */
ft_status ft_gen_sfts(ft_ctx ctx, int32_t n_det, const int32_t *n_sft, const double *t_mid,
                      double t_sft, int64_t first_bin, int32_t n_bins, const double *v_over_c,
                      const double *arms, uint64_t seed, uint32_t run, double t_ref,
                      const ft_injection *inj, int32_t n_inj, float *power_out);

/*
 * Batches (many independent runs in one launch: injection campaigns, uneven
 * sub-bands).  Each run has its own SFT subset, table and grid bank, given as
 * slices of shared arrays, and one toplist of length k over all its templates.
 */
typedef struct {
    uint64_t seed;          /* generated tables: Philox key of the run's noise           */
    uint32_t run_id;        /* generated tables: Philox counter word of the run          */
    int32_t sft_begin;      /* first SFT of the run in the batch's SFT arrays            */
    int32_t n_sft;          /* SFTs of the run (>= 1)                                    */
    int32_t n_bins;         /* table columns (1 .. 2^28 - 1)                             */
    int64_t first_bin;      /* absolute bin of column 0                                  */
    int64_t table_offset;   /* given tables: element offset of the run's [n_sft][n_bins] */
    int32_t f0_begin, n_f0; /* grid bank: slices of the batch's f0, f1 and sky arrays    */
    int32_t f1_begin, n_f1;
    int32_t sky_begin, n_sky;
    double t_ref;           /* reference time of the run's f0 and f1                     */
    ft_injection inj;       /* generated tables: injected signal (amp = 0: none)         */
} ft_run;

typedef struct {
    int32_t n_runs;
    int32_t k;              /* toplist length per run (1..512)                           */
    const ft_run *runs;     /* [n_runs]                                                  */
    int32_t n_sft_total;    /* length of the SFT arrays                                  */
    int32_t generate;       /* 1: tables generated on the GPU (as ft_gen_sfts) from the   */
                            /*    runs' seeds and injections; 0: tables given in `power`  */
    const double *t_mid;    /* [n_sft_total] mid-times (s)                               */
    const double *v_over_c; /* [n_sft_total][3]                                          */
    const double *arms;     /* [n_sft_total][6], required when generate = 1              */
    double t_sft;
    int64_t n_f0_total, n_f1_total, n_sky_total;
    const double *f0, *f1, *sky_xyz;
    int64_t power_len;      /* elements of `power` (generate = 0)                        */
    const float *power;     /* concatenated run tables (generate = 0)                    */
    int32_t tile;           /* 0: library choice per run (cached tuned tile of the run's */
                            /*    size class, else the cost model); FT_TILE_TUNE: tune   */
                            /*    uncached classes first; else a tile id for every run   */
    int32_t reserved;
} ft_batch;

/*
 * ft_eval_batch -- evaluate every run of a batch: (optionally) generate the
 * tables, evaluate all (run, tile) work items with one persistent kernel that
 * drains a shared queue, and select each run's exact toplist (as
 * ft_eval_templates with one sub-band covering the run).  use_graph = 1
 * captures the whole launch sequence in a HIP graph and launches it once.
 * Asynchronous; errors as ft_eval_templates.
 */
ft_status ft_eval_batch(ft_ctx ctx, const ft_batch *batch, int32_t use_graph);
/* Relaunch the HIP graph captured by the last ft_eval_batch(use_graph = 1)
 * on the same device buffers (the batch's inputs as then uploaded). */
ft_status ft_batch_replay(ft_ctx ctx);
/* GPU time (ms, HIP events on the context stream) of the last batch launch. */
ft_status ft_batch_time(ft_ctx ctx, double *ms);
/* Toplist of run `run` of the last batch (synchronises). */
ft_status ft_batch_toplist(ft_ctx ctx, int32_t run, ft_candidate *out, int32_t *n_out);
/* Detection labels of the last batch: labels[r] = 1 if the loudest critical
 * ratio of run r exceeds tau (the detection rule R(z; tau), Sec. V.B);
 * max_z[r] receives that critical ratio (either pointer may be NULL). */
ft_status ft_batch_labels(ft_ctx ctx, double tau, uint8_t *labels, double *max_z);

/*
 * Surrogate of the detection probability p_det (Sec. V, Eqs. pdet_abstract
 * and sampling): MLP 6 -> 256 -> 256 -> 256 -> 1 with GELU hidden units and a
 * sigmoid output, trained on detection labels with binary cross-entropy and
 * Adam, on the GPU (BF16 matrix-core products, FP32 accumulation and master
 * weights).  Raw inputs per sample: (h0/sqrt(S_n), cos iota, psi, sin delta,
 * alpha, f); features are (log of the first, the rest as given), standardised
 * as (g - shift)/scale.  Parameters (flat FP32, 133,633): W1 [256][6], b1,
 * W2 [256][256], b2, W3 [256][256], b3, W4 [256], b4.
 */
typedef struct ft_mlp_s *ft_mlp;
/* params: initial parameters (host or device) or NULL for He initialisation
 * from `seed`; max_batch: largest batch of any later call (>= 1). */
ft_status ft_mlp_create(ft_ctx ctx, const float *params, uint64_t seed, const float *feat_shift,
                        const float *feat_scale, int32_t max_batch, ft_mlp *out);
void ft_mlp_destroy(ft_mlp mlp);
ft_status ft_mlp_get_params(ft_mlp mlp, float *params);
/* p[i] = network output for raw inputs raw[i][6], i < n. */
ft_status ft_mlp_predict(ft_mlp mlp, const float *raw, int64_t n, float *p);
/* Mean BCE loss and its gradient (flat, like the parameters) on one batch. */
ft_status ft_mlp_loss_grad(ft_mlp mlp, const float *raw, const float *y, int32_t n, float *loss,
                           float *grad);
/* Adam training: `epochs` passes over n samples in batches of `batch`
 * (a fresh affine permutation of the samples per epoch from `seed`);
 * epoch_loss[e] (or NULL) receives the mean batch loss of epoch e. */
ft_status ft_mlp_train(ft_mlp mlp, const float *raw, const float *y, int64_t n, int32_t batch,
                       int32_t epochs, float lr, uint64_t seed, float *epoch_loss);

/* Tiles of the grid evaluation kernel (for the autotuner and tests); ids are
 * 1..ft_tile_count(), names describe run length L, f1 values JT, waves NW and
 * SFTs per LDS stage KS. */
int32_t ft_tile_count(void);
const char *ft_tile_name(int32_t tile);

/*
 * Tile autotuner (the batching form's tile choice).  A call with
 * tile = FT_TILE_TUNE whose shape class has no cached tile times candidate
 * tiles on the call's own data before evaluating:
 *   GRID bank   class = (n_f0, n_f1, n_sft, floor(log2 n_sky), Doppler
 *               half-width in bins, guard eligibility); every candidate runs
 *               over one contiguous range of the Doppler-ordered sky (about
 *               2.5e11 evaluations, or the whole bank if smaller)
 *   batch       class of a run = (floor(log2 n_f0), min(n_f1, 8), guard
 *               eligibility), runs with n_f0 >= 32 only (smaller f0 grids use
 *               the direct kernel); each pass launches every class's work
 *               items with its next candidate and times each class alone
 * Candidates are the tiles whose cost-model estimate (wasted lanes x VALU
 * operations per evaluation) is within 1.6x of the best and whose LDS window
 * fits; the fastest is cached per context and used by later calls of that
 * class with tile = 0 or FT_TILE_TUNE.  Tuning synchronises the stream and
 * overwrites the statistic buffer (the call then evaluates as usual).
 */
#define FT_TILE_TUNE (-1)

typedef struct {
    int32_t klass;       /* 0 for a GRID call; batch: 1 + class number              */
    int32_t tile;        /* candidate tile id (1-based)                             */
    int32_t chosen;      /* 1 for the tile kept for the class                       */
    int32_t reserved;
    double evals_per_s;  /* measured template-SFT evaluations per second            */
    double sample_evals; /* evaluations timed                                       */
} ft_tune_entry;

/* The timings of the most recent tuning in this context: up to `cap` entries
 * into out[], their number into *n_out, the wall time of the tuning (ms) into
 * *tune_ms (any pointer but n_out may be NULL). */
ft_status ft_tune_report(ft_ctx ctx, ft_tune_entry *out, int32_t cap, int32_t *n_out, double *tune_ms);
/* Forget every cached tile choice of the context. */
ft_status ft_tune_clear(ft_ctx ctx);

/*
 * Achievable rate of the grid kernel's gather-accumulate pattern for `tile`
 * (template-SFT evaluations per second): the tile's lanes gather JT runs of L
 * consecutive values per SFT step from an LDS window of row stride wtp floats
 * (0: the smallest multiple of 64 that holds the pattern) and add them into
 * FP32 accumulators flushed to FP64 every 32 steps, with no index arithmetic,
 * window staging or guard, at the tile's block size, LDS and register budget.
 * Timed with HIP events over 2048 workgroups x 2048 steps; synchronises.  The
 * denominator of the kernel's achieved fraction of its LDS gather ceiling.
 */
ft_status ft_probe_lds_gather(ft_ctx ctx, int32_t tile, int32_t wtp, double *evals_per_s);

/*
 * Chip ceilings measured on the device (the denominators of the roofline
 * fractions; vendor nominal figures are not measurements).
 *
 * ft_probe_lds_read: LDS read bandwidth (bytes per second, whole chip) of one
 * instruction form, FT_LDS_*: 4-wave workgroups, 8 per CU, each lane reading
 * 8 dwords per iteration of a 16 KB LDS array with consecutive lanes at
 * consecutive addresses; consume_all != 0 adds every dword read into an FP32
 * accumulator (the gather-sum's VALU load), 0 adds one per instruction.
 * Timed with HIP events over 2048 workgroups x 4096 iterations after a
 * warm-up launch; synchronises.
 *
 * ft_probe_hbm_read: read bandwidth of HBM (bytes per second) of a streaming
 * kernel (16 bytes per lane per load) over `bytes` of device memory (rounded
 * down to 16 B; at least 1 GiB, so the 256 MB last-level cache cannot hold
 * it), allocated by the call and freed before it returns; synchronises.
 */
enum {
    FT_LDS_B32 = 0,           /* ds_read_b32                                       */
    FT_LDS_READ2ST64 = 1,     /* ds_read2st64_b32: two rows of 64 dwords           */
    FT_LDS_READ2_ADJ = 2,     /* ds_read2_b32 of two adjacent dwords, 4-byte aligned */
    FT_LDS_B64 = 3,           /* ds_read_b64, 8-byte aligned                       */
    FT_LDS_B128 = 4,          /* ds_read_b128, 16-byte aligned                     */
    FT_LDS_READ2ST64_B64 = 5  /* ds_read2st64_b64: two 8-byte pairs 512 bytes apart */
};
ft_status ft_probe_lds_read(ft_ctx ctx, int32_t form, int32_t consume_all, double *bytes_per_s);
ft_status ft_probe_hbm_read(ft_ctx ctx, int64_t bytes, double *bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* FASTTRACKS_H */
