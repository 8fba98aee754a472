/*
 * FP64 CPU oracle for the short-coherence statistic -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU library.
 * Everything is plain, slow and sequential in the canonical order:
 *
 *   track      f_k   = (f0 + f1 * (t_k - t_ref)) * (1 + v_k . n)
 *              (Eq. track with a_p = 0 -- an isolated source -- plus a linear
 *               spindown term; the Doppler factor has the sign of Eq. track)
 *   bin        B_k   = floor(f_k * T_sft + 1/2)   (bins of width 1/T_sft,
 *                                                   Sec. IV.A resolution)
 *   statistic  S     = sum_k w_k * P[k][B_k - first_bin]
 *                                                  (Eq. short_coh_general)
 *   critical   z     = (S - 2 sum w) / (2 sqrt(sum w^2))
 *                      (mu_G, sigma_G of Sec. II.B.1; Eq. critical_ratio)
 *   toplist    the first K templates of each f0 sub-band under the total
 *              order (S descending, template index ascending).
 *
 * Operation order (fixed, no FMA contraction -- build with -ffp-contract=off):
 *   d = (vx*nx + vy*ny) + vz*nz ; g = 1 + d ; c = f1*dt ; a = f0 + c ;
 *   f = a*g ; x = f*T ; B = floor(x + 0.5) ; S accumulates in SFT order.
 *
 * Status codes: 0 ok, -1 invalid argument, -3 a track left the table.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_RANGE (-3)

/* Doppler factor 1 + v.n (Eq. track, detector-motion term). */
static double doppler_factor(const double *v, const double *n)
{
    double px = v[0] * n[0];
    double py = v[1] * n[1];
    double pz = v[2] * n[2];
    double d = px + py;
    d = d + pz;
    return 1.0 + d;
}

/* Absolute bin index of the track of (f0, f1) at an SFT with offset dt and
 * Doppler factor g. */
static int64_t track_bin(double f0, double f1, double dt, double g, double t_sft)
{
    double c = f1 * dt;
    double a = f0 + c;
    double f = a * g;
    double x = f * t_sft;
    return (int64_t)floor(x + 0.5);
}

static double weight_of(const float *weight, int64_t k)
{
    return weight ? (double)weight[k] : 1.0;
}

/* Bin indices of an arbitrary list of templates: bins[t*n_sft + k] = B (absolute). */
int ftor_bins_list(int32_t n_sft, const double *t_mid, double t_ref, double t_sft,
                   const double *v, int64_t n_tmpl, const double *f0, const double *f1,
                   const double *sky, int64_t *bins)
{
    if (n_sft <= 0 || n_tmpl < 0 || t_sft <= 0.0) return OR_E_INVALID;
    for (int64_t t = 0; t < n_tmpl; ++t) {
        for (int32_t k = 0; k < n_sft; ++k) {
            double g = doppler_factor(v + 3 * (int64_t)k, sky + 3 * t);
            double dt = t_mid[k] - t_ref;
            bins[t * n_sft + k] = track_bin(f0[t], f1[t], dt, g, t_sft);
        }
    }
    return OR_OK;
}

/* Statistic of an arbitrary list of templates.  *first_bad receives the first
 * template whose track leaves [first_bin, first_bin + n_bins), or -1. */
int ftor_eval_list(int32_t n_sft, const double *t_mid, double t_ref, double t_sft,
                   int64_t first_bin, int32_t n_bins, const float *power, const float *weight,
                   const double *v, int64_t n_tmpl, const double *f0, const double *f1,
                   const double *sky, double *s_out, int64_t *first_bad)
{
    if (n_sft <= 0 || n_bins <= 0 || n_tmpl < 0 || t_sft <= 0.0) return OR_E_INVALID;
    int64_t bad = -1;
    for (int64_t t = 0; t < n_tmpl; ++t) {
        double acc = 0.0;
        for (int32_t k = 0; k < n_sft; ++k) {
            double g = doppler_factor(v + 3 * (int64_t)k, sky + 3 * t);
            double dt = t_mid[k] - t_ref;
            int64_t b = track_bin(f0[t], f1[t], dt, g, t_sft) - first_bin;
            if (b < 0 || b >= n_bins) {
                if (bad < 0) bad = t;
                acc = NAN;
                break;
            }
            acc = acc + weight_of(weight, k) * (double)power[(int64_t)k * n_bins + b];
        }
        s_out[t] = acc;
    }
    if (first_bad) *first_bad = bad;
    return bad >= 0 ? OR_E_RANGE : OR_OK;
}

/* Statistic of a grid bank; template index t = (s*n_f1 + j)*n_f0 + i.
 * Sky points are independent, so they run on separate OpenMP threads; every
 * template still accumulates sequentially in SFT order. */
int ftor_eval_grid(int32_t n_sft, const double *t_mid, double t_ref, double t_sft,
                   int64_t first_bin, int32_t n_bins, const float *power, const float *weight,
                   const double *v, int64_t n_f0, const double *f0, int64_t n_f1,
                   const double *f1, int64_t n_sky, const double *sky, double *s_out,
                   int64_t *first_bad)
{
    if (n_sft <= 0 || n_bins <= 0 || n_f0 <= 0 || n_f1 <= 0 || n_sky < 0 || t_sft <= 0.0)
        return OR_E_INVALID;
    const int64_t per_sky = n_f0 * n_f1;
    int64_t bad = -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sky; ++s) {
        double *acc = s_out + s * per_sky;
        for (int64_t q = 0; q < per_sky; ++q) acc[q] = 0.0;
        int64_t local_bad = -1;
        for (int32_t k = 0; k < n_sft; ++k) {
            double g = doppler_factor(v + 3 * (int64_t)k, sky + 3 * s);
            double dt = t_mid[k] - t_ref;
            double w = weight_of(weight, k);
            const float *row = power + (int64_t)k * n_bins;
            for (int64_t j = 0; j < n_f1; ++j) {
                for (int64_t i = 0; i < n_f0; ++i) {
                    int64_t b = track_bin(f0[i], f1[j], dt, g, t_sft) - first_bin;
                    if (b < 0 || b >= n_bins) {
                        int64_t t = s * per_sky + j * n_f0 + i;
                        if (local_bad < 0 || t < local_bad) local_bad = t;
                        acc[j * n_f0 + i] = NAN;
                        continue;
                    }
                    acc[j * n_f0 + i] = acc[j * n_f0 + i] + w * (double)row[b];
                }
            }
        }
        if (local_bad >= 0) {
#pragma omp critical
            { if (bad < 0 || local_bad < bad) bad = local_bad; }
        }
    }
    if (first_bad) *first_bad = bad;
    return bad >= 0 ? OR_E_RANGE : OR_OK;
}

/* ---------------------------------------------------------------------------
 * Sources in circular binary systems (Eq. track with a_p > 0, no spindown).
 *
 *   f_k = f0 * (1 + v_k . n - a_p Omega cos(Omega (t_k - t_ref) - phi_b))
 *
 * (the orbital phase phi_b refers to t_ref).  Canonical operation order:
 *   d = (vx*nx + vy*ny) + vz*nz ; g = 1 + d ; ph = Omega*dt - phi_b ;
 *   cb = pcos(ph) ; e = (a_p*Omega)*cb ; h = g - e ; f = f0*h ; x = f*T ;
 *   B = floor(x + 0.5).
 * With a_p = 0, e = 0 and the bin equals the isolated track's with f1 = 0.
 *
 * pcos/psin: the project's FP64 cosine and sine, a fixed sequence of IEEE
 * additions and multiplications (so any implementation of the same sequence
 * gives the same bits):
 *   range reduction (Cody and Waite, 1980): q = floor(x*2/pi + 1/2),
 *     r = ((x - q*P1) - q*P2) - q*P3 with pi/2 = P1 + P2 + P3, P1 and P2 of
 *     33 significant bits (q*P1, q*P2 exact for |q| < 2^20, i.e. |x| < 1.6e6);
 *   Taylor polynomials on |r| <= pi/4 (truncation below 1e-19), Horner order:
 *     sin r = r + (r*r2)*p_s(r2), p_s = -1/3! + r2(1/5! - r2(1/7! - ... + r2/17!))
 *     cos r = (1 - r2/2) + (r2*r2)*p_c(r2), p_c = 1/4! - r2(1/6! - ... - r2/18!)
 *   quadrant n = q mod 4: cos x = (c, -s, -c, s)[n], sin x = (s, c, -s, -c)[n].
 * Coefficients are 1/n! rounded to double (hex literals).
 * ------------------------------------------------------------------------- */
#define PC_TWO_OVER_PI 0x1.45f306dc9c883p-1
#define PC_P1 0x1.921fb54400000p+0
#define PC_P2 0x1.0b4611a600000p-34
#define PC_P3 0x1.3198a2e037073p-69

static void psincos(double x, double *sin_out, double *cos_out)
{
    double t = x * PC_TWO_OVER_PI;
    double q = floor(t + 0.5);
    double r = x - q * PC_P1;
    r = r - q * PC_P2;
    r = r - q * PC_P3;
    double r2 = r * r;
    double ps = 0x1.952c77030ad4ap-49;            /*  1/17! */
    ps = ps * r2; ps = ps - 0x1.ae7f3e733b81fp-41; /* -1/15! */
    ps = ps * r2; ps = ps + 0x1.6124613a86d09p-33; /*  1/13! */
    ps = ps * r2; ps = ps - 0x1.ae64567f544e4p-26; /* -1/11! */
    ps = ps * r2; ps = ps + 0x1.71de3a556c734p-19; /*  1/9!  */
    ps = ps * r2; ps = ps - 0x1.a01a01a01a01ap-13; /* -1/7!  */
    ps = ps * r2; ps = ps + 0x1.1111111111111p-7;  /*  1/5!  */
    ps = ps * r2; ps = ps - 0x1.5555555555555p-3;  /* -1/3!  */
    double s = r + (r * r2) * ps;
    double pc = -0x1.6827863b97d97p-53;            /* -1/18! */
    pc = pc * r2; pc = pc + 0x1.ae7f3e733b81fp-45; /*  1/16! */
    pc = pc * r2; pc = pc - 0x1.93974a8c07c9dp-37; /* -1/14! */
    pc = pc * r2; pc = pc + 0x1.1eed8eff8d898p-29; /*  1/12! */
    pc = pc * r2; pc = pc - 0x1.27e4fb7789f5cp-22; /* -1/10! */
    pc = pc * r2; pc = pc + 0x1.a01a01a01a01ap-16; /*  1/8!  */
    pc = pc * r2; pc = pc - 0x1.6c16c16c16c17p-10; /* -1/6!  */
    pc = pc * r2; pc = pc + 0x1.5555555555555p-5;  /*  1/4!  */
    double c = (1.0 - 0.5 * r2) + (r2 * r2) * pc;
    int n = (int)((int64_t)q & 3);
    double cv = n == 0 ? c : n == 1 ? -s : n == 2 ? -c : s;
    double sv = n == 0 ? s : n == 1 ? c : n == 2 ? -s : -c;
    if (sin_out) *sin_out = sv;
    if (cos_out) *cos_out = cv;
}

/* The project cosine and sine of x[0..n) (|x| < 1.6e6). */
void ftor_pcos(int64_t n, const double *x, double *c_out, double *s_out)
{
    for (int64_t i = 0; i < n; ++i) psincos(x[i], s_out ? s_out + i : NULL, c_out ? c_out + i : NULL);
}

/* ---------------------------------------------------------------------------
 * plog: the project's FP64 natural logarithm, a fixed sequence of IEEE
 * operations (so any implementation of the same sequence gives the same bits):
 *   x = m 2^e exactly (frexp), m moved into [sqrt(1/2), sqrt(2)) by doubling;
 *   s = (m - 1)/(m + 1), z = s*s;
 *   ln m = 2 atanh(s) = 2s + s*(z*P(z)), P(z) = sum_{n=1..11} 2/(2n+1) z^(n-1)
 *     in Horner order (|s| <= 0.1716, the first omitted term is below 2^-57
 *     of ln m);
 *   ln x = e*LN2_HI + (e*LN2_LO + ln m), LN2_HI = ln 2 cut to 42 bits (so
 *     e*LN2_HI is exact), LN2_LO the rest rounded to double.
 * Defined for finite normal x > 0 (the Box-Muller uniforms lie in
 * [2^-54, 1)).  Coefficients are 2/(2n+1) rounded to double.
 * ------------------------------------------------------------------------- */
#define PL_SQRT_HALF 0x1.6a09e667f3bcdp-1
#define PL_LN2_HI 0x1.62e42fefa3800p-1
#define PL_LN2_LO 0x1.ef35793c76730p-45

static double plog(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < PL_SQRT_HALF) {
        m = m + m;
        e = e - 1;
    }
    double f = m - 1.0;
    double s = f / (m + 1.0);
    double z = s * s;
    double p = 0x1.642c8590b2164p-4;             /* 2/23 */
    p = p * z; p = p + 0x1.8618618618618p-4;     /* 2/21 */
    p = p * z; p = p + 0x1.af286bca1af28p-4;     /* 2/19 */
    p = p * z; p = p + 0x1.e1e1e1e1e1e1ep-4;     /* 2/17 */
    p = p * z; p = p + 0x1.1111111111111p-3;     /* 2/15 */
    p = p * z; p = p + 0x1.3b13b13b13b14p-3;     /* 2/13 */
    p = p * z; p = p + 0x1.745d1745d1746p-3;     /* 2/11 */
    p = p * z; p = p + 0x1.c71c71c71c71cp-3;     /* 2/9  */
    p = p * z; p = p + 0x1.2492492492492p-2;     /* 2/7  */
    p = p * z; p = p + 0x1.999999999999ap-2;     /* 2/5  */
    p = p * z; p = p + 0x1.5555555555555p-1;     /* 2/3  */
    double lm = (s + s) + s * (z * p);
    double de = (double)e;
    return de * PL_LN2_HI + (de * PL_LN2_LO + lm);
}

/* The project logarithm of x[0..n). */
void ftor_plog(int64_t n, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = plog(x[i]);
}

/* ---------------------------------------------------------------------------
 * Campaign noise (test data): Philox-4x32-10 (Salmon, Moraes, Dror and Shaw,
 * SC'11) with counter (bin b, SFT k + sft_offset, run, 0) and key (seed_lo,
 * seed_hi); the two 64-bit halves of its output, top 53 bits m, give the
 * uniforms (m + 1/2) 2^-53; Box-Muller (Box and Muller 1958):
 *   r = sqrt(-2 plog(u1)), th = (2 pi) u2, Re = r pcos(th), Im = r psin(th).
 * ------------------------------------------------------------------------- */
static void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int i = 0; i < 10; ++i) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

/* Philox-4x32-10 of n counters ctr[4n] under key (k0, k1) into out[4n]. */
void ftor_philox(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        philox4x32_10(c, k0, k1);
        for (int j = 0; j < 4; ++j) out[4 * i + j] = c[j];
    }
}

static double unit53(uint32_t hi, uint32_t lo)
{
    uint64_t m = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)m + 0.5) * 0x1p-53;
}

static void noise_pair(uint64_t seed, uint32_t run, uint32_t k, uint32_t b, double *re, double *im)
{
    uint32_t c[4] = {b, k, run, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    double u1 = unit53(c[0], c[1]);
    double u2 = unit53(c[2], c[3]);
    double r = sqrt(-2.0 * plog(u1));
    double th = (2.0 * 0x1.921fb54442d18p+1) * u2;
    double s, co;
    psincos(th, &s, &co);
    *re = r * co;
    *im = r * s;
}

/* (Re, Im) [n_sft][n_bins] of one run's noise. */
void ftor_noise_normals(uint64_t seed, uint32_t run, int32_t n_sft, int32_t n_bins, int64_t sft_offset,
                        double *re, double *im)
{
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < n_sft; ++k)
        for (int32_t b = 0; b < n_bins; ++b)
            noise_pair(seed, run, (uint32_t)(k + sft_offset), (uint32_t)b, re + (int64_t)k * n_bins + b,
                       im + (int64_t)k * n_bins + b);
}

/* FP32 power table [n_sft][n_bins] of one run: noise plus n_inj signals, signal
 * i adding amp[(i n_sft + k) 3 + m + 1] to Re at absolute bin
 * bin[i n_sft + k] + m (m = -1, 0, 1; bin INT64_MIN: none), in signal order. */
void ftor_gen_table(uint64_t seed, uint32_t run, int32_t n_sft, int32_t n_bins, int64_t sft_offset,
                    int64_t first_bin, int32_t n_inj, const int64_t *bin, const double *amp, float *out)
{
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < n_sft; ++k) {
        for (int32_t b = 0; b < n_bins; ++b) {
            double re, im;
            noise_pair(seed, run, (uint32_t)(k + sft_offset), (uint32_t)b, &re, &im);
            for (int32_t i = 0; i < n_inj; ++i) {
                int64_t q = (int64_t)i * n_sft + k;
                if (bin[q] == INT64_MIN) continue;
                int64_t m = first_bin + b - bin[q];
                if (m >= -1 && m <= 1) re = re + amp[3 * q + (m + 1)];
            }
            out[(int64_t)k * n_bins + b] = (float)(re * re + im * im);
        }
    }
}

/* Absolute bin of a binary-system template at an SFT (offset dt, velocity v). */
static int64_t binary_bin(double f0, const double *n, double ap, double omega, double phib,
                          const double *v, double dt, double t_sft)
{
    double g = doppler_factor(v, n);
    double ph = omega * dt;
    ph = ph - phib;
    double cb;
    psincos(ph, NULL, &cb);
    double aw = ap * omega;
    double e = aw * cb;
    double h = g - e;
    double f = f0 * h;
    double x = f * t_sft;
    return (int64_t)floor(x + 0.5);
}

/* Bins of binary templates: bins[t*n_sft + k]. */
int ftor_bins_binary(int32_t n_sft, const double *t_mid, double t_ref, double t_sft, const double *v,
                     int64_t n_tmpl, const double *f0, const double *sky, const double *ap,
                     const double *omega, const double *phib, int64_t *bins)
{
    if (n_sft <= 0 || n_tmpl < 0 || t_sft <= 0.0) return OR_E_INVALID;
    for (int64_t t = 0; t < n_tmpl; ++t)
        for (int32_t k = 0; k < n_sft; ++k)
            bins[t * n_sft + k] = binary_bin(f0[t], sky + 3 * t, ap[t], omega[t], phib[t],
                                             v + 3 * (int64_t)k, t_mid[k] - t_ref, t_sft);
    return OR_OK;
}

/* Statistic of binary templates (sequential FP64 sum in SFT order; templates
 * are independent and run on separate OpenMP threads). */
int ftor_eval_binary(int32_t n_sft, const double *t_mid, double t_ref, double t_sft, int64_t first_bin,
                     int32_t n_bins, const float *power, const float *weight, const double *v, int64_t n_tmpl,
                     const double *f0, const double *sky, const double *ap, const double *omega,
                     const double *phib, double *s_out, int64_t *first_bad)
{
    if (n_sft <= 0 || n_bins <= 0 || n_tmpl < 0 || t_sft <= 0.0) return OR_E_INVALID;
    int64_t bad = -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n_tmpl; ++t) {
        double acc = 0.0;
        for (int32_t k = 0; k < n_sft; ++k) {
            int64_t b = binary_bin(f0[t], sky + 3 * t, ap[t], omega[t], phib[t], v + 3 * (int64_t)k,
                                   t_mid[k] - t_ref, t_sft) - first_bin;
            if (b < 0 || b >= n_bins) {
#pragma omp critical
                { if (bad < 0 || t < bad) bad = t; }
                acc = NAN;
                break;
            }
            acc = acc + weight_of(weight, k) * (double)power[(int64_t)k * n_bins + b];
        }
        s_out[t] = acc;
    }
    if (first_bad) *first_bad = bad;
    return bad >= 0 ? OR_E_RANGE : OR_OK;
}

/* Noise-hypothesis moments: mu_G = 2 sum w, sigma_G = 2 sqrt(sum w^2)
 * (Sec. II.B.1), sums sequential in SFT order. */
void ftor_noise_moments(int32_t n_sft, const float *weight, double *mu, double *sigma)
{
    double sw = 0.0, sw2 = 0.0;
    for (int32_t k = 0; k < n_sft; ++k) {
        double w = weight_of(weight, k);
        sw = sw + w;
        sw2 = sw2 + w * w;
    }
    *mu = 2.0 * sw;
    *sigma = 2.0 * sqrt(sw2);
}

/* Critical ratio z = (S - mu_G)/sigma_G (Eq. critical_ratio). */
void ftor_critical_ratio(int64_t n, const double *s, int32_t n_sft, const float *weight,
                         double *z)
{
    double mu, sigma;
    ftor_noise_moments(n_sft, weight, &mu, &sigma);
    for (int64_t t = 0; t < n; ++t) z[t] = (s[t] - mu) / sigma;
}

/* Sub-band of each frequency: edges[j] <= f < edges[j+1]; -1 outside. */
void ftor_subband(int64_t n, const double *f, int32_t n_sub, const double *edges, int32_t *sub)
{
    for (int64_t t = 0; t < n; ++t) {
        int32_t r = -1;
        for (int32_t j = 0; j < n_sub; ++j)
            if (edges[j] <= f[t] && f[t] < edges[j + 1]) { r = j; break; }
        sub[t] = r;
    }
}

static const double *g_sort_s;
static int cmp_desc_s_asc_idx(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    double sa = g_sort_s[a], sb = g_sort_s[b];
    if (sa > sb) return -1;
    if (sa < sb) return 1;
    return (a < b) ? -1 : (a > b);
}

/* Toplist: for every sub-band j, out_idx[j*k + r] is the r-th template under
 * (S desc, index asc); out_n[j] counts them (<= k).  Not thread-safe. */
int ftor_toplist(int64_t n, const double *s, const int32_t *sub, int32_t n_sub, int32_t k,
                 int64_t *out_idx, int32_t *out_n)
{
    if (k <= 0 || n_sub <= 0) return OR_E_INVALID;
    int64_t *members = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!members) return OR_E_INVALID;
    for (int32_t j = 0; j < n_sub; ++j) {
        int64_t m = 0;
        for (int64_t t = 0; t < n; ++t)
            if (sub[t] == j) members[m++] = t;
        g_sort_s = s;
        qsort(members, (size_t)m, sizeof(int64_t), cmp_desc_s_asc_idx);
        int32_t cnt = (int32_t)(m < k ? m : k);
        for (int32_t r = 0; r < cnt; ++r) out_idx[(int64_t)j * k + r] = members[r];
        for (int32_t r = cnt; r < k; ++r) out_idx[(int64_t)j * k + r] = -1;
        out_n[j] = cnt;
    }
    free(members);
    return OR_OK;
}
