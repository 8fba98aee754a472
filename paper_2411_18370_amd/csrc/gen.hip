// Synthetic SFT tables for injection campaigns: circular complex Gaussian
// noise plus an optional continuous-wave signal (signal hypothesis of
// Sec. II.B.2), generated on the device.
//
// Noise: Re, Im ~ N(0, 1) per (SFT k, bin b), from the counter-based generator
// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) with counter
// (b, k, run, 0) and key (seed_lo, seed_hi); the two 64-bit halves of the
// output give two uniforms (m + 1/2) 2^-53 (m = top 53 bits) for the
// Box-Muller transform (Box and Muller 1958): r = sqrt(-2 ln u1),
// th = 2 pi u2, (Re, Im) = (r cos th, r sin th).  The logarithm, cosine and
// sine are the library's fixed sequences (lib_log, lib_sincos), dot products
// are summed (x0 y0 + x1 y1) + x2 y2, and square roots and divisions are
// correctly rounded, so the tables are one fixed sequence of IEEE operations
// and reproducible bit for bit by any implementation of it.
//
// Signal: in SFT k the track is at x_k = ((f0 + f1 dt_k) g_k) T bins (the
// canonical FP64 track), B_k = floor(x_k + 1/2), delta_k = x_k - B_k; power
// non-centrality rho_k^2 = T amp^2 (F+^2 A+^2 + Fx^2 Ax^2), amp = h0/sqrt(S_n),
// A+ = (1 + cos^2 iota)/2, Ax = cos iota; bins B_k + m (m = -1, 0, 1) receive
// sqrt(rho_k^2) |sinc(pi (delta_k - m))| added to Re.  Antenna patterns:
// F+ = D:e+, Fx = D:ex with D = (u u^T - w w^T)/2 from the arm unit vectors and
// (p, q) = (e_alpha, e_delta) rotated by psi.  Several signals superpose: each
// adds its amplitudes to Re in the order given.
//
// Batch runs generate only the columns their grid bank can reach (per SFT);
// the noise of a column is a function of (seed, run, SFT, column) alone, so
// those columns equal the full table's.
#include "ft_internal.h"

namespace ft {

namespace {

constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(PH_M0, c[0]), lo0 = PH_M0 * c[0];
        const uint32_t hi1 = __umulhi(PH_M1, c[2]), lo1 = PH_M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += PH_W0;
        k1 += PH_W1;
    }
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo)
{
    const uint64_t m = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)m + 0.5) * 0x1p-53;
}

__device__ __forceinline__ double sinc_pi(double d)
{
    const double y = M_PI * d;
    if (y == 0.0) return 1.0;
    double sy, cy;
    lib_sincos(y, sy, cy);
    return sy / y;
}

// Run r of a batch holding global index q, given exclusive prefix sums.
__device__ __forceinline__ int find_run(const int64_t *prefix, int n_runs, int64_t q)
{
    int lo = 0, hi = n_runs;  // last r with prefix[r] <= q
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Polarisation basis (p, q) of a source in direction n: (e_alpha, e_delta)
// rotated by psi (right ascension 0 at a pole).
__device__ __forceinline__ void source_frame(const double *n, double psi, double p[3], double q[3])
{
    const double n0 = n[0], n1 = n[1], n2 = n[2];
    const double rho = sqrt(n0 * n0 + n1 * n1);
    double ea[3], ed[3];
    if (rho > 0.0) {
        ea[0] = -n1 / rho;
        ea[1] = n0 / rho;
        ea[2] = 0.0;
        ed[0] = -n2 * n0 / rho;
        ed[1] = -n2 * n1 / rho;
        ed[2] = rho;
    } else {
        ea[0] = 0.0;
        ea[1] = 1.0;
        ea[2] = 0.0;
        ed[0] = -n2;
        ed[1] = 0.0;
        ed[2] = 0.0;
    }
    double cp, sp;
    lib_sincos(psi, sp, cp);
    for (int i = 0; i < 3; ++i) {
        p[i] = cp * ea[i] + sp * ed[i];
        q[i] = -sp * ea[i] + cp * ed[i];
    }
}

// Antenna patterns F+ = D:e+, Fx = D:ex with D = (u u^T - w w^T)/2 from the arm
// unit vectors arm = (u, w) and e+ = p p^T - q q^T, ex = p q^T + q p^T.
__device__ __forceinline__ void antenna(const double *arm, const double p[3], const double q[3], double &fp,
                                        double &fx)
{
    const double up = arm[0] * p[0] + arm[1] * p[1] + arm[2] * p[2];
    const double uq = arm[0] * q[0] + arm[1] * q[1] + arm[2] * q[2];
    const double wp = arm[3] * p[0] + arm[4] * p[1] + arm[5] * p[2];
    const double wq = arm[3] * q[0] + arm[4] * q[1] + arm[5] * q[2];
    fp = 0.5 * ((up * up - uq * uq) - (wp * wp - wq * wq));
    fx = up * uq - wp * wq;
}

// Per SFT of a run: injection bin and the three bin amplitudes.
// Column range of SFT k that the run's grid bank can reach: the canonical bin
// is monotone in f0, in c = f1 dt and in the Doppler factor g, so the range
// is spanned by the bank's extreme f0, c and g (g over the bank's sky points,
// or over all directions, 1 -+ |v|, for banks of more than 256 points).
__device__ void gen_band_one(const GenRun &g, int k)
{
    const double *v = g.v + 3 * (int64_t)k;
    double gmin, gmax;
    if (g.n_bank_sky <= 256) {
        gmin = 1e300;
        gmax = -1e300;
        for (int s = 0; s < g.n_bank_sky; ++s) {
            const double *n = g.bank_sky + 3 * (int64_t)s;
            const double gs = doppler_factor(v[0], v[1], v[2], n[0], n[1], n[2]);
            gmin = fmin(gmin, gs);
            gmax = fmax(gmax, gs);
        }
    } else {
        const double vabs = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) * (1.0 + 1e-12);
        gmin = 1.0 - vabs;
        gmax = 1.0 + vabs;
    }
    const double dt = g.t_mid[k] - g.t_ref;
    const double c1 = g.bank_f1_lo * dt, c2 = g.bank_f1_hi * dt;
    const int lo = bin_fp64(g.bank_f0_lo, fmin(c1, c2), gmin, g.t_sft) - (int)g.first_bin - 1;
    const int hi = bin_fp64(g.bank_f0_hi, fmax(c1, c2), gmax, g.t_sft) - (int)g.first_bin + 1;
    g.band[2 * k] = max(lo, 0);
    g.band[2 * k + 1] = min(hi, g.n_bins - 1);
}

__device__ void gen_prep_one(const GenRun &g, int k)
{
    if (g.band_mode) gen_band_one(g, k);
    if (g.amp == 0.0) {
        g.inj_bin[k] = INT32_MIN;
        return;
    }
    const double *v = g.v + 3 * (int64_t)k;
    const double gk = doppler_factor(v[0], v[1], v[2], g.sky[0], g.sky[1], g.sky[2]);
    const double dt = g.t_mid[k] - g.t_ref;
    const double c = g.f1 * dt;
    const double a = g.f0 + c;
    double h = gk;
    if (g.ap > 0.0) {  // binary orbit: h = g - (a_p Omega) cos(Omega dt - phi_b)
        double ph = g.omega * dt;
        ph = ph - g.phib;
        double sb, cb;
        lib_sincos(ph, sb, cb);
        const double e = (g.ap * g.omega) * cb;
        h = gk - e;
    }
    const double f = a * h;
    const double x = f * g.t_sft;
    const double B = floor(x + 0.5);
    const double delta = x - B;
    double p[3], q[3];
    source_frame(g.sky, g.psi, p, q);
    double fp, fx;
    antenna(g.arms + 6 * (int64_t)k, p, q, fp, fx);
    const double ap = 0.5 * (1.0 + g.cos_iota * g.cos_iota);
    const double ax = g.cos_iota;
    const double r2 = g.t_sft * g.amp * g.amp * (fp * fp * ap * ap + fx * fx * ax * ax);
    const double sr = sqrt(r2);
    for (int m = -1; m <= 1; ++m) g.inj_amp[3 * k + (m + 1)] = sr * fabs(sinc_pi(delta - (double)m));
    g.inj_bin[k] = (int32_t)B;
}

__global__ void gen_prep_kernel(const GenRun *runs, int n_runs, const int64_t *sft_prefix,
                                int64_t total_sft)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total_sft;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int r = find_run(sft_prefix, n_runs, q);
        gen_prep_one(runs[r], (int)(q - sft_prefix[r]));
    }
}

// Noise (and signals) of the table rows: each wavefront takes four SFT rows,
// sixteen lanes to a row, over the row's columns (its band for batch runs,
// which is a few tens of columns wide for a local bank).
constexpr int kRowLanes = 16;

__global__ __launch_bounds__(256) void gen_noise_kernel(const GenRun *runs, int n_runs,
                                                        const int64_t *row_prefix, int64_t total_rows)
{
    const int lane = threadIdx.x % kRowLanes;
    const int64_t group0 = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
    const int64_t n_groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
    for (int64_t q = group0; q < total_rows; q += n_groups) {
        const int rr = find_run(row_prefix, n_runs, q);
        const GenRun &g = runs[rr];
        const int k = (int)(q - row_prefix[rr]);
        int lo = 0, hi = g.n_bins - 1;
        if (g.band_mode) {
            lo = g.band[2 * k];
            hi = g.band[2 * k + 1];
        }
        float *row = g.table + (int64_t)k * g.n_bins;
        for (int b = lo + lane; b <= hi; b += kRowLanes) {
            uint32_t c[4] = {(uint32_t)b, (uint32_t)(k + g.sft_offset), g.run, 0u};
            philox4x32_10(c, (uint32_t)g.seed, (uint32_t)(g.seed >> 32));
            const double u1 = unit53(c[0], c[1]);
            const double u2 = unit53(c[2], c[3]);
            const double r = sqrt(-2.0 * lib_log(u1));
            const double th = 2.0 * M_PI * u2;
            double sth, cth;
            lib_sincos(th, sth, cth);
            double re = r * cth;
            const double im = r * sth;
            for (int i = 0; i < g.n_inj; ++i) {
                const int64_t ki = (int64_t)i * g.n_sft + k;
                const int32_t B = g.inj_bin[ki];
                if (B == INT32_MIN) continue;
                const int64_t m = g.first_bin + b - (int64_t)B;
                if (m >= -1 && m <= 1) re = re + g.inj_amp[3 * ki + (int)(m + 1)];
            }
            row[b] = (float)(re * re + im * im);
        }
    }
}
// Random template bank of sources in circular binary systems, uniform in the
// binary appendix's xi coordinates (Eq. unif_transform: up to constants xi is
// (f0^6, alpha, sin delta, a_p^3, Omega^4, phi_b)).  Template i draws six
// 53-bit uniforms from three Philox calls with counter (i_lo, i_hi, 0, 1 + j)
// and key (seed_lo, seed_hi) (the noise counters carry word 3 = 0), then
//   f0 = root6(lo^6 + u0 (hi^6 - lo^6)), alpha = alpha_lo + u1 (alpha_hi -
//   alpha_lo), sin delta = sdec_lo + u2 (sdec_hi - sdec_lo), a_p = root3(...u3...),
//   Omega = root4(...u4...), phi_b = phib_lo + u5 (phib_hi - phib_lo),
//   n = (cos delta cos alpha, cos delta sin alpha, sin delta), cos delta =
//   sqrt(1 - sin^2 delta), library cosine/sine of alpha.
// Roots: 12 Newton steps z <- z - (z^p - y)/(p z^(p-1)) from the linear
// interpolation lo + u (hi - lo), powers as z^3 = (z z) z, z^4 = (z z)(z z),
// z^5 = ((z z)(z z)) z, z^6 = ((z z) z)((z z) z): a fixed sequence of IEEE
// operations, so the bank is reproducible bit for bit.
template <int P>
__device__ __forceinline__ double xi_pow(double z)
{
    const double z2 = z * z;
    if (P == 2) return z2;
    if (P == 3) return z2 * z;
    if (P == 4) return z2 * z2;
    if (P == 5) return (z2 * z2) * z;
    const double z3 = z2 * z;
    return z3 * z3;
}

template <int P>
__device__ __forceinline__ double xi_root(double lo, double hi, double u)
{
    const double y = xi_pow<P>(lo) + u * (xi_pow<P>(hi) - xi_pow<P>(lo));
    double z = lo + u * (hi - lo);
    for (int it = 0; it < 12; ++it) z = z - (xi_pow<P>(z) - y) / ((double)P * xi_pow<P - 1>(z));
    return z;
}

__global__ __launch_bounds__(256) void gen_binary_bank_kernel(ft_binary_region reg, uint64_t seed, int64_t first,
                                                              int64_t n, double *f0, double *sky, double *ap,
                                                              double *omega, double *phib, BoxDiv div,
                                                              int32_t *box)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t t = (uint64_t)(first + i);
        double u[6];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), 0u, 1u + (uint32_t)j};
            philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            u[2 * j] = unit53(c[0], c[1]);
            u[2 * j + 1] = unit53(c[2], c[3]);
        }
        f0[i] = xi_root<6>(reg.f0_lo, reg.f0_hi, u[0]);
        const double alpha = reg.alpha_lo + u[1] * (reg.alpha_hi - reg.alpha_lo);
        const double sd = reg.sdec_lo + u[2] * (reg.sdec_hi - reg.sdec_lo);
        const double cd = sqrt(1.0 - sd * sd);
        double sa, ca;
        lib_sincos(alpha, sa, ca);
        sky[3 * i] = cd * ca;
        sky[3 * i + 1] = cd * sa;
        sky[3 * i + 2] = sd;
        ap[i] = xi_root<3>(reg.ap_lo, reg.ap_hi, u[3]);
        omega[i] = xi_root<4>(reg.omega_lo, reg.omega_hi, u[4]);
        phib[i] = reg.phib_lo + u[5] * (reg.phib_hi - reg.phib_lo);
        if (box) {
            // hyperbox of the template: b_d = floor(n_d u_d) (clamped), row-major
            int32_t b = 0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int bd = min((int)floor((double)div.n[d] * u[d]), div.n[d] - 1);
                b = b * div.n[d] + bd;
            }
            box[i] = b;
        }
    }
}

// Signal-response quantities of the semi-analytic sensitivity estimate
// (Sec. V.A: q = (mu_G, sigma_G, rho_hat_1^2, rho_hat_2^2)) for population
// samples (sky n_i, cos iota_i, psi_i), one lane per sample, sums sequential
// in SFT order with the per-SFT weights u_k (1 when absent):
//   mu_G = 2 sum u, sigma_G = 2 sqrt(sum u^2), rho1 = sum u rho_k, rho2 = sum u^2 rho_k,
//   rho_k = T_sft (F+^2 A+^2 + Fx^2 Ax^2), A+ = (1 + cos^2 iota)/2, Ax = cos iota
// (rho_hat^2 of Sec. II.B.2 with the two polarisations in quadrature; the
// power lost to the bin offset is applied by the caller).
__global__ __launch_bounds__(256) void q_sample_kernel(const double *arms, const float *weight, int n_sft,
                                                       double t_sft, const double *sky, const double *cos_iota,
                                                       const double *psi, int64_t n, double *q)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double p[3], qq[3];
        source_frame(sky + 3 * i, psi[i], p, qq);
        const double ci = cos_iota[i];
        const double ap = 0.5 * (1.0 + ci * ci);
        const double ax = ci;
        double s1 = 0.0, s2 = 0.0, r1 = 0.0, r2 = 0.0;
        for (int k = 0; k < n_sft; ++k) {
            double fp, fx;
            antenna(arms + 6 * (int64_t)k, p, qq, fp, fx);
            const double rk = t_sft * (fp * fp * ap * ap + fx * fx * ax * ax);
            const double u = weight ? (double)weight[k] : 1.0;
            s1 = s1 + u;
            s2 = s2 + u * u;
            r1 = r1 + u * rk;
            r2 = r2 + (u * u) * rk;
        }
        q[4 * i] = 2.0 * s1;
        q[4 * i + 1] = 2.0 * sqrt(s2);
        q[4 * i + 2] = r1;
        q[4 * i + 3] = r2;
    }
}

}  // namespace

hipError_t launch_q_sample(const double *arms, const float *weight, int n_sft, double t_sft, const double *sky,
                           const double *cos_iota, const double *psi, int64_t n, double *q, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(q_sample_kernel, dim3((unsigned)blocks), dim3(256), 0, s, arms, weight, n_sft, t_sft, sky,
                       cos_iota, psi, n, q);
    return hipGetLastError();
}

hipError_t launch_gen_binary_bank(const ft_binary_region &reg, uint64_t seed, int64_t first, int64_t n, double *f0,
                                  double *sky, double *ap, double *omega, double *phib, hipStream_t s,
                                  const BoxDiv *div, int32_t *box)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    const BoxDiv d = div ? *div : BoxDiv{{1, 1, 1, 1, 1, 1}};
    hipLaunchKernelGGL(gen_binary_bank_kernel, dim3((unsigned)blocks), dim3(256), 0, s, reg, seed, first, n, f0, sky,
                       ap, omega, phib, d, div ? box : nullptr);
    return hipGetLastError();
}

hipError_t launch_gen_tables(const GenRun *prep, int n_prep, const int64_t *prep_prefix, int64_t total_prep_sft,
                             const GenRun *runs, int n_runs, const int64_t *row_prefix, int64_t total_rows,
                             hipStream_t s)
{
    if (n_prep > 0 && total_prep_sft > 0) {
        int64_t b1 = (total_prep_sft + 255) / 256;
        if (b1 > 16384) b1 = 16384;
        hipLaunchKernelGGL(gen_prep_kernel, dim3((unsigned)b1), dim3(256), 0, s, prep, n_prep, prep_prefix,
                           total_prep_sft);
    }
    if (n_runs > 0 && total_rows > 0) {
        int64_t b2 = (total_rows + 15) / 16;  // sixteen rows per block
        if (b2 > 65536) b2 = 65536;
        hipLaunchKernelGGL(gen_noise_kernel, dim3((unsigned)b2), dim3(256), 0, s, runs, n_runs, row_prefix,
                           total_rows);
    }
    return hipGetLastError();
}

}  // namespace ft
