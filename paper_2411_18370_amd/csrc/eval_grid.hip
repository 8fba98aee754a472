// Grid-bank evaluation kernel: S(lambda) = sum_k w_k P[k][B_k] for every
// template of a Cartesian bank f0[n_f0] x f1[n_f1] x sky[n_sky]
// (Eq. short_coh_general; track of Eq. track with a_p = 0 plus spindown).
//
// Workgroup tile: 64*L consecutive f0 values (lane l owns the run
// [i0, i0 + L), i0 = tile_start + l*L) x JT f1 values x NW sky points (one per
// wave; sky points are visited in a Doppler-coherent order chosen by the
// host).  SFTs are processed in stages of KS, double-buffered: while stage p
// is accumulated, the table windows of stage p+1 stream from HBM/L2 straight
// into LDS (global_load_lds), and at every other stage the parameters of the
// next two stages are derived in one pass (a lane per (stage, f1, SFT), so
// that a wave's lanes are busy; parameters in a ring of three stages).
//   prepare(p): Doppler factor g[s][k] (canonical FP64 order), G = g*T_sft,
//      run-guard bounds, c[j][k] = f1_j*dt_k and h = c*G + 1/2 - u_lo - lo; then the
//      exact bin range [lo, hi] of the tile per SFT.  The FP64 bin is monotone
//      in each of f0, c and g and the tile is a Cartesian product, so lo/hi
//      are bins of actual templates: the range check against the table is
//      exact and hi - lo bounds the window.
//   stage(p): row k of the (weighted) power table, columns [lo, lo + wtp),
//      into LDS; columns are clamped into the table (a column outside it can
//      only be read after a range error, which is reported).
//   accumulate(p): for every f1 value each lane forms the estimate
//      t2 = d*G + H (one FP32 fused multiply-add, d = f0 - f0min of the tile,
//      H = f0min*G + h - lo formed in FP64 and rounded once) of
//      x + 1/2 - u_lo - lo for the first template of its run, takes
//      B = floor(t2) -- the LDS row offset of the bin -- and reads B, B+1, ...,
//      B+L-1 (one address per run from a wave-uniform row base, immediate
//      offsets; lanes hit distinct banks for odd L).
//
// Run guard.  |t~ - (x + 1/2)| and the rounding of every canonical evaluation
// are bounded by the host, together with the grid's deviation from uniform
// spacing dT/T_sft, by eta; the FP32 estimate adds the bound of est_err_fp32
// (both together are eta below).  With u = fract(t~) and e = dT*g - 1, template l of
// the run has canonical floor(x_l + 1/2) = floor(t~) + l whenever u + l*e lies
// in [eta, 1 - eta) for every l in [0, L) -- i.e. u in [u_lo, u_hi) with
// u_lo = eta + max(0, -(L-1)e), u_hi = 1 - eta - max(0, (L-1)e) (the expression
// is linear in l).  The kernel forms t2 = t~ - u_lo directly (h carries the
// shift); then u in [u_lo, u_hi) exactly when fract(t2) < u_hi - u_lo, and in
// that case floor(t2) = floor(t~): one compare per run.  The extra rounding of
// the shift is inside eta.  The values at the estimated bins are read first;
// for every f1 value where some lane of the wave fails, the wave then re-reads
// that f1 value's templates at their canonical FP64 bins.  Either way every bin
// equals the canonical FP64 bin.
//
// Whole-wave steps.  On a uniform grid with spacing near one bin, template m
// of the tile has x_m + 1/2 = x_0 + 1/2 + m (1 + e) up to eta, so its
// canonical bin is B0 + m for every m < n_in whenever u0 + m e stays in
// [eta, 1 - eta) at m = 0 and m = n_in - 1 (u0 = fract of the FP64 estimate
// at the first template).  The stage preparation checks this per (sky point,
// SFT, f1) in FP64 and keeps the row offset of B0 and a per-SFT mask; a step
// whose f1 values all pass reads at row offset + lane's first template + l,
// with no per-lane estimate, and the other steps take the run-guard path
// above.
//
// Sums: FP32 within aligned blocks of 32 SFTs, block sums accumulated in FP64.
//
// Sky-dependent weights (SKYW): the staged table holds u_k P (as without
// them), and each accumulation multiplies by the wave's factor
// ab_k(n) / sum_k' u_k' ab_k'(n) of its sky point (one FMA instead of the add),
// formed per SFT in the stage preparation.
#include "ft_internal.h"

#include <cstring>

namespace ft {

namespace {

// One SFT step of one sky point, as the accumulation reads it, in FP32:
// per f1 value H = f0min G + c G + 1/2 - u_lo - lo (so d G + H lands on the
// LDS row offset), G = g T_sft and w = u_hi - u_lo (the run-guard window,
// rounded down).  Two LDS reads per step.
template <int JT>
struct alignas(16) StepParams {
    float h[JT];
    float G, w;
};

// One SFT step of one sky point where the whole wave is certified: per f1
// value the LDS row offset (dwords from the stage's window buffer) of the
// canonical bin of the tile's first template; template m of the tile then has
// bin offset sb + m.
template <int JT>
struct alignas(16) WaveStep {
    int sb[JT];
};

template <int L, int JT, int NW, int KS>
struct StageParams {
    double g[NW][KS];                // canonical Doppler factor
    StepParams<JT> q[NW][KS];        // run-estimate parameters
    WaveStep<JT> ws[NW][KS];         // whole-wave bins (steps whose mask bit is set)
    double c[JT][KS];                // canonical f1 * dt
    float wt[NW][KS];                // sky-dependent weight factor (SKYW)
    int lo[KS];                      // first staged bin
};

template <int L, int JT, int NW, int KS>
struct Shared {
    static_assert(KS <= 64 && NW <= 16, "one lane per SFT of a stage");
    static_assert(SUM_BLOCK % KS == 0, "summation blocks end with a stage");
    // stages prepared per pass: two when both fit a wave's lanes
    static constexpr int NS = 2 * JT * KS <= 64 ? 2 : 1;
    StageParams<L, JT, NW, KS> p[3];  // stages p, p + 1, p + 2 (ring by stage % 3)
    double f0[64 * L];
    int lo_w[NW][NS * KS], hi_w[NW][NS * KS];  // per sky point bin ranges of the stages being prepared
    double vdt[2][4 * NS * KS];  // per pass: v/c [KS][3] then dt [KS] of each stage, prefetched a pass ahead
    double f1[JT], sky[NW][3];       // the tile's f1 values and sky points
    double norm[NW];                 // 1 / sum_k u_k ab_k(n) of the sky points (SKYW)
};

// Asynchronous copy of the velocities and time offsets of SFTs [k0, k0 + ks)
// into dst = [v (3 ks doubles) | pad | dt]: dwords 0..6 KS-1 hold v, dwords
// 6 KS..8 KS-1 hold dt.  Issued by wave 0; lanes past the stage's SFTs copy
// nothing.
template <int KS>
__device__ __forceinline__ void stage_vdt(const EvalRun &r, int k0, int ks, double *dst)
{
    const int lane = threadIdx.x & 63;
    const uint32_t *v = (const uint32_t *)(r.v + 3 * (int64_t)k0);
    const uint32_t *dt = (const uint32_t *)(r.dt + k0);
#pragma unroll
    for (int c = 0; c < (8 * KS + 63) / 64; ++c) {
        const int q = c * 64 + lane;
        const bool is_v = q < 6 * KS;
        const int e = is_v ? q : q - 6 * KS;
        if (q < 8 * KS && e < (is_v ? 6 * ks : 2 * ks))
            __builtin_amdgcn_global_load_lds(is_v ? v + e : dt + e, (uint32_t *)dst + c * 64, 4, 0, 0);
    }
}

__device__ __forceinline__ bool wave_all(bool p)
{
    return __builtin_amdgcn_ballot_w64(!p) == 0;
}

// LDS read of the rare guard-fallback path.  A volatile access keeps the
// compiler from merging it with the fast path's reads (which would force
// computed addresses on the fast path instead of immediate offsets).
typedef __attribute__((address_space(3))) const volatile float lds_vfloat;

__device__ __forceinline__ float slow_read(const float *p)
{
    return *(lds_vfloat *)p;
}



__device__ __forceinline__ void wait_loads()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

struct TileGeom {
    int i_base, i_last, n_in, j_base, j_last, s_base, s_last;
    double f0min, f0max;
};

// Bound (bins) on the error of the FP32 run estimate t2 = fma(d, G, H)
// against the FP64 estimate it replaces, for |d G| <= span and |t2| <= wtp + 2
// (the row offset of a bin inside the window; farther lanes fail the guard):
// the FP32 roundings of d and of G (each <= 2^-24 span), of H = t2 - d G
// (<= 2^-24 (wtp + 2 + span)) and of the fused multiply-add (<= 2^-24
// (wtp + 2)), plus 10^-9 for the FP64 roundings in forming H; 1% margin.
__device__ __forceinline__ double est_err_fp32(const EvalRun &r, const TileGeom &tg)
{
    const double span = (tg.f0max - tg.f0min) * r.t_sft * 1.01 + 1.0;
    return 0x1p-24 * (3.0 * span + 2.0 * ((double)r.wtp + 2.0)) * 1.01 + 1e-9;
}

// Window copies of SFT stage [k0, k0 + ks): rows k0 + kk, columns [lo_kk,
// lo_kk + wtp), wave w taking rows w, w + NW, ...; lo_kk is given by c0_of(kk)
// (wave-uniform).
template <int NW, typename C0>
__device__ __forceinline__ void window_dma(const EvalRun &r, int k0, int ks, float *wbuf, C0 c0_of)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wtp = r.wtp;
    for (int kk = wave; kk < ks; kk += NW) {
        const float *row = r.power_w + (int64_t)(k0 + kk) * r.n_bins;
        const int c0 = c0_of(kk) - r.first_bin;
        float *dst = wbuf + kk * wtp;
        if (c0 >= 0 && c0 <= r.n_bins - wtp) {
            // the whole window lies in the row: scalar base, one lane offset
            const float *src = row + c0;
            for (int x0 = 0; x0 < wtp; x0 += 64)
                __builtin_amdgcn_global_load_lds(src + x0 + lane, dst + x0, 4, 0, 0);
        } else {
            // columns clamped into the row (only after a reported range error
            // can a clamped column be read)
            for (int x0 = 0; x0 < wtp; x0 += 64) {
                const int col = min(max(c0 + lane + x0, 0), r.n_bins - 1);
                __builtin_amdgcn_global_load_lds(row + col, dst + x0, 4, 0, 0);
            }
        }
    }
}

// Parameters and exact windows of SFT stages s0 .. s0 + NS - 1 of a tile
// (one pass; with NS = 2, lane (st, jl, kk) for stage s0 + st, f1 value jl and
// SFT kk, so that the lanes are busy), then the asynchronous HBM/L2 -> LDS
// copies of stage s0's windows (stage s0 + 1's follow a stage later, from its
// stored first bins).  Every wave derives the parameters of its own sky point and that sky
// point's bin range over the tile's f0 and f1 values; one barrier publishes
// the ranges, and every wave takes their union for each SFT (the FP64 bin is
// monotone in f0, c and g, so the union is the exact range of the tile).
// Returns false, in every wave, if a window does not fit the LDS rows
// (flagged).
template <int L, int JT, int NW, int KS, bool SKYW>
__device__ __forceinline__ bool prepare_pair(const EvalRun &r, const TileGeom &tg, int s0,
                                             StageParams<L, JT, NW, KS> &P0, StageParams<L, JT, NW, KS> &P1,
                                             Shared<L, JT, NW, KS> &sh, float *wbuf0, uint64_t &wmask0,
                                             uint64_t &wmask1)
{
    constexpr int NS = Shared<L, JT, NW, KS>::NS;
    const int n_stage = (r.n_sft + KS - 1) / KS;
    const int n_st = NS > 1 && s0 + 1 < n_stage ? 2 : 1;
    const int ks0 = min(KS, r.n_sft - s0 * KS);
    const int ks1 = n_st > 1 ? min(KS, r.n_sft - (s0 + 1) * KS) : 0;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double T = r.t_sft;
    const double nx = sh.sky[wave][0], ny = sh.sky[wave][1], nz = sh.sky[wave][2];
    const double *vdt = sh.vdt[(s0 / NS) & 1];
    const double eta = r.eta + est_err_fp32(r, tg);
    constexpr int NP = JT * KS;            // (jl, kk) pairs of one stage
    constexpr int NQ = (NS * NP + 63) / 64;
    double hq[NQ];  // FP64 H of the lane's (st, jl, kk) before the shift by lo
    int b0q[NQ];    // bin of the tile's first template (valid where okq)
    bool okq[NQ];   // the whole tile's bins are b0q + m
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = lane + 64 * i;
        const int st = q / NP, jl = (q % NP) / KS, kk = q % KS;
        hq[i] = 0.0;
        b0q[i] = 0;
        okq[i] = false;
        if (st >= n_st || kk >= (st ? ks1 : ks0)) continue;
        StageParams<L, JT, NW, KS> &P = st ? P1 : P0;
        const double *vk = vdt + 4 * KS * st + 3 * kk;
        const double g = doppler_factor(vk[0], vk[1], vk[2], nx, ny, nz);
        const double G = g * T;
        const double dt = vdt[4 * KS * st + 3 * KS + kk];
        const double c = sh.f1[jl] * dt;
        const double e = r.dT * g - 1.0;
        const double eL = (double)(L - 1) * e;
        const double ulo = eta + fmax(0.0, -eL);
        hq[i] = ((c * G + 0.5) - ulo) + tg.f0min * G;  // shifted by lo below
        if (L > 1) {
            // whole-tile guard: FP64 estimate of x + 1/2 at the tile's first
            // template, then the run guard over all n_in templates (r.eta
            // bounds the estimate and the grid's spacing error at any offset)
            const double x0 = (c * G + 0.5) + tg.f0min * G;
            const double bf = floor(x0);
            const double u0 = x0 - bf;
            const double span = (double)(tg.n_in - 1) * e;
            okq[i] = u0 + fmin(0.0, span) >= r.eta && u0 + fmax(0.0, span) < 1.0 - r.eta;
            b0q[i] = (int)bf;
        }
        if (wave == 0) P.c[jl][kk] = c;
        if (jl == 0) {
            const int k0 = (s0 + st) * KS;
            P.g[wave][kk] = g;
            if (SKYW) P.wt[wave][kk] = (float)(sky_ab(r.arms + 6 * (int64_t)(k0 + kk), nx, ny, nz) * sh.norm[wave]);
            P.q[wave][kk].G = (float)G;
            // rounded down, so fract(t2) < w in FP32 implies it in real numbers
            if (L > 1) P.q[wave][kk].w = (float)((((1.0 - eta) - fmax(0.0, eL)) - ulo) * (1.0 - 0x1p-22));
            double cmin = c, cmax = c;
#pragma unroll
            for (int j = 1; j < JT; ++j) {
                const double cj = sh.f1[j] * dt;
                cmin = fmin(cmin, cj);
                cmax = fmax(cmax, cj);
            }
            sh.lo_w[wave][st * KS + kk] = bin_fp64(tg.f0min, cmin, g, T);
            sh.hi_w[wave][st * KS + kk] = bin_fp64(tg.f0max, cmax, g, T);
        }
    }
    __syncthreads();
    // the union over the sky points, lane st * KS + kk for stage s0 + st
    int lo = 0;
    bool bad = false;
    {
        const int st = lane / KS, kk = lane % KS;
        if (lane < NS * KS && st < n_st && kk < (st ? ks1 : ks0)) {
            lo = sh.lo_w[0][lane];
            int hi = sh.hi_w[0][lane];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                lo = min(lo, sh.lo_w[w][lane]);
                hi = max(hi, sh.hi_w[w][lane]);
            }
            uint32_t err = 0;
            if (lo < r.first_bin || hi - r.first_bin >= r.n_bins) err |= ERR_RANGE;
            if (hi - lo + L > r.wt) err |= ERR_WINDOW;
            if (wave == 0) {
                (st ? P1 : P0).lo[kk] = lo;
                if (err) atomicOr(r.err, err);
            }
            bad = (err & ERR_WINDOW) != 0;
        }
    }
    if (!wave_all(!bad)) return false;
    // shift the estimates to the first staged bin and round them to FP32 (each
    // lane its own entries; lo is an integer near the estimate, so the FP64
    // difference is exact to an ulp of the window width), and the whole-wave
    // row offsets with their step masks: bit kk is set when every f1 value of
    // step kk is certified and the tile's reads lie inside the window row
    wmask0 = 0;
    wmask1 = 0;
    if (L > 1) {
        const int span_rd = ((tg.n_in - 1) / L) * L + L;  // reads of the last run end here
        uint64_t okm[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = lane + 64 * i;
            const int st = q / NP, jl = (q % NP) / KS, kk = q % KS;
            bool ok = false;
            if (st < n_st && kk < (st ? ks1 : ks0)) {
                StageParams<L, JT, NW, KS> &P = st ? P1 : P0;
                int lo_k = sh.lo_w[0][st * KS + kk];
#pragma unroll
                for (int w = 1; w < NW; ++w) lo_k = min(lo_k, sh.lo_w[w][st * KS + kk]);
                P.q[wave][kk].h[jl] = (float)(hq[i] - (double)lo_k);
                const int off = b0q[i] - lo_k;
                ok = okq[i] && off >= 0 && off + span_rd <= r.wt;
                P.ws[wave][kk].sb[jl] = kk * r.wtp + (ok ? off : 0);
            }
            okm[i] = __builtin_amdgcn_ballot_w64(ok);
        }
        // KS divides 64, so the KS bits of one (stage, f1 value) lie in one
        // mask word
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            uint64_t m = KS >= 64 ? ~0ull : (1ull << KS) - 1;
#pragma unroll
            for (int jl = 0; jl < JT; ++jl) m &= okm[(st * NP + jl * KS) / 64] >> ((st * NP + jl * KS) % 64);
            if (st == 0) wmask0 = m;
            else wmask1 = n_st > 1 ? m : 0;
        }
    }

    // the velocities and time offsets of the next pass's stages (read by it,
    // after the end-of-stage waits)
    if (wave == 0) {
        double *dst = sh.vdt[((s0 + NS) / NS) & 1];
#pragma unroll
        for (int st = 0; st < NS; ++st)
            if ((s0 + NS + st) * KS < r.n_sft)
                stage_vdt<KS>(r, (s0 + NS + st) * KS, min(KS, r.n_sft - (s0 + NS + st) * KS), dst + 4 * KS * st);
    }
    window_dma<NW>(r, s0 * KS, ks0, wbuf0, [&](int kk) { return __builtin_amdgcn_readlane(lo, kk); });
    return true;
}

// Blocked summation: at the end of every aligned block of SUM_BLOCK SFTs the
// FP32 block sums move into the FP64 totals.
template <int L, int JT>
__device__ __forceinline__ void flush_block(const EvalRun &r, int k, float (&acc)[JT][L],
                                            double (&tot)[JT][L])
{
    if (r.sum_mode == FT_SUM_BLOCKED && ((k + 1) & (SUM_BLOCK - 1)) == 0) {
#pragma unroll
        for (int j = 0; j < JT; ++j)
#pragma unroll
            for (int l = 0; l < L; ++l) {
                tot[j][l] += (double)acc[j][l];
                acc[j][l] = 0.f;
            }
    }
}

// The step parameters of (sky point, SFT) read field by field (a whole-struct
// copy loses the alias information that keeps these LDS reads from waiting on
// the window copies in flight).
template <int L, int JT, int NW, int KS>
__device__ __forceinline__ StepParams<JT> load_step(const StageParams<L, JT, NW, KS> &P, int wave, int kk)
{
    StepParams<JT> q;
    q.G = P.q[wave][kk].G;
    q.w = P.q[wave][kk].w;
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) q.h[jl] = P.q[wave][kk].h[jl];
    return q;
}

template <int L, int JT, int NW, int KS>
__device__ __forceinline__ WaveStep<JT> load_wave_step(const StageParams<L, JT, NW, KS> &P, int wave, int kk)
{
    WaveStep<JT> q;
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) q.sb[jl] = P.ws[wave][kk].sb[jl];
    return q;
}

// Run estimates of one SFT step from its parameters (already in registers):
// B[jl] = floor(t2) with t2 = d G + H in FP32 (the LDS row offset of the
// run's first bin; d = f0 - f0min of the lane), and per f1 value the lanes (a
// wave mask) where a run fails the guard fract(t2) < w.  t2 >= -(eta + u_lo)
// (lo is the smallest bin of the tile), so a negative t2 has
// fract(t2) >= 1 - eta - u_lo >= w and fails.  Returns true if some run of
// the wave failed.
template <int JT>
__device__ __forceinline__ bool run_bins(float d_lane, const StepParams<JT> &q, int (&B)[JT], uint64_t (&fail)[JT])
{
    uint64_t any = 0;
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) {
        const float t = __builtin_fmaf(d_lane, q.G, q.h[jl]);
        B[jl] = (int)t;
        fail[jl] = __builtin_amdgcn_ballot_w64(!(__builtin_amdgcn_fractf(t) < q.w));
        any |= fail[jl];
    }
    return any != 0;
}

// Guard fallback of one SFT step: for every f1 value with a failing run, the
// values at the canonical FP64 bins of the lane's run replace the values read
// at the estimated bins (the other f1 values keep theirs).
template <int L, int JT, int NW, int KS>
__device__ __forceinline__ void canonical_fix(const StageParams<L, JT, NW, KS> &P, const Shared<L, JT, NW, KS> &sh,
                                              const TileGeom &tg, const float *wb, int base, int kk, int wave,
                                              int lane, double T, const uint64_t (&fail)[JT], float (&v)[JT][L])
{
    const double g = P.g[wave][kk];
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) {
        if (fail[jl] == 0) continue;
        const double c = P.c[jl][kk];
        int idx[L];
#pragma unroll
        for (int l = 0; l < L; ++l) idx[l] = base + bin_fp64(sh.f0[min(lane * L + l, tg.n_in - 1)], c, g, T);
#pragma unroll
        for (int l = 0; l < L; ++l) v[jl][l] = slow_read(wb + idx[l]);
    }
}

// Software-pipelined accumulation of one stage (run-length tiles).  Step kk
// reads the parameters of step kk+1 from LDS first, then issues its own
// gathers, then forms the bins of step kk+1 while those gathers are in flight,
// and only then adds the gathered values -- or, if some run of the wave failed
// the guard, replaces them by the values at the canonical bins first.  LDS
// returns in order, so the parameter reads never wait behind the gathers.
// The gathers are issued before the guard verdict: an estimate is within one
// bin of the canonical bin, the LDS rows carry that margin, and reads past
// the last row stay inside the workgroup's LDS allocation.
template <int L, int JT, int NW, int KS, bool SKYW>
__device__ __forceinline__ void accumulate_pipelined(const EvalRun &r, const StageParams<L, JT, NW, KS> &P,
                                                     const Shared<L, JT, NW, KS> &sh, const TileGeom &tg,
                                                     const float *wb, int wtp, int k0, int ks, int wave,
                                                     int lane, float d_lane, float (&acc)[JT][L],
                                                     double (&tot)[JT][L])
{
    const double T = r.t_sft;
    int B[JT];
    uint64_t fail[JT];
    bool any = run_bins<JT>(d_lane, load_step<L, JT, NW, KS>(P, wave, 0), B, fail);
    for (int kk = 0; kk < ks; ++kk) {
        const int kn = min(kk + 1, ks - 1);
        const StepParams<JT> qn = load_step<L, JT, NW, KS>(P, wave, kn);
        const float *wk = wb + kk * wtp;
        float v[JT][L];
#pragma unroll
        for (int jl = 0; jl < JT; ++jl)
#pragma unroll
            for (int l = 0; l < L; ++l) v[jl][l] = wk[B[jl] + l];
        int Bn[JT];
        uint64_t fn[JT];
        // keep the next bins ahead of the adds (the compiler would otherwise
        // sink them past the branch, after the wait for the gathers)
        const bool any_next = run_bins<JT>(d_lane, qn, Bn, fn);
#pragma unroll
        for (int jl = 0; jl < JT; ++jl) asm volatile("" ::"v"(Bn[jl]), "s"(fn[jl]));
        if (any)  // rare: some lane is within the guard margin of a bin edge
            canonical_fix<L, JT, NW, KS>(P, sh, tg, wb, kk * wtp - P.lo[kk], kk, wave, lane, T, fail, v);
        if (SKYW) {
            const float wt = P.wt[wave][kk];
#pragma unroll
            for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                for (int l = 0; l < L; ++l) acc[jl][l] = __builtin_fmaf(v[jl][l], wt, acc[jl][l]);
        } else {
#pragma unroll
            for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                for (int l = 0; l < L; ++l) acc[jl][l] += v[jl][l];
        }
        flush_block<L, JT>(r, k0 + kk, acc, tot);
#pragma unroll
        for (int jl = 0; jl < JT; ++jl) {
            B[jl] = Bn[jl];
            fail[jl] = fn[jl];
        }
        any = any_next;
    }
}

template <int L, int JT, int NW, int KS, bool PIPE, bool SKYW>
__device__ __forceinline__ void eval_tile(const EvalRun &r, int64_t b, float *win,
                                          Shared<L, JT, NW, KS> &sh)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nthreads = 64 * NW;

    const int tsky = (int)(b % r.tiles_sky);
    const int64_t rest = b / r.tiles_sky;
    const int tf1 = (int)(rest % r.tiles_f1);
    const int tf0 = (int)(rest / r.tiles_f1);

    TileGeom tg;
    tg.i_base = tf0 * 64 * L;
    tg.i_last = min(tg.i_base + 64 * L, r.n_f0) - 1;
    tg.n_in = tg.i_last - tg.i_base + 1;
    tg.j_base = tf1 * JT;
    tg.j_last = min(tg.j_base + JT, r.n_f1) - 1;
    tg.s_base = tsky * NW;
    tg.s_last = min(tg.s_base + NW, r.n_sky) - 1;
    tg.f0min = r.f0[tg.i_base];
    tg.f0max = r.f0[tg.i_last];

    const double T = r.t_sft;
    const int i0 = tg.i_base + lane * L;
    const double f0_lane = r.f0[min(i0, tg.i_last)];
    const float d_lane = (float)(f0_lane - tg.f0min);  // FP64 difference, one FP32 rounding
    const int wtp = r.wtp;

    __syncthreads();  // the previous tile's threads are done with the shared state
    if (L > 1)
        for (int q = threadIdx.x; q < 64 * L; q += nthreads)
            sh.f0[q] = r.f0[tg.i_base + min(q, tg.n_in - 1)];
    if (threadIdx.x < JT) sh.f1[threadIdx.x] = r.f1[min(tg.j_base + (int)threadIdx.x, tg.j_last)];
    if (threadIdx.x < 3 * NW) {
        const int sl = threadIdx.x / 3, d = threadIdx.x % 3;
        sh.sky[sl][d] = r.sky_tile[3 * (int64_t)min(tg.s_base + sl, tg.s_last) + d];
    }
    if (SKYW && threadIdx.x < NW) sh.norm[threadIdx.x] = r.sky_norm[r.sky_perm[min(tg.s_base + (int)threadIdx.x, tg.s_last)]];
    constexpr int NS = Shared<L, JT, NW, KS>::NS;
    if (wave == 0) {
        stage_vdt<KS>(r, 0, min(KS, r.n_sft), sh.vdt[0]);
        if (NS > 1 && KS < r.n_sft) stage_vdt<KS>(r, KS, min(KS, r.n_sft - KS), sh.vdt[0] + 4 * KS);
    }
    wait_loads();
    __syncthreads();

    float acc[JT][L];
    double tot[JT][L];
#pragma unroll
    for (int j = 0; j < JT; ++j)
#pragma unroll
        for (int l = 0; l < L; ++l) {
            acc[j][l] = 0.f;
            tot[j][l] = 0.0;
        }

    // the lane's first template in the tile (idle lanes repeat the last run)
    const int lane_off = min(lane, (tg.n_in - 1) / L) * L;
    const int n_stage = (r.n_sft + KS - 1) / KS;
    // whole-wave step masks of stages p, p + 1 and p + 2; stage parameters in
    // the ring sh.p[stage % 3], prepared NS stages per pass
    uint64_t wm0 = 0, wm1 = 0, wm2 = 0;
    if (!prepare_pair<L, JT, NW, KS, SKYW>(r, tg, 0, sh.p[0], sh.p[1], sh, win, wm0, wm1)) return;
    wait_loads();
    __syncthreads();

    int slot = 0;  // p % 3
    for (int p = 0; p < n_stage; ++p) {
        const int k0 = p * KS;
        const int ks = min(KS, r.n_sft - k0);
        const int cur = p & 1;
        const int s1 = slot == 2 ? 0 : slot + 1, s2 = s1 == 2 ? 0 : s1 + 1;
        if (p + 1 < n_stage) {
            float *wnext = win + (cur ^ 1) * KS * wtp;
            if ((p + 1) % NS == 0) {
                if (!prepare_pair<L, JT, NW, KS, SKYW>(r, tg, p + 1, sh.p[s1], sh.p[s2], sh, wnext, wm1, wm2))
                    return;
            } else {
                const StageParams<L, JT, NW, KS> &Pn = sh.p[s1];
                window_dma<NW>(r, (p + 1) * KS, min(KS, r.n_sft - (p + 1) * KS), wnext,
                               [&](int kk) { return Pn.lo[kk]; });
            }
        }
        const StageParams<L, JT, NW, KS> &P = sh.p[slot];
        const float *wb = win + cur * KS * wtp;
        const uint64_t wm = wm0;
        wm0 = wm1;
        wm1 = wm2;
        slot = s1;
        if (L > 1 && PIPE) {
            accumulate_pipelined<L, JT, NW, KS, SKYW>(r, P, sh, tg, wb, wtp, k0, ks, wave, lane, d_lane, acc, tot);
        } else
        for (int kk = 0; kk < ks; ++kk) {
            if (L == 1) {
                const int base = kk * wtp - P.lo[kk];
                const double g = P.g[wave][kk];
#pragma unroll
                for (int jl = 0; jl < JT; ++jl) {
                    const int B = bin_fp64(f0_lane, P.c[jl][kk], g, T);
                    if (SKYW) acc[jl][0] = __builtin_fmaf(wb[base + B], P.wt[wave][kk], acc[jl][0]);
                    else acc[jl][0] += wb[base + B];
                }
            } else {
                float v[JT][L];
                if ((wm >> kk) & 1) {
                    // the whole wave is certified: bins sb + lane_off + l
                    const WaveStep<JT> q = load_wave_step<L, JT, NW, KS>(P, wave, kk);
                    const float *wl = wb + lane_off;
#pragma unroll
                    for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                        for (int l = 0; l < L; ++l) v[jl][l] = wl[q.sb[jl] + l];
                } else {
                    // reads at the estimated bins first; the rare failing f1
                    // values (some lane within the guard margin of a bin edge)
                    // are then re-read at their canonical bins
                    const StepParams<JT> q = load_step<L, JT, NW, KS>(P, wave, kk);
                    int B[JT];
                    uint64_t fail[JT];
                    const bool any = run_bins<JT>(d_lane, q, B, fail);
                    const float *wk = wb + kk * wtp;
#pragma unroll
                    for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                        for (int l = 0; l < L; ++l) v[jl][l] = wk[B[jl] + l];
                    if (any)
                        canonical_fix<L, JT, NW, KS>(P, sh, tg, wb, kk * wtp - P.lo[kk], kk, wave, lane, T, fail, v);
                }
                if (SKYW) {
                    const float wt = P.wt[wave][kk];
#pragma unroll
                    for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                        for (int l = 0; l < L; ++l) acc[jl][l] = __builtin_fmaf(v[jl][l], wt, acc[jl][l]);
                } else {
#pragma unroll
                    for (int jl = 0; jl < JT; ++jl)
#pragma unroll
                        for (int l = 0; l < L; ++l) acc[jl][l] += v[jl][l];
                }
            }
        }
        // blocks of SUM_BLOCK SFTs end with a stage (KS divides SUM_BLOCK)
        if (!(L > 1 && PIPE) && r.sum_mode == FT_SUM_BLOCKED && ((k0 + ks) & (SUM_BLOCK - 1)) == 0) {
#pragma unroll
            for (int j = 0; j < JT; ++j)
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    tot[j][l] += (double)acc[j][l];
                    acc[j][l] = 0.f;
                }
        }
        wait_loads();
        __syncthreads();
    }

    // --- epilogue: write the statistic (original sky order) ----------------
    const int s = tg.s_base + wave;
    if (s > tg.s_last) return;
    const int64_t s_orig = r.sky_perm ? r.sky_perm[s] : s;
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) {
        const int j = tg.j_base + jl;
        if (j > tg.j_last) continue;
        const int64_t row = (s_orig * (r.n_f1_stride ? r.n_f1_stride : r.n_f1) + j) * r.n_f0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int i = i0 + l;
            if (i <= tg.i_last) r.stats[row + i] = (float)(tot[jl][l] + (double)acc[jl][l]);
        }
    }
}

// Grid-stride over tiles.  Blocks are dispatched round-robin over the 8 XCDs
// and the grid is a multiple of 8, so block b stays on XCD b % 8; each XCD is
// given a contiguous range of tiles (f0 tile slowest, sky tile fastest) so
// the table windows it stages stay in its L2.
// OCC > 0 asks the compiler for at least OCC waves per SIMD (the second
// launch-bounds argument: a register budget of 512 / OCC VGPRs per lane; with
// four-wave workgroups that is OCC workgroups per CU); 0 leaves the
// allocation free.
template <int L, int JT, int NW, int KS, int OCC, bool PIPE, bool SKYW>
__global__ __launch_bounds__(64 * NW, OCC > 0 ? OCC : 1) void eval_grid_kernel(EvalRun r)
{
    extern __shared__ float win[];  // [2][KS][wtp]
    __shared__ Shared<L, JT, NW, KS> sh;
    const int64_t nt = (int64_t)r.tiles_f0 * r.tiles_f1 * r.tiles_sky;
    const int64_t full = nt - (nt & 7);
    for (int64_t b0 = blockIdx.x; b0 < nt; b0 += gridDim.x) {
        const int64_t b = b0 < full ? (b0 & 7) * (full >> 3) + (b0 >> 3) : b0;
        eval_tile<L, JT, NW, KS, PIPE, SKYW>(r, b, win, sh);
    }
}

// Persistent batch kernel: workgroups pull (run, tile) items from a queue
// shared by every run of a batch until it is drained; each item is one tile of
// one run's grid bank.  The queue counter is reset by the launcher's preceding
// fill kernel, so the sequence can be captured in a HIP graph.
template <int L, int JT, int NW, int KS, int OCC, bool PIPE>
__global__ __launch_bounds__(64 * NW, OCC > 0 ? OCC : 1) void eval_batch_kernel(const EvalRun *runs,
                                                                                const int2 *items, int n_items,
                                                                                unsigned *counter)
{
    extern __shared__ float win[];
    __shared__ Shared<L, JT, NW, KS> sh;
    __shared__ int item_sh;
    for (;;) {
        __syncthreads();  // every thread has read the previous item
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(item_sh);
        if (item >= n_items) break;
        const int2 it = items[item];
        const EvalRun r = runs[__builtin_amdgcn_readfirstlane(it.x)];
        eval_tile<L, JT, NW, KS, PIPE, false>(r, __builtin_amdgcn_readfirstlane(it.y), win, sh);
    }
}

template <int L, int JT, int NW, int KS, int OCC, bool PIPE>
hipError_t launch_batch_t(const EvalRun *runs, const int2 *items, int n_items, int max_wtp,
                          unsigned *counter, int grid, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    const size_t lds = (size_t)2 * KS * max_wtp * sizeof(float);
    hipLaunchKernelGGL((eval_batch_kernel<L, JT, NW, KS, OCC, PIPE>), dim3((unsigned)grid), dim3(64 * NW), lds,
                       s, runs, items, n_items, counter);
    return hipGetLastError();
}

template <int L, int JT, int NW, int KS, int OCC, bool PIPE, bool SKYW = false>
hipError_t launch_t(const EvalRun &r, hipStream_t s)
{
    const int64_t nt = (int64_t)r.tiles_f0 * r.tiles_f1 * r.tiles_sky;
    if (nt <= 0) return hipSuccess;
    const size_t lds = (size_t)2 * KS * r.wtp * sizeof(float);
    // at most 2^22 blocks (work-items stay below 2^32); a multiple of 8 keeps
    // every block's tiles on one XCD
    int64_t grid = nt < (1 << 22) ? nt : (1 << 22);
    if (grid > 8) grid &= ~(int64_t)7;
    hipLaunchKernelGGL((eval_grid_kernel<L, JT, NW, KS, OCC, PIPE, SKYW>), dim3((unsigned)grid), dim3(64 * NW),
                       lds, s, r);
    return hipGetLastError();
}

// LDS gather probe: the accumulation pattern of a tile shape -- every lane
// gathers JT runs of L consecutive window values per SFT step from a staged
// window and adds them into FP32 accumulators flushed to FP64 every SUM_BLOCK
// steps -- with the index arithmetic, the staging and the guard removed.  Its
// rate is the achievable ceiling of the grid kernel's gather-accumulate part
// at the same occupancy (same block size, LDS and register budget).
template <int L, int JT, int NW, int KS, int OCC>
__global__ __launch_bounds__(64 * NW, OCC > 0 ? OCC : 1) void lds_probe_kernel(int n_step, int wtp,
                                                                                 float *out)
{
    extern __shared__ float win[];  // [2][KS][wtp]
    const int lane = threadIdx.x & 63;
    const int n_win = 2 * KS * wtp;
    for (int i = threadIdx.x; i < n_win; i += 64 * NW) win[i] = (float)(i & 1023) * 0.25f;
    __syncthreads();
    float acc[JT][L];
    double tot[JT][L];
#pragma unroll
    for (int j = 0; j < JT; ++j)
#pragma unroll
        for (int l = 0; l < L; ++l) {
            acc[j][l] = 0.f;
            tot[j][l] = 0.0;
        }
    // lane runs as in a tile: consecutive lanes L bins apart, f1 values a few
    // bins apart, the whole pattern shifted by a few bins from step to step
    const int span = 64 * L + 3 * JT + 8;
    const int room = wtp - span > 0 ? wtp - span : 0;
    for (int k = 0; k < n_step; ++k) {
        const int kk = k % (2 * KS);
        const int shift = room > 0 ? (k * 5) % room : 0;
        const float *wk = win + kk * wtp + shift;
#pragma unroll
        for (int jl = 0; jl < JT; ++jl) {
            const float *wp = wk + lane * L + 3 * jl;
#pragma unroll
            for (int l = 0; l < L; ++l) acc[jl][l] += wp[l];
        }
        if (((k + 1) & (SUM_BLOCK - 1)) == 0) {
#pragma unroll
            for (int j = 0; j < JT; ++j)
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    tot[j][l] += (double)acc[j][l];
                    acc[j][l] = 0.f;
                }
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < JT; ++j)
#pragma unroll
        for (int l = 0; l < L; ++l) sum += tot[j][l] + (double)acc[j][l];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)sum;
}

template <int L, int JT, int NW, int KS, int OCC>
hipError_t launch_probe_t(int n_blocks, int n_step, int wtp, float *out, hipStream_t s)
{
    const size_t lds = (size_t)2 * KS * wtp * sizeof(float);
    hipLaunchKernelGGL((lds_probe_kernel<L, JT, NW, KS, OCC>), dim3((unsigned)n_blocks), dim3(64 * NW), lds, s,
                       n_step, wtp, out);
    return hipGetLastError();
}

using Launcher = hipError_t (*)(const EvalRun &, hipStream_t);
using BatchLauncher = hipError_t (*)(const EvalRun *, const int2 *, int, int, unsigned *, int,
                                     hipStream_t);

using ProbeLauncher = hipError_t (*)(int, int, int, float *, hipStream_t);

struct TileEntry {
    TileCfg cfg;
    Launcher fn;
    BatchLauncher batch_fn;
    size_t static_lds;
    ProbeLauncher probe_fn;
    Launcher sky_fn;  // sky-dependent weights, or nullptr (no such form of the tile)
};

#define FT_TILE_X(id, L, JT, NW, KS, SKY)                                                          \
    {{id, "L" #L "_J" #JT "_W" #NW "_K" #KS, L, JT, NW, KS}, &launch_t<L, JT, NW, KS, 0, false>,        \
     &launch_batch_t<L, JT, NW, KS, 0, false>, sizeof(Shared<L, JT, NW, KS>), &launch_probe_t<L, JT, NW, KS, 0>, SKY}
#define FT_TILE(id, L, JT, NW, KS) FT_TILE_X(id, L, JT, NW, KS, nullptr)
#define FT_TILE_OX(id, L, JT, NW, KS, OCC, SKY)                                                    \
    {{id, "L" #L "_J" #JT "_W" #NW "_K" #KS "_O" #OCC, L, JT, NW, KS}, &launch_t<L, JT, NW, KS, OCC, false>, \
     &launch_batch_t<L, JT, NW, KS, OCC, false>, sizeof(Shared<L, JT, NW, KS>),                     \
     &launch_probe_t<L, JT, NW, KS, OCC>, SKY}
#define FT_TILE_O(id, L, JT, NW, KS, OCC) FT_TILE_OX(id, L, JT, NW, KS, OCC, nullptr)
#define FT_TILE_PX(id, L, JT, NW, KS, OCC, SKY)                                                     \
    {{id, "L" #L "_J" #JT "_W" #NW "_K" #KS "_O" #OCC "_P", L, JT, NW, KS}, &launch_t<L, JT, NW, KS, OCC, true>, \
     &launch_batch_t<L, JT, NW, KS, OCC, true>, sizeof(Shared<L, JT, NW, KS>),                     \
     &launch_probe_t<L, JT, NW, KS, OCC>, SKY}
#define FT_TILE_P(id, L, JT, NW, KS, OCC) FT_TILE_PX(id, L, JT, NW, KS, OCC, nullptr)

const TileEntry kTiles[] = {
    FT_TILE(0, 1, 1, 4, 16),
    FT_TILE_X(1, 1, 4, 4, 16, (&launch_t<1, 4, 4, 16, 0, false, true>)),
    FT_TILE(2, 3, 4, 4, 16),
    FT_TILE(3, 5, 4, 4, 16),
    FT_TILE(4, 5, 3, 4, 16),
    FT_TILE(5, 7, 3, 4, 16),
    FT_TILE(6, 5, 6, 4, 8),
    FT_TILE(7, 3, 6, 4, 16),
    FT_TILE(8, 5, 4, 4, 8),
    FT_TILE(9, 5, 4, 8, 8),
    FT_TILE(10, 3, 4, 8, 16),
    FT_TILE(11, 7, 2, 4, 16),
    FT_TILE(12, 9, 2, 4, 16),
    FT_TILE(13, 3, 8, 4, 8),
    FT_TILE(14, 1, 3, 4, 16),
    FT_TILE(15, 3, 3, 4, 16),
    FT_TILE(16, 5, 3, 4, 8),
    FT_TILE_OX(17, 5, 4, 4, 8, 4, (&launch_t<5, 4, 4, 8, 4, false, true>)),
    FT_TILE_O(18, 5, 4, 4, 8, 5),
    FT_TILE(19, 3, 6, 4, 8),
    FT_TILE_O(20, 3, 6, 4, 8, 4),
    FT_TILE_O(21, 3, 6, 4, 8, 5),
    FT_TILE_OX(22, 5, 3, 4, 8, 4, (&launch_t<5, 3, 4, 8, 4, false, true>)),
    FT_TILE_O(23, 3, 4, 4, 8, 5),
    FT_TILE_PX(24, 5, 4, 4, 8, 4, (&launch_t<5, 4, 4, 8, 4, true, true>)),
    FT_TILE_P(25, 5, 3, 4, 8, 4),
    FT_TILE_P(26, 3, 4, 4, 8, 4),
    FT_TILE_P(27, 5, 4, 4, 8, 3),
};

}  // namespace

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }

const TileCfg &tile_cfg(int id) { return kTiles[id].cfg; }

size_t tile_static_lds(int id) { return kTiles[id].static_lds; }

bool tile_has_sky_weights(int id) { return kTiles[id].sky_fn != nullptr; }

int tile_companion(int id, int jt)
{
    const TileCfg &c = kTiles[id].cfg;
    const char *tail = strstr(c.name, "_K");  // stage length, register budget, pipelining
    for (int i = 0; i < tile_count(); ++i) {
        const TileCfg &d = kTiles[i].cfg;
        if (d.L != c.L || d.NW != c.NW || d.KS != c.KS || d.JT != jt) continue;
        const char *t2 = strstr(d.name, "_K");
        if (tail && t2 && strcmp(tail, t2) == 0) return i;
    }
    return -1;
}

hipError_t launch_eval_grid(const EvalRun &run, const TileCfg &cfg, hipStream_t s)
{
    if (run.sky_norm) return kTiles[cfg.id].sky_fn ? kTiles[cfg.id].sky_fn(run, s) : hipErrorInvalidValue;
    return kTiles[cfg.id].fn(run, s);
}

hipError_t launch_eval_batch(const EvalRun *runs, const int2 *items, int n_items, int max_wtp,
                             unsigned *counter, int grid, const TileCfg &cfg, hipStream_t s)
{
    return kTiles[cfg.id].batch_fn(runs, items, n_items, max_wtp, counter, grid, s);
}

hipError_t launch_lds_probe(const TileCfg &cfg, int n_blocks, int n_step, int wtp, float *out, hipStream_t s)
{
    return kTiles[cfg.id].probe_fn(n_blocks, n_step, wtp, out, s);
}

}  // namespace ft
