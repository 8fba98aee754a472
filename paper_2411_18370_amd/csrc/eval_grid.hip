// Grid-bank evaluation kernel: S(lambda) = sum_k w_k P[k][B_k] for every
// template of a Cartesian bank f0[n_f0] x f1[n_f1] x sky[n_sky]
// (Eq. short_coh_general; track of Eq. track with a_p = 0 plus spindown).
//
// Workgroup tile: 64*L consecutive f0 values (lane l owns the run
// [i0, i0 + L), i0 = tile_start + l*L) x JT f1 values x NW sky points (one per
// wave).  SFTs are processed in stages of KS.  Per stage the workgroup
//   A. computes the Doppler factor g[s][k] of its sky points and c[j][k] =
//      f1_j * dt_k of its f1 values (FP64, canonical order);
//   B. derives, per SFT, the exact bin range [lo, hi] of the whole tile.  The
//      FP64 bin is monotone in each of f0, c and g, and the tile is a
//      Cartesian product, so lo/hi are the bins of two actual templates: the
//      range check against the table is exact, and hi - lo bounds the window;
//   C. copies row k of the power table, columns [lo, lo + wt), into LDS
//      (coalesced), pre-multiplied by the SFT weight;
//   D. accumulates: each lane computes the canonical FP64 bin B of the first
//      template of its run and reads B, B+1, ..., B+L-1 from LDS.
//
// Run guard (exactness of B + l).  With u = (x + 1/2) - B in [0, 1) and
// e = dT*g - 1 (dT = grid spacing * T_sft), the exact position of template l
// of the run is u + l*e + err with |err| <= eta, where eta bounds the FP64
// rounding of both evaluations and the grid's deviation from uniform spacing
// (computed on the host).  If u + l*e stays inside [eta, 1 - eta) for l = 1 and
// l = L-1 (and so for all l, by linearity) then floor = B + l exactly.  When
// any lane of the wave fails the guard the wave recomputes every template of
// the run with the canonical FP64 expression.
//
// Sums: FP32 within aligned blocks of 32 SFTs, block sums accumulated in FP64.
#include "ft_internal.h"

namespace ft {

namespace {

template <int L, int JT, int NW, int KS>
struct Shared {
    double g[NW][KS];
    double ulo[NW][KS];
    double uhi[NW][KS];
    double c[JT][KS];
    int lo[KS];
    int tile_bad;
};

template <int L, int JT, int NW, int KS>
__device__ __forceinline__ void eval_tile(const EvalRun &r, int64_t b, float *win,
                                          Shared<L, JT, NW, KS> &sh)
{
    auto &g_sh = sh.g;
    auto &ulo_sh = sh.ulo;
    auto &uhi_sh = sh.uhi;
    auto &c_sh = sh.c;
    auto &lo_sh = sh.lo;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nthreads = 64 * NW;

    const int tsky = (int)(b % r.tiles_sky);
    const int64_t rest = b / r.tiles_sky;
    const int tf1 = (int)(rest % r.tiles_f1);
    const int tf0 = (int)(rest / r.tiles_f1);

    const int i_base = tf0 * 64 * L;
    const int i_last = min(i_base + 64 * L, r.n_f0) - 1;
    const int j_base = tf1 * JT;
    const int j_last = min(j_base + JT, r.n_f1) - 1;
    const int s_base = tsky * NW;
    const int s_last = min(s_base + NW, r.n_sky) - 1;

    const double T = r.t_sft;
    const double f0min = r.f0[i_base];
    const double f0max = r.f0[i_last];
    const int i0 = i_base + lane * L;
    const double f0_lane = r.f0[min(i0, i_last)];
    const int wt = r.wt;

    float acc[JT][L];
    double tot[JT][L];
#pragma unroll
    for (int j = 0; j < JT; ++j)
#pragma unroll
        for (int l = 0; l < L; ++l) {
            acc[j][l] = 0.f;
            tot[j][l] = 0.0;
        }

    __syncthreads();  // the previous tile's threads are done with the shared state
    if (threadIdx.x == 0) sh.tile_bad = 0;
    for (int k0 = 0; k0 < r.n_sft; k0 += KS) {
        const int ks = min(KS, r.n_sft - k0);
        // --- A: Doppler factors, guard bounds, spindown offsets -------------
        for (int q = threadIdx.x; q < NW * KS; q += nthreads) {
            const int sl = q / KS, kk = q % KS;
            if (kk < ks) {
                const int s = min(s_base + sl, s_last);
                const double *vk = r.v + 3 * (int64_t)(k0 + kk);
                const double *n = r.sky + 3 * (int64_t)s;
                const double g = doppler_factor(vk[0], vk[1], vk[2], n[0], n[1], n[2]);
                g_sh[sl][kk] = g;
                if (L > 1) {
                    const double e = r.dT * g - 1.0;
                    const double eL = (double)(L - 1) * e;
                    ulo_sh[sl][kk] = r.eta + fmax(-e, -eL);
                    uhi_sh[sl][kk] = (1.0 - r.eta) - fmax(e, eL);
                }
            }
        }
        for (int q = threadIdx.x; q < JT * KS; q += nthreads) {
            const int jl = q / KS, kk = q % KS;
            if (kk < ks) c_sh[jl][kk] = r.f1[min(j_base + jl, j_last)] * r.dt[k0 + kk];
        }
        __syncthreads();
        // --- B: exact bin range of the tile per SFT -------------------------
        for (int kk = threadIdx.x; kk < ks; kk += nthreads) {
            double gmin = g_sh[0][kk], gmax = gmin;
#pragma unroll
            for (int sl = 1; sl < NW; ++sl) {
                gmin = fmin(gmin, g_sh[sl][kk]);
                gmax = fmax(gmax, g_sh[sl][kk]);
            }
            double cmin = c_sh[0][kk], cmax = cmin;
#pragma unroll
            for (int jl = 1; jl < JT; ++jl) {
                cmin = fmin(cmin, c_sh[jl][kk]);
                cmax = fmax(cmax, c_sh[jl][kk]);
            }
            const int lo = bin_fp64(f0min, cmin, gmin, T);
            const int hi = bin_fp64(f0max, cmax, gmax, T);
            uint32_t bad = 0;
            if (lo < r.first_bin || hi - r.first_bin >= r.n_bins) bad |= ERR_RANGE;
            if (hi - lo + L > wt) bad |= ERR_WINDOW;
            if (bad) {
                atomicOr(r.err, bad);
                if (bad & ERR_WINDOW) sh.tile_bad = 1;
            }
            lo_sh[kk] = lo;
        }
        __syncthreads();
        // A window wider than the allocation would read outside this SFT's
        // slice: the error is flagged and the tile's result is abandoned.
        if (sh.tile_bad) return;
        // --- C: stage the windows ------------------------------------------
        for (int kk = 0; kk < ks; ++kk) {
            const int col0 = lo_sh[kk] - r.first_bin;
            const float *row = r.power + (int64_t)(k0 + kk) * r.n_bins;
            const float w = r.weight ? r.weight[k0 + kk] : 1.f;
            for (int x = threadIdx.x; x < wt; x += nthreads) {
                const int col = col0 + x;
                float val = (col >= 0 && col < r.n_bins) ? row[col] : 0.f;
                win[kk * wt + x] = val * w;
            }
        }
        __syncthreads();
        // --- D: gather and accumulate --------------------------------------
        for (int kk = 0; kk < ks; ++kk) {
            const double g = g_sh[wave][kk];
            const int base = kk * wt - lo_sh[kk];
            double ulo = 0.0, uhi = 1.0;
            if (L > 1) {
                ulo = ulo_sh[wave][kk];
                uhi = uhi_sh[wave][kk];
            }
#pragma unroll
            for (int jl = 0; jl < JT; ++jl) {
                const double c = c_sh[jl][kk];
                const double a = f0_lane + c;
                const double f = a * g;
                const double x = f * T;
                const double t = x + 0.5;
                const int B = (int)t;
                const float *wp = win + (base + B);
                if (L == 1) {
                    acc[jl][0] += wp[0];
                } else {
                    const double u = t - (double)B;
                    const bool ok = (u >= ulo) && (u < uhi);
                    if (__all(ok)) {
#pragma unroll
                        for (int l = 0; l < L; ++l) acc[jl][l] += wp[l];
                    } else {
#pragma unroll
                        for (int l = 0; l < L; ++l) {
                            const int il = min(i0 + l, i_last);
                            const int Bl = bin_fp64(r.f0[il], c, g, T);
                            acc[jl][l] += win[base + Bl];
                        }
                    }
                }
            }
            if (r.sum_mode == FT_SUM_BLOCKED && ((k0 + kk + 1) & (SUM_BLOCK - 1)) == 0) {
#pragma unroll
                for (int j = 0; j < JT; ++j)
#pragma unroll
                    for (int l = 0; l < L; ++l) {
                        tot[j][l] += (double)acc[j][l];
                        acc[j][l] = 0.f;
                    }
            }
        }
        __syncthreads();
    }

    // --- epilogue: write the statistic -------------------------------------
    const int s = s_base + wave;
    if (s > s_last) return;
#pragma unroll
    for (int jl = 0; jl < JT; ++jl) {
        const int j = j_base + jl;
        if (j > j_last) continue;
        const int64_t row = ((int64_t)s * r.n_f1 + j) * r.n_f0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int i = i0 + l;
            if (i <= i_last) r.stats[row + i] = (float)(tot[jl][l] + (double)acc[jl][l]);
        }
    }
}

// Grid-stride over tiles.  Blocks are dispatched round-robin over the 8 XCDs
// and the grid is a multiple of 8, so block b stays on XCD b % 8; each XCD is
// given a contiguous range of tiles (f0 tile slowest, sky tile fastest) so
// the table windows it stages stay in its L2.
template <int L, int JT, int NW, int KS>
__global__ __launch_bounds__(64 * NW) void eval_grid_kernel(EvalRun r)
{
    extern __shared__ float win[];  // [KS][wt]
    __shared__ Shared<L, JT, NW, KS> sh;
    const int64_t nt = (int64_t)r.tiles_f0 * r.tiles_f1 * r.tiles_sky;
    const int64_t full = nt - (nt & 7);
    for (int64_t b0 = blockIdx.x; b0 < nt; b0 += gridDim.x) {
        const int64_t b = b0 < full ? (b0 & 7) * (full >> 3) + (b0 >> 3) : b0;
        eval_tile<L, JT, NW, KS>(r, b, win, sh);
    }
}

template <int L, int JT, int NW, int KS>
hipError_t launch_t(const EvalRun &r, hipStream_t s)
{
    const int64_t nt = (int64_t)r.tiles_f0 * r.tiles_f1 * r.tiles_sky;
    if (nt <= 0) return hipSuccess;
    const size_t lds = (size_t)KS * r.wt * sizeof(float);
    // at most 2^22 blocks (work-items stay below 2^32); a multiple of 8 keeps
    // every block's tiles on one XCD
    int64_t grid = nt < (1 << 22) ? nt : (1 << 22);
    if (grid > 8) grid &= ~(int64_t)7;
    hipLaunchKernelGGL((eval_grid_kernel<L, JT, NW, KS>), dim3((unsigned)grid), dim3(64 * NW),
                       lds, s, r);
    return hipGetLastError();
}

using Launcher = hipError_t (*)(const EvalRun &, hipStream_t);

struct TileEntry {
    TileCfg cfg;
    Launcher fn;
};

#define FT_TILE(id, L, JT, NW, KS) \
    {{id, "L" #L "_J" #JT "_W" #NW "_K" #KS, L, JT, NW, KS}, &launch_t<L, JT, NW, KS>}

const TileEntry kTiles[] = {
    FT_TILE(0, 1, 1, 4, 32),
    FT_TILE(1, 1, 4, 4, 32),
    FT_TILE(2, 3, 4, 4, 32),
    FT_TILE(3, 5, 4, 4, 32),
    FT_TILE(4, 5, 3, 4, 32),
    FT_TILE(5, 7, 3, 4, 32),
    FT_TILE(6, 5, 6, 4, 32),
    FT_TILE(7, 3, 6, 4, 32),
    FT_TILE(8, 5, 4, 4, 16),
    FT_TILE(9, 3, 4, 4, 16),
};

}  // namespace

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }

const TileCfg &tile_cfg(int id) { return kTiles[id].cfg; }

hipError_t launch_eval_grid(const EvalRun &run, const TileCfg &cfg, hipStream_t s)
{
    return kTiles[cfg.id].fn(run, s);
}

}  // namespace ft
