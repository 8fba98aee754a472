// Exact per-sub-band toplists (the list of loudest candidates per region of
// Secs. IV.B and VI) from the FP32 statistic.
//
// 1. Radix select (4 passes of 8-bit digits over the IEEE bits of S32, which
//    order like the values since S32 >= 0) finds K32, the exact K-th largest
//    FP32 statistic of each sub-band.
// 2. Every template with S32 >= K32 (1 - 2e)/(1 + 2e) is a candidate, where e
//    bounds |S32 - S64| / S relative to the sum: if K templates have
//    S32 >= K32 then the K-th largest S64 is >= K32/(1 + e), so every member of
//    the FP64 top-K has S32 >= K32 (1 - e)/(1 + e).  Candidates are compacted
//    per sub-band.
// 3. Each candidate is re-summed in FP64 in SFT order with canonical bins
//    (one wavefront per candidate: the 64 lanes form the weighted terms of
//    256 consecutive SFTs at a time, 4 per lane, and store them to LDS; lane 0
//    then adds them to the running sum one by one in SFT order, so the sum is
//    the plain sequential FP64 sum).
// 4. Candidates are ranked within their sub-band by (S64 desc, index asc);
//    ranks < K are the toplist, identical to sorting all FP64 statistics.
#include "ft_internal.h"

#include <algorithm>

namespace ft {

namespace {

constexpr uint32_t NAN_KEY = 0x7f800000u;  // keys above this are NaN
constexpr int ST = 8;                      // state words per segment
enum { S_PREFIX = 0, S_MASK = 1, S_KREM = 2, S_DONE = 3, S_THR = 4 };

__global__ void subband_map_kernel(const double *f0, int64_t n, const double *edges, int n_sub,
                                   int32_t *seg)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double f = f0[q];
        int lo = 0, hi = n_sub;  // find the last edge <= f
        if (!(edges[0] <= f) || !(f < edges[n_sub])) {
            seg[q] = -1;
            continue;
        }
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (edges[mid] <= f) lo = mid;
            else hi = mid;
        }
        seg[q] = lo;
    }
}

// Iterate the templates of a bank as rows: GRID rows are (s, j) pairs of
// n_f0 templates whose sub-band depends on i only; LIST rows are chunks.
struct Rows {
    int64_t n_rows, row_len, n_total;
    bool grid;
};

__device__ __forceinline__ int seg_at(const int32_t *seg_of, const Rows &rw, int64_t c,
                                      int64_t t)
{
    return rw.grid ? seg_of[c] : seg_of[t];
}

template <bool LDS>
__global__ __launch_bounds__(256) void hist_kernel(const float *stats, const int32_t *seg_of,
                                                   Rows rw, const uint32_t *state,
                                                   uint32_t *hist, int n_seg, int shift)
{
    extern __shared__ uint32_t hsh[];
    if (LDS) {
        for (int q = threadIdx.x; q < n_seg * 256; q += blockDim.x) hsh[q] = 0;
        __syncthreads();
    }
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        for (int64_t c = threadIdx.x; c < rw.row_len; c += blockDim.x) {
            const int64_t t = row * rw.row_len + c;
            if (t >= rw.n_total) break;
            const int sg = seg_at(seg_of, rw, c, t);
            if (sg < 0) continue;
            const uint32_t *st = state + (int64_t)sg * ST;
            if (st[S_DONE]) continue;
            const uint32_t key = __float_as_uint(stats[t]);
            if (key > NAN_KEY || (key & st[S_MASK]) != st[S_PREFIX]) continue;
            const uint32_t digit = (key >> shift) & 255u;
            if (LDS) atomicAdd(&hsh[sg * 256 + digit], 1u);
            else atomicAdd(&hist[(int64_t)sg * 256 + digit], 1u);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < n_seg * 256; q += blockDim.x)
            if (hsh[q]) atomicAdd(&hist[q], hsh[q]);
    }
}

// Grid banks: a row is one (sky, f1) pair of n_f0 templates and the sub-band
// depends on the f0 column only, so each thread owns the columns
// threadIdx.x + 256 i (i < COLS) of every row it visits and keeps their
// sub-band and selection state in registers; the rows stream through.
template <int COLS>
struct GridCols {
    int32_t sg[COLS];
    bool on[COLS];
};

template <int COLS>
__device__ __forceinline__ GridCols<COLS> grid_cols(const int32_t *seg_of, const Rows &rw)
{
    GridCols<COLS> g;
#pragma unroll
    for (int i = 0; i < COLS; ++i) {
        const int64_t c = threadIdx.x + 256 * i;
        g.sg[i] = c < rw.row_len ? seg_of[c] : -1;
        g.on[i] = g.sg[i] >= 0;
    }
    return g;
}

// Histogram pass over grid rows.  When every lane of the wave with a key for
// this column hits the same (sub-band, digit) -- the common case in the first
// passes, where a row's statistics share their leading bits -- one lane adds
// the wave's count.
template <int COLS>
__global__ __launch_bounds__(256) void hist_grid_kernel(const float *stats, const int32_t *seg_of, Rows rw,
                                                        const uint32_t *state, uint32_t *hist, int n_seg, int shift)
{
    extern __shared__ uint32_t hsh[];
    for (int q = threadIdx.x; q < n_seg * 256; q += blockDim.x) hsh[q] = 0;
    GridCols<COLS> g = grid_cols<COLS>(seg_of, rw);
    uint32_t mask[COLS], prefix[COLS];
#pragma unroll
    for (int i = 0; i < COLS; ++i) {
        const uint32_t *st = state + (int64_t)max(g.sg[i], 0) * ST;
        g.on[i] = g.on[i] && !st[S_DONE];
        mask[i] = st[S_MASK];
        prefix[i] = st[S_PREFIX];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        const float *rp = stats + row * rw.row_len;
#pragma unroll
        for (int i = 0; i < COLS; ++i) {
            int idx = -1;
            if (g.on[i]) {
                const uint32_t key = __float_as_uint(rp[threadIdx.x + 256 * i]);
                if (key <= NAN_KEY && (key & mask[i]) == prefix[i]) idx = g.sg[i] * 256 + (int)((key >> shift) & 255u);
            }
            const uint64_t valid = __builtin_amdgcn_ballot_w64(idx >= 0);
            if (valid == 0) continue;
            const int first = __builtin_ctzll(valid);
            const int lead = __builtin_amdgcn_readlane(idx, first);
            const uint64_t same = __builtin_amdgcn_ballot_w64(idx == lead);
            if (same == valid) {
                if (lane == first) atomicAdd(&hsh[lead], (uint32_t)__builtin_popcountll(valid));
            } else if (idx >= 0) {
                atomicAdd(&hsh[idx], 1u);
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_seg * 256; q += blockDim.x)
        if (hsh[q]) atomicAdd(&hist[q], hsh[q]);
}

// Candidates per sub-band over grid rows: counts kept per column in
// registers, added once per thread.
template <int COLS>
__global__ __launch_bounds__(256) void count_grid_kernel(const float *stats, const int32_t *seg_of, Rows rw,
                                                         const uint32_t *state, uint32_t *cnt, int n_seg)
{
    extern __shared__ uint32_t csh[];
    for (int q = threadIdx.x; q < n_seg; q += blockDim.x) csh[q] = 0;
    GridCols<COLS> g = grid_cols<COLS>(seg_of, rw);
    uint32_t thr[COLS], n[COLS];
#pragma unroll
    for (int i = 0; i < COLS; ++i) {
        thr[i] = state[(int64_t)max(g.sg[i], 0) * ST + S_THR];
        n[i] = 0;
    }
    __syncthreads();
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        const float *rp = stats + row * rw.row_len;
#pragma unroll
        for (int i = 0; i < COLS; ++i)
            if (g.on[i]) {
                const uint32_t key = __float_as_uint(rp[threadIdx.x + 256 * i]);
                n[i] += (key <= NAN_KEY && key >= thr[i]) ? 1u : 0u;
            }
    }
#pragma unroll
    for (int i = 0; i < COLS; ++i)
        if (g.on[i] && n[i]) atomicAdd(&csh[g.sg[i]], n[i]);
    __syncthreads();
    for (int q = threadIdx.x; q < n_seg; q += blockDim.x)
        if (csh[q]) atomicAdd(&cnt[q], csh[q]);
}

// Compaction of the candidates over grid rows.
template <int COLS>
__global__ __launch_bounds__(256) void scatter_grid_kernel(const float *stats, const int32_t *seg_of, Rows rw,
                                                           const uint32_t *state, const uint32_t *off,
                                                           uint32_t *fill, int64_t *cand, int64_t cap)
{
    GridCols<COLS> g = grid_cols<COLS>(seg_of, rw);
    uint32_t thr[COLS];
#pragma unroll
    for (int i = 0; i < COLS; ++i) thr[i] = state[(int64_t)max(g.sg[i], 0) * ST + S_THR];
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        const float *rp = stats + row * rw.row_len;
#pragma unroll
        for (int i = 0; i < COLS; ++i)
            if (g.on[i]) {
                const int64_t c = threadIdx.x + 256 * i;
                const uint32_t key = __float_as_uint(rp[c]);
                if (key <= NAN_KEY && key >= thr[i]) {
                    const int64_t pos = (int64_t)off[g.sg[i]] + atomicAdd(&fill[g.sg[i]], 1u);
                    if (pos < cap) cand[pos] = row * rw.row_len + c;
                }
            }
    }
}

// One thread per segment: choose the digit holding the k_rem-th largest key.
__global__ void scan_kernel(uint32_t *state, const uint32_t *hist, int n_seg, int shift,
                            double two_e)
{
    const int sg = blockIdx.x * blockDim.x + threadIdx.x;
    if (sg >= n_seg) return;
    uint32_t *st = state + (int64_t)sg * ST;
    if (st[S_DONE]) return;
    const uint32_t *h = hist + (int64_t)sg * 256;
    uint32_t k_rem = st[S_KREM], cum = 0;
    int found = -1;
    for (int d = 255; d >= 0; --d) {
        if (cum + h[d] >= k_rem) {
            found = d;
            break;
        }
        cum += h[d];
    }
    if (found < 0) {  // fewer than K members: all of them are candidates
        st[S_DONE] = 1;
        st[S_THR] = 0;
        return;
    }
    st[S_PREFIX] |= (uint32_t)found << shift;
    st[S_MASK] |= 255u << shift;
    st[S_KREM] = k_rem - cum;
    if (shift == 0) {
        const double kth = (double)__uint_as_float(st[S_PREFIX]);
        const double thr = kth * (1.0 - two_e) / (1.0 + two_e);
        float tf = (float)thr;
        if ((double)tf > thr) tf = nextafterf(tf, 0.f);
        if (!(tf > 0.f)) tf = 0.f;
        st[S_THR] = __float_as_uint(tf);
        st[S_DONE] = 1;
    }
}

template <bool LDS>
__global__ __launch_bounds__(256) void count_kernel(const float *stats, const int32_t *seg_of,
                                                    Rows rw, const uint32_t *state,
                                                    uint32_t *cnt, int n_seg)
{
    extern __shared__ uint32_t csh[];
    if (LDS) {
        for (int q = threadIdx.x; q < n_seg; q += blockDim.x) csh[q] = 0;
        __syncthreads();
    }
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        for (int64_t c = threadIdx.x; c < rw.row_len; c += blockDim.x) {
            const int64_t t = row * rw.row_len + c;
            if (t >= rw.n_total) break;
            const int sg = seg_at(seg_of, rw, c, t);
            if (sg < 0) continue;
            const uint32_t key = __float_as_uint(stats[t]);
            if (key > NAN_KEY || key < state[(int64_t)sg * ST + S_THR]) continue;
            if (LDS) atomicAdd(&csh[sg], 1u);
            else atomicAdd(&cnt[sg], 1u);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < n_seg; q += blockDim.x)
            if (csh[q]) atomicAdd(&cnt[q], csh[q]);
    }
}

__global__ void offsets_kernel(const uint32_t *cnt, uint32_t *off, int n_seg, int64_t cap,
                               uint32_t *err)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint64_t acc = 0;
    off[0] = 0;
    for (int s = 0; s < n_seg; ++s) {
        acc += cnt[s];
        off[s + 1] = (uint32_t)(acc < 0xffffffffull ? acc : 0xffffffffull);
    }
    if (acc > (uint64_t)cap) atomicOr(err, ERR_CAND_OVERFLOW);
}

__global__ __launch_bounds__(256) void scatter_kernel(const float *stats, const int32_t *seg_of,
                                                      Rows rw, const uint32_t *state,
                                                      const uint32_t *off, uint32_t *fill,
                                                      int64_t *cand, int64_t cap)
{
    for (int64_t row = blockIdx.x; row < rw.n_rows; row += gridDim.x) {
        for (int64_t c = threadIdx.x; c < rw.row_len; c += blockDim.x) {
            const int64_t t = row * rw.row_len + c;
            if (t >= rw.n_total) break;
            const int sg = seg_at(seg_of, rw, c, t);
            if (sg < 0) continue;
            const uint32_t key = __float_as_uint(stats[t]);
            if (key > NAN_KEY || key < state[(int64_t)sg * ST + S_THR]) continue;
            const int64_t pos = (int64_t)off[sg] + atomicAdd(&fill[sg], 1u);
            if (pos < cap) cand[pos] = t;
        }
    }
}

struct TemplateParams {
    double f0, f1, nx, ny, nz;
    double aw, omega, phib;  // binary-system list banks (aw = a_p Omega), else 0
};

__device__ __forceinline__ TemplateParams params_of(const EvalRun &r, bool grid, int64_t t)
{
    TemplateParams p;
    int64_t s;
    if (grid) {
        const int64_t i = t % r.n_f0;
        const int64_t rest = t / r.n_f0;
        const int64_t j = rest % r.n_f1;
        s = rest / r.n_f1;
        p.f0 = r.f0[i];
        p.f1 = r.f1[j];
    } else {
        s = t;
        p.f0 = r.f0[t];
        p.f1 = r.ap ? 0.0 : r.f1[t];
    }
    p.aw = p.omega = p.phib = 0.0;
    if (!grid && r.ap) {
        p.omega = r.omega[t];
        p.phib = r.phib[t];
        p.aw = r.ap[t] * p.omega;
    }
    p.nx = r.sky[3 * s];
    p.ny = r.sky[3 * s + 1];
    p.nz = r.sky[3 * s + 2];
    return p;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// FP64 re-summation of template t in SFT order by one wavefront: lanes form
// the terms of 64 RS_UNROLL SFTs at a time and publish them to the wave's LDS
// slice buf [2][64 RS_UNROLL], then lane 0 adds them one after another in SFT
// order (the result is lane 0's).  The weight is u_k, times ab_k(n) / sum_k'
// u_k' ab_k'(n) with sky-dependent weights.  With MOM the weight sums W1 =
// sum w and W2 = sum w^2 come out as well.  The terms of the next chunk are
// formed (their gathers issued) before the current chunk is added, so the
// gathers' latency overlaps the additions.
constexpr int RS_UNROLL = 4;
constexpr int RS_BUF = 2 * 64 * RS_UNROLL;  // doubles of LDS per wave


template <bool MOM>
__device__ __forceinline__ double rescore_one(const EvalRun &r, bool grid, int64_t t, int lane, uint32_t &bad,
                                              double *buf, double *w1 = nullptr, double *w2 = nullptr)
{
    const TemplateParams tp = params_of(r, grid, t);
    // sky-dependent weights: 1 / sum_k u_k ab_k(n) of the template's sky point
    // (grid: per sky point, precomputed; binary banks: per template, here)
    const bool bsky = !grid && r.arms;
    double inv = grid && r.sky_norm ? r.sky_norm[t / ((int64_t)r.n_f0 * r.n_f1)] : 0.0;
    if (bsky) inv = 1.0 / sky_norm_sum(r.arms, r.weight, r.n_sft, tp.nx, tp.ny, tp.nz, buf, lane);
    // terms of SFTs k0 + 64 j + lane, j < RS_UNROLL (0 past the last SFT)
    auto terms = [&](int k0, double (&val)[RS_UNROLL], double (&wk)[RS_UNROLL]) {
#pragma unroll
        for (int j = 0; j < RS_UNROLL; ++j) {
            const int k = k0 + 64 * j + lane;
            val[j] = 0.0;
            wk[j] = 0.0;
            if (k < r.n_sft) {
                const double *vk = r.v + 3 * (int64_t)k;
                const double g = doppler_factor(vk[0], vk[1], vk[2], tp.nx, tp.ny, tp.nz);
                int b = (r.ap ? bin_binary(tp.f0, g, tp.aw, tp.omega, tp.phib, r.dt[k], r.t_sft)
                              : bin_fp64(tp.f0, tp.f1 * r.dt[k], g, r.t_sft)) -
                        r.first_bin;
                if (b < 0 || b >= r.n_bins) {
                    bad = ERR_RANGE;
                    b = b < 0 ? 0 : r.n_bins - 1;
                }
                double w = r.weight ? (double)r.weight[k] : 1.0;
                if ((grid && r.sky_norm) || bsky) w = w * (sky_ab(r.arms + 6 * (int64_t)k, tp.nx, tp.ny, tp.nz) * inv);
                val[j] = w * (double)r.power[(int64_t)k * r.n_bins + b];
                wk[j] = w;
            }
        }
    };
    double acc = 0.0, sw = 0.0, sw2 = 0.0;
    double val[RS_UNROLL], wk[RS_UNROLL];
    terms(0, val, wk);
    for (int k0 = 0; k0 < r.n_sft; k0 += 64 * RS_UNROLL) {
        double nval[RS_UNROLL], nwk[RS_UNROLL];
        const bool more = k0 + 64 * RS_UNROLL < r.n_sft;
        if (more) terms(k0 + 64 * RS_UNROLL, nval, nwk);
#pragma unroll
        for (int j = 0; j < RS_UNROLL; ++j) {
            buf[64 * j + lane] = val[j];
            if (MOM) buf[64 * RS_UNROLL + 64 * j + lane] = wk[j];
        }
        wave_lds_sync();
        if (lane == 0) {
            const int m_all = min(64 * RS_UNROLL, r.n_sft - k0);
            int q = 0;
            for (; q + 8 <= m_all; q += 8) {
                double x[8], y[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    x[i] = buf[q + i];
                    if (MOM) y[i] = buf[64 * RS_UNROLL + q + i];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    acc = acc + x[i];
                    if (MOM) {
                        sw = sw + y[i];
                        sw2 = sw2 + y[i] * y[i];
                    }
                }
            }
            for (; q < m_all; ++q) {
                acc = acc + buf[q];
                if (MOM) {
                    const double y = buf[64 * RS_UNROLL + q];
                    sw = sw + y;
                    sw2 = sw2 + y * y;
                }
            }
        }
        wave_lds_sync();
        if (more) {
#pragma unroll
            for (int j = 0; j < RS_UNROLL; ++j) {
                val[j] = nval[j];
                wk[j] = nwk[j];
            }
        }
    }
    if (MOM) {
        *w1 = sw;
        *w2 = sw2;
    }
    return acc;
}

// FP64 re-summation of the candidates, one wavefront per candidate; with
// mom, also each candidate's sums of weights and squared weights.
__global__ __launch_bounds__(256) void rescore_kernel(EvalRun r, bool grid, const int64_t *cand,
                                                      const uint32_t *off, int n_seg,
                                                      int64_t cap, double *s64, double *mom)
{
    __shared__ double rs_buf[4 * RS_BUF];
    double *buf = rs_buf + (threadIdx.x >> 6) * RS_BUF;
    const int lane = threadIdx.x & 63;
    const int64_t total = min((int64_t)off[n_seg], cap);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    uint32_t bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < total;
         p += n_waves) {
        if (mom) {
            double w1, w2;
            const double acc = rescore_one<true>(r, grid, cand[p], lane, bad, buf, &w1, &w2);
            if (lane == 0) {
                s64[p] = acc;
                mom[2 * p] = w1;
                mom[2 * p + 1] = w2;
            }
        } else {
            const double acc = rescore_one<false>(r, grid, cand[p], lane, bad, buf);
            if (lane == 0) s64[p] = acc;
        }
    }
    if (bad) atomicOr(r.err, bad);
}

// FP64 re-summation of the templates of toplist entries top[0 .. n_out[0]):
// out[3p .. 3p+2] = (sum, W1, W2).
__global__ __launch_bounds__(256) void rescore_entries_kernel(EvalRun r, bool grid, const ft_candidate *top,
                                                              const int32_t *n_out, double *out)
{
    __shared__ double rs_buf[4 * RS_BUF];
    double *buf = rs_buf + (threadIdx.x >> 6) * RS_BUF;
    const int lane = threadIdx.x & 63;
    const int64_t total = n_out[0];
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    uint32_t bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < total; p += n_waves) {
        double w1, w2;
        const double acc = rescore_one<true>(r, grid, top[p].index, lane, bad, buf, &w1, &w2);
        if (lane == 0) {
            out[3 * p] = acc;
            out[3 * p + 1] = w1;
            out[3 * p + 2] = w2;
        }
    }
    if (bad) atomicOr(r.err, bad);
}

// Rank of each candidate within its sub-band under (S64 desc, index asc).
__global__ __launch_bounds__(256) void rank_kernel(EvalRun r, bool grid, const int64_t *cand,
                                                   const double *s64, const uint32_t *off,
                                                   int n_seg, int64_t cap, int k,
                                                   const double *mu_sigma, const double *mom,
                                                   ft_candidate *out)
{
    const int64_t total = min((int64_t)off[n_seg], cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_seg;  // segment: off[sg] <= p < off[sg+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if ((int64_t)off[mid] <= p) lo = mid;
            else hi = mid;
        }
        const int sg = lo;
        const int64_t q0 = off[sg];
        const int64_t q1 = min((int64_t)off[sg + 1], cap);
        const double sp = s64[p];
        const int64_t tp = cand[p];
        int64_t rank = 0;
        for (int64_t q = q0; q < q1 && rank < k; ++q) {
            const double sq = s64[q];
            rank += (sq > sp) || (sq == sp && cand[q] < tp);
        }
        if (rank < k) {
            const TemplateParams par = params_of(r, grid, tp);
            ft_candidate c;
            c.index = tp;
            c.sub = sg;
            c.s32 = r.stats[tp];
            c.f0 = par.f0;
            c.f1 = par.f1;
            c.n[0] = par.nx;
            c.n[1] = par.ny;
            c.n[2] = par.nz;
            c.s64 = sp;
            // sky-dependent weights: the moments of the template's sky point
            // (grid) or of the template's own weights (binary banks)
            double own[2];
            const double *ms = mu_sigma;
            if (grid && r.sky_ms) {
                ms = r.sky_ms + 2 * (tp / ((int64_t)r.n_f0 * r.n_f1));
            } else if (mom) {
                stat_moments(r.stat, mom[2 * p], mom[2 * p + 1], own);
                ms = own;
            }
            c.z = (sp - ms[0]) / ms[1];
            out[(int64_t)sg * k + rank] = c;
        }
    }
}

__global__ void n_out_kernel(const uint32_t *cnt, int n_seg, int k, int32_t *n_out)
{
    const int sg = blockIdx.x * blockDim.x + threadIdx.x;
    if (sg < n_seg) n_out[sg] = (int32_t)min(cnt[sg], (uint32_t)k);
}

__global__ void init_state_kernel(uint32_t *state, uint32_t *cnt, uint32_t *fill, int n_seg,
                                  int k)
{
    const int sg = blockIdx.x * blockDim.x + threadIdx.x;
    if (sg >= n_seg) return;
    uint32_t *st = state + (int64_t)sg * ST;
    st[S_PREFIX] = 0;
    st[S_MASK] = 0;
    st[S_KREM] = (uint32_t)k;
    st[S_DONE] = 0;
    st[S_THR] = 0;
    cnt[sg] = 0;
    fill[sg] = 0;
}

// ---------------------------------------------------------------------------
// Batches: one workgroup per run does the whole exact selection of that run
// (runs hold at most a few 1e5 templates): radix select in LDS, candidate
// compaction, FP64 re-summation (one wavefront per candidate) and ranking.
// SB_THREADS threads: the 16 wavefronts re-sum up to 16 candidates at once.
// ---------------------------------------------------------------------------
constexpr int SB_THREADS = 1024;

__global__ __launch_bounds__(SB_THREADS) void select_batch_kernel(const EvalRun *runs, int k, int cap,
                                                           int64_t *cand_all, double *s64_all,
                                                           ft_candidate *out, int32_t *n_out,
                                                           double *max_z, uint32_t *err)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t st_prefix, st_mask, st_krem, st_thr, st_done, n_cand;
    const int r = blockIdx.x;
    const EvalRun R = runs[r];
    const int64_t n_t = (int64_t)R.n_f0 * R.n_f1 * R.n_sky;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double N = (double)R.n_sft;
    const double two_e = 2.0 * (40.0 * 0x1p-24 + 4.0 * N * 0x1p-53);
    int64_t *cand = cand_all + (int64_t)r * cap;
    double *s64 = s64_all + (int64_t)r * cap;
    if (tid == 0) {
        st_prefix = 0;
        st_mask = 0;
        st_krem = (uint32_t)k;
        st_done = 0;
        st_thr = 0;
        n_cand = 0;
    }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        if (!st_done) {
            const uint32_t mask = st_mask, prefix = st_prefix;
            for (int64_t t = tid; t < n_t; t += SB_THREADS) {
                const uint32_t key = __float_as_uint(R.stats[t]);
                if (key > NAN_KEY || (key & mask) != prefix) continue;
                atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        if (tid == 0 && !st_done) {
            uint32_t cum = 0;
            int found = -1;
            for (int d = 255; d >= 0; --d) {
                if (cum + hist[d] >= st_krem) {
                    found = d;
                    break;
                }
                cum += hist[d];
            }
            if (found < 0) {
                st_done = 1;
                st_thr = 0;
            } else {
                st_prefix |= (uint32_t)found << shift;
                st_mask |= 255u << shift;
                st_krem -= cum;
                if (shift == 0) {
                    const double kth = (double)__uint_as_float(st_prefix);
                    const double thr = kth * (1.0 - two_e) / (1.0 + two_e);
                    float tf = (float)thr;
                    if ((double)tf > thr) tf = nextafterf(tf, 0.f);
                    if (!(tf > 0.f)) tf = 0.f;
                    st_thr = __float_as_uint(tf);
                    st_done = 1;
                }
            }
        }
        __syncthreads();
    }
    const uint32_t thr = st_thr;
    for (int64_t t = tid; t < n_t; t += SB_THREADS) {
        const uint32_t key = __float_as_uint(R.stats[t]);
        if (key > NAN_KEY || key < thr) continue;
        const uint32_t pos = atomicAdd(&n_cand, 1u);
        if (pos < (uint32_t)cap) cand[pos] = t;
    }
    __syncthreads();
    int nc = (int)n_cand;
    if (nc > cap) {
        if (tid == 0) atomicOr(err, ERR_CAND_OVERFLOW);
        nc = cap;
    }
    // FP64 re-summation in SFT order with canonical bins; the terms of the
    // next 64 SFTs are formed (their loads issued) before the current 64 are
    // added in order
    uint32_t bad = 0;
    for (int p = wave; p < nc; p += SB_THREADS / 64) {
        const TemplateParams tp = params_of(R, true, cand[p]);
        auto term = [&](int kq) {
            if (kq >= R.n_sft) return 0.0;
            const double *vk = R.v + 3 * (int64_t)kq;
            const double g = doppler_factor(vk[0], vk[1], vk[2], tp.nx, tp.ny, tp.nz);
            int b = bin_fp64(tp.f0, tp.f1 * R.dt[kq], g, R.t_sft) - R.first_bin;
            if (b < 0 || b >= R.n_bins) {
                bad = ERR_RANGE;
                b = b < 0 ? 0 : R.n_bins - 1;
            }
            const double w = R.weight ? (double)R.weight[kq] : 1.0;
            return w * (double)R.power[(int64_t)kq * R.n_bins + b];
        };
        double acc = 0.0;
        double val = term(lane);
        for (int k0 = 0; k0 < R.n_sft; k0 += 64) {
            const double nxt = term(k0 + 64 + lane);
            const int m = min(64, R.n_sft - k0);
            for (int l = 0; l < m; ++l) acc = acc + readlane_f64(val, l);
            val = nxt;
        }
        if (lane == 0) s64[p] = acc;
    }
    if (bad) atomicOr(err, bad);
    __syncthreads();
    const double mu = 2.0 * N, sigma = 2.0 * sqrt(N);
    for (int p = tid; p < nc; p += SB_THREADS) {
        const double sp = s64[p];
        const int64_t tp = cand[p];
        int rank = 0;
        for (int q = 0; q < nc && rank < k; ++q) {
            const double sq = s64[q];
            rank += (sq > sp) || (sq == sp && cand[q] < tp);
        }
        if (rank < k) {
            const TemplateParams par = params_of(R, true, tp);
            ft_candidate c;
            c.index = tp;
            c.sub = 0;
            c.s32 = R.stats[tp];
            c.f0 = par.f0;
            c.f1 = par.f1;
            c.n[0] = par.nx;
            c.n[1] = par.ny;
            c.n[2] = par.nz;
            c.s64 = sp;
            c.z = (sp - mu) / sigma;
            out[(int64_t)r * k + rank] = c;
            if (rank == 0) max_z[r] = c.z;
        }
    }
    if (tid == 0) n_out[r] = min(nc, k);
}

__global__ void labels_kernel(const double *max_z, int n_runs, double tau, uint8_t *labels)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_runs) labels[r] = max_z[r] > tau ? 1 : 0;
}

Rows rows_of(const EvalRun &r, bool grid)
{
    Rows rw;
    rw.grid = grid;
    if (grid) {
        rw.row_len = r.n_f0;
        rw.n_rows = (int64_t)r.n_sky * r.n_f1;
        rw.n_total = rw.n_rows * rw.row_len;
    } else {
        rw.row_len = 4096;
        rw.n_total = r.n_list;
        rw.n_rows = (r.n_list + rw.row_len - 1) / rw.row_len;
    }
    return rw;
}

unsigned blocks_for(int64_t n_rows) { return (unsigned)std::min<int64_t>(std::max<int64_t>(n_rows, 1), 8192); }

}  // namespace

hipError_t launch_select_batch(const EvalRun *runs, int n_runs, int k, int cap_per_run,
                               int64_t *cand, double *cand_s64, ft_candidate *out,
                               int32_t *n_out, double *max_z, uint32_t *err, hipStream_t s)
{
    if (n_runs <= 0) return hipSuccess;
    hipLaunchKernelGGL(select_batch_kernel, dim3((unsigned)n_runs), dim3(SB_THREADS), 0, s, runs, k,
                       cap_per_run, cand, cand_s64, out, n_out, max_z, err);
    return hipGetLastError();
}

hipError_t launch_labels(const double *max_z, int n_runs, double tau, uint8_t *labels,
                         hipStream_t s)
{
    if (n_runs <= 0) return hipSuccess;
    hipLaunchKernelGGL(labels_kernel, dim3((unsigned)((n_runs + 255) / 256)), dim3(256), 0, s,
                       max_z, n_runs, tau, labels);
    return hipGetLastError();
}

hipError_t launch_subband_map(const double *f0, int64_t n, const double *edges, int n_sub,
                              int32_t *seg, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(subband_map_kernel, dim3(g), dim3(256), 0, s, f0, n, edges, n_sub, seg);
    return hipGetLastError();
}

hipError_t launch_select(const EvalRun &r, bool grid, int n_seg, int k, double rel_err,
                         const SelectBufs &b, hipStream_t s)
{
    const Rows rw = rows_of(r, grid);
    const unsigned sg_blocks = (unsigned)((n_seg + 255) / 256);
    hipLaunchKernelGGL(init_state_kernel, dim3(sg_blocks), dim3(256), 0, s, b.state, b.cnt,
                       b.fill, n_seg, k);
    const bool lds_hist = n_seg * 256 <= 8192;
    const unsigned nb = blocks_for(rw.n_rows);
    // grid rows of at most 2048 templates: column-owning kernels
    const int cols = !grid || !lds_hist ? 0 : rw.row_len <= 1024 ? 4 : rw.row_len <= 2048 ? 8 : 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        hipError_t e = launch_fill_u32(b.hist, 0u, (int64_t)n_seg * 256, s);
        if (e != hipSuccess) return e;
        const size_t hl = (size_t)n_seg * 256 * sizeof(uint32_t);
        if (cols == 4)
            hipLaunchKernelGGL(hist_grid_kernel<4>, dim3(nb), dim3(256), hl, s, r.stats, b.seg_of_f0, rw, b.state,
                               b.hist, n_seg, shift);
        else if (cols == 8)
            hipLaunchKernelGGL(hist_grid_kernel<8>, dim3(nb), dim3(256), hl, s, r.stats, b.seg_of_f0, rw, b.state,
                               b.hist, n_seg, shift);
        else if (lds_hist)
            hipLaunchKernelGGL(hist_kernel<true>, dim3(nb), dim3(256),
                               (size_t)n_seg * 256 * sizeof(uint32_t), s, r.stats, b.seg_of_f0,
                               rw, b.state, b.hist, n_seg, shift);
        else
            hipLaunchKernelGGL(hist_kernel<false>, dim3(nb), dim3(256), 0, s, r.stats,
                               b.seg_of_f0, rw, b.state, b.hist, n_seg, shift);
        hipLaunchKernelGGL(scan_kernel, dim3(sg_blocks), dim3(256), 0, s, b.state, b.hist, n_seg,
                           shift, 2.0 * rel_err);
    }
    const bool lds_cnt = n_seg <= 8192;
    if (cols == 4)
        hipLaunchKernelGGL(count_grid_kernel<4>, dim3(nb), dim3(256), (size_t)n_seg * sizeof(uint32_t), s, r.stats,
                           b.seg_of_f0, rw, b.state, b.cnt, n_seg);
    else if (cols == 8)
        hipLaunchKernelGGL(count_grid_kernel<8>, dim3(nb), dim3(256), (size_t)n_seg * sizeof(uint32_t), s, r.stats,
                           b.seg_of_f0, rw, b.state, b.cnt, n_seg);
    else if (lds_cnt)
        hipLaunchKernelGGL(count_kernel<true>, dim3(nb), dim3(256),
                           (size_t)n_seg * sizeof(uint32_t), s, r.stats, b.seg_of_f0, rw,
                           b.state, b.cnt, n_seg);
    else
        hipLaunchKernelGGL(count_kernel<false>, dim3(nb), dim3(256), 0, s, r.stats, b.seg_of_f0,
                           rw, b.state, b.cnt, n_seg);
    hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(64), 0, s, b.cnt, b.off, n_seg, b.cap,
                       r.err);
    if (cols == 4)
        hipLaunchKernelGGL(scatter_grid_kernel<4>, dim3(nb), dim3(256), 0, s, r.stats, b.seg_of_f0, rw, b.state,
                           b.off, b.fill, b.cand, b.cap);
    else if (cols == 8)
        hipLaunchKernelGGL(scatter_grid_kernel<8>, dim3(nb), dim3(256), 0, s, r.stats, b.seg_of_f0, rw, b.state,
                           b.off, b.fill, b.cand, b.cap);
    else
        hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(256), 0, s, r.stats, b.seg_of_f0, rw,
                           b.state, b.off, b.fill, b.cand, b.cap);
    return hipGetLastError();
}

hipError_t launch_rescore_rank(const EvalRun &r, bool grid, int n_seg, int k,
                               const SelectBufs &b, hipStream_t s)
{
    double *mom = !grid && r.arms ? b.cand_mom : nullptr;  // binary banks with sky weights
    hipLaunchKernelGGL(rescore_kernel, dim3(2048), dim3(256), 0, s, r, grid, b.cand, b.off, n_seg,
                       b.cap, b.cand_s64, mom);
    hipLaunchKernelGGL(rank_kernel, dim3(1024), dim3(256), 0, s, r, grid, b.cand, b.cand_s64,
                       b.off, n_seg, b.cap, k, b.mu_sigma, mom, b.out);
    hipLaunchKernelGGL(n_out_kernel, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, s,
                       b.cnt, n_seg, k, b.n_out);
    return hipGetLastError();
}

// --- loudest template per hyperbox ------------------------------------------
__global__ void box_init_kernel(int64_t n_boxes, uint32_t *max32, int32_t *count, unsigned long long *max64,
                                unsigned long long *idx, uint32_t *n_cand)
{
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_boxes;
         b += (int64_t)gridDim.x * blockDim.x) {
        max32[b] = 0u;
        count[b] = 0;
        max64[b] = 0ull;
        idx[b] = ~0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) n_cand[threadIdx.x] = 0u;
}

// Statistics are >= 0, so their bit patterns order like their values.
__global__ void box_max_kernel(const float *stats, const int32_t *box, int64_t n, uint32_t *max32, int32_t *count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = box[i];
        atomicMax(max32 + b, __float_as_uint(stats[i]));
        atomicAdd(count + b, 1);
    }
}

// Candidates: S32 >= max32 (1 - 2 rel_err).  The template with the largest
// S64 of a box has S32 >= S64 (1 - rel) and the box's FP32 maximum is at most
// S64max (1 + rel), so it is always kept.
__global__ void box_cand_kernel(const float *stats, const int32_t *box, int64_t n, const uint32_t *max32, double keep,
                                int64_t *cand, uint32_t *n_cand, int64_t cap, uint32_t *err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double thr = (double)__uint_as_float(max32[box[i]]) * keep;
        if ((double)stats[i] >= thr) {
            const uint32_t pos = atomicAdd(n_cand + 1, 1u);
            if (pos < cap) cand[pos] = i;
            else atomicOr(err, ERR_CAND_OVERFLOW);
        }
    }
}

__global__ void box_pick_kernel(const int64_t *cand, const double *s64, const uint32_t *n_cand, int64_t cap,
                                const int32_t *box, unsigned long long *max64)
{
    const int64_t total = min((int64_t)n_cand[1], cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x)
        atomicMax(max64 + box[cand[p]], (unsigned long long)__double_as_longlong(s64[p]));
}

__global__ void box_index_kernel(const int64_t *cand, const double *s64, const uint32_t *n_cand, int64_t cap,
                                 const int32_t *box, const unsigned long long *max64, unsigned long long *idx)
{
    const int64_t total = min((int64_t)n_cand[1], cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = box[cand[p]];
        if ((unsigned long long)__double_as_longlong(s64[p]) == max64[b]) atomicMin(idx + b, (unsigned long long)cand[p]);
    }
}

__global__ void box_out_kernel(int64_t n_boxes, const int32_t *count, const unsigned long long *max64,
                               const unsigned long long *idx, const float *stats, const double *mu_sigma,
                               ft_box_result *out)
{
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_boxes;
         b += (int64_t)gridDim.x * blockDim.x) {
        ft_box_result r;
        r.count = count[b];
        if (r.count > 0) {
            r.index = (int64_t)idx[b];
            r.s32 = stats[r.index];
            r.s64 = __longlong_as_double((long long)max64[b]);
            r.z = (r.s64 - mu_sigma[0]) / mu_sigma[1];
        } else {
            r.index = -1;
            r.s32 = 0.f;
            r.s64 = 0.0;
            r.z = 0.0;
        }
        out[b] = r;
    }
}

hipError_t launch_box_max(const EvalRun &r, int64_t n, int64_t n_boxes, const BoxBufs &b, double rel_err,
                          hipStream_t s)
{
    const unsigned gb = (unsigned)std::min<int64_t>((n_boxes + 255) / 256, 8192);
    const unsigned gn = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(box_init_kernel, dim3(gb > 0 ? gb : 1), dim3(256), 0, s, n_boxes, b.max32, b.count, b.max64,
                       b.idx, b.n_cand);
    if (n <= 0) return hipGetLastError();
    hipLaunchKernelGGL(box_max_kernel, dim3(gn), dim3(256), 0, s, r.stats, b.box, n, b.max32, b.count);
    hipLaunchKernelGGL(box_cand_kernel, dim3(gn), dim3(256), 0, s, r.stats, b.box, n, b.max32, 1.0 - 2.0 * rel_err,
                       b.cand, b.n_cand, b.cap, r.err);
    return hipGetLastError();
}

hipError_t launch_box_pick(const EvalRun &r, int64_t n_boxes, const BoxBufs &b, const double *mu_sigma,
                           ft_box_result *out, hipStream_t s)
{
    const unsigned gb = (unsigned)std::min<int64_t>((n_boxes + 255) / 256, 8192);
    hipLaunchKernelGGL(rescore_kernel, dim3(2048), dim3(256), 0, s, r, false, b.cand, b.n_cand, 1, b.cap,
                       b.cand_s64, (double *)nullptr);
    hipLaunchKernelGGL(box_pick_kernel, dim3(1024), dim3(256), 0, s, b.cand, b.cand_s64, b.n_cand, b.cap, b.box,
                       b.max64);
    hipLaunchKernelGGL(box_index_kernel, dim3(1024), dim3(256), 0, s, b.cand, b.cand_s64, b.n_cand, b.cap, b.box,
                       b.max64, b.idx);
    hipLaunchKernelGGL(box_out_kernel, dim3(gb > 0 ? gb : 1), dim3(256), 0, s, n_boxes, b.count, b.max64, b.idx,
                       r.stats, mu_sigma, out);
    return hipGetLastError();
}

hipError_t launch_rescore_entries(const EvalRun &r, bool grid, const ft_candidate *top, const int32_t *n_out,
                                  double *out, hipStream_t s)
{
    hipLaunchKernelGGL(rescore_entries_kernel, dim3(64), dim3(256), 0, s, r, grid, top, n_out, out);
    return hipGetLastError();
}

}  // namespace ft
