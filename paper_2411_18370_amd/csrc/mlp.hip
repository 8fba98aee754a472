// Detection-probability surrogate: MLP 6 -> 256 -> 256 -> 256 -> 1, GELU
// hidden activations, sigmoid output, binary cross-entropy, Adam -- trained
// and run on the GPU.  It estimates p_det of Sec. V (Eqs. pdet_abstract and
// sampling) from injection parameters.
//
// The two 256 x 256 layers (forward, input-gradient and weight-gradient
// products) run on the matrix cores: v_mfma_f32_16x16x32_bf16, BF16 operands,
// FP32 accumulation; each wavefront owns a 32 x 32 output tile (2 x 2 MFMA
// blocks).  Master weights, biases, Adam moments, pre-activations and
// gradients are FP32; activations and the 256 x 256 weights feed the MFMAs in
// BF16.  The 6-wide input layer and the 1-wide output layer are VALU kernels.
//
// Parameter vector (flat FP32): W1 [256][6], b1 [256], W2 [256][256], b2,
// W3 [256][256], b3, W4 [256], b4 -- 133,633 values; Z_l = A_{l-1} W_l^T + b_l.
//
// One training step is ten launches: the input layer, two forward GEMMs, the
// output layer fused with its backward step, four backward GEMMs (the two
// weight-gradient products split over the batch into up to 8 slices so they
// fill more than 16 workgroups), one kernel of per-chunk column sums for every
// bias and the first and last layers, and one kernel that finishes every
// gradient entry (sum over chunks or slices, in a fixed order), applies Adam
// and adds the batch loss.  Every reduction is deterministic.
#include <algorithm>

#include "ft_internal.h"

namespace ft {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int H = 256;

__device__ __forceinline__ float gelu(float x)
{
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float x)
{
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
    return cdf + x * pdf;
}

enum { EPI_FWD = 0, EPI_BWD = 1, EPI_STORE = 2 };

// C[M][N] = A[M][K] B[K][N].  A_KMAJOR: A(m, k) = A[m*lda + k], else
// A(m, k) = A[k*lda + m].  B_KMAJOR: B(k, n) = B[n*ldb + k], else
// B(k, n) = B[k*ldb + n].  M, N multiples of 64, K and k_slice multiples of
// 32.  Workgroup z sums k in [z k_slice, min(K, (z + 1) k_slice)).  KC > 0
// fixes K = k_slice = KC at compile time: the k loop is unrolled, so every
// operand load is issued before the first product waits on one.
// Epilogues (ld = N):
//   EPI_FWD:   z = acc + bias[n]; zf[m][n] = z; act[m][n] = bf16(gelu(z))
//   EPI_BWD:   d = acc * gelu'(zprev[m][n]); zf[m][n] = d; act[m][n] = bf16(d)
//   EPI_STORE: zf[z][m][n] = acc (one partial product per slice z)
template <bool A_KMAJOR, bool B_KMAJOR, int EPI, int KC = 0>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const __bf16 *A, const __bf16 *B, int M,
                                                        int N, int K, int k_slice, int lda, int ldb,
                                                        const float *bias, const float *zprev,
                                                        float *zf, __bf16 *act)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int lr = lane & 15;        // row (A) / column (B) within a 16-block
    const int lk = (lane >> 4) * 8;  // first of the lane's 8 k values
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int k0, bf16x8 (&a)[2], bf16x8 (&b)[2]) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m0 + i * 16 + lr;
            if (A_KMAJOR) {
                a[i] = *(const bf16x8 *)(A + (int64_t)m * lda + k0 + lk);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) a[i][q] = A[(int64_t)(k0 + lk + q) * lda + m];
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + j * 16 + lr;
            if (B_KMAJOR) {
                b[j] = *(const bf16x8 *)(B + (int64_t)n * ldb + k0 + lk);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) b[j][q] = B[(int64_t)(k0 + lk + q) * ldb + n];
            }
        }
    };
    auto mma = [&](const bf16x8 (&a)[2], const bf16x8 (&b)[2]) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    };
    if (KC) {
        // every operand of the product is loaded before the first MFMA
        bf16x8 a[KC ? KC / 32 : 1][2], b[KC ? KC / 32 : 1][2];
#pragma unroll
        for (int t = 0; t < KC / 32; ++t) load(32 * t, a[t], b[t]);
        __builtin_amdgcn_sched_barrier(0);  // keep the scheduler from interleaving them again
#pragma unroll
        for (int t = 0; t < KC / 32; ++t) mma(a[t], b[t]);
    } else {
        const int k_begin = blockIdx.z * k_slice, k_end = min(K, k_begin + k_slice);
        if (EPI == EPI_STORE) zf += (int64_t)blockIdx.z * M * N;
        for (int k0 = k_begin; k0 < k_end; k0 += 32) {
            bf16x8 a[2], b[2];
            load(k0, a, b);
            mma(a, b);
        }
    }
    // output layout: lane holds column n0 + j*16 + lane%16, rows 4*(lane/16) + r
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + i * 16 + (lane >> 4) * 4 + r;
                const int64_t o = (int64_t)m * N + n;
                const float v = acc[i][j][r];
                if (EPI == EPI_FWD) {
                    const float z = v + bias[n];
                    zf[o] = z;
                    act[o] = (__bf16)gelu(z);
                } else if (EPI == EPI_BWD) {
                    const float d = v * gelu_grad(zprev[o]);
                    zf[o] = d;
                    act[o] = (__bf16)d;
                } else {
                    zf[o] = v;
                }
            }
        }
}

// Standardised features of sample idx(b): (log amp, cos iota, psi, sin delta,
// alpha, f) -> (g - shift)/scale.
__device__ __forceinline__ float feature(const float *raw, int64_t s, int i, const MlpConst &c)
{
    float g = raw[s * 6 + i];
    if (i == 0) g = logf(g);
    return (g - c.shift[i]) / c.scale[i];
}

__device__ __forceinline__ int64_t sample_index(int64_t b, const MlpConst &c)
{
    return c.perm_a == 0 ? c.base + b : (int64_t)((c.perm_a * (uint64_t)(c.base + b) + c.perm_c) % (uint64_t)c.n_total);
}

// Layer 1 (6 -> 256): x[b][i] features, z1, a1 = bf16(gelu(z1)).
__global__ void layer1_kernel(const float *raw, const float *params, MlpConst c, int bsz, int m_pad,
                              float *x, float *z1, __bf16 *a1)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)m_pad * H) return;
    const int b = (int)(q / H), o = (int)(q % H);
    if (b >= bsz) {  // padding rows: zero activations and features
        z1[q] = 0.f;
        a1[q] = (__bf16)0.f;
        if (o < 6) x[b * 6 + o] = 0.f;
        return;
    }
    const int64_t s = sample_index(b, c);
    const float *W1 = params;
    const float *b1 = params + H * 6;
    float z = b1[o];
    for (int i = 0; i < 6; ++i) z += W1[o * 6 + i] * feature(raw, s, i, c);
    if (o < 6) x[b * 6 + o] = feature(raw, s, o, c);
    z1[q] = z;
    a1[q] = (__bf16)gelu(z);
}

// Layer 4 (256 -> 1) and sigmoid, one wavefront per row of the padded batch.
// With labels it also forms the per-sample loss and the output-side backward
// step: dlogit = (p - y)/n and dZ3 = dlogit w4 * gelu'(z3) (zero on padding
// rows, which the weight-gradient products sum over).
__global__ void head_kernel(const __bf16 *a3, const float *z3, const float *params,
                            const float *labels, MlpConst c, int bsz, int m_pad, float inv_n,
                            float *logit, float *dlogit, float *prob, float *lossv, float *dz,
                            __bf16 *dzb)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= m_pad) return;
    const float *W4 = params + MLP_OFF_W4;
    if (b >= bsz) {
        if (labels)
            for (int i = lane; i < H; i += 64) {
                dz[(int64_t)b * H + i] = 0.f;
                dzb[(int64_t)b * H + i] = (__bf16)0.f;
            }
        return;
    }
    float s = 0.f;
    for (int i = lane; i < H; i += 64) s += W4[i] * (float)a3[(int64_t)b * H + i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);  // every lane holds the sum
    const float z = s + params[MLP_OFF_W4 + H];
    const float p = 1.f / (1.f + expf(-z));
    if (lane == 0) {
        logit[b] = z;
        if (prob) prob[b] = p;
    }
    if (!labels) return;
    const float y = labels[sample_index(b, c)];
    const float d = (p - y) * inv_n;
    if (lane == 0) {
        dlogit[b] = d;
        lossv[b] = fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
    }
    for (int i = lane; i < H; i += 64) {
        const int64_t q = (int64_t)b * H + i;
        const float v = d * W4[i] * gelu_grad(z3[q]);
        dz[q] = v;
        dzb[q] = (__bf16)v;
    }
}

// Column sums over the batch for every gradient entry that is not a 256 x 256
// weight, in chunks of MLP_RED_ROWS rows: part[c][q] = sum over the rows of
// chunk c.  Compact index q (MLP_RED_VEC entries):
//   [0, 6H)     W1 (unit j, input i at 6 j + i): dZ1[b][j] x[b][i]
//   [6H, 7H)    b1: dZ1[b][j]
//   [7H, 8H)    b2: dZ2[b][j]
//   [8H, 9H)    b3: dZ3[b][j]
//   [9H, 10H)   W4: dlogit[b] A3[b][j]
//   10H         b4: dlogit[b]
// Workgroup (c, section) handles one chunk of one section: wave w sums rows
// b0 + w, b0 + w + 4, ..., lane l units l + 64 u (u < 4), and the four wave
// sums are added in wave order.
__global__ __launch_bounds__(256) void grad_part_kernel(const float *dz1, const float *dz2,
                                                        const float *dz3, const float *dlogit,
                                                        const __bf16 *a3, const float *x, int bsz,
                                                        float *part)
{
    __shared__ float red[4][7 * H];
    const int c = blockIdx.x, sec = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b0 = c * MLP_RED_ROWS, b1 = min(b0 + MLP_RED_ROWS, bsz);
    float *mine = red[wave];
    float *out = part + (int64_t)c * MLP_RED_VEC;
    int n_red, at;  // entries of this section and their first compact index
    if (sec == 0) {
        float t[4][7];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 7; ++i) t[u][i] = 0.f;
#pragma unroll 4
        for (int b = b0 + wave; b < b1; b += 4) {
            float xi[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) xi[i] = x[b * 6 + i];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float d = dz1[(int64_t)b * H + lane + 64 * u];
#pragma unroll
                for (int i = 0; i < 6; ++i) t[u][i] += d * xi[i];
                t[u][6] += d;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = lane + 64 * u;
#pragma unroll
            for (int i = 0; i < 6; ++i) mine[6 * j + i] = t[u][i];
            mine[6 * H + j] = t[u][6];
        }
        n_red = 7 * H;
        at = 0;
    } else if (sec < 3) {
        const float *v = sec == 1 ? dz2 : dz3;
        float t[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int b = b0 + wave; b < b1; b += 4)
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] += v[(int64_t)b * H + lane + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) mine[lane + 64 * u] = t[u];
        n_red = H;
        at = (6 + sec) * H;
    } else {
        float t[4] = {0.f, 0.f, 0.f, 0.f}, tb = 0.f;
#pragma unroll 4
        for (int b = b0 + wave; b < b1; b += 4) {
            const float dl = dlogit[b];
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] += dl * (float)a3[(int64_t)b * H + lane + 64 * u];
            tb += dl;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) mine[lane + 64 * u] = t[u];
        if (lane == 0) mine[H] = tb;
        n_red = H + 1;
        at = 9 * H;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_red; q += 256)
        out[at + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// Finishes the gradient: g[i] = sum over chunks of part (compact entries) or
// over the slices of the split weight-gradient products (wpart [2][n_slices]
// [H][H], W2 then W3), each in index order.  With adam set, Adam (Kingma and
// Ba 2015, bias-corrected) updates theta and refreshes the BF16 copies of W2
// and W3 (row-major and transposed).  The last workgroup adds the batch's
// mean loss to *loss.
struct AdamArgs {
    bool on;
    float lr, b1, b2, eps, c1, c2;
};

__global__ __launch_bounds__(256) void grad_finish_kernel(const float *part, int n_chunks,
                                                          const float *wpart, int n_slices,
                                                          const float *lossv, int bsz, float inv_n,
                                                          float *loss, float *g, AdamArgs ad,
                                                          float *theta, float *m, float *v,
                                                          __bf16 *w2b, __bf16 *w3b, __bf16 *w2t,
                                                          __bf16 *w3t)
{
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ float red[256];
        float t = 0.f;
        for (int b = threadIdx.x; b < bsz; b += 256) t += lossv[b];
        red[threadIdx.x] = t;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss += red[0] * inv_n;
        return;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_N_PARAMS) return;
    float gi = 0.f;
    int wm = -1, r = 0, q = 0;
    if (i >= MLP_OFF_W2 && i < MLP_OFF_W2 + H * H) {
        wm = 0;
        r = i - MLP_OFF_W2;
    } else if (i >= MLP_OFF_W3 && i < MLP_OFF_W3 + H * H) {
        wm = 1;
        r = i - MLP_OFF_W3;
    } else if (i < MLP_OFF_W2) {
        q = i;  // W1, b1
    } else if (i < MLP_OFF_W3) {
        q = 7 * H + (i - MLP_OFF_W2 - H * H);  // b2
    } else if (i < MLP_OFF_W4) {
        q = 8 * H + (i - MLP_OFF_W3 - H * H);  // b3
    } else {
        q = 9 * H + (i - MLP_OFF_W4);  // W4, b4
    }
    if (wm >= 0) {
        const float *w = wpart + (int64_t)wm * n_slices * H * H + r;
        for (int z = 0; z < n_slices; ++z) gi += w[(int64_t)z * H * H];
    } else {
#pragma unroll 8
        for (int c = 0; c < n_chunks; ++c) gi += part[(int64_t)c * MLP_RED_VEC + q];
    }
    g[i] = gi;
    if (!ad.on) return;
    const float mi = ad.b1 * m[i] + (1.f - ad.b1) * gi;
    const float vi = ad.b2 * v[i] + (1.f - ad.b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - ad.lr * (mi / ad.c1) / (sqrtf(vi / ad.c2) + ad.eps);
    theta[i] = t;
    const int rt = (r % H) * H + r / H;  // W[o][i] -> Wt[i][o]
    if (wm == 0) {
        w2b[r] = (__bf16)t;
        w2t[rt] = (__bf16)t;
    }
    if (wm == 1) {
        w3b[r] = (__bf16)t;
        w3t[rt] = (__bf16)t;
    }
}

// BF16 copies of a 256 x 256 weight matrix, row-major and transposed.
__global__ void to_bf16_kernel(const float *src, __bf16 *dst, __bf16 *dst_t)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= H * H) return;
    dst[r] = (__bf16)src[r];
    dst_t[(r % H) * H + r / H] = (__bf16)src[r];
}

unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t mlp_refresh_bf16(const MlpBufs &m, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(H * H, 256)), dim3(256), 0, s,
                       m.theta + MLP_OFF_W2, m.w2b, m.w2t);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(H * H, 256)), dim3(256), 0, s,
                       m.theta + MLP_OFF_W3, m.w3b, m.w3t);
    return hipGetLastError();
}

// Forward pass of samples [c.base, c.base + bsz) (m_pad = bsz rounded up to 64).
hipError_t mlp_forward(const MlpBufs &m, const float *raw, const float *labels, const MlpConst &c,
                       int bsz, float *prob, hipStream_t s)
{
    const int m_pad = (bsz + 63) / 64 * 64;
    const dim3 g2(H / 64, m_pad / 64);
    hipLaunchKernelGGL(layer1_kernel, dim3(blocks((int64_t)m_pad * H, 256)), dim3(256), 0, s, raw,
                       m.theta, c, bsz, m_pad, m.x, m.z1, m.a1);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_FWD, H>), g2, dim3(256), 0, s, m.a1, m.w2b,
                       m_pad, H, H, H, H, H, m.theta + MLP_OFF_W2 + H * H, nullptr, m.z2, m.a2);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_FWD, H>), g2, dim3(256), 0, s, m.a2, m.w3b,
                       m_pad, H, H, H, H, H, m.theta + MLP_OFF_W3 + H * H, nullptr, m.z3, m.a3);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(labels ? m_pad : bsz, 4)), dim3(256), 0, s, m.a3,
                       m.z3, m.theta, labels, c, bsz, m_pad, 1.f / (float)bsz, m.logit, m.dlogit,
                       prob, m.lossv, m.dz3, m.dz3b);
    return hipGetLastError();
}

// Backward pass after mlp_forward with labels (which already formed dZ3):
// the gradient into m.grad, then, with adam, one Adam step t.
hipError_t mlp_backward(const MlpBufs &m, int bsz, const MlpAdamStep *adam, hipStream_t s)
{
    const int m_pad = (bsz + 63) / 64 * 64;
    const dim3 g2(H / 64, m_pad / 64);
    // the weight-gradient products sum over the batch in n_sl slices of >= 256 rows
    const int n_sl = std::max(1, std::min(MLP_MAX_SLICES, m_pad / 256));
    const int k_sl = (m_pad / n_sl + 31) / 32 * 32;
    const dim3 gw(H / 64, H / 64, n_sl);
    float *w2p = m.wpart, *w3p = m.wpart + (int64_t)n_sl * H * H;
    // layer 3: dW3 = dZ3^T A2, dZ2 = (dZ3 W3) * gelu'(Z2) (W3 read transposed, k-major)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false, EPI_STORE>), gw, dim3(256), 0, s, m.dz3b,
                       m.a2, H, H, m_pad, k_sl, H, H, nullptr, nullptr, w3p, nullptr);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_BWD, H>), g2, dim3(256), 0, s, m.dz3b, m.w3t,
                       m_pad, H, H, H, H, H, nullptr, m.z2, m.dz2, m.dz2b);
    // layer 2
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false, EPI_STORE>), gw, dim3(256), 0, s, m.dz2b,
                       m.a1, H, H, m_pad, k_sl, H, H, nullptr, nullptr, w2p, nullptr);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_BWD, H>), g2, dim3(256), 0, s, m.dz2b, m.w2t,
                       m_pad, H, H, H, H, H, nullptr, m.z1, m.dz1, m.dz1b);
    // column sums (biases, first and last layer), then every entry finished at once
    const int n_chunks = (bsz + MLP_RED_ROWS - 1) / MLP_RED_ROWS;
    hipLaunchKernelGGL(grad_part_kernel, dim3(n_chunks, 4), dim3(256), 0, s, m.dz1, m.dz2, m.dz3,
                       m.dlogit, m.a3, m.x, bsz, m.part);
    AdamArgs ad{false, 0.f, 0.9f, 0.999f, 1e-8f, 1.f, 1.f};
    if (adam) {
        ad.on = true;
        ad.lr = adam->lr;
        ad.c1 = 1.f - powf(ad.b1, (float)adam->t);
        ad.c2 = 1.f - powf(ad.b2, (float)adam->t);
    }
    hipLaunchKernelGGL(grad_finish_kernel, dim3(blocks(MLP_N_PARAMS, 256) + 1), dim3(256), 0, s,
                       m.part, n_chunks, m.wpart, n_sl, m.lossv, bsz, 1.f / (float)bsz, m.loss,
                       m.grad, ad, m.theta, m.m, m.v, m.w2b, m.w3b, m.w2t, m.w3t);
    return hipGetLastError();
}

}  // namespace ft
