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
// B(k, n) = B[k*ldb + n].  M, N multiples of 64, K a multiple of 32.
// Epilogues (ld = N):
//   EPI_FWD:   z = acc + bias[n]; zf[m][n] = z; act[m][n] = bf16(gelu(z))
//   EPI_BWD:   d = acc * gelu'(zprev[m][n]); zf[m][n] = d; act[m][n] = bf16(d)
//   EPI_STORE: zf[m][n] = acc
template <bool A_KMAJOR, bool B_KMAJOR, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const __bf16 *A, const __bf16 *B, int M,
                                                        int N, int K, int lda, int ldb,
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
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[2], b[2];
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
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
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

// Layer 4 (256 -> 1) + sigmoid + BCE: one wavefront per sample.
__global__ void head_kernel(const __bf16 *a3, const float *params, const float *labels,
                            MlpConst c, int bsz, float inv_n, float *logit, float *dlogit,
                            float *prob, float *loss_sum)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= bsz) return;
    const float *W4 = params + MLP_OFF_W4;
    float s = 0.f;
    for (int i = lane; i < H; i += 64) s += W4[i] * (float)a3[(int64_t)b * H + i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane != 0) return;
    const float z = s + params[MLP_OFF_W4 + H];
    const float p = 1.f / (1.f + expf(-z));
    logit[b] = z;
    if (prob) prob[b] = p;
    if (labels) {
        const float y = labels[sample_index(b, c)];
        dlogit[b] = (p - y) * inv_n;
        const float l = fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
        atomicAdd(loss_sum, l * inv_n);
    }
}

// dZ3 = (dlogit w4) * gelu'(z3), padded rows zero.
__global__ void head_back_kernel(const float *dlogit, const float *params, const float *z3,
                                 int bsz, int m_pad, float *dz, __bf16 *dzb)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)m_pad * H) return;
    const int b = (int)(q / H), i = (int)(q % H);
    const float d = b < bsz ? dlogit[b] * params[MLP_OFF_W4 + i] * gelu_grad(z3[q]) : 0.f;
    dz[q] = d;
    dzb[q] = (__bf16)d;
}

// Gradient reductions over the batch, in two deterministic stages: chunk c of
// RED_ROWS rows writes part[c][q] = sum over its rows of term(b, q); then
// out[q] = sum_c part[c][q] in chunk order.
//   RED_COL:  term = v[b][q], q < 256 (bias gradients)
//   RED_HEAD: term = dlogit[b] a3[b][q] for q < 256, dlogit[b] for q = 256
//             (output-layer weights and bias)
//   RED_L1:   the first layer: for hidden unit j, term = dz1[b][j] x[b][i] at
//             q = 6 j + i (i < 6, weights) and dz1[b][j] at q = 1536 + j
//             (bias), one thread per unit holding its seven sums
enum { RED_COL = 0, RED_HEAD = 1, RED_L1 = 2 };
constexpr int RED_ROWS = 16;

template <int MODE>
__global__ __launch_bounds__(256) void reduce_part_kernel(const float *v, const __bf16 *a3,
                                                          const float *x, int bsz, int n_out,
                                                          float *part)
{
    const int c = blockIdx.x;
    const int b0 = c * RED_ROWS, b1 = min(b0 + RED_ROWS, bsz);
    if (MODE == RED_L1) {
        const int j = threadIdx.x;  // blockDim.x == H
        float s[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int b = b0; b < b1; ++b) {
            const float d = v[(int64_t)b * H + j];
#pragma unroll
            for (int i = 0; i < 6; ++i) s[i] += d * x[b * 6 + i];
            s[6] += d;
        }
        float *out = part + (int64_t)c * n_out;
#pragma unroll
        for (int i = 0; i < 6; ++i) out[6 * j + i] = s[i];
        out[6 * H + j] = s[6];
        return;
    }
    for (int q = threadIdx.x; q < n_out; q += blockDim.x) {
        float s = 0.f;
        for (int b = b0; b < b1; ++b) {
            if (MODE == RED_COL) s += v[(int64_t)b * H + q];
            if (MODE == RED_HEAD) s += q < H ? v[b] * (float)a3[(int64_t)b * H + q] : v[b];
        }
        part[(int64_t)c * n_out + q] = s;
    }
}

__global__ void reduce_sum_kernel(const float *part, int n_chunks, int n_out, float *out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_out) return;
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * n_out + q];
    out[q] = s;
}

// Adam (Kingma and Ba 2015) with bias correction; refreshes the BF16 copies of
// the two 256 x 256 weight matrices.
__global__ void adam_kernel(float *theta, const float *g, float *m, float *v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2, __bf16 *w2b,
                            __bf16 *w3b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = t;
    if (i >= MLP_OFF_W2 && i < MLP_OFF_W2 + H * H) w2b[i - MLP_OFF_W2] = (__bf16)t;
    if (i >= MLP_OFF_W3 && i < MLP_OFF_W3 + H * H) w3b[i - MLP_OFF_W3] = (__bf16)t;
}

__global__ void to_bf16_kernel(const float *src, __bf16 *dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (__bf16)src[i];
}

unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int MODE>
void reduce_rows(const float *v, const __bf16 *a3, const float *x, int bsz, int n_out, float *part,
                 float *out, hipStream_t s)
{
    const int n_chunks = (bsz + RED_ROWS - 1) / RED_ROWS;
    hipLaunchKernelGGL(reduce_part_kernel<MODE>, dim3(n_chunks), dim3(256), 0, s, v, a3, x, bsz, n_out,
                       part);
    hipLaunchKernelGGL(reduce_sum_kernel, dim3(blocks(n_out, 256)), dim3(256), 0, s, part, n_chunks, n_out,
                       out);
}

}  // namespace

hipError_t mlp_refresh_bf16(const MlpBufs &m, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(H * H, 256)), dim3(256), 0, s,
                       m.theta + MLP_OFF_W2, m.w2b, H * H);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(H * H, 256)), dim3(256), 0, s,
                       m.theta + MLP_OFF_W3, m.w3b, H * H);
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
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_FWD>), g2, dim3(256), 0, s, m.a1, m.w2b,
                       m_pad, H, H, H, H, m.theta + MLP_OFF_W2 + H * H, nullptr, m.z2, m.a2);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, EPI_FWD>), g2, dim3(256), 0, s, m.a2, m.w3b,
                       m_pad, H, H, H, H, m.theta + MLP_OFF_W3 + H * H, nullptr, m.z3, m.a3);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(bsz, 4)), dim3(256), 0, s, m.a3, m.theta, labels, c,
                       bsz, 1.f / (float)bsz, m.logit, m.dlogit, prob, m.loss);
    return hipGetLastError();
}

// Backward pass after mlp_forward with labels: gradient into m.grad.
hipError_t mlp_backward(const MlpBufs &m, int bsz, hipStream_t s)
{
    const int m_pad = (bsz + 63) / 64 * 64;
    const dim3 g2(H / 64, m_pad / 64);
    const dim3 gw(H / 64, H / 64);
    float *g = m.grad;
    reduce_rows<RED_HEAD>(m.dlogit, m.a3, nullptr, bsz, H + 1, m.part, g + MLP_OFF_W4, s);
    hipLaunchKernelGGL(head_back_kernel, dim3(blocks((int64_t)m_pad * H, 256)), dim3(256), 0, s,
                       m.dlogit, m.theta, m.z3, bsz, m_pad, m.dz3, m.dz3b);
    // layer 3: dW3 = dZ3^T A2, db3 = colsum dZ3, dZ2 = (dZ3 W3) * gelu'(Z2)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false, EPI_STORE>), gw, dim3(256), 0, s, m.dz3b,
                       m.a2, H, H, m_pad, H, H, nullptr, nullptr, g + MLP_OFF_W3, nullptr);
    reduce_rows<RED_COL>(m.dz3, nullptr, nullptr, bsz, H, m.part, g + MLP_OFF_W3 + H * H, s);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false, EPI_BWD>), g2, dim3(256), 0, s, m.dz3b, m.w3b,
                       m_pad, H, H, H, H, nullptr, m.z2, m.dz2, m.dz2b);
    // layer 2
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false, EPI_STORE>), gw, dim3(256), 0, s, m.dz2b,
                       m.a1, H, H, m_pad, H, H, nullptr, nullptr, g + MLP_OFF_W2, nullptr);
    reduce_rows<RED_COL>(m.dz2, nullptr, nullptr, bsz, H, m.part, g + MLP_OFF_W2 + H * H, s);
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false, EPI_BWD>), g2, dim3(256), 0, s, m.dz2b, m.w2b,
                       m_pad, H, H, H, H, nullptr, m.z1, m.dz1, m.dz1b);
    // layer 1
    // weights and bias of the first layer are contiguous: g[0 .. 7H)
    reduce_rows<RED_L1>(m.dz1, nullptr, m.x, bsz, H * 7, m.part, g, s);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpBufs &m, float lr, int t, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(MLP_N_PARAMS, 256)), dim3(256), 0, s, m.theta, m.grad,
                       m.m, m.v, MLP_N_PARAMS, lr, b1, b2, 1e-8f, c1, c2, m.w2b, m.w3b);
    return hipGetLastError();
}

}  // namespace ft
