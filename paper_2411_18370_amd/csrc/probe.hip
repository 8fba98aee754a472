// Microbenchmarks of the chip ceilings that bound the statistic's kernels:
// the LDS read rate of each instruction form a gather can use, and the HBM
// read rate of a plain streaming kernel.  They are the measured denominators
// of the roofline fractions (the vendor's nominal figures are not).
//
// LDS read probe.  Every workgroup (4 waves) fills a 16 KB LDS array, then
// each lane reads 8 dwords per iteration in one of these forms (consecutive
// lanes at consecutive addresses, no bank conflicts unless stated):
//   FT_LDS_B32           8 x ds_read_b32, rows of 64 dwords
//   FT_LDS_READ2ST64     4 x ds_read2st64_b32 (two rows of 64 dwords each)
//   FT_LDS_READ2_ADJ     4 x ds_read2_b32 of two adjacent dwords at a 4-byte
//                        aligned address (lane l at dword 2l + 1: two passes
//                        over the banks per instruction)
//   FT_LDS_B64           4 x ds_read_b64, 8-byte aligned
//   FT_LDS_B128          2 x ds_read_b128, 16-byte aligned
//   FT_LDS_READ2ST64_B64 2 x ds_read2st64_b64 (two 8-byte pairs 512 bytes apart)
// With `consume_all` every dword read is added into an FP32 accumulator (one
// VALU add per dword, as a gather-sum does); otherwise one add per
// instruction and the other dwords are only kept live, so VALU issue cannot
// hide the LDS rate.  The base address moves every iteration so no read can
// be hoisted.
#include "ft_internal.h"

namespace ft {

namespace {

constexpr int PROBE_LDS_DWORDS = 4096;  // 16 KB per workgroup

__device__ __forceinline__ void keep(float x)
{
    asm volatile("" ::"v"(x));
}

// a compiler barrier between loads keeps them as separate instructions
__device__ __forceinline__ void no_merge()
{
    asm volatile("" ::: "memory");
}

template <int FORM, bool ALL>
__global__ __launch_bounds__(256) void lds_read_kernel(int n_iter, float *out)
{
    __shared__ __attribute__((aligned(16))) float buf[PROBE_LDS_DWORDS];
    for (int i = threadIdx.x; i < PROBE_LDS_DWORDS; i += 256) buf[i] = (float)(i & 255) * 0.5f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc0 = 0.f, acc1 = 0.f;
    for (int it = 0; it < n_iter; ++it) {
        // base in [0, 1536] dwords, a multiple of 512; reads span < 1024 + 4
        const int base = (it & 3) * 512;
        if (FORM == FT_LDS_B32) {
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const float x = buf[base + 64 * m + lane];
                if (ALL || m == 0) acc0 += x; else keep(x);
                no_merge();
            }
        } else if (FORM == FT_LDS_READ2ST64) {
#pragma unroll
            for (int m = 0; m < 8; m += 2) {
                const float x = buf[base + 64 * m + lane];
                const float y = buf[base + 64 * (m + 1) + lane];
                if (ALL) { acc0 += x; acc1 += y; } else { acc0 += x; keep(y); }
                no_merge();
            }
        } else if (FORM == FT_LDS_READ2_ADJ) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float *p = buf + base + 128 * m + 2 * lane + 1;
                const float x = p[0];
                const float y = p[1];
                if (ALL) { acc0 += x; acc1 += y; } else { acc0 += x; keep(y); }
                no_merge();
            }
        } else if (FORM == FT_LDS_B64) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float2 v = *(const float2 *)(buf + base + 128 * m + 2 * lane);
                if (ALL) { acc0 += v.x; acc1 += v.y; } else { acc0 += v.x; keep(v.y); }
                no_merge();
            }
        } else if (FORM == FT_LDS_READ2ST64_B64) {
#pragma unroll
            for (int m = 0; m < 4; m += 2) {
                const float2 v = *(const float2 *)(buf + base + 128 * m + 2 * lane);
                const float2 w = *(const float2 *)(buf + base + 128 * (m + 1) + 2 * lane);
                if (ALL) {
                    acc0 += v.x; acc1 += v.y; acc0 += w.x; acc1 += w.y;
                } else {
                    acc0 += v.x; keep(v.y); keep(w.x); keep(w.y);
                }
                no_merge();
            }
        } else {  // FT_LDS_B128
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const float4 v = *(const float4 *)(buf + base + 256 * m + 4 * lane);
                if (ALL) {
                    acc0 += v.x; acc1 += v.y; acc0 += v.z; acc1 += v.w;
                } else {
                    acc0 += v.x; keep(v.y); keep(v.z); keep(v.w);
                }
                no_merge();
            }
        }
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc0 + acc1;
}

// Streaming read of n16 16-byte words (grid-stride, 16 B per lane per load).
__global__ __launch_bounds__(256) void hbm_read_kernel(const float4 *p, int64_t n16, float *out)
{
    float a = 0.f, b = 0.f;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
        const float4 v = p[i];
        a += v.x + v.y;
        b += v.z + v.w;
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = a + b;
}

template <int FORM>
hipError_t launch_lds_read_t(bool all, int n_blocks, int n_iter, float *out, hipStream_t s)
{
    if (all)
        hipLaunchKernelGGL((lds_read_kernel<FORM, true>), dim3(n_blocks), dim3(256), 0, s, n_iter, out);
    else
        hipLaunchKernelGGL((lds_read_kernel<FORM, false>), dim3(n_blocks), dim3(256), 0, s, n_iter, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lds_read_probe(int form, bool consume_all, int n_blocks, int n_iter, float *out, hipStream_t s)
{
    switch (form) {
    case FT_LDS_B32: return launch_lds_read_t<FT_LDS_B32>(consume_all, n_blocks, n_iter, out, s);
    case FT_LDS_READ2ST64: return launch_lds_read_t<FT_LDS_READ2ST64>(consume_all, n_blocks, n_iter, out, s);
    case FT_LDS_READ2_ADJ: return launch_lds_read_t<FT_LDS_READ2_ADJ>(consume_all, n_blocks, n_iter, out, s);
    case FT_LDS_B64: return launch_lds_read_t<FT_LDS_B64>(consume_all, n_blocks, n_iter, out, s);
    case FT_LDS_B128: return launch_lds_read_t<FT_LDS_B128>(consume_all, n_blocks, n_iter, out, s);
    case FT_LDS_READ2ST64_B64: return launch_lds_read_t<FT_LDS_READ2ST64_B64>(consume_all, n_blocks, n_iter, out, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hbm_read_probe(const void *src, int64_t bytes, int n_blocks, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(hbm_read_kernel, dim3(n_blocks), dim3(256), 0, s, (const float4 *)src, bytes / 16, out);
    return hipGetLastError();
}

}  // namespace ft
