// Hardware ceilings measured on the device itself (benchmark harness, not
// part of the method): a streaming copy for the HBM bandwidth and, on a
// buffer that fits the 256 MB Infinity Cache and is copied several times in
// one launch, the cache bandwidth; FMA and exp2 chains for the VALU rates.
// The step kernels' measured fractions are reported against these as well as
// against the datasheet peaks.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace adk {
namespace {

constexpr int kCopyUnroll = 4;

// reps passes of dst[i] = src[i], i < n16, 16 bytes per lane and access,
// kCopyUnroll independent accesses in flight per lane.  With reps > 1 the
// same n16 elements are read and written again (the cache-resident case).
__global__ __launch_bounds__(kBlock) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                      int64_t n16, int64_t reps)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r = 0; r < reps; ++r) {
        int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        for (; i + (kCopyUnroll - 1) * stride < n16; i += kCopyUnroll * stride) {
            uint4 v[kCopyUnroll];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) dst[i + u * stride] = v[u];
        }
        for (; i < n16; i += stride) dst[i] = src[i];
    }
}

// One pass of dst[i] = src[i], one 16-byte access per lane: workgroup b
// copies the 4 KiB block b, so the workgroups in flight stream through one
// region of memory in address order.  On the MI355X this measured 6.2 TB/s
// (read + write, 1 GiB) where the grid-stride loop above measured 4.0-4.5
// at 4-32 workgroups per CU (5.4-5.6 with a contiguous 16 KiB block per
// workgroup and pass): the HBM ceiling takes this form.
__global__ __launch_bounds__(kBlock) void copy_block_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                            int64_t n16, int64_t first)
{
    const int64_t i = first + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

constexpr int kChains = 8;  // independent dependency chains per lane

// Every lane runs kChains chains of `iters` steps x <- fma(x, a, b) (T float
// or double) or x <- exp2(fma(x, a, b)) (EXP, float): a and b are kernel
// arguments, so nothing folds at compile time.  The caller passes a = 1,
// b = 0 (FMA) or a = b = 0 (EXP): every chain stays at 1 and out[lane] = 8.
template <class T, bool EXP>
__global__ __launch_bounds__(kBlock) void valu_kernel(T a, T b, int64_t iters, T *__restrict__ out)
{
    T x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = T(1);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            if constexpr (EXP)
                x[k] = __builtin_amdgcn_exp2f(fmaf(x[k], a, b));
            else
                x[k] = fma(x[k], a, b);
        }
    }
    T s = T(0);
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace
}  // namespace adk

int adk_ceiling_copy(void *dst, const void *src, int64_t bytes, int64_t reps, hipStream_t stream)
{
    if (bytes < 0 || reps < 1 || bytes % 16 != 0) return ADK_EINVAL;
    if (bytes > 0 && (!dst || !src)) return ADK_EINVAL;
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return ADK_OK;
    const int64_t need = (n16 + adk::kBlock - 1) / adk::kBlock;
    if (reps == 1) {
        // one block per workgroup, launches of at most 2^30 workgroups
        const int64_t maxg = (int64_t)1 << 30;
        for (int64_t g0 = 0; g0 < need; g0 += maxg) {
            const int64_t g = need - g0 < maxg ? need - g0 : maxg;
            hipLaunchKernelGGL(adk::copy_block_kernel, dim3((unsigned)g), dim3(adk::kBlock), 0, stream,
                               (const uint4 *)src, (uint4 *)dst, n16, g0 * adk::kBlock);
            if (hipGetLastError() != hipSuccess) return ADK_EDEVICE;
        }
        return ADK_OK;
    }
    const int64_t cap = (int64_t)adk::num_cus() * 8;
    const int grid = (int)(need < cap ? need : cap);
    hipLaunchKernelGGL(adk::copy_kernel, dim3(grid), dim3(adk::kBlock), 0, stream, (const uint4 *)src, (uint4 *)dst,
                       n16, reps);
    return hipGetLastError() == hipSuccess ? ADK_OK : ADK_EDEVICE;
}

int adk_ceiling_valu(int32_t kind, int64_t iters, void *out, int64_t nlanes, hipStream_t stream)
{
    if (kind < 0 || kind > 2 || iters < 0 || nlanes <= 0 || nlanes % adk::kBlock != 0 || !out) return ADK_EINVAL;
    if (nlanes / adk::kBlock > ((int64_t)1 << 30)) return ADK_ERANGE;
    const dim3 grid((unsigned)(nlanes / adk::kBlock));
    if (kind == 0)
        hipLaunchKernelGGL((adk::valu_kernel<float, false>), grid, dim3(adk::kBlock), 0, stream, 1.0f, 0.0f, iters,
                           (float *)out);
    else if (kind == 1)
        hipLaunchKernelGGL((adk::valu_kernel<double, false>), grid, dim3(adk::kBlock), 0, stream, 1.0, 0.0, iters,
                           (double *)out);
    else
        hipLaunchKernelGGL((adk::valu_kernel<float, true>), grid, dim3(adk::kBlock), 0, stream, 0.0f, 0.0f, iters,
                           (float *)out);
    return hipGetLastError() == hipSuccess ? ADK_OK : ADK_EDEVICE;
}
