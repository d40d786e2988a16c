// HIP kernels for gfx950 (templates; instantiated per precision and window
// width in inst.hip).
//
// One lane per mesh cell.  Cells are independent (Sec. 3, the analytic
// solution is computed cell by cell), so a step is a single streaming pass:
// coalesced structure-of-arrays loads of E, the window index and the window
// populations, per-cell arithmetic in registers, coalesced stores.  The gas
// coefficient table (a few KB) is staged in LDS once per workgroup of a
// grid-stride launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "adkion.h"
#include "chain.hpp"
#include "gas_table.hpp"

namespace adk {

constexpr int kBlock = 256;
constexpr int kCoefStride = 6;           // LDS: A + ln dt, alpha, B, c1, c2, c3
constexpr double kLog2e = 1.4426950408889634;
constexpr double kXMax = 1e30;           // cap of W dt (keeps inf out of the solver)

// Per-cell field terms of Eq. (1), in double: L = ln(E/E_a), R = E_a/E, u = E/E_a.
struct Field {
    double L, R, u;
    bool zero;
};

__device__ __forceinline__ Field field_terms(double E, double inv_Ea)
{
    Field f;
    const double EL = fabs(E);
    f.u = EL * inv_Ea;
    f.L = log(f.u);
    f.R = 1.0 / f.u;
    f.zero = (EL == 0.0);
    return f;
}

// Exponent of W_k dt (or of W_k when the LDS table holds A without ln dt) and
// the m-average polynomial, from the LDS row of level k.
__device__ __forceinline__ double rate_exponent(const double *row, const Field &f, double &poly)
{
    poly = fma(fma(fma(row[5], f.u, row[4]), f.u, row[3]), f.u, 1.0);
    return fma(-row[2], f.R, fma(row[1], f.L, row[0]));
}

template <class P>
struct RateEval;

template <>
struct RateEval<PolicyF64> {
    __device__ static __forceinline__ double x_of(const double *row, const Field &f)
    {
        double poly;
        const double y = rate_exponent(row, f, poly);
        double x = exp(y) * poly;
        x = f.zero ? 0.0 : x;
        return x < kXMax ? x : (x == x ? kXMax : x);
    }
};

template <>
struct RateEval<PolicyMixed> {
    __device__ static __forceinline__ float x_of(const double *row, const Field &f)
    {
        double poly;
        const double y = rate_exponent(row, f, poly);
        // 2^t with t split exactly in double: the integer part goes to the
        // exponent, only |f| <= 1/2 passes through the float exp2, so the
        // relative error stays ~1e-7 whatever the size of the exponent.
        double t = y * kLog2e;
        t = t < 120.0 ? t : (t == t ? 120.0 : t);
        t = t > -160.0 ? t : (t == t ? -160.0 : t);
        const double ti = rint(t);
        const float fr = (float)(t - ti);
        float x = ldexpf(exp2f(fr), (int)ti) * (float)poly;
        x = f.zero ? 0.0f : x;
        return x < (float)kXMax ? x : (x == x ? (float)kXMax : x);
    }
};

__device__ __forceinline__ void stage_coefficients(double *sc, const double *__restrict__ coef, int Z,
                                                   double ln_dt)
{
    for (int t = threadIdx.x; t < Z * kCoefStride; t += blockDim.x) {
        const int k = t / kCoefStride, f = t - k * kCoefStride;
        double v = coef[k * 8 + f];
        if (f == 0) v += ln_dt;
        sc[t] = v;
    }
    __syncthreads();
}

// Rates of the W window levels p..p+W-1 (0 past level Z-1).
template <class P, int W>
__device__ __forceinline__ void window_rates(const double *sc, int Z, int p, const Field &f,
                                             typename P::real (&x)[W])
{
    using R = typename P::real;
    static_for<0, W>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        const int k = p + s;
        const int kk = k < Z ? k : Z - 1;
        const R v = RateEval<P>::x_of(sc + kk * kCoefStride, f);
        x[s] = k < Z ? v : R(0);
    });
}

// ---------------------------------------------------------------------------
// ionize_step, compact layout: pops[(W+1)][n], slot s = level lo + s.
template <class P, int W>
__global__ __launch_bounds__(kBlock) void step_compact_kernel(
    const double *__restrict__ coef, int Z, double ln_dt, double inv_Ea, double eps,
    const typename P::real *__restrict__ E, typename P::real *__restrict__ pops,
    uint8_t *__restrict__ lo, int64_t n)
{
    using R = typename P::real;
    __shared__ double sc[ADK_MAX_Z * kCoefStride];
    stage_coefficients(sc, coef, Z, ln_dt);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += stride) {
        const double Ec = (double)E[c];
        int p = lo[c];
        p = p < Z ? p : Z;
        double N[W + 1];
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            N[s] = (double)pops[(int64_t)s * n + c];
        });
        // window shift at the start of the step; residual folded upward
        while (p < Z && N[0] < eps) {
            N[0] += N[1];
            static_for<1, W>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                N[s] = N[s + 1];
            });
            N[W] = 0.0;
            ++p;
        }
        const Field f = field_terms(Ec, inv_Ea);
        R x[W];
        window_rates<P, W>(sc, Z, p, f, x);
        double out[W + 1];
        chain_apply<P, W>(x, N, out);
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            pops[(int64_t)s * n + c] = (R)out[s];
        });
        lo[c] = (uint8_t)p;
    }
}

// ionize_step, full layout: pops[(Z+1)][n], row k = level k.
template <class P, int W>
__global__ __launch_bounds__(kBlock) void step_full_kernel(
    const double *__restrict__ coef, int Z, double ln_dt, double inv_Ea, double eps,
    const typename P::real *__restrict__ E, typename P::real *__restrict__ pops,
    uint8_t *__restrict__ lo, int64_t n)
{
    using R = typename P::real;
    __shared__ double sc[ADK_MAX_Z * kCoefStride];
    stage_coefficients(sc, coef, Z, ln_dt);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += stride) {
        const double Ec = (double)E[c];
        int p = lo[c];
        p = p < Z ? p : Z;
        const int p0 = p;
        double N[W + 1];
        N[0] = (double)pops[(int64_t)p * n + c];
        while (p < Z && N[0] < eps) {
            N[0] += (double)pops[(int64_t)(p + 1) * n + c];
            ++p;
        }
        static_for<1, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            N[s] = (p + s <= Z) ? (double)pops[(int64_t)(p + s) * n + c] : 0.0;
        });
        const Field f = field_terms(Ec, inv_Ea);
        R x[W];
        window_rates<P, W>(sc, Z, p, f, x);
        double out[W + 1];
        chain_apply<P, W>(x, N, out);
        for (int k = p0; k < p; ++k) pops[(int64_t)k * n + c] = R(0);
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            if (p + s <= Z) pops[(int64_t)(p + s) * n + c] = (R)out[s];
        });
        lo[c] = (uint8_t)p;
    }
}

// Chain advance with given rates W[w][n] (1/s), pops[(w+1)][n].
template <class P, int W>
__global__ __launch_bounds__(kBlock) void chain_advance_kernel(const typename P::real *__restrict__ Wr,
                                                               double dt, typename P::real *__restrict__ pops,
                                                               int64_t n)
{
    using R = typename P::real;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += stride) {
        R x[W];
        double N[W + 1];
        static_for<0, W>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            double v = (double)Wr[(int64_t)s * n + c] * dt;
            v = v < kXMax ? v : (v == v ? kXMax : v);
            x[s] = (R)v;
        });
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            N[s] = (double)pops[(int64_t)s * n + c];
        });
        double out[W + 1];
        chain_apply<P, W>(x, N, out);
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            pops[(int64_t)s * n + c] = (R)out[s];
        });
    }
}

// Rates W_out[j][i] = W_{k0+j}(E[i]) in 1/s (table staged with ln dt = 0).
template <class P>
__global__ __launch_bounds__(kBlock) void rates_kernel(const double *__restrict__ coef, int Z, int k0, int nk,
                                                       double inv_Ea, const typename P::real *__restrict__ E,
                                                       typename P::real *__restrict__ Wout, int64_t n)
{
    __shared__ double sc[ADK_MAX_Z * kCoefStride];
    stage_coefficients(sc, coef, Z, 0.0);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const Field f = field_terms((double)E[i], inv_Ea);
        for (int j = 0; j < nk; ++j) Wout[(int64_t)j * n + i] = RateEval<P>::x_of(sc + (k0 + j) * kCoefStride, f);
    }
}

// Launch helpers (one instantiation per precision and window width).
int grid_for(int64_t n);

template <class P, int W>
hipError_t launch_step(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                       const adk_window *win, hipStream_t st)
{
    using R = typename P::real;
    const int grid = grid_for(n);
    const double ln_dt = std::log(dt), inv_Ea = 1.0 / g->consts.E_a;
    if (win->layout == ADK_LAYOUT_COMPACT)
        hipLaunchKernelGGL((step_compact_kernel<P, W>), dim3(grid), dim3(kBlock), 0, st, g->d_coef, g->Z, ln_dt,
                           inv_Ea, win->eps, (const R *)E, (R *)pops, lo, n);
    else
        hipLaunchKernelGGL((step_full_kernel<P, W>), dim3(grid), dim3(kBlock), 0, st, g->d_coef, g->Z, ln_dt,
                           inv_Ea, win->eps, (const R *)E, (R *)pops, lo, n);
    return hipGetLastError();
}

template <class P, int W>
hipError_t launch_advance(const void *Wr, int64_t n, double dt, void *pops, hipStream_t st)
{
    using R = typename P::real;
    hipLaunchKernelGGL((chain_advance_kernel<P, W>), dim3(grid_for(n)), dim3(kBlock), 0, st, (const R *)Wr, dt,
                       (R *)pops, n);
    return hipGetLastError();
}

using StepFn = hipError_t (*)(const adk_gas *, const void *, int64_t, double, void *, uint8_t *,
                              const adk_window *, hipStream_t);
using AdvanceFn = hipError_t (*)(const void *, int64_t, double, void *, hipStream_t);

}  // namespace adk

// Non-template entry of each instantiation: adk_step_<prec>_<W>, adk_advance_<prec>_<W>.
#define ADK_DECLARE_INST(PREC, W)                                                                          \
    hipError_t adk_step_##PREC##_##W(const adk_gas *, const void *, int64_t, double, void *, uint8_t *,    \
                                     const adk_window *, hipStream_t);                                     \
    hipError_t adk_advance_##PREC##_##W(const void *, int64_t, double, void *, hipStream_t);
#define ADK_DECLARE_PREC(PREC)                                                                             \
    ADK_DECLARE_INST(PREC, 1)                                                                              \
    ADK_DECLARE_INST(PREC, 2)                                                                              \
    ADK_DECLARE_INST(PREC, 3)                                                                              \
    ADK_DECLARE_INST(PREC, 4)                                                                              \
    ADK_DECLARE_INST(PREC, 5)                                                                              \
    ADK_DECLARE_INST(PREC, 6)                                                                              \
    ADK_DECLARE_INST(PREC, 7)                                                                              \
    ADK_DECLARE_INST(PREC, 8)
ADK_DECLARE_PREC(f64)
ADK_DECLARE_PREC(mixed)
