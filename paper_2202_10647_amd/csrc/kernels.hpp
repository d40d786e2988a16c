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
constexpr double kLog2e = 1.4426950408889634;
// LDS row per level (base-2 exponent of W dt, field terms folded in):
//   t = a + alpha log2|E| - b / |E|,   W dt = 2^t (1 + c1 |E| + c2 |E|^2 + c3 |E|^3)
// a = (A + ln dt) log2(e) - alpha log2(E_a), b = B log2(e) E_a, c_j = c_j,orig / E_a^j.
// Rows Z..Z+kPadRows-1 hold a = -1e300 (rate 0), so windows reaching past
// level Z-1 need no per-level test.
constexpr int kCoefStride = 6;
constexpr int kPadRows = 8;
constexpr int kCoefRows = ADK_MAX_Z + kPadRows;
// log2 reduction table: 64 pairs (c_j, -log2 c_j), see fast_log2.
constexpr int kLogTable = 64;
// Cap of W dt.  Replacing a rate x_i > cap by the cap changes T by less than
// 0.37 / cap (the level empties either way; only x_{i+1}/x_i enters).
template <class R>
inline constexpr R kXMax = R(1e15);
template <>
inline constexpr float kXMax<float> = 1e12f;

// Launch arguments shared by the step kernels.
struct StepArgs {
    const double *tab;   // device table of the gas (kDevTableLen doubles)
    int Z;
    int has_poly;        // some level averages over m (c_j != 0)
    double ln_dt;
    double eps;
    double E_cut;        // below this |E| every rate of the gas is < 1e-30 per step
};

// Order in which a grid-stride kernel visits the chunks of its cells (kBlock
// cells per chunk for the step kernel, one wavefront's 64 for the surrogate):
// a permutation of the full chunks [0, chunks) (the last, partial chunk stays
// in place).  Chunk v goes to the first value below `chunks` on the orbit of
// v under Q = (odd multiply, xor-shift, odd multiply, xor-shift, bit
// reversal) on k bits, 2^k >= chunks: each step is a permutation of
// [0, 2^k), and the orbit is walked until it is back in range (cycle
// walking).  The dispatcher deals consecutive workgroups out to the XCDs and
// their CUs in turn; in cell order a field that is strong in one slab of the
// mesh (a laser pulse, whose z range falls on the same chunk residues in
// every row) lands on the few XCDs and CUs whose workgroups hold that slab,
// while the scattered order loads them alike.  Measured on the laser meshes
// (1M and 33.5M cells, mixed precision): 14.5 -> 10.8 us and 330 -> 275 us
// per step.
struct ChunkOrder {
    int64_t chunks;
    int bits;
};

__device__ __forceinline__ int64_t chunk_place(int64_t v, const ChunkOrder &o)
{
    if (v >= o.chunks || o.bits == 0) return v;
    const uint32_t mask = o.bits >= 32 ? 0xffffffffu : ((1u << o.bits) - 1u);
    const int sh = (o.bits + 1) / 2;
    uint32_t x = (uint32_t)v;
    do {
        x = (x * 0x9E3779B9u) & mask;
        x ^= x >> sh;
        x = (x * 0x85EBCA6Bu) & mask;
        x ^= x >> sh;
        x = __builtin_bitreverse32(x) >> (32 - o.bits);
    } while ((int64_t)x >= o.chunks);
    return (int64_t)x;
}

// Identity windows.  For each window start p < Z, the field below which
// every rate of the window p .. min(p + w, Z) - 1 is below kIdentityRate per
// step (the smallest of the levels' thresholds, rounded down): a cell under
// it with no shift due keeps its populations, which the exact step would
// change by less than w kIdentityRate of them (below FP64 rounding).
constexpr double kIdentityRate = 1e-16;
struct WinCut {
    float e[ADK_MAX_Z + 1];
};

// Host helpers (abi.hip).
WinCut window_cutoffs(const adk_gas *g, double dt, int w);
int num_cus();
int grid_for(int64_t n);
StepArgs step_args(const adk_gas *g, double dt, double eps);
ChunkOrder chunk_order(int64_t n, int64_t chunk = kBlock);

// log2 of a positive finite double v: v = m 2^k with m in [1/2, 1); the top
// six fraction bits of m select c_j ~ 1/m from the table, r = m c_j - 1 is
// formed with one rounding (|r| < 0.0078) and log2(1 + r) is a short series,
// so log2 v = k + (-log2 c_j) + r q(r).  D terms: D = 7 gives ~1e-19 (FP64
// path), D = 4 gives ~5e-12 (float path, where only ~1e-10 is needed).
template <int D>
__device__ __forceinline__ double fast_log2(double v, const double *slog)
{
    int k;
    const double m = frexp(v, &k);
    const unsigned hi = (unsigned)(__double_as_longlong(m) >> 32);
    const int j = (hi >> 14) & (kLogTable - 1);
    const double c = slog[2 * j], nlc = slog[2 * j + 1];
    const double r = fma(m, c, -1.0);
    double q = ((D & 1) ? -kLog2e : kLog2e) / (D + 1);
    static_for<0, D>([&](auto ii) {
        constexpr int i = D - 1 - decltype(ii)::value;
        q = fma(q, r, ((i & 1) ? -kLog2e : kLog2e) / (i + 1));
    });
    return fma(r, q, (double)k + nlc);
}

// 1/v from the hardware estimate and two Newton steps.
__device__ __forceinline__ double fast_rcp(double v)
{
    double r = __builtin_amdgcn_rcp(v);
    r = fma(r, fma(-v, r, 1.0), r);
    return fma(r, fma(-v, r, 1.0), r);
}

// Per-cell field terms of Eq. (1) in double: lg = log2|E|, inv = 1/|E|.
struct Field {
    double lg, inv, E;
};

template <int D>
__device__ __forceinline__ Field field_terms(double EL, const double *slog)
{
    // |E| = 0 (and non-finite |E|, whose cell is overwritten with NaN at the
    // end) is replaced by a tiny field: every rate underflows to exactly 0.
    Field f;
    f.E = EL > 1e-280 ? (EL <= 1e300 ? EL : 1.0) : 1e-280;
    f.lg = fast_log2<D>(f.E, slog);
    f.inv = fast_rcp(f.E);
    return f;
}

__device__ __forceinline__ double rate_exponent2(const double *row, const Field &f)
{
    return fma(-row[2], f.inv, fma(row[1], f.lg, row[0]));
}

__device__ __forceinline__ double mavg_poly(const double *row, const Field &f)
{
    return fma(fma(fma(row[5], f.E, row[4]), f.E, row[3]), f.E, 1.0);
}

template <class P>
struct RateEval;

template <>
struct RateEval<PolicyF64> {
    static constexpr int kLogTerms = 7;
    __device__ static __forceinline__ double x_of(const double *row, const Field &f, bool has_poly)
    {
        double x = exp2(rate_exponent2(row, f));
        if (has_poly) x *= mavg_poly(row, f);
        return x < kXMax<double> ? x : kXMax<double>;  // the cap (x is never NaN here)
    }
};

template <>
struct RateEval<PolicyMixed> {
    static constexpr int kLogTerms = 4;
    __device__ static __forceinline__ float x_of(const double *row, const Field &f, bool has_poly)
    {
        // 2^t with t split exactly in double: the integer part goes to the
        // exponent and only |fr| <= 1/2 passes through the float exp2, so the
        // relative error stays a few float ulps whatever the size of t.  The
        // lower bound keeps the integer part in range of the conversion (2^-160
        // is 0 in float; the field terms bound t above by |alpha| log2(1e300)
        // + a, far inside int); a t above 128 gives +inf, which the cap below
        // turns into kXMax (the m-average polynomial is at least 1, never 0).
        const double t = fmax(rate_exponent2(row, f), -160.0);
        const double ti = rint(t);
        // |t - ti| <= 1/2: the hardware exp2 (no range reduction needed)
        float x = ldexpf(__builtin_amdgcn_exp2f((float)(t - ti)), (int)ti);
        if (has_poly) x *= (float)mavg_poly(row, f);
        return __builtin_amdgcn_fmed3f(x, 0.0f, kXMax<float>);  // the cap (x >= 0, never NaN here)
    }
};

// Stage the prefolded coefficient rows (ln dt added to column 0) and the
// log2 table into LDS.  Device layout of a gas: kCoefRows x kCoefStride
// folded rows (see gas_table.cpp: fold_rows), then the 64 x 2 log2 table.
constexpr int kDevTableLen = kCoefRows * kCoefStride + 2 * kLogTable;

__device__ __forceinline__ void stage_coefficients(double *sc, const double *__restrict__ tab, double ln_dt)
{
    const double add = ln_dt * kLog2e;
    for (int t = threadIdx.x; t < kDevTableLen; t += blockDim.x) {
        const double v = tab[t];
        sc[t] = (t < kCoefRows * kCoefStride && t % kCoefStride == 0) ? v + add : v;
    }
    __syncthreads();
}

// Rates of the W window levels p..p+W-1 (0 past level Z-1: padded rows).
template <class P, int W>
__device__ __forceinline__ void window_rates(const double *sc, int p, const Field &f, bool has_poly,
                                             typename P::real (&x)[W])
{
    static_for<0, W>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        x[s] = RateEval<P>::x_of(sc + (p + s) * kCoefStride, f, has_poly);
    });
}

// ---------------------------------------------------------------------------
// ionize_step, compact layout: pops[(W+1)][n], slot s = level lo + s.
// Grid-stride loop, software pipelined: the loads of a lane's next cell are
// issued before the current cell is computed, so their latency overlaps the
// arithmetic.
template <class R, int W>
struct CellLoad {
    R E;
    R N[W + 1];
    uint8_t lo;
};

template <class R, int W>
__device__ __forceinline__ void load_cell(CellLoad<R, W> &d, const R *__restrict__ E, const R *__restrict__ pops,
                                          const uint8_t *__restrict__ lo, int64_t n, int64_t c)
{
    d.E = E[c];
    static_for<0, W + 1>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        d.N[s] = pops[(int64_t)s * n + c];
    });
    d.lo = lo[c];
}

// One cell of a compact-layout step from its loaded data: window shift,
// rates, exact chain update; the new window in o / olo.  Called by all
// active lanes of a wavefront together (the fast path and the solver use
// wavefront votes).
template <class P, int W>
__device__ __forceinline__ void step_cell_out(const CellLoad<typename P::real, W> &cur, const double *sc,
                                              const double *slog, int Z, bool has_poly, double eps, double E_cut,
                                              typename P::real (&o)[W + 1], int &olo)
{
    using R = typename P::real;
    const double EL = fabs((double)cur.E);
    int p = cur.lo;
    p = p < Z ? p : Z;
    // T = I for the whole wavefront: every cell is either fully stripped
    // (window [Z, Z], no rate) or below the field cutoff with no shift due
    if (__all(p >= Z || (EL < E_cut && (double)cur.N[0] >= eps))) {
        static_for<0, W + 1>([&](auto ss) { o[decltype(ss)::value] = cur.N[decltype(ss)::value]; });
        olo = p;
        return;
    }
    double N[W + 1];
    static_for<0, W + 1>([&](auto ss) { N[decltype(ss)::value] = (double)cur.N[decltype(ss)::value]; });
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
    const Field f = field_terms<RateEval<P>::kLogTerms>(EL, slog);
    R x[W];
    window_rates<P, W>(sc, p, f, has_poly, x);
    double out[W + 1];
    chain_apply<P, W>(x, N, out);
    const bool finite = EL <= 1.7976931348623157e308 || p >= Z;  // no rate when stripped
    static_for<0, W + 1>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        // slots past level Z hold no population (rounding of the top row);
        // a non-finite field makes the whole window NaN
        const R v = finite ? (R)out[s] : R(NAN);
        o[s] = (p + s <= Z) ? v : R(0);
    });
    olo = p;
}

template <class P, int W>
__device__ __forceinline__ void step_cell(const CellLoad<typename P::real, W> &cur, const double *sc,
                                          const double *slog, int Z, bool has_poly, double eps, double E_cut,
                                          typename P::real *__restrict__ pops, uint8_t *__restrict__ lo, int64_t n,
                                          int64_t c)
{
    typename P::real o[W + 1];
    int l;
    step_cell_out<P, W>(cur, sc, slog, Z, has_poly, eps, E_cut, o, l);
    static_for<0, W + 1>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        pops[(int64_t)s * n + c] = o[s];
    });
    lo[c] = (uint8_t)l;
}

// A wavefront whose 64 cells all take T = I (fully stripped, or below the
// field cutoff with no shift due) stores nothing: its windows are unchanged
// in place.  Grid-stride loop, software pipelined: the loads of a lane's
// next cell are issued before the current cell is computed, so their
// latency overlaps the arithmetic.
//
// With YIELD the kernel also writes the cell's electron yield of the step,
// dne[c] = sum_s (lo' + s) N'_s - sum_s (lo + s) N_s: the change of the mean
// charge (electrons released per atom), from the same registers.
template <class P, int W, bool YIELD>
__global__ __launch_bounds__(kBlock) void step_compact_kernel(StepArgs a, WinCut wc, ChunkOrder ord,
                                                              const typename P::real *__restrict__ E,
                                                              typename P::real *__restrict__ pops,
                                                              uint8_t *__restrict__ lo, int64_t n,
                                                              typename P::real *__restrict__ dne)
{
    using R = typename P::real;
    __shared__ double sc[kDevTableLen];
    __shared__ float scut[ADK_MAX_Z + 1];
    const double *slog = sc + kCoefRows * kCoefStride;
    const int Z = a.Z;
    for (int t = threadIdx.x; t <= ADK_MAX_Z; t += kBlock) scut[t] = wc.e[t];  // visible after the staging barrier
    // workgroup b takes chunks b, b + grid, ... of kBlock cells, each mapped
    // to a scattered place of the mesh (ChunkOrder)
    const int64_t nv = (n + kBlock - 1) / kBlock;
    int64_t v = blockIdx.x;
    int64_t c = chunk_place(v, ord) * kBlock + threadIdx.x;
    CellLoad<R, W> nxt;
    if (v < nv && c < n) load_cell(nxt, E, pops, lo, n, c);  // in flight while the table is staged
    stage_coefficients(sc, a.tab, a.ln_dt);
    for (; v < nv; v += gridDim.x) {
        const int64_t vn = v + gridDim.x;
        const int64_t cn = vn < nv ? chunk_place(vn, ord) * kBlock + threadIdx.x : n;
        const CellLoad<R, W> cur = nxt;
        if (cn < n) load_cell(nxt, E, pops, lo, n, cn);
        const int64_t cc = c;
        c = cn;
        if (cc >= n) continue;
        const int p = cur.lo < Z ? cur.lo : Z;
        const double ecut = p < Z ? (double)scut[p] : 0.0;
        if (__all(p >= Z || (fabs((double)cur.E) < ecut && (double)cur.N[0] >= a.eps))) {
            if (p != cur.lo) lo[cc] = (uint8_t)p;  // an index past Z is clamped
            if (YIELD) dne[cc] = R(0);
            continue;
        }
        R o[W + 1];
        int l;
        step_cell_out<P, W>(cur, sc, slog, Z, a.has_poly != 0, a.eps, ecut, o, l);
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            pops[(int64_t)s * n + cc] = o[s];
        });
        lo[cc] = (uint8_t)l;
        if (YIELD) {
            double q0 = 0.0, q1 = 0.0;
            static_for<0, W + 1>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                q0 = fma((double)(p + s), (double)cur.N[s], q0);
                q1 = fma((double)(l + s), (double)o[s], q1);
            });
            dne[cc] = (R)(q1 - q0);
        }
    }
}

// ionize_step, full layout: pops[(Z+1)][n], row k = level k.
template <class P, int W>
__global__ __launch_bounds__(kBlock) void step_full_kernel(StepArgs a, WinCut wc, const typename P::real *__restrict__ E,
                                                           typename P::real *__restrict__ pops,
                                                           uint8_t *__restrict__ lo, int64_t n)
{
    using R = typename P::real;
    __shared__ double sc[kDevTableLen];
    __shared__ float scut[ADK_MAX_Z + 1];
    const double *slog = sc + kCoefRows * kCoefStride;
    for (int t = threadIdx.x; t <= ADK_MAX_Z; t += kBlock) scut[t] = wc.e[t];  // visible after the staging barrier
    stage_coefficients(sc, a.tab, a.ln_dt);
    const int Z = a.Z;
    const bool has_poly = a.has_poly != 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += stride) {
        const double EL = fabs((double)E[c]);
        int p = lo[c];
        p = p < Z ? p : Z;
        const int p0 = p;
        double N[W + 1];
        N[0] = (double)pops[(int64_t)p * n + c];
        while (p < Z && N[0] < a.eps) {
            N[0] += (double)pops[(int64_t)(p + 1) * n + c];
            ++p;
        }
        static_for<1, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            N[s] = (p + s <= Z) ? (double)pops[(int64_t)(p + s) * n + c] : 0.0;
        });
        double out[W + 1];
        // the compact kernel's identity test (window under its identity
        // field, no shift due), so both layouts take the same path
        if (__all(p0 >= Z || (EL < (double)scut[p0] && p == p0))) {
            static_for<0, W + 1>([&](auto ss) { out[decltype(ss)::value] = N[decltype(ss)::value]; });
        } else {
            const Field f = field_terms<RateEval<P>::kLogTerms>(EL, slog);
            R x[W];
            window_rates<P, W>(sc, p, f, has_poly, x);
            chain_apply<P, W>(x, N, out);
        }
        const bool finite = EL <= 1.7976931348623157e308 || p >= Z;  // no rate when stripped
        for (int k = p0; k < p; ++k) pops[(int64_t)k * n + c] = R(0);
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            if (p + s <= Z) pops[(int64_t)(p + s) * n + c] = finite ? (R)out[s] : R(NAN);
        });
        lo[c] = (uint8_t)p;
    }
}

// Comparison baseline (not the method): the same step with the chain
// integrated by nsub explicit classical Runge-Kutta (RK4) substeps of
// dt / nsub instead of the analytic solution, rates frozen over the step as
// in the analytic method.  This is the sub-cycled ("fractional") time
// stepping that the exact solution avoids.  FP64, compact layout.
template <int W>
__device__ __forceinline__ void chain_deriv(const double (&x)[W], const double (&y)[W + 1], double (&d)[W + 1])
{
    d[0] = -x[0] * y[0];
    static_for<1, W>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        d[j] = fma(x[j - 1], y[j - 1], -x[j] * y[j]);
    });
    d[W] = x[W - 1] * y[W - 1];
}

template <int W>
__global__ __launch_bounds__(kBlock) void subcycle_kernel(StepArgs a, const double *__restrict__ E,
                                                          double *__restrict__ pops, uint8_t *__restrict__ lo,
                                                          int64_t n, int nsub)
{
    __shared__ double sc[kDevTableLen];
    const double *slog = sc + kCoefRows * kCoefStride;
    stage_coefficients(sc, a.tab, a.ln_dt);
    const int Z = a.Z;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const double h = 1.0 / nsub;  // substep in units of dt (x = W dt)
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += stride) {
        const double EL = fabs(E[c]);
        int p = lo[c];
        p = p < Z ? p : Z;
        double y[W + 1];
        static_for<0, W + 1>([&](auto ss) { y[decltype(ss)::value] = pops[(int64_t)decltype(ss)::value * n + c]; });
        while (p < Z && y[0] < a.eps) {
            y[0] += y[1];
            static_for<1, W>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                y[s] = y[s + 1];
            });
            y[W] = 0.0;
            ++p;
        }
        const Field f = field_terms<RateEval<PolicyF64>::kLogTerms>(EL, slog);
        double x[W];
        window_rates<PolicyF64, W>(sc, p, f, a.has_poly != 0, x);
        for (int it = 0; it < nsub; ++it) {
            double k1[W + 1], k2[W + 1], k3[W + 1], k4[W + 1], t[W + 1];
            chain_deriv<W>(x, y, k1);
            static_for<0, W + 1>([&](auto jj) { t[decltype(jj)::value] = fma(0.5 * h, k1[decltype(jj)::value], y[decltype(jj)::value]); });
            chain_deriv<W>(x, t, k2);
            static_for<0, W + 1>([&](auto jj) { t[decltype(jj)::value] = fma(0.5 * h, k2[decltype(jj)::value], y[decltype(jj)::value]); });
            chain_deriv<W>(x, t, k3);
            static_for<0, W + 1>([&](auto jj) { t[decltype(jj)::value] = fma(h, k3[decltype(jj)::value], y[decltype(jj)::value]); });
            chain_deriv<W>(x, t, k4);
            static_for<0, W + 1>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                y[j] += (h / 6.0) * (k1[j] + 2.0 * (k2[j] + k3[j]) + k4[j]);
            });
        }
        const bool finite = EL <= 1.7976931348623157e308 || p >= Z;
        static_for<0, W + 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            const double v = finite ? y[s] : NAN;
            pops[(int64_t)s * n + c] = (p + s <= Z) ? v : 0.0;
        });
        lo[c] = (uint8_t)p;
    }
}

template <int W>
hipError_t launch_subcycle(const adk_gas *g, const double *E, int64_t n, double dt, double *pops, uint8_t *lo,
                           double eps, int nsub, hipStream_t st)
{
    const StepArgs a = step_args(g, dt, eps);
    hipLaunchKernelGGL((subcycle_kernel<W>), dim3(grid_for(n)), dim3(kBlock), 0, st, a, E, pops, lo, n, nsub);
    return hipGetLastError();
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
            v = v < (double)kXMax<R> ? v : (v == v ? (double)kXMax<R> : v);
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

// Rates W_out[j][i] = W_{k0+j}(E[i]) in 1/s (table staged with ln dt = 0,
// evaluated in double and rounded to the output type).
template <class P>
__global__ __launch_bounds__(kBlock) void rates_kernel(StepArgs a, int k0, int nk,
                                                       const typename P::real *__restrict__ E,
                                                       typename P::real *__restrict__ Wout, int64_t n)
{
    __shared__ double sc[kDevTableLen];
    const double *slog = sc + kCoefRows * kCoefStride;
    stage_coefficients(sc, a.tab, 0.0);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double EL = fabs((double)E[i]);
        const Field f = field_terms<7>(EL, slog);
        const bool finite = EL <= 1.7976931348623157e308;
        for (int j = 0; j < nk; ++j) {
            const double *row = sc + (k0 + j) * kCoefStride;
            double x = exp2(rate_exponent2(row, f));
            if (a.has_poly) x *= mavg_poly(row, f);
            Wout[(int64_t)j * n + i] = (typename P::real)(finite ? x : NAN);
        }
    }
}

// Launch helpers (one instantiation per precision and window width).
int num_cus();
int grid_for(int64_t n);
StepArgs step_args(const adk_gas *g, double dt, double eps);

// Grid of a grid-stride kernel: every workgroup resident at once (occupancy
// from the compiled resource usage), no more groups than cells need.
// (The occupancy is cached per kernel: the template parameter is the kernel
// itself, so kernels of one signature do not share the cache.)
//
// With chunks_per_group > 0 the grid grows beyond the resident slots to about
// that many kBlock-cell chunks per workgroup: the surplus workgroups start as
// earlier ones retire, so a CU whose chunks happened to hold the expensive
// (ionizing) cells takes fewer of them, while each workgroup still loops over
// several chunks (one-ahead prefetch, table staged once per chunk run).
template <auto Kernel>
int resident_grid(int64_t n, int64_t chunks_per_group = 0)
{
    static int per_cu = 0;
    if (per_cu <= 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, Kernel, kBlock, 0) != hipSuccess || b <= 0) b = 4;
        per_cu = b;
    }
    const int64_t need = (n + kBlock - 1) / kBlock;
    int64_t grid = (int64_t)num_cus() * per_cu;
    if (chunks_per_group > 0) {
        int64_t spread = (need + chunks_per_group - 1) / chunks_per_group;
        spread = spread < ((int64_t)1 << 30) ? spread : ((int64_t)1 << 30);  // grid-stride covers the rest
        grid = spread > grid ? spread : grid;
    }
    return (int)(need < grid ? need : grid);
}

// Chunks per workgroup of the compact step kernel.  Measured on the 3D laser
// mesh (33.5M cells = 131,072 chunks, 2048 resident workgroups): all resident
// (64 chunks each) 273 us per step (mixed) / 566 us (FP64); 32 chunks 266 /
// 521; 16 chunks 249 / 525; 8 chunks 244 / 517; 4 chunks 250 / 533; one chunk
// per workgroup 318 / 648.  Meshes of up to 8 x resident chunks (the 1M-cell
// 2D mesh) keep the resident grid.
constexpr int64_t kStepChunksPerGroup = 8;

template <class P, int W>
hipError_t launch_step(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                       const adk_window *win, void *dne, hipStream_t st)
{
    using R = typename P::real;
    const StepArgs a = step_args(g, dt, win->eps);
    const WinCut wc = window_cutoffs(g, dt, W);
    if (win->layout == ADK_LAYOUT_COMPACT) {
        if (dne) {
            const int grid = resident_grid<step_compact_kernel<P, W, true>>(n, kStepChunksPerGroup);
            hipLaunchKernelGGL((step_compact_kernel<P, W, true>), dim3(grid), dim3(kBlock), 0, st, a, wc,
                               chunk_order(n), (const R *)E, (R *)pops, lo, n, (R *)dne);
        } else {
            const int grid = resident_grid<step_compact_kernel<P, W, false>>(n, kStepChunksPerGroup);
            hipLaunchKernelGGL((step_compact_kernel<P, W, false>), dim3(grid), dim3(kBlock), 0, st, a, wc,
                               chunk_order(n), (const R *)E, (R *)pops, lo, n, (R *)nullptr);
        }
    } else {
        const int grid = resident_grid<step_full_kernel<P, W>>(n);
        hipLaunchKernelGGL((step_full_kernel<P, W>), dim3(grid), dim3(kBlock), 0, st, a, wc, (const R *)E,
                           (R *)pops, lo, n);
    }
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
                              const adk_window *, void *, hipStream_t);
using AdvanceFn = hipError_t (*)(const void *, int64_t, double, void *, hipStream_t);

}  // namespace adk

// Non-template entry of each instantiation: adk_step_<prec>_<W>, adk_advance_<prec>_<W>.
#define ADK_DECLARE_INST(PREC, W)                                                                          \
    hipError_t adk_step_##PREC##_##W(const adk_gas *, const void *, int64_t, double, void *, uint8_t *,    \
                                     const adk_window *, void *, hipStream_t);                             \
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

// ionize_step for windows wider than ADK_MAX_W (wide.hip).
hipError_t adk_step_wide(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                         const adk_window *win, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched step over cells of several gases and window widths (plan).
// Cells are grouped by (gas, w) on the host; a tile is up to CPL*kBlock cells
// of one group, listed through a permutation of the cell index.  The widths
// of a plan are split into launch groups, each served by one launch of the
// kernel compiled for the group's widest window (its register budget, and so
// the waves a SIMD can hold, is that of the widest solver it contains).  One
// workgroup per tile, tiles in the host's order (heaviest first): the
// hardware dispatcher balances the load, with no device-wide counter (an
// atomic on one address from every workgroup serialises across the chip).
namespace adk {

constexpr int kPlanMaxGas = 8;
constexpr int kPlanMaxW = 6;

struct PlanGasArgs {
    const double *tab;
    int Z;
    int has_poly;
    double E_cut;
};

struct PlanArgs {
    PlanGasArgs gas[kPlanMaxGas];
    double ln_dt;
    double eps;
    int t0;      // first tile of the launch group
    int ntiles;  // tiles of the launch group
};

struct PlanTile {
    int32_t gas, w, start, count;
};

// A tile of one (gas, w) group: the gas table is staged while the first
// cells' loads are in flight; each lane then walks its CPL cells with the
// next cell's loads issued before the current one is computed.  A
// wavefront whose cells all take T = I stores nothing (as ionize_step).
template <class P, int W, int CPL>
__device__ __forceinline__ void plan_tile(const PlanTile &tile, const PlanGasArgs &g, double ln_dt, double eps,
                                          double *sc, const typename P::real *__restrict__ E,
                                          typename P::real *__restrict__ pops, uint8_t *__restrict__ lo, int64_t n,
                                          const int32_t *__restrict__ perm)
{
    using R = typename P::real;
    const double *slog = sc + kCoefRows * kCoefStride;
    const int end = tile.start + tile.count;
    int idx = tile.start + (int)threadIdx.x;
    CellLoad<R, W> nxt;
    int64_t cn = 0;
    if (idx < end) {
        cn = perm ? perm[idx] : idx;  // no permutation: the plan's own cell order
        load_cell(nxt, E, pops, lo, n, cn);
    }
    stage_coefficients(sc, g.tab, ln_dt);
    static_for<0, CPL>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if (idx < end) {
            const CellLoad<R, W> cur = nxt;
            const int64_t c = cn;
            if constexpr (k + 1 < CPL) {
                if (idx + kBlock < end) {
                    cn = perm ? perm[idx + kBlock] : idx + kBlock;
                    load_cell(nxt, E, pops, lo, n, cn);
                }
            }
            const int p = cur.lo < g.Z ? cur.lo : g.Z;
            if (__all(p >= g.Z || (fabs((double)cur.E) < g.E_cut && (double)cur.N[0] >= eps))) {
                if (p != cur.lo) lo[c] = (uint8_t)p;  // an index past Z is clamped
            } else {
                step_cell<P, W>(cur, sc, slog, g.Z, g.has_poly != 0, eps, g.E_cut, pops, lo, n, c);
            }
        }
        idx += kBlock;
    });
}

// Tiles of widths 1..WMAX (the host never hands a wider tile to it);
// workgroup b takes tile t0 + b.
template <class P, int WMAX, int CPL>
__global__ __launch_bounds__(kBlock) void plan_kernel(PlanArgs a, const typename P::real *__restrict__ E,
                                                      typename P::real *__restrict__ pops,
                                                      uint8_t *__restrict__ lo, int64_t n,
                                                      const int32_t *__restrict__ perm,
                                                      const PlanTile *__restrict__ tiles)
{
    __shared__ double sc[kDevTableLen];
    if ((int)blockIdx.x >= a.ntiles) return;
    const PlanTile tile = tiles[a.t0 + (int)blockIdx.x];
    // uniform selection (a dynamic index into the argument block would put
    // it in scratch memory)
    PlanGasArgs g = a.gas[0];
    static_for<1, kPlanMaxGas>([&](auto kk) {
        if (tile.gas == decltype(kk)::value) g = a.gas[decltype(kk)::value];
    });
    if constexpr (WMAX == 1) {
        plan_tile<P, 1, CPL>(tile, g, a.ln_dt, a.eps, sc, E, pops, lo, n, perm);
    } else {
        static_for<1, WMAX + 1>([&](auto ww) {
            constexpr int w = decltype(ww)::value;
            if (tile.w == w) plan_tile<P, w, CPL>(tile, g, a.ln_dt, a.eps, sc, E, pops, lo, n, perm);
        });
    }
}

template <class P, int WMAX, int CPL>
hipError_t launch_plan(const PlanArgs &a, const void *E, void *pops, uint8_t *lo, int64_t n, const int32_t *perm,
                       const PlanTile *tiles, hipStream_t st)
{
    using R = typename P::real;
    hipLaunchKernelGGL((plan_kernel<P, WMAX, CPL>), dim3(a.ntiles), dim3(kBlock), 0, st, a, (const R *)E,
                       (R *)pops, lo, n, perm, tiles);
    return hipGetLastError();
}

using PlanLaunchFn = hipError_t (*)(const PlanArgs &, const void *, void *, uint8_t *, int64_t, const int32_t *,
                                    const PlanTile *, hipStream_t);

}  // namespace adk

// adk_plan_launch_<prec>_<wmax>_<cpl>
#define ADK_DECLARE_PLAN_CPL(PREC, WMAX, CPL)                                                              \
    hipError_t adk_plan_launch_##PREC##_##WMAX##_##CPL(const adk::PlanArgs &, const void *, void *,        \
                                                       uint8_t *, int64_t, const int32_t *,                \
                                                       const adk::PlanTile *, hipStream_t);
#define ADK_DECLARE_PLAN(PREC, WMAX)      \
    ADK_DECLARE_PLAN_CPL(PREC, WMAX, 1)   \
    ADK_DECLARE_PLAN_CPL(PREC, WMAX, 2)   \
    ADK_DECLARE_PLAN_CPL(PREC, WMAX, 4)
#define ADK_DECLARE_PLAN_PREC(PREC) \
    ADK_DECLARE_PLAN(PREC, 1)       \
    ADK_DECLARE_PLAN(PREC, 2)       \
    ADK_DECLARE_PLAN(PREC, 3)       \
    ADK_DECLARE_PLAN(PREC, 4)       \
    ADK_DECLARE_PLAN(PREC, 5)       \
    ADK_DECLARE_PLAN(PREC, 6)
ADK_DECLARE_PLAN_PREC(f64)
ADK_DECLARE_PLAN_PREC(mixed)
