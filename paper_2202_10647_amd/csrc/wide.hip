// Wide windows (9 <= w <= 63 rates, up to the whole chain): one wavefront
// per cell; the shared device code (rate ranking, the sorted Newton table,
// the hole recurrence) is in wide.hpp.
#include "wide.hpp"

namespace adk {
namespace {

// One cell, all 64 lanes.  LDS: s, e, mm (sorted rate, e^{-s}, max(1, s)),
// Nb (window populations), cid (chain index of a sorted position), pos (sorted
// position of a chain index), D (triangular table), V (one column per lane).
template <class R>
__device__ void wide_cell(const StepArgs &a, int W, bool full, int64_t c,
                          double EL, int p0, const R *__restrict__ E, R *__restrict__ pops,
                          uint8_t *__restrict__ lo, int64_t n, double *s, double *e, double *mm, double *Nb,
                          int *cid, int *pos, double *D, double *V)
{
    (void)E;
    const int lane = wide_lane();
    const int Z = a.Z;
    wave_sync();  // the previous cell's reads of LDS are done
    double Ns = 0.0;
    if (lane <= W) {
        if (full) {
            const int lev = p0 + lane;
            Ns = lev <= Z ? (double)pops[(int64_t)lev * n + c] : 0.0;
        } else {
            Ns = (double)pops[(int64_t)lane * n + c];
        }
    }
    // window shift at the start of the step; the residual folds upward
    int p = p0;
    while (p < Z && __shfl(Ns, 0) < a.eps) {
        const double up = __shfl_down(Ns, 1);
        Ns = lane == 0 ? Ns + up : (lane < W ? up : 0.0);
        ++p;
    }
    const bool finite = EL <= 1.7976931348623157e308 || p >= Z;
    double out = Ns;
    if (finite && p < Z) {
        const Field f = field_terms<RateEval<PolicyF64>::kLogTerms>(EL, a.tab + kCoefRows * kCoefStride);
        double x = 0.0;
        const int lev = p + lane;
        if (lane < W && lev < Z) {
            double row[kCoefStride];
            for (int k = 0; k < kCoefStride; ++k) row[k] = a.tab[lev * kCoefStride + k];
            row[0] += a.ln_dt * kLog2e;  // the fold of ln dt that staging applies
            x = RateEval<PolicyF64>::x_of(row, f, a.has_poly != 0);
        }
        // Only slots [q_lo, top] change by more than 1e-30.  q_lo, q_hi: the
        // lowest and highest slot holding at least 1e-30; slot j can receive
        // at most sum_i N_i prod_{k=i}^{j-1} x_k / (j-i)! (g <= 1/n!), so the
        // last slot K reached by a term of 1e-30 or more bounds the flow, and
        // slot K+1, made absorbing, takes the (negligible) rest.
        const bool sig = lane <= W && !(fabs(Ns) < kWideNegligible);
        const unsigned long long pop = __ballot(sig);
        if (pop) {
            const int q_lo = __ffsll((long long)pop) - 1;
            const int q_hi = 63 - __clzll((long long)pop);
            double *lx = V, *lnN = V + (W + 1);  // scratch before the solve (slots 0..W)
            if (lane <= W) {
                lx[lane] = lane < W ? log(x) : -INFINITY;
                lnN[lane] = sig ? log(fabs(Ns)) : -INFINITY;
            }
            wave_sync();
            bool reach = false;
            if (lane >= q_lo && lane <= W) {
                double best = lnN[lane], path = 0.0;
                for (int i = lane - 1; i >= q_lo && path > -INFINITY; --i) {
                    path += lx[i];
                    best = fmax(best, lnN[i] + path - kLogFact.v[lane - i]);
                }
                reach = best >= kWideNegligibleLog;
            }
            const unsigned long long rb = __ballot(reach);
            const int K = max(q_hi, 63 - __clzll((long long)(rb | 1ull)));
            const int top = min(W, K + 1);
            const int Wp = top - q_lo;  // rates of the sub-window
            wave_sync();
            if (Wp > 0) {
                const int src = lane + q_lo < 64 ? lane + q_lo : 63;
                const double xs = __shfl(x, src), Nsub = __shfl(Ns, src);
                const double r =
                    chain_sub<true>(Wp, lane < Wp ? xs : 0.0, lane <= Wp ? Nsub : 0.0, to_lds(s), to_lds(e), to_lds(mm),
                                    to_lds(Nb), to_lds(cid), to_lds(pos), to_lds(D), to_lds(V), W);
                const double back = __shfl(r, lane - q_lo >= 0 ? lane - q_lo : 0);
                if (lane >= q_lo && lane <= top) out = back;
            }
        }
    }
    if (lane <= W) {
        const int lev = p + lane;
        const double v = finite ? out : (double)NAN;
        if (full) {
            if (lev <= Z) pops[(int64_t)lev * n + c] = (R)v;
        } else {
            pops[(int64_t)lane * n + c] = lev <= Z ? (R)v : R(0);
        }
    }
    // full layout: levels below the new window are empty
    if (full && lane < p - p0) pops[(int64_t)(p0 + lane) * n + c] = R(0);
    if (lane == 0) lo[c] = (uint8_t)p;
}

template <class R>
// Four wavefronts per SIMD where LDS allows it (windows up to about 20
// rates); the register cap spills a few registers.
__global__ __launch_bounds__(kWideBlock, 4) void wide_step_kernel(StepArgs a, int W, int full, const R *__restrict__ E,
                                                               R *__restrict__ pops, uint8_t *__restrict__ lo,
                                                               int64_t n)
{
    extern __shared__ __align__(16) double wl[];
    int *cid = (int *)(wl + 256);
    int *pos = cid + 64;  // followed by 64 doubles of log rates (chain_sub)
    double *D = wl + 384;
    double *V = D + W * (W + 1) / 2;
    const int lane = wide_lane();
    const int Z = a.Z;
    for (int64_t base = (int64_t)blockIdx.x * kWideBlock; base < n; base += (int64_t)gridDim.x * kWideBlock) {
        // lane-per-cell test: fully stripped, or below the field cutoff with
        // no shift due (T = I): only an index past Z is clamped
        const int64_t c0 = base + lane;
        const bool valid = c0 < n;
        int p0 = Z, l0 = 0;
        double EL0 = 0.0, N00 = 0.0;
        if (valid) {
            EL0 = fabs((double)E[c0]);
            l0 = lo[c0];
            p0 = l0 < Z ? l0 : Z;
            N00 = (double)pops[(full ? (int64_t)p0 : 0) * n + c0];
        }
        const bool ident = !valid || p0 >= Z || (EL0 < a.E_cut && N00 >= a.eps);
        if (valid && ident && p0 != l0) lo[c0] = (uint8_t)p0;
        unsigned long long todo = __ballot(!ident);
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const double EL = __shfl(EL0, src);
            const int p = __shfl(p0, src);
            wide_cell<R>(a, W, full != 0, base + src, EL, p, E, pops, lo, n, wl, wl + 64, wl + 128, wl + 192, cid,
                         pos, D, V);
        }
    }
}

template <class R>
hipError_t launch_wide(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                       const adk_window *win, hipStream_t st)
{
    const StepArgs a = step_args(g, dt, win->eps);
    const int W = win->w;
    const size_t dyn = sizeof(double) * wide_wave_doubles(W, true);
    static int per_cu[ADK_MAX_WIDE_W + 1] = {};  // occupancy per width (LDS grows with W)
    int b = per_cu[W];
    if (b <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, wide_step_kernel<R>, kWideBlock, dyn) != hipSuccess ||
            b <= 0)
            b = 1;
        per_cu[W] = b;
    }
    const int64_t need = (n + kWideBlock - 1) / kWideBlock;
    const int64_t cap = (int64_t)num_cus() * b;
    const int grid = (int)(need < cap ? need : cap);
    hipLaunchKernelGGL(wide_step_kernel<R>, dim3(grid), dim3(kWideBlock), dyn, st, a, W,
                       win->layout == ADK_LAYOUT_FULL ? 1 : 0, (const R *)E, (R *)pops, lo, n);
    return hipGetLastError();
}

// Chain advance with given rates W[w][n] (1/s) for windows wider than the
// lane-per-cell path: one wavefront per cell, the same solution (chain_sub),
// no window shift.
template <class R>
__global__ __launch_bounds__(kWideBlock) void wide_advance_kernel(int W, const R *__restrict__ Wr, double dt,
                                                                  R *__restrict__ pops, int64_t n)
{
    extern __shared__ __align__(16) double wl[];
    int *cid = (int *)(wl + 256);
    int *pos = cid + 64;
    double *D = wl + 384;
    double *V = D + W * (W + 1) / 2;
    const int lane = wide_lane();
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        wave_sync();  // the previous cell's reads of LDS are done
        double x = 0.0;
        if (lane < W) {
            const double v = (double)Wr[(int64_t)lane * n + c] * dt;
            x = v < (double)kXMax<R> ? v : (v == v ? (double)kXMax<R> : v);
        }
        const double Nk = lane <= W ? (double)pops[(int64_t)lane * n + c] : 0.0;
        const double r = chain_sub<false>(W, x, Nk, to_lds(wl), to_lds(wl + 64), to_lds(wl + 128), to_lds(wl + 192),
                                          to_lds(cid), to_lds(pos), to_lds(D), to_lds(V), W);
        if (lane <= W) pops[(int64_t)lane * n + c] = (R)r;
    }
}

template <class R>
hipError_t launch_wide_advance(int W, const void *Wr, int64_t n, double dt, void *pops, hipStream_t st)
{
    const size_t dyn = sizeof(double) * wide_wave_doubles(W, false);
    static int per_cu[ADK_MAX_WIDE_W + 1] = {};
    int b = per_cu[W];
    if (b <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, wide_advance_kernel<R>, kWideBlock, dyn) !=
                hipSuccess ||
            b <= 0)
            b = 1;
        per_cu[W] = b;
    }
    const int64_t cap = (int64_t)num_cus() * b;
    const int grid = (int)(n < cap ? n : cap);
    hipLaunchKernelGGL(wide_advance_kernel<R>, dim3(grid), dim3(kWideBlock), dyn, st, W, (const R *)Wr, dt,
                       (R *)pops, n);
    return hipGetLastError();
}

}  // namespace
}  // namespace adk

hipError_t adk_advance_wide(int w, const void *Wr, int64_t n, double dt, void *pops, adk_prec prec, hipStream_t st)
{
    return prec == ADK_F64 ? adk::launch_wide_advance<double>(w, Wr, n, dt, pops, st)
                           : adk::launch_wide_advance<float>(w, Wr, n, dt, pops, st);
}

hipError_t adk_step_wide(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                         const adk_window *win, hipStream_t st)
{
    return win->prec == ADK_F64 ? adk::launch_wide<double>(g, E, n, dt, pops, lo, win, st)
                                : adk::launch_wide<float>(g, E, n, dt, pops, lo, win, st);
}
