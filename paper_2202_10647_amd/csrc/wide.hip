// Wide windows (9 <= w <= 63 rates, up to the whole chain): one wavefront
// per cell.
//
// A window this wide does not fit the per-lane register tables of the
// narrow path, so the 64 lanes of a wavefront share one cell.  The step is
// the same (shift at the start, rates of Eq. (1) frozen over dt, exact
// solution of the chain, Sec. 3); the transition entries
//     T[j][i] = (x_i ... x_{j-1}) g(x_i, ..., x_j)
// (g the sign-adjusted divided difference of e^{-x}) come from one table over
// the sorted rates instead of one table per chain range:
//   * the rates are ranked (lane k holds x_k), and the scaled Newton table
//     ghat[a][b] = g(s_a..s_b) prod_{a<k<=b} max(1, s_k) of the sorted points
//     is built one diagonal per step in LDS, a diagonal entry per lane; an
//     entry whose spread is below the threshold of its order comes from the
//     Taylor series of the divided difference about its smallest point
//     (McCurdy, Ng and Parlett 1984);
//   * a chain range [i..j] is a subset of the sorted points.  Its hull
//     [a..b] in sorted order (a, b: positions of its smallest and largest
//     rate) may contain holes (rates of levels outside the range).  With a
//     the smallest point and h > a a hole, the identity
//         g(S) = g(S - {a} + {h}) + (s_h - s_a) g(S + {h})
//     fills holes one at a time, smallest last; both sets on the right have
//     one hole less, and the sets reached form a triangle over (start, holes
//     filled), so g(S) costs (holes + 1)^2 / 2 fused steps from the entries
//     ghat[a+t][b].  Every term is non-negative: nothing cancels.  In scaled
//     form, V_t <- (V_{t+1} m_{a+t+1} + (s_h - s_{a+t}) V_t) / m_h.
//   * lane j accumulates row j, N'_j = sum_i T[j][i] N_i; the top slot takes
//     what the rows leave (conservation).
// All arithmetic is double; populations are stored in the precision's type.
//
// LDS bounds how many of these latency-bound wavefronts a CU holds, so it
// goes to the cells only: each wavefront (one per workgroup) has its region
// (sorted rates, the triangular table, and the per-lane columns of the hole
// recurrence, W - 1 entries for each of the W lanes that use them), and the
// rate coefficients and the log2 table, read once per cell, come from the
// gas's device table through the caches instead of being staged.
#include "kernels.hpp"

namespace adk {
namespace {

constexpr int kWideBlock = 64;  // one wavefront per workgroup

__device__ __forceinline__ int wide_lane() { return threadIdx.x; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int tri(int a, int b) { return b * (b + 1) / 2 + a; }

// Newton below this spread for an entry of n + 1 points (FP64 accuracy; the
// rounding of the recurrence grows ~ n / spread per order).
__device__ __forceinline__ double wide_delta(int n)
{
    return n == 1 ? 0.1 : (n <= 3 ? 0.5 : (n <= 5 ? 1.0 : (n <= 7 ? 1.5 : 2.0)));
}

constexpr int kTaylorMaxTerms = 120;
constexpr double kWideNegligible = 1e-30;  // populations and transfers below this are left out
constexpr double kWideNegligibleLog = -69.07755278982137;  // log(1e-30)

struct LogFactTable {
    double v[64];
    constexpr LogFactTable() : v()
    {
        // log k! by summing log k in double at compile time would need a
        // constexpr log; store ln k! from the factorial table instead
        double f = 1.0;
        v[0] = 0.0;
        for (int k = 1; k < 64; ++k) {
            f *= (double)k;
            v[k] = ln_constexpr(f);
        }
    }
    static constexpr double ln_constexpr(double x)
    {
        // x = 2^e * m, m in [1, 2): ln x = e ln 2 + ln m, ln m from the
        // atanh series of (m - 1) / (m + 1) (|t| <= 1/3, 40 terms)
        int ex = 0;
        while (x >= 2.0) {
            x *= 0.5;
            ++ex;
        }
        const double t = (x - 1.0) / (x + 1.0), t2 = t * t;
        double sum = 0.0, pw = t;
        for (int k = 0; k < 40; ++k) {
            sum += pw / (2 * k + 1);
            pw *= t2;
        }
        return ex * 0.69314718055994530942 + 2.0 * sum;
    }
};
__constant__ inline constexpr LogFactTable kLogFact{};

struct InvFactLong {
    double v[192];  // 1/k!, 0 past the double range
    constexpr InvFactLong() : v()
    {
        v[0] = 1.0;
        for (int k = 1; k < 192; ++k) v[k] = v[k - 1] / (double)k;
    }
};
__constant__ inline constexpr InvFactLong kInvFactL{};

constexpr double kWideClusterSpread = 2.0;  // largest spread any order's threshold sends to the series

// Taylor series about s_a for every entry [a..a+k], k = 1..nmax, of lane a's
// row in one pass (the points s_{a+1..a+nmax} lie within kWideClusterSpread
// of s_a):  g(s_a..s_{a+k}) = e^{-s_a} sum_m (-1)^m h_m(y_1..y_k) / (k+m)!,
// y_t = s_{a+t} - s_a, where h_m(y_1..y_k) = y_k h_{m-1}(y_1..y_k) +
// h_m(y_1..y_{k-1}) builds every k from the one below in the same sweep.
// The partial sums accumulate in D[a][a+k] (written by this lane only), the
// h values in this lane's column of hv; on return D holds ghat.
__device__ void taylor_row(const double *s, const double *e, const double *mm, double *D, int a, int nmax,
                           double *hv, int lane, int vs)
{
    const double sa = s[a];
    for (int k = 1; k <= nmax; ++k) {
        hv[(k - 1) * vs + lane] = 1.0;
        D[tri(a, a + k)] = kInvFactL.v[k];
    }
    double sgn = 1.0;
    for (int m = 1; m < kTaylorMaxTerms; ++m) {
        sgn = -sgn;
        double prev = 0.0;  // h_m() of no variables is 0 for m >= 1
        bool conv = true;
        for (int k = 1; k <= nmax; ++k) {
            const double hk = fma(s[a + k] - sa, hv[(k - 1) * vs + lane], prev);
            hv[(k - 1) * vs + lane] = hk;
            prev = hk;
            const double term = sgn * hk * kInvFactL.v[k + m];
            const double acc = D[tri(a, a + k)] + term;
            D[tri(a, a + k)] = acc;
            conv = conv && !(fabs(term) > 1e-17 * acc);
        }
        if (conv) break;
    }
    const double ea = e[a];
    double scale = 1.0;
    for (int k = 1; k <= nmax; ++k) {
        scale *= mm[a + k];
        // e^{-s_a} underflowing makes the entry 0 (and the scale could be huge)
        D[tri(a, a + k)] = ea == 0.0 ? 0.0 : ea * D[tri(a, a + k)] * scale;
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    static_for<0, 6>([&](auto kk) { v += __shfl_xor(v, 1 << decltype(kk)::value); });
    return v;
}

// The exact update of a window of Wp rates held one per lane (x_k in lane k
// for k < Wp, N_k in lane k for k <= Wp; zero elsewhere): returns N'_k in
// lane k.  All 64 lanes call it together.  V: per-lane columns of the hole
// recurrence, entry t of lane k at V[t vs + k] (vs >= Wp, t <= Wp - 2).
__device__ double chain_sub(int Wp, double x, double Nk, double *s, double *e, double *mm, double *Nb, int *cid,
                            int *pos, double *D, double *V, int vs)
{
    double *ls = (double *)(pos + 64);  // log of the sorted rates
    const int lane = wide_lane();
    // rank of x_k among the window's rates (ties by chain index)
    int rank = 0;
    for (int k = 0; k < Wp; ++k) {
        const double xk = __shfl(x, k);
        rank += (xk < x || (xk == x && k < lane)) ? 1 : 0;
    }
    if (lane < Wp) {
        s[rank] = x;
        e[rank] = exp(-x);
        mm[rank] = fmax(1.0, x);
        ls[rank] = log(x);
        cid[rank] = lane;
        pos[lane] = rank;
    }
    if (lane <= Wp) Nb[lane] = Nk;
    wave_sync();
    // scaled Newton table of the sorted rates: the series for every entry
    // within kWideClusterSpread (one pass per row), then one order per step,
    // Newton where the spread reaches the order's threshold
    if (lane < Wp) {
        D[tri(lane, lane)] = e[lane];
        int nmax = 0;
        while (lane + nmax + 1 < Wp && s[lane + nmax + 1] - s[lane] < kWideClusterSpread) ++nmax;
        if (nmax > 0) taylor_row(s, e, mm, D, lane, nmax, V, lane, vs);
    }
    wave_sync();
    for (int ord = 1; ord < Wp; ++ord) {
        if (lane < Wp - ord) {
            const int lo_ = lane, hi = lane + ord;
            const double spread = s[hi] - s[lo_];
            if (spread >= wide_delta(ord))
                D[tri(lo_, hi)] =
                    PolicyF64::quot(fma(D[tri(lo_, hi - 1)], mm[hi], -D[tri(lo_ + 1, hi)] * mm[lo_ + 1]), spread);
        }
        wave_sync();
    }
    // row j = lane: N'_j = sum_{i <= j} T[j][i] N_i
    double acc = 0.0;
    if (lane < Wp) {
        const int j = lane;
        const double mj = fmax(1.0, x);
        double Rp = 1.0;  // prod_{k=i}^{j-1} min(x_k, 1)
        double lb = 0.0;  // log of prod_{k=i}^{j-1} x_k / (j-i)!, which bounds T[j][i] (g <= 1/n!)
        int A = pos[j], B = A;
        for (int i = j; i >= 0; --i) {
            const int pi = pos[i];
            if (i < j) {
                const double xi = s[pi];
                Rp *= fmin(xi, 1.0);
                if (Rp == 0.0) break;  // every lower source reaches row j through a zero rate
                lb += ls[pi] - kLogFact.v[j - i] + kLogFact.v[j - i - 1];  // log x_i - log (j-i)
            }
            A = min(A, pi);
            B = max(B, pi);
            const double Ni = Nb[i];
            // a source whose contribution is below 1e-30 is skipped (every
            // skipped term is bounded by N_i prod x / (j-i)!)
            if (Ni == 0.0 || fmin(lb, 0.0) + log(fabs(Ni)) < kWideNegligibleLog) continue;
            const int holes = (B - A + 1) - (j - i + 1);
            double G;
            if (holes == 0) {
                G = D[tri(A, B)];
            } else {
                for (int t = 0; t <= holes; ++t) V[t * vs + lane] = D[tri(A + t, B)];
                int cnt = holes;
                for (int q = B; q > A && cnt > 0; --q) {
                    const int ci = cid[q];
                    if (ci >= i && ci <= j) continue;
                    --cnt;
                    const double rh = 1.0 / mm[q];
                    const double sq = s[q];
                    double cur = V[lane];
                    for (int t = 0; t <= cnt; ++t) {
                        const double nxt = V[(t + 1) * vs + lane];
                        V[t * vs + lane] = fma(nxt, mm[A + t + 1], (sq - s[A + t]) * cur) * rh;
                        cur = nxt;
                    }
                }
                G = V[lane];
            }
            acc = fma(Rp * (mm[A] / mj) * G, Ni, acc);
        }
    }
    // the top slot keeps what the rows leave (columns of T sum to one)
    const double total = wave_sum(lane <= Wp ? Nk : 0.0);
    const double rows = wave_sum(lane < Wp ? acc : 0.0);
    const double top = fmax(total - rows, 0.0);
    wave_sync();  // LDS reads done before the next use
    return lane < Wp ? acc : (lane == Wp ? top : 0.0);
}

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
                const double r = chain_sub(Wp, lane < Wp ? xs : 0.0, lane <= Wp ? Nsub : 0.0, s, e, mm, Nb, cid,
                                           pos, D, V, W);
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

// Doubles of one wavefront's LDS region for width W: s, e, mm, Nb, cid and
// pos, log rates (384), the triangular table, and the per-lane columns
// ((W - 1) W >= 2 (W + 1), which also holds the scratch of the reach test).
constexpr size_t wide_wave_doubles(int W)
{
    return 384 + (size_t)W * (W + 1) / 2 + (size_t)(W - 1) * W;
}

template <class R>
__global__ __launch_bounds__(kWideBlock) void wide_step_kernel(StepArgs a, int W, int full, const R *__restrict__ E,
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
    const size_t dyn = sizeof(double) * wide_wave_doubles(W);
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

}  // namespace
}  // namespace adk

hipError_t adk_step_wide(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                         const adk_window *win, hipStream_t st)
{
    return win->prec == ADK_F64 ? adk::launch_wide<double>(g, E, n, dt, pops, lo, win, st)
                                : adk::launch_wide<float>(g, E, n, dt, pops, lo, win, st);
}
