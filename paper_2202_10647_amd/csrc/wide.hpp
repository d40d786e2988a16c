// Wide windows: one cell per wavefront, or per aligned group of 16 lanes
// (shared by the wide ionize_step path, adk_chain_advance and the adaptive
// window's wide tiers).
//
// A window this wide does not fit the per-lane register tables of the
// narrow path, so the lanes of a wavefront (or of a 16-lane group, for
// windows of up to 15 rates) share one cell.  The step is
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
// LDS bounds how many of these latency-bound cells a CU holds, so it goes to
// the cells only: each cell has its region (sorted rates, the triangular
// table, and the per-lane columns of the hole recurrence, W - 1 entries for
// each of the W lanes that use them), and the rate coefficients and the log2
// table, read once per cell, come from the gas's device table through the
// caches instead of being staged.
#pragma once
#include "kernels.hpp"

namespace adk {
namespace {

constexpr int kWideBlock = 64;  // one wavefront per workgroup

__device__ __forceinline__ int wide_lane() { return threadIdx.x; }

// A cell's lanes: the whole wavefront (G = 64) or an aligned group of G
// lanes of it (the adaptive window's groups of 16, four cells per
// wavefront).  Votes, sums and exchanges stay within the group, so a cell's
// result does not depend on the cells beside it.
template <int G>
struct Lanes {
    static_assert(G == 16 || G == 32 || G == 64, "a cell's lanes are 16, 32 or 64");
    // (a whole-wavefront cell runs in a one-wavefront workgroup)
    static __device__ __forceinline__ int lane() { return G == 64 ? (int)threadIdx.x : (int)(threadIdx.x & (G - 1)); }
    static __device__ __forceinline__ unsigned long long ballot(bool p)
    {
        const unsigned long long b = __ballot(p);
        if constexpr (G == 64) return b;
        else return (b >> (threadIdx.x & 63 & ~(G - 1))) & ((1ull << G) - 1ull);
    }
    static __device__ __forceinline__ bool any(bool p) { return ballot(p) != 0ull; }
    template <class T>
    static __device__ __forceinline__ T shfl(T v, int k)  // lane k of the group, 0 <= k < G
    {
        if constexpr (G == 64) return __shfl(v, k);
        else return __shfl(v, k, G);
    }
    template <class T>
    static __device__ __forceinline__ T down1(T v)  // the next lane's value (own value in the last lane)
    {
        if constexpr (G == 64) return __shfl_down(v, 1);
        else return __shfl_down(v, 1, G);
    }
    static __device__ __forceinline__ double sum(double v)
    {
        static_for<0, (G == 64 ? 6 : (G == 32 ? 5 : 4))>([&](auto kk) { v += __shfl_xor(v, 1 << decltype(kk)::value); });
        return v;
    }
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int tri(int a, int b) { return b * (b + 1) / 2 + a; }

// The solver's tables live in LDS.  Its functions are not inlined (they
// would hold the caller's registers), so their pointers carry the LDS
// address space: through plain (generic) pointers every table access would
// be a flat memory instruction, on the vector memory path, instead of an
// LDS one.
#define ADK_LDS __attribute__((address_space(3)))
using ldsd = ADK_LDS double;
using ldsi = ADK_LDS int;
using ldsf = ADK_LDS float;
template <class T>
__device__ __forceinline__ ADK_LDS T *to_lds(T *p)
{
    return (ADK_LDS T *)p;
}

// Newton below this spread for an entry of n + 1 points (FP64 accuracy; the
// rounding of the recurrence grows ~ n / spread per order).
__device__ __forceinline__ double wide_delta(int n)
{
    return n == 1 ? 0.1 : (n <= 3 ? 0.5 : (n <= 5 ? 1.0 : (n <= 7 ? 1.5 : 2.0)));
}

constexpr int kTaylorMaxTerms = 120;
constexpr int kTaylorRegRow = 8;  // series rows of up to this many entries are summed in registers
constexpr double kWideNegligible = 1e-30;  // populations and transfers below this are left out
constexpr double kWideNegligibleLog = -69.07755278982137;  // log(1e-30)

struct LogFactTable {
    double v[72];
    constexpr LogFactTable() : v()
    {
        // log k! by summing log k in double at compile time would need a
        // constexpr log; store ln k! from the factorial table instead
        double f = 1.0;
        v[0] = 0.0;
        for (int k = 1; k < 72; ++k) {
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
__device__ void taylor_row(const ldsd *s, const ldsd *e, const ldsd *mm, ldsd *D, int a, int nmax, ldsd *hv,
                           int lane, int vs)
{
    const double sa = s[a];
    if (nmax <= kTaylorRegRow) {
        // short rows in registers: the same sums, no LDS round trip per term
        double y[kTaylorRegRow], h[kTaylorRegRow], acc[kTaylorRegRow];
#pragma unroll
        for (int k = 0; k < kTaylorRegRow; ++k) {
            y[k] = k < nmax ? s[a + k + 1] - sa : 0.0;
            h[k] = 1.0;
            acc[k] = kInvFactL.v[k + 1];
        }
        double sgn = 1.0;
        for (int m = 1; m < kTaylorMaxTerms; ++m) {
            sgn = -sgn;
            double prev = 0.0;
            bool conv = true;
#pragma unroll
            for (int k = 0; k < kTaylorRegRow; ++k) {
                if (k < nmax) {
                    const double hk = fma(y[k], h[k], prev);
                    h[k] = hk;
                    prev = hk;
                    const double term = sgn * hk * kInvFactL.v[k + 1 + m];
                    acc[k] += term;
                    conv = conv && !(fabs(term) > 1e-17 * acc[k]);
                }
            }
            if (conv) break;
        }
        const double ea = e[a];
        double scale = 1.0;
#pragma unroll
        for (int k = 0; k < kTaylorRegRow; ++k) {
            if (k < nmax) {
                scale *= mm[a + k + 1];
                D[tri(a, a + k + 1)] = ea == 0.0 ? 0.0 : ea * acc[k] * scale;
            }
        }
        return;
    }
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

constexpr double kWideUlp = 1.1102230246251565e-16;  // 2^-53
constexpr double kWideSeriesErr = 1e-15;              // relative error of a series entry (spread < 2)
constexpr double kWideTableTol = 1e-13;               // table entries above this bound take the squaring
constexpr double kSquareMax = 1024.0;                 // points squared: s <= kSquareMax (j <= 10)

// Entries of the sorted table among the points s_0..s_{r-1} <= kSquareMax by
// scaling and squaring (see chain_sub), then the entries with larger points
// again by the Newton / series rule on top of them.  LDS: D (table), V
// (scratch of (vs - 1) vs doubles), and 192 doubles after V for the scaled
// points.  All G lanes of the cell call it.
template <int G>
__device__ void square_block(int Wp, const ldsd *s, const ldsd *mm, ldsd *D, ldsd *V, int vs)
{
    const int lane = Lanes<G>::lane();
    const int r = __popcll(Lanes<G>::ballot(lane < Wp && s[lane] <= kSquareMax));  // sorted ascending
    if (r < 2) return;
    const double smax = s[r - 1];
    int j = 0;
    while (j < 10 && ldexp(1.0, j) < smax) ++j;
    ldsd *ss = V + (size_t)(vs - 1) * vs, *ee = ss + G, *ms = ee + G;
    if (lane < r) {
        ss[lane] = ldexp(s[lane], -j);
        ee[lane] = exp(-ss[lane]);
        ms[lane] = ldexp(mm[lane], -j);  // the scale max(1, s) and the factor 2^-j per order
    }
    wave_sync();
    if (lane < r) {
        D[tri(lane, lane)] = ee[lane];
        if (lane + 1 < r) taylor_row(ss, ee, ms, D, lane, r - 1 - lane, V, lane, vs);
    }
    wave_sync();
    const int nent = r * (r + 1) / 2;  // entries [a][b], b < r: the first nent of the table
    ldsd *src = D, *dst = V;
    for (int it = 0; it < j; ++it) {
        for (int t = lane; t < nent; t += G) {
            int b = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
            while (b * (b + 1) / 2 > t) --b;
            while ((b + 1) * (b + 2) / 2 <= t) ++b;
            const int a = t - b * (b + 1) / 2;
            double acc = 0.0;
            for (int c = a; c <= b; ++c) acc = fma(src[tri(a, c)], src[tri(c, b)], acc);
            dst[t] = acc;
        }
        wave_sync();
        ldsd *tmp = src;
        src = dst;
        dst = tmp;
    }
    if (src != D) {
        for (int t = lane; t < nent; t += G) D[t] = src[t];
        wave_sync();
    }
    if (r < Wp) {
        for (int ord = 1; ord < Wp; ++ord) {
            if (lane < Wp - ord && lane + ord >= r) {
                const int lo_ = lane, hi = lane + ord;
                const double spread = s[hi] - s[lo_];
                if (spread >= wide_delta(ord))
                    D[tri(lo_, hi)] =
                        PolicyF64::quot(fma(D[tri(lo_, hi - 1)], mm[hi], -D[tri(lo_ + 1, hi)] * mm[lo_ + 1]), spread);
            }
            wave_sync();
        }
    }
}

// The table entries' relative error bounds as kept in LDS: a float per entry
// on a wavefront; on a group of fewer lanes the float's upper 16 bits (the
// bfloat16 grid), rounded up so that a stored bound still bounds, which
// halves the table and lets a CU hold one more wavefront of such groups.
template <int G, bool HALF = (G < 64)>
struct EtStore {
    using type = ADK_LDS float;
    static constexpr size_t kBytes = sizeof(float);
    __device__ static void put(type *p, int i, float v) { p[i] = v; }
    __device__ static float get(const type *p, int i) { return p[i]; }
};
template <int G>
struct EtStore<G, true> {
    using type = ADK_LDS unsigned short;
    static constexpr size_t kBytes = sizeof(unsigned short);
    // v >= 0 and finite (bounds are clamped to 1e30): adding 0xffff before
    // the shift moves every value off the grid up to the next grid point
    __device__ static void put(type *p, int i, float v)
    {
        p[i] = (unsigned short)((__float_as_uint(v) + 0xffffu) >> 16);
    }
    __device__ static float get(const type *p, int i) { return __uint_as_float((unsigned)p[i] << 16); }
};

// Row j = lane of the update, N'_j = sum_{i <= j} T[j][i] N_i (lanes below
// Wp), and in err a bound on its absolute rounding error from the table
// entries' relative bounds Et: the hole recurrence combines non-negative
// terms, so a term's relative error is at most the largest of its entries'
// plus the recurrence's own rounding.
template <bool ERR, int G>
__device__ __forceinline__ double chain_rows(int Wp, double x, const ldsd *s, const ldsd *mm, const ldsd *Nb,
                                             const ldsi *cid, const ldsi *pos, const ldsd *ls, const ldsd *lNb,
                                             const ldsd *D, const typename EtStore<G>::type *Et, ldsd *V,
                                             int vs, double &err)
{
    const int lane = Lanes<G>::lane();
    double acc = 0.0;
    err = 0.0;
    if (lane < Wp) {
        const int j = lane;
        const double mj = fmax(1.0, x);
        double Rp = 1.0;  // prod_{k=i}^{j-1} min(x_k, 1)
        double lb = 0.0;  // log of prod_{k=i}^{j-1} x_k / (j-i)!, which bounds T[j][i] (g <= 1/n!)
        int A = pos[j], B = A;
        // d = j - i counts the steps down from the row: the same on every
        // lane still in the loop, so the factorial table is read with a
        // uniform index
        for (int d = 0; d <= j; ++d) {
            const int i = j - d;
            const int pi = pos[i];
            if (d > 0) {
                const double xi = s[pi];
                Rp *= fmin(xi, 1.0);
                if (Rp == 0.0) break;  // every lower source reaches row j through a zero rate
                lb += ls[pi] - kLogFact.v[d] + kLogFact.v[d - 1];  // log x_i - log (j-i)
            }
            A = min(A, pi);
            B = max(B, pi);
            const double Ni = Nb[i];
            // a source whose contribution is below 1e-30 is skipped (every
            // skipped term is bounded by N_i prod x / (j-i)!)
            if (Ni == 0.0 || fmin(lb, 0.0) + lNb[i] < kWideNegligibleLog) continue;
            const int holes = (B - A + 1) - (j - i + 1);
            double gS, eG = 0.0;
            if (holes == 0) {
                gS = D[tri(A, B)];
                if constexpr (ERR) eG = (double)EtStore<G>::get(Et, tri(A, B));
            } else {
                for (int t = 0; t <= holes; ++t) {
                    V[t * vs + lane] = D[tri(A + t, B)];
                    if constexpr (ERR) eG = fmax(eG, (double)EtStore<G>::get(Et, tri(A + t, B)));
                }
                if constexpr (ERR) eG += (double)((holes + 1) * (holes + 2)) * kWideUlp;
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
                gS = V[lane];
            }
            const double term = Rp * (mm[A] / mj) * gS * Ni;
            acc += term;
            if constexpr (ERR) err = fma(fabs(term), eG + 8.0 * kWideUlp, err);
        }
    }
    return acc;
}

// The exact update of a window of Wp rates held one per lane (x_k in lane k
// for k < Wp, N_k in lane k for k <= Wp; zero elsewhere; lanes counted
// within the cell's G lanes, Wp < G): returns N'_k in lane k.  All G lanes
// of the cell call it together.  V: per-lane columns of the hole
// recurrence, entry t of lane k at V[t vs + k] (vs >= Wp, t <= Wp - 2).
template <bool POSTERIOR, int G = 64>
__device__ double chain_sub(int Wp, double x, double Nk, ldsd *s, ldsd *e, ldsd *mm, ldsd *Nb, ldsi *cid, ldsi *pos,
                            ldsd *D, ldsd *V, int vs)
{
    ldsd *ls = (ldsd *)(pos + G);  // log of the sorted rates
    const int lane = Lanes<G>::lane();
    // rank of x_k among the window's rates (ties by chain index)
    int rank = 0;
    for (int k = 0; k < Wp; ++k) {
        const double xk = Lanes<G>::shfl(x, k);
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
    // relative error bounds of the entries: over the squaring's scaled points
    // after their first G doubles (log |N_i| while the rows are taken); they
    // are read only by the rows taken before any squaring
    using Ets = EtStore<G>;
    typename Ets::type *Et = (typename Ets::type *)(V + (size_t)(vs - 1) * vs + G);
    if (lane < Wp) {
        D[tri(lane, lane)] = e[lane];
        if constexpr (POSTERIOR) Ets::put(Et, tri(lane, lane), (float)(4.0 * kWideUlp));
        int nmax = 0;
        while (lane + nmax + 1 < Wp && s[lane + nmax + 1] - s[lane] < kWideClusterSpread) ++nmax;
        if (nmax > 0) taylor_row(s, e, mm, D, lane, nmax, V, lane, vs);
    }
    wave_sync();
    // Newton orders, each entry with a bound on its relative rounding error:
    // e = (|A| e_A + |B| e_B) / |A - B| + 4 ulp for A - B over the spread
    // (A, B the two entries below it, scaled), 1e-15 for a series entry.
    // Lane a carries the bound of its entry [a][a+ord-1]; entry
    // [a+1][a+ord] is lane a+1's.
    double eprev = 4.0 * kWideUlp, emax = 0.0;
    bool cancelled = false;  // an entry whose two terms cancelled exactly (its relative bound is void)
    for (int ord = 1; ord < Wp; ++ord) {
        const double enb = Lanes<G>::down1(eprev);
        double ecur = eprev;
        if (lane < Wp - ord) {
            const int lo_ = lane, hi = lane + ord;
            const double spread = s[hi] - s[lo_];
            if (spread >= wide_delta(ord)) {
                const double A = D[tri(lo_, hi - 1)] * mm[hi], B = D[tri(lo_ + 1, hi)] * mm[lo_ + 1];
                D[tri(lo_, hi)] = PolicyF64::quot(A - B, spread);
                ecur = (fabs(A) * eprev + fabs(B) * enb) / fabs(A - B) + 4.0 * kWideUlp;
                cancelled = cancelled || (A == B && A != 0.0);
            } else {
                ecur = kWideSeriesErr;
            }
            // (0/0 of two vanishing entries gives NaN: the entry is 0 and so
            // is its error; an exact cancellation of nonzero terms is flagged)
            if constexpr (POSTERIOR) Ets::put(Et, tri(lo_, hi), ecur == ecur ? (float)fmin(ecur, 1e30) : 0.0f);
            emax = fmax(emax, ecur);  // (NaN ignored, as above)
        }
        eprev = ecur;
        wave_sync();
    }
    // Many points within a band of a few tens (a dense cluster of rates)
    // defeat both branches: the recurrence's rounding grows with every order.
    // Then the entries among the points up to kSquareMax come from scaling and
    // squaring instead (McCurdy, Ng and Parlett 1984; the table is exp(-J) for
    // J upper bidiagonal with the points on its diagonal and ones above it, and
    // with the signs of g its entries are non-negative, so products lose
    // nothing): the points scaled by 2^-j (all within [0, 1]) take the series
    // for every entry, the scaled table (entries of exp(-J/2^j), a factor
    // 2^-j per order, times the same max(1, s) scale) is squared j times, and
    // the entries that involve larger points are redone on top of it.
    // When an entry's bound exceeds kWideTableTol: without POSTERIOR the
    // table is squared before the rows are taken; with it the rows are taken
    // first, with a bound on their rounding from the entries' bounds weighted
    // by what each term contributes (all rows together, which also bounds the
    // top slot), and the table is squared and the rows taken again only when
    // that bound exceeds kWideTableTol.  POSTERIOR pays off where the entries
    // with large bounds carry negligible terms: a full chain, most of whose
    // levels hold almost nothing, and, as measured, the adaptive window's
    // cells on the 3D pulse; where such entries matter it costs one more pass
    // over the rows.
    const bool suspect = Lanes<G>::any(emax > kWideTableTol) || Lanes<G>::any(cancelled);
    if (suspect && !POSTERIOR) square_block<G>(Wp, s, mm, D, V, vs);
    // log |N_i| once per source, in the squaring's scratch after the columns
    // (rewritten after a squaring, which uses that scratch)
    ldsd *lNb = V + (size_t)(vs - 1) * vs;
    if (lane <= Wp) lNb[lane] = Nk != 0.0 ? log(fabs(Nk)) : -INFINITY;
    wave_sync();
    double err;
    double acc = chain_rows<POSTERIOR, G>(Wp, x, s, mm, Nb, cid, pos, ls, lNb, D, Et, V, vs, err);
    if (suspect && POSTERIOR) {
        const double errsum = Lanes<G>::sum(lane < Wp ? err : 0.0);
        if (!(errsum <= kWideTableTol) || Lanes<G>::any(cancelled)) {
            wave_sync();
            square_block<G>(Wp, s, mm, D, V, vs);
            if (lane <= Wp) lNb[lane] = Nk != 0.0 ? log(fabs(Nk)) : -INFINITY;
            wave_sync();
            acc = chain_rows<false, G>(Wp, x, s, mm, Nb, cid, pos, ls, lNb, D, Et, V, vs, err);
        }
    }
    // the top slot keeps what the rows leave (columns of T sum to one)
    const double total = Lanes<G>::sum(lane <= Wp ? Nk : 0.0);
    const double rows = Lanes<G>::sum(lane < Wp ? acc : 0.0);
    const double top = fmax(total - rows, 0.0);
    wave_sync();  // LDS reads done before the next use
    return lane < Wp ? acc : (lane == Wp ? top : 0.0);
}

// Doubles of one cell's LDS region for width W and G lanes: s, e, mm, Nb,
// cid and pos, log rates (6 G), the triangular table, the per-lane columns
// ((W - 1) W >= 2 (W + 1), which also holds the scratch of the reach test
// and of the squaring), then the squaring's scaled points (3 G; the first G
// hold log |N_i| while the rows are taken), and, for chain_sub<true>, the
// entries' error bounds (EtStore, triangular) over the last 2 G of those
// points and past them as far as they need.
template <int G = 64>
constexpr size_t wide_cell_doubles(int W, bool bounds)
{
    const size_t tri = (size_t)W * (W + 1) / 2, cols = (size_t)(W - 1) * W;
    const size_t et = (tri * EtStore<G>::kBytes + sizeof(double) - 1) / sizeof(double);
    return 7 * (size_t)G + tri + cols + (bounds && et > 2 * (size_t)G ? et : 2 * (size_t)G);
}
constexpr size_t wide_wave_doubles(int W, bool bounds) { return wide_cell_doubles<64>(W, bounds); }

}  // namespace
}  // namespace adk
