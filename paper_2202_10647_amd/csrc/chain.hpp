// Device-side exact solution of the windowed ionization chain over one step.
//
// The window holds populations N_0..N_W (levels lo..lo+W), rates x_k = W_k dt
// for k < W and an absorbing top.  With rates frozen over the step (Sec. 3,
// constant-rate assumption) the update is N' = T N, T = exp(dt A) for the
// lower-bidiagonal A of Eq. (3).  The eigen expansion of Eqs. (4)-(5) (and
// its explicit 4-level form, Eqs. (6)-(9)) is, entry by entry, the Bateman
// solution
//     T[j][i] = (x_i x_{i+1} ... x_{j-1}) * g(x_i, ..., x_j),   i <= j < W,
// where g(S) = (-1)^n f[S] is the signed divided difference of f(x) = e^{-x}
// over the n+1 points of S.  The absorbing row follows from conservation
// (columns of A sum to zero): T[W][i] = (1 - e^{-x_i}) - sum_{i<j<W} T[j][i],
// with 1 - e^{-x_i} evaluated without cancellation.
//
// Evaluation of g, which is symmetric in its points and positive:
//   * two points a <= b: g = (e^{-a} - e^{-b}) / (b - a) when b - a is not
//     small, else e^{-a} phi(b - a) with the series
//     phi(d) = (1 - e^{-d})/d = sum_k (-d)^k / (k+1)!;
//   * three or more points: the points of the range are sorted and the Newton
//     recurrence g[a..b] = (g[a..b-1] - g[a+1..b]) / (s_b - s_a) is used
//     where s_b - s_a is not small; clustered entries come from the Taylor
//     series of the divided difference about the smallest point (McCurdy, Ng
//     and Parlett 1984),
//         g[a..b] = e^{-s_a} sum_m (-1)^m h_m(s_{a+1}-s_a, ..., s_b-s_a)/(n+m)!,
//     h_m the complete homogeneous symmetric polynomials, summed in double
//     until the terms are negligible for every lane of the wavefront.
// No formula divides by a small rate difference, so equal, zero and
// crossing rates need no special case.
//
// Windows of up to three rates run in the policy's type (float for the mixed
// policy, with its three-point series in double).  Wider windows tabulate in
// double for either policy: products of up to eight capped rates (x <= 1e15)
// and the divided differences stay inside the double range, so nothing is
// rescaled, and the Newton recurrence can run down to small spreads.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace adk {

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F &&>(f));
    }
}

struct InvFactTable {
    double v[64];
    constexpr InvFactTable() : v()
    {
        double f = 1.0;
        v[0] = 1.0;
        for (int k = 1; k < 64; ++k) {
            f *= (double)k;
            v[k] = 1.0 / f;
        }
    }
};
inline constexpr InvFactTable kInvFact{};

// (-1)^m / (n+m)! indexed [n][m] for the Taylor branch (m is wave-uniform,
// so the loads are scalar).
struct TaylorCoefTable {
    double v[10][40];
    constexpr TaylorCoefTable() : v()
    {
        InvFactTable f{};
        for (int n = 0; n < 10; ++n)
            for (int m = 0; m < 40; ++m) v[n][m] = (m & 1) ? -f.v[n + m] : f.v[n + m];
    }
};
__constant__ inline constexpr TaylorCoefTable kTaylorCoef{};

// Precision policies.  `real` is the storage / main arithmetic type; the
// Taylor branch of 3+ clustered points always runs in double.
struct PolicyF64 {
    using real = double;
    static constexpr double kDeltaPhi = 0.1;       // 2-point: series below, difference above
    static constexpr int kPhiDegree = 10;          // 0.1^11/12! < 1e-19
    static constexpr double kDelta3 = 0.5;         // Taylor below this spread (three points, windows
                                                   // of up to three rates)
    static constexpr double kTaylorRelTol = 1e-17;
    static constexpr double kSkipProduct = 1e-18;  // rate products below this: entry is 0
    // windows of four or more rates (double tables): Newton below this
    // spread for a table of L points (index L), series tolerance.  Rounding
    // of the recurrence grows ~ L! / delta^(L-2); these keep it near 1e-13.
    static constexpr double kGenDelta[9] = {0.0, 0.0, 0.1, 0.5, 0.5, 1.0, 1.0, 1.5, 1.5};
    static constexpr double kGenTaylorTol = 1e-17;
    __device__ static __forceinline__ double expneg(double x) { return exp(-x); }
    // a / b from the hardware reciprocal estimate refined by Newton steps
    // (no IEEE division sequence; ~1 ulp)
    __device__ static __forceinline__ double quot(double a, double b)
    {
        double r = __builtin_amdgcn_rcp(b);
        r = fma(r, fma(-b, r, 1.0), r);
        r = fma(r, fma(-b, r, 1.0), r);
        const double q = a * r;
        return fma(fma(-b, q, a), r, q);
    }
};

struct PolicyMixed {
    using real = float;
    static constexpr double kDeltaPhi = 0.5;
    static constexpr int kPhiDegree = 7;           // 0.5^8/9! ~ 1.1e-8, below float rounding
    static constexpr double kDelta3 = 1.0;
    static constexpr double kTaylorRelTol = 1e-9;
    static constexpr double kSkipProduct = 1e-12;
    // double tables for windows of four or more rates, rounding of the
    // recurrence kept near 1e-9 (float results)
    static constexpr double kGenDelta[9] = {0.0, 0.0, 1e-3, 0.01, 0.01, 0.03, 0.1, 0.25, 0.5};
    static constexpr double kGenTaylorTol = 1e-9;
    __device__ static __forceinline__ float expneg(float x) { return __expf(-x); }
    __device__ static __forceinline__ float quot(float a, float b)
    {
        return a * __builtin_amdgcn_rcpf(b);
    }
};

// phi(d) = sum_{k=0}^{K} (-d)^k / (k+1)!  (Horner)
template <int K, class R>
__device__ __forceinline__ R phi_series(R d)
{
    R acc = R((K & 1) ? -kInvFact.v[K + 1] : kInvFact.v[K + 1]);
    static_for<0, K>([&](auto kk) {
        constexpr int k = K - 1 - decltype(kk)::value;
        acc = fma(acc, d, R((k & 1) ? -kInvFact.v[k + 1] : kInvFact.v[k + 1]));
    });
    return acc;
}

// g of two sorted points a <= b with exps ea, eb.
template <class P>
__device__ __forceinline__ typename P::real g2_sorted(typename P::real a, typename P::real b,
                                                      typename P::real ea, typename P::real eb)
{
    using R = typename P::real;
    const R d = b - a;
    const R diff = P::quot(ea - eb, d);
    const R ser = ea * phi_series<P::kPhiDegree>(d);
    return d >= R(P::kDeltaPhi) ? diff : ser;
}

// 1 - e^{-x} without cancellation (e = e^{-x}).
template <class P>
__device__ __forceinline__ typename P::real one_minus_exp(typename P::real x, typename P::real e)
{
    using R = typename P::real;
    return x >= R(P::kDeltaPhi) ? R(1) - e : x * phi_series<P::kPhiDegree>(x);
}

// Compare-exchange of sorted position (A, B) carrying the exp values.
template <int A, int B, class R, int L>
__device__ __forceinline__ void cswap(R (&s)[L], R (&e)[L])
{
    const bool sw = s[A] > s[B];
    const R sa = sw ? s[B] : s[A], sb = sw ? s[A] : s[B];
    const R ea = sw ? e[B] : e[A], eb = sw ? e[A] : e[B];
    s[A] = sa;
    s[B] = sb;
    e[A] = ea;
    e[B] = eb;
}

// Ascending sort of L <= 9 points (with their exp values).
template <int L, class R>
__device__ __forceinline__ void sort_points(R (&s)[L], R (&e)[L])
{
    if constexpr (L == 2) {
        cswap<0, 1>(s, e);
    } else if constexpr (L == 3) {
        cswap<0, 1>(s, e);
        cswap<1, 2>(s, e);
        cswap<0, 1>(s, e);
    } else if constexpr (L == 4) {
        cswap<0, 1>(s, e);
        cswap<2, 3>(s, e);
        cswap<0, 2>(s, e);
        cswap<1, 3>(s, e);
        cswap<1, 2>(s, e);
    } else {
        static_for<0, L>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, L / 2 + 1>([&](auto qq) {
                constexpr int a = 2 * decltype(qq)::value + (r & 1);
                if constexpr (a + 1 < L) cswap<a, a + 1>(s, e);
            });
        });
    }
}

// Taylor branch for sorted points s[A..B] (B > A), in double, summed
// until the terms are below the tolerance relative to the sum in every
// active lane: returns g[A..B].
template <class P, int A, int B, int L>
__device__ __forceinline__ double taylor_dd(const double (&s)[L], double ea)
{
    constexpr int n = B - A;  // number of variables s_k - s_A, k = A+1..B
    double y[n], h[n];
    static_for<0, n>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        y[v] = s[A + 1 + v] - s[A];
        h[v] = 1.0;
    });
    double acc = kInvFact.v[n];
    double c_next = kTaylorCoef.v[n][1];
    for (int m = 1; m < 39; ++m) {
        // the next coefficient's (scalar) load is issued a step ahead
        const double c = c_next;
        c_next = kTaylorCoef.v[n][m + 1];
        // h^(1)_m = y_1 h^(1)_{m-1};  h^(k)_m = y_k h^(k)_{m-1} + h^(k-1)_m
        h[0] *= y[0];
        static_for<1, n>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            h[v] = fma(y[v], h[v], h[v - 1]);
        });
        const double term = c * h[n - 1];
        acc += term;
        if (__all(!(fabs(term) > P::kGenTaylorTol * acc))) break;
    }
    return ea * acc;
}

// Newton table of L >= 2 sorted points (double): tab[a][b] = g[s_a..s_b]
// for a < b; an entry of three or more points whose spread is below the
// policy's threshold for tables of L points is taken from the Taylor series
// instead.
template <class P, int L>
__device__ __forceinline__ void dd_table(const double (&s)[L], const double (&e)[L], double (&tab)[L][L])
{
    constexpr double delta = P::kGenDelta[L];
    // pairs: difference quotient, or the phi series below 0.1 (branch-free)
    static_for<0, L - 1>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        tab[a][a + 1] = g2_sorted<PolicyF64>(s[a], s[a + 1], e[a], e[a + 1]);
    });
    static_for<2, L>([&](auto ll) {
        constexpr int len = decltype(ll)::value;
        static_for<0, L - len>([&](auto aa) {
            constexpr int a = decltype(aa)::value;
            constexpr int b = a + len;
            const double spread = s[b] - s[a];
            double t;
            if (spread >= delta)
                t = PolicyF64::quot(tab[a][b - 1] - tab[a + 1][b], spread);
            else
                t = taylor_dd<P, a, b>(s, e[a]);
            tab[a][b] = t;
        });
    });
}

// g over L >= 2 sorted points (double).
template <class P, int L>
__device__ __forceinline__ double dd_sorted(const double (&s)[L], const double (&e)[L])
{
    double tab[L][L];
    dd_table<P, L>(s, e, tab);
    return tab[0][L - 1];
}

// T[J][I] for the chain range [I..J] of rate points (J - I >= 2), 0 when the
// rate product is negligible in every lane of the wavefront.
template <class P, int W, int I, int J>
__device__ __forceinline__ double range_entry(const double (&x)[W], const double (&ex)[W])
{
    constexpr int L = J - I + 1;
    double prod = 1.0;
    static_for<I, J>([&](auto kk) { prod *= x[decltype(kk)::value]; });
    if (!__any(prod >= P::kSkipProduct)) return 0.0;
    double s[L], e[L];
    static_for<0, L>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        s[k] = x[I + k];
        e[k] = ex[I + k];
    });
    sort_points<L>(s, e);
    // a range clustered as a whole needs its top entry only: one series
    double g;
    if (s[L - 1] - s[0] < P::kGenDelta[L])
        g = taylor_dd<P, 0, L - 1>(s, e[0]);
    else
        g = dd_sorted<P, L>(s, e);
    return prod * g;
}

// g of two points in any order.
template <class P>
__device__ __forceinline__ typename P::real g_pair(typename P::real a, typename P::real b, typename P::real ea,
                                                   typename P::real eb)
{
    using R = typename P::real;
    const bool sw = a > b;
    const R lo = sw ? b : a, hi = sw ? a : b;
    const R elo = sw ? eb : ea, ehi = sw ? ea : eb;
    return g2_sorted<P>(lo, hi, elo, ehi);
}

// Taylor series of g over three points mn <= md <= mx (double, adaptive).
template <class P, class R>
__device__ __forceinline__ double taylor3(R mn, R md, R mx, R emn)
{
    const double y1 = (double)md - (double)mn, y2 = (double)mx - (double)mn;
    double h1 = 1.0, h2 = 1.0, acc = 0.5;
    for (int m = 1; m < 39; ++m) {
        h1 *= y1;
        h2 = fma(y2, h2, h1);
        const double term = kTaylorCoef.v[2][m] * h2;
        acc += term;
        if (__all(!(fabs(term) > P::kTaylorRelTol * acc))) break;
    }
    return (double)emn * acc;
}

// Windows of up to three rates: the only range of three points is [0..2],
// whose divided difference reuses the pair values of the neighbouring
// entries.  With rates capped at 1e12 no product leaves the float range.
template <class P, int W>
__device__ __forceinline__ void chain_apply_small(const typename P::real (&x)[W], const double (&N)[W + 1],
                                                  double (&out)[W + 1])
{
    using R = typename P::real;
    R ex[W];
    double om[W];
    static_for<0, W>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        ex[k] = P::expneg(x[k]);
        om[k] = (double)one_minus_exp<P>(x[k], ex[k]);
    });
    if constexpr (W == 1) {
        out[0] = (double)ex[0] * N[0];
        out[1] = fma(om[0], N[0], N[1]);
    } else if constexpr (W == 2) {
        const double T10 = (double)(x[0] * g_pair<P>(x[0], x[1], ex[0], ex[1]));
        out[0] = (double)ex[0] * N[0];
        out[1] = fma(T10, N[0], (double)ex[1] * N[1]);
        double t0 = om[0] - T10;
        t0 = t0 < 0.0 ? 0.0 : t0;
        out[2] = fma(t0, N[0], fma(om[1], N[1], N[2]));
    } else {
        const R x0 = x[0], x1 = x[1], x2 = x[2];
        const R e0 = ex[0], e1 = ex[1], e2 = ex[2];
        const R g01 = g_pair<P>(x0, x1, e0, e1);
        const R g12 = g_pair<P>(x1, x2, e1, e2);
        const double T10 = (double)(x0 * g01), T21 = (double)(x1 * g12);
        double T20 = 0.0;
        const double prod = (double)x0 * (double)x1;
        if (__any(prod >= P::kSkipProduct)) {
            // g[S] = (g[S \ max] - g[S \ min]) / (max - min)
            const bool x1_mid = (x0 <= x1 && x1 <= x2) || (x0 >= x1 && x1 >= x2);
            R g02 = R(0);
            if (__any(!x1_mid)) g02 = g_pair<P>(x0, x2, e0, e2);
            const int imax = (x0 >= x1 && x0 >= x2) ? 0 : (x1 >= x2 ? 1 : 2);
            const int imin = (x0 <= x1 && x0 <= x2) ? 0 : (x1 <= x2 ? 1 : 2);
            // pair without point m: m = 0 -> (1,2), 1 -> (0,2), 2 -> (0,1)
            const R g_lo = imax == 0 ? g12 : (imax == 1 ? g02 : g01);
            const R g_hi = imin == 0 ? g12 : (imin == 1 ? g02 : g01);
            const R mn = x0 < x1 ? (x0 < x2 ? x0 : x2) : (x1 < x2 ? x1 : x2);
            const R mx = x0 > x1 ? (x0 > x2 ? x0 : x2) : (x1 > x2 ? x1 : x2);
            const R spread = mx - mn;
            R g3;
            if (spread >= R(P::kDelta3)) {
                g3 = P::quot(g_lo - g_hi, spread);
            } else {
                const R a01 = x0 < x1 ? x0 : x1, b01 = x0 < x1 ? x1 : x0;
                const R md = b01 < x2 ? b01 : (a01 > x2 ? a01 : x2);
                const R emn = imin == 0 ? e0 : (imin == 1 ? e1 : e2);
                g3 = (R)taylor3<P>(mn, md, mx, emn);
            }
            T20 = prod * (double)g3;
        }
        out[0] = (double)e0 * N[0];
        out[1] = fma(T10, N[0], (double)e1 * N[1]);
        out[2] = fma(T20, N[0], fma(T21, N[1], (double)e2 * N[2]));
        double t0 = om[0] - T10 - T20, t1 = om[1] - T21;
        t0 = t0 < 0.0 ? 0.0 : t0;
        t1 = t1 < 0.0 ? 0.0 : t1;
        out[3] = fma(t0, N[0], fma(t1, N[1], fma(om[2], N[2], N[3])));
    }
}

template <class P, int W>
__device__ __forceinline__ void chain_apply_general(const typename P::real (&x)[W], const double (&N)[W + 1],
                                                    double (&out)[W + 1]);

// Weak rates.  When every rate of the window is at most kWeakRate in every
// lane of the wavefront (the edge of a pulse, where the steep rate law leaves
// most ionizing cells), N' = exp(dt A) N is summed as its Taylor series to
// order kWeakOrder: y_0 = N, y_k = (dt A) y_{k-1} / k, N' = sum_k y_k, with
// (dt A y)_j = x_{j-1} y_{j-1} - x_j y_j and inflow only into the absorbing
// top slot.  Since ||dt A||_1 <= 2 max x, the remainder is at most
// (2 max x)^(K+1) / (K+1)! of the window's population: 2.7e-16 for 1e-3 and
// K = 4, below the rounding of the exact forms.  Every power of A has zero
// column sums, so the truncated series conserves the population up to
// rounding.  The terms are formed in the policy's type (each is at most
// 2e-3 of the population, so float terms cost < 1e-10) and summed onto the
// populations in double.
constexpr double kWeakRate = 1e-3;
constexpr int kWeakOrder = 4;

template <class P, int W>
__device__ __forceinline__ bool chain_apply_weak(const typename P::real (&x)[W], const double (&N)[W + 1],
                                                 double (&out)[W + 1])
{
    using R = typename P::real;
    R xm = R(0);
    static_for<0, W>([&](auto kk) { xm = fmax(xm, x[decltype(kk)::value]); });
    if (!__all(xm <= R(kWeakRate))) return false;
    R y[W + 1];
    static_for<0, W + 1>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        y[j] = (R)N[j];
        out[j] = N[j];
    });
    static_for<1, kWeakOrder + 1>([&](auto kk) {
        constexpr R inv = R(1) / R(decltype(kk)::value);
        R z[W + 1];
        z[0] = -x[0] * y[0];
        static_for<1, W>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            z[j] = fma(x[j - 1], y[j - 1], -x[j] * y[j]);
        });
        z[W] = x[W - 1] * y[W - 1];
        static_for<0, W + 1>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            y[j] = z[j] * inv;
            out[j] += (double)y[j];
        });
    });
    return true;
}

// N' = T N for one cell.  Identity when no lane of the wavefront has a
// nonzero rate; the weak-rate series when every rate is small.
template <class P, int W>
__device__ __forceinline__ void chain_apply(const typename P::real (&x)[W], const double (&N)[W + 1],
                                            double (&out)[W + 1])
{
    using R = typename P::real;
    bool active = false;
    static_for<0, W>([&](auto kk) { active |= !(x[decltype(kk)::value] == R(0)); });
    if (!__any(active)) {
        static_for<0, W + 1>([&](auto jj) { out[decltype(jj)::value] = N[decltype(jj)::value]; });
        return;
    }
    if (chain_apply_weak<P, W>(x, N, out)) return;
    if constexpr (W <= 3) {
        chain_apply_small<P, W>(x, N, out);
    } else {
        chain_apply_general<P, W>(x, N, out);
    }
}

// Windows of four or more rates, in double for either policy.  Double range
// holds every product of up to eight capped rates and every divided
// difference, so no scaling is needed, and double rounding lets the Newton
// recurrence run down to much smaller spreads than float would (the series
// then converges in a few terms).
template <class P, int W>
__device__ __forceinline__ void chain_apply_general(const typename P::real (&x)[W], const double (&N)[W + 1],
                                                    double (&out)[W + 1])
{
    double xd[W], ex[W], om[W];
    static_for<0, W>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        xd[k] = (double)x[k];
        ex[k] = exp(-xd[k]);
        om[k] = one_minus_exp<PolicyF64>(xd[k], ex[k]);
    });
    // T[j][i] for i <= j < W
    double T[W][W];
    static_for<0, W>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        T[i][i] = ex[i];
        if constexpr (i + 1 < W) {
            const double a = xd[i], b = xd[i + 1];
            const bool sw = a > b;
            const double lo = sw ? b : a, hi = sw ? a : b;
            const double elo = sw ? ex[i + 1] : ex[i], ehi = sw ? ex[i] : ex[i + 1];
            T[i + 1][i] = xd[i] * g2_sorted<PolicyF64>(lo, hi, elo, ehi);
        }
    });
    // Rates monotone along the window (the usual case: deeper levels ionize
    // more slowly) in every lane: the chain order is the sorted order,
    // reversed where the rates fall, and one table over the W points gives
    // every range.  Otherwise each range is sorted and tabulated on its own.
    bool inc = true, dec = true;
    static_for<0, W - 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        inc = inc && xd[k] <= xd[k + 1];
        dec = dec && xd[k] >= xd[k + 1];
    });
    if (__all(inc || dec)) {
        double s[W], e[W], tab[W][W];
        static_for<0, W>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            s[k] = dec ? xd[W - 1 - k] : xd[k];
            e[k] = dec ? ex[W - 1 - k] : ex[k];
        });
        dd_table<P, W>(s, e, tab);
        static_for<2, W>([&](auto dd) {
            constexpr int d = decltype(dd)::value;
            static_for<0, W - d>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                double prod = 1.0;
                static_for<i, i + d>([&](auto kk) { prod *= xd[decltype(kk)::value]; });
                // chain range [i..i+d] = sorted positions [i..i+d], or
                // [W-1-i-d..W-1-i] where the rates fall
                const double g = dec ? tab[W - 1 - i - d][W - 1 - i] : tab[i][i + d];
                T[i + d][i] = prod * g;
            });
        });
    } else {
        static_for<2, W>([&](auto dd) {
            constexpr int d = decltype(dd)::value;
            static_for<0, W - d>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                T[i + d][i] = range_entry<P, W, i, i + d>(xd, ex);
            });
        });
    }
    static_for<0, W>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        double acc = T[j][j] * N[j];
        static_for<0, j>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            acc = fma(T[j][i], N[i], acc);
        });
        out[j] = acc;
    });
    // absorbing top: column sums of T are one
    double top = N[W];
    static_for<0, W>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        double t = om[i];
        static_for<i + 1, W>([&](auto jj) { t -= T[decltype(jj)::value][i]; });
        t = t < 0.0 ? 0.0 : t;  // rounding only; NaN passes through
        top = fma(t, N[i], top);
    });
    out[W] = top;
}

}  // namespace adk
