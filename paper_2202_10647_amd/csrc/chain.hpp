// Device-side exact solution of the windowed ionization chain over one step.
//
// The window holds populations N_0..N_W (levels lo..lo+W), rates x_k = W_k dt
// for k < W and an absorbing top (x_W = 0).  With rates frozen over the step
// (Sec. 3, constant-rate assumption) the update is N' = T N, T = exp(dt A)
// for the lower-bidiagonal A of Eq. (3).  The eigen expansion of Eqs. (4)-(5)
// (and its explicit 4-level form, Eqs. (6)-(9)) is, entry by entry, the
// Bateman solution
//     T[j][i] = (x_i x_{i+1} ... x_{j-1}) * g(x_i, ..., x_j),   j >= i,
// where g(S) = (-1)^n f[S] is the signed divided difference of f(x) = e^{-x}
// over the n+1 points of S.  g is symmetric in its points and positive, so it
// is evaluated on the points of each chain range sorted ascending with the
// Newton recurrence
//     g[a..b] = (g[a..b-1] - g[a+1..b]) / (s_b - s_a),
// which loses accuracy only when s_b - s_a is small.  Those entries are taken
// from the Taylor series of the divided difference about the smallest point
// (McCurdy, Ng and Parlett 1984):
//     g[a..b] = e^{-s_a} sum_m (-1)^m h_m(s_{a+1}-s_a, ..., s_b-s_a) / (n+m)!
// with h_m the complete homogeneous symmetric polynomials.  This is the
// divided-difference form of the paper's 1/(W_i - W_j) coefficients: it has
// no division by a rate difference, so equal, zero and crossing rates need no
// special case.
//
// Scaling: synthetic gases reach x ~ 1e10 per step, where the products of
// rates and the divided differences over- and underflow.  The table stores
// ghat[a..b] = g[a..b] * prod_{k=a+1..b} m_k with m_k = max(1, s_k), whose
// recurrence is ghat[a..b] = (ghat[a..b-1] m_b - ghat[a+1..b] m_{a+1}) /
// (s_b - s_a), and the rate product becomes prod (x_k / m_k) times a ratio of
// m's <= 1, so no intermediate leaves the range of the storage type.
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
    double v[48];
    constexpr InvFactTable() : v()
    {
        double f = 1.0;
        v[0] = 1.0;
        for (int k = 1; k < 48; ++k) {
            f *= (double)k;
            v[k] = 1.0 / f;
        }
    }
};
inline constexpr InvFactTable kInvFact{};

// Precision policies.  `real` is the storage / main arithmetic type; the
// Taylor branch always runs in double.
struct PolicyF64 {
    using real = double;
    static constexpr double kDeltaSmallW = 0.5, kDeltaLargeW = 1.0;
    static constexpr int kMSmallW = 16, kMLargeW = 20;
    __device__ static __forceinline__ double expneg(double x) { return exp(-x); }
    __device__ static __forceinline__ double quot(double a, double b) { return a / b; }
};

struct PolicyMixed {
    using real = float;
    static constexpr double kDeltaSmallW = 1.0, kDeltaLargeW = 2.0;
    static constexpr int kMSmallW = 13, kMLargeW = 17;
    __device__ static __forceinline__ float expneg(float x) { return __expf(-x); }
    __device__ static __forceinline__ float quot(float a, float b)
    {
        return a * __builtin_amdgcn_rcpf(b);
    }
};

template <class P, int W>
struct DDParams {
    static constexpr double delta = (W <= 4) ? P::kDeltaSmallW : P::kDeltaLargeW;
    static constexpr int M = (W <= 4) ? P::kMSmallW : P::kMLargeW;
};

template <class R>
__device__ __forceinline__ R scale_of(R s)
{
    return s > R(1) ? s : R(1);
}

// Chain point K of the window: rate x_K for K < W, the absorbing top (0) at K = W.
template <int W, int K, class R>
__device__ __forceinline__ R point(const R (&x)[W])
{
    if constexpr (K < W)
        return x[K];
    else
        return R(0);
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
        // odd-even transposition network: L rounds
        static_for<0, L>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, L / 2 + 1>([&](auto qq) {
                constexpr int a = 2 * decltype(qq)::value + (r & 1);
                if constexpr (a + 1 < L) cswap<a, a + 1>(s, e);
            });
        });
    }
}

// Taylor branch for the sorted points s[A..B] (A < B), in double:
// g[A..B] * prod_{k=A+1..B} m_k.
template <int A, int B, int M, class R, int L>
__device__ __forceinline__ double taylor_scaled(const R (&s)[L], R ea)
{
    constexpr int n = B - A;
    const double base = (double)s[A];
    double h[M + 1];
    h[0] = 1.0;
    static_for<1, M + 1>([&](auto mm) { h[decltype(mm)::value] = 0.0; });
    double msc = 1.0;
    static_for<A + 1, B + 1>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const double y = (double)s[v] - base;
        msc *= (double)scale_of(s[v]);
        static_for<1, M + 1>([&](auto mm) {
            constexpr int m = decltype(mm)::value;
            h[m] = fma(y, h[m - 1], h[m]);
        });
    });
    double tot = 0.0;
    static_for<0, M + 1>([&](auto mm) {
        constexpr int m = M - decltype(mm)::value;
        constexpr double c = (m & 1) ? -kInvFact.v[n + m] : kInvFact.v[n + m];
        tot = fma(c, h[m], tot);
    });
    return (double)ea * tot * msc;
}

// Full scaled table over L sorted points: tab[a][b] = ghat[a..b] for a <= b.
template <class P, int W, int L>
__device__ __forceinline__ void dd_table(const typename P::real (&s)[L], const typename P::real (&e)[L],
                                         typename P::real (&tab)[L][L])
{
    using R = typename P::real;
    constexpr R delta = (R)DDParams<P, W>::delta;
    constexpr int M = DDParams<P, W>::M;
    R msc[L];
    static_for<0, L>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        tab[a][a] = e[a];
        msc[a] = scale_of(s[a]);
    });
    static_for<1, L>([&](auto ll) {
        constexpr int len = decltype(ll)::value;
        static_for<0, L - len>([&](auto aa) {
            constexpr int a = decltype(aa)::value;
            constexpr int b = a + len;
            const R spread = s[b] - s[a];
            R t;
            if (spread >= delta) {
                t = P::quot(tab[a][b - 1] * msc[b] - tab[a + 1][b] * msc[a + 1], spread);
            } else {
                t = (R)taylor_scaled<a, b, M>(s, e[a]);
            }
            tab[a][b] = t;
        });
    });
}

// Accumulate out[j] += T[j][i] N[i] for all i <= j of the window.
// x[0..W-1] rates, ex[0..W] = exp(-x) with ex[W] = 1.
// General path: every chain range is sorted on its own.
template <class P, int W>
__device__ __forceinline__ void chain_apply_general(const typename P::real (&x)[W],
                                                    const typename P::real (&ex)[W + 1],
                                                    const double (&N)[W + 1], double (&out)[W + 1])
{
    using R = typename P::real;
    static_for<0, W + 1>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        out[j] = (double)ex[j] * N[j];
    });
    static_for<0, W>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        R rho = R(1);  // prod_{k=i}^{j-1} x_k / m_k
        static_for<i + 1, W + 1>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            constexpr int L = j - i + 1;
            rho *= x[j - 1] / scale_of(x[j - 1]);
            R s[L], e[L];
            static_for<0, L>([&](auto kk) {
                constexpr int k = decltype(kk)::value;
                s[k] = point<W, i + k>(x);
                e[k] = ex[i + k];
            });
            sort_points<L>(s, e);
            R tab[L][L];
            dd_table<P, W, L>(s, e, tab);
            const R mj = scale_of(point<W, j>(x));
            const double Tji = (double)rho * (double)tab[0][L - 1] * ((double)scale_of(s[0]) / (double)mj);
            out[j] = fma(Tji, N[i], out[j]);
        });
    });
}

// Monotone path: valid when x_0 >= x_1 >= ... >= x_{W-1} >= 0, so every chain
// range is already sorted (descending) and one table over the reversed points
// serves all ranges: chain range [i..j] is sorted range [W-j .. W-i].
template <class P, int W>
__device__ __forceinline__ void chain_apply_monotone(const typename P::real (&x)[W],
                                                     const typename P::real (&ex)[W + 1],
                                                     const double (&N)[W + 1], double (&out)[W + 1])
{
    using R = typename P::real;
    constexpr int L = W + 1;
    R s[L], e[L];
    static_for<0, L>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        constexpr int c = W - k;  // chain index of sorted position k
        s[k] = point<W, c>(x);
        e[k] = ex[c];
    });
    R tab[L][L];
    dd_table<P, W, L>(s, e, tab);
    static_for<0, W + 1>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        out[j] = (double)ex[j] * N[j];
    });
    static_for<0, W>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        R rho = R(1);
        static_for<i + 1, W + 1>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            rho *= x[j - 1] / scale_of(x[j - 1]);
            const double Tji = (double)rho * (double)tab[W - j][W - i];
            out[j] = fma(Tji, N[i], out[j]);
        });
    });
}

// N' = T N for one cell.  Wave-uniform dispatch: identity when no lane of the
// wave has a nonzero rate, the single-table path when every lane's rates are
// non-increasing along the window, the general path otherwise.
template <class P, int W>
__device__ __forceinline__ void chain_apply(const typename P::real (&x)[W], const double (&N)[W + 1],
                                            double (&out)[W + 1])
{
    using R = typename P::real;
    bool active = false, mono = true;
    static_for<0, W>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        active |= !(x[k] == R(0));
        if constexpr (k + 1 < W) mono &= (x[k] >= x[k + 1]);
    });
    if (!__any(active)) {
        static_for<0, W + 1>([&](auto jj) { out[decltype(jj)::value] = N[decltype(jj)::value]; });
        return;
    }
    R ex[W + 1];
    static_for<0, W>([&](auto kk) { ex[decltype(kk)::value] = P::expneg(x[decltype(kk)::value]); });
    ex[W] = R(1);
    if (__all(mono)) {
        chain_apply_monotone<P, W>(x, ex, N, out);
    } else {
        chain_apply_general<P, W>(x, ex, N, out);
    }
}

}  // namespace adk
