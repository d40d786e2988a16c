/*
 * adk_oracle.c -- plain, slow, FP64 CPU oracle for the multi-level ADK
 * ionization step (Cheng & Samulyak, "Efficient numerical algorithm for
 * multi-level ionization of high-atomic-number gases").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The HIP library never
 * links, includes or calls anything here, and this file includes nothing from
 * it: the two share no code, headers, tables or constants.
 *
 * What it computes, per mesh cell and independently of every other cell
 * (Sec. 3, the remark after Eq. (5) that solutions are computed cell by cell):
 *   1. ADK rate of every charge state by Eq. (1), evaluated literally as the
 *      printed product of factors (pow/exp/sqrt, integer factorials).
 *   2. The rate chain of Eq. (2) / matrix form Eq. (3) restricted to the
 *      locally-reduced window [p, top] (Sec. 3, the reduced 4-level system,
 *      Eqs. (6)-(9)): top = min(p + w, Z) is absorbing within the step.
 *   3. Rates frozen over the step (Sec. 3, the constant-rate assumption), so
 *      the exact update is N(t+dt) = expm(dt * A_window) N(t): the same result
 *      as the eigen-expansion Eqs. (4)-(5), computed here by a Taylor series
 *      with scaling and squaring in quad precision, which needs no distinct
 *      eigenvalues.
 *   4. Window shift at the START of the step (Sec. 3, the cut-off criterion
 *      paragraph after Eq. (9)): while p < Z and N_p < eps the residual N_p
 *      is folded into N_{p+1} and p is incremented.
 *
 * Readings of the paper that this file takes (silent or garbled passages):
 *   - E_L = |E|; E_L == 0 gives W = 0 (limit of the exp factor of Eq. (1)).
 *   - A rate whose exp factor exp(-2 E_a (Q/n*)^3 / (3 E_L)) is below the
 *     smallest normal double is taken as zero (such rates are < 1e-200/s).
 *   - Level k (charge k -> k+1) uses Q = k + 1 and the k-th listed ionization
 *     potential U[k]; n* = Q sqrt(U_H / U[k]) (Sec. 2, text after Eq. (1)).
 *   - "e" in (2e/n*)^(2n*) is Euler's number.
 *   - m < 0 in the level table means: average the rate over the projections
 *     m = -l..l with equal weight.
 *   - The residual population at a window shift is folded upward, which
 *     conserves the total exactly.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 72 /* largest chain matrix handled: Z + 1 <= 72 */

static double orc_fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

/*
 * Eq. (1), literally: W_lm for one electron with orbital number l and
 * projection |m| = am, in s^-1.  U in eV, E in GV/m.
 * consts = {omega_a [s^-1], E_a [GV/m], U_H [eV]} (Sec. 2, text after Eq. (1)).
 * Pinned by hand-simplified closed forms at n* = 1, 2 and 3 (which fix the
 * n* dependence of every factor), the charge scaling law, the |m| and l
 * factors and, at non-integer n*, the whole field dependence (the paper
 * prints no rate values).
 */
double orc_rate_lm(double U, int Q, int l, int am, double E, const double *consts)
{
    const double omega_a = consts[0], E_a = consts[1], U_H = consts[2];
    const double EL = fabs(E);
    if (EL == 0.0) return 0.0;
    const double ns = (double)Q * sqrt(U_H / U);
    const double Q3 = (double)Q * Q * Q;
    const double n3 = ns * ns * ns;
    const double f_sqrt = sqrt(3.0 * n3 * EL / (M_PI * Q3 * E_a));
    const double f_q2 = (double)Q * Q / (2.0 * ns * ns);
    const double f_stirling = pow(2.0 * M_E / ns, 2.0 * ns);
    const double f_tunnel = exp(-2.0 * E_a / (3.0 * EL) * pow((double)Q / ns, 3.0));
    /* Tunnelling factor below the normal range: the rate is below ~1e-200/s
     * (W dt < 1e-215 for fs steps) and is taken as zero; this also keeps the
     * product from inheriting the lost precision of a subnormal factor. */
    if (f_tunnel < DBL_MIN) return 0.0;
    const double f_lm = (2.0 * l + 1.0) * orc_fact(l + am) /
                        (2.0 * M_PI * ns * pow(2.0, am) * orc_fact(am) * orc_fact(l - am));
    const double f_pow = pow(2.0 * E_a * Q3 / (EL * n3), 2.0 * ns - am - 1.0);
    return omega_a * f_sqrt * f_q2 * f_stirling * f_tunnel * f_lm * f_pow;
}

/* Rate of level k of a gas: fixed |m|, or the equal-weight average over
 * m = -l..l when m < 0. */
double orc_level_rate(double U, int Q, int l, int m, double E, const double *consts)
{
    if (m >= 0) return orc_rate_lm(U, Q, l, m, E, consts);
    double s = 0.0;
    for (int mm = -l; mm <= l; ++mm) s += orc_rate_lm(U, Q, l, abs(mm), E, consts);
    return s / (2.0 * l + 1.0);
}

/* W_out[j][i] = rate of level k0 + j at field E[i], j < nk, i < n. */
void orc_rates(int Z, const double *U, const int8_t *l, const int8_t *m, const double *consts,
               const double *E, int64_t n, int k0, int nk, double *W_out)
{
    (void)Z;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < nk; ++j) {
            const int k = k0 + j;
            W_out[(int64_t)j * n + i] = orc_level_rate(U[k], k + 1, l[k], m[k], E[i], consts);
        }
}

/* Quad precision (IEEE binary128, software arithmetic): the squaring phase
 * of the matrix exponential multiplies rounding errors by up to 2^s, and the
 * synthetic gases reach dt*W ~ 1e10 (s ~ 35), so the oracle works in a
 * format whose rounding (1e-34) stays far below the GPU tolerances. */
typedef __float128 qreal;

/* C = A * B for n x n row-major matrices. */
static void orc_matmul(int n, const qreal *A, const qreal *B, qreal *C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            qreal s = 0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

/*
 * T = exp(M) for an n x n row-major matrix: scale M by 2^-s so that its
 * 1-norm is at most 1/2, sum the Taylor series to degree 30, square s times.
 * Quad precision throughout; the result is rounded to double.
 */
void orc_expm(int n, const double *M, double *T)
{
    qreal S[n * n], term[n * n], acc[n * n], tmp[n * n];
    double norm = 0.0;
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(M[i * n + j]);
        if (c > norm) norm = c;
    }
    int s = 0;
    while (norm > 0.5 && s < 1100) { norm *= 0.5; ++s; }
    for (int i = 0; i < n * n; ++i) S[i] = (qreal)ldexp(M[i], -s);
    for (int i = 0; i < n * n; ++i) acc[i] = term[i] = 0;
    for (int i = 0; i < n; ++i) acc[i * n + i] = term[i * n + i] = 1;
    for (int k = 1; k <= 30; ++k) {
        orc_matmul(n, term, S, tmp);
        for (int i = 0; i < n * n; ++i) {
            term[i] = tmp[i] / (qreal)k;
            acc[i] += term[i];
        }
    }
    for (int r = 0; r < s; ++r) {
        orc_matmul(n, acc, acc, tmp);
        memcpy(acc, tmp, sizeof(qreal) * (size_t)n * (size_t)n);
    }
    for (int i = 0; i < n * n; ++i) T[i] = (double)acc[i];
}

/*
 * Advance populations N[0..n-1] over dt under the lower-bidiagonal chain of
 * Eq. (3) restricted to n levels, rates W[0..n-2] (s^-1), last level
 * absorbing: N <- expm(dt A) N.
 */
static void orc_advance_window(int n, const double *W, double dt, double *N)
{
    if (n < 2) return;
    double A[n * n], T[n * n], out[n];
    memset(A, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int i = 0; i + 1 < n; ++i) {
        A[i * n + i] = -W[i] * dt;
        A[(i + 1) * n + i] = W[i] * dt;
    }
    orc_expm(n, A, T);
    for (int i = 0; i < n; ++i) {
        qreal s = 0;
        for (int j = 0; j < n; ++j) s += (qreal)T[i * n + j] * (qreal)N[j];
        out[i] = (double)s;
    }
    memcpy(N, out, sizeof(double) * (size_t)n);
}

/*
 * Chain advance with given rates and no window logic:
 * pops[(w+1)][ncells] SoA, W[w][ncells] SoA (s^-1).
 */
void orc_chain_advance(int w, int64_t ncells, const double *W, double dt, double *pops)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
        double N[ORC_MAXN], Wc[ORC_MAXN];
        for (int s = 0; s <= w; ++s) N[s] = pops[(int64_t)s * ncells + c];
        for (int s = 0; s < w; ++s) Wc[s] = W[(int64_t)s * ncells + c];
        orc_advance_window(w + 1, Wc, dt, N);
        for (int s = 0; s <= w; ++s) pops[(int64_t)s * ncells + c] = N[s];
    }
}

/*
 * One ionization step for every cell.
 * layout 0 (compact): pops[(w+1)][ncells], slot s holds level p + s.
 * layout 1 (full):    pops[(Z+1)][ncells], row k holds level k.
 * p[ncells]: lowest window level, updated in place (values above Z read as Z).
 */
void orc_ionize_step(int Z, const double *U, const int8_t *l, const int8_t *m,
                     const double *consts, int64_t ncells, const double *E, double dt,
                     int w, double eps, int layout, double *pops, uint8_t *p)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < ncells; ++c) {
        double N[ORC_MAXN], W[ORC_MAXN];
        for (int k = 0; k <= Z; ++k) N[k] = 0.0;
        int lo = p[c] > Z ? Z : p[c];
        if (layout == 0) {
            for (int s = 0; s <= w; ++s)
                if (lo + s <= Z) N[lo + s] = pops[(int64_t)s * ncells + c];
        } else {
            for (int k = 0; k <= Z; ++k) N[k] = pops[(int64_t)k * ncells + c];
        }
        /* window shift at the start of the step, residual folded upward */
        while (lo < Z && N[lo] < eps) {
            N[lo + 1] += N[lo];
            N[lo] = 0.0;
            ++lo;
        }
        const int top = lo + w < Z ? lo + w : Z;
        for (int k = lo; k < top; ++k) W[k - lo] = orc_level_rate(U[k], k + 1, l[k], m[k], E[c], consts);
        orc_advance_window(top - lo + 1, W, dt, N + lo);
        if (layout == 0) {
            for (int s = 0; s <= w; ++s)
                pops[(int64_t)s * ncells + c] = (lo + s <= Z) ? N[lo + s] : 0.0;
        } else {
            for (int k = 0; k <= Z; ++k) pops[(int64_t)k * ncells + c] = N[k];
        }
        p[c] = (uint8_t)lo;
    }
}

/*
 * Bound on the population that passes slot t of a window during the step in
 * the full chain (Eq. (3) with every level above the window present):
 *     leak(t) = sum_{s <= t, N_s != 0} N_s x_s x_{s+1} ... x_t / (t - s + 1)!,
 * x_k = W_{p+k} dt.  A particle that starts at slot s has passed slot t once
 * the t - s + 1 exponential waiting times of slots s..t sum to at most dt,
 * and that probability is at most prod x / (t - s + 1)! (the density of such
 * a sum is at most prod W u^(n-1)/(n-1)!).  The window with its top at slot t
 * holds that population back (Sec. 3: the top absorbs), and changes nothing
 * below slot t, so leak(t) bounds its difference from the full chain.
 */
static double orc_leak(const double *N, const double *x, int t)
{
    double L = 0.0;
    for (int s = 0; s <= t; ++s) {
        if (N[s] == 0.0) continue;
        double term = N[s];
        for (int k = s; k <= t; ++k) term *= x[k];
        L += term / orc_fact(t - s + 1);
    }
    return L;
}

/*
 * One step with an adaptive window: the reduced system of Sec. 3 ("specified
 * independently for each computational cell"), here with a top that moves up
 * per cell and step so that the population the absorbing top holds back
 * stays below tol.
 *   pops[(wmax+1)][ncells]: slot s holds level p + s for s <= wc (slots above
 *     wc are read as zero and written as zero);
 *   p[ncells]: lowest window level (values above Z read as Z);
 *   wc[ncells]: rates in the window (its top is slot wc).
 * Per cell:
 *   1. window shift at the start of the step (as orc_ionize_step); the top
 *      level stays, so wc drops by the number of shifts (not below 0);
 *   2. t0 = min(max(wmin, wc), Z - p);
 *   3. top = t0, then while top < min(wmax, Z - p) and not leak(top) <= tol:
 *      top += 1 (a NaN leak widens);
 *   4. exact solve of the window [p, p + top], top absorbing;
 *   5. slots 0..wmax stored (zero above top), wc = top.
 * force_top (may be NULL): a value >= 0 replaces step 3 for that cell.
 * top_out, leak_top, leak_below (may be NULL): the top taken, leak at it,
 * and leak one slot lower (-1 when top == t0).  leaks (may be NULL,
 * [(wmax+1)][ncells]): leak(t) for t = t0..room after the shift, -1 elsewhere.
 */
void orc_adaptive_step(int Z, const double *U, const int8_t *l, const int8_t *m, const double *consts,
                       int64_t ncells, const double *E, double dt, int wmin, int wmax, double eps, double tol,
                       double *pops, uint8_t *p, uint8_t *wc, const int *force_top, int *top_out,
                       double *leak_top, double *leak_below, double *leaks)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < ncells; ++c) {
        double N[ORC_MAXN], x[ORC_MAXN], W[ORC_MAXN];
        for (int k = 0; k < ORC_MAXN; ++k) N[k] = 0.0;
        int lo = p[c] > Z ? Z : p[c];
        int w = wc[c] > wmax ? wmax : wc[c];
        for (int s = 0; s <= w; ++s)
            if (lo + s <= Z) N[s] = pops[(int64_t)s * ncells + c];
        /* window shift at the start of the step, residual folded upward */
        while (lo < Z && N[0] < eps) {
            N[1] += N[0];
            for (int s = 0; s < wmax; ++s) N[s] = N[s + 1];
            N[wmax] = 0.0;
            ++lo;
            w = w > 0 ? w - 1 : 0;
        }
        const int room = Z - lo < wmax ? Z - lo : wmax;
        int t0 = w > wmin ? w : wmin;
        if (t0 > Z - lo) t0 = Z - lo;
        for (int k = 0; k <= room && lo + k < Z; ++k) {
            W[k] = orc_level_rate(U[lo + k], lo + k + 1, l[lo + k], m[lo + k], E[c], consts);
            x[k] = W[k] * dt;
        }
        if (leaks)
            for (int t = 0; t <= wmax; ++t)
                leaks[(int64_t)t * ncells + c] = (t >= t0 && t <= room) ? orc_leak(N, x, t) : -1.0;
        int top = t0;
        if (force_top && force_top[c] >= 0) {
            top = force_top[c];
        } else {
            while (top < room && !(orc_leak(N, x, top) <= tol)) ++top;
        }
        if (top_out) top_out[c] = top;
        if (leak_top) leak_top[c] = lo + top < Z ? orc_leak(N, x, top) : 0.0;
        if (leak_below) leak_below[c] = top > t0 ? orc_leak(N, x, top - 1) : -1.0;
        orc_advance_window(top + 1, W, dt, N);
        for (int s = 0; s <= wmax; ++s) pops[(int64_t)s * ncells + c] = s <= top ? N[s] : 0.0;
        p[c] = (uint8_t)lo;
        wc[c] = (uint8_t)top;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
