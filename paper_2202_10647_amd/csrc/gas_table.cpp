// Host side of the library: gas-table builder (log-domain coefficients of
// Eq. (1)), argument validation helpers and the gas object.
//
// Eq. (1) (Sec. 2) written in logs.  With L = ln(E/E_a), R = E_a/E and
// p = 2n* - |m| - 1 every factor is a power of E or a constant:
//   ln W = A + alpha L - B R
//   alpha = 1/2 - p                      (sqrt(E) factor and the power p of 1/E)
//   B     = (2/3) (Q/n*)^3                (tunnelling exponent)
//   A     = ln omega_a + (1/2) ln(3 n*^3 / (pi Q^3)) + ln(Q^2 / (2 n*^2))
//         + 2n* ln(2e/n*) + ln C_lm + p ln(2 Q^3 / n*^3)
//   C_lm  = (2l+1)(l+|m|)! / (2 pi n* 2^|m| |m|! (l-|m|)!)
// For the m-average (1/(2l+1)) sum_{m=-l..l} W_{l|m|}, the |m| = j term has
// alpha_j = alpha_0 + j and the same B, so the average is
//   W = exp(A_0 + alpha_0 L - B R) (1 + sum_{j>=1} c_j u^j),  u = E/E_a,
// with A_0 including the weight 1/(2l+1) and c_j = exp(A_j - A_0) including
// the weight 2/(2l+1) of the +-j pair.
#include "gas_table.hpp"

#include <cmath>
#include <cstring>

namespace adk {

static double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

static double level_logA(double Q, double ns, int l, int am, const adk_constants &c)
{
    const double p = 2.0 * ns - am - 1.0;
    const double Clm = (2.0 * l + 1.0) * factorial(l + am) /
                       (2.0 * M_PI * ns * std::ldexp(1.0, am) * factorial(am) * factorial(l - am));
    return std::log(c.omega_a) + 0.5 * std::log(3.0 * ns * ns * ns / (M_PI * Q * Q * Q)) +
           std::log(Q * Q / (2.0 * ns * ns)) + 2.0 * ns * std::log(2.0 * M_E / ns) + std::log(Clm) +
           p * std::log(2.0 * Q * Q * Q / (ns * ns * ns));
}

adk_constants resolve_constants(const adk_constants *consts)
{
    if (consts) return *consts;
    adk_constants c;
    c.omega_a = 4.13e16;
    c.E_a = 510.0;
    c.U_H = 27.21 / 2.0;
    return c;
}

int validate_desc(const adk_gas_desc *d, const adk_constants *consts)
{
    if (!d) return ADK_EINVAL;
    if (d->Z < 1 || d->Z > ADK_MAX_Z) return ADK_ERANGE;
    if (!d->U_eV || !d->l || !d->m) return ADK_EINVAL;
    for (int k = 0; k < d->Z; ++k) {
        const double U = d->U_eV[k];
        if (!(U > 0.0) || !std::isfinite(U)) return ADK_EINVAL;
        const int l = d->l[k], m = d->m[k];
        if (l < 0 || l > 3) return ADK_EINVAL;
        if (m != ADK_M_AVERAGE && (m < 0 || m > l)) return ADK_EINVAL;
    }
    if (consts) {
        if (!(consts->omega_a > 0.0) || !std::isfinite(consts->omega_a)) return ADK_EINVAL;
        if (!(consts->E_a > 0.0) || !std::isfinite(consts->E_a)) return ADK_EINVAL;
        if (!(consts->U_H > 0.0) || !std::isfinite(consts->U_H)) return ADK_EINVAL;
    }
    return ADK_OK;
}

void build_coeffs(const adk_gas_desc &d, const adk_constants &c, double *coef)
{
    for (int k = 0; k < d.Z; ++k) {
        double *out = coef + 8 * k;
        for (int i = 0; i < 8; ++i) out[i] = 0.0;
        const double Q = (double)(k + 1);
        const double ns = Q * std::sqrt(c.U_H / d.U_eV[k]);
        const int l = d.l[k];
        const double B = (2.0 / 3.0) * std::pow(Q / ns, 3.0);
        if (d.m[k] == ADK_M_AVERAGE) {
            const double A0 = level_logA(Q, ns, l, 0, c) + std::log(1.0 / (2.0 * l + 1.0));
            out[0] = A0;
            out[1] = 1.5 - 2.0 * ns;
            for (int j = 1; j <= l; ++j) {
                const double Aj = level_logA(Q, ns, l, j, c) + std::log(2.0 / (2.0 * l + 1.0));
                out[2 + j] = std::exp(Aj - A0);
            }
        } else {
            const int am = d.m[k];
            out[0] = level_logA(Q, ns, l, am, c);
            out[1] = 1.5 - 2.0 * ns + am;
        }
        out[2] = B;
    }
}

// Field below which the rate of every level is below 1e-30 per step.  Per
// level the base-2 exponent t(u) = a2 + alpha log2 u - b2/u (u = E/E_a)
// increases up to u* = b2 ln2 / (-alpha) (all u when alpha >= 0), and the
// m-average factor increases with u, so ln(W dt) is increasing on (0, u*]:
// bisection on ln u gives the crossing of ln(1e-30), or u* when the level
// stays below it.  The minimum over the levels (less a margin) is returned.
double field_cutoff(const adk_gas &g, double dt)
{
    const double target = std::log(1e-30);
    const double ln2 = std::log(2.0), log2e = 1.0 / ln2;
    double cut = INFINITY;
    for (int k = 0; k < g.Z; ++k) {
        const double *r = g.h_coef + 8 * k;
        const double a2 = (r[0] + std::log(dt)) * log2e, al = r[1], b2 = r[2] * log2e;
        auto lnx = [&](double lu) {
            const double u = std::exp(lu);
            const double poly = 1.0 + u * (r[3] + u * (r[4] + u * r[5]));
            return (a2 + al * lu * log2e - b2 / u) * ln2 + std::log(poly);
        };
        const double lu_star = al < 0.0 ? std::log(b2 * ln2 / -al) : std::log(1e8);
        double lo = std::log(1e-30), hi = lu_star;
        if (!(lnx(hi) > target)) {
            cut = std::fmin(cut, std::exp(hi));
            continue;
        }
        if (lnx(lo) > target) return 0.0;  // no usable cutoff
        for (int it = 0; it < 200 && hi - lo > 1e-12; ++it) {
            const double mid = 0.5 * (lo + hi);
            (lnx(mid) > target ? hi : lo) = mid;
        }
        cut = std::fmin(cut, std::exp(lo));
    }
    if (!std::isfinite(cut)) cut = 1e8;
    return cut * g.consts.E_a * (1.0 - 1e-9);
}

void level_thresholds(const adk_gas &g, double dt, double theta, float *thr)
{
    const double target = std::log(theta);
    const double ln2 = std::log(2.0), log2e = 1.0 / ln2;
    for (int k = 0; k < g.Z; ++k) {
        const double *r = g.h_coef + 8 * k;
        const double a2 = (r[0] + std::log(dt)) * log2e, al = r[1], b2 = r[2] * log2e;
        auto lnx = [&](double lu) {
            const double u = std::exp(lu);
            const double poly = 1.0 + u * (r[3] + u * (r[4] + u * r[5]));
            return (a2 + al * lu * log2e - b2 / u) * ln2 + std::log(poly);
        };
        const double lu_star = al < 0.0 ? std::log(b2 * ln2 / -al) : std::log(1e8);
        double lo = std::log(1e-30), hi = lu_star;
        if (!(lnx(hi) > target)) {  // below theta at every field
            thr[k] = INFINITY;
            continue;
        }
        if (lnx(lo) > target) {
            thr[k] = 0.0f;
            continue;
        }
        for (int it = 0; it < 200 && hi - lo > 1e-12; ++it) {
            const double mid = 0.5 * (lo + hi);
            (lnx(mid) > target ? hi : lo) = mid;
        }
        // rounded down: every field below thr[k] is below the crossing
        thr[k] = std::nextafter((float)(std::exp(lo) * g.consts.E_a * (1.0 - 1e-9)), 0.0f);
    }
}

}  // namespace adk

extern "C" int adk_gas_coeffs(const adk_gas_desc *desc, const adk_constants *consts, double *coef_out)
{
    const int st = adk::validate_desc(desc, consts);
    if (st != ADK_OK) return st;
    if (!coef_out) return ADK_EINVAL;
    adk::build_coeffs(*desc, adk::resolve_constants(consts), coef_out);
    return ADK_OK;
}
