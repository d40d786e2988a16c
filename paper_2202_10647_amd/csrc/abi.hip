// C-ABI entry points of libadkion: host validation (before any device call),
// gas objects, and dispatch to the per-(precision, window) kernel
// instantiations compiled from inst.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "kernels.hpp"

// Adaptive window (adapt.hip).
hipError_t adk_step_adaptive(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                             uint8_t *wc, const adk_adaptive *win, void *work, unsigned long long *counters,
                             hipStream_t st);
size_t adk_adaptive_work_bytes_impl(int64_t ncells);
// Chain advance for windows wider than ADK_MAX_W (wide.hip).
hipError_t adk_advance_wide(int w, const void *Wr, int64_t n, double dt, void *pops, adk_prec prec, hipStream_t st);

namespace adk {

// ---------------------------------------------------------------------------
static int g_num_cu = 0;

int num_cus()
{
    if (g_num_cu <= 0) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            g_num_cu = cu;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

int grid_for(int64_t n)
{
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)num_cus() * 8;
    return (int)(blocks < cap ? blocks : cap);
}

ChunkOrder chunk_order(int64_t n, int64_t chunk)
{
    ChunkOrder o;
    o.chunks = n / chunk;
    o.bits = 0;
    if (o.chunks >= 2 && o.chunks <= ((int64_t)1 << 31))
        while (((int64_t)1 << o.bits) < o.chunks) ++o.bits;
    return o;
}

WinCut window_cutoffs(const adk_gas *g, double dt, int w)
{
    adk_gas *mg = const_cast<adk_gas *>(g);
    std::lock_guard<std::mutex> lock(mg->cut_mu);
    if (mg->wcut_dt != dt || mg->wcut_w != w) {
        float lvl[ADK_MAX_Z];
        level_thresholds(*g, dt, kIdentityRate, lvl);  // rounded down per level
        for (int p = 0; p <= ADK_MAX_Z; ++p) {
            float e = 0.0f;  // p >= Z: fully stripped, never compared
            if (p < g->Z) {
                e = INFINITY;
                for (int k = p; k < p + w && k < g->Z; ++k) e = std::fmin(e, lvl[k]);
            }
            mg->wcut[p] = e;
        }
        mg->wcut_dt = dt;
        mg->wcut_w = w;
    }
    WinCut c;
    for (int p = 0; p <= ADK_MAX_Z; ++p) c.e[p] = mg->wcut[p];
    return c;
}

StepArgs step_args(const adk_gas *g, double dt, double eps)
{
    StepArgs a;
    a.tab = g->d_coef;
    a.Z = g->Z;
    a.has_poly = g->has_poly;
    a.ln_dt = std::log(dt);
    a.eps = eps;
    adk_gas *mg = const_cast<adk_gas *>(g);
    std::lock_guard<std::mutex> lock(mg->cut_mu);
    if (mg->cut_dt != dt) {
        mg->cut_E = field_cutoff(*g, dt);
        mg->cut_dt = dt;
    }
    a.E_cut = mg->cut_E;
    return a;
}

// Reduction table of fast_log2: bin j of the mantissa m in [1/2, 1) (top six
// fraction bits) has centre m_j = (1 + (j + 1/2)/64)/2; c_j is 1/m_j rounded
// to a float (so that m c_j is exact for float inputs) and -log2 c_j is
// evaluated in long double.
static void log2_table(double *t)
{
    for (int j = 0; j < kLogTable; ++j) {
        const double mj = 0.5 * (1.0 + (j + 0.5) / kLogTable);
        const double c = (double)(float)(1.0 / mj);
        t[2 * j] = c;
        t[2 * j + 1] = (double)(-std::log2((long double)c));
    }
}

// Rows of the LDS rate table (see kernels.hpp): for level k,
// a = A log2(e) - alpha log2(E_a) (ln dt log2(e) is added at staging),
// alpha, b = B log2(e) E_a, c_j / E_a^j; rows Z.. have a = -1e300 (rate 0).
static void fold_rows(const adk_gas &g, double *rows)
{
    const double log2e = 1.4426950408889634, Ea = g.consts.E_a, l2Ea = std::log2(Ea);
    for (int k = 0; k < kCoefRows; ++k) {
        double *r = rows + kCoefStride * k;
        for (int f = 0; f < kCoefStride; ++f) r[f] = 0.0;
        if (k < g.Z) {
            const double *c = g.h_coef + 8 * k;
            r[0] = c[0] * log2e - c[1] * l2Ea;
            r[1] = c[1];
            r[2] = c[2] * log2e * Ea;
            r[3] = c[3] / Ea;
            r[4] = c[4] / (Ea * Ea);
            r[5] = c[5] / (Ea * Ea * Ea);
        } else {
            r[0] = -1e300;
        }
    }
}

static const StepFn kStepF64[ADK_MAX_W + 1] = {nullptr, adk_step_f64_1, adk_step_f64_2, adk_step_f64_3,
                                               adk_step_f64_4, adk_step_f64_5, adk_step_f64_6,
                                               adk_step_f64_7, adk_step_f64_8};
static const StepFn kStepMixed[ADK_MAX_W + 1] = {nullptr, adk_step_mixed_1, adk_step_mixed_2, adk_step_mixed_3,
                                                 adk_step_mixed_4, adk_step_mixed_5, adk_step_mixed_6,
                                                 adk_step_mixed_7, adk_step_mixed_8};
static const AdvanceFn kAdvF64[ADK_MAX_W + 1] = {nullptr, adk_advance_f64_1, adk_advance_f64_2,
                                                 adk_advance_f64_3, adk_advance_f64_4, adk_advance_f64_5,
                                                 adk_advance_f64_6, adk_advance_f64_7, adk_advance_f64_8};
static const AdvanceFn kAdvMixed[ADK_MAX_W + 1] = {nullptr, adk_advance_mixed_1, adk_advance_mixed_2,
                                                   adk_advance_mixed_3, adk_advance_mixed_4,
                                                   adk_advance_mixed_5, adk_advance_mixed_6,
                                                   adk_advance_mixed_7, adk_advance_mixed_8};

static int status_of(hipError_t e)
{
    if (e == hipSuccess) return ADK_OK;
    if (e == hipErrorOutOfMemory) return ADK_ENOMEM;
    return ADK_EDEVICE;
}

static bool valid_prec(int p) { return p == ADK_F64 || p == ADK_MIXED; }

}  // namespace adk

using namespace adk;

extern "C" {

const char *adk_version(void) { return "adkion 0.1.0 (gfx950)"; }

const char *adk_strerror(int status)
{
    switch (status) {
    case ADK_OK: return "ok";
    case ADK_EINVAL: return "invalid argument";
    case ADK_ERANGE: return "value out of supported range";
    case ADK_EDEVICE: return "HIP device error";
    case ADK_ENOMEM: return "device allocation failed";
    default: return "unknown status";
    }
}

int adk_gas_create(const adk_gas_desc *desc, const adk_constants *consts, adk_gas **out)
{
    if (!out) return ADK_EINVAL;
    *out = nullptr;
    const int st = validate_desc(desc, consts);
    if (st != ADK_OK) return st;
    adk_gas *g = new (std::nothrow) adk_gas();
    if (!g) return ADK_ENOMEM;
    g->Z = desc->Z;
    g->consts = resolve_constants(consts);
    build_coeffs(*desc, g->consts, g->h_coef);
    for (int k = 0; k < g->Z; ++k)
        if (g->h_coef[8 * k + 3] != 0.0 || g->h_coef[8 * k + 4] != 0.0 || g->h_coef[8 * k + 5] != 0.0)
            g->has_poly = 1;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return ADK_EDEVICE;
    }
    // device buffer: folded rows, then the log2 reduction table
    double staging[kDevTableLen];
    fold_rows(*g, staging);
    log2_table(staging + kCoefRows * kCoefStride);
    const size_t bytes = sizeof(double) * kDevTableLen;
    hipError_t e = hipMalloc((void **)&g->d_coef, bytes);
    if (e != hipSuccess) {
        delete g;
        return status_of(e);
    }
    e = hipMemcpy(g->d_coef, staging, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(g->d_coef);
        delete g;
        return status_of(e);
    }
    *out = g;
    return ADK_OK;
}

int adk_gas_destroy(adk_gas *gas)
{
    if (!gas) return ADK_OK;
    const hipError_t e = gas->d_coef ? hipFree(gas->d_coef) : hipSuccess;
    delete gas;
    return status_of(e);
}

int adk_gas_levels(const adk_gas *gas) { return gas ? gas->Z : ADK_EINVAL; }

int adk_rates(const adk_gas *gas, const void *E, int64_t n, int32_t k0, int32_t nk, void *W_out, adk_prec prec,
              hipStream_t stream)
{
    if (!gas || n < 0 || !valid_prec(prec)) return ADK_EINVAL;
    if (n > 0 && (!E || !W_out)) return ADK_EINVAL;
    if (k0 < 0 || nk < 1 || (int64_t)k0 + nk > gas->Z) return ADK_ERANGE;
    if (n == 0) return ADK_OK;
    const StepArgs a = step_args(gas, 1.0, 0.0);
    if (prec == ADK_F64)
        hipLaunchKernelGGL((rates_kernel<PolicyF64>), dim3(grid_for(n)), dim3(kBlock), 0, stream, a, k0, nk,
                           (const double *)E, (double *)W_out, n);
    else
        hipLaunchKernelGGL((rates_kernel<PolicyMixed>), dim3(grid_for(n)), dim3(kBlock), 0, stream, a, k0, nk,
                           (const float *)E, (float *)W_out, n);
    return status_of(hipGetLastError());
}

int adk_chain_advance(int32_t w, const void *W, int64_t ncells, double dt, void *pops, adk_prec prec,
                      hipStream_t stream)
{
    if (ncells < 0 || !valid_prec(prec)) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (w < 1 || w > ADK_MAX_WIDE_W) return ADK_ERANGE;
    if (ncells > 0 && (!W || !pops)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    if (w > ADK_MAX_W) return status_of(adk_advance_wide(w, W, ncells, dt, pops, prec, stream));
    const hipError_t e = (prec == ADK_F64 ? kAdvF64 : kAdvMixed)[w](W, ncells, dt, pops, stream);
    return status_of(e);
}

int ionize_step(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops, uint8_t *lo,
                const adk_window *win, hipStream_t stream)
{
    if (!gas || !win || ncells < 0) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (!(win->eps >= 0.0) || !std::isfinite(win->eps)) return ADK_EINVAL;
    if (!valid_prec(win->prec)) return ADK_EINVAL;
    if (win->layout != ADK_LAYOUT_COMPACT && win->layout != ADK_LAYOUT_FULL) return ADK_EINVAL;
    if (win->w < 1 || win->w > ADK_MAX_WIDE_W || win->w > gas->Z) return ADK_ERANGE;
    if (ncells > 0 && (!E || !pops || !lo)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    if (win->w > ADK_MAX_W) return status_of(adk_step_wide(gas, E, ncells, dt, pops, lo, win, stream));
    const hipError_t e = (win->prec == ADK_F64 ? kStepF64 : kStepMixed)[win->w](gas, E, ncells, dt, pops, lo,
                                                                               win, nullptr, stream);
    return status_of(e);
}

size_t adk_adaptive_work_bytes(int64_t ncells) { return adk_adaptive_work_bytes_impl(ncells); }

int ionize_step_adaptive(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops, uint8_t *lo,
                         uint8_t *wc, const adk_adaptive *win, void *work, size_t work_bytes,
                         unsigned long long *counters, hipStream_t stream)
{
    if (!gas || !win || ncells < 0) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (!(win->eps >= 0.0) || !std::isfinite(win->eps)) return ADK_EINVAL;
    if (!(win->tol >= 0.0)) return ADK_EINVAL;
    if (!valid_prec(win->prec)) return ADK_EINVAL;
    if (win->wmax < 1 || win->wmax > ADK_MAX_WIDE_W || win->wmax > gas->Z || win->wmin < 0 ||
        win->wmin > win->wmax)
        return ADK_ERANGE;
    if (ncells >= ((int64_t)1 << 31)) return ADK_ERANGE;
    if (ncells > 0 && (!E || !pops || !lo || !wc || !work)) return ADK_EINVAL;
    if (ncells > 0 && work_bytes < adk_adaptive_work_bytes_impl(ncells)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    return status_of(adk_step_adaptive(gas, E, ncells, dt, pops, lo, wc, win, work, counters, stream));
}

int ionize_step_yield(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops, uint8_t *lo,
                      const adk_window *win, void *dne, hipStream_t stream)
{
    if (!win || win->layout != ADK_LAYOUT_COMPACT) return ADK_EINVAL;
    if (ncells > 0 && !dne) return ADK_EINVAL;
    if (!gas || ncells < 0) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (!(win->eps >= 0.0) || !std::isfinite(win->eps)) return ADK_EINVAL;
    if (!valid_prec(win->prec)) return ADK_EINVAL;
    if (win->w < 1 || win->w > ADK_MAX_W || win->w > gas->Z) return ADK_ERANGE;
    if (ncells > 0 && (!E || !pops || !lo)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    const hipError_t e = (win->prec == ADK_F64 ? kStepF64 : kStepMixed)[win->w](gas, E, ncells, dt, pops, lo,
                                                                               win, dne, stream);
    return status_of(e);
}

}  // extern "C"
