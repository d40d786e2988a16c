/*
 * adkion.h -- C ABI of the MI355X (gfx950) multi-level ADK ionization library.
 *
 * Method: Cheng & Samulyak, "Efficient numerical algorithm for multi-level
 * ionization of high-atomic-number gases".  Per mesh cell, independently
 * (Sec. 3, remark after Eq. (5)): ADK rates of the charge states from the
 * local field (Eq. (1)), then the exact solution over one step of the linear
 * ionization chain (Eqs. (2)-(3)) with rates frozen over the step (Sec. 3,
 * constant-rate assumption; eigen form Eqs. (4)-(5)), restricted to the
 * locally-reduced window of levels (Sec. 3, reduced system, Eqs. (6)-(9)).
 *
 * Conventions shared by every entry point:
 *   - Return value: ADK_OK (0) or a negative ADK_E* status.  Nothing throws
 *     or aborts.  Arguments are validated on the host before any device call.
 *   - Array arguments are DEVICE pointers owned by the caller (for example the
 *     data pointer of a device tensor) unless a comment says "host".  The
 *     library never frees or keeps them.
 *   - Work is enqueued asynchronously on `stream` (NULL = the null stream);
 *     results are ready after the caller synchronises that stream.
 *   - Units: E in GV/m, dt in s, rates in 1/s, populations are fractions.
 *   - Precision ADK_F64: E, populations and rates are double.
 *     ADK_MIXED: E, populations and rates are float; the rate exponent, the
 *     log/reciprocal of the field and the near-coincident-rate branch of the
 *     chain solution are evaluated in double.
 *   - Layout: structure of arrays, cell index fastest: element (row r, cell c)
 *     is at [r * ncells + c].
 */
#ifndef ADKION_H
#define ADKION_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ADK_OK = 0,
    ADK_EINVAL = -1,  /* invalid argument (null pointer, size, range, enum)    */
    ADK_ERANGE = -2,  /* value outside a supported range (e.g. Z, window width) */
    ADK_EDEVICE = -3, /* a HIP call failed (no device, launch failure, ...)     */
    ADK_ENOMEM = -4   /* device allocation failed                               */
};

#define ADK_MAX_Z 64     /* largest number of ionization levels of a gas        */
#define ADK_MAX_W 8      /* widest window: active rates per cell (populations w+1) */
#define ADK_M_AVERAGE -1 /* projection code: average the rate over m = -l..l     */

/* Physical constants of Eq. (1) (Sec. 2, text after Eq. (1)). */
typedef struct {
    double omega_a; /* atomic unit frequency, 1/s          (paper: 4.13e16) */
    double E_a;     /* atomic unit of field, GV/m          (paper: 510)     */
    double U_H;     /* hydrogen ionization potential, eV   (27.21 / 2)      */
} adk_constants;

/* Level table of one gas (host arrays, read during adk_gas_create only).
 * Level k = 0..Z-1 ionizes charge k -> k+1 and uses Q = k+1 and U_eV[k]
 * (Sec. 2, definitions after Eq. (1)); n* = Q sqrt(U_H / U_eV[k]).
 * l[k] >= 0 is the orbital number of the electron removed, m[k] its projection
 * |m| (0 <= m <= l), or ADK_M_AVERAGE for the equal-weight average over
 * m = -l..l (Sec. 3, quantum numbers per electron, Fig. 1 discussion). */
typedef struct {
    int32_t Z;
    const double *U_eV;
    const int8_t *l;
    const int8_t *m;
} adk_gas_desc;

typedef enum { ADK_F64 = 0, ADK_MIXED = 1 } adk_prec;

/* ADK_LAYOUT_COMPACT: pops[(w+1)][ncells], slot s holds level lo[c] + s
 *   (slots past level Z hold 0).  Levels outside the window are zero by
 *   construction, so this is the paper's reduced per-cell storage (Sec. 3,
 *   memory paragraph: w+1 values and the index p instead of Z+1 values).
 * ADK_LAYOUT_FULL: pops[(Z+1)][ncells], row k holds level k. */
typedef enum { ADK_LAYOUT_COMPACT = 0, ADK_LAYOUT_FULL = 1 } adk_layout;

/* Locally-reduced window (Sec. 3, reduced system and cut-off criterion after
 * Eq. (9)).  w = number of active rates: the window holds populations
 * lo..top with top = min(lo + w, Z), top absorbing within the step; the
 * paper's "4-level system" is w = 3.  eps = shift threshold: at the start of a
 * step, while lo < Z and N_lo < eps, N_lo is added to N_lo+1, set to 0, and lo
 * is incremented (comparison in double). */
typedef struct {
    int32_t w;       /* 1 <= w <= min(Z, ADK_MAX_W)       */
    double eps;      /* >= 0 and finite; 0 disables shifts */
    adk_layout layout;
    adk_prec prec;
} adk_window;

typedef struct adk_gas adk_gas; /* opaque; immutable after create; owns a device table */

/* Library version string (static storage). */
const char *adk_version(void);

/* Text for a status code (static storage). */
const char *adk_strerror(int status);

/* Build the per-level log-domain rate coefficients of Eq. (1) on the host:
 * ln W_k(E) = A_k + alpha_k ln(E/E_a) - B_k E_a/E + ln(1 + sum_j c_kj (E/E_a)^j),
 * coef[k*8 + 0..5] = {A_k, alpha_k, B_k, c_k1, c_k2, c_k3}, coef[k*8+6..7] = 0.
 * Host-only (no device call).  consts may be NULL (paper values).
 * Errors: ADK_EINVAL for null desc/arrays/out, U <= 0 or non-finite, l < 0,
 * l > 3, m outside [0, l] and not ADK_M_AVERAGE; ADK_ERANGE for Z outside
 * [1, ADK_MAX_Z]. */
int adk_gas_coeffs(const adk_gas_desc *desc, const adk_constants *consts, double *coef_out);

/* Create a gas: validates like adk_gas_coeffs, then allocates and uploads the
 * coefficient table to the current device (synchronously).  *out receives
 * the handle; on error *out is set to NULL.  ADK_EDEVICE/ADK_ENOMEM on HIP
 * failure. */
int adk_gas_create(const adk_gas_desc *desc, const adk_constants *consts, adk_gas **out);

/* Destroy a gas and free its device table.  NULL is accepted.  The caller
 * must ensure no enqueued work still uses it. */
int adk_gas_destroy(adk_gas *gas);

/* Number of levels Z of a gas (host), or ADK_EINVAL for NULL. */
int adk_gas_levels(const adk_gas *gas);

/* ADK rates, Eq. (1) (Sec. 2): W_out[j][i] = W_{k0+j}(|E[i]|) in 1/s for
 * j < nk, i < n.  E[n] and W_out[nk][n] are device arrays of the precision's
 * type.  E == 0 gives 0; NaN gives NaN.  Errors: ADK_EINVAL (null pointers
 * with n > 0, n < 0, bad prec), ADK_ERANGE (k0 < 0, nk < 1, k0 + nk > Z). */
int adk_rates(const adk_gas *gas, const void *E, int64_t n, int32_t k0, int32_t nk,
              void *W_out, adk_prec prec, hipStream_t stream);

/* Exact chain advance with given rates (Eqs. (2)-(5) on a window of w+1
 * levels, top absorbing, no window shift): pops[(w+1)][ncells] <-
 * expm(dt A(W)) pops, with W[w][ncells] in 1/s (rates >= 0).  The update is
 * the analytic (Bateman / divided-difference) solution, valid for equal,
 * zero and crossing rates.  Errors: ADK_EINVAL (null pointers with ncells > 0,
 * ncells < 0, dt <= 0 or non-finite, bad prec), ADK_ERANGE (w outside
 * [1, ADK_MAX_W]). */
int adk_chain_advance(int32_t w, const void *W, int64_t ncells, double dt, void *pops,
                      adk_prec prec, hipStream_t stream);

/* One ionization step for ncells independent cells (the hot path):
 * 1. window shift at the start of the step from the input populations;
 * 2. rates of levels lo..top-1 from E[c] by Eq. (1), frozen over dt;
 * 3. pops of levels lo..top <- expm(dt A) pops (analytic solution).
 * E[ncells], pops (see adk_layout) and lo[ncells] (uint8, lowest window level
 * p; values above Z are read as Z) are device arrays; pops and lo are updated
 * in place.  ncells == 0 is a no-op.  Non-finite E gives non-finite
 * populations in that cell only.  Errors: ADK_EINVAL (null pointers with
 * ncells > 0, ncells < 0, dt <= 0 or non-finite, eps < 0 or non-finite, bad
 * enums), ADK_ERANGE (w outside [1, min(Z, ADK_MAX_W)]). */
int ionize_step(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops,
                uint8_t *lo, const adk_window *win, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched step over cells of several gases with uneven window widths.
 * Cells are independent (Sec. 3), so one launch can serve a mesh whose cells
 * carry different gases (for example a dopant in a host gas) and different
 * window widths w (Sec. 3, reduced system of 3 or 4 levels, chosen per cell).
 */
#define ADK_PLAN_MAX_GAS 8
#define ADK_PLAN_MAX_W 6

typedef struct adk_plan adk_plan; /* opaque: grouping of the cells, tiles, tuning */

typedef struct {
    int32_t ngas;            /* gases of the plan                                   */
    int32_t nbuckets;        /* non-empty (gas, w) groups                           */
    int32_t ntiles;          /* tiles of cells_per_lane * 256 cells of one group    */
    int32_t cells_per_lane;  /* 1, 2 or 4 (autotuned, cached, or fixed by caller)   */
    int32_t grid;            /* workgroups of the persistent launch                 */
    int32_t rows;            /* population rows of the plan layout: max w + 1       */
    int32_t from_cache;      /* 1 when cells_per_lane came from ADK_TUNE_CACHE      */
    double tuned_us;         /* best trial launch time of the autotuner (0 if none) */
} adk_plan_info;

/* Create a plan over ncells cells: cell c uses gases[cell_gas[c]] with window
 * width cell_w[c] (1 <= w <= min(Z, ADK_PLAN_MAX_W)).  gases (host array of
 * ngas handles, which must outlive the plan), cell_gas and cell_w are host
 * arrays read during the call.  Populations use the compact layout with
 * info.rows rows: pops[rows][ncells], slot s of cell c = level lo[c] + s for
 * s <= cell_w[c] (other rows are not touched).  cells_per_lane = 0 runs the
 * autotuner (timed trials on scratch device buffers of the plan's size;
 * result cached in the file named by ADK_TUNE_CACHE when set), 1, 2 or 4 fixes
 * it.  Synchronous; allocates device memory.  Errors: ADK_EINVAL (null
 * pointers, bad prec, eps < 0 or non-finite, cells_per_lane not in
 * {0,1,2,4}), ADK_ERANGE (ngas outside [1, ADK_PLAN_MAX_GAS], a cell's gas
 * index or width out of range, ncells >= 2^31 - 256), ADK_EDEVICE/ADK_ENOMEM. */
int adk_plan_create(const adk_gas *const *gases, int32_t ngas, const uint8_t *cell_gas, const uint8_t *cell_w,
                    int64_t ncells, adk_prec prec, double eps, int32_t cells_per_lane, adk_plan **out);

/* One ionization step of every cell of the plan (same semantics per cell as
 * ionize_step with the cell's gas and width): one persistent launch on stream.
 * E[ncells], pops[rows][ncells], lo[ncells] are device arrays of the plan's
 * precision.  Allocates nothing and never synchronises, so it may be captured
 * into a hipGraph; consecutive launches of one plan must be ordered (one
 * stream).  Errors: ADK_EINVAL (null plan or arrays, dt <= 0 or non-finite). */
int adk_plan_step(adk_plan *plan, const void *E, double dt, void *pops, uint8_t *lo, hipStream_t stream);

/* Host query of the plan's grouping and tuning.  ADK_EINVAL for NULL. */
int adk_plan_get_info(const adk_plan *plan, adk_plan_info *info);

/* Free a plan (NULL accepted); no enqueued step may still use it. */
int adk_plan_destroy(adk_plan *plan);

/* Synthetic field generator for tests and benchmarks (an input generator,
 * not part of the method): E[i] = exp(ln E_lo + u (ln E_hi - ln E_lo)) with
 * u = (z >> 11) 2^-53, z the SplitMix64 finaliser of
 * seed + 0x9E3779B97F4A7C15 * (step * n + i + 1) (Steele, Lea & Flood 2014),
 * so every (seed, step, cell) has its own log-uniform value.  Device array E
 * of the precision's type.  Errors: ADK_EINVAL (n < 0, step < 0, E_lo <= 0,
 * E_hi < E_lo, null E with n > 0, bad prec). */
int adk_field_hash(void *E, int64_t n, uint64_t seed, int64_t step, double E_lo, double E_hi, adk_prec prec,
                   hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ADKION_H */
