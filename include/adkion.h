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

#ifdef __cplusplus
}
#endif
#endif /* ADKION_H */
