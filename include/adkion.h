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

#include <stddef.h>
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
#define ADK_MAX_WIDE_W 63 /* widest window of ionize_step (w > ADK_MAX_W: one wavefront per cell) */
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
    int32_t w;       /* 1 <= w <= min(Z, ADK_MAX_WIDE_W)  */
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
 * zero and crossing rates.  Windows up to ADK_MAX_W rates run one cell per
 * lane, wider ones (up to ADK_MAX_WIDE_W) one cell per wavefront in double
 * arithmetic; there a table of divided differences whose rounding bound
 * exceeds 1e-13 (dozens of rates within a band of a few tens per step) is
 * recomputed by scaling and squaring.  Errors: ADK_EINVAL (null pointers
 * with ncells > 0, ncells < 0, dt <= 0 or non-finite, bad prec), ADK_ERANGE
 * (w outside [1, ADK_MAX_WIDE_W]). */
int adk_chain_advance(int32_t w, const void *W, int64_t ncells, double dt, void *pops,
                      adk_prec prec, hipStream_t stream);

/* One ionization step for ncells independent cells (the hot path):
 * 1. window shift at the start of the step from the input populations;
 * 2. rates of levels lo..top-1 from E[c] by Eq. (1), frozen over dt;
 * 3. pops of levels lo..top <- expm(dt A) pops (analytic solution).
 * E[ncells], pops (see adk_layout) and lo[ncells] (uint8, lowest window level
 * p; values above Z are read as Z) are device arrays; pops and lo are updated
 * in place.  ncells == 0 is a no-op.  Non-finite E gives non-finite
 * populations in that cell only.  Windows up to ADK_MAX_W rates run one cell
 * per lane; wider windows (up to ADK_MAX_WIDE_W, so w = Z with eps = 0 is the
 * full chain of Sec. 3's comparison for Z <= 63) run one cell per wavefront,
 * in double arithmetic for either precision.  A cell with no shift due whose
 * window rates are all below 1e-16 per step (windows up to ADK_MAX_W) keeps
 * its populations: the exact step would change them by less than 3e-16.
 * Errors: ADK_EINVAL (null pointers with ncells > 0, ncells < 0, dt <= 0 or
 * non-finite, eps < 0 or non-finite, bad enums), ADK_ERANGE (w outside
 * [1, min(Z, ADK_MAX_WIDE_W)]). */
int ionize_step(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops,
                uint8_t *lo, const adk_window *win, hipStream_t stream);

/* ionize_step (compact layout) that also writes each cell's electron yield
 * of the step, the quantity the particle code downstream turns into new
 * electrons (Sec. 1 and Sec. 4; electron density from the charge-state
 * populations, Fig. 2(c)): dne[c] = sum_s (lo'+s) N'_s - sum_s (lo+s) N_s,
 * the change of the mean charge per atom (lo' and N' after the step, lo read
 * as min(lo, Z)).  dne[ncells] is a device array of the precision's type,
 * computed in double from the same registers as the populations.  Errors: as
 * ionize_step (but w at most ADK_MAX_W), and ADK_EINVAL for a layout other
 * than ADK_LAYOUT_COMPACT or a null dne with ncells > 0. */
int ionize_step_yield(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops,
                      uint8_t *lo, const adk_window *win, void *dne, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Adaptive window.  The reduced system of Sec. 3 is "specified independently
 * for each computational cell"; here each cell's window also chooses its own
 * width, step by step, so that it follows populations that spread over more
 * levels than a fixed window holds (a slowly ionizing level below a fast
 * cascade).  Per cell and step:
 *   1. the window shift at the start of the step (cut-off criterion after
 *      Eq. (9), as ionize_step); the top level stays, so the width wc drops
 *      by the number of shifts (not below 0);
 *   2. the top slot t starts at min(max(wmin, wc), Z - lo) and moves up,
 *      at most to min(wmax, Z - lo), while leak(t) > tol (or is NaN), where
 *        leak(t) = sum_{s <= t, N_s != 0} N_s x_s x_{s+1} ... x_t / (t-s+1)!,
 *      x_k = W_{lo+k} dt, bounds the population the full chain (Eq. (3)
 *      with every level) moves past slot t within the step: the absorbing
 *      top holds back at most leak(t), and below the top the window's
 *      solution is the full chain's;
 *   3. the window [lo, lo + t] is solved exactly (Eqs. (4)-(5)), top
 *      absorbing; wc = t.
 * With tol = 0 and wmax >= Z - lo the result is the full chain; with
 * wmin = wmax = w it is ionize_step with window w.  Cells whose window fits
 * three rates run one per lane in a sweep of the mesh, those that fit eight
 * one per lane over a list of them, wider ones on 16 lanes each (four cells
 * per wavefront) while their slots fit, else one per wavefront (double
 * arithmetic), up to ADK_MAX_WIDE_W rates.
 */
typedef struct {
    int32_t wmin; /* 0 <= wmin <= wmax: narrowest window (rates)                 */
    int32_t wmax; /* 1 <= wmax <= min(Z, ADK_MAX_WIDE_W): widest; rows wmax + 1  */
    double eps;   /* shift threshold, >= 0 and finite (as adk_window)            */
    double tol;   /* leak tolerance per step, >= 0 (not NaN)                     */
    adk_prec prec;
} adk_adaptive;

/* Bytes of the device workspace ionize_step_adaptive needs for ncells cells
 * (a bit mask of the cells handed from the first to the second tier, a list
 * of those handed to the third, a list of those the third passes on to the
 * fourth, and their lengths):
 * 256 + 32 ceil(ncells / 256) + 8 ncells. */
size_t adk_adaptive_work_bytes(int64_t ncells);

/* One step with adaptive windows for ncells cells (compact layout):
 * E[ncells], pops[(wmax+1)][ncells] (slot s holds level lo + s for s <= wc;
 * slots above wc are not read and are written as zero when the window
 * leaves them), lo[ncells] (uint8, values above Z read as Z) and wc[ncells]
 * (uint8, rates in the window, values above wmax read as wmax; start with
 * wmin) are device arrays of the precision's type, updated in place.  work
 * is a device buffer of at least adk_adaptive_work_bytes(ncells) bytes that
 * the call uses as scratch (contents need no initialisation; calls sharing
 * one workspace must be ordered).  counters (device, 2 x uint64, may be
 * NULL) are incremented by: [0] cells listed for the wide tiers (window
 * wider than eight rates), [1] cells whose top the storage limit wmax held
 * back with leak above tol.  A cell below the gas's field cutoff (every rate
 * below 1e-30 per step) with no shift due keeps its populations when
 * tol >= 1e-30.  Five launches on stream (clear the lists, lane-per-cell
 * sweep, lane-per-cell tier over the cells it marked, 16-lane tier over the
 * cells that one listed, wavefront-per-cell tier over the cells the 16-lane
 * tier passed on); allocates nothing and never synchronises.  Results do not depend
 * on timing: repeated calls on the same inputs agree bit for bit.
 * Errors: ADK_EINVAL (null gas/win, null arrays or work with ncells > 0,
 * ncells < 0, work_bytes too small, dt <= 0 or non-finite, eps < 0 or
 * non-finite, tol < 0 or NaN, bad prec), ADK_ERANGE (wmin/wmax outside the
 * ranges above, ncells >= 2^31). */
int ionize_step_adaptive(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops, uint8_t *lo,
                         uint8_t *wc, const adk_adaptive *win, void *work, size_t work_bytes,
                         unsigned long long *counters, hipStream_t stream);

/* Comparison baseline, not the method: ionize_step (compact layout, ADK_F64)
 * with the chain integrated by nsub explicit classical Runge-Kutta substeps
 * of dt/nsub instead of its analytic solution (rates frozen over the step,
 * window shift and top as in ionize_step).  Sub-cycled time stepping of
 * the rate equations is what the exact solution of Sec. 3 replaces (Sec. 1);
 * this entry point measures that cost and its error on identical inputs.
 * Arrays as ionize_step (double).  Errors: as ionize_step, and ADK_EINVAL
 * for nsub < 1, a precision other than ADK_F64 or a layout other than
 * ADK_LAYOUT_COMPACT. */
int adk_subcycle_step(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops, uint8_t *lo,
                      const adk_window *win, int32_t nsub, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched step over cells of several gases with uneven window widths.
 * Cells are independent (Sec. 3), so one launch can serve a mesh whose cells
 * carry different gases (for example a dopant in a host gas) and different
 * window widths w (Sec. 3, reduced system of 3 or 4 levels, chosen per cell).
 */
#define ADK_PLAN_MAX_GAS 8
#define ADK_PLAN_MAX_W 6
/* A window width with at least this many cells gets a launch of its own,
 * compiled for that width; runs of smaller widths share one launch compiled
 * for the widest of them. */
#define ADK_PLAN_SOLO_CELLS (1 << 19)
/* Storage order of the arrays a plan steps (adk_plan_create's layout):
 * ADK_PLAN_MESH_ORDER: E, pops and lo are indexed by mesh cell; each tile
 *   gathers its cells through the plan's permutation (a sparse dopant's
 *   cells lie scattered over many cache lines).
 * ADK_PLAN_GROUPED: the arrays hold the cells in the plan's order
 *   (adk_plan_order), each (gas, w) group contiguous, as a code that stores
 *   each species' cells in arrays of its own does; every access of a tile
 *   is then contiguous.  The caller keeps its populations in that order
 *   and supplies the field in it. */
#define ADK_PLAN_MESH_ORDER 0
#define ADK_PLAN_GROUPED 1

typedef struct adk_plan adk_plan; /* opaque: grouping of the cells, tiles, tuning */

typedef struct {
    int32_t ngas;            /* gases of the plan                                     */
    int32_t nbuckets;        /* non-empty (gas, w) groups                             */
    int32_t ntiles;          /* tiles of cells_per_lane * 256 cells of one group      */
    int32_t cells_per_lane;  /* of the launch with the most cells (1, 2 or 4)         */
    int32_t grid;            /* workgroups of the launch with the most cells (= tiles) */
    int32_t rows;            /* population rows of the plan layout: max w + 1         */
    int32_t from_cache;      /* 1 when every tuned launch's choice came from the cache */
    double tuned_us;         /* sum of the best trial times of the tuned launches     */
    int32_t nlaunches;       /* kernel launches per step (launch groups)              */
    /* per launch, in launch order (widest windows first): */
    int32_t launch_wmax[ADK_PLAN_MAX_W];   /* widest window it serves              */
    int32_t launch_cpl[ADK_PLAN_MAX_W];    /* cells per lane (1, 2 or 4)            */
    int32_t launch_grid[ADK_PLAN_MAX_W];   /* workgroups (one per tile)             */
    int32_t launch_tiles[ADK_PLAN_MAX_W];  /* tiles                                 */
    int64_t launch_cells[ADK_PLAN_MAX_W];  /* cells                                 */
    int32_t layout;                        /* ADK_PLAN_MESH_ORDER or ADK_PLAN_GROUPED */
} adk_plan_info;

/* Create a plan over ncells cells: cell c uses gases[cell_gas[c]] with window
 * width cell_w[c] (1 <= w <= min(Z, ADK_PLAN_MAX_W)).  gases (host array of
 * ngas handles, which must outlive the plan), cell_gas and cell_w are host
 * arrays read during the call.  Populations use the compact layout with
 * info.rows rows: pops[rows][ncells], slot s of cell c = level lo[c] + s for
 * s <= cell_w[c] (other rows are not touched).  The widths are split into
 * launch groups (ADK_PLAN_SOLO_CELLS).  cells_per_lane = 0 runs the
 * autotuner for each launch group (timed trials on scratch device buffers of
 * the plan's size; result cached in the file named by ADK_TUNE_CACHE when
 * set; a line of that file that does not parse is skipped), 1, 2 or 4
 * fixes it for every launch.  layout: ADK_PLAN_MESH_ORDER or
 * ADK_PLAN_GROUPED (the order of the arrays adk_plan_step is given; cell_gas
 * and cell_w are always in mesh order).  Synchronous; allocates device
 * memory.  Errors: ADK_EINVAL (null pointers, bad prec, eps < 0 or
 * non-finite, cells_per_lane not in {0,1,2,4}, unknown layout), ADK_ERANGE (ngas outside
 * [1, ADK_PLAN_MAX_GAS], a cell's gas index or width out of range,
 * ncells >= 2^31 - 256), ADK_EDEVICE/ADK_ENOMEM. */
int adk_plan_create(const adk_gas *const *gases, int32_t ngas, const uint8_t *cell_gas, const uint8_t *cell_w,
                    int64_t ncells, adk_prec prec, double eps, int32_t cells_per_lane, int32_t layout,
                    adk_plan **out);

/* The plan's cell order: order[i] = the mesh cell (index into cell_gas /
 * cell_w of adk_plan_create) at plan position i, for i < ncells; each
 * (gas, w) group is one contiguous run, mesh order kept within it.  With
 * ADK_PLAN_GROUPED, element i of E, lo and every pops row belongs to mesh
 * cell order[i].  order: host array of ncells int32, written.  Errors:
 * ADK_EINVAL (null plan, null order with ncells > 0). */
int adk_plan_order(const adk_plan *plan, int32_t *order);

/* One ionization step of every cell of the plan (same semantics per cell as
 * ionize_step with the cell's gas and width): one launch per launch group
 * (one workgroup per tile).  The launch group with the most cells runs on
 * stream; the others run on a stream of the plan that is forked from stream
 * (an event recorded on stream) and joined back into it (stream waits on an
 * event recorded after them), so the sparse groups overlap the dense one and
 * the step as a whole is ordered on stream like a single launch.
 * E[ncells], pops[rows][ncells], lo[ncells] are device arrays of the plan's
 * precision.  Allocates nothing and never synchronises, so it may be captured
 * into a hipGraph (the fork and join become parallel branches); consecutive
 * steps of one plan must be ordered (one stream), and one plan must not be
 * stepped from several host threads at once (its side stream and events are
 * shared).  Errors: ADK_EINVAL (null plan or arrays, dt <= 0 or non-finite),
 * ADK_EDEVICE. */
int adk_plan_step(adk_plan *plan, const void *E, double dt, void *pops, uint8_t *lo, hipStream_t stream);

/* hipGraph path of the batched step: nsteps more steps of the plan with the
 * arguments of its last adk_plan_step (same E, dt, pops, lo: a field held
 * constant over nsteps steps, e.g. an ionization sub-cycle inside one field
 * step), launched as one graph on stream.  The graph (every launch group of
 * every step, the side-stream fork and join as parallel branches) is captured
 * on the plan's own stream on first use and cached; it is captured again when
 * nsteps or the last step's arguments change.  When stream is itself being
 * captured, the steps are enqueued on it directly (they join the caller's
 * graph).  Results equal nsteps calls of adk_plan_step bit for bit.
 * nsteps == 0 is a no-op.  Errors: ADK_EINVAL (null plan, nsteps < 0, no
 * adk_plan_step before), ADK_EDEVICE. */
int adk_plan_graph_replay(adk_plan *plan, int32_t nsteps, hipStream_t stream);

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


/* Hardware ceilings for the measurement harness (not part of the method).
 * adk_ceiling_copy: reps passes of a 16-byte-per-lane streaming copy of
 * `bytes` bytes from src to dst (device buffers, not overlapping; bytes a
 * multiple of 16).  One pass (one 4 KiB block per workgroup, in address
 * order) over a large buffer measures the HBM bandwidth, several passes (a
 * grid-stride loop of resident workgroups) over a buffer that fits the
 * 256 MB Infinity Cache its bandwidth; bytes moved = 2 x bytes x reps.
 * adk_ceiling_valu: nlanes lanes (a multiple of 256) each run 8 independent
 * chains of `iters` steps: kind 0 x <- fma(x, 1, 0) in float, kind 1 the
 * same in double, kind 2 x <- exp2(fma(x, 0, 0)) in float; out[nlanes] (float
 * for kinds 0 and 2, double for kind 1) receives 8 per lane.  Work per launch:
 * 16 x iters x nlanes flops (kinds 0, 1) or 8 x iters x nlanes exp2 (kind 2).
 * Both are asynchronous on stream.  Errors: ADK_EINVAL (null buffers, bytes
 * not a multiple of 16 or negative, reps < 1, kind not 0..2, iters < 0,
 * nlanes not a positive multiple of 256), ADK_ERANGE (more than 2^30
 * workgroups), ADK_EDEVICE. */
int adk_ceiling_copy(void *dst, const void *src, int64_t bytes, int64_t reps, hipStream_t stream);
int adk_ceiling_valu(int32_t kind, int64_t iters, void *out, int64_t nlanes, hipStream_t stream);


/* ---------------------------------------------------------------------------
 * Band-column surrogate.  The exact step (Eqs. (2)-(5)) moves the population
 * of a source level k to k, k+1, k+2, ...; within the reduced window of
 * Sec. 3 (three rates, absorbing top) only four destinations matter: k, k+1,
 * k+2 and "k+3 or beyond", which the window top absorbs.  A small network
 * predicts that column, P(k -> k+d), d = 0..3, from (|E|, dt, k):
 *
 *   u = log10|E| and v = log10(dt omega_a) (dt in units of tau_a = 1/omega_a),
 *       each mapped from its trained range onto [-1, 1];
 *   z1 = W1u u + W1v v + W1e emb[k] + b1, h1 = relu(z1)   (FP32)
 *   h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3), z4 = W4 h3 + b4
 *        (bfloat16 operands on the matrix cores, FP32 accumulation)
 *   P = softmax(z4)  (FP32): non-negative, sums to 1, so a step built from such
 *        columns conserves the total population.
 *
 * Parameters: one flat FP32 vector, weights stored [out][in], blocks in this
 * order: emb[Z][16], W1u[64], W1v[64], W1e[64][16], b1[64], W2[64][64],
 * b2[64], W3[64][64], b3[64], W4[4][64], b4[4]; adk_mlp_nparams(Z) entries.
 * Training minimises the batch mean of the cross entropy -sum_d P_d log Q_d
 * against exact columns from the FP64 analytic solver, with Adam (Kingma &
 * Ba 2015) and a cosine learning-rate schedule.  Every reduction of the
 * training step has a fixed order, so training is bitwise reproducible.
 */
#define ADK_MLP_HIDDEN 64
#define ADK_MLP_EMB 16
#define ADK_MLP_BAND 4

typedef struct adk_mlp adk_mlp; /* opaque: FP32 master weights, Adam moments, training buffers.
                                  * Calls on one network use its scratch buffers: order them (one
                                  * stream, or synchronise between streams). */

typedef struct {
    double E_lo, E_hi;   /* trained field range, GV/m (0 < E_lo < E_hi)        */
    double dt_lo, dt_hi; /* trained step range, s (0 < dt_lo < dt_hi)         */
} adk_mlp_range;         /* NULL => [10, 5000] GV/m and [0.02, 0.2] fs          */

typedef struct {
    int64_t nsamples;    /* training set size (samples 0..nsamples-1 of seed)  */
    int32_t iters;       /* Adam steps to take in this call                     */
    int32_t total_iters; /* horizon of the cosine schedule (>= 1)               */
    int32_t batch;       /* samples per step, 1..nsamples                       */
    double lr, lr_min;   /* schedule lr(t) = lr_min + (lr - lr_min)(1 + cos(pi min(t,T)/T))/2 */
    uint64_t seed;       /* training-set seed                                   */
} adk_train_cfg;

/* Number of FP32 parameters for a gas of Z levels: 16 Z + 9796; -1 if Z is
 * outside [1, ADK_MAX_Z]. */
int64_t adk_mlp_nparams(int32_t Z);

/* Create a network for `gas` (its Z and omega_a) from host FP32 parameters
 * params[adk_mlp_nparams(Z)] (copied; initial values are the caller's, e.g. a
 * seeded draw).  range NULL => defaults above.  Adam moments start at zero,
 * step count 0.  Synchronous; allocates device memory.  Errors: ADK_EINVAL
 * (null gas/params/out, range not ordered or not positive/finite, non-finite
 * parameter), ADK_EDEVICE/ADK_ENOMEM. */
int adk_mlp_create(const adk_gas *gas, const float *params, const adk_mlp_range *range, adk_mlp **out);

/* Free a network (NULL accepted); no enqueued work may still use it. */
int adk_mlp_destroy(adk_mlp *mlp);

/* Host copies of the state: params, Adam moments m and v (each
 * [adk_mlp_nparams(Z)], any may be NULL) and the number of Adam steps taken
 * (step may be NULL).  Synchronous.  ADK_EINVAL for a NULL mlp. */
int adk_mlp_get_state(const adk_mlp *mlp, float *params, float *m, float *v, int64_t *step);

/* Exact band columns from the FP64 analytic solver (training targets):
 * for sample i, the step dt[i] of a unit population at level k[i] with a
 * window of three rates and absorbing top (Eqs. (2)-(5) restricted as in
 * Sec. 3), i.e. cols[d][i] = T[k+d, k] for d < 3 and the remainder for d = 3;
 * levels past Z carry no rate.  Device arrays E[n] (double, GV/m), dt[n]
 * (double, s), k[n] (int32, 0 <= k < Z), cols[4][n] (double).  Errors:
 * ADK_EINVAL (null gas or arrays with n > 0, n < 0).  k outside [0, Z) or
 * dt <= 0 yields NaN columns for that sample. */
int adk_band_columns(const adk_gas *gas, const double *E, const double *dt, const int32_t *k, int64_t n,
                     double *cols, hipStream_t stream);

/* Network output Q[4][n] (float, device) for device inputs E[n], dt[n]
 * (double) and k[n] (int32, clamped to [0, Z-1]).  Errors: ADK_EINVAL. */
int adk_mlp_forward(const adk_mlp *mlp, const double *E, const double *dt, const int32_t *k, int64_t n,
                    float *Q, hipStream_t stream);

/* adk_mlp_forward that also writes, for testing the network element by
 * element, each sample's float32 pre-activations of layers 1-3 before their
 * rounding to bfloat16 and its four logits: Zt[n][196] (device floats), row
 * i = z1[64], z2[64], z3[64] (hidden units in order) then z4[4].  Q and the
 * evaluation are those of adk_mlp_forward (the same kernel code).  Errors:
 * ADK_EINVAL. */
int adk_mlp_forward_trace(const adk_mlp *mlp, const double *E, const double *dt, const int32_t *k, int64_t n,
                          float *Q, float *Zt, hipStream_t stream);

/* Loss and gradient of the current parameters over the n given samples
 * (targets from adk_band_columns, computed inside): grad[adk_mlp_nparams(Z)]
 * and loss[1] are device floats.  The backward pass treats the bfloat16
 * rounding of the forward pass as the identity.  Allocates scratch on first
 * use of a larger n.  Errors: ADK_EINVAL (null arguments, n < 1, gas with
 * another Z than the network's), ADK_EDEVICE/ADK_ENOMEM. */
int adk_mlp_loss_grad(adk_mlp *mlp, const adk_gas *gas, const double *E, const double *dt, const int32_t *k,
                      int64_t n, float *grad, float *loss, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): adk_mlp_loss_grad without any allocation.  Same arguments and
 * results as adk_mlp_loss_grad (the same kernels, the same summation order),
 * for n <= ADK_MLP_NOALLOC_MAX_SAMPLES samples; the network is not modified.
 * Its scratch (activations, partial gradients, sample features, about 8.4 MB)
 * is one file-scope device array of the library that each GPU holds until
 * the process ends; every buffer in it is written before it is read, and
 * calls that overlap on one GPU share it and race (order them).  Calls no
 * hipMalloc or hipFree; the first call on a device looks up that device's
 * copy of the array.  Errors: as adk_mlp_loss_grad, ADK_ERANGE for n above
 * the maximum, ADK_EDEVICE when the array cannot be located. */
#define ADK_MLP_NOALLOC_MAX_SAMPLES 4096
int adk_mlp_loss_grad_noalloc(const adk_mlp *mlp, const adk_gas *gas, const double *E, const double *dt,
                              const int32_t *k, int64_t n, float *grad, float *loss, hipStream_t stream);

/* Train on the analytic solver's columns: the training set is samples
 * 0..nsamples-1 of cfg->seed (sample i: E log-uniform in the field range, dt
 * log-uniform in the step range, k uniform in 0..Z-1, from three uniforms
 * u_j = (z >> 11) 2^-53, z the SplitMix64 finaliser of
 * seed + 0x9E3779B97F4A7C15 * (3i + j + 1), j = 0, 1, 2), generated and
 * labelled on the device.  Adam step t (counted over the life of the
 * network, so training may be split over calls or resumed from a saved
 * state) uses batch number t mod floor(nsamples / batch).  Adam: beta1 0.9,
 * beta2 0.999, epsilon 1e-8.  loss_out (host, may be NULL) receives the batch
 * loss of each step taken; the call then synchronises the stream.  Errors:
 * ADK_EINVAL (null arguments, iters < 0, total_iters < 1, batch < 1 or >
 * nsamples, lr or lr_min negative or non-finite, gas with another Z than the
 * network's), ADK_EDEVICE/ADK_ENOMEM. */
int adk_mlp_train(adk_mlp *mlp, const adk_gas *gas, const adk_train_cfg *cfg, float *loss_out,
                  hipStream_t stream);

/* Save the whole state (parameters, Adam moments, step count, ranges) to a
 * binary file; adk_mlp_load restores it for `gas` (same Z) so that further
 * training continues bitwise as if uninterrupted.  Synchronous.  Errors:
 * ADK_EINVAL (null arguments, unreadable/unwritable or malformed file, Z
 * mismatch), ADK_EDEVICE/ADK_ENOMEM. */
int adk_mlp_save(const adk_mlp *mlp, const char *path);
int adk_mlp_load(const adk_gas *gas, const char *path, adk_mlp **out);

/* Rate below which a source level's column is the identity in the
 * surrogate step: W_k dt < ADK_SURROGATE_NEGLIGIBLE on the rising branch of
 * Eq. (1) keeps the level's population to within that fraction. */
#define ADK_SURROGATE_NEGLIGIBLE 1e-9

/* One ionization step in surrogate form (compact layout, float populations):
 * the window shift at the start of the step is that of ionize_step; then a
 * cell whose |E| lies in the trained field range (and dt in the trained step
 * range) advances with band columns, one per source level of its window,
 * destinations past the window top lumped into the top: the network's
 * column, or the identity column for a source level whose rate at this
 * field is negligible (W_k dt < ADK_SURROGATE_NEGLIGIBLE, judged by a
 * per-level field threshold computed on the host once per dt); every other
 * cell takes the analytic step of ionize_step (ADK_MIXED).  win->prec
 * must be ADK_MIXED, win->layout ADK_LAYOUT_COMPACT, 1 <= win->w <= 3.
 * A cell whose |E| lies below its window's identity field (every rate of
 * the window below 1e-16 per step) with no shift due is left unchanged on
 * either path, as ionize_step leaves it.
 * counters (device, 2 x uint64, may be NULL) are incremented by: [0] cells
 * with a window below the top level that took the analytic step (out of the
 * trained range, not left unchanged as above) with |E| at or above the gas's
 * field cutoff (below it the step is only the window shift), [1] (cell,
 * source level) pairs evaluated by the network (negligible sources
 * excluded).
 * Allocates nothing and never synchronises.  Errors: ADK_EINVAL (null
 * arguments with ncells > 0, dt <= 0 or non-finite, eps < 0, prec or layout
 * other than above, network and gas of different Z), ADK_ERANGE (w outside
 * [1, 3] or w > Z). */
int adk_surrogate_step(const adk_gas *gas, const adk_mlp *mlp, const void *E, int64_t ncells, double dt,
                       void *pops, uint8_t *lo, const adk_window *win, unsigned long long *counters,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ADKION_H */
