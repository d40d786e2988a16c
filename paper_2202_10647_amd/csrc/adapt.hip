// Adaptive window (ionize_step_adaptive): the reduced system of Sec. 3, set
// independently for each cell, with a top that moves up per cell and step.
//
// Per cell: the window shift at the start of the step (cut-off criterion
// after Eq. (9)) moves the bottom up and keeps the top level, so the width wc
// drops by the shifts; then the top slot t starts at max(wmin, wc) (clipped
// to level Z) and moves up while the leak
//     leak(t) = sum_{s <= t, N_s != 0} N_s x_s ... x_t / (t - s + 1)!
// exceeds the tolerance (x_k = W_{lo+k} dt).  leak(t) bounds the population
// the full chain moves past slot t within the step (a particle starting at
// slot s has passed slot t once t - s + 1 exponential waiting times sum to
// at most dt, probability at most prod x / (t - s + 1)!), which is exactly
// what the absorbing top holds back: below the top the window's solution is
// the full chain's.  The window [lo, lo + t] is then solved exactly.
//
// Three tiers:
//   * narrow, one lane per cell over the whole mesh: cells whose top stays
//     within slot kNarrowW solve in registers with the narrow path's chain
//     solution (chain_apply), rates above their own top set to zero, which
//     makes the top absorbing and leaves the slots above it empty; the
//     other cells (and cells already wider than kNarrowW) are marked in a
//     bit mask in the workspace (one 64-bit word per wavefront of the sweep)
//     and left untouched;
//   * middle, one lane per marked cell: the same with windows of up to
//     kMidW rates (a register table too large for the mesh-wide sweep,
//     whose occupancy it would cut).  Each workgroup takes a fixed range of
//     mask words and packs its marked cells densely by a prefix sum, so a
//     cell always shares its wavefront with the same cells: the chain
//     solution takes wavefront-wide shortcuts (weak rates, negligible
//     entries, monotone rates), and a fixed grouping keeps every step
//     reproducible bit for bit.  Cells wider still are listed (atomics) for
//   * wide: the wide path's sorted-table solution (chain_sub), up to
//     ADK_MAX_WIDE_W rates, first on 16 lanes per listed cell, four cells
//     per wavefront (every vote, exchange and sum confined to the cell's
//     lanes, a quarter of the LDS per cell, so more cells are in flight per
//     CU); a cell whose slots do not fit 16 lanes is left untouched and
//     listed again, for one wavefront each.  A cell's result does not depend
//     on its place in either list, nor on the cells beside it.
// A step is five launches on the stream: clear the list headers, narrow,
// middle, groups of 16 lanes, wavefronts.  No allocation and no host
// synchronisation, so a step can be captured in a HIP graph.
#include "wide.hpp"

namespace adk {
namespace {

constexpr int kNarrowW = 3;  // widest window the mesh-wide lane-per-cell tier solves
constexpr int kMidW = 8;     // widest window the lane-per-cell tier over listed cells solves

struct AdaptArgs {
    int wmin, wmax;
    double tol;
};

struct AdaptHeader {
    uint32_t count;       // cells listed for the wide tier (groups of 16 lanes)
    uint32_t count_wave;  // cells of that list passed on to one wavefront each
    uint32_t pad[62];
};

// Workspace: the wide tier's list header, the narrow tier's mask (one word
// per wavefront of the sweep: 4 per 256-cell chunk of the scattered order),
// then the wide tier's list and the list of its cells passed on to one
// wavefront each (ncells entries each).
struct AdaptWork {
    AdaptHeader *hdr;
    unsigned long long *mask;
    int32_t *list;
    int32_t *list_wave;
    int64_t nwords;
};

__host__ __device__ inline int64_t adapt_mask_words(int64_t n) { return 4 * ((n + kBlock - 1) / kBlock); }

__host__ __device__ inline AdaptWork adapt_work(void *work, int64_t n)
{
    AdaptWork w;
    w.hdr = (AdaptHeader *)work;
    w.mask = (unsigned long long *)(w.hdr + 1);
    w.nwords = adapt_mask_words(n);
    w.list = (int32_t *)(w.mask + w.nwords);
    w.list_wave = w.list + n;
    return w;
}

__global__ void adaptive_clear_kernel(AdaptHeader *h)
{
    if (threadIdx.x == 0) {
        h->count = 0u;
        h->count_wave = 0u;
    }
}

// Appends the lanes with go set to a list: one atomic per wavefront.  All
// lanes of the wavefront call it.
__device__ __forceinline__ void list_cells(bool go, int64_t c, AdaptHeader *hdr, int32_t *list,
                                           unsigned long long *counters)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(go);
    if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) {
            const int cnt = __popcll(mask);
            base = atomicAdd(&hdr->count, (uint32_t)cnt);
            if (counters) atomicAdd(&counters[0], (unsigned long long)cnt);
        }
        base = __shfl(base, leader);
        if (go) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)c;
    }
}

// leak(t) for t = 0..W of one lane's window (double; products of at most
// W + 1 capped rates stay in range), populations N[0..W], rates x[0..W].
template <int W, class R>
__device__ __forceinline__ void leak_all(const double (&N)[W + 1], const R (&x)[W + 1], double (&L)[W + 1])
{
    static_for<0, W + 1>([&](auto tt) {
        constexpr int t = decltype(tt)::value;
        double acc = 0.0, c = 1.0;
        static_for<0, t + 1>([&](auto qq) {
            constexpr int s = t - decltype(qq)::value;  // s = t, t-1, ..., 0
            constexpr double inv = 1.0 / (t - s + 1);
            c *= (double)x[s] * inv;  // prod x_s..x_t / (t-s+1)!
            acc += N[s] != 0.0 ? N[s] * c : 0.0;
        });
        L[t] = acc;
    });
}

// One cell of a lane-per-cell tier of windows up to W rates (c valid when
// `valid`): shift, top by the leak test, exact solve of the window.  Returns
// true when the cell needs a wider window; it is then left untouched for
// the next tier.
template <class P, int W>
__device__ __forceinline__ bool adaptive_lane_cell(const StepArgs &a, const AdaptArgs &ad, const double *sc,
                                                   const double *slog, int64_t c, bool valid,
                                                   const typename P::real *__restrict__ E,
                                                   typename P::real *__restrict__ pops, uint8_t *__restrict__ lo,
                                                   uint8_t *__restrict__ wc, int64_t n,
                                                   unsigned long long *__restrict__ counters)
{
    using R = typename P::real;
    const int Z = a.Z;
    double EL = 0.0;
    int p = Z, w_in = 0;
    double N[W + 1];
    static_for<0, W + 1>([&](auto ss) { N[decltype(ss)::value] = 0.0; });
    if (valid) {
        EL = fabs((double)E[c]);
        const int l0 = lo[c];
        p = l0 < Z ? l0 : Z;
        const int w0 = wc[c];
        w_in = w0 < ad.wmax ? w0 : ad.wmax;
        N[0] = (double)pops[c];
    }
    // windows already wider than this tier go to the next one
    const bool wide_now = valid && p < Z && w_in > W;
    static_for<1, W + 1>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        if (valid && !wide_now && s <= w_in) N[s] = (double)pops[(int64_t)s * n + c];
    });
    // fully stripped, or every rate of the gas below 1e-30 per step with
    // no shift due: the step moves less than 1e-30 of the population, and
    // with a tolerance of at least 1e-30 the top stays at max(wmin, wc)
    const bool quiet = !valid || p >= Z || (ad.tol >= 1e-30 && EL < a.E_cut && N[0] >= a.eps);
    bool go_wide = wide_now && !quiet;
    if (!__all(quiet) && !quiet && !wide_now) {
        int w = w_in;
        while (p < Z && N[0] < a.eps) {
            N[0] += N[1];
            static_for<1, W>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                N[s] = N[s + 1];
            });
            N[W] = 0.0;
            ++p;
            w = w > 0 ? w - 1 : 0;
        }
        const int room = min(ad.wmax, Z - p);
        const int t0 = min(max(ad.wmin, w), Z - p);
        R x[W + 1];
        const Field f = field_terms<RateEval<P>::kLogTerms>(EL, slog);
        window_rates<P, W + 1>(sc, p, f, a.has_poly != 0, x);
        double L[W + 1];
        leak_all<W>(N, x, L);
        // top: the lowest slot t in [t0, room) with leak(t) <= tol, else
        // room (a NaN leak widens); above slot W it is the next tier's
        int top = t0;
        bool found = false;
        static_for<0, W + 1>([&](auto tt) {
            constexpr int t = decltype(tt)::value;
            if (!found && t >= t0 && t < room) {
                if (L[t] <= ad.tol) found = true;
                else top = t + 1;
            }
        });
        if (!found) top = top > room ? top : room;  // every tested slot leaks: top = room
        if (top > W) {
            go_wide = true;
        } else {
            // the storage limit held the top back (its own leak above tol)
            double Ltop = 0.0;
            static_for<0, W + 1>([&](auto tt) {
                constexpr int t = decltype(tt)::value;
                Ltop = t == top ? L[t] : Ltop;  // selects, not a dynamic index
            });
            if (counters && !found && top < Z - p && !(Ltop <= ad.tol)) atomicAdd(&counters[1], 1ull);
            const bool finite = EL <= 1.7976931348623157e308;
            R xw[W];
            static_for<0, W>([&](auto kk) {
                constexpr int k = decltype(kk)::value;
                xw[k] = k < top ? x[k] : R(0);
            });
            double out[W + 1];
            chain_apply<P, W>(xw, N, out);
            // slots above the top received only rounding residue of the
            // absorbing row: it goes to the top, they hold zero
            double extra = 0.0;
            static_for<1, W + 1>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                const bool above = s > top;
                extra += above ? out[s] : 0.0;
                out[s] = above ? 0.0 : out[s];
            });
            static_for<0, W + 1>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                out[s] += s == top ? extra : 0.0;
            });
            const int wst = max(w_in, top);
            static_for<0, W + 1>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                if (s <= wst) pops[(int64_t)s * n + c] = finite ? (R)out[s] : R(NAN);
            });
            lo[c] = (uint8_t)p;
            wc[c] = (uint8_t)top;
        }
    }
    if (valid && quiet) {
        // T = I: only an index past Z or a width below wmin changes
        const int w_new = p >= Z ? 0 : min(max(ad.wmin, w_in), Z - p);
        if (p != lo[c]) lo[c] = (uint8_t)p;
        if (w_new != wc[c]) wc[c] = (uint8_t)w_new;
    }
    return go_wide;
}

// Narrow tier: every cell of the mesh, one lane each, in the scattered
// chunk order of the step kernel; wider cells go to the middle tier's list.
template <class P>
__global__ __launch_bounds__(kBlock) void adaptive_narrow_kernel(StepArgs a, AdaptArgs ad, ChunkOrder ord,
                                                                 const typename P::real *__restrict__ E,
                                                                 typename P::real *__restrict__ pops,
                                                                 uint8_t *__restrict__ lo, uint8_t *__restrict__ wc,
                                                                 int64_t n,
                                                                 unsigned long long *__restrict__ mask,
                                                                 unsigned long long *__restrict__ counters)
{
    __shared__ double sc[kDevTableLen];
    const double *slog = sc + kCoefRows * kCoefStride;
    stage_coefficients(sc, a.tab, a.ln_dt);
    const int64_t nv = (n + kBlock - 1) / kBlock;
    for (int64_t v = blockIdx.x; v < nv; v += gridDim.x) {
        const int64_t c = chunk_place(v, ord) * kBlock + threadIdx.x;
        const bool go = adaptive_lane_cell<P, kNarrowW>(a, ad, sc, slog, c, c < n, E, pops, lo, wc, n, counters);
        const unsigned long long m = __ballot(go);
        if ((threadIdx.x & 63) == 0) mask[v * 4 + (threadIdx.x >> 6)] = m;  // every word, every step
    }
}

// Position of the k-th set bit (k < popcount) of a 64-bit word.
__device__ __forceinline__ int select_bit(unsigned long long w, unsigned k)
{
    int pos = 0;
    static_for<0, 6>([&](auto ii) {
        constexpr int half = 32 >> decltype(ii)::value;
        const unsigned low = (unsigned)__popcll(w & ((1ull << half) - 1ull));
        if (k >= low) {
            k -= low;
            w >>= half;
            pos += half;
        }
    });
    return pos;
}

constexpr int kMidSeg = 2048;  // mask words per segment of the middle tier (8 per thread)

// Middle tier: workgroup b takes mask words [b per, (b + 1) per), segment by
// segment: the marked cells of a segment get their ranks by a prefix sum of
// the words' bit counts and are processed 256 at a time in rank order (a
// fixed grouping, independent of timing).  Wider cells go to the wide
// tier's list (counted in counters[0]).
template <class P>
__global__ __launch_bounds__(kBlock) void adaptive_mid_kernel(StepArgs a, AdaptArgs ad, ChunkOrder ord,
                                                              const typename P::real *__restrict__ E,
                                                              typename P::real *__restrict__ pops,
                                                              uint8_t *__restrict__ lo, uint8_t *__restrict__ wc,
                                                              int64_t n, const unsigned long long *__restrict__ mask,
                                                              int64_t nwords, int64_t per,
                                                              AdaptHeader *__restrict__ hdr,
                                                              int32_t *__restrict__ list,
                                                              unsigned long long *__restrict__ counters)
{
    constexpr int kPer = kMidSeg / kBlock;  // words per thread in a segment
    __shared__ double sc[kDevTableLen];
    __shared__ unsigned long long smask[kMidSeg];
    __shared__ uint32_t spre[kMidSeg + 1];
    __shared__ uint32_t swave[kBlock / 64];
    const double *slog = sc + kCoefRows * kCoefStride;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t w0 = (int64_t)blockIdx.x * per;
    const int64_t w1 = w0 + per < nwords ? w0 + per : nwords;
    bool staged = false;
    for (int64_t s0 = w0; s0 < w1; s0 += kMidSeg) {
        // bit counts of this thread's kPer words, then an exclusive prefix
        // sum over the workgroup
        uint32_t cnt[kPer], tot = 0;
        static_for<0, kPer>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const int64_t wd = s0 + threadIdx.x * kPer + i;
            const unsigned long long m = wd < w1 ? mask[wd] : 0ull;
            smask[threadIdx.x * kPer + i] = m;
            cnt[i] = (uint32_t)__popcll(m);
            tot += cnt[i];
        });
        uint32_t x = tot;
        static_for<0, 6>([&](auto dd) {
            constexpr int d = 1 << decltype(dd)::value;
            const uint32_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        });
        if (lane == 63) swave[wid] = x;
        __syncthreads();
        uint32_t excl = x - tot;
        for (int k = 0; k < wid; ++k) excl += swave[k];
        static_for<0, kPer>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            spre[threadIdx.x * kPer + i] = excl;
            excl += cnt[i];
        });
        if (threadIdx.x == kBlock - 1) spre[kMidSeg] = excl;
        __syncthreads();
        const uint32_t C = spre[kMidSeg];  // marked cells of the segment (uniform)
        if (C > 0 && !staged) {
            stage_coefficients(sc, a.tab, a.ln_dt);
            staged = true;
        }
        for (uint32_t base = 0; base < C; base += kBlock) {
            const uint32_t r = base + threadIdx.x;
            const bool valid = r < C;
            int64_t c = 0;
            if (valid) {
                // the word holding rank r: the last j with spre[j] <= r
                int lo_ = 0, hi_ = kMidSeg - 1;
                while (lo_ < hi_) {
                    const int mid = (lo_ + hi_ + 1) >> 1;
                    if (spre[mid] <= r) lo_ = mid;
                    else hi_ = mid - 1;
                }
                const int bit = select_bit(smask[lo_], r - spre[lo_]);
                const int64_t wd = s0 + lo_;
                c = chunk_place(wd >> 2, ord) * kBlock + (wd & 3) * 64 + bit;
            }
            const bool go = adaptive_lane_cell<P, kMidW>(a, ad, sc, slog, c, valid, E, pops, lo, wc, n, counters);
            list_cells(go, c, hdr, list, counters);
        }
        __syncthreads();  // the segment's LDS is read before the next one is written
    }
}

// Wide tier: one wavefront per listed cell (double arithmetic).  LDS as the
// wide ionize_step path (wide_wave_doubles) plus the leak scratch.
// One listed cell on G lanes (a wavefront, or a group of 16 of it): shift,
// leak test, exact solve by chain_sub.  A group checks the rows' rounding
// after taking them and squares the table only when that check fails
// (chain_sub<true>): most tables whose entries' a-priori bounds call for the
// squaring yield rows well within the tolerance here (3D pulse: the step
// 36.7 -> 26.9 ms).  A wavefront's cell squares on the a-priori bound.  With G < 64 a cell whose slots do
// not fit the group (its window already 16 rates or more, or its top above
// slot 15) is left untouched and listed in list_wave (returns false).
template <class R, int G>
__device__ void adaptive_cell(const StepArgs &a, const AdaptArgs &ad, int64_t c, const R *__restrict__ E,
                              R *__restrict__ pops, uint8_t *__restrict__ lo, uint8_t *__restrict__ wc, int64_t n,
                              double *s, double *e, double *mm, double *Nb, int *cid, int *pos, double *D, double *V,
                              int vs, double *lx, double *lN, AdaptHeader *__restrict__ hdr,
                              int32_t *__restrict__ list_wave, unsigned long long *__restrict__ counters)
{
    using L = Lanes<G>;
    const int lane = L::lane();
    const int Z = a.Z;
    const int wmax = ad.wmax;
    auto pass_on = [&]() {
        if (lane == 0) list_wave[atomicAdd(&hdr->count_wave, 1u)] = (int32_t)c;
    };
    wave_sync();  // the previous cell's reads of LDS are done
    const double EL = fabs((double)E[c]);
    const int l0 = lo[c];
    int p = l0 < Z ? l0 : Z;
    const int w0 = wc[c];
    const int w_in = w0 < wmax ? w0 : wmax;
    if (G < 64 && w_in >= G) {
        pass_on();
        return;
    }
    double Ns = lane <= w_in ? (double)pops[(int64_t)lane * n + c] : 0.0;
    int w = w_in;
    while (p < Z && L::shfl(Ns, 0) < a.eps) {
        const double up = L::down1(Ns);
        Ns = lane == 0 ? Ns + up : (lane < wmax && lane < G - 1 ? up : 0.0);
        ++p;
        w = w > 0 ? w - 1 : 0;
    }
    const int room = min(wmax, Z - p);
    const int t0 = min(max(ad.wmin, w), Z - p);
    const bool finite = EL <= 1.7976931348623157e308 || p >= Z;
    double out = Ns;
    int top = t0;
    if (p < Z) {
        const Field f = field_terms<RateEval<PolicyF64>::kLogTerms>(EL, a.tab + kCoefRows * kCoefStride);
        double x = 0.0;
        if (lane <= room && p + lane < Z) {
            double row[kCoefStride];
            for (int k = 0; k < kCoefStride; ++k) row[k] = a.tab[(p + lane) * kCoefStride + k];
            row[0] += a.ln_dt * kLog2e;
            x = RateEval<PolicyF64>::x_of(row, f, a.has_poly != 0);
        }
        // leak(t) of lane t: on a wavefront in the log domain (products of
        // many capped rates leave the double range); within 16 slots the
        // products of at most 16 rates (each at most kXMax) stay in range,
        // and a running product takes the place of an exponential per term
        double leak = 0.0;
        if constexpr (G < 64) {
            if (lane <= room) {
                lx[lane] = x;
                lN[lane] = fabs(Ns);
            }
            wave_sync();
            if (lane >= t0 && lane <= room) {
                double prod = 1.0;
                for (int d = 0; d <= lane; ++d) {  // d = lane - q: uniform over the lanes in the loop
                    const int q = lane - d;
                    prod *= lx[q];
                    if (lN[q] != 0.0) leak = fma(lN[q] * prod, kInvFactL.v[d + 1], leak);
                }
            }
        } else {
            if (lane <= room) {
                lx[lane] = log(x);
                lN[lane] = Ns != 0.0 ? log(fabs(Ns)) : -INFINITY;
            }
            wave_sync();
            if (lane >= t0 && lane <= room) {
                double path = 0.0;
                for (int q = lane; q >= 0; --q) {
                    path += lx[q];
                    if (lN[q] > -INFINITY) leak += exp(lN[q] + path - kLogFact.v[lane - q + 1]);
                }
            }
        }
        // top: the lowest slot t in [t0, room) with leak(t) <= tol (a NaN
        // leak widens), else room
        const unsigned long long okm = L::ballot(lane >= t0 && lane < room && leak <= ad.tol);
        if (G < 64 && !okm && room >= G) {
            // the top lies above the group's slots
            wave_sync();
            pass_on();
            return;
        }
        top = okm ? __ffsll((long long)okm) - 1 : room;
        // the storage limit held the top back
        const bool held = !okm && room < Z - p && !(L::shfl(leak, room) <= ad.tol);
        if (held && counters && lane == 0) atomicAdd(&counters[1], 1ull);
        wave_sync();
        if (top > 0 && finite) {
            const double r =
                chain_sub<(G < 64), G>(top, lane < top ? x : 0.0, lane <= top ? Ns : 0.0, to_lds(s), to_lds(e), to_lds(mm),
                                    to_lds(Nb), to_lds(cid), to_lds(pos), to_lds(D), to_lds(V), vs);
            if (lane <= top) out = r;
        }
    }
    const int wst = max(w_in, top);
    if (lane <= wst) {
        const double v = finite ? (lane <= top ? out : 0.0) : (double)NAN;
        pops[(int64_t)lane * n + c] = (R)v;
    }
    if (lane == 0) {
        lo[c] = (uint8_t)p;
        wc[c] = (uint8_t)(p >= Z ? 0 : top);
    }
}

// LDS doubles of one cell on a wavefront, windows up to W rates: chain_sub's
// region and the leak test's logs (2 x 64).
constexpr size_t adaptive_wave_doubles(int W) { return wide_cell_doubles<64>(W, false) + 128; }

// Cells of the list, four per wavefront (16 lanes each): windows of up to
// kGroupW rates (slots 0..15); the others go on to list_wave.
constexpr int kGroupLanes = 16;
constexpr int kGroupsPerWave = 64 / kGroupLanes;
constexpr int kGroupW = kGroupLanes - 1;  // widest window of a group, also its column stride
// LDS doubles of one group's cell: chain_sub's region for kGroupW rates with
// the entries' error bounds; the leak test's scratch lies in its columns,
// which are used only after it (LDS bounds how many of these wavefronts a CU
// holds)
constexpr size_t kGroupCellDoubles = wide_cell_doubles<kGroupLanes>(kGroupW, true);

template <class R>
__global__ __launch_bounds__(kWideBlock) void adaptive_group_kernel(StepArgs a, AdaptArgs ad,
                                                                    const R *__restrict__ E, R *__restrict__ pops,
                                                                    uint8_t *__restrict__ lo,
                                                                    uint8_t *__restrict__ wc, int64_t n,
                                                                    AdaptHeader *__restrict__ hdr,
                                                                    const int32_t *__restrict__ list,
                                                                    int32_t *__restrict__ list_wave,
                                                                    unsigned long long *__restrict__ counters)
{
    constexpr int G = kGroupLanes;
    extern __shared__ __align__(16) double wl[];
    const int grp = threadIdx.x / G;
    double *base = wl + (size_t)grp * kGroupCellDoubles;
    int *cid = (int *)(base + 4 * G);
    int *pos = cid + G;
    double *D = base + 6 * G;
    double *V = D + kGroupW * (kGroupW + 1) / 2;
    double *lx = V;  // the leak test's rates and populations, before the solve uses V
    double *lN = V + G;
    const uint32_t count = hdr->count;
    for (uint32_t i = blockIdx.x * kGroupsPerWave + grp; i < count; i += gridDim.x * kGroupsPerWave) {
        const int64_t c = list[i];
        adaptive_cell<R, G>(a, ad, c, E, pops, lo, wc, n, base, base + G, base + 2 * G, base + 3 * G, cid, pos, D,
                            V, kGroupW, lx, lN, hdr, list_wave, counters);
    }
}

// Cells passed on by the groups, one per wavefront.
template <class R>
__global__ __launch_bounds__(kWideBlock) void adaptive_wide_kernel(StepArgs a, AdaptArgs ad,
                                                                   const R *__restrict__ E, R *__restrict__ pops,
                                                                   uint8_t *__restrict__ lo,
                                                                   uint8_t *__restrict__ wc, int64_t n,
                                                                   AdaptHeader *__restrict__ hdr,
                                                                   const int32_t *__restrict__ list_wave,
                                                                   unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) double wl[];
    const int W = ad.wmax;
    int *cid = (int *)(wl + 256);
    int *pos = cid + 64;
    double *D = wl + 384;
    double *V = D + W * (W + 1) / 2;
    double *lx = wl + wide_wave_doubles(W, false);
    double *lN = lx + 64;
    const uint32_t count = hdr->count_wave;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t c = list_wave[i];
        adaptive_cell<R, 64>(a, ad, c, E, pops, lo, wc, n, wl, wl + 64, wl + 128, wl + 192, cid, pos, D, V, W, lx,
                             lN, hdr, nullptr, counters);
    }
}

template <class P>
hipError_t launch_adaptive(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                           uint8_t *wc, const adk_adaptive *win, void *work, unsigned long long *counters,
                           hipStream_t st)
{
    using R = typename P::real;
    const StepArgs a = step_args(g, dt, win->eps);
    AdaptArgs ad;
    ad.wmin = win->wmin;
    ad.wmax = win->wmax;
    ad.tol = win->tol;
    const AdaptWork wk = adapt_work(work, n);
    hipLaunchKernelGGL(adaptive_clear_kernel, dim3(1), dim3(64), 0, st, wk.hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const ChunkOrder ord = chunk_order(n);
    const int grid = resident_grid<adaptive_narrow_kernel<P>>(n, kStepChunksPerGroup);
    hipLaunchKernelGGL((adaptive_narrow_kernel<P>), dim3(grid), dim3(kBlock), 0, st, a, ad, ord, (const R *)E,
                       (R *)pops, lo, wc, n, wk.mask, counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the middle tier: the resident workgroups, each a fixed range of words
    const int mgrid = resident_grid<adaptive_mid_kernel<P>>(n);
    const int64_t per = (wk.nwords + mgrid - 1) / mgrid;
    hipLaunchKernelGGL((adaptive_mid_kernel<P>), dim3(mgrid), dim3(kBlock), 0, st, a, ad, ord, (const R *)E,
                       (R *)pops, lo, wc, n, (const unsigned long long *)wk.mask, wk.nwords, per, wk.hdr, wk.list,
                       counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // groups of 16 lanes over the list: the resident workgroups (one
    // wavefront each, LDS bound)
    {
        const size_t gdyn = sizeof(double) * kGroupsPerWave * kGroupCellDoubles;
        static int gper_cu = 0;
        if (gper_cu <= 0) {
            int b = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, adaptive_group_kernel<R>, kWideBlock, gdyn) !=
                    hipSuccess ||
                b <= 0)
                b = 1;
            gper_cu = b;
        }
        const int64_t need = (n + kWideBlock - 1) / kWideBlock;
        const int64_t cap = (int64_t)num_cus() * gper_cu;
        const int ggrid = (int)(need < cap ? need : cap);
        hipLaunchKernelGGL(adaptive_group_kernel<R>, dim3(ggrid), dim3(kWideBlock), gdyn, st, a, ad, (const R *)E,
                           (R *)pops, lo, wc, n, wk.hdr, (const int32_t *)wk.list, wk.list_wave, counters);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t dyn = sizeof(double) * adaptive_wave_doubles(ad.wmax);
    static int per_cu[ADK_MAX_WIDE_W + 1] = {};  // occupancy per widest window (LDS grows with it)
    int b = per_cu[ad.wmax];
    if (b <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, adaptive_wide_kernel<R>, kWideBlock, dyn) !=
                hipSuccess ||
            b <= 0)
            b = 1;
        per_cu[ad.wmax] = b;
    }
    const int64_t need = (n + kWideBlock - 1) / kWideBlock;
    const int64_t cap = (int64_t)num_cus() * b;
    const int wgrid = (int)(need < cap ? need : cap);
    hipLaunchKernelGGL(adaptive_wide_kernel<R>, dim3(wgrid), dim3(kWideBlock), dyn, st, a, ad, (const R *)E,
                       (R *)pops, lo, wc, n, wk.hdr, (const int32_t *)wk.list_wave, counters);
    return hipGetLastError();
}

}  // namespace
}  // namespace adk

size_t adk_adaptive_work_bytes_impl(int64_t ncells)
{
    const int64_t n = ncells > 0 ? ncells : 0;
    return sizeof(adk::AdaptHeader) + sizeof(unsigned long long) * (size_t)adk::adapt_mask_words(n) +
           2 * sizeof(int32_t) * (size_t)n;
}

hipError_t adk_step_adaptive(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                             uint8_t *wc, const adk_adaptive *win, void *work, unsigned long long *counters,
                             hipStream_t st)
{
    return win->prec == ADK_F64
               ? adk::launch_adaptive<adk::PolicyF64>(g, E, n, dt, pops, lo, wc, win, work, counters, st)
               : adk::launch_adaptive<adk::PolicyMixed>(g, E, n, dt, pops, lo, wc, win, work, counters, st);
}
