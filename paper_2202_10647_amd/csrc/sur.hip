// Surrogate form of the ionization step (compact layout, float populations).
//
// A wavefront takes 64 cells at a time, its chunks of the mesh in the
// scattered order of the step kernel (ChunkOrder), so the network's work in
// the pulse spreads over all XCDs and CUs (3D laser mesh: 1309 -> 938 us per
// step against chunks in mesh order).  The window shift at the start of the
// step is that of the analytic step.  Cells whose |E| lies in the network's
// trained range then advance with predicted band columns, one per source level of
// the window: the (cell, source) pairs whose rate is not negligible are
// packed into a list in LDS, evaluated 16 at a time (the matrix-core tile),
// and each cell reads its columns back.  Cells outside the range take the
// analytic chain solution (mixed precision); a wavefront runs each branch
// only if one of its lanes needs it.
#include "mlp.hpp"

namespace adk {
namespace {

// Visibility of this wavefront's LDS writes to its own later reads (a
// wavefront's LDS operations execute in order; the fences keep the compiler
// from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup per CU: 12 wavefronts (three per SIMD, what the register
// file holds at this kernel's register count) share one chunk counter.
// Against workgroups of 4 wavefronts, the 3D pulse step measured 711 -> 671 us.
constexpr int kSurWaves = 12;
constexpr int kSurBlock = 64 * kSurWaves;

// Dynamic LDS: the layer-1 table ctab[Z][kCtabStride], then per wavefront
// 64 W slots of 16 bytes: the (cell, source) pairs that need the network
// (u and level k), overwritten by their columns once evaluated.
template <int W>
constexpr size_t sur_dyn_bytes(int Z)
{
    return (size_t)Z * kCtabStride * sizeof(float) + (size_t)kSurWaves * 64 * W * sizeof(f32x4);
}

template <int W>
__global__ __launch_bounds__(kSurBlock, 3) void surrogate_kernel(SurArgs a, const float *__restrict__ E,
                                                                 float *__restrict__ pops, uint8_t *__restrict__ lo,
                                                                 int64_t n, ChunkOrder ord)
{
    __shared__ double sc[kDevTableLen];
    __shared__ MlpShared ms;
    // thresholds of levels 0..Z-1, then infinite ones up to level Z + W - 1
    // (a window's slots past the last level need no clamp)
    static_assert(W <= 4, "threshold padding");
    __shared__ float sthr[ADK_MAX_Z + 4];
    __shared__ float scut[ADK_MAX_Z + 1];
    __shared__ unsigned next_chunk;
    extern __shared__ __align__(16) unsigned char dyn[];
    const int Z = a.st.Z;
    const int lane = threadIdx.x & 63;
    float *ctab = (float *)dyn;
    // a group reads its pairs before it writes their columns into the same
    // slots, and no other group touches them
    f32x4 *slot = (f32x4 *)(dyn + (size_t)Z * kCtabStride * sizeof(float)) + (threadIdx.x >> 6) * 64 * W;
    if (threadIdx.x == 0) next_chunk = 0u;  // visible after staging
    for (int t = threadIdx.x; t < Z + W; t += blockDim.x) sthr[t] = t < Z ? a.thr[t] : INFINITY;
    for (int t = threadIdx.x; t <= ADK_MAX_Z; t += blockDim.x) scut[t] = a.cut.e[t];  // visible after staging
    stage_coefficients(sc, a.st.tab, a.st.ln_dt);
    stage_mlp(ms, ctab, a.prm, a.L, a.v, true);
    const double *slog = sc + kCoefRows * kCoefStride;
    const bool has_poly = a.st.has_poly != 0;
    unsigned long long n_fb = 0, n_eval = 0;

    // Workgroup b owns the chunk indices [b per, (b + 1) per) (scattered over
    // the mesh by ChunkOrder), and its wavefronts take them one at a time
    // from a counter in LDS: a chunk's cost depends on how many of its cells
    // the pulse has reached, and a fixed share per wavefront would leave the
    // launch waiting for the wavefronts that drew the most of them.  A cell's
    // result does not depend on which wavefront takes it.
    //
    // Wavefront-uniform loop: every lane stays active for the matrix ops.
    // The next chunk's cells are loaded while this one is worked on (the
    // network and the column sums hide their HBM latency), and handed over
    // to the loop's working registers before this chunk's stores: the
    // vector-memory counter retires loads and stores in the order they were
    // issued, so a wait for the loads after the stores (at the top of the
    // next iteration) would also wait for the stores.
    const int64_t nchunks = (n + 63) / 64;
    const int64_t per = (nchunks + gridDim.x - 1) / gridDim.x;
    // uniform values, held in scalar registers (so is what is derived from
    // them: the chunk's place under ChunkOrder is a scalar loop)
    auto uniform = [](int64_t x) -> int64_t {
        const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)x);
        const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
        return (int64_t)(((uint64_t)hi32 << 32) | lo32);
    };
    const int64_t vb = uniform((int64_t)blockIdx.x * per);
    const int64_t ve = uniform(vb + per < nchunks ? vb + per : nchunks);
    auto take = [&]() -> int64_t {
        unsigned t = 0u;
        if (lane == 0) t = atomicAdd(&next_chunk, 1u);
        return vb + (int64_t)__builtin_amdgcn_readfirstlane(t);
    };
    // the network's weight operands stay in registers for the whole loop
    // (loading them per chunk measured 17 % of the wavefronts' time)
    MlpRegs r;
    load_regs(r, ms, lane);
    MlpBias bs;
    if constexpr (kBiasRegs > 0) load_bias(bs, ms, lane);
    int64_t vt = take();
    int64_t cn = vt < ve ? chunk_place(vt, ord) * 64 + lane : n;
    // lanes past the end load the last cell (any in-bounds address) and
    // drop it at the hand-over; n > 0 whenever the loop runs
    CellLoad<float, W> nxt;
    if (n > 0) load_cell(nxt, E, pops, lo, n, cn < n ? cn : n - 1);
    int64_t ch;  // the handed-over chunk: its cells, field and window bottom
    float Eh, Nh[W + 1];
    int loh;
    auto handover = [&]() __attribute__((always_inline)) {
        const bool ok = cn < n;
        ch = cn;
        Eh = ok ? nxt.E : 0.0f;
#pragma unroll
        for (int s = 0; s <= W; ++s) Nh[s] = ok ? nxt.N[s] : 0.0f;
        loh = ok ? (int)nxt.lo : Z;
        // the values pass through an empty asm statement, so that they count
        // as computed here (after the wait for the loads) and the stores that
        // follow stay after it
        asm volatile("" : "+v"(Eh), "+v"(loh)::"memory");
#pragma unroll
        for (int s = 0; s <= W; ++s) asm volatile("" : "+v"(Nh[s])::"memory");
    };
    handover();
    while (vt < ve) {
        const int64_t c = ch;
        const bool valid = c < n;
        const float Ef = Eh;
        float Nf[W + 1];
#pragma unroll
        for (int s = 0; s <= W; ++s) Nf[s] = Nh[s];
        const int lo0 = loh;
        vt = take();
        cn = vt < ve ? chunk_place(vt, ord) * 64 + lane : n;
        load_cell(nxt, E, pops, lo, n, cn < n ? cn : n - 1);
        int p = lo0 < Z ? lo0 : Z;
        const double EL = fabs((double)Ef);
        // a cell under its window's identity field (every rate of the
        // window below 1e-16 per step) with no shift due is left as it is,
        // as ionize_step leaves it: the exact step would move less than
        // 3e-16, and for a field in the trained range every source is then
        // negligible, so the network's form is the identity too
        const bool idle = p >= Z || (EL < (double)scut[p] && (double)Nf[0] >= a.st.eps);
        if (__all(idle)) {
            handover();
            if (valid && p != lo0) lo[c] = (uint8_t)p;  // windows unchanged in place
            continue;
        }
        double N[W + 1];
#pragma unroll
        for (int s = 0; s <= W; ++s) N[s] = (double)Nf[s];
        while (p < Z && N[0] < a.st.eps) {
            N[0] += N[1];
#pragma unroll
            for (int s = 1; s < W; ++s) N[s] = N[s + 1];
            N[W] = 0.0;
            ++p;
        }
        const bool act = p < Z && !idle;
        const bool in = EL >= a.E_lo && EL <= a.E_hi;
        const bool use_mlp = act && in;
        const bool use_an = act && !in;
        // float from here on: stored values, and for the network's cells also
        // the populations it redistributes (its columns are float)
        float out[W + 1];
#pragma unroll
        for (int s = 0; s <= W; ++s) out[s] = (float)N[s];

        if (__any(use_an)) {
            const Field f = field_terms<RateEval<PolicyMixed>::kLogTerms>(EL, slog);
            float x[W];
            window_rates<PolicyMixed, W>(sc, p, f, has_poly, x);
            double o2[W + 1];
            chain_apply<PolicyMixed, W>(x, N, o2);
            if (use_an) {
#pragma unroll
                for (int s = 0; s <= W; ++s) out[s] = (float)o2[s];
            }
        }

        const int top = act ? (W < Z - p ? W : Z - p) : 0;  // absorbing slot
        if (__any(use_mlp)) {
            // the (cell, source) pairs that need the network, packed densely:
            // a source level whose rate is negligible at this field (W dt <
            // 1e-9, |E| below its threshold) keeps its population (identity
            // column) without an evaluation
            const float u = fmaf(__log2f(fabsf(Ef)), a.au, a.bu);
            const float Eabs = fabsf(Ef);
            const float *lthr = sthr + p;  // p <= Z
            const int rowb = __mul24(p, (int)(kCtabStride * sizeof(float)));  // byte offset of level p's layer-1 row
            int cnt = 0;
            int pos[W];
            bool need[W];
#pragma unroll
            for (int s = 0; s < W; ++s) {
                // every lane reads its threshold (thresholds are 0, positive
                // or infinite) and a lane with no pair in slot s tests -1
                // against it, so that one compare gives the mask and the
                // ballot takes it as it is
                const float thr = lthr[s];
                const float x = (use_mlp & (s < top)) ? Eabs : -1.0f;
                need[s] = !(x < thr);
                const unsigned long long m = __ballot(need[s]);
                pos[s] = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                // the pair: u and the byte offset of level k's layer-1 row
                if (need[s])
                    slot[pos[s]] = (f32x4){u, __int_as_float(rowb + s * (int)(kCtabStride * sizeof(float))), 0.0f, 0.0f};
                cnt += __popcll(m);
            }
            // the list is padded to whole passes with a pair that evaluates
            // harmlessly (u = 0, level 0), so that every lane of a pass reads
            // its own slot; the padding's columns are not stored
            // (a pass reads u and the row offset, the slot's first two words)
            const int cpad = (cnt + 15) & ~15;
            if (lane < cpad - cnt) *(uint2 *)(slot + cnt + lane) = make_uint2(0u, 0u);
            wave_lds_sync();
            if (cnt > 0) {
                // 16 pairs per pass; four passes in a row add their logits
                // into one tile (pass j's samples land in lane group j & 3),
                // which then takes one softmax for 64 pairs.  Slots of a
                // block are read by its passes before the block's columns
                // overwrite them
                f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                const f32x4 *mine = slot + (lane & 15);
                // byte offset of this lane group's b2 units and b4 copy,
                // renewed (as far as the compiler knows) on every pass
                int ob = (int)(4 * sizeof(float)) * (lane >> 4);
                f32x2 cqn = *(const f32x2 *)mine;
                for (int g0 = 0; g0 < cnt; g0 += 16) {
                    asm volatile("" : "+v"(ob));
                    const int qo = (g0 >> 4) & 3;
                    const f32x2 cq = cqn;
                    // the next pass's pair, read during this pass
                    cqn = *(const f32x2 *)(mine + (g0 + 16 < cnt ? g0 + 16 : g0));
                    mlp_logits_into(r, bs, (const float *)((const char *)ms.b2 + ob),
                                    (const float *)((const char *)ms.b4 + ob),
                                    (const float *)((const char *)ctab + __float_as_int(cq.y)), cq.x, qo, z);
                    if (qo == 3 || g0 + 16 >= cnt) {
                        float zm, lse;
                        const f32x4 Q = softmax4(z, zm, lse);
                        const int tb = (g0 & ~63) + lane;
                        if (tb < cnt) slot[tb] = Q;
                    }
                }
                wave_lds_sync();
            }
            n_eval += (unsigned long long)cnt;
            // N' = sum over source slots s of column_s x N[s] (float);
            // destinations past the top slot are lumped into it, which keeps
            // its own population
            float acc[W + kBand];
#pragma unroll
            for (int j = 0; j < W + kBand; ++j) acc[j] = 0.0f;
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const f32x4 Q = need[s] ? slot[pos[s]] : (f32x4){1.0f, 0.0f, 0.0f, 0.0f};
                const float ns = s < top ? out[s] : 0.0f;  // = N[s] on the network's cells
#pragma unroll
                for (int d = 0; d < kBand; ++d) acc[s + d] = fmaf(Q[d], ns, acc[s + d]);
            }
            float Ntop = 0.0f, tail = 0.0f;
#pragma unroll
            for (int j = 0; j <= W; ++j) Ntop = j == top ? out[j] : Ntop;
#pragma unroll
            for (int j = 0; j < W + kBand; ++j) tail += j >= top ? acc[j] : 0.0f;
            if (use_mlp) {
#pragma unroll
                for (int j = 0; j <= W; ++j) out[j] = j < top ? acc[j] : (j == top ? Ntop + tail : 0.0f);
            }
        }

        n_fb += (unsigned long long)__popcll(__ballot(use_an && EL >= a.st.E_cut));

        handover();
        if (valid) {
            const bool finite = EL <= 1.7976931348623157e308 || p >= Z;
#pragma unroll
            for (int s = 0; s <= W; ++s) {
                const float v = finite ? out[s] : NAN;
                pops[(int64_t)s * n + c] = (p + s <= Z) ? v : 0.0f;
            }
            lo[c] = (uint8_t)p;
        }
    }
    if (a.counters && lane == 0) {
        if (n_fb) atomicAdd(a.counters, n_fb);
        if (n_eval) atomicAdd(a.counters + 1, n_eval);
    }
}

template <int W>
hipError_t launch(const SurArgs &a, const float *E, float *pops, uint8_t *lo, int64_t n, hipStream_t st)
{
    const size_t dyn = sur_dyn_bytes<W>(a.st.Z);
    static int per_cu[ADK_MAX_Z + 1] = {};  // occupancy per level count (LDS grows with Z)
    int b = per_cu[a.st.Z];
    if (b <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, surrogate_kernel<W>, kSurBlock, dyn) != hipSuccess ||
            b <= 0)
            b = 1;
        per_cu[a.st.Z] = b;
    }
    const int64_t need = (n + kSurBlock - 1) / kSurBlock;
    const int64_t cap = (int64_t)num_cus() * b;
    const int grid = (int)(need < cap ? need : cap);
    hipLaunchKernelGGL(surrogate_kernel<W>, dim3(grid), dim3(kSurBlock), dyn, st, a, E, pops, lo, n,
                       chunk_order(n, 64));
    return hipGetLastError();
}

}  // namespace
}  // namespace adk

hipError_t adk_surrogate_launch_1(const adk::SurArgs &a, const float *E, float *p, uint8_t *lo, int64_t n,
                                  hipStream_t st)
{
    return adk::launch<1>(a, E, p, lo, n, st);
}
hipError_t adk_surrogate_launch_2(const adk::SurArgs &a, const float *E, float *p, uint8_t *lo, int64_t n,
                                  hipStream_t st)
{
    return adk::launch<2>(a, E, p, lo, n, st);
}
hipError_t adk_surrogate_launch_3(const adk::SurArgs &a, const float *E, float *p, uint8_t *lo, int64_t n,
                                  hipStream_t st)
{
    return adk::launch<3>(a, E, p, lo, n, st);
}
