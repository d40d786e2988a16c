// Surrogate form of the ionization step (compact layout, float populations).
//
// A wavefront takes 64 cells.  The window shift at the start of the step is
// that of the analytic step.  Cells whose |E| lies in the network's trained
// range then advance with predicted band columns: for each source slot s of
// the window the wavefront evaluates the network on 4 groups of 16 cells (the
// matrix-core tile), and the owner lane of each cell collects its columns by
// lane shuffles.  Cells outside the range take the analytic chain solution
// (mixed precision); a wavefront runs each branch only if one of its lanes
// needs it.
#include "mlp.hpp"

namespace adk {
namespace {

template <int W>
__global__ __launch_bounds__(kBlock, 3) void surrogate_kernel(SurArgs a, const float *__restrict__ E,
                                                           float *__restrict__ pops, uint8_t *__restrict__ lo,
                                                           int64_t n)
{
    __shared__ double sc[kDevTableLen];
    __shared__ MlpShared ms;
    stage_coefficients(sc, a.st.tab, a.st.ln_dt);
    stage_mlp(ms, a.prm, a.L, a.v, true);
    const double *slog = sc + kCoefRows * kCoefStride;
    const int Z = a.st.Z;
    const bool has_poly = a.st.has_poly != 0;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    unsigned long long n_fb = 0, n_eval = 0;

    // wavefront-uniform loop: every lane stays active for the matrix ops
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        const int64_t c = base + lane;
        const bool valid = c < n;
        float Ef = 0.0f;
        float Nf[W + 1];
        int p = Z;
#pragma unroll
        for (int s = 0; s <= W; ++s) Nf[s] = 0.0f;
        if (valid) {
            Ef = E[c];
#pragma unroll
            for (int s = 0; s <= W; ++s) Nf[s] = pops[(int64_t)s * n + c];
            p = lo[c];
            p = p < Z ? p : Z;
        }
        const double EL = fabs((double)Ef);
        if (__all(p >= Z || (EL < a.E_fast && (double)Nf[0] >= a.st.eps))) {
            if (valid) {
#pragma unroll
                for (int s = 0; s <= W; ++s) pops[(int64_t)s * n + c] = Nf[s];
                lo[c] = (uint8_t)p;
            }
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
        const bool act = p < Z;
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
            // weight operands reloaded per wavefront pass (not held across
            // the analytic branch)
            MlpRegs r;
            load_regs(r, *(const MlpShared *)((const char *)&ms + opaque_zero()), lane);
            const float u = fmaf(__log2f(fabsf(Ef)), a.au, a.bu);
            // inputs of sample n of group q come from the cell of lane 16 q + n
            float uq[4];
            int pq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uq[q] = __shfl(u, 16 * q + (lane & 15));
                pq[q] = __shfl(p, 16 * q + (lane & 15));
            }
            const int g = lane >> 4;
            // N' = sum over source slots s of column_s x N[s] (float: the
            // columns themselves are float); destinations past the top slot
            // are lumped into it, which keeps its own population
            float acc[W + kBand];
#pragma unroll
            for (int j = 0; j < W + kBand; ++j) acc[j] = 0.0f;
#pragma unroll
            for (int s = 0; s < W; ++s) {
                float Qs[kBand] = {};
                // groups of 16 cells with no cell needing source slot s are skipped
                const unsigned long long need = __ballot(use_mlp && s < top);
#pragma unroll 1
                for (int q = 0; q < 4; ++q) {
                    if (((need >> (16 * q)) & 0xFFFFull) == 0) continue;
                    const float un = q == 0 ? uq[0] : (q == 1 ? uq[1] : (q == 2 ? uq[2] : uq[3]));
                    const int pn = q == 0 ? pq[0] : (q == 1 ? pq[1] : (q == 2 ? pq[2] : pq[3]));
                    const int k = pn + s < Z - 1 ? pn + s : Z - 1;
                    bf16x8 h1[2], h2[2], h3[2];
                    // the logits of the cell of lane 16 q + n land in that lane
                    const f32x4 z = mlp_logits<false>(r, ms.b2 + opaque_zero(), ms.ctab + k * kH, un, 0.0f, q,
                                                      h1, h2, h3);
                    float zm, lse;
                    const f32x4 Q = softmax4(z, zm, lse);
                    if (g == q) {
#pragma unroll
                        for (int d = 0; d < kBand; ++d) Qs[d] = Q[d];
                    }
                }
                const float ns = s < top ? out[s] : 0.0f;  // = N[s] on the network's cells
#pragma unroll
                for (int d = 0; d < kBand; ++d) acc[s + d] = fmaf(Qs[d], ns, acc[s + d]);
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
#pragma unroll
        for (int s = 0; s < W; ++s) n_eval += (unsigned long long)__popcll(__ballot(use_mlp && s < top));

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
    static int per_cu = 0;
    if (per_cu <= 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, surrogate_kernel<W>, kBlock, 0) != hipSuccess || b <= 0)
            b = 2;
        per_cu = b;
    }
    const int64_t need = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)num_cus() * per_cu;
    const int grid = (int)(need < cap ? need : cap);
    hipLaunchKernelGGL(surrogate_kernel<W>, dim3(grid), dim3(kBlock), 0, st, a, E, pops, lo, n);
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
