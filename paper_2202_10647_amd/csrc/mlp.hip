// Band-column surrogate: exact training targets from the FP64 analytic
// solver, the network's forward pass on the matrix cores, an FP32 backward
// pass, Adam, the training loop, checkpoints, and the C-ABI entry points
// (the surrogate-form step kernel itself is in sur.hip).
//
// Training is deterministic: every sum of the backward pass runs in a fixed
// order (per-workgroup partial gradients over fixed chunks of the batch, then
// a chunk-ordered reduction), and no atomics are used.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "mlp.hpp"

namespace adk {
namespace {

constexpr int kCh = 32;       // samples per backward workgroup
constexpr double kNegligibleXdt = ADK_SURROGATE_NEGLIGIBLE;
constexpr int kPS = kH + 1;   // padded LDS row stride of the backward pass
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t splitmix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double u01(uint64_t seed, uint64_t ctr)
{
    return (double)(splitmix(seed + kGamma * ctr) >> 11) * 0x1.0p-53;
}

__device__ inline float bf16_round(float x) { return (float)(__bf16)x; }

// Exact band column of a unit population at level k (FP64 analytic step with
// a window of three rates, absorbing top, no shift).  The staged table holds
// no ln dt; the per-sample log2 dt is added to column 0 of each row.
__device__ inline void band_column(const double *sc, const double *slog, int Z, bool has_poly, double E, double dt,
                                   int k, double (&col)[kBand])
{
    const bool ok = k >= 0 && k < Z && dt > 0.0 && dt <= 1.7976931348623157e308;
    const int kk = ok ? k : 0;
    const double EL = fabs(E);
    const Field f = field_terms<RateEval<PolicyF64>::kLogTerms>(EL, slog);
    const double add = ok ? log2(dt) : 0.0;
    double x[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        double row[kCoefStride];
#pragma unroll
        for (int j = 0; j < kCoefStride; ++j) row[j] = sc[(kk + s) * kCoefStride + j];
        row[0] += add;
        x[s] = RateEval<PolicyF64>::x_of(row, f, has_poly);
    }
    const double N[4] = {1.0, 0.0, 0.0, 0.0};
    chain_apply<PolicyF64, 3>(x, N, col);
    const bool finite = ok && EL <= 1.7976931348623157e308;
#pragma unroll
    for (int j = 0; j < kBand; ++j) col[j] = finite ? col[j] : (double)NAN;
}

struct DataArgs {
    const double *tab;
    int Z, has_poly;
    // sampler, used when no sample arrays are given
    uint64_t seed;
    int64_t first;
    double lE0, lEs, lt0, lts;
    // features
    float au, bu;
    double av, bv, omega_a;
    int labels;  // compute the exact columns
};

// Samples -> features (U, V, K) and, with labels, exact columns as float
// P[n][4] (training) and/or double cols[4][n] (adk_band_columns).
__global__ __launch_bounds__(kBlock) void data_kernel(DataArgs a, const double *__restrict__ E,
                                                      const double *__restrict__ dt, const int32_t *__restrict__ k,
                                                      int64_t n, float *__restrict__ U, float *__restrict__ V,
                                                      uint8_t *__restrict__ K, float *__restrict__ P,
                                                      double *__restrict__ cols)
{
    __shared__ double sc[kDevTableLen];
    if (a.labels) stage_coefficients(sc, a.tab, 0.0);  // uniform over the workgroup
    const double *slog = sc + kCoefRows * kCoefStride;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double e, d;
        int kk;
        if (E) {
            e = E[i];
            d = dt[i];
            kk = k[i];
        } else {
            const uint64_t j = 3ull * (uint64_t)(a.first + i);
            e = exp(a.lE0 + u01(a.seed, j + 1) * a.lEs);
            d = exp(a.lt0 + u01(a.seed, j + 2) * a.lts);
            kk = (int)floor(u01(a.seed, j + 3) * a.Z);
            kk = kk < a.Z - 1 ? kk : a.Z - 1;
        }
        if (a.labels) {
            double col[kBand];
            band_column(sc, slog, a.Z, a.has_poly != 0, e, d, kk, col);
            if (cols)
#pragma unroll
                for (int j = 0; j < kBand; ++j) cols[(int64_t)j * n + i] = col[j];
            if (P)
#pragma unroll
                for (int j = 0; j < kBand; ++j) P[i * kBand + j] = (float)col[j];
        }
        if (U) {
            U[i] = fmaf(__log2f((float)fabs(e)), a.au, a.bu);
            V[i] = (float)(a.av * log2(d * a.omega_a) + a.bv);
            K[i] = (uint8_t)(kk < 0 ? 0 : (kk < a.Z ? kk : a.Z - 1));
        }
    }
}

struct FwdArgs {
    const float *prm;
    MlpLayout L;
    const float *U, *V;
    const uint8_t *K;
    const float *P;   // targets [.][4] (training) or null
    int64_t off, n;   // samples off..off+n-1 of U, V, K, P
    float inv_n;
    __bf16 *H1, *H2, *H3;  // activations [n][64] (training) or null
    float *dZ4;            // (Q - P) / n, [n][4]
    float *lossv;          // per-sample cross entropy [n]
    float *Q;              // network output [4][n] or null
    float *Zt;             // pre-activations and logits [n][kTraceRow] (fwd_kernel<true>) or null
};

constexpr int kTraceRow = 3 * kH + kBand;  // z1, z2, z3 (float32, before rounding), logits z4

__device__ __forceinline__ void store_h(__bf16 *H, int64_t row, int g, const bf16x8 (&h)[2])
{
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        bf16x4 lo4 = {h[c][0], h[c][1], h[c][2], h[c][3]};
        bf16x4 hi4 = {h[c][4], h[c][5], h[c][6], h[c][7]};
        *(bf16x4 *)(H + row * kH + hid(c, g, 0)) = lo4;
        *(bf16x4 *)(H + row * kH + hid(c, g, 4)) = hi4;
    }
}

template <bool TRACE>
__global__ __launch_bounds__(kBlock) void fwd_kernel(FwdArgs a)
{
    __shared__ MlpShared s;
    __shared__ float ctab[ADK_MAX_Z * kCtabStride];
    stage_mlp(s, ctab, a.prm, a.L, 0.0f, false);
    const int lane = threadIdx.x & 63, g = lane >> 4, nn = lane & 15;
    MlpRegs r;
    load_regs(r, s, lane);
    const int64_t ngroups = (a.n + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t grp = wave; grp < ngroups; grp += nwaves) {
        const int64_t i = grp * 16 + nn;
        const bool ok = i < a.n;
        const int64_t ii = ok ? i : a.n - 1;
        const int64_t si = a.off + ii;
        const int k = a.K[si];
        bf16x8 h1[2], h2[2], h3[2];
        float *zt = (TRACE && ok) ? a.Zt + ii * kTraceRow : nullptr;
        const f32x4 z = mlp_logits<true, TRACE>(r, s.b2 + opaque_zero(), ctab + k * kCtabStride, a.U[si], a.V[si], 0, h1,
                                                h2, h3, zt);
        if (TRACE && ok && g == 0) {
#pragma unroll
            for (int j = 0; j < kBand; ++j) zt[3 * kH + j] = z[j];
        }
        if (ok && a.H1) {
            store_h(a.H1, ii, g, h1);
            store_h(a.H2, ii, g, h2);
            store_h(a.H3, ii, g, h3);
        }
        if (ok && g == 0) {
            float zm, lse;
            const f32x4 q = softmax4(z, zm, lse);
            if (a.Q)
#pragma unroll
                for (int j = 0; j < kBand; ++j) a.Q[(int64_t)j * a.n + ii] = q[j];
            if (a.P) {
                float l = 0.0f;
#pragma unroll
                for (int j = 0; j < kBand; ++j) {
                    const float pj = a.P[si * kBand + j];
                    a.dZ4[ii * kBand + j] = (q[j] - pj) * a.inv_n;
                    if (pj > 0.0f) l -= pj * (z[j] - zm - lse);
                }
                a.lossv[ii] = l;
            }
        }
    }
}

// Offsets of one workgroup's partial gradient: the dense blocks, then the
// per-level sums of the layer-1 delta (emb, W1e and b1 follow from them).
struct PartLayout {
    int W1u, W1v, W2, b2, W3, b3, W4, b4, dc, n;
    static PartLayout of(int Z)
    {
        PartLayout P{};
        int o = 0;
        P.W1u = o; o += kH;
        P.W1v = o; o += kH;
        P.W2 = o; o += kH * kH;
        P.b2 = o; o += kH;
        P.W3 = o; o += kH * kH;
        P.b3 = o; o += kH;
        P.W4 = o; o += kBand * kH;
        P.b4 = o; o += kBand;
        P.dc = o; o += Z * kH;
        P.n = o;
        return P;
    }
};

struct BwdArgs {
    const float *prm;
    MlpLayout L;
    PartLayout PL;
    const float *U, *V;
    const uint8_t *K;
    int64_t off, n;
    const __bf16 *H1, *H2, *H3;
    const float *dZ4;
    float *part;  // [nchunks][PL.n]
};

struct BwdShared {
    float Wt[kH * kPS];   // weights of the current layer (bf16 values) [o][i]
    float Da[kCh * kPS];  // deltas [s][unit]
    float Db[kCh * kPS];
    float Hs[kCh * kPS];  // activation entering the current layer [s][i]
    float W4s[kBand * kH];
    float Us[kCh], Vs[kCh];
    int Ks[kCh];
};

__device__ void bwd_load_h(BwdShared &sh, const __bf16 *H, int64_t s0, int ns)
{
    for (int t = threadIdx.x; t < kCh * kH; t += blockDim.x) {
        const int s = t / kH, i = t % kH;
        sh.Hs[s * kPS + i] = s < ns ? (float)H[(s0 + s) * kH + i] : 0.0f;
    }
}

// One hidden layer: gradients of W (out x in) and b from the delta Din of its
// output, then the delta of its input Dout = (h > 0) W^T Din.
__device__ void bwd_layer(BwdShared &sh, const float *__restrict__ prm, int offW, const __bf16 *H, int64_t s0,
                          int ns, const float *Din, float *Dout, float *out, int pW, int pb)
{
    const int tid = threadIdx.x;
    for (int t = tid; t < kH * kH; t += blockDim.x) sh.Wt[(t / kH) * kPS + t % kH] = bf16_round(prm[offW + t]);
    bwd_load_h(sh, H, s0, ns);
    __syncthreads();
    {
        const int o0 = 4 * (tid / 16), i0 = 4 * (tid % 16);
        float acc[4][4] = {};
        for (int s = 0; s < kCh; ++s) {
            float d[4], h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                d[j] = Din[s * kPS + o0 + j];
                h[j] = sh.Hs[s * kPS + i0 + j];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(d[x], h[y], acc[x][y]);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) out[pW + (o0 + x) * kH + i0 + y] = acc[x][y];
    }
    if (tid < kH) {
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc += Din[s * kPS + tid];
        out[pb + tid] = acc;
    }
    {
        const int s = tid / 8, i0 = 8 * (tid % 8);
        float acc[8] = {};
        for (int o = 0; o < kH; ++o) {
            const float d = Din[s * kPS + o];
#pragma unroll
            for (int y = 0; y < 8; ++y) acc[y] = fmaf(sh.Wt[o * kPS + i0 + y], d, acc[y]);
        }
#pragma unroll
        for (int y = 0; y < 8; ++y) Dout[s * kPS + i0 + y] = sh.Hs[s * kPS + i0 + y] > 0.0f ? acc[y] : 0.0f;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void bwd_kernel(BwdArgs a)
{
    static_assert(kBlock == kBand * kH && kBlock == kCh * 8 && kBlock == 16 * 16, "thread mapping");
    __shared__ BwdShared sh;
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kCh;
    const int ns = (int)(a.n - s0 < kCh ? a.n - s0 : kCh);
    float *out = a.part + (int64_t)blockIdx.x * a.PL.n;
    const float *prm = a.prm;

    // layer 4: delta of the logits
    for (int t = tid; t < kCh * kBand; t += blockDim.x) {
        const int s = t / kBand, j = t % kBand;
        sh.Da[s * kPS + j] = s < ns ? a.dZ4[(s0 + s) * kBand + j] : 0.0f;
    }
    for (int t = tid; t < kBand * kH; t += blockDim.x) sh.W4s[t] = bf16_round(prm[a.L.W4 + t]);
    if (tid < kCh) {
        const bool ok = tid < ns;
        sh.Us[tid] = ok ? a.U[a.off + s0 + tid] : 0.0f;
        sh.Vs[tid] = ok ? a.V[a.off + s0 + tid] : 0.0f;
        sh.Ks[tid] = ok ? (int)a.K[a.off + s0 + tid] : -1;
    }
    bwd_load_h(sh, a.H3, s0, ns);
    __syncthreads();
    {
        const int j = tid / kH, i = tid % kH;
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc = fmaf(sh.Da[s * kPS + j], sh.Hs[s * kPS + i], acc);
        out[a.PL.W4 + j * kH + i] = acc;
    }
    if (tid < kBand) {
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc += sh.Da[s * kPS + tid];
        out[a.PL.b4 + tid] = acc;
    }
    for (int t = tid; t < kCh * kH; t += blockDim.x) {
        const int s = t / kH, i = t % kH;
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < kBand; ++j) acc = fmaf(sh.W4s[j * kH + i], sh.Da[s * kPS + j], acc);
        sh.Db[s * kPS + i] = sh.Hs[s * kPS + i] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // layers 3 and 2
    bwd_layer(sh, prm, a.L.W3, a.H2, s0, ns, sh.Db, sh.Da, out, a.PL.W3, a.PL.b3);
    bwd_layer(sh, prm, a.L.W2, a.H1, s0, ns, sh.Da, sh.Db, out, a.PL.W2, a.PL.b2);
    // layer 1: delta in Db
    if (tid < kH) {
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc = fmaf(sh.Db[s * kPS + tid], sh.Us[s], acc);
        out[a.PL.W1u + tid] = acc;
    } else if (tid < 2 * kH) {
        const int i = tid - kH;
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc = fmaf(sh.Db[s * kPS + i], sh.Vs[s], acc);
        out[a.PL.W1v + i] = acc;
    }
    for (int t = tid; t < a.L.Z * kH; t += blockDim.x) {
        const int k = t / kH, i = t % kH;
        float acc = 0.0f;
        for (int s = 0; s < kCh; ++s) acc += sh.Ks[s] == k ? sh.Db[s * kPS + i] : 0.0f;
        out[a.PL.dc + t] = acc;
    }
}

// Sum of the workgroups' partial gradients, chunk by chunk in order.
__global__ __launch_bounds__(kBlock) void reduce_kernel(const float *__restrict__ part, int nchunks, int plen,
                                                        float *__restrict__ red)
{
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < plen; e += gridDim.x * kBlock) {
        float acc = 0.0f;
        for (int c = 0; c < nchunks; ++c) acc += part[(int64_t)c * plen + e];
        red[e] = acc;
    }
}

// Gradient in parameter order; emb, W1e and b1 from the per-level delta sums
// dc[k] = sum over samples of level k of the layer-1 delta.
__global__ __launch_bounds__(kBlock) void finish_kernel(const float *__restrict__ prm, MlpLayout L, PartLayout PL,
                                                        const float *__restrict__ red, float *__restrict__ grad)
{
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < L.n; e += gridDim.x * kBlock) {
        float gv;
        if (e < L.W1u) {  // emb[k][j] = sum_h W1e[h][j] dc[k][h]
            const int k = (e - L.emb) / kEmb, j = (e - L.emb) % kEmb;
            float acc = 0.0f;
            for (int h = 0; h < kH; ++h) acc = fmaf(prm[L.W1e + h * kEmb + j], red[PL.dc + k * kH + h], acc);
            gv = acc;
        } else if (e < L.W1v) {
            gv = red[PL.W1u + e - L.W1u];
        } else if (e < L.W1e) {
            gv = red[PL.W1v + e - L.W1v];
        } else if (e < L.b1) {  // W1e[h][j] = sum_k dc[k][h] emb[k][j]
            const int h = (e - L.W1e) / kEmb, j = (e - L.W1e) % kEmb;
            float acc = 0.0f;
            for (int k = 0; k < L.Z; ++k) acc = fmaf(red[PL.dc + k * kH + h], prm[L.emb + k * kEmb + j], acc);
            gv = acc;
        } else if (e < L.W2) {
            const int h = e - L.b1;
            float acc = 0.0f;
            for (int k = 0; k < L.Z; ++k) acc += red[PL.dc + k * kH + h];
            gv = acc;
        } else {  // W2, b2, W3, b3, W4, b4 are contiguous in both layouts
            gv = red[PL.W2 + e - L.W2];
        }
        grad[e] = gv;
    }
}

// Batch mean of the per-sample losses: one workgroup, fixed summation order.
__global__ __launch_bounds__(kBlock) void loss_kernel(const float *__restrict__ lossv, int64_t n, float inv_n,
                                                      float *__restrict__ out)
{
    __shared__ float red[kBlock];
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += lossv[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * inv_n;
}

__global__ __launch_bounds__(kBlock) void adam_kernel(float *__restrict__ prm, float *__restrict__ m,
                                                      float *__restrict__ v, const float *__restrict__ g, int n,
                                                      float lr, float b1, float b2, float c1, float c2, float eps)
{
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        const float ge = g[e];
        const float me = fmaf(b1, m[e], (1.0f - b1) * ge);
        const float ve = fmaf(b2, v[e], (1.0f - b2) * ge * ge);
        m[e] = me;
        v[e] = ve;
        prm[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
    }
}

}  // namespace
}  // namespace adk

// ---------------------------------------------------------------------------
using namespace adk;

struct adk_mlp {
    int Z = 0;
    MlpLayout L{};
    PartLayout PL{};
    adk_mlp_range range{};
    double omega_a = 0.0;
    float *prm = nullptr, *m = nullptr, *v = nullptr;
    int64_t step = 0;
    // training set
    uint64_t data_seed = 0;
    int64_t data_n = 0;
    const adk_gas *data_gas = nullptr;
    float *U = nullptr, *V = nullptr, *P = nullptr;
    uint8_t *K = nullptr;
    // batch scratch (cap samples)
    int64_t cap = 0;
    __bf16 *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
    float *dZ4 = nullptr, *lossv = nullptr, *part = nullptr, *red = nullptr, *grad = nullptr;
    float *losses = nullptr;
    int64_t nlosses = 0;
    // features/targets of caller-given samples (adk_mlp_loss_grad)
    int64_t xcap = 0;
    float *xU = nullptr, *xV = nullptr, *xP = nullptr;
    uint8_t *xK = nullptr;
};

namespace {

int status_of(hipError_t e)
{
    if (e == hipSuccess) return ADK_OK;
    if (e == hipErrorOutOfMemory) return ADK_ENOMEM;
    return ADK_EDEVICE;
}

template <class T>
int dev_alloc(T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) return ADK_OK;
    return status_of(hipMalloc((void **)p, sizeof(T) * (size_t)count));
}

template <class T>
void dev_free(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

bool valid_range(const adk_mlp_range &r)
{
    return std::isfinite(r.E_lo) && std::isfinite(r.E_hi) && std::isfinite(r.dt_lo) && std::isfinite(r.dt_hi) &&
           r.E_lo > 0.0 && r.E_hi > r.E_lo && r.dt_lo > 0.0 && r.dt_hi > r.dt_lo;
}

MlpFeatures features(const adk_mlp &m)
{
    const double l2 = std::log10(2.0);
    const double e0 = std::log10(m.range.E_lo), e1 = std::log10(m.range.E_hi);
    const double t0 = std::log10(m.range.dt_lo * m.omega_a), t1 = std::log10(m.range.dt_hi * m.omega_a);
    MlpFeatures F;
    F.au = (float)(l2 / (0.5 * (e1 - e0)));
    F.bu = (float)(-0.5 * (e0 + e1) / (0.5 * (e1 - e0)));
    F.av = l2 / (0.5 * (t1 - t0));
    F.bv = -0.5 * (t0 + t1) / (0.5 * (t1 - t0));
    return F;
}

DataArgs data_args(const adk_gas *gas, const adk_mlp &m)
{
    DataArgs a{};
    a.tab = gas->d_coef;
    a.Z = gas->Z;
    a.has_poly = gas->has_poly;
    const MlpFeatures F = features(m);
    a.au = F.au;
    a.bu = F.bu;
    a.av = F.av;
    a.bv = F.bv;
    a.omega_a = m.omega_a;
    a.lE0 = std::log(m.range.E_lo);
    a.lEs = std::log(m.range.E_hi) - a.lE0;
    a.lt0 = std::log(m.range.dt_lo);
    a.lts = std::log(m.range.dt_hi) - a.lt0;
    return a;
}

int small_grid(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)num_cus() * 4;
    return (int)(b < 1 ? 1 : (b < cap ? b : cap));
}

void free_scratch(adk_mlp *m)
{
    dev_free(m->H1);
    dev_free(m->H2);
    dev_free(m->H3);
    dev_free(m->dZ4);
    dev_free(m->lossv);
    dev_free(m->part);
    dev_free(m->red);
    m->cap = 0;
}

int ensure_scratch(adk_mlp *m, int64_t n)
{
    if (!m->grad) {
        int st = dev_alloc(&m->grad, m->L.n);
        if (st) return st;
    }
    if (n <= m->cap) return ADK_OK;
    free_scratch(m);
    const int64_t nch = (n + kCh - 1) / kCh;
    int st = dev_alloc(&m->H1, n * kH);
    if (!st) st = dev_alloc(&m->H2, n * kH);
    if (!st) st = dev_alloc(&m->H3, n * kH);
    if (!st) st = dev_alloc(&m->dZ4, n * kBand);
    if (!st) st = dev_alloc(&m->lossv, n);
    if (!st) st = dev_alloc(&m->part, nch * m->PL.n);
    if (!st) st = dev_alloc(&m->red, m->PL.n);
    if (st) {
        free_scratch(m);
        return st;
    }
    m->cap = n;
    return ADK_OK;
}

// Device buffers of one gradient pass over n samples: activations, output
// deltas, per-sample losses, per-chunk partial gradients and their sum, and
// the gradient itself.
struct GradBufs {
    __bf16 *H1, *H2, *H3;
    float *dZ4, *lossv, *part, *red, *grad;
};

GradBufs bufs_of(adk_mlp *m) { return {m->H1, m->H2, m->H3, m->dZ4, m->lossv, m->part, m->red, m->grad}; }

// forward (storing activations), loss, backward and gradient of samples
// off..off+n-1 of (U, V, K, P); the gradient lands in B.grad, the loss in *loss.
hipError_t grad_pass(const adk_mlp *m, const GradBufs &B, const float *U, const float *V, const uint8_t *K,
                     const float *P, int64_t off, int64_t n, float *loss, hipStream_t st)
{
    FwdArgs f{};
    f.prm = m->prm;
    f.L = m->L;
    f.U = U;
    f.V = V;
    f.K = K;
    f.P = P;
    f.off = off;
    f.n = n;
    f.inv_n = (float)(1.0 / (double)n);
    f.H1 = B.H1;
    f.H2 = B.H2;
    f.H3 = B.H3;
    f.dZ4 = B.dZ4;
    f.lossv = B.lossv;
    const int64_t waves = (n + 15) / 16;
    const int64_t gmax = (int64_t)num_cus() * 2;
    int64_t g = (waves + 3) / 4;
    g = g < gmax ? g : gmax;
    hipLaunchKernelGGL(fwd_kernel<false>, dim3((int)g), dim3(kBlock), 0, st, f);
    BwdArgs b{};
    b.prm = m->prm;
    b.L = m->L;
    b.PL = m->PL;
    b.U = U;
    b.V = V;
    b.K = K;
    b.off = off;
    b.n = n;
    b.H1 = B.H1;
    b.H2 = B.H2;
    b.H3 = B.H3;
    b.dZ4 = B.dZ4;
    b.part = B.part;
    const int nch = (int)((n + kCh - 1) / kCh);
    hipLaunchKernelGGL(bwd_kernel, dim3(nch), dim3(kBlock), 0, st, b);
    hipLaunchKernelGGL(reduce_kernel, dim3(small_grid(m->PL.n)), dim3(kBlock), 0, st, (const float *)B.part, nch,
                       m->PL.n, B.red);
    hipLaunchKernelGGL(finish_kernel, dim3(small_grid(m->L.n)), dim3(kBlock), 0, st, (const float *)m->prm, m->L,
                       m->PL, (const float *)B.red, B.grad);
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kBlock), 0, st, (const float *)B.lossv, n, f.inv_n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of adk_mlp_loss_grad_noalloc: one file-scope device array (each GPU
// holds its own copy), laid out for ADK_MLP_NOALLOC_MAX_SAMPLES samples and a
// gas of up to ADK_MAX_Z levels.  Every buffer in it is written in full
// before it is read within a call, so nothing needs clearing; calls that
// overlap on one GPU share it and race.
constexpr int64_t kNaN = ADK_MLP_NOALLOC_MAX_SAMPLES;
constexpr int64_t kNaPL = 2 * kH + 2 * (kH * kH + kH) + kBand * kH + kBand + (int64_t)ADK_MAX_Z * kH;  // PartLayout n
constexpr int64_t kNaChunks = (kNaN + kCh - 1) / kCh;
constexpr size_t na_round(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaH = na_round(sizeof(__bf16) * kNaN * kH);
constexpr size_t kNaDZ4 = na_round(sizeof(float) * kNaN * kBand);
constexpr size_t kNaLoss = na_round(sizeof(float) * kNaN);
constexpr size_t kNaPart = na_round(sizeof(float) * kNaChunks * kNaPL);
constexpr size_t kNaRed = na_round(sizeof(float) * kNaPL);
constexpr size_t kNaX = na_round(sizeof(float) * kNaN);
constexpr size_t kNaXP = na_round(sizeof(float) * kNaN * kBand);
constexpr size_t kNaXK = na_round(sizeof(uint8_t) * kNaN);
constexpr size_t kNaBytes = 3 * kNaH + kNaDZ4 + kNaLoss + kNaPart + kNaRed + 2 * kNaX + kNaXP + kNaXK;

__device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current); nullptr on failure.
void *na_scratch(int dev)
{
    if (dev < 0 || dev >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_na_ptr[dev] = ptr;
    }
    return g_na_ptr[dev];
}

constexpr char kMagic[8] = {'A', 'D', 'K', 'M', 'L', 'P', '0', '1'};

struct FileHeader {
    char magic[8];
    int32_t Z, nparams;
    adk_mlp_range range;
    double omega_a;
    int64_t step;
};

}  // namespace

extern "C" {

int64_t adk_mlp_nparams(int32_t Z)
{
    if (Z < 1 || Z > ADK_MAX_Z) return -1;
    return MlpLayout::of(Z).n;
}

int adk_mlp_create(const adk_gas *gas, const float *params, const adk_mlp_range *range, adk_mlp **out)
{
    if (!gas || !params || !out) return ADK_EINVAL;
    *out = nullptr;
    adk_mlp_range r{10.0, 5000.0, 0.02e-15, 0.2e-15};
    if (range) r = *range;
    if (!valid_range(r)) return ADK_EINVAL;
    const MlpLayout L = MlpLayout::of(gas->Z);
    for (int i = 0; i < L.n; ++i)
        if (!std::isfinite(params[i])) return ADK_EINVAL;
    adk_mlp *m = new (std::nothrow) adk_mlp;
    if (!m) return ADK_ENOMEM;
    m->Z = gas->Z;
    m->L = L;
    m->PL = PartLayout::of(gas->Z);
    m->range = r;
    m->omega_a = gas->consts.omega_a;
    int st = dev_alloc(&m->prm, L.n);
    if (!st) st = dev_alloc(&m->m, L.n);
    if (!st) st = dev_alloc(&m->v, L.n);
    if (!st) st = status_of(hipMemcpy(m->prm, params, sizeof(float) * L.n, hipMemcpyHostToDevice));
    if (!st) st = status_of(hipMemset(m->m, 0, sizeof(float) * L.n));
    if (!st) st = status_of(hipMemset(m->v, 0, sizeof(float) * L.n));
    if (st) {
        adk_mlp_destroy(m);
        return st;
    }
    *out = m;
    return ADK_OK;
}

int adk_mlp_destroy(adk_mlp *m)
{
    if (!m) return ADK_OK;
    dev_free(m->prm);
    dev_free(m->m);
    dev_free(m->v);
    dev_free(m->U);
    dev_free(m->V);
    dev_free(m->P);
    dev_free(m->K);
    free_scratch(m);
    dev_free(m->grad);
    dev_free(m->losses);
    dev_free(m->xU);
    dev_free(m->xV);
    dev_free(m->xP);
    dev_free(m->xK);
    delete m;
    return ADK_OK;
}

int adk_mlp_get_state(const adk_mlp *m, float *params, float *mo, float *vo, int64_t *step)
{
    if (!m) return ADK_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return ADK_EDEVICE;
    const size_t bytes = sizeof(float) * (size_t)m->L.n;
    if (params && hipMemcpy(params, m->prm, bytes, hipMemcpyDeviceToHost) != hipSuccess) return ADK_EDEVICE;
    if (mo && hipMemcpy(mo, m->m, bytes, hipMemcpyDeviceToHost) != hipSuccess) return ADK_EDEVICE;
    if (vo && hipMemcpy(vo, m->v, bytes, hipMemcpyDeviceToHost) != hipSuccess) return ADK_EDEVICE;
    if (step) *step = m->step;
    return ADK_OK;
}

int adk_band_columns(const adk_gas *gas, const double *E, const double *dt, const int32_t *k, int64_t n,
                     double *cols, hipStream_t stream)
{
    if (!gas || n < 0) return ADK_EINVAL;
    if (n > 0 && (!E || !dt || !k || !cols)) return ADK_EINVAL;
    if (n == 0) return ADK_OK;
    DataArgs a{};
    a.tab = gas->d_coef;
    a.Z = gas->Z;
    a.has_poly = gas->has_poly;
    a.labels = 1;
    hipLaunchKernelGGL(data_kernel, dim3(small_grid(n)), dim3(kBlock), 0, stream, a, E, dt, k, n, (float *)nullptr,
                       (float *)nullptr, (uint8_t *)nullptr, (float *)nullptr, cols);
    return status_of(hipGetLastError());
}

namespace {

// Features (and, with a gas, exact float columns) of caller-given samples
// into U, V, K (and P).
int launch_given(const adk_mlp *m, const adk_gas *gas, const double *E, const double *dt, const int32_t *k,
                 int64_t n, float *U, float *V, uint8_t *K, float *P, hipStream_t stream)
{
    DataArgs a = gas ? data_args(gas, *m) : DataArgs{};
    if (!gas) {
        const MlpFeatures F = features(*m);
        a.Z = m->Z;
        a.au = F.au;
        a.bu = F.bu;
        a.av = F.av;
        a.bv = F.bv;
        a.omega_a = m->omega_a;
    }
    a.labels = gas ? 1 : 0;
    hipLaunchKernelGGL(data_kernel, dim3(small_grid(n)), dim3(kBlock), 0, stream, a, E, dt, k, n, U, V, K,
                       gas ? P : (float *)nullptr, (double *)nullptr);
    return status_of(hipGetLastError());
}

// Features (and, with a gas, exact float columns) of caller-given samples in
// the mlp's x-buffers.
int prepare_given(adk_mlp *m, const adk_gas *gas, const double *E, const double *dt, const int32_t *k, int64_t n,
                  hipStream_t stream)
{
    if (n > m->xcap) {
        dev_free(m->xU);
        dev_free(m->xV);
        dev_free(m->xP);
        dev_free(m->xK);
        m->xcap = 0;
        int st = dev_alloc(&m->xU, n);
        if (!st) st = dev_alloc(&m->xV, n);
        if (!st) st = dev_alloc(&m->xP, n * kBand);
        if (!st) st = dev_alloc(&m->xK, n);
        if (st) return st;
        m->xcap = n;
    }
    return launch_given(m, gas, E, dt, k, n, m->xU, m->xV, m->xK, m->xP, stream);
}

}  // namespace

int adk_mlp_forward(const adk_mlp *m, const double *E, const double *dt, const int32_t *k, int64_t n, float *Q,
                    hipStream_t stream)
{
    if (!m || n < 0) return ADK_EINVAL;
    if (n > 0 && (!E || !dt || !k || !Q)) return ADK_EINVAL;
    if (n == 0) return ADK_OK;
    adk_mlp *mm = const_cast<adk_mlp *>(m);
    int st = prepare_given(mm, nullptr, E, dt, k, n, stream);
    if (st) return st;
    FwdArgs f{};
    f.prm = m->prm;
    f.L = m->L;
    f.U = mm->xU;
    f.V = mm->xV;
    f.K = mm->xK;
    f.n = n;
    f.inv_n = 1.0f;
    f.Q = Q;
    const int64_t waves = (n + 15) / 16;
    const int64_t gmax = (int64_t)num_cus() * 2;
    int64_t g = (waves + 3) / 4;
    g = g < gmax ? g : gmax;
    hipLaunchKernelGGL(fwd_kernel<false>, dim3((int)g), dim3(kBlock), 0, stream, f);
    return status_of(hipGetLastError());
}

int adk_mlp_forward_trace(const adk_mlp *m, const double *E, const double *dt, const int32_t *k, int64_t n,
                          float *Q, float *Zt, hipStream_t stream)
{
    if (!m || n < 0) return ADK_EINVAL;
    if (n > 0 && (!E || !dt || !k || !Q || !Zt)) return ADK_EINVAL;
    if (n == 0) return ADK_OK;
    adk_mlp *mm = const_cast<adk_mlp *>(m);
    int st = prepare_given(mm, nullptr, E, dt, k, n, stream);
    if (st) return st;
    FwdArgs f{};
    f.prm = m->prm;
    f.L = m->L;
    f.U = mm->xU;
    f.V = mm->xV;
    f.K = mm->xK;
    f.n = n;
    f.inv_n = 1.0f;
    f.Q = Q;
    f.Zt = Zt;
    const int64_t waves = (n + 15) / 16;
    const int64_t gmax = (int64_t)num_cus() * 2;
    int64_t g = (waves + 3) / 4;
    g = g < gmax ? g : gmax;
    hipLaunchKernelGGL(fwd_kernel<true>, dim3((int)g), dim3(kBlock), 0, stream, f);
    return status_of(hipGetLastError());
}

int adk_mlp_loss_grad(adk_mlp *m, const adk_gas *gas, const double *E, const double *dt, const int32_t *k,
                      int64_t n, float *grad, float *loss, hipStream_t stream)
{
    if (!m || !gas || !E || !dt || !k || !grad || !loss || n < 1) return ADK_EINVAL;
    if (gas->Z != m->Z) return ADK_EINVAL;
    int st = ensure_scratch(m, n);
    if (!st) st = prepare_given(m, gas, E, dt, k, n, stream);
    if (st) return st;
    hipError_t e = grad_pass(m, bufs_of(m), m->xU, m->xV, m->xK, m->xP, 0, n, loss, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad, m->grad, sizeof(float) * (size_t)m->L.n, hipMemcpyDeviceToDevice, stream);
    return status_of(e);
}

int adk_mlp_loss_grad_noalloc(const adk_mlp *m, const adk_gas *gas, const double *E, const double *dt,
                              const int32_t *k, int64_t n, float *grad, float *loss, hipStream_t stream)
{
    if (!m || !gas || !E || !dt || !k || !grad || !loss || n < 1) return ADK_EINVAL;
    if (gas->Z != m->Z) return ADK_EINVAL;
    if (n > ADK_MLP_NOALLOC_MAX_SAMPLES) return ADK_ERANGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ADK_EDEVICE;
    unsigned char *base = (unsigned char *)na_scratch(dev);
    if (!base) return ADK_EDEVICE;
    GradBufs B{};
    size_t o = 0;
    B.H1 = (__bf16 *)(base + o); o += kNaH;
    B.H2 = (__bf16 *)(base + o); o += kNaH;
    B.H3 = (__bf16 *)(base + o); o += kNaH;
    B.dZ4 = (float *)(base + o); o += kNaDZ4;
    B.lossv = (float *)(base + o); o += kNaLoss;
    B.part = (float *)(base + o); o += kNaPart;
    B.red = (float *)(base + o); o += kNaRed;
    float *xU = (float *)(base + o); o += kNaX;
    float *xV = (float *)(base + o); o += kNaX;
    float *xP = (float *)(base + o); o += kNaXP;
    uint8_t *xK = (uint8_t *)(base + o); o += kNaXK;
    B.grad = grad;  // the gradient goes straight to the caller's buffer
    int st = launch_given(m, gas, E, dt, k, n, xU, xV, xK, xP, stream);
    if (st) return st;
    return status_of(grad_pass(m, B, xU, xV, xK, xP, 0, n, loss, stream));
}

int adk_mlp_train(adk_mlp *m, const adk_gas *gas, const adk_train_cfg *cfg, float *loss_out, hipStream_t stream)
{
    if (!m || !gas || !cfg) return ADK_EINVAL;
    if (gas->Z != m->Z) return ADK_EINVAL;
    if (cfg->iters < 0 || cfg->total_iters < 1 || cfg->nsamples < 1 || cfg->batch < 1 ||
        cfg->batch > cfg->nsamples)
        return ADK_EINVAL;
    if (!std::isfinite(cfg->lr) || !std::isfinite(cfg->lr_min) || cfg->lr < 0.0 || cfg->lr_min < 0.0)
        return ADK_EINVAL;
    if (cfg->iters == 0) return ADK_OK;
    int st = ensure_scratch(m, cfg->batch);
    if (st) return st;
    // training set: samples 0..nsamples-1 of the seed, labelled on the device
    if (m->data_seed != cfg->seed || m->data_n != cfg->nsamples || m->data_gas != gas || !m->U) {
        dev_free(m->U);
        dev_free(m->V);
        dev_free(m->P);
        dev_free(m->K);
        m->data_n = 0;
        const int64_t n = cfg->nsamples;
        st = dev_alloc(&m->U, n);
        if (!st) st = dev_alloc(&m->V, n);
        if (!st) st = dev_alloc(&m->P, n * kBand);
        if (!st) st = dev_alloc(&m->K, n);
        if (st) return st;
        DataArgs a = data_args(gas, *m);
        a.seed = cfg->seed;
        a.first = 0;
        a.labels = 1;
        hipLaunchKernelGGL(data_kernel, dim3(small_grid(n)), dim3(kBlock), 0, stream, a, (const double *)nullptr,
                           (const double *)nullptr, (const int32_t *)nullptr, n, m->U, m->V, m->K, m->P,
                           (double *)nullptr);
        st = status_of(hipGetLastError());
        if (st) return st;
        m->data_seed = cfg->seed;
        m->data_n = n;
        m->data_gas = gas;
    }
    if (m->nlosses < cfg->iters) {
        dev_free(m->losses);
        m->nlosses = 0;
        st = dev_alloc(&m->losses, cfg->iters);
        if (st) return st;
        m->nlosses = cfg->iters;
    }
    const int64_t nbatches = cfg->nsamples / cfg->batch;
    const double b1 = 0.9, b2 = 0.999;
    const double T = (double)cfg->total_iters;
    for (int it = 0; it < cfg->iters; ++it) {
        const int64_t t = m->step;  // steps taken before this one
        const int64_t off = (t % nbatches) * cfg->batch;
        hipError_t e = grad_pass(m, bufs_of(m), m->U, m->V, m->K, m->P, off, cfg->batch, m->losses + it, stream);
        const double tt = (double)(t < cfg->total_iters ? t : cfg->total_iters);
        const double lr = cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(M_PI * tt / T));
        const double c1 = 1.0 / (1.0 - std::pow(b1, (double)(t + 1)));
        const double c2 = 1.0 / (1.0 - std::pow(b2, (double)(t + 1)));
        if (e == hipSuccess) {
            hipLaunchKernelGGL(adam_kernel, dim3(small_grid(m->L.n)), dim3(kBlock), 0, stream, m->prm, m->m, m->v,
                               (const float *)m->grad, m->L.n, (float)lr, (float)b1, (float)b2, (float)c1,
                               (float)c2, 1e-8f);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return status_of(e);
        ++m->step;
    }
    if (loss_out) {
        hipError_t e = hipMemcpyAsync(loss_out, m->losses, sizeof(float) * (size_t)cfg->iters,
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return status_of(e);
    }
    return ADK_OK;
}

int adk_mlp_save(const adk_mlp *m, const char *path)
{
    if (!m || !path) return ADK_EINVAL;
    std::vector<float> buf(3 * (size_t)m->L.n);
    int64_t step = 0;
    int st = adk_mlp_get_state(m, buf.data(), buf.data() + m->L.n, buf.data() + 2 * m->L.n, &step);
    if (st) return st;
    FileHeader h{};
    std::memcpy(h.magic, kMagic, sizeof(kMagic));
    h.Z = m->Z;
    h.nparams = m->L.n;
    h.range = m->range;
    h.omega_a = m->omega_a;
    h.step = step;
    FILE *f = std::fopen(path, "wb");
    if (!f) return ADK_EINVAL;
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? ADK_OK : ADK_EINVAL;
}

int adk_mlp_load(const adk_gas *gas, const char *path, adk_mlp **out)
{
    if (!gas || !path || !out) return ADK_EINVAL;
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return ADK_EINVAL;
    FileHeader h{};
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, kMagic, sizeof(kMagic)) == 0 &&
              h.Z == gas->Z && h.nparams == MlpLayout::of(gas->Z).n && h.step >= 0 && valid_range(h.range);
    std::vector<float> buf;
    if (ok) {
        buf.resize(3 * (size_t)h.nparams);
        ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
        char extra;
        ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the state
    }
    std::fclose(f);
    if (!ok) return ADK_EINVAL;
    adk_mlp *m = nullptr;
    int st = adk_mlp_create(gas, buf.data(), &h.range, &m);
    if (st) return st;
    m->omega_a = h.omega_a;
    const size_t bytes = sizeof(float) * (size_t)h.nparams;
    st = status_of(hipMemcpy(m->m, buf.data() + h.nparams, bytes, hipMemcpyHostToDevice));
    if (!st) st = status_of(hipMemcpy(m->v, buf.data() + 2 * (size_t)h.nparams, bytes, hipMemcpyHostToDevice));
    if (st) {
        adk_mlp_destroy(m);
        return st;
    }
    m->step = h.step;
    *out = m;
    return ADK_OK;
}

int adk_surrogate_step(const adk_gas *gas, const adk_mlp *m, const void *E, int64_t ncells, double dt, void *pops,
                       uint8_t *lo, const adk_window *win, unsigned long long *counters, hipStream_t stream)
{
    if (!gas || !m || !win || ncells < 0) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (!(win->eps >= 0.0) || !std::isfinite(win->eps)) return ADK_EINVAL;
    if (win->prec != ADK_MIXED || win->layout != ADK_LAYOUT_COMPACT) return ADK_EINVAL;
    if (gas->Z != m->Z) return ADK_EINVAL;
    if (win->w < 1 || win->w > 3 || win->w > gas->Z) return ADK_ERANGE;
    if (ncells > 0 && (!E || !pops || !lo)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    SurArgs a{};
    a.st = step_args(gas, dt, win->eps);
    a.prm = m->prm;
    a.L = m->L;
    const MlpFeatures F = features(*m);
    a.au = F.au;
    a.bu = F.bu;
    a.v = (float)(F.av * std::log2(dt * m->omega_a) + F.bv);
    const bool dt_ok = dt >= m->range.dt_lo && dt <= m->range.dt_hi;
    a.E_lo = dt_ok ? m->range.E_lo : INFINITY;
    a.E_hi = dt_ok ? m->range.E_hi : -INFINITY;
    a.cut = window_cutoffs(gas, dt, win->w);  // (takes the gas's lock itself)
    a.counters = counters;
    {
        adk_gas *g = const_cast<adk_gas *>(gas);
        std::lock_guard<std::mutex> lock(g->cut_mu);
        if (g->thr_dt != dt) {
            level_thresholds(*g, dt, kNegligibleXdt, g->thr_E);
            g->thr_dt = dt;
        }
        for (int k = 0; k < ADK_MAX_Z; ++k) a.thr[k] = k < gas->Z ? g->thr_E[k] : 0.0f;
    }
    hipError_t e;
    switch (win->w) {
    case 1: e = adk_surrogate_launch_1(a, (const float *)E, (float *)pops, lo, ncells, stream); break;
    case 2: e = adk_surrogate_launch_2(a, (const float *)E, (float *)pops, lo, ncells, stream); break;
    default: e = adk_surrogate_launch_3(a, (const float *)E, (float *)pops, lo, ncells, stream); break;
    }
    return status_of(e);
}

}  // extern "C"
