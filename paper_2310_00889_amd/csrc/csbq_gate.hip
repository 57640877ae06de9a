// csbq_gate.hip -- learned correction-tier gate (not part of the paper's
// method; its criterion, the error estimates of Section 3.2, stays the fallback):
//   k_gate_features    cheap per-pair features from the sampled circles
//   k_gate_mlp         inference: bf16 MFMA (v_mfma_f32_16x16x16_bf16), FP32
//                      accumulation, one 16-pair tile per wavefront step
//   k_gate_select      predicted tier; pairs to escalate to the criterion
//   k_gate_train_step  FP32 forward + backward over a minibatch (one block of
//                      64 threads per sample range, thread j = hidden unit j)
//   k_gate_reduce      deterministic sum of the per-block gradients
//   k_gate_adam        Adam update (Kingma & Ba, 2015)
//   k_gate_labels      training labels: cheapest tier whose correction agrees
//                      with the special quadrature to the label tolerance
#include <hip/hip_runtime.h>

#include <algorithm>

#include "csbq_gate.hpp"
#include "csbq_math.hpp"

namespace csbq {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f)
{
    // round to nearest even (finite inputs)
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(hi, fmaxf(lo, v)); }

// ---------------------------------------------------------------------------
// features of a (target, element) pair, from the element's NCIRC sampled
// circles (GL circles and panel ends): distances and trapezoid decay rates,
// the position of the closest circle, the element's shape and the density's
// band limits.  An on-surface target on its own element gets feature 11 = 1.
// ---------------------------------------------------------------------------
__global__ void k_gate_features(int64_t P, const int* __restrict__ order, const int* __restrict__ pe,
                                const int* __restrict__ pt, const double* __restrict__ xt, int64_t T,
                                const int64_t* __restrict__ tnode, const double* __restrict__ circ,
                                const ElemInfo* __restrict__ info, const int* __restrict__ band, float ltol,
                                float* __restrict__ feat)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int64_t p = order ? (int64_t)order[q] : q;
    const int e = pe[p];
    const int64_t t = pt[p];
    const ElemInfo inf = info[e];
    const double x[3] = {xt[t], xt[T + t], xt[2 * T + t]};
    const int64_t nd = tnode ? tnode[t] : -1;
    const double* cc = circ + (int64_t)e * NCIRC * CIRQ;
    double bd = 1e300, ba = 1e300;
    int kd = 0;
    for (int k = 0; k < NCIRC; ++k) {
        const double* c = cc + k * CIRQ;
        const double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
        const double z = v[0] * c[3] + v[1] * c[4] + v[2] * c[5];
        const double rho = sqrt(fmax(0.0, v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - z * z));
        const double ae = fabs(c[6]);
        const double dr = rho - ae;
        const double d2 = dr * dr + z * z;
        const double cha = (rho > 0.0 && ae > 1e-300) ? d2 / (2.0 * rho * ae) : 1e300;
        if (d2 < bd) {
            bd = d2;
            kd = k;
        }
        ba = fmin(ba, cha);
    }
    const double half = 0.5 * (inf.c - inf.a), mid = 0.5 * (inf.a + inf.c);
    const double xn = (cc[kd * CIRQ + 8] - mid) / half;
    const double dmin = sqrt(bd) + 1e-300;
    const double spd = fmax(cc[kd * CIRQ + 7], 1e-300);
    const double rho_flat = bernstein_rho(xn, dmin / spd / half, -1.0, 1.0);
    const double dc = sqrt((x[0] - inf.cen[0]) * (x[0] - inf.cen[0]) + (x[1] - inf.cen[1]) * (x[1] - inf.cen[1]) +
                           (x[2] - inf.cen[2]) * (x[2] - inf.cen[2]));
    float f[GATE_NF];
    f[0] = clampf((float)log10(dmin / inf.eps_max), -8.f, 4.f);
    f[1] = clampf((float)log10(fmax(ba, 1e-300)), -8.f, 8.f);
    f[2] = (float)fabs(xn);
    f[3] = clampf((float)log10(half * inf.smax / inf.eps_max), -3.f, 3.f);
    f[4] = (float)(inf.fb - 1);
    f[5] = band[2 * e] / 16.f;
    f[6] = band[2 * e + 1] / 16.f;
    f[7] = clampf((float)log10(dc / inf.rad + 1e-300), -4.f, 4.f);
    f[8] = clampf((float)log10(dmin / (half * inf.smax)), -8.f, 4.f);
    f[9] = clampf((float)log10(fmax(log(rho_flat), 1e-12)), -12.f, 3.f);
    f[10] = ltol / 10.f;
    f[11] = (nd >= 0 && nd / NPE == e) ? 1.f : 0.f;
    for (int k = GATE_NU; k < GATE_NF; ++k) f[k] = 0.f;
    float4* o = reinterpret_cast<float4*>(feat + p * GATE_NF);
    for (int k = 0; k < GATE_NF / 4; ++k) o[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

// ---------------------------------------------------------------------------
// inference.  Fragments of v_mfma_f32_16x16x16_bf16 (one 64-lane wavefront):
//   A (16 x 16, row-major M x K): lane l holds A[l % 16][4 (l / 16) + i], i < 4
//   B (16 x 16, K x N):           lane l holds B[4 (l / 16) + i][l % 16]
//   D (16 x 16 FP32):             lane l holds D[4 (l / 16) + i][l % 16]
// Weights arrive pre-arranged as B fragments (bf16, [fragment][lane][4]);
// activations go through LDS as bf16 rows so the next layer reads A
// fragments as one 8-byte load per lane.
// ---------------------------------------------------------------------------
constexpr int GM_WAVES = 4;
// s_waitcnt immediate that waits for the wave's LDS operations only
// (lgkmcnt 0; vmcnt and expcnt at their maxima, so a feature load in flight
// is not waited for)
constexpr int LDS_DONE = 0xC07F;

__global__ __launch_bounds__(64 * GM_WAVES) void k_gate_mlp(int64_t P, const float* __restrict__ feat,
                                                            const uint16_t* __restrict__ wfrag,
                                                            const float* __restrict__ bias, float tau_esc,
                                                            int8_t* __restrict__ tier, uint8_t* __restrict__ esc,
                                                            float* __restrict__ logits)
{
    __shared__ __attribute__((aligned(16))) unsigned short wl[GATE_NFRAG * GATE_FRAG_ELEMS];
    __shared__ float bl[GATE_NBIAS];
    __shared__ __attribute__((aligned(16))) unsigned short hl[GM_WAVES][16][GATE_H + 8];
    __shared__ float zl[GM_WAVES][16][17];
    for (int i = threadIdx.x; i < GATE_NFRAG * GATE_FRAG_ELEMS; i += blockDim.x) wl[i] = wfrag[i];
    for (int i = threadIdx.x; i < GATE_NBIAS; i += blockDim.x) bl[i] = bias[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;   // A row / B,D column; k quarter
    const v4s* wf = reinterpret_cast<const v4s*>(wl);
    const int64_t ntile = (P + 15) / 16, tstep = (int64_t)gridDim.x * GM_WAVES;
    // lane (r, q) holds features 4q .. 4q + 3 of the tile's pair r; the next
    // tile's are loaded while this one is computed
    auto load_feat = [&](int64_t tl) {
        const int64_t p = tl * 16 + r;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tl < ntile && p < P) v = reinterpret_cast<const float4*>(feat + p * GATE_NF)[q];
        return v;
    };
    float4 vnext = load_feat((int64_t)blockIdx.x * GM_WAVES + wv);
    for (int64_t tile = (int64_t)blockIdx.x * GM_WAVES + wv; tile < ntile; tile += tstep) {
        const int64_t p0 = tile * 16;
        const float4 v = vnext;
        vnext = load_feat(tile + tstep);
        // feature 11 (own element) of pair r sits in lane r + 32 (q = 2, w)
        const float own = __shfl(v.w, r + 32, 64);
        // layer 1: A = features of the tile's 16 pairs
        v4s a;
        {
            a[0] = (short)f2bf(v.x);
            a[1] = (short)f2bf(v.y);
            a[2] = (short)f2bf(v.z);
            a[3] = (short)f2bf(v.w);
        }
        int fo = 0;   // fragment offset
        int bo = 0;   // bias offset
#pragma unroll
        for (int layer = 0; layer < 3; ++layer) {
            const int nk = layer == 0 ? 1 : 4;
            v4s ak[4];
            if (layer == 0) {
                ak[0] = a;
            } else {
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    ak[kb] = *reinterpret_cast<const v4s*>(&hl[wv][r][kb * 16 + 4 * q]);
            }
            v4f acc[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    if (kb < nk)
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ak[kb], wf[(fo + kb * 4 + nb) * 64 + lane],
                                                                           acc[nb], 0, 0, 0);
                }
            }
            fo += nk * 4;
            // bias, ReLU, back to LDS as bf16 rows (the next layer's A)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float h = fmaxf(acc[nb][i] + bl[bo + nb * 16 + r], 0.f);
                    hl[wv][4 * q + i][nb * 16 + r] = f2bf(h);
                }
            bo += GATE_H;
            __builtin_amdgcn_s_waitcnt(LDS_DONE);
            __builtin_amdgcn_wave_barrier();
        }
        // output layer: 64 -> 16 (GATE_NO used)
        v4f z = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const v4s ah = *reinterpret_cast<const v4s*>(&hl[wv][r][kb * 16 + 4 * q]);
            z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, wf[(fo + kb) * 64 + lane], z, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) zl[wv][4 * q + i][r] = z[i] + bl[bo + r];
        __builtin_amdgcn_s_waitcnt(LDS_DONE);
        __builtin_amdgcn_wave_barrier();
        if (lane < 16) {
            const int64_t p = p0 + lane;
            if (p < P) {
                float s[GATE_NO];
                int tr = 0;
                for (int k = 0; k < GATE_NO; ++k) {
                    const float zz = zl[wv][lane][k];
                    s[k] = 1.f / (1.f + __expf(-zz));
                    if (logits) logits[p * GATE_NO + k] = zz;
                }
                // predicted tier: the last ordinal output above one half
                for (int k = 0; k < GATE_NO; ++k)
                    if (s[k] > 0.5f) tr = k + 1;
                const bool up = tr < GATE_NO && s[tr] > tau_esc;   // risk that the tier is too low
                tier[p] = (int8_t)tr;
                esc[p] = (uint8_t)((up || tr == TIER_FULL || own > 0.5f) ? 1 : 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// final tier of the confident pairs; flags (in element-major order) of the
// pairs the criterion decides
// On an element closed at its ends (fb == 2) the far-field rule already is the
// 32 x 32 rule of tier 1, so a tier-1 correction would be zero: a predicted
// tier 1 there means "the far-field rule is not enough" and becomes tier 2.
__global__ void k_gate_select(int64_t P, const int* __restrict__ perm, const int* __restrict__ pe,
                              const ElemInfo* __restrict__ info, const uint8_t* __restrict__ esc,
                              const int8_t* __restrict__ tier_mlp, int8_t* __restrict__ tier,
                              uint8_t* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int p = perm[i];
    const uint8_t f = esc[p];
    flag[i] = f;
    if (!f) {
        int8_t tr = tier_mlp[p];
        if (tr == TIER_UP1 && info[pe[p]].fb == 2) tr = TIER_UP2;
        tier[p] = tr;
    }
}

// ---------------------------------------------------------------------------
// training: FP32 forward and backward over samples [off + b spb, off +
// (b + 1) spb) of the permuted set, gradients of the weighted ordinal
// cross-entropy  sum_k -(w_k y_k log s_k + (1 - y_k) log(1 - s_k)),
// y_k = [label > k], accumulated per block (thread j owns unit j's weights).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_gate_train_step(int64_t off, int64_t n, int spb,
                                                        const int64_t* __restrict__ perm,
                                                        const float* __restrict__ feat,
                                                        const int8_t* __restrict__ label,
                                                        const float* __restrict__ W, const float* __restrict__ posw,
                                                        float* __restrict__ partial)
{
    __shared__ float w[GATE_NW];
    __shared__ float xs[GATE_NF], h1[GATE_H], h2[GATE_H], h3[GATE_H], dz[GATE_NO], d3[GATE_H], d2[GATE_H];
    __shared__ float lsum[GATE_NO];
    const int j = threadIdx.x;
    for (int i = j; i < GATE_NW; i += 64) w[i] = W[i];
    float g1[GATE_NF], g2[GATE_H], g3[GATE_H], g4[GATE_NO];
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gb4 = 0.f, loss = 0.f;
    for (int k = 0; k < GATE_NF; ++k) g1[k] = 0.f;
    for (int k = 0; k < GATE_H; ++k) g2[k] = g3[k] = 0.f;
    for (int k = 0; k < GATE_NO; ++k) g4[k] = 0.f;
    __syncthreads();
    const int64_t s0 = off + (int64_t)blockIdx.x * spb;
    const int64_t s1 = min(off + n, s0 + spb);
    for (int64_t s = s0; s < s1; ++s) {
        const int64_t idx = perm[s];
        if (j < GATE_NF) xs[j] = feat[idx * GATE_NF + j];
        const int y = label[idx];
        __syncthreads();
        float a1 = w[GB1 + j];
        for (int k = 0; k < GATE_NF; ++k) a1 = fmaf(w[GW1 + k * GATE_H + j], xs[k], a1);
        h1[j] = fmaxf(a1, 0.f);
        __syncthreads();
        float a2 = w[GB2 + j];
        for (int k = 0; k < GATE_H; ++k) a2 = fmaf(w[GW2 + k * GATE_H + j], h1[k], a2);
        h2[j] = fmaxf(a2, 0.f);
        __syncthreads();
        float a3 = w[GB3 + j];
        for (int k = 0; k < GATE_H; ++k) a3 = fmaf(w[GW3 + k * GATE_H + j], h2[k], a3);
        h3[j] = fmaxf(a3, 0.f);
        __syncthreads();
        if (j < GATE_NO) {
            float z = w[GB4 + j];
            for (int k = 0; k < GATE_H; ++k) z = fmaf(w[GW4 + k * GATE_NO + j], h3[k], z);
            const float yk = (y > j) ? 1.f : 0.f;
            const float wk = posw[j];
            // log s = -softplus(-z), log(1 - s) = -softplus(z)
            const float sp_pos = fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z)));    // softplus(z)
            const float sp_neg = sp_pos - z;                                    // softplus(-z)
            loss += wk * yk * sp_neg + (1.f - yk) * sp_pos;
            const float sg = 1.f / (1.f + __expf(-z));
            dz[j] = -wk * yk * (1.f - sg) + (1.f - yk) * sg;
        }
        __syncthreads();
        // output layer
        float e3 = 0.f;
        for (int c = 0; c < GATE_NO; ++c) {
            g4[c] = fmaf(h3[j], dz[c], g4[c]);
            e3 = fmaf(w[GW4 + j * GATE_NO + c], dz[c], e3);
        }
        if (j < GATE_NO) gb4 += dz[j];
        const float dd3 = a3 > 0.f ? e3 : 0.f;
        d3[j] = dd3;
        __syncthreads();
        gb3 += dd3;
        float e2 = 0.f;
        for (int k = 0; k < GATE_H; ++k) {
            g3[k] = fmaf(h2[k], dd3, g3[k]);
            e2 = fmaf(w[GW3 + j * GATE_H + k], d3[k], e2);
        }
        const float dd2 = a2 > 0.f ? e2 : 0.f;
        d2[j] = dd2;
        __syncthreads();
        gb2 += dd2;
        float e1 = 0.f;
        for (int k = 0; k < GATE_H; ++k) {
            g2[k] = fmaf(h1[k], dd2, g2[k]);
            e1 = fmaf(w[GW2 + j * GATE_H + k], d2[k], e1);
        }
        const float dd1 = a1 > 0.f ? e1 : 0.f;
        gb1 += dd1;
        for (int k = 0; k < GATE_NF; ++k) g1[k] = fmaf(xs[k], dd1, g1[k]);
        __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * (GATE_NW + 1);
    for (int k = 0; k < GATE_NF; ++k) out[GW1 + k * GATE_H + j] = g1[k];
    for (int k = 0; k < GATE_H; ++k) {
        out[GW2 + k * GATE_H + j] = g2[k];
        out[GW3 + k * GATE_H + j] = g3[k];
    }
    for (int c = 0; c < GATE_NO; ++c) out[GW4 + j * GATE_NO + c] = g4[c];
    out[GB1 + j] = gb1;
    out[GB2 + j] = gb2;
    out[GB3 + j] = gb3;
    if (j < GATE_NO) {
        out[GB4 + j] = gb4;
        lsum[j] = loss;
    }
    __syncthreads();
    if (j == 0) out[GATE_NW] = lsum[0] + lsum[1] + lsum[2] + lsum[3];
}

__global__ void k_gate_reduce(int nblk, const float* __restrict__ partial, float scale, float* __restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > GATE_NW) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * (GATE_NW + 1) + i];
    grad[i] = s * scale;
}

__global__ void k_gate_adam(float* __restrict__ W, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= GATE_NW) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// label = the cheapest tier whose correction agrees with the special
// quadrature to thr (per output kind, in the unscaled sums): 0 = skip
// (agreement of zero), 1..3 = the upsampled rules, else 4
__global__ void k_gate_labels(int64_t P, const double* __restrict__ c1, const double* __restrict__ c2,
                              const double* __restrict__ c3, const double* __restrict__ cf, double thr_s,
                              double thr_d, int8_t* __restrict__ label)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double* cs[4] = {nullptr, c1, c2, c3};
    int lab = TIER_FULL;
    for (int k = 0; k < 4; ++k) {
        double es = 0.0, ed = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double ref_s = cf[p * 6 + c], ref_d = cf[p * 6 + 3 + c];
            const double vs = k ? cs[k][p * 6 + c] : 0.0, vd = k ? cs[k][p * 6 + 3 + c] : 0.0;
            es = fmax(es, fabs(vs - ref_s));
            ed = fmax(ed, fabs(vd - ref_d));
        }
        if (es <= thr_s && ed <= thr_d) {
            lab = k;
            break;
        }
    }
    label[p] = (int8_t)lab;
}

#define GATE_LAUNCH_CHECK()                             \
    do {                                                \
        hipError_t e_ = hipGetLastError();              \
        if (e_ != hipSuccess) return (int)e_;           \
    } while (0)

int launch_gate_features(hipStream_t st, int64_t P, const int* order, const int* pe, const int* pt, const double* xt,
                         int64_t T, const int64_t* tnode, const double* circ, const ElemInfo* info, const int* band,
                         float ltol, float* feat)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_gate_features, dim3((unsigned)((P + 127) / 128)), dim3(128), 0, st, P, order, pe, pt, xt, T,
                       tnode, circ, info, band, ltol, feat);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_mlp(hipStream_t st, int64_t P, const float* feat, const uint16_t* wfrag, const float* bias,
                    float tau_esc, int8_t* tier, uint8_t* esc, float* logits)
{
    if (P == 0) return 0;
    const int64_t ntile = (P + 15) / 16;
    const int64_t want = (ntile + GM_WAVES - 1) / GM_WAVES;
    const unsigned grid = (unsigned)std::min<int64_t>(want, 256 * 16);
    hipLaunchKernelGGL(k_gate_mlp, dim3(grid), dim3(64 * GM_WAVES), 0, st, P, feat, wfrag, bias, tau_esc, tier, esc,
                       logits);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_select(hipStream_t st, int64_t P, const int* perm, const int* pe, const ElemInfo* info,
                       const uint8_t* esc, const int8_t* tier_mlp, int8_t* tier, uint8_t* flag)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_gate_select, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, perm, pe, info, esc,
                       tier_mlp, tier, flag);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_train_step(hipStream_t st, int nblk, int spb, int64_t off, int64_t n, const int64_t* perm,
                           const float* feat, const int8_t* label, const float* W, const float* posw, float* partial)
{
    hipLaunchKernelGGL(k_gate_train_step, dim3(nblk), dim3(64), 0, st, off, n, spb, perm, feat, label, W, posw,
                       partial);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_reduce(hipStream_t st, int nblk, const float* partial, float scale, float* grad)
{
    hipLaunchKernelGGL(k_gate_reduce, dim3((GATE_NW + 1 + 255) / 256), dim3(256), 0, st, nblk, partial, scale, grad);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_adam(hipStream_t st, float* W, const float* grad, float* m, float* v, float lr, float b1, float b2,
                     float eps, int step)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_gate_adam, dim3((GATE_NW + 255) / 256), dim3(256), 0, st, W, grad, m, v, lr, b1, b2, eps, c1,
                       c2);
    GATE_LAUNCH_CHECK();
    return 0;
}

int launch_gate_labels(hipStream_t st, int64_t P, const double* c_up1, const double* c_up2, const double* c_up3,
                       const double* c_full, double thr_s, double thr_d, int8_t* label)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_gate_labels, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, c_up1, c_up2, c_up3,
                       c_full, thr_s, thr_d, label);
    GATE_LAUNCH_CHECK();
    return 0;
}

}  // namespace csbq
