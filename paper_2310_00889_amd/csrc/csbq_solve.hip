// csbq_solve.hip -- device kernels of the boundary-integral solves (Section 4):
// GMRES's inner products and updates, the projector L onto the rigid-body
// motions of every body (Section 4.2, the orthogonal projector built from the
// translations and rotations of each body), rigid-body fields (the completion
// flow density and the recovered rigid motion) and the assembly of the
// combined-field operator from the two layer potentials.
//
// Every reduction runs in a fixed order (per-block partial sums, then one
// block over the partials), so a solve is bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "csbq_solve.hpp"

namespace csbq {

namespace {

constexpr int RB = 256;   // threads of a reduction block

__device__ inline double block_sum(double v, double* red /*[RB / 64]*/)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < RB / 64; ++k) s += red[k];
    __syncthreads();
    return s;   // valid in thread 0
}

// partial[j][b] = sum over block b's slice of V[j][i] * w[i]
__global__ __launch_bounds__(RB) void k_mdot_partial(int64_t n, int k, const double* __restrict__ V, int64_t ld,
                                                    const double* __restrict__ w, int64_t slice,
                                                    double* __restrict__ partial)
{
    __shared__ double red[RB / 64];
    const int b = blockIdx.x;
    const int64_t i0 = (int64_t)b * slice, i1 = min(n, i0 + slice);
    for (int j = 0; j < k; ++j) {
        const double* v = V + (int64_t)j * ld;
        double s = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += RB) s = fma(v[i], w[i], s);
        s = block_sum(s, red);
        if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + b] = s;
    }
}

// out[j] (+)= sum_b partial[j][b], in order of b
__global__ __launch_bounds__(RB) void k_mdot_final(int k, int nb, const double* __restrict__ partial,
                                                  double* __restrict__ out, int accumulate)
{
    __shared__ double red[RB / 64];
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
        // contiguous ranges per thread keep the order fixed
        const int per = (nb + RB - 1) / RB;
        const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
        for (int b = b0; b < b1; ++b) s += partial[(int64_t)j * nb + b];
        s = block_sum(s, red);
        if (threadIdx.x == 0) out[j] = accumulate ? out[j] + s : s;
    }
}

// w[i] += sgn * sum_j h[j] V[j][i]
__global__ void k_maxpy(int64_t n, int k, const double* __restrict__ V, int64_t ld, const double* __restrict__ h,
                        double sgn, double* __restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(h[j], V[(int64_t)j * ld + i], s);
    w[i] = fma(sgn, s, w[i]);
}

// y = a x + b y
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = b == 0.0 ? a * x[i] : fma(a, x[i], b * y[i]);
}

// Combined-field operator from the layer potentials of tau (Section 4.1, the
// slender combined-field form): y = tau/2 + D4 tau + eta S tau (+ extra),
// with D4 = dsign * (the evaluator's double layer).  Stokes: dsign = -1 (the
// evaluator's stresslet gives c, c/2, 0 inside, on, outside for a constant
// density, and the integral equations of Section 4 take the double layer of
// the opposite orientation, under which rigid motions lie in the null space of
// I/2 + D4); Laplace: dsign = +1 (dG/dn_y gives -1, -1/2, 0, the orientation
// of Section 4.1's exterior equation).
__global__ void k_combine(int64_t n, const double* __restrict__ tau, const double* __restrict__ usl,
                          const double* __restrict__ udl, double eta, double dsign, const double* __restrict__ extra,
                          double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = fma(0.5, tau[i], fma(eta, usl[i], dsign * udl[i]));
    if (extra) v += extra[i];
    y[i] = v;
}

// Per body (one block each): surface centroid c, area A, first moment M1 =
// sum w (y - c) and second moment J2 = sum w (y - c)(y - c)^T (xx xy xz yy yz
// zz), with the smooth quadrature weights.  geo[b] = c(3) A M1(3) J2(6).
__global__ __launch_bounds__(RB) void k_body_geometry(const int64_t* __restrict__ boff, const double* __restrict__ ny,
                                                      const double* __restrict__ nw, int64_t N,
                                                      double* __restrict__ geo)
{
    __shared__ double red[RB / 64];
    __shared__ double cen[4];
    const int b = blockIdx.x;
    const int64_t n0 = boff[b], n1 = boff[b + 1];
    double s[4] = {0, 0, 0, 0};
    for (int64_t n = n0 + threadIdx.x; n < n1; n += RB) {
        const double w = nw[n];
        s[0] += w;
        for (int d = 0; d < 3; ++d) s[1 + d] = fma(w, ny[d * N + n], s[1 + d]);
    }
    for (int q = 0; q < 4; ++q) {
        const double t = block_sum(s[q], red);
        if (threadIdx.x == 0) cen[q] = t;
    }
    __syncthreads();
    const double A = cen[0];
    const double c[3] = {cen[1] / A, cen[2] / A, cen[3] / A};
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = n0 + threadIdx.x; n < n1; n += RB) {
        const double w = nw[n];
        const double r[3] = {ny[n] - c[0], ny[N + n] - c[1], ny[2 * N + n] - c[2]};
        for (int d = 0; d < 3; ++d) m[d] = fma(w, r[d], m[d]);
        m[3] = fma(w * r[0], r[0], m[3]);
        m[4] = fma(w * r[0], r[1], m[4]);
        m[5] = fma(w * r[0], r[2], m[5]);
        m[6] = fma(w * r[1], r[1], m[6]);
        m[7] = fma(w * r[1], r[2], m[7]);
        m[8] = fma(w * r[2], r[2], m[8]);
    }
    double* g = geo + (int64_t)b * 13;
    for (int q = 0; q < 9; ++q) {
        const double t = block_sum(m[q], red);
        if (threadIdx.x == 0) g[4 + q] = t;
    }
    if (threadIdx.x == 0) {
        g[0] = c[0];
        g[1] = c[1];
        g[2] = c[2];
        g[3] = A;
    }
}

// Per body: the moments of a density against the raw rigid-body basis
// (translations e_k and rotations e_k x (y - c)): mom[b] = (sum w sigma,
// sum w (y - c) x sigma); then coef[b] = Ginv[b] mom[b] (the projection's
// coefficients in that basis).
__global__ __launch_bounds__(RB) void k_body_project(const int64_t* __restrict__ boff, const double* __restrict__ ny,
                                                     const double* __restrict__ nw, int64_t N,
                                                     const double* __restrict__ geo, const double* __restrict__ Ginv,
                                                     const double* __restrict__ sigma, double* __restrict__ coef)
{
    __shared__ double red[RB / 64];
    __shared__ double mom[6];
    const int b = blockIdx.x;
    const int64_t n0 = boff[b], n1 = boff[b + 1];
    const double* g = geo + (int64_t)b * 13;
    const double c[3] = {g[0], g[1], g[2]};
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t n = n0 + threadIdx.x; n < n1; n += RB) {
        const double w = nw[n];
        const double s[3] = {sigma[3 * n], sigma[3 * n + 1], sigma[3 * n + 2]};
        const double r[3] = {ny[n] - c[0], ny[N + n] - c[1], ny[2 * N + n] - c[2]};
        for (int d = 0; d < 3; ++d) m[d] = fma(w, s[d], m[d]);
        m[3] = fma(w, r[1] * s[2] - r[2] * s[1], m[3]);
        m[4] = fma(w, r[2] * s[0] - r[0] * s[2], m[4]);
        m[5] = fma(w, r[0] * s[1] - r[1] * s[0], m[5]);
    }
    for (int q = 0; q < 6; ++q) {
        const double t = block_sum(m[q], red);
        if (threadIdx.x == 0) mom[q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double* Gi = Ginv + (int64_t)b * 36 + threadIdx.x * 6;
        double v = 0.0;
        for (int q = 0; q < 6; ++q) v = fma(Gi[q], mom[q], v);
        coef[(int64_t)b * 6 + threadIdx.x] = v;
    }
}

// out[n] = base[n] + scale * (a_b + beta_b x (y_n - c_b)) for the body b of
// node n (base may be null: zero)
__global__ void k_rigid_field(int64_t N, int B, const int64_t* __restrict__ boff, const double* __restrict__ ny,
                              const double* __restrict__ geo, const double* __restrict__ coef, double scale,
                              const double* __restrict__ base, double* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int lo = 0, hi = B;   // boff[lo] <= n < boff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= n) lo = mid; else hi = mid;
    }
    const double* g = geo + (int64_t)lo * 13;
    const double* cf = coef + (int64_t)lo * 6;
    const double r[3] = {ny[n] - g[0], ny[N + n] - g[1], ny[2 * N + n] - g[2]};
    const double v[3] = {cf[0] + cf[4] * r[2] - cf[5] * r[1], cf[1] + cf[5] * r[0] - cf[3] * r[2],
                         cf[2] + cf[3] * r[1] - cf[4] * r[0]};
    for (int d = 0; d < 3; ++d) out[3 * n + d] = (base ? base[3 * n + d] : 0.0) + scale * v[d];
}

// node ids 0..n-1
__global__ void k_iota64(int64_t n, int64_t* __restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

#define SOLVE_CHECK()                         \
    do {                                      \
        hipError_t e_ = hipGetLastError();    \
        if (e_ != hipSuccess) return (int)e_; \
    } while (0)

int mdot_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096)); }

int launch_mdot(hipStream_t st, int64_t n, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, int accumulate)
{
    if (k <= 0) return 0;
    const int nb = mdot_blocks(n);
    const int64_t slice = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(RB), 0, st, n, k, V, ld, w, slice, partial);
    SOLVE_CHECK();
    hipLaunchKernelGGL(k_mdot_final, dim3(1), dim3(RB), 0, st, k, nb, partial, out, accumulate);
    SOLVE_CHECK();
    return 0;
}

int launch_maxpy(hipStream_t st, int64_t n, int k, const double* V, int64_t ld, const double* h, double sgn,
                 double* w)
{
    if (k <= 0 || n == 0) return 0;
    hipLaunchKernelGGL(k_maxpy, dim3(grid_of(n, 256)), dim3(256), 0, st, n, k, V, ld, h, sgn, w);
    SOLVE_CHECK();
    return 0;
}

int launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y)
{
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_axpby, dim3(grid_of(n, 256)), dim3(256), 0, st, n, a, x, b, y);
    SOLVE_CHECK();
    return 0;
}

int launch_combine(hipStream_t st, int64_t n, const double* tau, const double* usl, const double* udl, double eta,
                   double dsign, const double* extra, double* y)
{
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_combine, dim3(grid_of(n, 256)), dim3(256), 0, st, n, tau, usl, udl, eta, dsign, extra, y);
    SOLVE_CHECK();
    return 0;
}

int launch_body_geometry(hipStream_t st, int B, const int64_t* boff, const double* ny, const double* nw, int64_t N,
                         double* geo)
{
    hipLaunchKernelGGL(k_body_geometry, dim3(B), dim3(RB), 0, st, boff, ny, nw, N, geo);
    SOLVE_CHECK();
    return 0;
}

int launch_body_project(hipStream_t st, int B, const int64_t* boff, const double* ny, const double* nw, int64_t N,
                        const double* geo, const double* Ginv, const double* sigma, double* coef)
{
    hipLaunchKernelGGL(k_body_project, dim3(B), dim3(RB), 0, st, boff, ny, nw, N, geo, Ginv, sigma, coef);
    SOLVE_CHECK();
    return 0;
}

int launch_rigid_field(hipStream_t st, int64_t N, int B, const int64_t* boff, const double* ny, const double* geo,
                       const double* coef, double scale, const double* base, double* out)
{
    if (N == 0) return 0;
    hipLaunchKernelGGL(k_rigid_field, dim3(grid_of(N, 256)), dim3(256), 0, st, N, B, boff, ny, geo, coef, scale,
                       base, out);
    SOLVE_CHECK();
    return 0;
}

int launch_iota64(hipStream_t st, int64_t n, int64_t* v)
{
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_iota64, dim3(grid_of(n, 256)), dim3(256), 0, st, n, v);
    SOLVE_CHECK();
    return 0;
}

}  // namespace csbq
