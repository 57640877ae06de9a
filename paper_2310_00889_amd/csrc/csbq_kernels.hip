// csbq_kernels.hip -- gfx950 kernels of the Stokes layer-potential evaluator.
//
// Pipeline of one evaluation (each step cites the passage of the paper it
// implements):
//   k_expand        surface nodes, normals, smooth weights (Section 3.1,
//                   weights of the Nystrom rule in Section 3.2.1)
//   k_expand_up     upsampled tensor rules of each element (x2 and x4 in s
//                   and t) used as cheap corrections for mildly near pairs
//   k_prep_sigma    sigma*w, Fourier coefficients of the density on every GL
//                   circle, and the density's band limits
//   k_sigma_up      density on the upsampled rules (interpolation in s and t)
//   k_far           smooth Nystrom sum over every source (Section 3.2.1)
//   k_search_*      candidate (target, element) pairs: bounding ball of the
//                   element grown by its near-region radius (Section 3.2.1)
//   k_classify      per pair: closest circle, GL (Bernstein ellipse) and
//                   trapezoid error estimates -> correction tier
//   k_corr_up       upsampled tiers: upsampled rule minus the smooth rule
//   k_corr_full     special quadrature (Sections 3.2.2-3.2.4) minus the
//                   smooth rule, one wavefront per pair
//   k_reduce        far sum + corrections in a fixed order per target
#include <hip/hip_runtime.h>

#include <mutex>

#include "csbq_kernels.hpp"
#include "csbq_math.hpp"

namespace csbq {

__constant__ double c_gx[NS];        // GL nodes on [-1,1], ascending
__constant__ double c_gw[NS];        // GL weights
__constant__ double c_lam[NS];       // barycentric weights of the GL nodes
__constant__ double c_D[NS * NS];    // differentiation matrix on [-1,1]
__constant__ double c_T[NS * NS];    // Legendre transform: coef_k = sum_i T[k][i] f_i
__constant__ double c_cos[NT];       // cos(2 pi j / NT)
__constant__ double c_sin[NT];
__constant__ double c_cos128[128];   // cos(2 pi k / 128), for trapezoid rules of nt, 2nt, 4nt points
__constant__ double c_sin128[128];

static constexpr double PI = 3.14159265358979323846;

int upload_constants(const double* gx, const double* gw, const double* lam, const double* D, const double* T)
{
    double cs[NT], sn[NT];
    for (int j = 0; j < NT; ++j) {
        cs[j] = cos(2.0 * PI * j / NT);
        sn[j] = sin(2.0 * PI * j / NT);
    }
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_gx), gx, sizeof(double) * NS)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_gw), gw, sizeof(double) * NS)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_lam), lam, sizeof(double) * NS)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_D), D, sizeof(double) * NS * NS)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_T), T, sizeof(double) * NS * NS)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_cos), cs, sizeof(double) * NT)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_sin), sn, sizeof(double) * NT)) != hipSuccess) return (int)e;
    double c128[128], s128[128];
    for (int j = 0; j < 128; ++j) {
        c128[j] = cos(2.0 * PI * j / 128);
        s128[j] = sin(2.0 * PI * j / 128);
    }
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_cos128), c128, sizeof(double) * 128)) != hipSuccess) return (int)e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_sin128), s128, sizeof(double) * 128)) != hipSuccess) return (int)e;
    return 0;
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double xh = 0.5 * x;
    double e = fma(-xh, y * y, 0.5);   // y <- y (3/2 - x y^2 / 2)
    y = fma(y, e, y);
    e = fma(-xh, y * y, 0.5);
    return fma(y, e, y);
}

// 1/sqrt(x) for x > 0 from the hardware estimate y (relative error about
// 5e-8) and one Newton step, y (3 - x y^2) / 2: the step leaves a relative
// error of 1.5 e^2 + O(e^3) < 1e-14 for an estimate error e, always low.
__device__ __forceinline__ double rsqrt_nr1(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return (0.5 * y) * fma(-x, y * y, 3.0);
}

// 2/sqrt(rr) of a squared distance, 0 for rr == 0 (a source at the target
// itself): rsqrt_nr1 without its factor 1/2, which the callers take out of
// their sums as an exact power of two.  The estimate of 0 is +inf; clearing
// its high word leaves +0 before the Newton step, so the coincident pair adds
// nothing.  rr is a sum of squares of coordinate differences: its high word
// is zero only for rr = 0 or |r| below 1e-154.
__device__ __forceinline__ double rsqrt2_or_zero(double rr)
{
    const double y0 = __builtin_amdgcn_rsq(rr);
    const int hi = (__double2hiint(rr) == 0) ? 0 : __double2hiint(y0);
    const double y = __hiloint2double(hi, __double2loint(y0));
    return y * fma(-rr, y * y, 3.0);
}

// One source record (y, n, sigma*w as five 16-byte pairs A..F) against one
// target x, accumulated in scaled form: with q = 2/r, sa += q (sigma w),
// sb += q^3 (r.sigma w) r and sd += q^5 (r.n)(r.sigma w) r, i.e. 2, 8 and 32
// times the single-layer's two parts and the double-layer term.
__device__ __forceinline__ void pair_scaled(const double x[3], double2 A, double2 B, double2 C, double2 D, double2 F,
                                            double sa[3], double sb[3], double sd[3])
{
    // A = (y0, y1), B = (y2, n0), C = (n1, n2), D = (w0, w1), F = (w2, -)
    const double r0 = x[0] - A.x, r1 = x[1] - A.y, r2 = x[2] - B.x;
    const double rr = fma(r0, r0, fma(r1, r1, r2 * r2));
    const double q = rsqrt2_or_zero(rr);   // branch-free self term
    const double rs = fma(r0, D.x, fma(r1, D.y, r2 * F.x));
    const double rn = fma(r0, B.y, fma(r1, C.x, r2 * C.y));
    const double q2 = q * q;
    const double b = rs * (q * q2);
    const double cD = (rn * b) * q2;
    sa[0] = fma(q, D.x, sa[0]);
    sa[1] = fma(q, D.y, sa[1]);
    sa[2] = fma(q, F.x, sa[2]);
    sb[0] = fma(b, r0, sb[0]);
    sb[1] = fma(b, r1, sb[1]);
    sb[2] = fma(b, r2, sb[2]);
    sd[0] = fma(cD, r0, sd[0]);
    sd[1] = fma(cD, r1, sd[1]);
    sd[2] = fma(cD, r2, sd[2]);
}

// The Laplace pair (Section 4.1: G = 1/(4 pi |r|) and its normal derivative
// (r.n)/(4 pi |r|^3)) on the scalar density held in the record's first
// component: sa[0] += q (sigma w), sd[0] += q^3 (r.n)(sigma w), i.e. 2 and 8
// times the single and double layers' terms (the 1/(4 pi) is applied last).
__device__ __forceinline__ void pair_scaled_lap(const double x[3], double2 A, double2 B, double2 C, double2 D,
                                                double sa[3], double sd[3])
{
    const double r0 = x[0] - A.x, r1 = x[1] - A.y, r2 = x[2] - B.x;
    const double rr = fma(r0, r0, fma(r1, r1, r2 * r2));
    const double q = rsqrt2_or_zero(rr);
    const double rn = fma(r0, B.y, fma(r1, C.x, r2 * C.y));
    const double qw = q * D.x;
    sa[0] += qw;
    sd[0] = fma(rn * qw, q * q, sd[0]);
}

template <int KER>
__device__ __forceinline__ void pair_acc(const double x[3], double2 A, double2 B, double2 C, double2 D, double2 F,
                                         double sa[3], double sb[3], double sd[3])
{
    if constexpr (KER == KER_LAPLACE)
        pair_scaled_lap(x, A, B, C, D, sa, sd);
    else
        pair_scaled(x, A, B, C, D, F, sa, sb, sd);
}

// the six output slots (S: 0..2, D: 3..5) of the scaled sums; the Laplace
// layers fill slots 0 and 3 only
template <int KER>
__device__ __forceinline__ void scaled_out(const double sa[3], const double sb[3], const double sd[3], double o[6])
{
    if constexpr (KER == KER_LAPLACE) {
        o[0] = 0.5 * sa[0];
        o[3] = 0.125 * sd[0];
        o[1] = o[2] = o[4] = o[5] = 0.0;
    } else {
        for (int d = 0; d < 3; ++d) {
            o[d] = fma(0.5, sa[d], 0.125 * sb[d]);
            o[3 + d] = 0.03125 * sd[d];
        }
    }
}

// interpolate the CLQ centerline quantities of element data clq (layout
// [CLQ][NS]) at normalised x, then build the frame
__device__ inline void frame_at_x(const double* __restrict__ clq, double x, Frame& f)
{
    double l[NS];
    bary_weights(x, c_gx, c_lam, l);
    double q[CLQ];
#pragma unroll
    for (int k = 0; k < CLQ; ++k) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) v += l[i] * clq[k * NS + i];
        q[k] = v;
    }
    frame_from_q(q, f);
}

// 1/x from the hardware reciprocal refined by two Newton steps (~1 ulp)
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = r * fma(-x, r, 2.0);
    return r * fma(-x, r, 2.0);
}

// barycentric weights (as bary_weights / bary_weights_rel) with refined
// hardware reciprocals in place of divisions
__device__ inline void bary_weights_rcp(double x, double* l)
{
    double sum = 0.0;
    int hit = -1;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double dx = x - c_gx[i];
        if (dx == 0.0) hit = i;
        l[i] = c_lam[i] * rcp_nr(dx);
        sum += l[i];
    }
    if (hit >= 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) l[i] = (i == hit) ? 1.0 : 0.0;
        return;
    }
    const double is = rcp_nr(sum);
#pragma unroll
    for (int i = 0; i < NS; ++i) l[i] *= is;
}

// As bary_weights_rel_rcp with the node offsets and barycentric weights read
// from a per-wavefront table (LDS): tab[2 i] = x_i0 - x_i (exactly 0 at i0, so
// that x - x_i0 = du there), tab[2 i + 1] = lam_i.  Read inside a loop with
// barriers, the table is not kept in registers across the loop (the
// constants, and the 16 masks of a test against i0, would be).
__device__ inline void bary_weights_rel_tab(const double* tab, double du, double* l)
{
    int hit = -1;
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double dx = tab[2 * i] + du;
        if (dx == 0.0) hit = i;
        l[i] = tab[2 * i + 1] * rcp_nr(dx == 0.0 ? 1.0 : dx);
        sum += l[i];
    }
    if (hit >= 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) l[i] = (i == hit) ? 1.0 : 0.0;
        return;
    }
    const double is = rcp_nr(sum);
#pragma unroll
    for (int i = 0; i < NS; ++i) l[i] *= is;
}

__device__ inline void bary_weights_rel_rcp(int i0, double du, double* l)
{
    // a node that falls on a GL node (x - x_i == 0 exactly, e.g. the nodes
    // of a sub-panel that is the whole panel) takes that node's values
    int hit = -1;
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double dx = (i == i0) ? du : (c_gx[i0] - c_gx[i]) + du;
        if (dx == 0.0) hit = i;
        l[i] = c_lam[i] * rcp_nr(dx == 0.0 ? 1.0 : dx);
        sum += l[i];
    }
    if (hit >= 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) l[i] = (i == hit) ? 1.0 : 0.0;
        return;
    }
    const double is = rcp_nr(sum);
#pragma unroll
    for (int i = 0; i < NS; ++i) l[i] *= is;
}

// position/tangent/radius only (for the distance searches of the
// classification, which only steer estimates): barycentric interpolation with
// the weights formed on the fly from the hardware reciprocal refined by two
// Newton steps (~1 ulp); a node hit (x equal to a GL node) takes the node's
// values.  The node loop is only partly unrolled so that the element's data
// is read in the loop rather than held in registers.
__device__ inline void circle_at_x(const double* __restrict__ clq, double x, double* X, double* t, double* E)
{
    double xp[3] = {0.0, 0.0, 0.0}, e = 0.0, sum = 0.0;
    X[0] = X[1] = X[2] = 0.0;
    int hit = -1;
#pragma unroll 2
    for (int i = 0; i < NS; ++i) {
        const double dx = x - c_gx[i];
        if (dx == 0.0) hit = i;
        double r = __builtin_amdgcn_rcp(dx);
        r = r * fma(-dx, r, 2.0);
        r = r * fma(-dx, r, 2.0);
        const double li = c_lam[i] * r;
        sum += li;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            X[d] += li * clq[(Q_X + d) * NS + i];
            xp[d] += li * clq[(Q_XP + d) * NS + i];
        }
        e += li * clq[Q_E * NS + i];
    }
    if (hit >= 0) {
        for (int d = 0; d < 3; ++d) {
            X[d] = clq[(Q_X + d) * NS + hit];
            xp[d] = clq[(Q_XP + d) * NS + hit];
        }
        e = clq[Q_E * NS + hit];
    } else {
        double is = __builtin_amdgcn_rcp(sum);
        is = is * fma(-sum, is, 2.0);
        is = is * fma(-sum, is, 2.0);
        for (int d = 0; d < 3; ++d) {
            X[d] *= is;
            xp[d] *= is;
        }
        e *= is;
    }
    *E = e;
    double it = rsqrt_nr(dot3(xp, xp));
    for (int d = 0; d < 3; ++d) t[d] = xp[d] * it;
}

__device__ inline void circle_dist(const double* X, const double* t, double E, const double* x, double* d2, double* cha)
{
    double v[3] = {x[0] - X[0], x[1] - X[1], x[2] - X[2]};
    double z = dot3(v, t);
    double r2 = fmax(0.0, dot3(v, v) - z * z);
    double rho = sqrt(r2);
    // a circle of vanishing radius (the pole of a body of revolution, where the
    // interpolated radius may even be a tiny negative number) gives a constant
    // angular integrand: no trapezoid error
    const double ae = fabs(E);
    double dr = rho - ae;
    *d2 = dr * dr + z * z;
    *cha = (rho > 0.0 && ae > 1e-300) ? *d2 / (2.0 * rho * ae) : 1e300;
}

// ---------------------------------------------------------------------------
// geometry expansion (Section 3.1, Section 3.2.1 weights)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_expand(int E, const double* __restrict__ xc, const double* __restrict__ eps,
                                                const double* __restrict__ e1, const double* __restrict__ sa,
                                                const double* __restrict__ sc, const int* __restrict__ esign,
                                                const int* __restrict__ ebody, const int* __restrict__ egroup, double* __restrict__ clq,
                                                double* __restrict__ circ, ElemInfo* __restrict__ info,
                                                double* __restrict__ ny, double* __restrict__ nn,
                                                double* __restrict__ nw, int64_t N, int closed_fb)
{
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ double sq[CLQ * NS];
    __shared__ double red[512];
    __shared__ double cen[3];
    const double a = sa[e], c = sc[e];
    const double ds = 2.0 / (c - a);
    if (tid < NS * 3) {
        int i = tid / 3, d = tid % 3;
        sq[(Q_X + d) * NS + i] = xc[((int64_t)e * NS + i) * 3 + d];
        sq[(Q_F + d) * NS + i] = e1[((int64_t)e * NS + i) * 3 + d];
    }
    if (tid < NS) sq[Q_E * NS + tid] = eps[(int64_t)e * NS + tid];
    __syncthreads();
    // first derivatives of x_c, eps, e1 (spectral differentiation on the panel);
    // samples are centred first so the O(|x_c|) offset does not enter the
    // rounding of the differentiated values
    if (tid < NS * 7) {
        int i = tid % NS, k = tid / NS;
        int src = (k < 3) ? (Q_X + k) : (k == 3 ? Q_E : Q_F + (k - 4));
        int dst = (k < 3) ? (Q_XP + k) : (k == 3 ? Q_EP : Q_FP + (k - 4));
        double m = 0.0;
        for (int j = 0; j < NS; ++j) m += sq[src * NS + j];
        m *= 1.0 / NS;
        double v = 0.0;
        for (int j = 0; j < NS; ++j) v += c_D[i * NS + j] * (sq[src * NS + j] - m);
        sq[dst * NS + i] = v * ds;
    }
    __syncthreads();
    if (tid < NS * 3) {
        int i = tid % NS, d = tid / NS;
        double m = 0.0;
        for (int j = 0; j < NS; ++j) m += sq[(Q_XP + d) * NS + j];
        m *= 1.0 / NS;
        double v = 0.0;
        for (int j = 0; j < NS; ++j) v += c_D[i * NS + j] * (sq[(Q_XP + d) * NS + j] - m);
        sq[(Q_XPP + d) * NS + i] = v * ds;
    }
    __syncthreads();
    if (tid < CLQ * NS) clq[(int64_t)e * CLQ * NS + tid] = sq[tid];
    // nodes
    const int i = tid / NT, j = tid % NT;
    double q[CLQ];
    for (int k = 0; k < CLQ; ++k) q[k] = sq[k * NS + i];
    Frame f;
    frame_from_q(q, f);
    double y[3], ys[3], yt[3];
    surface_at(f, c_cos[j], c_sin[j], y, ys, yt);
    double jn[3];
    cross3(yt, ys, jn);
    double J = sqrt(dot3(jn, jn));
    double sg = (double)esign[e];
    const int64_t n = (int64_t)e * NPE + tid;
    for (int d = 0; d < 3; ++d) {
        ny[d * N + n] = y[d];
        nn[d * N + n] = sg * jn[d] / J;
    }
    nw[n] = J * c_gw[i] * (0.5 * (c - a)) * (2.0 * PI / NT);
    // bounding-ball centre = mean node
    for (int d = 0; d < 3; ++d) {
        red[tid] = y[d];
        __syncthreads();
        for (int s = 256; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) cen[d] = red[0] / NPE;
        __syncthreads();
    }
    // circles: GL circles and the two panel ends
    double rad = 0.0, epsm = 0.0, smx = 0.0;
    if (tid < NCIRC) {
        Frame g;
        double xn;
        if (tid == 0)
            xn = -1.0;
        else if (tid == NCIRC - 1)
            xn = 1.0;
        else
            xn = c_gx[tid - 1];
        frame_at_x(sq, xn, g);
        double sp = speed_bound(g);
        double* cp = circ + ((int64_t)e * NCIRC + tid) * CIRQ;
        for (int d = 0; d < 3; ++d) {
            cp[d] = g.X[d];
            cp[3 + d] = g.t[d];
        }
        cp[6] = g.E;
        cp[7] = sp;
        cp[8] = 0.5 * (a + c) + 0.5 * (c - a) * xn;
        double dx[3] = {g.X[0] - cen[0], g.X[1] - cen[1], g.X[2] - cen[2]};
        rad = sqrt(dot3(dx, dx)) + fabs(g.E);
        epsm = fabs(g.E);
        smx = sp;
    }
    // block max of rad, epsm, smx
    double vals[3] = {rad, epsm, smx};
    double outv[3];
    for (int k = 0; k < 3; ++k) {
        red[tid] = vals[k];
        __syncthreads();
        for (int s = 256; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
            __syncthreads();
        }
        outv[k] = red[0];
        __syncthreads();
    }
    if (tid == 0) {
        ElemInfo inf;
        inf.a = a;
        inf.c = c;
        for (int d = 0; d < 3; ++d) inf.cen[d] = cen[d];
        inf.rad = outv[0] * 1.02 + 0.01 * outv[1];
        inf.eps_max = outv[1];
        inf.smax = outv[2];
        inf.sign = esign[e];
        inf.body = ebody[e];
        // a cross-section that closes at a panel end (a body of revolution
        // described in polar angle, e.g. a sphere as one element) makes the
        // s-integrand converge slowly far away: its far-field rule is the
        // up_ns(0)-point Gauss rule in s (closed_fb = 2), or its own nodes
        // with the upsampled rule as a correction wherever the estimates ask
        // for it (closed_fb = 1)
        const double* cp0 = circ + (int64_t)e * NCIRC * CIRQ;
        const double eend = fmin(fabs(cp0[6]), fabs(cp0[(NCIRC - 1) * CIRQ + 6]));
        inf.closed = eend < 1e-3 * outv[1];
        inf.fb = inf.closed ? closed_fb : 1;
        inf.group = egroup[e];
        inf.shape = SHAPE_OTHER;   // set by the host's shape test
        info[e] = inf;
    }
}

// Upsampled whole-panel tensor rule of tier k (or a far-field rule): ns_f
// Gauss-Legendre nodes on the whole panel in s (gx_f, gw_f on [-1,1]) times
// nt_f uniform angles.  Block = one s-row (nt_f threads), grid = (E, ns_f);
// element e's points start at e * ns_f * nt_f, or at eoff[e] (-1: none).
__global__ __launch_bounds__(128) void k_expand_up(int E, int ns_f, int nt_f, const double* __restrict__ gx_f,
                                                   const double* __restrict__ gw_f, const double* __restrict__ clq,
                                                   const ElemInfo* __restrict__ info, double* __restrict__ cpy,
                                                   double* __restrict__ cpn, double* __restrict__ cpw,
                                                   int64_t Mtot, const int64_t* __restrict__ eoff)
{
    const int e = blockIdx.x, p = blockIdx.y, q = threadIdx.x;
    const int64_t Mf = (int64_t)ns_f * nt_f;
    const int64_t m0 = eoff ? eoff[e] : (int64_t)e * Mf;
    if (m0 < 0) return;
    const ElemInfo inf = info[e];
    Frame fr;
    frame_at_x(clq + (int64_t)e * CLQ * NS, gx_f[p], fr);
    double th = 2.0 * PI * q / nt_f;
    double st, ct;
    sincos(th, &st, &ct);
    double y[3], ys[3], yt[3], jn[3];
    surface_at(fr, ct, st, y, ys, yt);
    cross3(yt, ys, jn);
    double J = sqrt(dot3(jn, jn));
    const int64_t m = m0 + (int64_t)p * nt_f + q;
    for (int d = 0; d < 3; ++d) {
        cpy[d * Mtot + m] = y[d];
        cpn[d * Mtot + m] = inf.sign * jn[d] / J;
    }
    cpw[m] = J * gw_f[p] * (0.5 * (inf.c - inf.a)) * (2.0 * PI / nt_f);
}

// Far-field (base) source set: each element contributes its own nodes (fb = 1)
// or its tier-0 rule (fb = 2); boff[e] is the element's first base source.
__global__ void k_base_build(int E, const ElemInfo* __restrict__ info, const int64_t* __restrict__ boff,
                             const double* __restrict__ ny, const double* __restrict__ nn,
                             const double* __restrict__ nw, int64_t N, const double* __restrict__ c0y,
                             const double* __restrict__ c0n, const double* __restrict__ c0w, int64_t M0,
                             double* __restrict__ by, double* __restrict__ bn, double* __restrict__ bw, int64_t Nb)
{
    const int e = blockIdx.x;
    const int fb = info[e].fb;
    const int64_t o = boff[e];
    const int cnt = fb == 2 ? (int)up_pts(0) : NPE;
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        int64_t src = fb == 2 ? (int64_t)e * up_pts(0) + k : (int64_t)e * NPE + k;
        const double* sy = fb == 2 ? c0y : ny;
        const double* sn = fb == 2 ? c0n : nn;
        const double* swt = fb == 2 ? c0w : nw;
        const int64_t ld = fb == 2 ? M0 : N;
        for (int d = 0; d < 3; ++d) {
            by[d * Nb + o + k] = sy[d * ld + src];
            bn[d * Nb + o + k] = sn[d * ld + src];
        }
        bw[o + k] = swt[src];
    }
}

// ---------------------------------------------------------------------------
// density preparation
// ---------------------------------------------------------------------------
// sigma*w (SoA), Fourier coefficients on each GL circle sh[e][i][l][6], and the
// band limits (highest Legendre degree Ms and Fourier mode Mt above eta times
// the element's largest coefficient; eta < 0: the full band).
__global__ __launch_bounds__(512) void k_prep_sigma(int E, const double* __restrict__ sigma,
                                                    const double* __restrict__ nw, int64_t N,
                                                    double* __restrict__ sw, double* __restrict__ sh,
                                                    int* __restrict__ band, double eta)
{
    const int e = blockIdx.x, tid = threadIdx.x;
    __shared__ double sg[3][NS][NT];
    __shared__ double shl[NS * NSH];
    __shared__ double amp[NS + NMODE];
    const int i = tid / NT, j = tid % NT;
    const int64_t n = (int64_t)e * NPE + tid;
    double w = nw[n];
    for (int d = 0; d < 3; ++d) {
        double s = sigma[n * 3 + d];
        sg[d][i][j] = s;
        sw[d * N + n] = s * w;
    }
    if (tid < NS + NMODE) amp[tid] = 0.0;
    __syncthreads();
    for (int o = tid; o < NS * NSH; o += blockDim.x) {
        int row = o / NSH, k = o % NSH;
        int l = k / 6, r = k % 6;
        int comp = r % 3;
        bool isb = r >= 3;
        double acc = 0.0;
        if (!(isb && (l == 0 || l == NT / 2))) {
            for (int jj = 0; jj < NT; ++jj) {
                int ph = (l * jj) % NT;
                acc += sg[comp][row][jj] * (isb ? c_sin[ph] : c_cos[ph]);
            }
        }
        double fac = (l == 0 || l == NT / 2) ? 1.0 / NT : 2.0 / NT;
        double v = acc * fac;
        shl[o] = v;
        sh[(int64_t)e * NS * NSH + o] = v;
    }
    __syncthreads();
    // Fourier band: amplitude of each mode over rows and components
    if (tid < NMODE) {
        double m = 0.0;
        for (int row = 0; row < NS; ++row)
            for (int r = 0; r < 6; ++r) m = fmax(m, fabs(shl[row * NSH + tid * 6 + r]));
        amp[NS + tid] = m;
    }
    // Legendre band along s: coefficient k of every angle and component
    if (tid < NS) {
        double m = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int jj = 0; jj < NT; ++jj) {
                double v = 0.0;
                for (int ii = 0; ii < NS; ++ii) v += c_T[tid * NS + ii] * sg[d][ii][jj];
                m = fmax(m, fabs(v));
            }
        amp[tid] = m;
    }
    __syncthreads();
    if (tid == 0) {
        double ms = 0.0, mt = 0.0;
        for (int k = 0; k < NS; ++k) ms = fmax(ms, amp[k]);
        for (int l = 0; l < NMODE; ++l) mt = fmax(mt, amp[NS + l]);
        int Ms = 0, Mt = 0;
        for (int k = 0; k < NS; ++k)
            if (amp[k] > eta * ms) Ms = k;
        for (int l = 0; l < NMODE; ++l)
            if (amp[NS + l] > eta * mt) Mt = l;
        if (eta < 0.0) {   // the widest band any density can have
            Ms = NS - 1;
            Mt = NMODE - 1;
        }
        band[2 * e] = Ms;
        band[2 * e + 1] = Mt;
    }
}

// density times weight on the upsampled whole-panel rule (ns_f x nt_f):
// sigma(s_p, t_q) from the GL-circle Fourier coefficients interpolated to s_p
// (Lup: ns_f x NS Lagrange matrix) and synthesised at t_q.
__global__ __launch_bounds__(256) void k_sigma_up(int E, int ns_f, int nt_f, const double* __restrict__ sh,
                                                  const double* __restrict__ Lup, const double* __restrict__ cpw,
                                                  double* __restrict__ swf, int64_t Mtot,
                                                  const int64_t* __restrict__ eoff)
{
    const int e = blockIdx.x, tid = threadIdx.x;
    const int64_t Mf = (int64_t)ns_f * nt_f;
    const int64_t m0 = eoff ? eoff[e] : (int64_t)e * Mf;
    if (m0 < 0) return;
    __shared__ double shl[NS * NSH];
    __shared__ double A[NS * NSH];
    for (int o = tid; o < NS * NSH; o += blockDim.x) shl[o] = sh[(int64_t)e * NS * NSH + o];
    __syncthreads();
    for (int rb = 0; rb < ns_f; rb += NS) {
        // coefficients at s-points rb .. min(rb + 16, ns_f) - 1
        const int nr = min(NS, ns_f - rb);
        for (int o = tid; o < nr * NSH; o += blockDim.x) {
            int r = o / NSH, k = o % NSH;
            int pp = rb + r;
            double v = 0.0;
            for (int ii = 0; ii < NS; ++ii) v += Lup[pp * NS + ii] * shl[ii * NSH + k];
            A[o] = v;
        }
        __syncthreads();
        for (int o = tid; o < nr * nt_f; o += blockDim.x) {
            int r = o / nt_f, q = o % nt_f;
            double th = 2.0 * PI * q / nt_f;
            double s1, c1;
            sincos(th, &s1, &c1);
            const double* ar = A + r * NSH;
            double v0 = ar[0], v1 = ar[1], v2 = ar[2];
            double cl = 1.0, sl = 0.0;
            for (int l = 1; l < NMODE; ++l) {
                double cn = cl * c1 - sl * s1;
                sl = sl * c1 + cl * s1;
                cl = cn;
                v0 += ar[l * 6 + 0] * cl + ar[l * 6 + 3] * sl;
                v1 += ar[l * 6 + 1] * cl + ar[l * 6 + 4] * sl;
                v2 += ar[l * 6 + 2] * cl + ar[l * 6 + 5] * sl;
            }
            int64_t m = m0 + (int64_t)(rb + r) * nt_f + q;
            double w = cpw[m];
            swf[0 * Mtot + m] = v0 * w;
            swf[1 * Mtot + m] = v1 * w;
            swf[2 * Mtot + m] = v2 * w;
        }
        __syncthreads();
    }
}

// density times weight on the base (far-field) source set
__global__ void k_sigma_base(int E, const ElemInfo* __restrict__ info, const int64_t* __restrict__ boff,
                             const double* __restrict__ sw, int64_t N, const double* __restrict__ swf0, int64_t M0,
                             double* __restrict__ bsw, int64_t Nb)
{
    const int e = blockIdx.x;
    const int fb = info[e].fb;
    const int64_t o = boff[e];
    const int cnt = fb == 2 ? (int)up_pts(0) : NPE;
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        for (int d = 0; d < 3; ++d)
            bsw[d * Nb + o + k] = fb == 2 ? swf0[d * M0 + (int64_t)e * up_pts(0) + k] : sw[d * N + (int64_t)e * NPE + k];
    }
}

// ---------------------------------------------------------------------------
// targets
// ---------------------------------------------------------------------------
// Target coordinates (node position for an on-surface target) and group: the
// node's element group, else the caller's group (0 without a list).
__global__ void k_targets(int64_t T, const double* __restrict__ x, const int64_t* __restrict__ tnode,
                          const int* __restrict__ tgrp_in, int G, const ElemInfo* __restrict__ info,
                          const double* __restrict__ ny, int64_t N, double* __restrict__ xt,
                          int* __restrict__ tgroup, int* __restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    int64_t nd = tnode ? tnode[t] : -1;
    if (nd >= N) {
        atomicOr(err, FLAG_NODE_RANGE);
        nd = -1;
    }
    for (int d = 0; d < 3; ++d) {
        double v = (nd >= 0) ? ny[d * N + nd] : (x ? x[t * 3 + d] : 0.0);
        xt[d * T + t] = v;
    }
    int g = (nd >= 0) ? info[nd / NPE].group : (tgrp_in ? tgrp_in[t] : 0);
    if (g < 0 || g >= G) {
        atomicOr(err, FLAG_GROUP_RANGE);
        g = 0;
    }
    tgroup[t] = g;
}

// first target of every group (gstart preset to -1); flags targets that are
// not ordered by group
__global__ void k_group_bounds(int64_t T, const int* __restrict__ tgroup, int64_t* __restrict__ gstart,
                               int* __restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int g = tgroup[t];
    if (t == 0 || tgroup[t - 1] != g) gstart[g] = t;
    if (t > 0 && tgroup[t - 1] > g) atomicOr(err, FLAG_GROUP_ORDER);
}

__global__ void k_fill_i64(int64_t n, int64_t* __restrict__ v, int64_t val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

// ---------------------------------------------------------------------------
// smooth Nystrom sum (Section 3.2.1): targets x sources
// ---------------------------------------------------------------------------
constexpr int FAR_REC = 10;     // LDS record of a source (upsampled corrections): y(3) n(3) sigma*w(3), padded

// bounding box of the block's points (lo/hi per coordinate; +-inf if none)
__device__ inline void block_box(double* lo, double* hi, double* red /*[2][3][FAR_BLOCK / 64]*/)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        double a = lo[d], b = hi[d];
        for (int o = 32; o > 0; o >>= 1) {
            a = fmin(a, __shfl_xor(a, o, 64));
            b = fmax(b, __shfl_xor(b, o, 64));
        }
        if (lane == 0) {
            red[d * (FAR_BLOCK / 64) + wv] = a;
            red[(3 + d) * (FAR_BLOCK / 64) + wv] = b;
        }
    }
    __syncthreads();
    for (int d = 0; d < 3; ++d) {
        double a = red[d * (FAR_BLOCK / 64)], b = red[(3 + d) * (FAR_BLOCK / 64)];
        for (int k = 1; k < FAR_BLOCK / 64; ++k) {
            a = fmin(a, red[d * (FAR_BLOCK / 64) + k]);
            b = fmax(b, red[(3 + d) * (FAR_BLOCK / 64) + k]);
        }
        lo[d] = a;
        hi[d] = b;
    }
    __syncthreads();
}

// Source ranges [seg[2 q], seg[2 q + 1]) of segments q0 .. q0 + nq - 1
// (nq <= 64) of a block, written to LDS by the first nq threads: for an
// element chunk, element tl.e0 + q's coarsest far-field rule whose radii
// from the element's centre (for its points in s and its angles) the block's
// target box [lo, hi] keeps clear of, else its base rule; for a plain chunk,
// its source range.
__device__ __forceinline__ void far_segments(const FarTile& tl, const FarSplit& spl, int q0, int nq, const double* lo,
                                             const double* hi, int64_t* seg)
{
    const int l = threadIdx.x;
    if (l >= nq) return;
    int64_t a = tl.s0, b = tl.s0 + tl.sn;
    if (tl.e1 > tl.e0) {
        const int e = tl.e0 + q0 + l;
        a = spl.boff[e];
        b = spl.boff[e + 1];
        if (spl.rc) {
            const ElemInfo& inf = spl.info[e];
            double g2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double g = fmax(0.0, fmax(lo[d] - inf.cen[d], inf.cen[d] - hi[d]));
                g2 += g * g;
            }
            // the radii grow as the rules coarsen (+inf outside the element's
            // own range): the coarsest admissible number of points in s, then
            // of angles
            int i = -1, j = 0;
            for (int ii = 0; ii < NFS; ++ii) {
                const double r = spl.rc[(int64_t)ii * spl.E + e];
                if (g2 >= r * r) i = ii;
            }
            for (int jj = 1; jj < NFT; ++jj) {
                const double r = spl.rc[(int64_t)(NFS + jj - 1) * spl.E + e];
                if (g2 >= r * r) j = jj;
            }
            if (i >= 0) {
                const int k = i * NFT + j;
                const int64_t o = spl.loff[(int64_t)k * spl.E + e];
                if (o >= 0) {   // else the element's base rule
                    a = o;
                    b = o + far_pts(k);
                }
            }
        }
    }
    seg[2 * l] = a;
    seg[2 * l + 1] = b;
}

// a value every lane holds alike, made provably uniform (scalar registers)
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// bounding box of a block's targets, stored in box[0..5] (lo, hi) in LDS
template <int TPT>
__device__ __forceinline__ void target_box(const double x[TPT][3], int64_t tb, int64_t tend, double* box,
                                           double* red)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
#pragma unroll
    for (int u = 0; u < TPT; ++u)
        if (tb + u * FAR_BLOCK < tend)
            for (int d = 0; d < 3; ++d) {
                lo[d] = fmin(lo[d], x[u][d]);
                hi[d] = fmax(hi[d], x[u][d]);
            }
    block_box(lo, hi, red);
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            box[d] = lo[d];
            box[3 + d] = hi[d];
        }
    __syncthreads();
}

// Each thread owns TPT targets and walks its block's source chunk; a
// source's record is read at wave-uniform addresses (scalar loads through the
// scalar cache, shared by the block's four waves), so it costs no vector
// memory, LDS or barrier and every load serves 64 TPT pairs.
template <int TPT, int KER>
__device__ __forceinline__ void far_range(const double x[TPT][3], const double* __restrict__ sy,
                                          const double* __restrict__ sn, const double* __restrict__ ssw, int64_t N,
                                          int64_t c0, int64_t c1, double sa[TPT][3], double sb[TPT][3],
                                          double sd[TPT][3])
{
#pragma unroll 4
    for (int64_t k = c0; k < c1; ++k) {
        const double2 A = {sy[k], sy[N + k]}, B = {sy[2 * N + k], sn[k]}, C = {sn[N + k], sn[2 * N + k]},
                      D = {ssw[k], ssw[N + k]}, F = {ssw[2 * N + k], 0.0};
#pragma unroll
        for (int u = 0; u < TPT; ++u) pair_acc<KER>(x[u], A, B, C, D, F, sa[u], sb[u], sd[u]);
    }
}

template <int TPT, int KER>
__global__ __launch_bounds__(FAR_BLOCK) void k_far(int64_t T, const double* __restrict__ xt,
                                                   const double* __restrict__ sy, const double* __restrict__ sn,
                                                   const double* __restrict__ ssw, int64_t N,
                                                   const FarTile* __restrict__ tiles, double* __restrict__ part,
                                                   FarSplit spl)
{
    __shared__ double red[6 * (FAR_BLOCK / 64)];
    __shared__ double box[6];
    __shared__ int64_t seg[2 * 64];
    const int tid = threadIdx.x;
    const FarTile tl = tiles[blockIdx.x];
    const int64_t tb = tl.t0 + tid, tend = tl.t0 + tl.tn;
    double x[TPT][3], sa[TPT][3], sb[TPT][3], sd[TPT][3];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int64_t t = tb + u * FAR_BLOCK;
        const bool ok = t < tend;
        x[u][0] = ok ? xt[t] : 0.0;
        x[u][1] = ok ? xt[T + t] : 0.0;
        x[u][2] = ok ? xt[2 * T + t] : 0.0;
        for (int d = 0; d < 3; ++d) sa[u][d] = sb[u][d] = sd[u][d] = 0.0;
    }
    // a plain source range, or the far-field rules of whole elements, in
    // batches of up to 64 segments whose ranges are staged in LDS
    if (tl.e1 > tl.e0 && spl.rc) target_box<TPT>(x, tb, tend, box, red);
    const int nseg = tl.e1 > tl.e0 ? tl.e1 - tl.e0 : 1;
    int64_t npts = 0;
    for (int q0 = 0; q0 < nseg; q0 += 64) {
        const int nq = min(64, nseg - q0);
        far_segments(tl, spl, q0, nq, box, box + 3, seg);
        __syncthreads();
        for (int q = 0; q < nq; ++q) {
            const int64_t a = uniform64(seg[2 * q]), b = uniform64(seg[2 * q + 1]);
            far_range<TPT, KER>(x, sy, sn, ssw, N, a, b, sa, sb, sd);
            npts += b - a;
        }
        __syncthreads();
    }
    if (spl.pairs && tid == 0) spl.pairs[blockIdx.x] = npts * tl.tn;
    double* p = part + (int64_t)tl.chunk * 6 * T;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int64_t t = tb + u * FAR_BLOCK;
        if (t < tend) {
            double o[6];
            scaled_out<KER>(sa[u], sb[u], sd[u], o);
            for (int k = 0; k < 6; ++k)
                if (KER != KER_LAPLACE || k == 0 || k == 3) p[k * T + t] = o[k];
        }
    }
}

// Mixed-precision smooth sum.  r = x - y is formed in FP64 (so a pair keeps
// its relative accuracy whatever the coordinates' magnitude) and the kernel
// is evaluated in FP32, summed in FP32 over one tile of FAR_BLOCK sources and
// then into FP64 accumulators.  Sources closer than sqrt(near2) to a target
// are evaluated and summed in FP64 from the FP64 record: their terms are the
// large ones that the near corrections later cancel against an FP64
// subtraction of the same terms, so they must carry FP64 rounding only.
// Whole tiles whose bounding box is farther than that from the block's
// targets skip the per-pair test.
struct __attribute__((aligned(16))) FarRecMx {
    double y0, y1, y2;
    float n0, n1, n2, w0, w1, w2;    // FP32 copy for the far part
    double n[3], w[3];               // FP64 values for the near part
};

template <int TPT>
__global__ __launch_bounds__(FAR_BLOCK) void k_far_mx(int64_t T, const double* __restrict__ xt,
                                                      const double* __restrict__ sy, const double* __restrict__ sn,
                                                      const double* __restrict__ ssw, int64_t N,
                                                      const FarTile* __restrict__ tiles, double near2,
                                                      double* __restrict__ part, FarSplit spl)
{
    __shared__ FarRecMx src[FAR_BLOCK];
    __shared__ double red[6 * (FAR_BLOCK / 64)];
    __shared__ int64_t seg[2 * 64];
    const int tid = threadIdx.x;
    const FarTile tl = tiles[blockIdx.x];
    const int64_t tb = tl.t0 + tid, tend = tl.t0 + tl.tn;
    const float near2f = (float)near2;
    double x[TPT][3], us[TPT][3], ud[TPT][3];
    double tlo[3] = {INFINITY, INFINITY, INFINITY}, thi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int64_t t = tb + u * FAR_BLOCK;
        const bool ok = t < tend;
        x[u][0] = ok ? xt[t] : 0.0;
        x[u][1] = ok ? xt[T + t] : 0.0;
        x[u][2] = ok ? xt[2 * T + t] : 0.0;
        for (int d = 0; d < 3; ++d) {
            us[u][d] = ud[u][d] = 0.0;
            if (ok) {
                tlo[d] = fmin(tlo[d], x[u][d]);
                thi[d] = fmax(thi[d], x[u][d]);
            }
        }
    }
    block_box(tlo, thi, red);
    // one source range [c0, c1)
    auto sum_range = [&](int64_t c0, int64_t c1) {
        for (int64_t base = c0; base < c1; base += FAR_BLOCK) {
            const int64_t k = base + tid;
            double slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
            if (k < c1) {
                FarRecMx r;
                r.y0 = sy[k];
                r.y1 = sy[N + k];
                r.y2 = sy[2 * N + k];
                for (int d = 0; d < 3; ++d) {
                    r.n[d] = sn[d * N + k];
                    r.w[d] = ssw[d * N + k];
                }
                r.n0 = (float)r.n[0];
                r.n1 = (float)r.n[1];
                r.n2 = (float)r.n[2];
                r.w0 = (float)r.w[0];
                r.w1 = (float)r.w[1];
                r.w2 = (float)r.w[2];
                src[tid] = r;
                slo[0] = shi[0] = r.y0;
                slo[1] = shi[1] = r.y1;
                slo[2] = shi[2] = r.y2;
            }
            block_box(slo, shi, red);   // also the barrier after the tile is stored
            double gap2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double g = fmax(0.0, fmax(tlo[d] - shi[d], slo[d] - thi[d]));
                gap2 += g * g;
            }
            const bool near_tile = !(gap2 >= near2 && gap2 > 0.0);   // uniform over the block
            const int nin = (int)min((int64_t)FAR_BLOCK, c1 - base);
            float fs[TPT][3], fd[TPT][3];
#pragma unroll
            for (int u = 0; u < TPT; ++u)
                for (int d = 0; d < 3; ++d) fs[u][d] = fd[u][d] = 0.0f;
            if (!near_tile) {
#pragma unroll 2
                for (int kk = 0; kk < nin; ++kk) {
                    const FarRecMx& R = src[kk];
                    const double y0 = R.y0, y1 = R.y1, y2 = R.y2;
                    const float n0 = R.n0, n1 = R.n1, n2 = R.n2, w0 = R.w0, w1 = R.w1, w2 = R.w2;
#pragma unroll
                    for (int u = 0; u < TPT; ++u) {
                        const float r0 = (float)(x[u][0] - y0), r1 = (float)(x[u][1] - y1), r2 = (float)(x[u][2] - y2);
                        const float rr = fmaf(r0, r0, fmaf(r1, r1, r2 * r2));
                        const float ir = __builtin_amdgcn_rsqf(rr);   // rr > 0: the tile is away from every target
                        const float rs = fmaf(r0, w0, fmaf(r1, w1, r2 * w2));
                        const float rn = fmaf(r0, n0, fmaf(r1, n1, r2 * n2));
                        const float ir2 = ir * ir;
                        const float b = rs * (ir * ir2);
                        const float cD = (rn * b) * ir2;
                        fs[u][0] = fmaf(ir, w0, fmaf(b, r0, fs[u][0]));
                        fs[u][1] = fmaf(ir, w1, fmaf(b, r1, fs[u][1]));
                        fs[u][2] = fmaf(ir, w2, fmaf(b, r2, fs[u][2]));
                        fd[u][0] = fmaf(cD, r0, fd[u][0]);
                        fd[u][1] = fmaf(cD, r1, fd[u][1]);
                        fd[u][2] = fmaf(cD, r2, fd[u][2]);
                    }
                }
            } else {
                for (int kk = 0; kk < nin; ++kk) {
                    const FarRecMx& R = src[kk];
#pragma unroll
                    for (int u = 0; u < TPT; ++u) {
                        const double d0 = x[u][0] - R.y0, d1 = x[u][1] - R.y1, d2 = x[u][2] - R.y2;
                        const float r0 = (float)d0, r1 = (float)d1, r2 = (float)d2;
                        const float rr = fmaf(r0, r0, fmaf(r1, r1, r2 * r2));
                        if (rr < near2f) {
                            const double rr64 = fma(d0, d0, fma(d1, d1, d2 * d2));
                            const double irn = rsqrt_nr1(rr64);
                            const double ir = rr64 > 0.0 ? irn : 0.0;
                            const double rs = fma(d0, R.w[0], fma(d1, R.w[1], d2 * R.w[2]));
                            const double rn = fma(d0, R.n[0], fma(d1, R.n[1], d2 * R.n[2]));
                            const double ir2 = ir * ir;
                            const double b = rs * (ir * ir2);
                            const double cD = (rn * b) * ir2;
                            us[u][0] = fma(ir, R.w[0], fma(b, d0, us[u][0]));
                            us[u][1] = fma(ir, R.w[1], fma(b, d1, us[u][1]));
                            us[u][2] = fma(ir, R.w[2], fma(b, d2, us[u][2]));
                            ud[u][0] = fma(cD, d0, ud[u][0]);
                            ud[u][1] = fma(cD, d1, ud[u][1]);
                            ud[u][2] = fma(cD, d2, ud[u][2]);
                        } else {
                            const float ir = __builtin_amdgcn_rsqf(rr);
                            const float rs = fmaf(r0, R.w0, fmaf(r1, R.w1, r2 * R.w2));
                            const float rn = fmaf(r0, R.n0, fmaf(r1, R.n1, r2 * R.n2));
                            const float ir2 = ir * ir;
                            const float b = rs * (ir * ir2);
                            const float cD = (rn * b) * ir2;
                            fs[u][0] = fmaf(ir, R.w0, fmaf(b, r0, fs[u][0]));
                            fs[u][1] = fmaf(ir, R.w1, fmaf(b, r1, fs[u][1]));
                            fs[u][2] = fmaf(ir, R.w2, fmaf(b, r2, fs[u][2]));
                            fd[u][0] = fmaf(cD, r0, fd[u][0]);
                            fd[u][1] = fmaf(cD, r1, fd[u][1]);
                            fd[u][2] = fmaf(cD, r2, fd[u][2]);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < TPT; ++u)
                for (int d = 0; d < 3; ++d) {
                    us[u][d] += (double)fs[u][d];
                    ud[u][d] += (double)fd[u][d];
                }
            __syncthreads();
        }
    };
    const int nseg = tl.e1 > tl.e0 ? tl.e1 - tl.e0 : 1;
    int64_t npts = 0;
    for (int q0 = 0; q0 < nseg; q0 += 64) {
        const int nq = min(64, nseg - q0);
        far_segments(tl, spl, q0, nq, tlo, thi, seg);
        __syncthreads();
        for (int q = 0; q < nq; ++q) {
            const int64_t a = uniform64(seg[2 * q]), b = uniform64(seg[2 * q + 1]);
            sum_range(a, b);
            npts += b - a;
        }
        __syncthreads();
    }
    if (spl.pairs && tid == 0) spl.pairs[blockIdx.x] = npts * tl.tn;
    double* p = part + (int64_t)tl.chunk * 6 * T;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int64_t t = tb + u * FAR_BLOCK;
        if (t < tend) {
            p[0 * T + t] = us[u][0];
            p[1 * T + t] = us[u][1];
            p[2 * T + t] = us[u][2];
            p[3 * T + t] = ud[u][0];
            p[4 * T + t] = ud[u][1];
            p[5 * T + t] = ud[u][2];
        }
    }
}

// ---------------------------------------------------------------------------
// near-pair search (candidates) and classification
// ---------------------------------------------------------------------------
__global__ void k_search(int64_t T, const int* __restrict__ tgroup, const int* __restrict__ gel,
                         const double* __restrict__ xt, const int64_t* __restrict__ tnode,
                         const ElemInfo* __restrict__ info, const double* __restrict__ rnear,
                         const int64_t* __restrict__ off, int* __restrict__ cnt, int* __restrict__ pe,
                         int* __restrict__ pt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double x[3] = {xt[t], xt[T + t], xt[2 * T + t]};
    int own = (tnode && tnode[t] >= 0) ? (int)(tnode[t] / NPE) : -1;
    int n = 0;
    int64_t o = off ? off[t] : 0;
    const int g = tgroup[t];
    for (int e = gel[g]; e < gel[g + 1]; ++e) {
        const ElemInfo& inf = info[e];
        double dx = x[0] - inf.cen[0], dy = x[1] - inf.cen[1], dz = x[2] - inf.cen[2];
        double R = inf.rad + rnear[e];
        bool cand = (dx * dx + dy * dy + dz * dz < R * R) || e == own;
        if (cand) {
            if (off) {
                pe[o + n] = e;
                pt[o + n] = (int)t;
            }
            ++n;
        }
    }
    if (!off) cnt[t] = n;
}

// worst Bernstein parameter of s* = sr + i si over f equal sub-panels of [a,c]
__device__ inline double rho_subpanels(double sr, double si, double a, double c, int f)
{
    double h = (c - a) / f;
    double best = 1e300;
    for (int k = 0; k < f; ++k) best = fmin(best, bernstein_rho(sr, si, a + k * h, a + (k + 1) * h));
    return best;
}

// --- complex arithmetic for the contact-point search
struct cx {
    double r, i;
};
__device__ __forceinline__ cx cadd(cx a, cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cx csub(cx a, cx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cx cmul(cx a, cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cx cdiv(cx a, cx b)
{
    double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// Circle-contact function at the complex (normalised) parameter z: the
// product d^2 d'^2 of the squared distances from the target to the circle at z
// and to its antipodal continuation, d^2 d'^2 = (|v|^2 + eps^2)^2 -
// 4 eps^2 (|v|^2 - (v.x_c')^2/|x_c'|^2), v = x - x_c(z) (bilinear products).
// The angular integral I(x, s) is analytic in s except where this vanishes,
// so its zero nearest to the panel sets the Gauss-Legendre convergence rate.
__device__ inline cx contact_fn(const double* __restrict__ clq, cx z, const double* x)
{
    // barycentric sums at the complex point in one pass (no stored weights)
    cx sum = {0.0, 0.0};
    cx X[3] = {{0, 0}, {0, 0}, {0, 0}}, Xp[3] = {{0, 0}, {0, 0}, {0, 0}}, E = {0, 0};
    // partly unrolled: a full unroll lets the compiler hoist all 112 element
    // values out of the root iteration into registers
#pragma unroll 2
    for (int i = 0; i < NS; ++i) {
        const double dr = z.r - c_gx[i], di = z.i;
        const double q = dr * dr + di * di;
        double rq = __builtin_amdgcn_rcp(q);
        rq = rq * fma(-q, rq, 2.0);  // one Newton step on the hardware reciprocal
        const double inv = c_lam[i] * rq;
        const cx li = {dr * inv, -di * inv};  // lam / (z - x_i)
        sum = cadd(sum, li);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double a = clq[(Q_X + d) * NS + i], b = clq[(Q_XP + d) * NS + i];
            X[d].r += li.r * a;
            X[d].i += li.i * a;
            Xp[d].r += li.r * b;
            Xp[d].i += li.i * b;
        }
        const double ee = clq[Q_E * NS + i];
        E.r += li.r * ee;
        E.i += li.i * ee;
    }
    const cx isum = cdiv({1.0, 0.0}, sum);
    for (int d = 0; d < 3; ++d) {
        X[d] = cmul(X[d], isum);
        Xp[d] = cmul(Xp[d], isum);
    }
    E = cmul(E, isum);
    cx vv = {0, 0}, xx = {0, 0}, vx = {0, 0};
    for (int d = 0; d < 3; ++d) {
        cx v = csub({x[d], 0.0}, X[d]);
        vv = cadd(vv, cmul(v, v));
        xx = cadd(xx, cmul(Xp[d], Xp[d]));
        vx = cadd(vx, cmul(v, Xp[d]));
    }
    cx EE = cmul(E, E);
    cx A = cadd(vv, EE);
    cx z2 = cdiv(cmul(vx, vx), xx);
    return csub(cmul(A, A), cmul({4.0 * EE.r, 4.0 * EE.i}, csub(vv, z2)));
}

// Bernstein parameter (relative to [-1,1]) of the zero of the contact
// function found by secant iterations started above the closest real point
// xr at the height h0 of the locally flat estimate; returns 1e300 and leaves
// (zr, zi) untouched if the iteration does not converge.  (A second start at
// h0 / 5 finds zeros that change no tier the method-generated labels need:
// on the 200-sphere pipe the criterion without it still has no pair below its
// label at 1e-13 of max |u|.)
__device__ inline double contact_root(const double* __restrict__ clq, const double* x, double xr, double h0,
                                      double* zr, double* zi)
{
    cx z0 = {xr, h0};
    cx z1 = {xr + 0.05 * h0, 1.1 * h0};
    cx f0 = contact_fn(clq, z0, x), f1 = contact_fn(clq, z1, x);
    bool ok = false;
    for (int it = 0; it < 30; ++it) {
        cx df = csub(f1, f0);
        if (df.r == 0.0 && df.i == 0.0) break;
        cx step = cdiv(cmul(f1, csub(z1, z0)), df);
        z0 = z1;
        f0 = f1;
        z1 = csub(z1, step);
        if (!(fabs(z1.r) < 8.0 && fabs(z1.i) < 8.0)) break;
        f1 = contact_fn(clq, z1, x);
        // a tight stop: a looser one (1e-7) also accepts iterates still
        // wandering far from any zero, and the estimate turns pessimistic
        if (sqrt(step.r * step.r + step.i * step.i) < 1e-9 * (1.0 + fabs(z1.r) + fabs(z1.i))) {
            ok = true;
            break;
        }
    }
    if (!ok || !(fabs(z1.i) > 1e-9)) return 1e300;
    *zr = z1.r;
    *zi = fabs(z1.i);
    return bernstein_rho(z1.r, fabs(z1.i), -1.0, 1.0);
}

// The contact zero for a sphere given as one element in its polar angle
// (x_c = c + a cos(pi t) A, eps = a sin(pi t), t the panel's normalised
// parameter; the host's shape test admits only such elements): the circle
// at u = pi t passes through x where D^2 + a^2 = 2 a D cos(u - phi), with
// D = |x - c| and phi the polar angle of x - c about A, so the zero is
// u = phi + i acosh(1 + (D - a)^2 / (2 a D)), at xn = 2 u / pi - 1 in the
// panel's normalised variable: what the secant search converges to, without
// its iterations.  The end circles give c and a A.  Returns the zero's
// Bernstein parameter, or 1e300 where the zero is on the real axis (as the
// search does).
__device__ inline double sphere_contact_root(const double* __restrict__ cc, const double* x, double* zr, double* zi)
{
    const double* p0 = cc;                        // xn = -1 (t = 0): c + a A
    const double* p1 = cc + (NCIRC - 1) * CIRQ;   // xn = +1 (t = 1): c - a A
    double r[3], A[3];
    for (int d = 0; d < 3; ++d) {
        A[d] = 0.5 * (p0[d] - p1[d]);
        r[d] = x[d] - 0.5 * (p0[d] + p1[d]);
    }
    const double a = sqrt(dot3(A, A)), D = sqrt(dot3(r, r));
    if (!(a > 0.0) || !(D > 0.0)) return 1e300;
    const double cphi = fmin(1.0, fmax(-1.0, dot3(r, A) / (a * D)));
    const double im = 2.0 / PI * acosh1p((D - a) * (D - a) / (2.0 * a * D));
    if (!(im > 1e-9)) return 1e300;
    *zr = 2.0 / PI * acos(cphi) - 1.0;
    *zi = im;
    return bernstein_rho(*zr, im, -1.0, 1.0);
}

__device__ __forceinline__ cx csqrt_(cx z)
{
    const double m = hypot(z.r, z.i);
    return {sqrt(0.5 * (m + z.r)), copysign(sqrt(0.5 * fmax(m - z.r, 0.0)), z.i)};
}

// principal arccosine: -i log(z + i sqrt(1 - z^2))
__device__ __forceinline__ cx cacos_(cx z)
{
    const cx s = csqrt_(csub({1.0, 0.0}, cmul(z, z)));
    const cx t = {z.r - s.i, z.i + s.r};
    return {atan2(t.i, t.r), -log(hypot(t.r, t.i))};
}

// The contact zero for a torus-arc element (centerline C + R (cos psi U +
// sin psi V), psi = psi0 + psi1 xn, constant radius r; certified by the
// host): with the target at azimuth psi_x, distance P from the axis through
// C along U x V and height Z, the contact function is a quadratic in
// w = P cos(psi - psi_x):
//   4 (R^2 - r^2) w^2 - 4 R (A - 2 r^2) w + A^2 - 4 r^2 (R^2 + Z^2),
//   A = P^2 + R^2 + Z^2 + r^2,
// so its zeros are psi = psi_x +- arccos(w / P) for its two roots w.  Of
// these, the one with the smallest Bernstein parameter in xn; 1e300 where
// none is off the real axis (as the search does).
__device__ inline double torus_contact_root(const double* __restrict__ tp, const double* x, double* zr, double* zi)
{
    const double R = tp[9], r = tp[10], psi0 = tp[11], psi1 = tp[12];
    double dv[3], nz[3];
    for (int d = 0; d < 3; ++d) dv[d] = x[d] - tp[d];
    cross3(tp + 3, tp + 6, nz);
    const double X = dot3(dv, tp + 3), Y = dot3(dv, tp + 6), Z = dot3(dv, nz);
    const double P2 = X * X + Y * Y, P = sqrt(P2);
    if (!(P > 1e-12 * R)) return 1e300;
    const double psx = atan2(Y, X);
    const double A = P2 + R * R + Z * Z + r * r;
    const double a2 = 4.0 * (R * R - r * r), a1 = -4.0 * R * (A - 2.0 * r * r);
    const double a0 = A * A - 4.0 * r * r * (R * R + Z * Z);
    const cx sq = csqrt_({a1 * a1 - 4.0 * a2 * a0, 0.0});
    double best = 1e300;
    for (int k = 0; k < 2; ++k) {
        const cx w = {(-a1 + (k ? -sq.r : sq.r)) / (2.0 * a2), (k ? -sq.i : sq.i) / (2.0 * a2)};
        const cx al = cacos_({w.r / P, w.i / P});
        for (int sg = -1; sg <= 1; sg += 2) {
            const double xr = (psx + sg * al.r - psi0) / psi1, xi = fabs(sg * al.i / psi1);
            if (!(xi > 1e-9)) continue;
            const double rho = bernstein_rho(xr, xi, -1.0, 1.0);
            if (rho < best) {
                best = rho;
                *zr = xr;
                *zi = xi;
            }
        }
    }
    return best;
}

// Closest circle and fastest trapezoid decay for a sphere element (as in
// sphere_contact_root: circles at u = pi t about the axis A through c, radius
// a sin u).  The target's distance from the axis, rho, is the same for every
// circle, so d^2(u) = (rho - a sin u)^2 + (z - a cos u)^2 (z its height along
// A) is least at the target's polar angle, (D - a)^2, and
// cosh a - 1 = d^2(u) / (2 rho a sin u) is least where cos u = 2 a z / (D^2 + a^2).
__device__ inline void sphere_minima(const double* __restrict__ cc, const double* x, double* d2c, double* xd,
                                     double* chac)
{
    const double* p0 = cc;                        // xn = -1: c + a A
    const double* p1 = cc + (NCIRC - 1) * CIRQ;   // xn = +1: c - a A
    double r[3], A[3];
    for (int d = 0; d < 3; ++d) {
        A[d] = 0.5 * (p0[d] - p1[d]);
        r[d] = x[d] - 0.5 * (p0[d] + p1[d]);
    }
    const double a = sqrt(dot3(A, A)), D2 = dot3(r, r), D = sqrt(D2);
    if (!(a > 0.0) || !(D > 0.0)) return;   // keep the sampled minima
    const double z = dot3(r, A) / a, rho = sqrt(fmax(0.0, D2 - z * z));
    *d2c = (D - a) * (D - a);
    *xd = 2.0 / PI * acos(fmin(1.0, fmax(-1.0, z / D))) - 1.0;
    const double cu = 2.0 * a * z / (D2 + a * a), su = sqrt(fmax(0.0, 1.0 - cu * cu));
    const double dr = rho - a * su, dz = z - a * cu;
    *chac = (rho > 0.0 && su > 0.0) ? (dr * dr + dz * dz) / (2.0 * rho * a * su) : 1e300;
}

// Closest circle and fastest trapezoid decay for a torus-arc element (as in
// torus_contact_root).  For the circle at psi = psi_x + delta, with
// c = cos delta and q = |(P c - R, Z)| the target's distance from its centre
// within its plane, d^2 = P^2 sin^2 delta + (q - r)^2 and cosh a - 1 =
// d^2 / (2 q r) = (P^2 + R^2 + Z^2 + r^2 - 2 P R c) / (2 q r) - 1, whose only
// critical point in c is P c - R = -2 R Z^2 / (P^2 - R^2 + Z^2 + r^2), while
// d^2 is least at delta = 0.  The minima over the panel's angles are among
// those points and the panel ends.
__device__ inline void torus_minima(const double* __restrict__ tp, const double* x, double* d2c, double* xd,
                                    double* chac)
{
    const double R = tp[9], r = tp[10], psi0 = tp[11], psi1 = tp[12];
    double dv[3], nz[3];
    for (int d = 0; d < 3; ++d) dv[d] = x[d] - tp[d];
    cross3(tp + 3, tp + 6, nz);
    const double X = dot3(dv, tp + 3), Y = dot3(dv, tp + 6), Z = dot3(dv, nz);
    const double P = sqrt(X * X + Y * Y);
    if (!(P > 1e-12 * R)) return;   // keep the sampled minima
    const double psx = atan2(Y, X);
    // the panel's angles relative to the target's, centred in (-pi, pi]
    const double pm = psi0, hw = fabs(psi1);
    const double dm = remainder(pm - psx, 2.0 * PI), da = dm - hw, db = dm + hw;
    double cand[5];
    int nc = 0;
    cand[nc++] = da;
    cand[nc++] = db;
    if (da < 0.0 && db > 0.0) cand[nc++] = 0.0;
    const double den = P * P - R * R + Z * Z + r * r;
    if (den != 0.0) {
        const double cs = (R - 2.0 * R * Z * Z / den) / P;
        if (cs >= -1.0 && cs <= 1.0) {
            const double al = acos(cs);
            if (al >= da && al <= db) cand[nc++] = al;
            if (-al >= da && -al <= db) cand[nc++] = -al;
        }
    }
    double bd = 1e300, ba = 1e300, bdel = 0.0;
    for (int k = 0; k < nc; ++k) {
        double sn, c;
        sincos(cand[k], &sn, &c);
        const double q = hypot(P * c - R, Z), dq = q - r;
        const double d2 = P * P * sn * sn + dq * dq;
        const double cha = q > 0.0 ? d2 / (2.0 * q * r) : 1e300;
        if (d2 < bd) {
            bd = d2;
            bdel = cand[k];
        }
        ba = fmin(ba, cha);
    }
    *d2c = bd;
    *chac = ba;
    *xd = fmin(1.0, fmax(-1.0, (bdel - dm) / psi1));
}

// normalised parameter of sampled circle k: the panel ends and the GL nodes
__device__ __forceinline__ double circle_xn(int k)
{
    return k == 0 ? -1.0 : (k == NCIRC - 1 ? 1.0 : c_gx[k - 1]);
}

// the bracket around sampled circle kc (the GL gaps on both sides) and its
// grid step
__device__ __forceinline__ void circle_bracket(int kc, double* lo, double* hi, double* h)
{
    *lo = circle_xn(max(kc - 1, 0));
    *hi = circle_xn(min(kc + 1, NCIRC - 1));
    *h = (*hi - *lo) / (CGRID - 1);
}

// The bracket grids do not depend on the target: their circles are built
// once per element, one thread per (bracket, grid point).
__global__ __launch_bounds__(NCIRC * CGRID) void k_grid_circles(int E, const double* __restrict__ clq,
                                                                 double* __restrict__ grid)
{
    const int e = blockIdx.x, k = threadIdx.x / CGRID, i = threadIdx.x % CGRID;
    double lo, hi, h;
    circle_bracket(k, &lo, &hi, &h);
    double X[3], tt[3], EE;
    circle_at_x(clq + (int64_t)e * CLQ * NS, lo + i * h, X, tt, &EE);
    double* g = grid + (((int64_t)e * NCIRC + k) * CGRID + i) * GRQ;
    for (int d = 0; d < 3; ++d) {
        g[d] = X[d];
        g[3 + d] = tt[d];
    }
    g[6] = EE;
    g[7] = 0.0;
}

// Pairs are visited in element-major order (perm), so the lanes of a
// wavefront read the same element's data.
__global__ __launch_bounds__(128) void k_classify(int64_t P, const int* __restrict__ perm, const int* __restrict__ pe,
                           const int* __restrict__ pt, const double* __restrict__ xt, int64_t T,
                           const int64_t* __restrict__ tnode, const double* __restrict__ clq,
                           const double* __restrict__ circ, const double* __restrict__ grid,
                           const ElemInfo* __restrict__ info, const double* __restrict__ tor,
                           const int* __restrict__ band, GateConsts gc, int8_t* __restrict__ tier,
                           double* __restrict__ cls)
{
    const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= P) return;
    const int64_t p = perm[ii];
    const int e = pe[p];
    const int64_t t = pt[p];
    const ElemInfo inf = info[e];
    double x[3] = {xt[t], xt[T + t], xt[2 * T + t]};
    const int64_t nd = tnode ? tnode[t] : -1;
    double* cp = cls + p * 4;
    if (nd >= 0 && nd / NPE == e) {
        int i0 = (int)((nd % NPE) / NT);
        cp[0] = 0.5 * (inf.a + inf.c) + 0.5 * (inf.c - inf.a) * c_gx[i0];
        cp[1] = 0.0;
        cp[2] = circ[((int64_t)e * NCIRC + 1 + i0) * CIRQ + 7];
        cp[3] = 0.0;
        tier[p] = TIER_FULL;
        return;
    }
    const double* cc = circ + (int64_t)e * NCIRC * CIRQ;
    const double* cq = clq + (int64_t)e * CLQ * NS;
    double bd = 1e300, ba = 1e300;
    int kd = 0, ka = 0;
    for (int k = 0; k < NCIRC; ++k) {
        double d2, cha;
        circle_dist(cc + k * CIRQ, cc + k * CIRQ + 3, cc[k * CIRQ + 6], x, &d2, &cha);
        if (d2 < bd) { bd = d2; kd = k; }
        if (cha < ba) { ba = cha; ka = k; }
    }
    // closest circle (minimum of d^2 over the two GL gaps around the sampled
    // minimum) and fastest trapezoid decay (minimum of cosh a - 1, likewise):
    // for each, a 9-point grid over its bracket, then two parabolic steps; on
    // a sphere element both minima in closed form
    double d2c = bd, chac = ba, xd = circle_xn(kd);
    const double* tp = tor + (int64_t)e * TOR_Q;
    if (inf.shape == SHAPE_SPHERE) {
        sphere_minima(cc, x, &d2c, &xd, &chac);
    } else if (tp[TOR_Q - 1] != 0.0) {
        torus_minima(tp, x, &d2c, &xd, &chac);
    } else {
        auto eval = [&](double xn, double* d2, double* cha) {
            double X[3], tt[3], EE;
            circle_at_x(cq, xn, X, tt, &EE);
            circle_dist(X, tt, EE, x, d2, cha);
        };
        // vertex of the parabola through (x - dx, fl), (x, fc), (x + dx, fr)
        auto vertex = [](double xc, double dx, double fl, double fc, double fr) {
            const double den = fl - 2.0 * fc + fr;
            if (!(den > 0.0) || fl >= 1e299 || fr >= 1e299) return xc;
            return xc + 0.5 * dx * (fl - fr) / den;
        };
        for (int which = 0; which < 2; ++which) {
            const int kc = which ? ka : kd;
            double lo, hi, h;
            circle_bracket(kc, &lo, &hi, &h);
            const double* gk = grid + ((int64_t)e * NCIRC + kc) * CGRID * GRQ;
            // running minimum of the grid with its neighbours (no indexed arrays)
            double m = 1e300, ml = 1e300, mr = 1e300, pv = 1e300, xm = lo;
            int im = -1;
            for (int i = 0; i < CGRID; ++i) {
                double vd, va;
                const double xi = lo + i * h;
                const double* gi = gk + i * GRQ;
                circle_dist(gi, gi + 3, gi[6], x, &vd, &va);
                const double v = which ? va : vd;
                if (im == i - 1) mr = v;
                if (v < m) {
                    m = v;
                    ml = pv;
                    mr = 1e300;
                    im = i;
                    xm = xi;
                }
                pv = v;
            }
            const double xv = fmin(hi, fmax(lo, vertex(xm, h, ml, m, mr)));
            const double dx = 0.125 * h;
            double g[3];
            for (int k = 0; k < 3; ++k) {
                double vd, va;
                const double xk = fmin(hi, fmax(lo, xv + (k - 1) * dx));
                eval(xk, &vd, &va);
                g[k] = which ? va : vd;
                if (g[k] < m) {
                    m = g[k];
                    xm = xk;
                }
            }
            {
                double vd, va;
                const double xk = fmin(hi, fmax(lo, vertex(xv, dx, g[0], g[1], g[2])));
                eval(xk, &vd, &va);
                const double v = which ? va : vd;
                if (v < m) {
                    m = v;
                    xm = xk;
                }
            }
            if (which) {
                chac = fmin(chac, m);
            } else if (m < d2c) {
                d2c = m;
                xd = xm;
            }
        }
    }
    // speed bound near the closest circle
    double spd = fmax(cc[kd * CIRQ + 7], cc[min(kd + 1, NCIRC - 1) * CIRQ + 7]);
    spd = fmax(spd, cc[max(kd - 1, 0) * CIRQ + 7]);
    const double dc = sqrt(d2c);
    const double ac = acosh1p(chac);
    // singularity of the s-integrand: locally flat estimate s_c + i d/speed, or
    // the nearest zero of the contact function if that is closer
    const double half = 0.5 * (inf.c - inf.a), mid = 0.5 * (inf.a + inf.c);
    double zr = xd, zi = dc / spd / half;
    const double rho_lin = bernstein_rho(zr, zi, -1.0, 1.0);
    double rr = xd, ri = zi;
    double rho_root = inf.shape == SHAPE_SPHERE ? sphere_contact_root(cc, x, &rr, &ri)
                      : tp[TOR_Q - 1] != 0.0    ? torus_contact_root(tp, x, &rr, &ri)
                                                : contact_root(cq, x, xd, fmax(zi, 1e-6), &rr, &ri);
    if (rho_root < rho_lin) {
        zr = rr;
        zi = ri;
    }
    const double sr = mid + half * zr, si = half * zi;
    cp[0] = sr;
    cp[1] = si;
    cp[2] = 1.0;
    cp[3] = ac;
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    // Gauss-Legendre error on the whole panel ~ rho^-(2n - Ms) for a density of
    // degree Ms; trapezoid error ~ exp(-(nt - Mt - extra) a)
    const double rho = bernstein_rho(sr, si, inf.a, inf.c);
    const double lrho = log(rho);
    const double lt = log(gc.tol);
    int8_t tr = TIER_FULL;
    for (int k = -1; k < NUP; ++k) {
        const int nsr = k < 0 ? NS * inf.fb : up_ns(k);
        const int ntr = k < 0 ? NT : up_nt(k);
        if (k >= 0 && nsr <= NS * inf.fb && ntr <= NT) continue;   // no finer than the base rule
        const double les = log(gc.cs) - (double)(2 * nsr - Ms) * lrho;
        const double let = log(gc.ct) - (double)(ntr - Mt - gc.extra_modes) * ac;
        if (les <= lt && let <= lt) {
            tr = (int8_t)(k + 1);
            break;
        }
    }
    tier[p] = tr;
}

// candidate radius of each element (the distance beyond which the plain rule
// meets the tolerance by the same estimates)
__global__ void k_rnear(int E, const ElemInfo* __restrict__ info, const double* __restrict__ circ,
                        const int* __restrict__ band, GateConsts gc, double* __restrict__ rnear)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const ElemInfo inf = info[e];
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    double areq = log(gc.ct / gc.tol) / (double)(NT - Mt - gc.extra_modes);
    double dth = inf.eps_max * (exp(areq) - 1.0);
    double rreq = pow(gc.cs / gc.tol, 1.0 / (double)(2 * NS * inf.fb - Ms));
    double h = 0.5 * (inf.c - inf.a);
    double ds = inf.smax * h * 0.5 * (rreq - 1.0 / rreq);
    // an element whose cross-section closes at an end (a sphere in polar
    // angle): the contact zero leaves the real axis only logarithmically with
    // distance, cosh(pi Im s / (c - a)) ~ distance / (2 radius)
    const double* cc = circ + (int64_t)e * NCIRC * CIRQ;
    double e0 = fabs(cc[6]), e1 = fabs(cc[(NCIRC - 1) * CIRQ + 6]);
    if (fmin(e0, e1) < 1e-3 * inf.eps_max) {
        double imphi = 3.14159265358979323846 * 0.25 * (rreq - 1.0 / rreq);
        ds = fmax(ds, 2.0 * inf.rad * cosh(fmin(imphi, 40.0)));
    }
    rnear[e] = 1.05 * fmax(dth, ds) + 1e-12;
    // the distances from the centre beyond which the smooth sum may take
    // far_ns(i) Gauss points in s, and far_nt(j) angles, for the element, by
    // the same estimates; at least the candidate radius.  An element whose
    // base rule is the 32-point rule (closed at an end) takes i in [0, 3),
    // any other i in [2, 5) (its base is its own 16 points, the candidate
    // radius).
    const bool base32 = inf.fb == 2;
    const int i0 = far_i0(base32);
    for (int i = 0; i < NFS; ++i) {
        double rc = INFINITY;
        const int ex = 2 * far_ns(i) - Ms;
        if (i >= i0 && i < i0 + FAR_NI && ex > 0) {
            if (!base32 && i == i0) {
                rc = inf.rad + rnear[e];
            } else {
                const double rq = pow(gc.cs / gc.tol, 1.0 / (double)ex);
                double dsi = inf.smax * h * 0.5 * (rq - 1.0 / rq);
                if (inf.closed)
                    dsi = fmax(dsi, 2.0 * inf.rad * cosh(fmin(3.14159265358979323846 * 0.25 * (rq - 1.0 / rq), 40.0)));
                rc = inf.rad + fmax(1.05 * dsi + 1e-12, rnear[e]);
            }
        }
        rnear[(int64_t)(1 + i) * E + e] = rc;
    }
    for (int j = 1; j < NFT; ++j) {
        double rc = INFINITY;
        const int ex = far_nt(j) - Mt - gc.extra_modes;
        if (ex > 0) {
            const double dtj = inf.eps_max * (exp(log(gc.ct / gc.tol) / (double)ex) - 1.0);
            rc = inf.rad + fmax(1.05 * dtj + 1e-12, rnear[e]);
        }
        rnear[(int64_t)(NFS + j) * E + e] = rc;
    }
}

// ---------------------------------------------------------------------------
// sort keys: element (for the classification order) and tier*E + element
// (for the correction buckets); values are pair indices
// ---------------------------------------------------------------------------
__global__ void k_iota(int64_t P, int* __restrict__ v)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) v[p] = (int)p;
}

__global__ void k_tier_keys(int64_t P, int E, const int8_t* __restrict__ tier, const int* __restrict__ pe,
                            int* __restrict__ key, int* __restrict__ val)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    key[p] = (int)tier[p] * E + pe[p];
    val[p] = (int)p;
}

// ---------------------------------------------------------------------------
// upsampled tiers: upsampled rule minus smooth rule, one wavefront per 64
// pairs of one element; the element's correction points are staged in LDS
// ---------------------------------------------------------------------------
// wave w covers sorted[ws[4w] .. ws[4w] + ws[4w+1]) of element ws[4w+2]
// with the rule of tier index ws[4w+3]: the element's tier rule (Mf points)
// plus its base rule with negated weight, staged in LDS 64 points at a time.
// One launch serves every tier, so the host can order the wavefronts by cost.
static_assert(NUP == 3, "k_corr_up selects among three tiers' rules");
static_assert(up_ns(1) == up_ns(0) && up_nt(1) == 2 * up_nt(0) && up_nt(0) == NT,
              "the 32 x 64 rule contains the closed-end far-field rule at its even angles");
template <int KER>
__global__ __launch_bounds__(64) void k_corr_up(UpRules ur, const int* __restrict__ ws,
                                                const int* __restrict__ sorted, const int* __restrict__ pt,
                                                const double* __restrict__ xt, int64_t T,
                                                const ElemInfo* __restrict__ info,
                                                const int64_t* __restrict__ boff, const double* __restrict__ by,
                                                const double* __restrict__ bn, const double* __restrict__ bsw,
                                                int64_t Nb, double* __restrict__ corr)
{
    // one wavefront per run of up to UP_PAIRS pairs of one element, UP_TPT
    // pairs per lane; rule points staged through LDS as 16-byte-pair records
    __shared__ __attribute__((aligned(16))) double src[64 * FAR_REC];
    const int w = blockIdx.x, lane = threadIdx.x;
    const int e = ws[4 * w + 2], ti = ws[4 * w + 3];
    const double* __restrict__ cpy = ti == 0 ? ur.y[0] : (ti == 1 ? ur.y[1] : ur.y[2]);
    const double* __restrict__ cpn = ti == 0 ? ur.n[0] : (ti == 1 ? ur.n[1] : ur.n[2]);
    const double* __restrict__ swf = ti == 0 ? ur.sw[0] : (ti == 1 ? ur.sw[1] : ur.sw[2]);
    const int64_t Mf = ti == 0 ? ur.Mf[0] : (ti == 1 ? ur.Mf[1] : ur.Mf[2]);
    const int64_t Mtot = ti == 0 ? ur.Mtot[0] : (ti == 1 ? ur.Mtot[1] : ur.Mtot[2]);
    int64_t p[UP_TPT];
    double x[UP_TPT][3], sa[UP_TPT][3], sb[UP_TPT][3], sd[UP_TPT][3];
#pragma unroll
    for (int u = 0; u < UP_TPT; ++u) {
        const int k = lane + 64 * u;
        p[u] = (k < ws[4 * w + 1]) ? (int64_t)sorted[(int64_t)ws[4 * w] + k] : -1;
        const int64_t t = p[u] >= 0 ? pt[p[u]] : -1;
        x[u][0] = t >= 0 ? xt[t] : 0.0;
        x[u][1] = t >= 0 ? xt[T + t] : 0.0;
        x[u][2] = t >= 0 ? xt[2 * T + t] : 0.0;
        for (int d = 0; d < 3; ++d) sa[u][d] = sb[u][d] = sd[u][d] = 0.0;
    }
    const int64_t nbase = boff[e + 1] - boff[e];
    // An element whose far-field rule is the 32 x 32 tensor rule (closed
    // ends) has those points among the 32 x 64 rule's, as its even angles,
    // with twice the weight: the 32 x 64 correction is then the alternating
    // sum over the 32 x 64 points alone (odd angles +, even angles -).
    const bool alt = ti == 1 && info[e].fb == 2;
    for (int pass = 0; pass < (alt ? 1 : 2); ++pass) {
        // pass 0: the upsampled rule; pass 1: minus the element's far-field rule
        const double* py = pass ? by : cpy;
        const double* pn = pass ? bn : cpn;
        const double* psw = pass ? bsw : swf;
        const int64_t ld = pass ? Nb : Mtot;
        const int64_t base0 = pass ? boff[e] : (int64_t)e * Mf;
        const int64_t cnt = pass ? nbase : Mf;
        for (int64_t base = 0; base < cnt; base += 64) {
            const int64_t m = base0 + base + lane;
            const double sg = pass ? -1.0 : (alt && !((base + lane) & 1) ? -1.0 : 1.0);
            if (base + lane < cnt) {
                double* r = src + lane * FAR_REC;
                r[0] = py[m];
                r[1] = py[ld + m];
                r[2] = py[2 * ld + m];
                r[3] = pn[m];
                r[4] = pn[ld + m];
                r[5] = pn[2 * ld + m];
                r[6] = sg * psw[m];
                r[7] = sg * psw[ld + m];
                r[8] = sg * psw[2 * ld + m];
                r[9] = 0.0;
            }
            __syncthreads();
            const int nin = (int)min((int64_t)64, cnt - base);
#pragma unroll 2
            for (int kk = 0; kk < nin; ++kk) {
                const double2* r2 = reinterpret_cast<const double2*>(src + kk * FAR_REC);
                const double2 A = r2[0], B = r2[1], C = r2[2], D = r2[3], F = r2[4];
#pragma unroll
                for (int u = 0; u < UP_TPT; ++u) pair_acc<KER>(x[u], A, B, C, D, F, sa[u], sb[u], sd[u]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int u = 0; u < UP_TPT; ++u) {
        if (p[u] >= 0) {
            double o[6];
            scaled_out<KER>(sa[u], sb[u], sd[u], o);
            for (int k = 0; k < 6; ++k) corr[p[u] * 6 + k] = o[k];
        }
    }
}

// ---------------------------------------------------------------------------
// special quadrature (Sections 3.2.2-3.2.4), one wavefront per pair
// ---------------------------------------------------------------------------
struct RuleTables {
    const int* off;       // [nb+1] offsets of the theta-rules (bracket b at index b-1)
    const double* th;     // nodes
    const double* w;      // weights
    const double* cs;     // cos, sin and 1 - cos of every node (same layout)
    const double* sn;
    const double* omc;
    int nb;
    const double* lx;     // log rule nodes on (0,1), singular at 0
    const double* lw;
    int nl;
    // whole-element singular s-rules (Section 3.2.4): set k, target GL index
    // i has nodes wd[woff[k NS + i] ..) as offsets from the i-th GL node in
    // the element variable v in [-1, 1], with weights ww for the integral
    // over v.  Sets 0..wnb-1: cylinders of aspect [2^(wb_lo + k),
    // 2^(wb_lo + k + 1)); set wsph (if >= 0): the sphere.  wany: the cylinder
    // rules also on open elements of other shapes.  wnb = 0 and wsph < 0
    // disable them.
    const int* woff;
    const double* wd;
    const double* ww;
    int wb_lo, wnb, wl0, wsph, wany;
};

// Wavefront-wide sum (64 lanes).
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wavefront per (target, element) pair, s-nodes taken in batches of SB.
//  1. lanes 0..SB-1, one s-node each: node, weight, interpolation weights;
//     all lanes: the centerline quantities at the s-nodes (an MFMA product);
//     lanes 0..SB-1 again: circle frame, the target's coordinates relative to
//     the circle and the choice of theta-rule -> one record per s-node in LDS;
//  2. all lanes: the density's Fourier coefficients (modes up to the measured
//     band) interpolated to the batch's s-nodes (an MFMA product);
//  3. all lanes: the batch's (s-node, theta-node) points as one flat list of
//     mirror pairs, 64 pairs at a time.  With the target's radial direction
//     b0 and b0p = t x b0 as basis, r = z t + (dr + eps(1 - cos phi)) b0 -
//     eps sin phi b0p, and the area element and r.n reduce to the scalars
//     g = |x_c'| + eps (e1'.t cos + e2'.t sin) and eps' (|y_t x y_s| =
//     eps sqrt(g^2 + eps'^2)), so a point costs half a Fourier synthesis and
//     a handful of flops.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int SB = 16;
static_assert(SB == 16, "the coefficient interpolation uses 16-row MFMA tiles");
enum { R_E = 0, R_EP, R_SP, R_A13, R_A23, R_Z, R_DR, R_T, R_B0 = R_T + 3, R_B0P = R_B0 + 3, R_W = R_B0P + 3, R_C0,
       R_S0, R_WQ, NREC };
constexpr int QVS = CLQ + 1;   // row stride of the interpolated centerline quantities
static_assert(CLQ <= 32, "the centerline interpolation uses two 16-column MFMA tiles");

// Modes of the special-quadrature kernel (MODE_*, csbq_kernels.hpp): the
// density route (corrections for the given density), the count of its rows
// per pair, and the rows of the correction matrix in the density's
// coefficient basis.
struct MatrixOut {
    const int64_t* roff;   // first row of each pair (by block), MODE_MATRIX
    double* V;             // [rows][CORR_NC][NT]: kernel components times basis functions, summed over a node's angles
    double* L;             // [rows][NS]: interpolation weights of the node from the GL rows
    int* count;            // [pairs]: rows of each pair, MODE_COUNT
    const double* lup0;    // [up_ns(0)][NS]: GL rows -> the closed-end far-field rule's rows
    const double* bw;      // [Nb]: weights of the far-field rule's points
};

// Correction-matrix rows of one pair (one wavefront).  Row m of the pair is a
// quadrature node s_m in s (an s-node of the special rule, or a row of the
// element's far-field rule with negated weights); its entries are
//   V[m][c][k] = sum over the node's angles q of w_q K_c(x, y(s_m, t_q)) b_k(t_q),
// K_c the six symmetric components of the single layer (W J (I/|r| +
// r r^T/|r|^3) up to the constant 1/(8 pi)) and of the double layer (W (r.n)
// r r^T/|r|^5, up to -3/(4 pi)), b_k the density's trigonometric basis (cos
// k t for k = 0..16, then sin k t for k = 1..15, at absolute angles t).  With
// L[m][i] the interpolation weights of s_m from the GL rows, the correction of
// the density with coefficients sigma^_{i,k} is sum_{m,i,k,c} L[m][i]
// V[m][c][k] sigma^_{i,k}.  The sums over angles run as FP64 MFMA 16x16x4
// products: four angles at a time, lane l holding component (l mod 16) of
// angle l / 16 and basis function (l mod 16) there.
constexpr int CORR_NC = 12;   // symmetric components: S (xx xy xz yy yz zz), D (same)
__device__ __forceinline__ void sym_pair(int c, int& a, int& b)
{
    const int cc = c % 6;
    a = cc < 3 ? 0 : (cc < 5 ? 1 : 2);
    b = cc < 3 ? cc : (cc < 5 ? cc - 2 : 2);
}

// component `row` (0..11, else 0) of the Stokes kernel pair at r, scaled by the
// single-layer factor aS = W J / |r| and the double-layer factor cD = W (r.n) / |r|^5
__device__ __forceinline__ double sym_component(int row, const double r[3], double aS, double ir2, double cD)
{
    if (row >= CORR_NC) return 0.0;
    int a, b;
    sym_pair(row, a, b);
    const double rab = r[a] * r[b];
    return row < 6 ? aS * ((a == b ? 1.0 : 0.0) + ir2 * rab) : cD * rab;
}

// basis functions of lane column k (0..15) at angle t: cos k t (first block),
// sin k t (second; cos 16 t in column 0)
__device__ __forceinline__ void basis_pair(int k, double t, double& b0, double& b1)
{
    double sn, cs;
    sincos((double)(k ? k : NT / 2) * t, &sn, &cs);
    b0 = k ? cs : 1.0;
    b1 = k ? sn : cs;
}

__device__ __forceinline__ void matrix_row_store(const MatrixOut& mo, int64_t row, int lane, v4d acc0, v4d acc1)
{
    const int g4 = lane >> 4, k = lane & 15;
    double* Vr = mo.V + row * (CORR_NC * NT);
#pragma unroll
    for (int i = 0; i < 3; ++i) {   // rows g4 + 4i < 12 of the MFMA tile
        const int c = g4 + 4 * i;
        Vr[c * NT + k] = acc0[i];
        Vr[c * NT + NT / 2 + k] = acc1[i];
    }
}

template <int KER>
__device__ void matrix_rows_special(int nb, int base, int lane, const double (*rec)[NREC], const int* rq_off,
                                    const int* rq_step, const int* npt, const double* lwl, const RuleTables& rt,
                                    double sgn, const MatrixOut& mo)
{
    static_assert(KER == KER_STOKES, "the correction matrix is built for the Stokes pair");
    const int g4 = lane >> 4, col = lane & 15;
    for (int j = 0; j < nb; ++j) {
        const double* R = rec[j];
        const int ro = rq_off[j];
        const bool trap = ro < 0;
        const int np_ = npt[j];
        const double c0 = R[R_C0], s0t = R[R_S0];
        const double th0 = atan2(s0t, c0);
        const double E = R[R_E], Ep = R[R_EP], z = R[R_Z], dr = R[R_DR];
        const double sp_ = R[R_SP], a13 = R[R_A13], a23 = R[R_A23];
        v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < np_; q0 += 4) {
            const int q = q0 + g4;
            double av = 0.0, bv0 = 0.0, bv1 = 0.0;
            if (q < np_) {
                double cth, sth, cph, sph, omc, wq, th;
                if (trap) {
                    const int ix = q * rq_step[j];
                    cth = c_cos128[ix];
                    sth = c_sin128[ix];
                    th = 2.0 * PI * q / np_;
                    cph = fma(cth, c0, sth * s0t);
                    sph = fma(sth, c0, -cth * s0t);
                    omc = 1.0 - cph;
                    wq = R[R_WQ];
                } else {
                    const int qq = ro + q;
                    cph = rt.cs[qq];
                    sph = rt.sn[qq];
                    omc = rt.omc[qq];
                    wq = rt.w[qq];
                    th = th0 + rt.th[qq];
                    cth = fma(c0, cph, -s0t * sph);
                    sth = fma(s0t, cph, c0 * sph);
                }
                const double W = R[R_W] * wq;
                const double gq = sp_ + a13 * cth + a23 * sth;
                const double jq = fma(gq, gq, Ep * Ep);
                const double J = E * (jq * rsqrt_nr1(jq));
                const double A = dr + E * omc, B = -E * sph;
                double r[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) r[d] = z * R[R_T + d] + A * R[R_B0 + d] + B * R[R_B0P + d];
                const double rr = z * z + A * A + B * B;
                const double ir = rr > 0.0 ? rsqrt_nr1(rr) : 0.0;
                const double ir2 = ir * ir;
                const double rn = sgn * E * (gq * (dr * cph - E * omc) - Ep * z);
                av = sym_component(col, r, W * J * ir, ir2, W * rn * ir2 * ir2 * ir);
                basis_pair(col, th, bv0, bv1);
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv1, acc1, 0, 0, 0);
        }
        const int64_t row = mo.roff[blockIdx.x] + base + j;
        matrix_row_store(mo, row, lane, acc0, acc1);
        if (lane < NS) mo.L[row * NS + lane] = lwl[j * NS + lane];
    }
}

// rows of the element's far-field rule (nbrows rows of NT angles at bo..),
// with negated weights: the rule the smooth sum applied, which the correction
// replaces (a source at the target itself contributes nothing)
template <int KER>
__device__ void matrix_rows_base(int nbrows, int S, int lane, const double x[3], int64_t bo,
                                 const double* __restrict__ by, const double* __restrict__ bn, int64_t Nb,
                                 const MatrixOut& mo, bool closed)
{
    static_assert(KER == KER_STOKES, "the correction matrix is built for the Stokes pair");
    const int g4 = lane >> 4, col = lane & 15;
    for (int rr_ = 0; rr_ < nbrows; ++rr_) {
        v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < NT; q0 += 4) {
            const int q = q0 + g4;
            const int64_t n = bo + (int64_t)rr_ * NT + q;
            const double r[3] = {x[0] - by[n], x[1] - by[Nb + n], x[2] - by[2 * Nb + n]};
            const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double ir = rr > 0.0 ? rsqrt_nr1(rr) : 0.0;
            const double ir2 = ir * ir;
            const double w = -mo.bw[n];
            const double rn = r[0] * bn[n] + r[1] * bn[Nb + n] + r[2] * bn[2 * Nb + n];
            const double av = sym_component(col, r, w * ir, ir2, w * rn * ir2 * ir2 * ir);
            double bv0, bv1;
            basis_pair(col, 2.0 * PI * q / NT, bv0, bv1);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv1, acc1, 0, 0, 0);
        }
        const int64_t row = mo.roff[blockIdx.x] + S + rr_;
        matrix_row_store(mo, row, lane, acc0, acc1);
        if (lane < NS) mo.L[row * NS + lane] = closed ? mo.lup0[rr_ * NS + lane] : (lane == rr_ ? 1.0 : 0.0);
    }
}

template <int KER, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_corr_full(const int* __restrict__ listf, const int* __restrict__ pe,
                                                  const int* __restrict__ pt, const double* __restrict__ xt,
                                                  int64_t T, const int64_t* __restrict__ tnode,
                                                  const double* __restrict__ clq, const double* __restrict__ sh,
                                                  const ElemInfo* __restrict__ info, const int* __restrict__ band,
                                                  const double* __restrict__ cls,
                                                  const int64_t* __restrict__ boff, const double* __restrict__ by,
                                                  const double* __restrict__ bn, const double* __restrict__ bsw,
                                                  int64_t Nb, RuleTables rt, GateConsts gc,
                                                  double* __restrict__ corr, int* __restrict__ err,
                                                  int* __restrict__ work, int cstride, MatrixOut mo)
{
    // cf: [SB][cstride] density coefficients at the batch's s-nodes, cstride =
    // 6 (largest band + 1) over all elements (dynamic LDS, at least
    // SB x (NS + QVS) doubles).  The same space holds the bisection stack
    // while the s-rule is built, and each batch's interpolation weights
    // [SB][NS] and centerline quantities [SB][QVS] from phase 1 until phase 2
    // has read them, which keeps the block's LDS small enough for three waves
    // per SIMD.
    extern __shared__ __attribute__((aligned(16))) double cf[];
    double* const lwl = cf;
    double* const qv = cf + SB * NS;   // phase 1b output [SB][QVS]
    double* const st_lo = cf;
    double* const st_hi = cf + 48;
    __shared__ __attribute__((aligned(16))) double rec[SB][NREC];
    __shared__ int rq_off[SB], rq_step[SB], npt[SB], pref[SB + 1];
    __shared__ double sub_lo[MAXSUB], sub_hi[MAXSUB];
    __shared__ int sub_ty[MAXSUB], soff[MAXSUB + 1];
    __shared__ int nsub, wrule;
    // reference GL node i0 (the target's own node, else the node nearest the
    // singularity): E0, Xp0[3], sp0, t0[3], then bn[3] (own) or the target's
    // offset xr[3] = x - x_c(s_i0), and z_ref = xr.t0, k_ref = |xr|^2 - E0^2
    __shared__ double f0d[16];
    // the barycentric table of the reference node: x_i0 - x_i and lam_i
    __shared__ double bwt[2 * NS];
    // the pair's scalars, read where they are used inside the s-node loop
    // rather than held in registers across it: s0, hw, the normal's sign, the
    // three trapezoid thresholds, the target x[3]
    __shared__ double pq[9];
    enum { PQ_S0 = 0, PQ_HW, PQ_SGN, PQ_TRAP, PQ_X = PQ_TRAP + 3 };
    const int lane = threadIdx.x;
    const int64_t p = listf[blockIdx.x];
    const int e = pe[p];
    const int64_t t = pt[p];
    const ElemInfo inf = info[e];
    const double x[3] = {xt[t], xt[T + t], xt[2 * T + t]};
    // the element's centerline data, read at wave-uniform addresses
    const double* __restrict__ sq = clq + (int64_t)e * CLQ * NS;
    const int64_t nd = tnode ? tnode[t] : -1;
    const bool own = nd >= 0 && nd / NPE == e;
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    const int ncoef = 6 * (Mt + 1);
    // thresholds on the circle's cosh(alpha) - 1 above which a trapezoid rule
    // of nt, 2nt or 4nt points meets the tolerance (Section 3.2.2)
    if (lane == 0) {
        const double lg = log(gc.ct / gc.tol);
        for (int k = 0; k < 3; ++k) pq[PQ_TRAP + k] = cosh(lg / (double)((NT << k) - Mt - gc.extra_modes)) - 1.0;
        pq[PQ_HW] = 0.5 * (inf.c - inf.a);
        pq[PQ_SGN] = (double)inf.sign;
        for (int d = 0; d < 3; ++d) pq[PQ_X + d] = x[d];
    }
    const double* __restrict__ she = sh + (int64_t)e * NS * NSH;
    __syncthreads();
    // Every s-node and circle is placed relative to a reference GL node i0 of
    // the element: its parameter as an offset from s_i0 and its centerline
    // data as differences from the samples there.  Near the target these
    // offsets are small and keep their relative accuracy, whereas absolute
    // parameters (rounded to ~1e-16 of s) would move quadrature nodes by a
    // relative 1e-16 / (distance in s): 2e-9 of the double layer at 1e-7 from
    // the surface.
    int i0 = 0;
    double s0 = 0.0;
    {
        if (own) {
            i0 = (int)((nd % NPE) / NT);
        } else {
            // the GL node nearest the singularity's real part
            const double xr = (cls[p * 4 + 0] - inf.a) / (0.5 * (inf.c - inf.a)) - 1.0;
            double best = 1e300;
            for (int i = 0; i < NS; ++i) {
                const double dd = fabs(c_gx[i] - xr);
                if (dd < best) {
                    best = dd;
                    i0 = i;
                }
            }
        }
        s0 = 0.5 * (inf.a + inf.c) + 0.5 * (inf.c - inf.a) * c_gx[i0];
        if (lane == 0) pq[PQ_S0] = s0;
        if (lane < NS) {
            bwt[2 * lane] = lane == i0 ? 0.0 : c_gx[i0] - c_gx[lane];
            bwt[2 * lane + 1] = c_lam[lane];
        }
        if (lane == 0) {
            double q0[CLQ];
            for (int k = 0; k < CLQ; ++k) q0[k] = sq[k * NS + i0];
            Frame f0;
            frame_from_q(q0, f0);
            f0d[0] = f0.E;
            for (int d = 0; d < 3; ++d) {
                f0d[1 + d] = f0.Xp[d];
                f0d[5 + d] = f0.t[d];
            }
            f0d[4] = f0.sp;
            if (own) {
                const int j0 = (int)(nd % NT);
                for (int d = 0; d < 3; ++d) f0d[8 + d] = f0.e1[d] * c_cos[j0] + f0.e2[d] * c_sin[j0];
            } else {
                double xr[3], xx = 0.0;
                for (int d = 0; d < 3; ++d) {
                    xr[d] = x[d] - q0[Q_X + d];
                    f0d[8 + d] = xr[d];
                    xx += xr[d] * xr[d];
                }
                f0d[11] = dot3(xr, f0.t);
                f0d[12] = xx - f0.E * f0.E;
            }
        }
    }
    // ---- s-rule: list of sub-panels (lane 0)
    if (lane == 0) {
        int ns_ = 0;
        const double a = inf.a, c = inf.c;
        // whole-element singular rule (Section 3.2.4, second part) for an
        // on-surface target on an open element whose aspect at the target,
        // A = (element length at the target's speed) / radius = 2 hw |x_c'| / eps,
        // falls in a tabulated bracket; closed cross-sections (the rules'
        // cylinders have none) and bands beyond the rules' modes keep the
        // general form below
        int wr = -1;
        if (own && Mt <= rt.wl0) {
            if (inf.shape == SHAPE_SPHERE && rt.wsph >= 0) {
                wr = rt.wsph * NS + i0;
            } else if (rt.wnb > 0 && !inf.closed && (inf.shape == SHAPE_CYLINDER || rt.wany)) {
                const double A = (c - a) * f0d[4] / f0d[0];
                if (A > 0.0 && A < 1e300) {
                    int ex;
                    frexp(A, &ex);   // A in [2^(ex-1), 2^ex)
                    const int b = ex - 1 - rt.wb_lo;
                    if (b >= 0 && b < rt.wnb) wr = b * NS + i0;
                }
            }
        }
        wrule = wr;
        if (wr >= 0) {
            sub_lo[0] = a;
            sub_hi[0] = c;
            sub_ty[0] = SUB_WHOLE;
            ns_ = 1;
        } else if (own) {
            // dyadic refinement toward s0 down to ~eps/speed, log-singular
            // panels on both sides of s0 (Section 3.2.4, general form).  The
            // panel size is also cut by the density's Fourier band: the
            // modal Green's function of mode l turns from its log form to
            // decay at ~eps/l from the circle, so at band Mt the log rule
            // (p log u + q, degree < 16) must cover eps/(Mt/4) at most (a
            // density of every mode up to 16 left 1e-6 with eps/speed
            // panels, 2e-11 with a quarter of that)
            const double hmin = gc.hmin_fac * sq[Q_E * NS + i0] / cls[p * 4 + 2] * (Mt > 4 ? 4.0 / Mt : 1.0);
            for (int side = 0; side < 2; ++side) {
                double L = side ? (c - s0) : (s0 - a);
                int lev = 0;
                while (L > hmin && lev < 40 && ns_ < MAXSUB - 2) {
                    double u0 = 0.5 * L, u1 = L;
                    sub_lo[ns_] = side ? s0 + u0 : s0 - u1;
                    sub_hi[ns_] = side ? s0 + u1 : s0 - u0;
                    sub_ty[ns_] = SUB_GL;
                    ++ns_;
                    L *= 0.5;
                    ++lev;
                }
                sub_lo[ns_] = side ? s0 : s0 - L;
                sub_hi[ns_] = side ? s0 + L : s0;
                sub_ty[ns_] = side ? SUB_LOG_LO : SUB_LOG_HI;
                ++ns_;
            }
        } else {
            // adaptive bisection until the target is outside every sub-panel's
            // near region (Section 3.2.3), judged by the Bernstein parameter of
            // the s-integrand's nearest singularity
            const double sr = cls[p * 4 + 0], si_ = cls[p * 4 + 1];
            const double rreq = pow(gc.cs / gc.tol, 1.0 / (double)(2 * NS - Ms));
            // rho(sub-panel) >= rreq  <=>  s* lies outside the Bernstein
            // ellipse of parameter rreq (semi-axes A h, B h about the
            // sub-panel's midpoint, h its half-length):
            // (x B)^2 + (y A)^2 >= (A B h)^2, no root or division
            const double EA = 0.5 * (rreq + 1.0 / rreq), EB = 0.5 * (rreq - 1.0 / rreq);
            const double EA2 = EA * EA, EB2 = EB * EB, EAB2 = EA2 * EB2, y2A = si_ * si_ * EA2;
            int sp = 0;
            st_lo[sp] = a;
            st_hi[sp] = c;
            ++sp;
            while (sp > 0) {
                --sp;
                double lo = st_lo[sp], hi = st_hi[sp];
                const double xm = sr - 0.5 * (lo + hi), hh = 0.5 * (hi - lo);
                bool ok = xm * xm * EB2 + y2A >= EAB2 * hh * hh;
                if (ok || (hi - lo) < 1e-12 * (c - a) || sp + 2 > 48 || ns_ + sp + 2 > MAXSUB) {
                    if (!ok) atomicOr(err, FLAG_SRULE_LIMIT);
                    sub_lo[ns_] = lo;
                    sub_hi[ns_] = hi;
                    sub_ty[ns_] = SUB_GL;
                    ++ns_;
                } else {
                    double mid = 0.5 * (lo + hi);
                    st_lo[sp] = mid;  // right half first so the left is processed next
                    st_hi[sp] = hi;
                    ++sp;
                    st_lo[sp] = lo;
                    st_hi[sp] = mid;
                    ++sp;
                }
            }
        }
        soff[0] = 0;
        for (int k = 0; k < ns_; ++k)
            soff[k + 1] = soff[k] + (sub_ty[k] == SUB_GL ? NS
                                    : sub_ty[k] == SUB_WHOLE ? rt.woff[wr + 1] - rt.woff[wr] : rt.nl);
        nsub = ns_;
    }
    __syncthreads();
    const int nsb = nsub;
    const int S = soff[nsb];
    const int nbrows = inf.fb == 2 ? up_ns(0) : NS;   // rows of the element's far-field rule
    if constexpr (MODE == MODE_COUNT) {
        if (lane == 0) mo.count[blockIdx.x] = S + nbrows;
        return;
    }
    double a0 = 0, a1 = 0, a2 = 0, b0_ = 0, b1_ = 0, b2_ = 0;
    int n_theta = 0;
    for (int base = 0; base < S; base += SB) {
        const int nb = min(SB, S - base);
        // ---- 1a. one s-node per lane: node, weight, interpolation weights
        double ws = 0.0;
        if (lane < nb) {
            const int g = base + lane;
            int lo_i = 0, hi_i = nsb;   // soff[lo_i] <= g < soff[hi_i]
            while (hi_i - lo_i > 1) {
                int mid = (lo_i + hi_i) >> 1;
                if (soff[mid] <= g) lo_i = mid; else hi_i = mid;
            }
            const int m = g - soff[lo_i];
            const double lo = sub_lo[lo_i], hi = sub_hi[lo_i];
            const int ty = sub_ty[lo_i];
            double s, u;
            if (ty == SUB_GL) {
                s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * c_gx[m];
                ws = 0.5 * (hi - lo) * c_gw[m];
                // offset from s_i0 formed from differences (lo - s0 is exact
                // for nearby sub-panels), not from the rounded absolute s
                u = own ? s - pq[PQ_S0] : (lo - pq[PQ_S0]) + 0.5 * (hi - lo) * (1.0 + c_gx[m]);
            } else if (ty == SUB_WHOLE) {
                // tabulated node offsets from the target's GL node: u is
                // formed without the absolute parameter
                const int o = rt.woff[wrule] + m;
                u = pq[PQ_HW] * rt.wd[o];
                s = pq[PQ_S0] + u;
                ws = pq[PQ_HW] * rt.ww[o];
            } else if (ty == SUB_LOG_LO) {
                u = (hi - lo) * rt.lx[m];
                s = lo + u;
                ws = (hi - lo) * rt.lw[m];
            } else {
                u = -(hi - lo) * rt.lx[m];
                s = hi + u;
                ws = (hi - lo) * rt.lw[m];
            }
            double lw[NS];
            bary_weights_rel_tab(bwt, u / pq[PQ_HW], lw);
#pragma unroll
            for (int i = 0; i < NS; ++i) lwl[lane * NS + i] = lw[i];
        }
        __syncthreads();
        // ---- 1b. centerline quantities at the batch's s-nodes: [nb x NS]
        // weights times the element's [NS x CLQ] samples (on the target's own
        // element, differences from the samples at the target's GL node), as
        // FP64 MFMA 16x16x4 tiles in the layout of phase 2
        {
            const int r = lane & 15, qq = lane >> 4;
            double wa[NS / 4];
#pragma unroll
            for (int ks = 0; ks < NS / 4; ++ks) wa[ks] = (r < nb) ? lwl[r * NS + 4 * ks + qq] : 0.0;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int col = cb * 16 + r;
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < NS / 4; ++ks) {
                    double bv = 0.0;
                    if (col < CLQ) bv = sq[col * NS + 4 * ks + qq] - sq[col * NS + i0];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[ks], bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = qq + 4 * i;
                    if (row < nb && col < CLQ) qv[row * QVS + col] = acc[i];
                }
            }
        }
        __syncthreads();
        // ---- 1c. one s-node per lane: frame, local coordinates, theta-rule
        if (lane < nb) {
            Frame fr;
            CircleLocal cl;
            {
                double q[CLQ];
                const double* dq = qv + lane * QVS;   // differences from the reference node's samples
#pragma unroll
                for (int k = 0; k < CLQ; ++k) q[k] = sq[k * NS + i0] + dq[k];
                frame_from_q(q, fr);
                Frame f0;
                f0.E = f0d[0];
                for (int d = 0; d < 3; ++d) {
                    f0.Xp[d] = f0d[1 + d];
                    f0.t[d] = f0d[5 + d];
                }
                f0.sp = f0d[4];
                const double v3[3] = {f0d[8], f0d[9], f0d[10]};
                if (own)
                    circle_local_rel(fr, f0, v3, dq, cl);
                else
                    circle_local_off(fr, f0, v3, f0d[11], f0d[12], dq, cl);
            }
            // theta-rule for this circle (Section 3.2.2): trapezoid of nt, 2nt
            // or 4nt points if the estimate allows, else the bracket's
            // generalized Chebyshev rule
            int ntr = 0, rb = 0;
            for (int k = 0; k < 3 && !ntr; ++k)
                if (cl.cha >= pq[PQ_TRAP + k]) ntr = NT << k;
            if (!ntr) {
                int ex;
                frexp(sqrt(cl.d2) / fr.E, &ex);   // alpha in [2^(ex-1), 2^ex)
                int b = 1 - ex;
                if (b < 1) {
                    ntr = 4 * NT;
                } else {
                    if (b > rt.nb) {
                        b = rt.nb;
                        atomicOr(err, FLAG_THETA_CLAMP);
                    }
                    rb = b;
                }
            }
            double* R = rec[lane];
            R[R_E] = fr.E;
            R[R_EP] = fr.Ep;
            R[R_SP] = fr.sp;
            R[R_A13] = fr.E * dot3(fr.e1p, fr.t);
            R[R_A23] = fr.E * dot3(fr.e2p, fr.t);
            R[R_Z] = cl.z;
            R[R_DR] = cl.dr;
            for (int d = 0; d < 3; ++d) {
                R[R_T + d] = fr.t[d];
                R[R_B0 + d] = cl.b0[d];
                R[R_B0P + d] = cl.b0p[d];
            }
            R[R_W] = ws;
            // closest angle theta0 of the circle: (cos, sin) of the radial direction
            R[R_C0] = dot3(cl.b0, fr.e1);
            R[R_S0] = dot3(cl.b0, fr.e2);
            R[R_WQ] = ntr ? 2.0 * PI / ntr : 0.0;
            rq_off[lane] = ntr ? -1 : rt.off[rb - 1];
            rq_step[lane] = ntr ? 128 / ntr : 0;
            npt[lane] = ntr ? ntr : rt.off[rb] - rt.off[rb - 1];
        }
        __syncthreads();
        if constexpr (MODE == MODE_MATRIX) {
            matrix_rows_special<KER>(nb, base, lane, rec, rq_off, rq_step, npt, lwl, rt, pq[PQ_SGN], mo);
            __syncthreads();
            continue;
        }
        // ---- 2. density coefficients at the batch's s-nodes
        if (lane == 0) {
            pref[0] = 0;
            for (int j = 0; j < nb; ++j) pref[j + 1] = pref[j] + npt[j] / 2;   // point pairs
        }
        // coefficients at the s-nodes = [nb x NS] interpolation weights times
        // the [NS x ncoef] GL-row coefficients: FP64 MFMA 16x16x4 tiles
        // (A: lane l holds W[l % 16][4 ks + l / 16]; B: C[4 ks + l / 16][l % 16];
        // D: lane l holds rows l / 16 + 4 i, i < 4, of column l % 16)
        {
            const int r = lane & 15, qq = lane >> 4;
            double wa[NS / 4];
#pragma unroll
            for (int ks = 0; ks < NS / 4; ++ks) wa[ks] = (r < nb) ? lwl[r * NS + 4 * ks + qq] : 0.0;
            __syncthreads();   // the weights are read before cf overwrites them
            for (int cb = 0; cb * 16 < ncoef; ++cb) {
                const int col = cb * 16 + r;
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < NS / 4; ++ks) {
                    const double bv = (col < ncoef) ? she[(4 * ks + qq) * NSH + col] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[ks], bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = qq + 4 * i;
                    if (row < nb && col < ncoef) cf[row * cstride + col] = acc[i];
                }
            }
        }
        __syncthreads();
        // s-nodes with a tabulated rule: coefficients turned to the closest
        // angle theta0, (a, b)_l -> (a cos l theta0 + b sin l theta0,
        // b cos l theta0 - a sin l theta0), so that the series is in phi
        if (lane < 3 * nb) {
            const int jj = lane / 3, d = lane - 3 * jj;
            if (rq_off[jj] >= 0) {
                const double c0 = rec[jj][R_C0], s0t = rec[jj][R_S0];
                double* Cj = cf + jj * cstride;
                double cl = c0, sl = s0t;
                for (int l = 1; l <= Mt; ++l) {
                    const double a = Cj[6 * l + d], b = Cj[6 * l + 3 + d];
                    Cj[6 * l + d] = fma(a, cl, b * sl);
                    Cj[6 * l + 3 + d] = fma(b, cl, -a * sl);
                    const double cn = fma(cl, c0, -sl * s0t);
                    sl = fma(sl, c0, cl * s0t);
                    cl = cn;
                }
            }
        }
        __syncthreads();
        // ---- 3. the batch's points in mirror pairs, one pair per lane and
        // step: a trapezoid node theta with theta + pi, a tabulated rule's node
        // theta0 + phi with theta0 - phi (the rules are symmetric, equal
        // weights).  Both points share one Fourier recurrence in psi (theta,
        // resp. phi): with the sums Ce, Co of the cosine terms of even and odd
        // modes and Se, So of the sine terms, the pair's densities are
        // T = Ce + Co + Se + So and, for the trapezoid, (Ce + Se) - (Co + So)
        // (cos l(psi + pi) = (-1)^l cos l psi), for the rule (Ce + Co) -
        // (Se + So) (sine terms odd in phi).
        const int Pb = pref[nb];
        int j = 0;
        for (int P = lane; P < Pb; P += 64) {
            while (P >= pref[j + 1]) ++j;
            const int k = P - pref[j];
            const double* R = rec[j];
            const double c0 = R[R_C0], s0t = R[R_S0];
            const int ro = rq_off[j];
            const bool trap = ro < 0;
            double ca, sa, wq, cth[2], sth[2], cph[2], sph[2], omc[2];
            if (trap) {
                const int ix = k * rq_step[j];
                ca = c_cos128[ix];
                sa = c_sin128[ix];
                const double cp = fma(ca, c0, sa * s0t), sp = fma(sa, c0, -ca * s0t);   // phi = theta - theta0
                cth[0] = ca;
                sth[0] = sa;
                cth[1] = -ca;
                sth[1] = -sa;
                cph[0] = cp;
                sph[0] = sp;
                cph[1] = -cp;
                sph[1] = -sp;
                omc[0] = 1.0 - cp;
                omc[1] = 1.0 + cp;
                wq = R[R_WQ];
            } else {
                const int q = ro + (npt[j] >> 1) + k;   // the positive half of the rule
                ca = rt.cs[q];
                sa = rt.sn[q];
                const double om = rt.omc[q];
                wq = rt.w[q];
                cth[0] = fma(c0, ca, -s0t * sa);
                sth[0] = fma(s0t, ca, c0 * sa);
                cth[1] = fma(c0, ca, s0t * sa);
                sth[1] = fma(s0t, ca, -c0 * sa);
                cph[0] = cph[1] = ca;
                sph[0] = sa;
                sph[1] = -sa;
                omc[0] = omc[1] = om;
            }
            n_theta += 2;
            // density by Fourier synthesis over the measured band (the
            // Laplace layers' scalar density is component 0)
            constexpr int NC = KER == KER_LAPLACE ? 1 : 3;
            const double* C = cf + j * cstride;
            double Ce[3] = {C[0], C[1], C[2]}, Co[3] = {0.0, 0.0, 0.0}, Se[3] = {0.0, 0.0, 0.0},
                   So[3] = {0.0, 0.0, 0.0};
            double cl = ca, sl = sa;
            int l = 1;
            for (; l + 1 <= Mt; l += 2) {
                const double* Cl = C + 6 * l;
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    Co[d] = fma(Cl[d], cl, Co[d]);
                    So[d] = fma(Cl[3 + d], sl, So[d]);
                }
                double cn = fma(cl, ca, -sl * sa);
                sl = fma(sl, ca, cl * sa);
                cl = cn;
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    Ce[d] = fma(Cl[6 + d], cl, Ce[d]);
                    Se[d] = fma(Cl[9 + d], sl, Se[d]);
                }
                cn = fma(cl, ca, -sl * sa);
                sl = fma(sl, ca, cl * sa);
                cl = cn;
            }
            if (l <= Mt) {
                const double* Cl = C + 6 * l;
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    Co[d] = fma(Cl[d], cl, Co[d]);
                    So[d] = fma(Cl[3 + d], sl, So[d]);
                }
            }
            double v[2][3];
#pragma unroll
            for (int d = 0; d < NC; ++d) {
                v[0][d] = (Ce[d] + Co[d]) + (Se[d] + So[d]);
                v[1][d] = trap ? (Ce[d] + Se[d]) - (Co[d] + So[d]) : (Ce[d] + Co[d]) - (Se[d] + So[d]);
            }
            const double E = R[R_E], Ep = R[R_EP], z = R[R_Z], dr = R[R_DR];
            const double sp_ = R[R_SP], a13 = R[R_A13], a23 = R[R_A23], W = R[R_W] * wq;
            double tv[3], b0v[3], b0pv[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                tv[d] = R[R_T + d];
                b0v[d] = R[R_B0 + d];
                b0pv[d] = R[R_B0P + d];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double gq = sp_ + a13 * cth[u] + a23 * sth[u];
                // g^2 + eps'^2 > 0 on any admissible tube (eps * curvature < 1)
                const double jq = fma(gq, gq, Ep * Ep);
                const double J = E * (jq * rsqrt_nr1(jq));
                const double A = dr + E * omc[u], B = -E * sph[u];
                double r[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) r[d] = z * tv[d] + A * b0v[d] + B * b0pv[d];
                const double rr = z * z + A * A + B * B;
                const double ir = rr > 0.0 ? rsqrt_nr1(rr) : 0.0;
                const double ir2 = ir * ir;
                const double rn = pq[PQ_SGN] * E * (gq * (dr * cph[u] - E * omc[u]) - Ep * z);
                const double aS = W * J * ir;
                if constexpr (KER == KER_LAPLACE) {
                    a0 = fma(aS, v[u][0], a0);
                    b0_ = fma(W * rn * ir * ir2, v[u][0], b0_);
                } else {
                    const double rs = r[0] * v[u][0] + r[1] * v[u][1] + r[2] * v[u][2];
                    const double bS = aS * rs * ir2;
                    const double cD = W * rn * rs * ir2 * ir2 * ir;
                    a0 += aS * v[u][0] + bS * r[0];
                    a1 += aS * v[u][1] + bS * r[1];
                    a2 += aS * v[u][2] + bS * r[2];
                    b0_ += cD * r[0];
                    b1_ += cD * r[1];
                    b2_ += cD * r[2];
                }
            }
        }
        __syncthreads();
    }
    const int64_t bo = boff[e], bc = boff[e + 1] - boff[e];
    const double xe[3] = {pq[PQ_X], pq[PQ_X + 1], pq[PQ_X + 2]};   // the target, kept in LDS through the loop
    if constexpr (MODE == MODE_MATRIX) {
        matrix_rows_base<KER>(nbrows, S, lane, xe, bo, by, bn, Nb, mo, inf.fb == 2);
        return;
    }
    // minus the element's far-field (base) rule (self term zero)
    for (int64_t k = lane; k < bc; k += 64) {
        int64_t n = bo + k;
        double r0 = xe[0] - by[n], r1 = xe[1] - by[Nb + n], r2 = xe[2] - by[2 * Nb + n];
        double rr = r0 * r0 + r1 * r1 + r2 * r2;
        double ir = rr > 0.0 ? rsqrt_nr1(rr) : 0.0;
        double ir2 = ir * ir;
        double w0 = bsw[n], w1 = bsw[Nb + n], w2 = bsw[2 * Nb + n];
        double rn = r0 * bn[n] + r1 * bn[Nb + n] + r2 * bn[2 * Nb + n];
        if constexpr (KER == KER_LAPLACE) {
            a0 -= ir * w0;
            b0_ -= rn * w0 * ir * ir2;
        } else {
            double rs = r0 * w0 + r1 * w1 + r2 * w2;
            double b = rs * ir * ir2;
            double cD = rn * rs * ir2 * ir2 * ir;
            a0 -= ir * w0 + b * r0;
            a1 -= ir * w1 + b * r1;
            a2 -= ir * w2 + b * r2;
            b0_ -= cD * r0;
            b1_ -= cD * r1;
            b2_ -= cD * r2;
        }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    b0_ = wave_sum(b0_);
    b1_ = wave_sum(b1_);
    b2_ = wave_sum(b2_);
    for (int o = 32; o > 0; o >>= 1) n_theta += __shfl_xor(n_theta, o, 64);
    if (lane == 0) {
        double* o = corr + p * 6;
        o[0] = a0;
        o[1] = a1;
        o[2] = a2;
        o[3] = b0_;
        o[4] = b1_;
        o[5] = b2_;
        int* wk = work + (int64_t)WORK_STRIDE * blockIdx.x;
        wk[0] = n_theta;
        wk[1] = S;
        wk[2] = n_theta * Mt;
        wk[3] = S * (Mt + 1);
        wk[4] = wrule >= 0;
    }
}

// ---------------------------------------------------------------------------
// correction matrix: assembly from the rows, and its application
// ---------------------------------------------------------------------------
// E[p][c][i][k] = sum over the pair's rows m of L[m][i] V[m][c][k]: a
// [NS x rows] . [rows x CORR_NC NT] product per pair as FP64 MFMA 16x16x4
// tiles (four wavefronts per pair, six 16-column tiles each).
constexpr int EMAT = CORR_NC * NS * NT;   // doubles of one pair's matrix
__global__ __launch_bounds__(256) void k_emat(int npairs, const int64_t* __restrict__ roff,
                                              const double* __restrict__ V, const double* __restrict__ L,
                                              int64_t p0, double* __restrict__ Em)
{
    const int p = blockIdx.x;
    if (p >= npairs) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, qq = lane >> 4;
    const int64_t m0 = roff[p], m1 = roff[p + 1];
    constexpr int TPW = CORR_NC * NT / 16 / 4;   // column tiles per wavefront
    v4d acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t m = m0; m < m1; m += 4) {
        const int64_t mm = m + qq;
        const bool ok = mm < m1;
        const double a = ok ? L[mm * NS + r] : 0.0;   // A = L^T: lane holds L[m + l/16][l mod 16]
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int colt = (wv * TPW + t) * 16 + r;
            const double b = ok ? V[mm * (CORR_NC * NT) + colt] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
    }
    double* E = Em + (p0 + p) * (int64_t)EMAT;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int colt = (wv * TPW + t) * 16 + r;   // column (c, k) = c * NT + k
        const int c = colt / NT, k = colt % NT;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = qq + 4 * j;
            E[(c * NS + i) * NT + k] = acc[t][j];
        }
    }
}

// corrections of the pairs from their matrices and the density's GL-circle
// Fourier coefficients (sh: a_l at 6 l + d, b_l at 6 l + 3 + d): one wavefront
// per pair, eight (row, basis function) slots per lane; the matrix is read
// once, coalesced (bandwidth bound)
__global__ __launch_bounds__(64) void k_emat_apply(int npairs, const int* __restrict__ listf,
                                                   const int* __restrict__ pe, const double* __restrict__ Em,
                                                   const double* __restrict__ sh, double* __restrict__ corr)
{
    const int w = blockIdx.x, lane = threadIdx.x;
    if (w >= npairs) return;
    const int64_t p = listf[w];
    const double* E = Em + (int64_t)w * EMAT;
    const double* she = sh + (int64_t)pe[p] * NS * NSH;
    double o[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 2
    for (int sl = lane; sl < NS * NT; sl += 64) {
        const int i = sl / NT, k = sl % NT;
        const int off = k < NT / 2 ? 6 * k : (k == NT / 2 ? 6 * (NT / 2) : 6 * (k - NT / 2) + 3);
        const double s0 = she[i * NSH + off], s1 = she[i * NSH + off + 1], s2 = she[i * NSH + off + 2];
        double e[CORR_NC];
#pragma unroll
        for (int c = 0; c < CORR_NC; ++c) e[c] = E[c * (NS * NT) + sl];
        // symmetric S (xx xy xz yy yz zz) and D blocks times (s0 s1 s2)
        o[0] += e[0] * s0 + e[1] * s1 + e[2] * s2;
        o[1] += e[1] * s0 + e[3] * s1 + e[4] * s2;
        o[2] += e[2] * s0 + e[4] * s1 + e[5] * s2;
        o[3] += e[6] * s0 + e[7] * s1 + e[8] * s2;
        o[4] += e[7] * s0 + e[9] * s1 + e[10] * s2;
        o[5] += e[8] * s0 + e[10] * s1 + e[11] * s2;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = wave_sum(o[q]);
    if (lane == 0)
        for (int q = 0; q < 6; ++q) corr[p * 6 + q] = o[q];
}

// ---------------------------------------------------------------------------
// final reduction: far chunks in order, then the pair corrections in CSR order
// ---------------------------------------------------------------------------
// Stokes: u_S = u[0..2] / (8 pi), u_D = -3 u[3..5] / (4 pi) (three components
// per target); Laplace: u_S = u[0] / (4 pi), u_D = u[3] / (4 pi) (one each).
__global__ void k_reduce(int64_t T, const int* __restrict__ tgroup, const int* __restrict__ gnchunk,
                         const double* __restrict__ part, const int64_t* __restrict__ off,
                         const int8_t* __restrict__ tier, const double* __restrict__ corr,
                         double* __restrict__ usl, double* __restrict__ udl, int ker)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double u[6] = {0, 0, 0, 0, 0, 0};
    const int nchunk = gnchunk[tgroup[t]];
    const int kstep = ker == KER_LAPLACE ? 3 : 1;   // Laplace: slots 0 and 3 only
    for (int c = 0; c < nchunk; ++c)
        for (int k = 0; k < 6; k += kstep) u[k] += part[((int64_t)c * 6 + k) * T + t];
    if (off) {
        for (int64_t p = off[t]; p < off[t + 1]; ++p) {
            if (tier[p] == TIER_SKIP) continue;
            for (int k = 0; k < 6; k += kstep) u[k] += corr[p * 6 + k];
        }
    }
    if (ker == KER_LAPLACE) {
        const double cL = 1.0 / (4.0 * PI);
        if (usl) usl[t] = cL * u[0];
        if (udl) udl[t] = cL * u[3];
        return;
    }
    const double cS = 1.0 / (8.0 * PI), cD = -3.0 / (4.0 * PI);
    for (int d = 0; d < 3; ++d) {
        if (usl) usl[t * 3 + d] = cS * u[d];
        if (udl) udl[t * 3 + d] = cD * u[3 + d];
    }
}

// scalar density (Laplace) into the first component of a 3-component array
__global__ void k_scalar_to_vec(int64_t N, const double* __restrict__ s, double* __restrict__ v)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    v[3 * n] = s[n];
    v[3 * n + 1] = 0.0;
    v[3 * n + 2] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
#define LAUNCH_CHECK()                               \
    do {                                             \
        hipError_t e_ = hipGetLastError();           \
        if (e_ != hipSuccess) return (int)e_;        \
    } while (0)

int launch_expand(hipStream_t st, int E, const double* xc, const double* eps, const double* e1, const double* sa,
                  const double* sc, const int* esign, const int* ebody, const int* egroup, double* clq, double* circ,
                  ElemInfo* info, double* ny, double* nn, double* nw, int64_t N, int closed_fb)
{
    if (closed_fb != 1 && closed_fb != 2) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_expand, dim3(E), dim3(512), 0, st, E, xc, eps, e1, sa, sc, esign, ebody, egroup, clq, circ,
                       info, ny, nn, nw, N, closed_fb);
    LAUNCH_CHECK();
    return 0;
}

int launch_expand_up(hipStream_t st, int E, int ns_f, int nt_f, const double* gx_f, const double* gw_f,
                     const double* clq, const ElemInfo* info, double* cpy, double* cpn, double* cpw, int64_t Mtot,
                     const int64_t* eoff)
{
    hipLaunchKernelGGL(k_expand_up, dim3(E, ns_f), dim3(nt_f), 0, st, E, ns_f, nt_f, gx_f, gw_f, clq, info, cpy, cpn,
                       cpw, Mtot, eoff);
    LAUNCH_CHECK();
    return 0;
}

int launch_base_build(hipStream_t st, int E, const ElemInfo* info, const int64_t* boff, const double* ny,
                      const double* nn, const double* nw, int64_t N, const double* c0y, const double* c0n,
                      const double* c0w, int64_t M0, double* by, double* bn, double* bw, int64_t Nb)
{
    hipLaunchKernelGGL(k_base_build, dim3(E), dim3(256), 0, st, E, info, boff, ny, nn, nw, N, c0y, c0n, c0w, M0, by,
                       bn, bw, Nb);
    LAUNCH_CHECK();
    return 0;
}

int launch_prep_sigma(hipStream_t st, int E, const double* sigma, const double* nw, int64_t N, double* sw,
                      double* sh, int* band, double eta, const ElemInfo* info, const double* circ, GateConsts gc,
                      double* rnear)
{
    hipLaunchKernelGGL(k_prep_sigma, dim3(E), dim3(512), 0, st, E, sigma, nw, N, sw, sh, band, eta);
    LAUNCH_CHECK();
    if (rnear) {
        hipLaunchKernelGGL(k_rnear, dim3((E + 127) / 128), dim3(128), 0, st, E, info, circ, band, gc, rnear);
        LAUNCH_CHECK();
    }
    return 0;
}

// a density whose band exceeds the one a frozen evaluation plan was built
// for (FLAG_BAND): the plan's rules were chosen for the narrower band
__global__ void k_band_check(int E, const int* __restrict__ band_new, const int* __restrict__ band_plan,
                             int* __restrict__ err)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    if (band_new[2 * e] > band_plan[2 * e] || band_new[2 * e + 1] > band_plan[2 * e + 1]) atomicOr(err, FLAG_BAND);
}

__global__ void k_fill_i32(int64_t n, int* __restrict__ v, int val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

int launch_band_check(hipStream_t st, int E, const int* band_new, const int* band_plan, int* err)
{
    hipLaunchKernelGGL(k_band_check, dim3((E + 127) / 128), dim3(128), 0, st, E, band_new, band_plan, err);
    LAUNCH_CHECK();
    return 0;
}

int launch_fill_i32(hipStream_t st, int64_t n, int* v, int val)
{
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, val);
    LAUNCH_CHECK();
    return 0;
}

int launch_sigma_up(hipStream_t st, int E, int ns_f, int nt_f, const double* sh, const double* Lup, const double* cpw,
                    double* swf, int64_t Mtot, const int64_t* eoff)
{
    hipLaunchKernelGGL(k_sigma_up, dim3(E), dim3(256), 0, st, E, ns_f, nt_f, sh, Lup, cpw, swf, Mtot, eoff);
    LAUNCH_CHECK();
    return 0;
}

int launch_sigma_base(hipStream_t st, int E, const ElemInfo* info, const int64_t* boff, const double* sw, int64_t N,
                      const double* swf0, int64_t M0, double* bsw, int64_t Nb)
{
    hipLaunchKernelGGL(k_sigma_base, dim3(E), dim3(256), 0, st, E, info, boff, sw, N, swf0, M0, bsw, Nb);
    LAUNCH_CHECK();
    return 0;
}

int launch_targets(hipStream_t st, int64_t T, const double* x, const int64_t* tnode, const int* tgrp_in, int G,
                   const ElemInfo* info, const double* ny, int64_t N, double* xt, int* tgroup, int64_t* gstart,
                   int* err)
{
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st, (int64_t)G, gstart,
                       (int64_t)-1);
    LAUNCH_CHECK();
    if (T == 0) return 0;
    const dim3 grid((unsigned)((T + 255) / 256));
    hipLaunchKernelGGL(k_targets, grid, dim3(256), 0, st, T, x, tnode, tgrp_in, G, info, ny, N, xt, tgroup, err);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_group_bounds, grid, dim3(256), 0, st, T, tgroup, gstart, err);
    LAUNCH_CHECK();
    return 0;
}

int launch_far(hipStream_t st, int64_t T, const double* xt, const double* sy, const double* sn, const double* ssw,
               int64_t N, const FarTile* tiles, int ntiles, double* part, bool mixed, double near2, int tpt, int ker,
               const FarSplit& spl)
{
    if (ntiles == 0) return 0;
    if (mixed && ker != KER_STOKES) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)ntiles), blk(FAR_BLOCK);
#define CSBQ_FAR(K)                                                                                                 \
    if (mixed)                                                                                                      \
        hipLaunchKernelGGL(k_far_mx<K>, grid, blk, 0, st, T, xt, sy, sn, ssw, N, tiles, near2, part, spl);         \
    else if (ker == KER_LAPLACE)                                                                                    \
        hipLaunchKernelGGL((k_far<K, KER_LAPLACE>), grid, blk, 0, st, T, xt, sy, sn, ssw, N, tiles, part, spl);     \
    else                                                                                                            \
        hipLaunchKernelGGL((k_far<K, KER_STOKES>), grid, blk, 0, st, T, xt, sy, sn, ssw, N, tiles, part, spl);
    switch (tpt) {
    case 1: CSBQ_FAR(1) break;
    case 2: CSBQ_FAR(2) break;
    case 4: CSBQ_FAR(4) break;
    default: return (int)hipErrorInvalidValue;
    }
#undef CSBQ_FAR
    LAUNCH_CHECK();
    return 0;
}

int launch_search(hipStream_t st, int64_t T, const int* tgroup, const int* gel, const double* xt,
                  const int64_t* tnode, const ElemInfo* info, const double* rnear, const int64_t* off, int* cnt,
                  int* pe, int* pt)
{
    if (T == 0) return 0;
    hipLaunchKernelGGL(k_search, dim3((unsigned)((T + 127) / 128)), dim3(128), 0, st, T, tgroup, gel, xt, tnode,
                       info, rnear, off, cnt, pe, pt);
    LAUNCH_CHECK();
    return 0;
}

int launch_grid_circles(hipStream_t st, int E, const double* clq, double* grid)
{
    if (E == 0) return 0;
    hipLaunchKernelGGL(k_grid_circles, dim3(E), dim3(NCIRC * CGRID), 0, st, E, clq, grid);
    LAUNCH_CHECK();
    return 0;
}

int launch_classify(hipStream_t st, int64_t P, const int* perm, const int* pe, const int* pt, const double* xt,
                    int64_t T, const int64_t* tnode, const double* clq, const double* circ, const double* grid,
                    const ElemInfo* info, const double* tor, const int* band, GateConsts gc, int8_t* tier, double* cls)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)((P + 127) / 128)), dim3(128), 0, st, P, perm, pe, pt, xt, T, tnode,
                       clq, circ, grid, info, tor, band, gc, tier, cls);
    LAUNCH_CHECK();
    return 0;
}

int launch_iota(hipStream_t st, int64_t P, int* v)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, v);
    LAUNCH_CHECK();
    return 0;
}

int launch_tier_keys(hipStream_t st, int64_t P, int E, const int8_t* tier, const int* pe, int* key, int* val)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_tier_keys, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, E, tier, pe, key, val);
    LAUNCH_CHECK();
    return 0;
}

int launch_corr_up(hipStream_t st, const UpRules& ur, int nwaves, const int* ws, const int* sorted, const int* pt,
                   const double* xt, int64_t T, const ElemInfo* info, const int64_t* boff, const double* by,
                   const double* bn, const double* bsw, int64_t Nb, double* corr, int ker)
{
    if (nwaves == 0) return 0;
    if (ker == KER_LAPLACE)
        hipLaunchKernelGGL(k_corr_up<KER_LAPLACE>, dim3(nwaves), dim3(64), 0, st, ur, ws, sorted, pt, xt, T, info, boff,
                           by, bn, bsw, Nb, corr);
    else
        hipLaunchKernelGGL(k_corr_up<KER_STOKES>, dim3(nwaves), dim3(64), 0, st, ur, ws, sorted, pt, xt, T, info, boff,
                           by, bn, bsw, Nb, corr);
    LAUNCH_CHECK();
    return 0;
}

int launch_corr_full(hipStream_t st, int nfull, const int* listf, const int* pe, const int* pt, const double* xt,
                     int64_t T, const int64_t* tnode, const double* clq, const double* sh, const ElemInfo* info,
                     const int* band, const double* cls, const int64_t* boff, const double* by, const double* bn,
                     const double* bsw, int64_t Nb, const RuleArgs& ra, GateConsts gc, double* corr, int* err,
                     int* work, int mt_max, int ker, int mode, const MatrixRows* mr)
{
    if (nfull == 0) return 0;
    if (mt_max < 0 || mt_max >= NMODE) return (int)hipErrorInvalidValue;
    if (mode != MODE_DENSITY && (ker != KER_STOKES || !mr)) return (int)hipErrorInvalidValue;
    if (ra.wnb < 0 || ((ra.wnb > 0 || ra.wsph >= 0) && (!ra.woff || !ra.wd || !ra.ww)))
        return (int)hipErrorInvalidValue;
    RuleTables rt{ra.roff, ra.rth, ra.rw, ra.rcs, ra.rsn, ra.romc, ra.nb, ra.lx, ra.lw, ra.nl,
                  ra.woff, ra.wd, ra.ww, ra.wb_lo, ra.wnb, ra.wl0, ra.wsph, ra.wany};
    const int cstride = 6 * (mt_max + 1);
    // at least the phase-1 weights and centerline quantities (and the stack)
    const size_t lds = (size_t)SB * (cstride > NS + QVS ? cstride : NS + QVS) * sizeof(double);
    MatrixOut mo{};
    if (mr) mo = MatrixOut{mr->roff, mr->V, mr->L, mr->count, mr->lup0, mr->bw};
    if (ker == KER_LAPLACE)
        hipLaunchKernelGGL((k_corr_full<KER_LAPLACE, MODE_DENSITY>), dim3(nfull), dim3(64), lds, st, listf, pe, pt, xt,
                           T, tnode, clq, sh, info, band, cls, boff, by, bn, bsw, Nb, rt, gc, corr, err, work, cstride,
                           mo);
    else if (mode == MODE_COUNT)
        hipLaunchKernelGGL((k_corr_full<KER_STOKES, MODE_COUNT>), dim3(nfull), dim3(64), lds, st, listf, pe, pt, xt,
                           T, tnode, clq, sh, info, band, cls, boff, by, bn, bsw, Nb, rt, gc, corr, err, work, cstride,
                           mo);
    else if (mode == MODE_MATRIX)
        hipLaunchKernelGGL((k_corr_full<KER_STOKES, MODE_MATRIX>), dim3(nfull), dim3(64), lds, st, listf, pe, pt, xt,
                           T, tnode, clq, sh, info, band, cls, boff, by, bn, bsw, Nb, rt, gc, corr, err, work, cstride,
                           mo);
    else
        hipLaunchKernelGGL((k_corr_full<KER_STOKES, MODE_DENSITY>), dim3(nfull), dim3(64), lds, st, listf, pe, pt, xt,
                           T, tnode, clq, sh, info, band, cls, boff, by, bn, bsw, Nb, rt, gc, corr, err, work, cstride,
                           mo);
    LAUNCH_CHECK();
    return 0;
}

int launch_reduce(hipStream_t st, int64_t T, const int* tgroup, const int* gnchunk, const double* part,
                  const int64_t* off, const int8_t* tier, const double* corr, double* usl, double* udl, int ker)
{
    if (T == 0) return 0;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, T, tgroup, gnchunk, part, off,
                       tier, corr, usl, udl, ker);
    LAUNCH_CHECK();
    return 0;
}

int launch_emat(hipStream_t st, int npairs, const int64_t* roff, const double* V, const double* L, int64_t p0,
                double* Em)
{
    if (npairs == 0) return 0;
    hipLaunchKernelGGL(k_emat, dim3(npairs), dim3(256), 0, st, npairs, roff, V, L, p0, Em);
    LAUNCH_CHECK();
    return 0;
}

int launch_emat_apply(hipStream_t st, int npairs, const int* listf, const int* pe, const double* Em, const double* sh,
                      double* corr)
{
    if (npairs == 0) return 0;
    hipLaunchKernelGGL(k_emat_apply, dim3(npairs), dim3(64), 0, st, npairs, listf, pe, Em, sh, corr);
    LAUNCH_CHECK();
    return 0;
}

int launch_scalar_to_vec(hipStream_t st, int64_t N, const double* s, double* v)
{
    if (N == 0) return 0;
    hipLaunchKernelGGL(k_scalar_to_vec, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, s, v);
    LAUNCH_CHECK();
    return 0;
}


// ---------------------------------------------------------------------------
// allocation-free smooth sum: scratch in a static device array
// ---------------------------------------------------------------------------
// One copy per device, zero-initialised when the code object loads and held
// until the process ends.  Host code never passes this name to a kernel: the
// device address comes from scratch_address().
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

int scratch_address(int device, void** out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return (int)e;
        if (cur != device) return (int)hipErrorInvalidDevice;   // the caller makes `device` current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return 0;
}

// Block list of a single-geometry smooth sum (target block a = i / nch, source
// chunk c = i % nch, so consecutive blocks -- one per XCD -- take consecutive
// chunks), the group's chunk count and a cleared flag word.
__global__ void k_noalloc_setup(int ntiles, int nch, int64_t T, int64_t N, int tb, int64_t chunk,
                                FarTile* __restrict__ tiles, int* __restrict__ gnchunk, int* __restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        gnchunk[0] = nch;
        err[0] = 0;
    }
    if (i >= ntiles) return;
    const int a = i / nch, c = i - a * nch;
    const int64_t t0 = (int64_t)a * tb, s0 = (int64_t)c * chunk;
    FarTile f;
    f.t0 = t0;
    f.s0 = s0;
    f.tn = (int32_t)min((int64_t)tb, T - t0);
    f.sn = (int32_t)min(chunk, N - s0);
    f.chunk = c;
    f.e0 = f.e1 = 0;   // a plain source range
    f.pad_ = 0;
    tiles[i] = f;
}

int launch_noalloc_setup(hipStream_t st, int ntiles, int nch, int64_t T, int64_t N, int tb, int64_t chunk,
                         FarTile* tiles, int* gnchunk, int* err)
{
    hipLaunchKernelGGL(k_noalloc_setup, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, ntiles, nch, T, N,
                       tb, chunk, tiles, gnchunk, err);
    LAUNCH_CHECK();
    return 0;
}

}  // namespace csbq
