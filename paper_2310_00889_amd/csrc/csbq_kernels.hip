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
//   k_corr_up       tier x2/x4: upsampled rule minus the smooth rule
//   k_corr_full     special quadrature (Sections 3.2.2-3.2.4) minus the
//                   smooth rule, one wavefront per pair
//   k_reduce        far sum + corrections in a fixed order per target
#include <hip/hip_runtime.h>

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
    return 0;
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    h = x * y;
    e = fma(-h, y, 1.0);
    return fma(0.5 * y, e, y);
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

// position/tangent/radius only (for distance searches)
__device__ inline void circle_at_x(const double* __restrict__ clq, double x, double* X, double* t, double* E)
{
    double l[NS];
    bary_weights(x, c_gx, c_lam, l);
    double xp[3];
    for (int d = 0; d < 3; ++d) {
        double v = 0.0, vp = 0.0;
        for (int i = 0; i < NS; ++i) {
            v += l[i] * clq[(Q_X + d) * NS + i];
            vp += l[i] * clq[(Q_XP + d) * NS + i];
        }
        X[d] = v;
        xp[d] = vp;
    }
    double e = 0.0;
    for (int i = 0; i < NS; ++i) e += l[i] * clq[Q_E * NS + i];
    *E = e;
    double is = 1.0 / sqrt(dot3(xp, xp));
    for (int d = 0; d < 3; ++d) t[d] = xp[d] * is;
}

__device__ inline void circle_dist(const double* X, const double* t, double E, const double* x, double* d2, double* cha)
{
    double v[3] = {x[0] - X[0], x[1] - X[1], x[2] - X[2]};
    double z = dot3(v, t);
    double r2 = fmax(0.0, dot3(v, v) - z * z);
    double rho = sqrt(r2);
    double dr = rho - E;
    *d2 = dr * dr + z * z;
    *cha = rho > 0.0 ? *d2 / (2.0 * rho * E) : 1e300;
}

// ---------------------------------------------------------------------------
// geometry expansion (Section 3.1, Section 3.2.1 weights)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_expand(int E, const double* __restrict__ xc, const double* __restrict__ eps,
                                                const double* __restrict__ e1, const double* __restrict__ sa,
                                                const double* __restrict__ sc, const int* __restrict__ esign,
                                                const int* __restrict__ ebody, double* __restrict__ clq,
                                                double* __restrict__ circ, ElemInfo* __restrict__ info,
                                                double* __restrict__ ny, double* __restrict__ nn,
                                                double* __restrict__ nw, int64_t N)
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
        info[e] = inf;
    }
}

// Upsampled tensor rule of tier factor f: f sub-panels of NS GL nodes in s,
// f*NT uniform angles.  Block = one s-row (f*NT threads), grid = (E, f*NS).
// Points of element e start at e*Mf (Mf = f^2 NPE + NPE; the last NPE slots
// hold the element's own nodes, filled by k_cp_nodes).
__global__ __launch_bounds__(128) void k_expand_up(int E, int f, const double* __restrict__ clq,
                                                   const ElemInfo* __restrict__ info, double* __restrict__ cpy,
                                                   double* __restrict__ cpn, double* __restrict__ cpw,
                                                   int64_t Mtot)
{
    const int e = blockIdx.x, p = blockIdx.y, q = threadIdx.x;
    const int ntf = f * NT;
    const int64_t Mf = (int64_t)f * f * NPE + NPE;
    const ElemInfo inf = info[e];
    const int k = p / NS, g = p % NS;
    // normalised position of GL node g of sub-panel k in [-1,1]
    const double xn = -1.0 + (2.0 * k + 1.0 + c_gx[g]) / f;
    Frame fr;
    frame_at_x(clq + (int64_t)e * CLQ * NS, xn, fr);
    double th = 2.0 * PI * q / ntf;
    double st, ct;
    sincos(th, &st, &ct);
    double y[3], ys[3], yt[3], jn[3];
    surface_at(fr, ct, st, y, ys, yt);
    cross3(yt, ys, jn);
    double J = sqrt(dot3(jn, jn));
    const int64_t m = (int64_t)e * Mf + (int64_t)p * ntf + q;
    for (int d = 0; d < 3; ++d) {
        cpy[d * Mtot + m] = y[d];
        cpn[d * Mtot + m] = inf.sign * jn[d] / J;
    }
    cpw[m] = J * c_gw[g] * (0.5 * (inf.c - inf.a) / f) * (2.0 * PI / ntf);
}

__global__ void k_cp_nodes(int E, int f, const double* __restrict__ ny, const double* __restrict__ nn,
                           const double* __restrict__ nw, int64_t N, double* __restrict__ cpy,
                           double* __restrict__ cpn, double* __restrict__ cpw, int64_t Mtot)
{
    const int64_t Mf = (int64_t)f * f * NPE + NPE;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)E * NPE) return;
    int64_t e = idx / NPE, r = idx % NPE;
    int64_t m = e * Mf + (int64_t)f * f * NPE + r;
    for (int d = 0; d < 3; ++d) {
        cpy[d * Mtot + m] = ny[d * N + idx];
        cpn[d * Mtot + m] = nn[d * N + idx];
    }
    cpw[m] = -nw[idx];
}

// ---------------------------------------------------------------------------
// density preparation
// ---------------------------------------------------------------------------
// sigma*w (SoA), Fourier coefficients on each GL circle sh[e][i][l][6], and the
// band limits (highest Legendre degree Ms and Fourier mode Mt above eta).
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
        band[2 * e] = Ms;
        band[2 * e + 1] = Mt;
    }
}

// density times weight on the upsampled rule of factor f (and -sigma*w on the
// element's own nodes): sigma(s_p, t_q) from the GL-circle Fourier
// coefficients interpolated to s_p and synthesised at t_q.
__global__ __launch_bounds__(256) void k_sigma_up(int E, int f, const double* __restrict__ sh,
                                                  const double* __restrict__ Lup, const double* __restrict__ cpw,
                                                  const double* __restrict__ sw, int64_t N,
                                                  double* __restrict__ swf, int64_t Mtot)
{
    const int e = blockIdx.x, tid = threadIdx.x;
    const int ntf = f * NT;
    const int64_t Mf = (int64_t)f * f * NPE + NPE;
    __shared__ double shl[NS * NSH];
    __shared__ double A[NS * NSH];
    for (int o = tid; o < NS * NSH; o += blockDim.x) shl[o] = sh[(int64_t)e * NS * NSH + o];
    __syncthreads();
    for (int rb = 0; rb < f; ++rb) {
        // coefficients at the 16 s-points of sub-panel rb
        for (int o = tid; o < NS * NSH; o += blockDim.x) {
            int r = o / NSH, k = o % NSH;
            int p = rb * NS + r;
            double v = 0.0;
            for (int ii = 0; ii < NS; ++ii) v += Lup[p * NS + ii] * shl[ii * NSH + k];
            A[o] = v;
        }
        __syncthreads();
        for (int o = tid; o < NS * ntf; o += blockDim.x) {
            int r = o / ntf, q = o % ntf;
            double th = 2.0 * PI * q / ntf;
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
            int64_t m = (int64_t)e * Mf + (int64_t)(rb * NS + r) * ntf + q;
            double w = cpw[m];
            swf[0 * Mtot + m] = v0 * w;
            swf[1 * Mtot + m] = v1 * w;
            swf[2 * Mtot + m] = v2 * w;
        }
        __syncthreads();
    }
    for (int r = tid; r < NPE; r += blockDim.x) {
        int64_t m = (int64_t)e * Mf + (int64_t)f * f * NPE + r;
        int64_t n = (int64_t)e * NPE + r;
        for (int d = 0; d < 3; ++d) swf[d * Mtot + m] = -sw[d * N + n];
    }
}

// ---------------------------------------------------------------------------
// targets
// ---------------------------------------------------------------------------
__global__ void k_targets(int64_t T, const double* __restrict__ x, const int64_t* __restrict__ tnode,
                          const double* __restrict__ ny, int64_t N, double* __restrict__ xt,
                          int* __restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    int64_t nd = tnode ? tnode[t] : -1;
    if (nd >= N) {
        atomicOr(err, 1);
        nd = -1;
    }
    for (int d = 0; d < 3; ++d) {
        double v = (nd >= 0) ? ny[d * N + nd] : (x ? x[t * 3 + d] : 0.0);
        xt[d * T + t] = v;
    }
}

// ---------------------------------------------------------------------------
// smooth Nystrom sum (Section 3.2.1): targets x sources, sources staged in LDS
// ---------------------------------------------------------------------------
constexpr int FAR_BLOCK = 256;

__global__ __launch_bounds__(FAR_BLOCK) void k_far(int64_t T, const double* __restrict__ xt,
                                                   const double* __restrict__ sy, const double* __restrict__ sn,
                                                   const double* __restrict__ ssw, int64_t N, int64_t chunk,
                                                   double* __restrict__ part)
{
    __shared__ double ly[3][FAR_BLOCK], ln_[3][FAR_BLOCK], ls[3][FAR_BLOCK];
    const int tid = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * FAR_BLOCK + tid;
    const bool ok = t < T;
    double x0 = 0, x1 = 0, x2 = 0;
    if (ok) {
        x0 = xt[t];
        x1 = xt[T + t];
        x2 = xt[2 * T + t];
    }
    double s0 = 0, s1 = 0, s2 = 0, d0 = 0, d1 = 0, d2 = 0;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = min(N, c0 + chunk);
    for (int64_t base = c0; base < c1; base += FAR_BLOCK) {
        const int64_t k = base + tid;
        if (k < c1) {
            ly[0][tid] = sy[k];
            ly[1][tid] = sy[N + k];
            ly[2][tid] = sy[2 * N + k];
            ln_[0][tid] = sn[k];
            ln_[1][tid] = sn[N + k];
            ln_[2][tid] = sn[2 * N + k];
            ls[0][tid] = ssw[k];
            ls[1][tid] = ssw[N + k];
            ls[2][tid] = ssw[2 * N + k];
        }
        __syncthreads();
        const int nin = (int)min((int64_t)FAR_BLOCK, c1 - base);
#pragma unroll 4
        for (int kk = 0; kk < nin; ++kk) {
            double r0 = x0 - ly[0][kk], r1 = x1 - ly[1][kk], r2 = x2 - ly[2][kk];
            double rr = fma(r0, r0, fma(r1, r1, r2 * r2));
            double ir = rr > 0.0 ? rsqrt_nr(rr) : 0.0;
            double w0 = ls[0][kk], w1 = ls[1][kk], w2 = ls[2][kk];
            double rs = fma(r0, w0, fma(r1, w1, r2 * w2));
            double rn = fma(r0, ln_[0][kk], fma(r1, ln_[1][kk], r2 * ln_[2][kk]));
            double ir2 = ir * ir;
            double b = rs * ir * ir2;
            double cD = rn * rs * ir2 * ir2 * ir;
            s0 = fma(ir, w0, fma(b, r0, s0));
            s1 = fma(ir, w1, fma(b, r1, s1));
            s2 = fma(ir, w2, fma(b, r2, s2));
            d0 = fma(cD, r0, d0);
            d1 = fma(cD, r1, d1);
            d2 = fma(cD, r2, d2);
        }
        __syncthreads();
    }
    if (ok) {
        double* p = part + (int64_t)blockIdx.y * 6 * T;
        p[0 * T + t] = s0;
        p[1 * T + t] = s1;
        p[2 * T + t] = s2;
        p[3 * T + t] = d0;
        p[4 * T + t] = d1;
        p[5 * T + t] = d2;
    }
}

// ---------------------------------------------------------------------------
// near-pair search (candidates) and classification
// ---------------------------------------------------------------------------
__global__ void k_search(int64_t T, int E, const double* __restrict__ xt, const int64_t* __restrict__ tnode,
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
    for (int e = 0; e < E; ++e) {
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

// golden-section minimisation of a distance-like function of s over [lo, hi]
template <typename F>
__device__ inline double golden_min(F fn, double lo, double hi, int iters, double* fmin_out)
{
    const double gr = 0.6180339887498949;
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = fn(x1), f2 = fn(x2);
    for (int it = 0; it < iters; ++it) {
        if (f1 < f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - gr * (hi - lo);
            f1 = fn(x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + gr * (hi - lo);
            f2 = fn(x2);
        }
    }
    double fl = fn(lo), fh = fn(hi);
    double best = x1, fb = f1;
    if (f2 < fb) { best = x2; fb = f2; }
    if (fl < fb) { best = lo; fb = fl; }
    if (fh < fb) { best = hi; fb = fh; }
    *fmin_out = fb;
    return best;
}

// worst Bernstein parameter of s* = sr + i si over f equal sub-panels of [a,c]
__device__ inline double rho_subpanels(double sr, double si, double a, double c, int f)
{
    double h = (c - a) / f;
    double best = 1e300;
    for (int k = 0; k < f; ++k) best = fmin(best, bernstein_rho(sr, si, a + k * h, a + (k + 1) * h));
    return best;
}

__global__ void k_classify(int64_t P, const int* __restrict__ pe, const int* __restrict__ pt,
                           const double* __restrict__ xt, int64_t T, const int64_t* __restrict__ tnode,
                           const double* __restrict__ clq, const double* __restrict__ circ,
                           const ElemInfo* __restrict__ info, const int* __restrict__ band, GateConsts gc,
                           int8_t* __restrict__ tier, double* __restrict__ cls)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
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
    auto xn_of = [&](int k) { return k == 0 ? -1.0 : (k == NCIRC - 1 ? 1.0 : c_gx[k - 1]); };
    auto fd = [&](double xn) {
        double X[3], tt[3], EE, d2, cha;
        circle_at_x(cq, xn, X, tt, &EE);
        circle_dist(X, tt, EE, x, &d2, &cha);
        return d2;
    };
    auto fa = [&](double xn) {
        double X[3], tt[3], EE, d2, cha;
        circle_at_x(cq, xn, X, tt, &EE);
        circle_dist(X, tt, EE, x, &d2, &cha);
        return cha;
    };
    double d2c, chac;
    double xd = golden_min(fd, xn_of(max(kd - 1, 0)), xn_of(min(kd + 1, NCIRC - 1)), 40, &d2c);
    golden_min(fa, xn_of(max(ka - 1, 0)), xn_of(min(ka + 1, NCIRC - 1)), 40, &chac);
    d2c = fmin(d2c, bd);
    chac = fmin(chac, ba);
    const double sc_ = 0.5 * (inf.a + inf.c) + 0.5 * (inf.c - inf.a) * xd;
    // speed bound at the closest circle (interpolated between neighbouring circles' bounds)
    double spd = fmax(cc[kd * CIRQ + 7], cc[min(kd + 1, NCIRC - 1) * CIRQ + 7]);
    spd = fmax(spd, cc[max(kd - 1, 0) * CIRQ + 7]);
    const double dc = sqrt(d2c);
    const double ac = acosh1p(chac);
    cp[0] = sc_;
    cp[1] = dc;
    cp[2] = spd;
    cp[3] = ac;
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    int8_t tr = TIER_FULL;
    const int facs[3] = {1, 2, 4};
    for (int fi = 0; fi < 3; ++fi) {
        int f = facs[fi];
        double rho = rho_subpanels(sc_, dc / spd, inf.a, inf.c, f);
        double es = gc.cs * pow(rho, -(double)(2 * NS - Ms));
        double et = gc.ct * exp(-(double)(f * NT - Mt - gc.extra_modes) * ac);
        if (es <= gc.tol && et <= gc.tol) {
            tr = (f == 1) ? TIER_SKIP : (f == 2 ? TIER_UP2 : TIER_UP4);
            break;
        }
    }
    tier[p] = tr;
}

// near-region radius of each element from its band limits (candidate filter)
__global__ void k_rnear(int E, const ElemInfo* __restrict__ info, const int* __restrict__ band, GateConsts gc,
                        double* __restrict__ rnear)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const ElemInfo inf = info[e];
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    double areq = log(gc.ct / gc.tol) / (double)(NT - Mt - gc.extra_modes);
    double dth = inf.eps_max * (exp(areq) - 1.0);
    double rreq = pow(gc.cs / gc.tol, 1.0 / (double)(2 * NS - Ms));
    double h = 0.5 * (inf.c - inf.a);
    double ds = inf.smax * h * 0.5 * (rreq - 1.0 / rreq);
    rnear[e] = 1.05 * fmax(dth, ds) + 1e-12;
}

// ---------------------------------------------------------------------------
// correction buckets
// ---------------------------------------------------------------------------
__global__ void k_bucket_count(int64_t P, const int8_t* __restrict__ tier, const int* __restrict__ pe,
                               int* __restrict__ cnt2, int* __restrict__ cnt4, int* __restrict__ nfull)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int8_t tr = tier[p];
    if (tr == TIER_UP2) atomicAdd(cnt2 + pe[p], 1);
    if (tr == TIER_UP4) atomicAdd(cnt4 + pe[p], 1);
    if (tr == TIER_FULL) atomicAdd(nfull, 1);
}

__global__ void k_bucket_fill(int64_t P, const int8_t* __restrict__ tier, const int* __restrict__ pe,
                              int* __restrict__ cur2, int* __restrict__ cur4, int* __restrict__ curf,
                              int64_t* __restrict__ list2, int64_t* __restrict__ list4, int64_t* __restrict__ listf)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int8_t tr = tier[p];
    if (tr == TIER_UP2) list2[atomicAdd(cur2 + pe[p], 1)] = p;
    if (tr == TIER_UP4) list4[atomicAdd(cur4 + pe[p], 1)] = p;
    if (tr == TIER_FULL) listf[atomicAdd(curf, 1)] = p;
}

// ---------------------------------------------------------------------------
// tier x2 / x4: upsampled rule minus smooth rule, one wavefront per 64 pairs
// of one element; the element's correction points are staged in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_corr_up(int f, const int* __restrict__ wave_elem,
                                                const int64_t* __restrict__ list, const int* __restrict__ pt,
                                                const double* __restrict__ xt, int64_t T,
                                                const double* __restrict__ cpy, const double* __restrict__ cpn,
                                                const double* __restrict__ swf, int64_t Mtot,
                                                double* __restrict__ corr)
{
    __shared__ double ly[3][64], ln_[3][64], ls[3][64];
    const int w = blockIdx.x, lane = threadIdx.x;
    const int e = wave_elem[w];
    const int64_t p = list[(int64_t)w * 64 + lane];
    const int64_t Mf = (int64_t)f * f * NPE + NPE;
    double x0 = 0, x1 = 0, x2 = 0;
    if (p >= 0) {
        int64_t t = pt[p];
        x0 = xt[t];
        x1 = xt[T + t];
        x2 = xt[2 * T + t];
    }
    double s0 = 0, s1 = 0, s2 = 0, d0 = 0, d1 = 0, d2 = 0;
    const int64_t base0 = (int64_t)e * Mf;
    for (int64_t base = 0; base < Mf; base += 64) {
        int64_t m = base0 + base + lane;
        ly[0][lane] = cpy[m];
        ly[1][lane] = cpy[Mtot + m];
        ly[2][lane] = cpy[2 * Mtot + m];
        ln_[0][lane] = cpn[m];
        ln_[1][lane] = cpn[Mtot + m];
        ln_[2][lane] = cpn[2 * Mtot + m];
        ls[0][lane] = swf[m];
        ls[1][lane] = swf[Mtot + m];
        ls[2][lane] = swf[2 * Mtot + m];
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 64; ++kk) {
            double r0 = x0 - ly[0][kk], r1 = x1 - ly[1][kk], r2 = x2 - ly[2][kk];
            double rr = fma(r0, r0, fma(r1, r1, r2 * r2));
            double ir = rr > 0.0 ? rsqrt_nr(rr) : 0.0;
            double w0 = ls[0][kk], w1 = ls[1][kk], w2 = ls[2][kk];
            double rs = fma(r0, w0, fma(r1, w1, r2 * w2));
            double rn = fma(r0, ln_[0][kk], fma(r1, ln_[1][kk], r2 * ln_[2][kk]));
            double ir2 = ir * ir;
            double b = rs * ir * ir2;
            double cD = rn * rs * ir2 * ir2 * ir;
            s0 = fma(ir, w0, fma(b, r0, s0));
            s1 = fma(ir, w1, fma(b, r1, s1));
            s2 = fma(ir, w2, fma(b, r2, s2));
            d0 = fma(cD, r0, d0);
            d1 = fma(cD, r1, d1);
            d2 = fma(cD, r2, d2);
        }
        __syncthreads();
    }
    if (p >= 0) {
        double* o = corr + p * 6;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
        o[3] = d0;
        o[4] = d1;
        o[5] = d2;
    }
}

// ---------------------------------------------------------------------------
// special quadrature (Sections 3.2.2-3.2.4), one wavefront per pair
// ---------------------------------------------------------------------------
struct RuleTables {
    const int* off;       // [nb+1] offsets of the theta-rules (bracket b at index b-1)
    const double* th;     // nodes
    const double* w;      // weights
    int nb;
    const double* lx;     // log rule nodes on (0,1), singular at 0
    const double* lw;
    int nl;
};

__global__ __launch_bounds__(64) void k_corr_full(const int64_t* __restrict__ listf, const int* __restrict__ pe,
                                                  const int* __restrict__ pt, const double* __restrict__ xt,
                                                  int64_t T, const int64_t* __restrict__ tnode,
                                                  const double* __restrict__ clq, const double* __restrict__ sh,
                                                  const ElemInfo* __restrict__ info, const int* __restrict__ band,
                                                  const double* __restrict__ cls, const double* __restrict__ ny,
                                                  const double* __restrict__ nn, const double* __restrict__ sw,
                                                  int64_t N, RuleTables rt, GateConsts gc,
                                                  double* __restrict__ corr, int* __restrict__ err,
                                                  int* __restrict__ work)
{
    __shared__ double sq[CLQ * NS];
    __shared__ double shl[NS * NSH];
    __shared__ double sub_lo[MAXSUB], sub_hi[MAXSUB];
    __shared__ int sub_ty[MAXSUB];
    __shared__ int nsub;
    __shared__ double lw_[NS];
    __shared__ double qi[CLQ];
    __shared__ double dqi[CLQ];
    __shared__ double si[NSH];
    __shared__ double red[64];
    const int lane = threadIdx.x;
    const int64_t p = listf[blockIdx.x];
    const int e = pe[p];
    const int64_t t = pt[p];
    const ElemInfo inf = info[e];
    const double x[3] = {xt[t], xt[T + t], xt[2 * T + t]};
    for (int o = lane; o < CLQ * NS; o += 64) sq[o] = clq[(int64_t)e * CLQ * NS + o];
    for (int o = lane; o < NS * NSH; o += 64) shl[o] = sh[(int64_t)e * NS * NSH + o];
    const int64_t nd = tnode ? tnode[t] : -1;
    const bool own = nd >= 0 && nd / NPE == e;
    const int Ms = band[2 * e], Mt = band[2 * e + 1];
    __syncthreads();
    // on-surface target: its node (i0, j0), the node's frame and radial direction
    int i0 = 0;
    double s0 = 0.0;
    Frame f0;
    double bn[3] = {0, 0, 0};
    if (own) {
        i0 = (int)((nd % NPE) / NT);
        const int j0 = (int)(nd % NT);
        s0 = 0.5 * (inf.a + inf.c) + 0.5 * (inf.c - inf.a) * c_gx[i0];
        double q0[CLQ];
        for (int k = 0; k < CLQ; ++k) q0[k] = sq[k * NS + i0];
        frame_from_q(q0, f0);
        for (int d = 0; d < 3; ++d) bn[d] = f0.e1[d] * c_cos[j0] + f0.e2[d] * c_sin[j0];
    }
    // ---- s-rule: list of sub-panels (lane 0)
    if (lane == 0) {
        int ns_ = 0;
        const double a = inf.a, c = inf.c;
        if (own) {
            // dyadic refinement toward s0 down to ~eps/speed, log-singular
            // panels on both sides of s0 (Section 3.2.4, general form)
            const int i0 = (int)((nd % NPE) / NT);
            const double s0 = 0.5 * (a + c) + 0.5 * (c - a) * c_gx[i0];
            const double hmin = gc.hmin_fac * sq[Q_E * NS + i0] / cls[p * 4 + 2];
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
            // near region (Section 3.2.3): Bernstein parameter of s* = s_c + i d/speed
            const double sr = cls[p * 4 + 0], si_ = cls[p * 4 + 1] / cls[p * 4 + 2];
            const double expo = (double)(2 * NS - Ms);
            double st_lo[48], st_hi[48];
            int sp = 0;
            st_lo[sp] = a;
            st_hi[sp] = c;
            ++sp;
            while (sp > 0) {
                --sp;
                double lo = st_lo[sp], hi = st_hi[sp];
                double rho = bernstein_rho(sr, si_, lo, hi);
                bool ok = gc.cs * pow(rho, -expo) <= gc.tol;
                if (ok || (hi - lo) < 1e-12 * (c - a) || sp + 2 > 48 || ns_ + sp + 2 > MAXSUB) {
                    if (!ok) atomicOr(err, 2);
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
        nsub = ns_;
    }
    __syncthreads();
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int nsb = nsub;
    int n_theta = 0, n_snode = 0;
    for (int sb = 0; sb < nsb; ++sb) {
        const double lo = sub_lo[sb], hi = sub_hi[sb];
        const int ty = sub_ty[sb];
        const int nnod = (ty == SUB_GL) ? NS : rt.nl;
        for (int m = 0; m < nnod; ++m) {
            double s, ws, u;
            if (ty == SUB_GL) {
                s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * c_gx[m];
                ws = 0.5 * (hi - lo) * c_gw[m];
                u = s - s0;
            } else if (ty == SUB_LOG_LO) {
                u = (hi - lo) * rt.lx[m];
                s = lo + u;
                ws = (hi - lo) * rt.lw[m];
            } else {
                u = -(hi - lo) * rt.lx[m];
                s = hi + u;
                ws = (hi - lo) * rt.lw[m];
            }
            const double xn = (2.0 * s - inf.a - inf.c) / (inf.c - inf.a);
            // interpolation weights, centerline quantities and density coefficients at s
            if (lane == 0) {
                if (own)
                    bary_weights_rel(i0, 2.0 * u / (inf.c - inf.a), c_gx, c_lam, lw_);
                else
                    bary_weights(xn, c_gx, c_lam, lw_);
            }
            __syncthreads();
            if (lane < CLQ) {
                if (own) {
                    const double q0 = sq[lane * NS + i0];
                    double v = 0.0;
                    for (int i = 0; i < NS; ++i) v += lw_[i] * (sq[lane * NS + i] - q0);
                    dqi[lane] = v;
                    qi[lane] = q0 + v;
                } else {
                    double v = 0.0;
                    for (int i = 0; i < NS; ++i) v += lw_[i] * sq[lane * NS + i];
                    qi[lane] = v;
                }
            }
            for (int k = lane; k < NSH; k += 64) {
                double v = 0.0;
                for (int i = 0; i < NS; ++i) v += lw_[i] * shl[i * NSH + k];
                si[k] = v;
            }
            __syncthreads();
            Frame fr;
            frame_from_q(qi, fr);
            CircleLocal cl;
            if (own)
                circle_local_rel(fr, f0, bn, dqi, cl);
            else
                circle_local(fr, x, cl);
            // theta-rule for this circle (Section 3.2.2): trapezoid of nt, 2nt or
            // 4nt points if the estimate allows, else the bracket's Chebyshev rule
            const double a_ = acosh1p(cl.cha);
            int ntr = 0;
            for (int f = 1; f <= 4; f *= 2) {
                if (gc.ct * exp(-(double)(f * NT - Mt - gc.extra_modes) * a_) <= gc.tol) {
                    ntr = f * NT;
                    break;
                }
            }
            int rb = 0;
            double th0 = 0.0;
            if (ntr == 0) {
                double alpha = sqrt(cl.d2) / fr.E;
                int b = (alpha > 0.0) ? (int)floor(-log2(alpha)) + 1 : rt.nb;
                if (b < 1) {
                    ntr = 4 * NT;
                } else {
                    if (b > rt.nb) {
                        b = rt.nb;
                        atomicOr(err, 4);
                    }
                    rb = b;
                }
            }
            // angle of the closest circle point
            {
                double c1 = dot3(cl.b0, fr.e1), s1 = dot3(cl.b0, fr.e2);
                th0 = atan2(s1, c1);
            }
            const int nq = ntr ? ntr : (rt.off[rb] - rt.off[rb - 1]);
            n_theta += nq;
            ++n_snode;
            for (int q = lane; q < nq; q += 64) {
                double phi, wq;
                if (ntr) {
                    double th = 2.0 * PI * q / ntr;
                    phi = th - th0;
                    wq = 2.0 * PI / ntr;
                } else {
                    phi = rt.th[rt.off[rb - 1] + q];
                    wq = rt.w[rt.off[rb - 1] + q];
                }
                const double th = th0 + phi;
                double sth, cth;
                sincos(th, &sth, &cth);
                // density by Fourier synthesis
                double v0 = si[0], v1 = si[1], v2 = si[2];
                double clv = 1.0, slv = 0.0;
                for (int l = 1; l < NMODE; ++l) {
                    double cn = clv * cth - slv * sth;
                    slv = slv * cth + clv * sth;
                    clv = cn;
                    v0 += si[l * 6 + 0] * clv + si[l * 6 + 3] * slv;
                    v1 += si[l * 6 + 1] * clv + si[l * 6 + 4] * slv;
                    v2 += si[l * 6 + 2] * clv + si[l * 6 + 5] * slv;
                }
                // geometry: dy/ds, dy/dt and r = x - y in the circle's local frame
                double y[3], ys[3], yt[3];
                surface_at(fr, cth, sth, y, ys, yt);
                double sp_, cp_;
                sincos(phi, &sp_, &cp_);
                double hs = sin(0.5 * phi);
                double rb0 = cl.dr + 2.0 * fr.E * hs * hs;
                double rbp = -fr.E * sp_;
                double r[3];
                for (int d = 0; d < 3; ++d) r[d] = cl.z * fr.t[d] + rb0 * cl.b0[d] + rbp * cl.b0p[d];
                double jn[3];
                cross3(yt, ys, jn);
                double J = sqrt(dot3(jn, jn));
                double rr = dot3(r, r);
                if (!(rr > 0.0)) continue;
                double ir = 1.0 / sqrt(rr);
                double ir2 = ir * ir;
                double W = ws * wq;
                double sig[3] = {v0, v1, v2};
                double rs = dot3(r, sig);
                double rn = inf.sign * dot3(r, jn);
                double aS = W * J * ir, bS = W * J * rs * ir * ir2;
                double cD = W * rn * rs * ir2 * ir2 * ir;
                for (int d = 0; d < 3; ++d) {
                    acc[d] += aS * sig[d] + bS * r[d];
                    acc[3 + d] += cD * r[d];
                }
            }
            __syncthreads();
        }
    }
    // minus the smooth rule of this element (self term zero)
    for (int k = lane; k < NPE; k += 64) {
        int64_t n = (int64_t)e * NPE + k;
        double r0 = x[0] - ny[n], r1 = x[1] - ny[N + n], r2 = x[2] - ny[2 * N + n];
        double rr = r0 * r0 + r1 * r1 + r2 * r2;
        if (!(rr > 0.0)) continue;
        double ir = 1.0 / sqrt(rr);
        double ir2 = ir * ir;
        double w0 = sw[n], w1 = sw[N + n], w2 = sw[2 * N + n];
        double rs = r0 * w0 + r1 * w1 + r2 * w2;
        double rn = r0 * nn[n] + r1 * nn[N + n] + r2 * nn[2 * N + n];
        double b = rs * ir * ir2;
        double cD = rn * rs * ir2 * ir2 * ir;
        acc[0] -= ir * w0 + b * r0;
        acc[1] -= ir * w1 + b * r1;
        acc[2] -= ir * w2 + b * r2;
        acc[3] -= cD * r0;
        acc[4] -= cD * r1;
        acc[5] -= cD * r2;
    }
    for (int k = 0; k < 6; ++k) {
        red[lane] = acc[k];
        __syncthreads();
        for (int s = 32; s > 0; s >>= 1) {
            if (lane < s) red[lane] += red[lane + s];
            __syncthreads();
        }
        if (lane == 0) corr[p * 6 + k] = red[0];
        __syncthreads();
    }
    if (lane == 0) {
        work[2 * blockIdx.x] = n_theta;
        work[2 * blockIdx.x + 1] = n_snode;
    }
}

// ---------------------------------------------------------------------------
// final reduction: far chunks in order, then the pair corrections in CSR order
// ---------------------------------------------------------------------------
__global__ void k_reduce(int64_t T, int nchunk, const double* __restrict__ part, const int64_t* __restrict__ off,
                         const int8_t* __restrict__ tier, const double* __restrict__ corr,
                         double* __restrict__ usl, double* __restrict__ udl)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double u[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < nchunk; ++c)
        for (int k = 0; k < 6; ++k) u[k] += part[((int64_t)c * 6 + k) * T + t];
    if (off) {
        for (int64_t p = off[t]; p < off[t + 1]; ++p) {
            if (tier[p] == TIER_SKIP) continue;
            for (int k = 0; k < 6; ++k) u[k] += corr[p * 6 + k];
        }
    }
    const double cS = 1.0 / (8.0 * PI), cD = -3.0 / (4.0 * PI);
    for (int d = 0; d < 3; ++d) {
        if (usl) usl[t * 3 + d] = cS * u[d];
        if (udl) udl[t * 3 + d] = cD * u[3 + d];
    }
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
                  const double* sc, const int* esign, const int* ebody, double* clq, double* circ, ElemInfo* info,
                  double* ny, double* nn, double* nw, int64_t N)
{
    hipLaunchKernelGGL(k_expand, dim3(E), dim3(512), 0, st, E, xc, eps, e1, sa, sc, esign, ebody, clq, circ, info,
                       ny, nn, nw, N);
    LAUNCH_CHECK();
    return 0;
}

int launch_expand_up(hipStream_t st, int E, int f, const double* clq, const ElemInfo* info, const double* ny,
                     const double* nn, const double* nw, int64_t N, double* cpy, double* cpn, double* cpw,
                     int64_t Mtot)
{
    hipLaunchKernelGGL(k_expand_up, dim3(E, f * NS), dim3(f * NT), 0, st, E, f, clq, info, cpy, cpn, cpw, Mtot);
    LAUNCH_CHECK();
    int64_t tot = (int64_t)E * NPE;
    hipLaunchKernelGGL(k_cp_nodes, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, E, f, ny, nn, nw, N, cpy,
                       cpn, cpw, Mtot);
    LAUNCH_CHECK();
    return 0;
}

int launch_prep_sigma(hipStream_t st, int E, const double* sigma, const double* nw, int64_t N, double* sw,
                      double* sh, int* band, double eta, const ElemInfo* info, GateConsts gc, double* rnear)
{
    hipLaunchKernelGGL(k_prep_sigma, dim3(E), dim3(512), 0, st, E, sigma, nw, N, sw, sh, band, eta);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rnear, dim3((E + 127) / 128), dim3(128), 0, st, E, info, band, gc, rnear);
    LAUNCH_CHECK();
    return 0;
}

int launch_sigma_up(hipStream_t st, int E, int f, const double* sh, const double* Lup, const double* cpw,
                    const double* sw, int64_t N, double* swf, int64_t Mtot)
{
    hipLaunchKernelGGL(k_sigma_up, dim3(E), dim3(256), 0, st, E, f, sh, Lup, cpw, sw, N, swf, Mtot);
    LAUNCH_CHECK();
    return 0;
}

int launch_targets(hipStream_t st, int64_t T, const double* x, const int64_t* tnode, const double* ny, int64_t N,
                   double* xt, int* err)
{
    hipLaunchKernelGGL(k_targets, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, T, x, tnode, ny, N, xt, err);
    LAUNCH_CHECK();
    return 0;
}

int launch_far(hipStream_t st, int64_t T, const double* xt, const double* sy, const double* sn, const double* ssw,
               int64_t N, int64_t chunk, int nchunk, double* part)
{
    dim3 grid((unsigned)((T + FAR_BLOCK - 1) / FAR_BLOCK), (unsigned)nchunk);
    hipLaunchKernelGGL(k_far, grid, dim3(FAR_BLOCK), 0, st, T, xt, sy, sn, ssw, N, chunk, part);
    LAUNCH_CHECK();
    return 0;
}

int launch_search(hipStream_t st, int64_t T, int E, const double* xt, const int64_t* tnode, const ElemInfo* info,
                  const double* rnear, const int64_t* off, int* cnt, int* pe, int* pt)
{
    hipLaunchKernelGGL(k_search, dim3((unsigned)((T + 127) / 128)), dim3(128), 0, st, T, E, xt, tnode, info, rnear,
                       off, cnt, pe, pt);
    LAUNCH_CHECK();
    return 0;
}

int launch_classify(hipStream_t st, int64_t P, const int* pe, const int* pt, const double* xt, int64_t T,
                    const int64_t* tnode, const double* clq, const double* circ, const ElemInfo* info,
                    const int* band, GateConsts gc, int8_t* tier, double* cls)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)((P + 127) / 128)), dim3(128), 0, st, P, pe, pt, xt, T, tnode, clq,
                       circ, info, band, gc, tier, cls);
    LAUNCH_CHECK();
    return 0;
}

int launch_bucket_count(hipStream_t st, int64_t P, const int8_t* tier, const int* pe, int* cnt2, int* cnt4,
                        int* nfull)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, tier, pe, cnt2, cnt4,
                       nfull);
    LAUNCH_CHECK();
    return 0;
}

int launch_bucket_fill(hipStream_t st, int64_t P, const int8_t* tier, const int* pe, int* cur2, int* cur4,
                       int* curf, int64_t* list2, int64_t* list4, int64_t* listf)
{
    if (P == 0) return 0;
    hipLaunchKernelGGL(k_bucket_fill, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, tier, pe, cur2, cur4,
                       curf, list2, list4, listf);
    LAUNCH_CHECK();
    return 0;
}

int launch_corr_up(hipStream_t st, int f, int nwaves, const int* wave_elem, const int64_t* list, const int* pt,
                   const double* xt, int64_t T, const double* cpy, const double* cpn, const double* swf,
                   int64_t Mtot, double* corr)
{
    if (nwaves == 0) return 0;
    hipLaunchKernelGGL(k_corr_up, dim3(nwaves), dim3(64), 0, st, f, wave_elem, list, pt, xt, T, cpy, cpn, swf, Mtot,
                       corr);
    LAUNCH_CHECK();
    return 0;
}

int launch_corr_full(hipStream_t st, int nfull, const int64_t* listf, const int* pe, const int* pt, const double* xt,
                     int64_t T, const int64_t* tnode, const double* clq, const double* sh, const ElemInfo* info,
                     const int* band, const double* cls, const double* ny, const double* nn, const double* sw,
                     int64_t N, const int* roff, const double* rth, const double* rw, int nb, const double* lx,
                     const double* lw, int nl, GateConsts gc, double* corr, int* err, int* work)
{
    if (nfull == 0) return 0;
    RuleTables rt{roff, rth, rw, nb, lx, lw, nl};
    hipLaunchKernelGGL(k_corr_full, dim3(nfull), dim3(64), 0, st, listf, pe, pt, xt, T, tnode, clq, sh, info, band,
                       cls, ny, nn, sw, N, rt, gc, corr, err, work);
    LAUNCH_CHECK();
    return 0;
}

int launch_reduce(hipStream_t st, int64_t T, int nchunk, const double* part, const int64_t* off, const int8_t* tier,
                  const double* corr, double* usl, double* udl)
{
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, T, nchunk, part, off, tier,
                       corr, usl, udl);
    LAUNCH_CHECK();
    return 0;
}

}  // namespace csbq
