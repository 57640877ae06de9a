// csbq_solve.cpp -- boundary-integral solves on the evaluator (Section 4):
// the slender combined-field Stokes Dirichlet problem and the slender
// combined-field mobility problem, each solved by restarted GMRES whose
// operator applications replay one frozen evaluation plan (csbq_plan /
// csbq_apply over every surface node).
//
// Operators (D below is the double layer of Section 4, the negative of the
// evaluator's u_dl; see k_combine):
//   Dirichlet (Section 4.1, slender combined field):  K sigma = u0,
//       K = I/2 + D + eta S;  u = (D + eta S)[sigma] off the surface.
//   Mobility (Section 4.2, slender mobility combined field):
//       (K (I - L) + L) sigma = u_s - S nu,
//       L the orthogonal projector (smooth-weight inner product) onto the
//       rigid motions of each body, nu = a_b + beta_b x (y - c_b) the
//       completion density with the given force and torque, and the rigid
//       motion of every body recovered as -L sigma.
// The vector work (inner products, updates, projections) runs in the kernels
// of csbq_solve.hip; the host keeps only GMRES's small Hessenberg system.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "csbq_ctx.hpp"
#include "csbq_solve.hpp"

namespace {

// Inverse of a symmetric positive definite 6x6 matrix by Cholesky; false if
// the matrix is not positive definite.
bool spd_inverse6(const double* G, double* Ginv)
{
    double L[36] = {0};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = G[i * 6 + j];
            for (int k = 0; k < j; ++k) s -= L[i * 6 + k] * L[j * 6 + k];
            if (i == j) {
                if (!(s > 0)) return false;
                L[i * 6 + i] = std::sqrt(s);
            } else {
                L[i * 6 + j] = s / L[j * 6 + j];
            }
        }
    // columns of G^{-1}: solve L L^T x = e_c
    for (int c = 0; c < 6; ++c) {
        double y[6], x[6];
        for (int i = 0; i < 6; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[i * 6 + k] * y[k];
            y[i] = s / L[i * 6 + i];
        }
        for (int i = 5; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < 6; ++k) s -= L[k * 6 + i] * x[k];
            x[i] = s / L[i * 6 + i];
        }
        for (int i = 0; i < 6; ++i) Ginv[i * 6 + c] = x[i];
    }
    return true;
}

// Gram matrix of the raw rigid-body basis of one body in the smooth-weight
// inner product: translations e_i and rotations e_i x r (r = y - c), from the
// body's area A, first moment M1 = sum w r and second moment J2 = sum w r r^T.
void rigid_gram(const double* geo, double* G)
{
    const double A = geo[3];
    const double* M1 = geo + 4;
    const double J[3][3] = {{geo[7], geo[8], geo[9]}, {geo[8], geo[10], geo[11]}, {geo[9], geo[11], geo[12]}};
    const double tr = J[0][0] + J[1][1] + J[2][2];
    auto eps3 = [](int i, int j, int k) -> double {
        if (i == j || j == k || i == k) return 0.0;
        return ((i == 0 && j == 1) || (i == 1 && j == 2) || (i == 2 && j == 0)) ? 1.0 : -1.0;
    };
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            G[i * 6 + j] = (i == j) ? A : 0.0;
            // (e_i, e_j x r) = sum w e_i . (e_j x r) = (e_j x M1)_i
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += eps3(i, j, k) * M1[k];
            G[i * 6 + 3 + j] = v;
            G[(3 + j) * 6 + i] = v;
            // (e_i x r, e_j x r) = sum w (|r|^2 delta_ij - r_i r_j)
            G[(3 + i) * 6 + 3 + j] = (i == j ? tr : 0.0) - J[i][j];
        }
}

}  // namespace

// per-body data of the rigid-body projector: centroids, moments, inverse Gram
// matrices (device), and their host copies
static int rigid_setup(csbq_ctx* ctx, std::vector<double>& geo_h, std::vector<double>& ginv_h)
{
    const int B = ctx->n_bodies;
    ALLOC(ctx->s_boff, (size_t)B + 1);
    ALLOC(ctx->s_geo, (size_t)B * 13);
    ALLOC(ctx->s_ginv, (size_t)B * 36);
    ALLOC(ctx->s_coef, (size_t)B * 6);
    HIPC(hipMemcpyAsync(ctx->s_boff.p, ctx->h_body_off.data(), ((size_t)B + 1) * sizeof(int64_t),
                        hipMemcpyHostToDevice, ctx->stream));
    LCHK(launch_body_geometry(ctx->stream, B, ctx->s_boff.p, ctx->ny.p, ctx->nw.p, ctx->N, ctx->s_geo.p));
    geo_h.assign((size_t)B * 13, 0.0);
    HIPC(hipMemcpyAsync(geo_h.data(), ctx->s_geo.p, geo_h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    ginv_h.assign((size_t)B * 36, 0.0);
    for (int b = 0; b < B; ++b) {
        double G[36];
        rigid_gram(&geo_h[(size_t)b * 13], G);
        if (!spd_inverse6(G, &ginv_h[(size_t)b * 36]))
            return ctx->fail(CSBQ_EINVAL, "a body's rigid-motion Gram matrix is singular");
    }
    HIPC(hipMemcpyAsync(ctx->s_ginv.p, ginv_h.data(), ginv_h.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CSBQ_OK;
}

// the plan every operator application replays: all surface nodes as
// on-surface targets, rules and tiers for the full band
static int operator_plan(csbq_ctx* ctx, const double* dens)
{
    const int64_t N = ctx->N;
    ALLOC(ctx->s_tn, (size_t)N);
    ALLOC(ctx->s_usl, (size_t)N * ctx->nc());
    ALLOC(ctx->s_udl, (size_t)N * ctx->nc());
    LCHK(launch_iota64(ctx->stream, N, ctx->s_tn.p));
    ctx->full_band = true;
    int rc = csbq_plan(ctx, dens, N, nullptr, ctx->s_tn.p, nullptr, ctx->s_usl.p, ctx->s_udl.p, CSBQ_DEVICE);
    ctx->full_band = false;
    return rc;
}

// restarted GMRES with classical Gram-Schmidt applied twice; x (device, n
// doubles) must be zero on entry and holds the solution on return
static int gmres(csbq_ctx* ctx, const csbq_solve_options& o, int64_t n,
                 const std::function<int(const double*, double*)>& A, const double* b, double* x, int32_t* iters)
{
    hipStream_t st = ctx->stream;
    const int m = std::max(1, std::min(o.restart, o.max_iter));
    ALLOC(ctx->s_V, (size_t)(m + 1) * n);
    ALLOC(ctx->s_w, (size_t)n);
    ALLOC(ctx->s_h, (size_t)2 * (m + 2));
    ALLOC(ctx->s_part, (size_t)mdot_blocks(n) * (m + 2));
    double* V = ctx->s_V.p;
    double* w = ctx->s_w.p;
    double* hd = ctx->s_h.p;
    double* part = ctx->s_part.p;
    auto norm = [&](const double* v, double* out) -> int {
        LCHK(launch_mdot(st, n, 1, v, n, v, part, hd, 0));
        double s = 0.0;
        HIPC(hipMemcpyAsync(&s, hd, 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        *out = std::sqrt(s);
        return CSBQ_OK;
    };
    int rc;
    double bnorm = 0.0;
    if ((rc = norm(b, &bnorm))) return rc;
    *iters = 0;
    if (bnorm == 0.0) {
        LCHK(launch_axpby(st, n, 0.0, b, 0.0, x));
        return CSBQ_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 2), y(m);
    int total = 0;
    bool x_zero = true;   // the initial guess is zero: r = b without an application
    while (true) {
        // r = b - A x into w
        if (x_zero) {
            LCHK(launch_axpby(st, n, 1.0, b, 0.0, w));
        } else {
            if ((rc = A(x, w))) return rc;
            LCHK(launch_axpby(st, n, 1.0, b, -1.0, w));
        }
        x_zero = false;
        double beta = 0.0;
        if ((rc = norm(w, &beta))) return rc;
        if (beta <= o.tol * bnorm || total >= o.max_iter) break;
        LCHK(launch_axpby(st, n, 1.0 / beta, w, 0.0, V));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool done = false;
        for (; k < m && total < o.max_iter; ++k) {
            if ((rc = A(V + (size_t)k * n, w))) return rc;
            ++total;
            // two passes of classical Gram-Schmidt; the coefficients stay on the device
            LCHK(launch_mdot(st, n, k + 1, V, n, w, part, hd, 0));
            LCHK(launch_maxpy(st, n, k + 1, V, n, hd, -1.0, w));
            LCHK(launch_mdot(st, n, k + 1, V, n, w, part, hd + (m + 2), 0));
            LCHK(launch_maxpy(st, n, k + 1, V, n, hd + (m + 2), -1.0, w));
            std::vector<double> h2(k + 1);
            HIPC(hipMemcpyAsync(h.data(), hd, (k + 1) * 8, hipMemcpyDeviceToHost, st));
            HIPC(hipMemcpyAsync(h2.data(), hd + (m + 2), (k + 1) * 8, hipMemcpyDeviceToHost, st));
            double hk1 = 0.0;
            if ((rc = norm(w, &hk1))) return rc;   // synchronises
            for (int i = 0; i <= k; ++i) h[i] += h2[i];
            h[k + 1] = hk1;
            if (hk1 > 0.0) LCHK(launch_axpby(st, n, 1.0 / hk1, w, 0.0, V + (size_t)(k + 1) * n));
            // previous Givens rotations, then a new one for row k+1
            for (int i = 0; i < k; ++i) {
                const double t = cs[i] * h[i] + sn[i] * h[i + 1];
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                h[i] = t;
            }
            const double den = std::hypot(h[k], h[k + 1]);
            cs[k] = den > 0 ? h[k] / den : 1.0;
            sn[k] = den > 0 ? h[k + 1] / den : 0.0;
            h[k] = den;
            h[k + 1] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            for (int i = 0; i <= k; ++i) H[(size_t)k * (m + 1) + i] = h[i];
            if (std::fabs(g[k + 1]) <= o.tol * bnorm || hk1 == 0.0) {
                ++k;
                done = true;
                break;
            }
        }
        // x += V y, H y = g (upper triangular, k columns)
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[(size_t)j * (m + 1) + i] * y[j];
            y[i] = s / H[(size_t)i * (m + 1) + i];
        }
        HIPC(hipMemcpyAsync(hd, y.data(), k * 8, hipMemcpyHostToDevice, st));
        LCHK(launch_maxpy(st, n, k, V, n, hd, 1.0, x));
        HIPC(hipStreamSynchronize(st));
        if (done || total >= o.max_iter) break;
    }
    *iters = total;
    return CSBQ_OK;
}

// ||b - A x|| / ||b|| with one more operator application
static int true_residual(csbq_ctx* ctx, int64_t n, const std::function<int(const double*, double*)>& A,
                         const double* b, const double* x, double* rel)
{
    hipStream_t st = ctx->stream;
    double* w = ctx->s_w.p;
    double* hd = ctx->s_h.p;
    int rc;
    if ((rc = A(x, w))) return rc;
    LCHK(launch_axpby(st, n, 1.0, b, -1.0, w));
    LCHK(launch_mdot(st, n, 1, w, n, w, ctx->s_part.p, hd, 0));
    LCHK(launch_mdot(st, n, 1, b, n, b, ctx->s_part.p, hd + 1, 0));
    double s[2] = {0, 0};
    HIPC(hipMemcpyAsync(s, hd, 16, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    *rel = s[1] > 0 ? std::sqrt(s[0] / s[1]) : 0.0;
    return CSBQ_OK;
}

static int solve_checks(csbq_ctx* ctx, const csbq_solve_options* o, int mem)
{
    if (!ctx->have_geom) return ctx->fail(CSBQ_ESTATE, "set_geometry must be called first");
    if (ctx->G != 1) return ctx->fail(CSBQ_EINVAL, "solves take a single geometry (not a batch of groups)");
    if (!o || !(o->eta > 0) || !std::isfinite(o->eta))
        return ctx->fail(CSBQ_EINVAL, "the single-layer weight eta must be positive");
    if (!(o->tol > 0) || o->max_iter < 1 || o->restart < 1)
        return ctx->fail(CSBQ_EINVAL, "GMRES needs tol > 0, max_iter >= 1 and restart >= 1");
    if (mem != CSBQ_HOST && mem != CSBQ_DEVICE) return ctx->fail(CSBQ_EINVAL, "bad mem flag");
    return CSBQ_OK;
}

// caller array (host or device, n doubles) -> device buffer
static int stage_in(csbq_ctx* ctx, DBuf<double>& buf, const double* src, int64_t n, int mem)
{
    ALLOC(buf, (size_t)n);
    if (mem == CSBQ_HOST)
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(src[i])) return ctx->fail(CSBQ_EINVAL, "input has NaN/Inf");
    HIPC(hipMemcpyAsync(buf.p, src, (size_t)n * 8, mem == CSBQ_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                        ctx->stream));
    return CSBQ_OK;
}

static int stage_out(csbq_ctx* ctx, double* dst, const double* src, int64_t n, int mem)
{
    if (!dst) return CSBQ_OK;
    HIPC(hipMemcpyAsync(dst, src, (size_t)n * 8, mem == CSBQ_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        ctx->stream));
    return CSBQ_OK;
}

extern "C" {

void csbq_default_solve_options(csbq_solve_options* o)
{
    if (!o) return;
    o->eta = 1.0;
    o->tol = 1e-10;
    o->max_iter = 200;
    o->restart = 60;
}

int csbq_solve_dirichlet(csbq_ctx* ctx, const csbq_solve_options* o, const double* u0, double* sigma,
                         csbq_solve_info* info, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    int rc;
    if ((rc = solve_checks(ctx, o, mem))) return rc;
    if (!u0 || !sigma) return ctx->fail(CSBQ_EINVAL, "missing boundary data or output");
    HIPC(hipSetDevice(ctx->opt.device));
    const int64_t n = ctx->N * ctx->nc();
    const double dsign = ctx->ker == KER_LAPLACE ? 1.0 : -1.0;
    hipStream_t st = ctx->stream;
    if ((rc = stage_in(ctx, ctx->s_b, u0, n, mem))) return rc;
    ALLOC(ctx->s_x, (size_t)n);
    if ((rc = operator_plan(ctx, ctx->s_b.p))) return rc;
    LCHK(launch_axpby(st, n, 0.0, ctx->s_b.p, 0.0, ctx->s_x.p));
    const double eta = o->eta;
    std::function<int(const double*, double*)> A = [&](const double* in, double* out) -> int {
        int r = csbq_apply(ctx, in, ctx->s_usl.p, ctx->s_udl.p, CSBQ_DEVICE);
        if (r) return r;
        LCHK(launch_combine(st, n, in, ctx->s_usl.p, ctx->s_udl.p, eta, dsign, nullptr, out));
        return CSBQ_OK;
    };
    int32_t it = 0;
    if ((rc = gmres(ctx, *o, n, A, ctx->s_b.p, ctx->s_x.p, &it))) return rc;
    double rel = 0.0;
    if ((rc = true_residual(ctx, n, A, ctx->s_b.p, ctx->s_x.p, &rel))) return rc;
    if ((rc = stage_out(ctx, sigma, ctx->s_x.p, n, mem))) return rc;
    HIPC(hipStreamSynchronize(st));
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
    }
    return CSBQ_OK;
}

int csbq_solve_mobility(csbq_ctx* ctx, const csbq_solve_options* o, const double* force, const double* torque,
                        const double* u_slip, double* sigma, double* nu, double* rigid, double* centers,
                        csbq_solve_info* info, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    int rc;
    if ((rc = solve_checks(ctx, o, mem))) return rc;
    if (!force || !torque) return ctx->fail(CSBQ_EINVAL, "missing forces or torques");
    if (ctx->ker != KER_STOKES) return ctx->fail(CSBQ_EINVAL, "the mobility problem is a Stokes problem");
    HIPC(hipSetDevice(ctx->opt.device));
    const int B = ctx->n_bodies;
    for (int k = 0; k < 3 * B; ++k)
        if (!std::isfinite(force[k]) || !std::isfinite(torque[k]))
            return ctx->fail(CSBQ_EINVAL, "forces and torques must be finite");
    const int64_t N = ctx->N, n = N * 3;
    hipStream_t st = ctx->stream;
    std::vector<double> geo, ginv;
    if ((rc = rigid_setup(ctx, geo, ginv))) return rc;
    // completion density: G (a, beta) = (F, T) per body
    std::vector<double> ab((size_t)B * 6);
    for (int b = 0; b < B; ++b) {
        const double ft[6] = {force[3 * b], force[3 * b + 1], force[3 * b + 2],
                              torque[3 * b], torque[3 * b + 1], torque[3 * b + 2]};
        for (int i = 0; i < 6; ++i) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += ginv[(size_t)b * 36 + i * 6 + k] * ft[k];
            ab[(size_t)b * 6 + i] = s;
        }
    }
    ALLOC(ctx->s_nu, (size_t)n);
    ALLOC(ctx->s_b, (size_t)n);
    ALLOC(ctx->s_x, (size_t)n);
    ALLOC(ctx->s_tau, (size_t)n);
    ALLOC(ctx->s_lsig, (size_t)n);
    HIPC(hipMemcpyAsync(ctx->s_coef.p, ab.data(), ab.size() * 8, hipMemcpyHostToDevice, st));
    LCHK(launch_rigid_field(st, N, B, ctx->s_boff.p, ctx->ny.p, ctx->s_geo.p, ctx->s_coef.p, 1.0, nullptr,
                            ctx->s_nu.p));
    if ((rc = operator_plan(ctx, ctx->s_nu.p))) return rc;
    // right-hand side u_s - S nu (the plan's evaluation of nu left S nu in s_usl)
    if (u_slip) {
        if ((rc = stage_in(ctx, ctx->s_b, u_slip, n, mem))) return rc;
        LCHK(launch_axpby(st, n, -1.0, ctx->s_usl.p, 1.0, ctx->s_b.p));
    } else {
        LCHK(launch_axpby(st, n, -1.0, ctx->s_usl.p, 0.0, ctx->s_b.p));
    }
    LCHK(launch_axpby(st, n, 0.0, ctx->s_b.p, 0.0, ctx->s_x.p));
    const double eta = o->eta;
    // (K (I - L) + L) in: coefficients of L in, tau = in - L in, K tau + L in
    std::function<int(const double*, double*)> A = [&](const double* in, double* out) -> int {
        LCHK(launch_body_project(st, B, ctx->s_boff.p, ctx->ny.p, ctx->nw.p, N, ctx->s_geo.p, ctx->s_ginv.p, in,
                                 ctx->s_coef.p));
        LCHK(launch_rigid_field(st, N, B, ctx->s_boff.p, ctx->ny.p, ctx->s_geo.p, ctx->s_coef.p, -1.0, in,
                                ctx->s_tau.p));
        LCHK(launch_rigid_field(st, N, B, ctx->s_boff.p, ctx->ny.p, ctx->s_geo.p, ctx->s_coef.p, 1.0, nullptr,
                                ctx->s_lsig.p));
        int r = csbq_apply(ctx, ctx->s_tau.p, ctx->s_usl.p, ctx->s_udl.p, CSBQ_DEVICE);
        if (r) return r;
        LCHK(launch_combine(st, n, ctx->s_tau.p, ctx->s_usl.p, ctx->s_udl.p, eta, -1.0, ctx->s_lsig.p, out));
        return CSBQ_OK;
    };
    int32_t it = 0;
    if ((rc = gmres(ctx, *o, n, A, ctx->s_b.p, ctx->s_x.p, &it))) return rc;
    double rel = 0.0;
    if ((rc = true_residual(ctx, n, A, ctx->s_b.p, ctx->s_x.p, &rel))) return rc;
    // rigid motion -L sigma; the density of the representation (I - L) sigma
    LCHK(launch_body_project(st, B, ctx->s_boff.p, ctx->ny.p, ctx->nw.p, N, ctx->s_geo.p, ctx->s_ginv.p, ctx->s_x.p,
                             ctx->s_coef.p));
    LCHK(launch_rigid_field(st, N, B, ctx->s_boff.p, ctx->ny.p, ctx->s_geo.p, ctx->s_coef.p, -1.0, ctx->s_x.p,
                            ctx->s_tau.p));
    std::vector<double> coef((size_t)B * 6);
    HIPC(hipMemcpyAsync(coef.data(), ctx->s_coef.p, coef.size() * 8, hipMemcpyDeviceToHost, st));
    if ((rc = stage_out(ctx, sigma, ctx->s_tau.p, n, mem))) return rc;
    if ((rc = stage_out(ctx, nu, ctx->s_nu.p, n, mem))) return rc;
    HIPC(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
        if (rigid)
            for (int i = 0; i < 6; ++i) rigid[(size_t)b * 6 + i] = -coef[(size_t)b * 6 + i];
        if (centers)
            for (int i = 0; i < 3; ++i) centers[(size_t)b * 3 + i] = geo[(size_t)b * 13 + i];
    }
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
    }
    return CSBQ_OK;
}

}  // extern "C"
