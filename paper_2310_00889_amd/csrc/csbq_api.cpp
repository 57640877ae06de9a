// csbq_api.cpp -- C ABI of the gfx950 Stokes layer-potential evaluator
// (declared in include/csbq.h): context, device memory, table loading and the
// sequencing of the kernels of one evaluation.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "csbq_ctx.hpp"
#include <algorithm>
#include <random>

using namespace csbq;

namespace {

const char* kPhaseNames[] = {"prep", "far", "search", "classify", "bucket", "corr_up", "corr_full", "reduce"};

// Gauss-Legendre nodes by Newton iteration on the Legendre recurrence, with
// the closed-form barycentric weights (-1)^i sqrt((1-x_i^2) w_i) of the GL
// nodes and the spectral differentiation matrix built from them.
void gl_tables(int n, double* x, double* w, double* lam, double* D, double* T)
{
    for (int i = 0; i < n; ++i) {
        // i-th root in ascending order
        double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (p0 - z * p1) / (1.0 - z * z);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (p0 - z * p1) / (1.0 - z * z);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    for (int i = 0; i < n; ++i) lam[i] = ((i % 2) ? -1.0 : 1.0) * std::sqrt((1.0 - x[i] * x[i]) * w[i]);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double v = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * n + j] = v;
            s += v;
        }
        D[i * n + i] = -s;
    }
    for (int i = 0; i < n; ++i) {
        double p0 = 1.0, p1 = x[i];
        for (int k = 0; k < n; ++k) {
            double pk;
            if (k == 0)
                pk = 1.0;
            else if (k == 1)
                pk = x[i];
            else {
                double p2 = ((2 * k - 1) * x[i] * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
                pk = p2;
            }
            T[k * n + i] = 0.5 * (2 * k + 1) * w[i] * pk;
        }
    }
}

void lagrange_row(int n, const double* x, const double* lam, double xi, double* row)
{
    double s = 0.0;
    int hit = -1;
    for (int i = 0; i < n; ++i) {
        double d = xi - x[i];
        if (d == 0.0) hit = i;
        row[i] = lam[i] / (d == 0.0 ? 1.0 : d);
        s += row[i];
    }
    if (hit >= 0) {
        for (int i = 0; i < n; ++i) row[i] = (i == hit) ? 1.0 : 0.0;
        return;
    }
    for (int i = 0; i < n; ++i) row[i] /= s;
}

std::string default_table_dir()
{
    Dl_info info;
    if (dladdr((void*)&csbq_default_options, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t k = p.find_last_of('/');
        std::string dir = (k == std::string::npos) ? std::string(".") : p.substr(0, k);
        return dir + "/tables";
    }
    return "tables";
}

}  // namespace


static void plan_drop(csbq_ctx* ctx);

static_assert(CSBQ_NOALLOC_MAX_TARGETS == NOALLOC_MAX_TARGETS && CSBQ_NOALLOC_MAX_NODES == NOALLOC_MAX_NODES,
              "limits of the allocation-free smooth sum");
static_assert(CSBQ_FLAG_NODE_RANGE == FLAG_NODE_RANGE && CSBQ_FLAG_SRULE_LIMIT == FLAG_SRULE_LIMIT &&
                  CSBQ_FLAG_THETA_CLAMP == FLAG_THETA_CLAMP && CSBQ_FLAG_GROUP_RANGE == FLAG_GROUP_RANGE &&
                  CSBQ_FLAG_GROUP_ORDER == FLAG_GROUP_ORDER && CSBQ_FLAG_BAND == FLAG_BAND,
              "flag bits of the C ABI and the kernels");


extern "C" {

void csbq_default_options(csbq_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->quad_tol = 1e-12;
    opt->precision = CSBQ_FP64;
    opt->gate = CSBQ_GATE_CRITERION;
    opt->device = 0;
    opt->stream = nullptr;
    opt->table_dir = nullptr;
    opt->kernel = CSBQ_KERNEL_STOKES;
    opt->srule = CSBQ_SRULE_AUTO;
    opt->far_rule = CSBQ_FAR_AUTO;
}

const char* csbq_last_error(const csbq_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static bool file_exists(const std::string& path)
{
    FILE* f = std::fopen(path.c_str(), "rb");
    if (f) std::fclose(f);
    return f != nullptr;
}

// Rule tables of a context: with quad_tol >= 1e-8 the ones built to 1e-8
// (rules_t8.bin, srules_t8.bin: fewer nodes) where the table directory holds
// them, else those built to 1e-13 / 1e-12 (rules.bin, srules.bin).
static std::string table_name(const csbq_ctx* ctx, const char* base)
{
    const std::string loose = std::string(base) + "_t8.bin";
    if (ctx->opt.quad_tol >= 1e-8 && file_exists(ctx->table_dir + "/" + loose)) return loose;
    return std::string(base) + ".bin";
}

static int load_tables(csbq_ctx* ctx)
{
    const std::string path = ctx->table_dir + "/" + table_name(ctx, "rules");
    ctx->table_path = path;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return ctx->fail(CSBQ_ETABLE, "cannot open " + path);
    char magic[8];
    int32_t ver, nb, l0;
    double tol;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CSBQRUL1", 8) == 0 &&
              std::fread(&ver, 4, 1, f) == 1 && std::fread(&nb, 4, 1, f) == 1 && std::fread(&l0, 4, 1, f) == 1 &&
              std::fread(&tol, 8, 1, f) == 1 && nb > 0 && nb < 64;
    std::vector<int> off(1, 0);
    std::vector<double> th, w;
    for (int b = 0; ok && b < nb; ++b) {
        int32_t m;
        ok = std::fread(&m, 4, 1, f) == 1 && m > 0 && m <= MAXRULE;
        if (!ok) break;
        size_t o = th.size();
        th.resize(o + m);
        w.resize(o + m);
        ok = std::fread(th.data() + o, 8, m, f) == (size_t)m && std::fread(w.data() + o, 8, m, f) == (size_t)m;
        off.push_back((int)th.size());
    }
    int32_t ml = 0;
    std::vector<double> lx, lw;
    if (ok) ok = std::fread(&ml, 4, 1, f) == 1 && ml > 0 && ml <= MAXLOG;
    if (ok) {
        lx.resize(ml);
        lw.resize(ml);
        ok = std::fread(lx.data(), 8, ml, f) == (size_t)ml && std::fread(lw.data(), 8, ml, f) == (size_t)ml;
    }
    std::fclose(f);
    if (!ok) return ctx->fail(CSBQ_ETABLE, "malformed rule table " + path);
    // the special quadrature evaluates each theta-rule in mirror pairs
    // (phi, -phi): every rule must be symmetric with equal mirrored weights
    for (size_t b = 0; b + 1 < off.size(); ++b) {
        const int o = off[b], m = off[b + 1] - off[b];
        bool sym = m % 2 == 0;
        for (int q = 0; sym && q < m / 2; ++q)
            sym = th[o + q] == -th[o + m - 1 - q] && w[o + q] == w[o + m - 1 - q] && th[o + m - 1 - q] > 0.0;
        if (!sym) return ctx->fail(CSBQ_ETABLE, "theta-rule " + std::to_string(b + 1) + " is not symmetric in " + path);
    }
    std::vector<double> cs_(th.size()), sn_(th.size()), omc_(th.size());
    for (size_t q = 0; q < th.size(); ++q) {
        cs_[q] = std::cos(th[q]);
        sn_[q] = std::sin(th[q]);
        double h = std::sin(0.5 * th[q]);
        omc_[q] = 2.0 * h * h;   // 1 - cos, without cancellation near 0
    }
    ALLOC(ctx->rcs, th.size());
    ALLOC(ctx->rsn, th.size());
    ALLOC(ctx->romc, th.size());
    HIPC(hipMemcpy(ctx->rcs.p, cs_.data(), th.size() * 8, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->rsn.p, sn_.data(), th.size() * 8, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->romc.p, omc_.data(), th.size() * 8, hipMemcpyHostToDevice));
    ALLOC(ctx->roff, off.size());
    ALLOC(ctx->rth, th.size());
    ALLOC(ctx->rw, w.size());
    ALLOC(ctx->lx, lx.size());
    ALLOC(ctx->lw, lw.size());
    HIPC(hipMemcpy(ctx->roff.p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->rth.p, th.data(), th.size() * 8, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->rw.p, w.data(), w.size() * 8, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->lx.p, lx.data(), lx.size() * 8, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->lw.p, lw.data(), lw.size() * 8, hipMemcpyHostToDevice));
    ctx->nb = nb;
    ctx->nl = ml;
    return CSBQ_OK;
}

// density times weight on the coarser far-field rules (from the Fourier
// coefficients on the GL circles, as on the upsampled rules), straight into
// the base source set; nothing is allocated, so an evaluation plan's replay
// can run it
static int sigma_far(csbq_ctx* ctx, hipStream_t st)
{
    for (int k = 0; k < NFL; ++k) {
        if (!ctx->far_used[k]) continue;
        const int i = k / NFT;
        int r = launch_sigma_up(st, ctx->E, far_ns(i), far_nt(k % NFT), ctx->sh.p, ctx->Lfar[i].p, ctx->bw.p,
                                ctx->bsw.p, ctx->Nb, ctx->loff.p + (int64_t)k * ctx->E);
        if (r) return r;
    }
    return 0;
}

// Whole-element singular s-rules (Section 3.2.4, second part), written by
// tables/gen_srules.py: per cylinder aspect bracket and target GL index, then
// (optionally) per target GL index of the sphere element, node offsets from
// the GL node in the element variable v in [-1, 1] and their weights.
static int load_srules(csbq_ctx* ctx)
{
    const std::string path = ctx->table_dir + "/" + table_name(ctx, "srules");
    ctx->srule_path = path;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return ctx->fail(CSBQ_ETABLE, "cannot open " + path);
    char magic[8];
    int32_t ver, ns, b_lo, nb, nsph, l0, npoly;
    double tol;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CSBQSRL2", 8) == 0 &&
              std::fread(&ver, 4, 1, f) == 1 && std::fread(&ns, 4, 1, f) == 1 && std::fread(&b_lo, 4, 1, f) == 1 &&
              std::fread(&nb, 4, 1, f) == 1 && std::fread(&nsph, 4, 1, f) == 1 && std::fread(&l0, 4, 1, f) == 1 &&
              std::fread(&npoly, 4, 1, f) == 1 && std::fread(&tol, 8, 1, f) == 1 && ns == NS && nb >= 0 &&
              nb <= 64 && (nb == 0 || (b_lo >= 2 && b_lo + nb <= 31)) && (nsph == 0 || nsph == 1) && l0 >= 0 &&
              l0 <= NT;
    std::vector<int> off(1, 0);
    std::vector<double> d, w;
    for (int k = 0; ok && k < (nb + nsph) * NS; ++k) {
        int32_t m;
        ok = std::fread(&m, 4, 1, f) == 1 && m > 0 && m <= MAXWHOLE;
        if (!ok) break;
        const size_t o = d.size();
        d.resize(o + m);
        w.resize(o + m);
        ok = std::fread(d.data() + o, 8, m, f) == (size_t)m && std::fread(w.data() + o, 8, m, f) == (size_t)m;
        // nodes inside the element, off the target, ascending
        const double xi = ctx->gx[k % NS];
        for (int j = 0; ok && j < m; ++j)
            ok = std::isfinite(d[o + j]) && std::isfinite(w[o + j]) && d[o + j] != 0.0 && xi + d[o + j] > -1.0 &&
                 xi + d[o + j] < 1.0 && (j == 0 || d[o + j] > d[o + j - 1]);
        off.push_back((int)d.size());
    }
    std::fclose(f);
    if (!ok) return ctx->fail(CSBQ_ETABLE, "malformed whole-element rule table " + path);
    ALLOC(ctx->woff, off.size());
    ALLOC(ctx->wd, d.size() + 1);
    ALLOC(ctx->ww, w.size() + 1);
    HIPC(hipMemcpy(ctx->woff.p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!d.empty()) {
        HIPC(hipMemcpy(ctx->wd.p, d.data(), d.size() * 8, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->ww.p, w.data(), w.size() * 8, hipMemcpyHostToDevice));
    }
    ctx->wb_lo = b_lo;
    ctx->wnb = nb;
    ctx->wl0 = l0;
    ctx->wsph = nsph ? nb : -1;
    return CSBQ_OK;
}

static RuleArgs rule_args(const csbq_ctx* ctx)
{
    const bool on = ctx->opt.srule != CSBQ_SRULE_GENERAL;
    return RuleArgs{ctx->roff.p, ctx->rth.p, ctx->rw.p, ctx->nb, ctx->lx.p, ctx->lw.p, ctx->nl, ctx->rcs.p,
                    ctx->rsn.p, ctx->romc.p, ctx->woff.p, ctx->wd.p, ctx->ww.p, ctx->wb_lo, on ? ctx->wnb : 0,
                    ctx->wl0, on ? ctx->wsph : -1, ctx->opt.srule == CSBQ_SRULE_WHOLE ? 1 : 0};
}

// Shape of an element for the whole-element singular s-rules, from its GL
// samples (xc [NS][3], eps [NS], e1 [NS][3] at the nodes gx of [-1, 1], D the
// differentiation matrix there):
//  * SHAPE_SPHERE: x_c = c + a cos(pi t) q, eps = a sin(pi t), t = (v + 1)/2,
//    |q| = 1, with constant e1, to 1e-12 of the element's size (the sphere
//    rules' family exactly);
//  * SHAPE_CYLINDER: constant speed |x_c'| (to 1e-9), bend (largest curvature
//    times the element's length) at most 0.06, radius varying by at most
//    10 % and e1 turning by at most 0.25 rad over the element, none of which
//    moved the cylinder rules by more than ~1e-13 in measurements (the rules
//    are exact on straight cylinders of constant radius; at bend 0.13 they
//    missed by 1.5e-12, at 0.79 by 7e-9; a 0.1 % speed variation cost 1e-10);
//  * SHAPE_OTHER otherwise.
static int element_shape(const double* xc, const double* eps, const double* e1, const double* gx, const double* D)
{
    auto dot3 = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto n3 = [&](const double* v) { return std::sqrt(dot3(v, v)); };
    auto cross3 = [](const double* a, const double* b, double* c) {
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
    };
    // sphere: x_c = c + a cos(pi t) q, eps = a sin(pi t), constant e1
    {
        const double tol = 1e-12;
        const double e1n = n3(e1);
        bool ok = e1n > 0.0;
        for (int i = 1; ok && i < NS; ++i)
            for (int d = 0; ok && d < 3; ++d) ok = std::fabs(e1[3 * i + d] - e1[d]) <= tol * e1n;
        const double PI_ = 3.14159265358979323846;
        const double c0 = std::cos(PI_ * 0.5 * (gx[0] + 1.0)), c1 = std::cos(PI_ * 0.5 * (gx[NS - 1] + 1.0));
        double aq[3], c[3];
        for (int d = 0; d < 3; ++d) {
            aq[d] = (xc[d] - xc[3 * (NS - 1) + d]) / (c0 - c1);
            c[d] = xc[d] - c0 * aq[d];
        }
        const double a = n3(aq);
        ok = ok && a > 0.0;
        for (int i = 0; ok && i < NS; ++i) {
            const double t = PI_ * 0.5 * (gx[i] + 1.0);
            ok = std::fabs(eps[i] - a * std::sin(t)) <= tol * a;
            for (int d = 0; ok && d < 3; ++d) ok = std::fabs(xc[3 * i + d] - (c[d] + std::cos(t) * aq[d])) <= tol * a;
        }
        if (ok) return SHAPE_SPHERE;
    }
    // cylinder rules: constant speed, small bend, taper and e1 turn
    double xp[NS][3], xpp[NS][3];
    for (int i = 0; i < NS; ++i)
        for (int d = 0; d < 3; ++d) {
            double s1 = 0.0;
            for (int j = 0; j < NS; ++j) s1 += D[i * NS + j] * xc[3 * j + d];
            xp[i][d] = s1;
        }
    for (int i = 0; i < NS; ++i)
        for (int d = 0; d < 3; ++d) {
            double s2 = 0.0;
            for (int j = 0; j < NS; ++j) s2 += D[i * NS + j] * xp[j][d];
            xpp[i][d] = s2;
        }
    double spmin = 1e300, spmax = 0.0, spsum = 0.0, kmax = 0.0, emin = 1e300, emax = 0.0;
    for (int i = 0; i < NS; ++i) {
        const double sp = n3(xp[i]);
        double cr[3];
        cross3(xp[i], xpp[i], cr);
        spmin = std::fmin(spmin, sp);
        spmax = std::fmax(spmax, sp);
        spsum += sp;
        kmax = std::fmax(kmax, n3(cr) / (sp * sp * sp));
        emin = std::fmin(emin, eps[i]);
        emax = std::fmax(emax, eps[i]);
    }
    const double spm = spsum / NS;
    if (!(spmin > 0.0) || !(emin > 0.0)) return SHAPE_OTHER;
    if (spmax - spmin > 1e-9 * spm) return SHAPE_OTHER;
    if (kmax * 2.0 * spm > 0.06) return SHAPE_OTHER;
    if (emax > 1.1 * emin) return SHAPE_OTHER;
    // e1 at both ends, each without its tangential part: the angle between them
    double u0[3], u1[3];
    {
        const double* a = e1;
        const double* b = e1 + 3 * (NS - 1);
        const double* t0 = xp[0];
        const double* t1 = xp[NS - 1];
        const double at = dot3(a, t0) / dot3(t0, t0), bt = dot3(b, t1) / dot3(t1, t1);
        for (int d = 0; d < 3; ++d) {
            u0[d] = a[d] - at * t0[d];
            u1[d] = b[d] - bt * t1[d];
        }
    }
    const double cu = dot3(u0, u1) / (n3(u0) * n3(u1));
    if (!(cu >= std::cos(0.25))) return SHAPE_OTHER;
    return SHAPE_CYLINDER;
}

// A torus-arc element (a section of a tube of constant radius r about a
// circle of radius R > r): centerline x_c = C + R (cos psi U + sin psi V) with
// psi = psi0 + psi1 xn linear in the panel's normalised variable xn.  Then
// the classification's contact zero has a closed form.  out[TOR_Q]: C, U, V,
// R, r, psi0, psi1 and a flag (1 = such an element, else all 0).
static void element_torus(const double* xc, const double* eps, const double* gx, double* out)
{
    auto dot3 = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto cross3 = [](const double* a, const double* b, double* c) {
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
    };
    for (int k = 0; k < TOR_Q; ++k) out[k] = 0.0;
    const double tol = 1e-11;
    const double r = eps[0];
    if (!(r > 0.0)) return;
    for (int i = 1; i < NS; ++i)
        if (std::fabs(eps[i] - r) > tol * r) return;
    // the circle through the first, middle and last centerline points
    const double* p0 = xc;
    const double* pm = xc + 3 * (NS / 2);
    const double* p1 = xc + 3 * (NS - 1);
    double ab[3], ac[3], n[3];
    for (int d = 0; d < 3; ++d) {
        ab[d] = pm[d] - p0[d];
        ac[d] = p1[d] - p0[d];
    }
    cross3(ab, ac, n);
    const double nn = dot3(n, n);
    if (!(nn > 1e-24 * dot3(ac, ac) * dot3(ac, ac))) return;   // (nearly) straight
    double t1[3], t2[3], c[3];
    cross3(n, ab, t1);
    cross3(ac, n, t2);
    for (int d = 0; d < 3; ++d) c[d] = p0[d] + (dot3(ac, ac) * t1[d] + dot3(ab, ab) * t2[d]) / (2.0 * nn);
    double u[3], v[3], nz[3];
    for (int d = 0; d < 3; ++d) u[d] = p0[d] - c[d];
    const double R = std::sqrt(dot3(u, u));
    if (!(R > r * (1.0 + 1e-6))) return;
    for (int d = 0; d < 3; ++d) {
        u[d] /= R;
        nz[d] = n[d] / std::sqrt(nn);
    }
    cross3(nz, u, v);
    // every point on that circle, at an angle linear in xn
    double psi[NS], gm = 0.0, pmn = 0.0;
    for (int i = 0; i < NS; ++i) {
        double q[3];
        for (int d = 0; d < 3; ++d) q[d] = xc[3 * i + d] - c[d];
        if (std::fabs(dot3(q, nz)) > tol * R || std::fabs(std::sqrt(dot3(q, q)) - R) > tol * R) return;
        psi[i] = std::atan2(dot3(q, v), dot3(q, u));
        gm += gx[i] / NS;
        pmn += psi[i] / NS;
    }
    double sxy = 0.0, sxx = 0.0;
    for (int i = 0; i < NS; ++i) {
        sxy += (gx[i] - gm) * (psi[i] - pmn);
        sxx += (gx[i] - gm) * (gx[i] - gm);
    }
    const double psi1 = sxy / sxx, psi0 = pmn - psi1 * gm;
    if (!(std::fabs(psi1) > 0.0) || std::fabs(psi1) > 1.5) return;   // an arc of at most 3 rad
    for (int i = 0; i < NS; ++i)
        if (std::fabs(psi[i] - (psi0 + psi1 * gx[i])) > tol) return;
    for (int d = 0; d < 3; ++d) {
        out[d] = c[d];
        out[3 + d] = u[d];
        out[6 + d] = v[d];
    }
    out[9] = R;
    out[10] = r;
    out[11] = psi0;
    out[12] = psi1;
    out[TOR_Q - 1] = 1.0;
}

int csbq_create(const csbq_options* opt, csbq_ctx** out)
{
    if (!out) return CSBQ_EINVAL;
    *out = nullptr;
    csbq_ctx* ctx = new (std::nothrow) csbq_ctx();
    if (!ctx) return CSBQ_ENOMEM;
    if (opt)
        ctx->opt = *opt;
    else
        csbq_default_options(&ctx->opt);
    if (!(ctx->opt.quad_tol > 0)) ctx->opt.quad_tol = 1e-12;
    if (ctx->opt.gate != CSBQ_GATE_CRITERION && ctx->opt.gate != CSBQ_GATE_MLP) {
        delete ctx;
        return CSBQ_EINVAL;
    }
    if (ctx->opt.precision != CSBQ_FP64 && ctx->opt.precision != CSBQ_MIXED) {
        delete ctx;
        return CSBQ_EINVAL;
    }
    // the Laplace layers run in FP64 under the error-estimate criterion (the
    // mixed-precision sum and the learned gate are built for the Stokes pair)
    if ((ctx->opt.kernel != CSBQ_KERNEL_STOKES && ctx->opt.kernel != CSBQ_KERNEL_LAPLACE) ||
        (ctx->opt.kernel == CSBQ_KERNEL_LAPLACE &&
         (ctx->opt.precision != CSBQ_FP64 || ctx->opt.gate != CSBQ_GATE_CRITERION))) {
        delete ctx;
        return CSBQ_EINVAL;
    }
    if (ctx->opt.srule != CSBQ_SRULE_AUTO && ctx->opt.srule != CSBQ_SRULE_WHOLE &&
        ctx->opt.srule != CSBQ_SRULE_GENERAL) {
        delete ctx;
        return CSBQ_EINVAL;
    }
    if (ctx->opt.far_rule != CSBQ_FAR_AUTO && ctx->opt.far_rule != CSBQ_FAR_BASE) {
        delete ctx;
        return CSBQ_EINVAL;
    }
    ctx->far_split = ctx->opt.far_rule == CSBQ_FAR_AUTO;
    ctx->ker = ctx->opt.kernel == CSBQ_KERNEL_LAPLACE ? KER_LAPLACE : KER_STOKES;
    ctx->table_dir = ctx->opt.table_dir ? std::string(ctx->opt.table_dir) : default_table_dir();
    ctx->opt.table_dir = nullptr;
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || ctx->opt.device < 0 || ctx->opt.device >= ndev) {
        std::fprintf(stderr, "csbq_create: no usable device (%s, %d devices)\n", hipGetErrorString(he), ndev);
        (void)hipGetLastError();
        delete ctx;
        return CSBQ_EHIP;
    }
    if ((he = hipSetDevice(ctx->opt.device)) != hipSuccess) {
        std::fprintf(stderr, "csbq_create: hipSetDevice: %s\n", hipGetErrorString(he));
        delete ctx;
        return CSBQ_EHIP;
    }
    if (ctx->opt.stream) {
        ctx->stream = (hipStream_t)ctx->opt.stream;
    } else {
        if ((he = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) {
            std::fprintf(stderr, "csbq_create: hipStreamCreate: %s\n", hipGetErrorString(he));
            delete ctx;
            return CSBQ_EHIP;
        }
        ctx->own_stream = true;
    }
    double D[NS * NS], T[NS * NS];
    gl_tables(NS, ctx->gx, ctx->gw, ctx->lam, D, T);
    std::memcpy(ctx->Dgl, D, sizeof D);
    if (int uc = upload_constants(ctx->gx, ctx->gw, ctx->lam, D, T)) {
        std::fprintf(stderr, "csbq_create: constant upload failed (%d: %s)\n", uc,
                     hipGetErrorString(hipGetLastError()));
        csbq_destroy(ctx);
        return CSBQ_EHIP;
    }
    int rc = load_tables(ctx);
    if (!rc && ctx->opt.srule != CSBQ_SRULE_GENERAL) rc = load_srules(ctx);
    if (rc) {
        std::fprintf(stderr, "csbq: %s\n", ctx->err.c_str());
        csbq_destroy(ctx);
        return rc;
    }
    ctx->gc.tol = ctx->opt.quad_tol;
    ctx->gc.cs = 1000.0;
    ctx->gc.ct = 1000.0;
    ctx->gc.hmin_fac = 1.0;
    ctx->gc.extra_modes = 2;
    ctx->closed_fb = 2;
    {
        void* sp = nullptr;
        if (int se = scratch_address(ctx->opt.device, &sp)) {
            std::fprintf(stderr, "csbq_create: scratch address lookup failed (%s)\n",
                         hipGetErrorString((hipError_t)se));
            csbq_destroy(ctx);
            return CSBQ_EHIP;
        }
        ctx->scratch = (unsigned char*)sp;
    }
    for (int k = 0; k < kNPhase; ++k) {
        ctx->ph[k].name = kPhaseNames[k];
        (void)hipEventCreate(&ctx->ph[k].a);
        (void)hipEventCreate(&ctx->ph[k].b);
    }
    *out = ctx;
    return CSBQ_OK;
}

int csbq_destroy(csbq_ctx* ctx)
{
    if (!ctx) return CSBQ_EINVAL;
    (void)hipSetDevice(ctx->opt.device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int k = 0; k < kNPhase; ++k) {
        if (ctx->ph[k].a) (void)hipEventDestroy(ctx->ph[k].a);
        if (ctx->ph[k].b) (void)hipEventDestroy(ctx->ph[k].b);
    }
    ctx->roff.release();
    ctx->rth.release();
    ctx->rw.release();
    ctx->lx.release();
    ctx->lw.release();
    ctx->rcs.release();
    ctx->rsn.release();
    ctx->romc.release();
    ctx->woff.release();
    ctx->wd.release();
    ctx->ww.release();
    ctx->g_xc.release();
    ctx->g_eps.release();
    ctx->g_e1.release();
    ctx->g_sa.release();
    ctx->g_sc.release();
    ctx->g_sign.release();
    ctx->g_body.release();
    ctx->clq.release();
    ctx->circ.release();
    ctx->gridc.release();
    ctx->ny.release();
    ctx->nn.release();
    ctx->nw.release();
    ctx->info.release();
    ctx->boff.release();
    ctx->by.release();
    ctx->bn.release();
    ctx->bw.release();
    ctx->bsw.release();
    for (int k = 0; k < NUP; ++k) {
        ctx->cpy[k].release();
        ctx->cpn[k].release();
        ctx->cpw[k].release();
        ctx->Lup[k].release();
        ctx->upx[k].release();
        ctx->upw[k].release();
        ctx->swf[k].release();
    }
    ctx->wdesc.release();
    ctx->sig_d.release();
    ctx->x_d.release();
    ctx->usl_d.release();
    ctx->udl_d.release();
    ctx->tn_d.release();
    ctx->sw.release();
    ctx->sh.release();
    ctx->rnear.release();
    ctx->xt.release();
    ctx->part.release();
    ctx->cls.release();
    ctx->corr.release();
    ctx->band.release();
    ctx->cnt.release();
    ctx->pe.release();
    ctx->pt.release();
    ctx->kin.release();
    ctx->kout.release();
    ctx->vin.release();
    ctx->perm.release();
    ctx->sorted.release();
    ctx->runs_key.release();
    ctx->runs_cnt.release();
    ctx->nruns.release();
    ctx->err_d.release();
    ctx->work.release();
    ctx->off.release();
    ctx->tier.release();
    ctx->cub_tmp.release();
    plan_drop(ctx);
    if (ctx->plan.e0) (void)hipEventDestroy(ctx->plan.e0);
    if (ctx->plan.e1) (void)hipEventDestroy(ctx->plan.e1);
    if (ctx->plan.gst) (void)hipStreamDestroy(ctx->plan.gst);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return CSBQ_OK;
}

int csbq_synchronize(csbq_ctx* ctx)
{
    if (!ctx) return CSBQ_EINVAL;
    HIPC(hipStreamSynchronize(ctx->stream));
    return CSBQ_OK;
}

int csbq_eval_flags(csbq_ctx* ctx, int32_t* flags)
{
    if (!ctx || !flags) return CSBQ_EINVAL;
    if (ctx->flags_pending && ctx->flags_src) {
        int f = 0;
        HIPC(hipSetDevice(ctx->opt.device));
        HIPC(hipMemcpyAsync(&f, ctx->flags_src, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        ctx->last_err_flags = f;
        ctx->flags_pending = false;
    }
    *flags = ctx->last_err_flags;
    return CSBQ_OK;
}

int csbq_num_nodes(const csbq_ctx* ctx, int64_t* n)
{
    if (!ctx || !n) return CSBQ_EINVAL;
    if (!ctx->have_geom) return CSBQ_ESTATE;
    *n = ctx->N;
    return CSBQ_OK;
}

}  // extern "C"

// copy `n` elements from caller memory (host or device) into a device buffer
template <typename T>
static int to_device(csbq_ctx* ctx, DBuf<T>& buf, const T* src, size_t n, int mem)
{
    ALLOC(buf, n);
    if (n == 0) return CSBQ_OK;
    HIPC(hipMemcpyAsync(buf.p, src, n * sizeof(T), mem == CSBQ_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        ctx->stream));
    return CSBQ_OK;
}

extern "C" {

int csbq_set_geometry(csbq_ctx* ctx, int32_t n_bodies, const int32_t* n_panels, const int32_t* normal_sign,
                      const double* s_break, const double* xc, const double* eps, const double* e1, int32_t ns,
                      int32_t nt, int mem)
{
    return csbq_set_geometry_batch(ctx, n_bodies, nullptr, n_panels, normal_sign, s_break, xc, eps, e1, ns, nt, mem);
}

int csbq_set_geometry_batch(csbq_ctx* ctx, int32_t n_bodies, const int32_t* body_group, const int32_t* n_panels,
                            const int32_t* normal_sign, const double* s_break, const double* xc, const double* eps,
                            const double* e1, int32_t ns, int32_t nt, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (ns != NS || nt != NT) return ctx->fail(CSBQ_EINVAL, "the library supports ns=16, nt=32 only");
    if (n_bodies < 1 || !n_panels || !normal_sign || !s_break || !xc || !eps || !e1)
        return ctx->fail(CSBQ_EINVAL, "missing geometry arrays");
    if (mem != CSBQ_HOST && mem != CSBQ_DEVICE) return ctx->fail(CSBQ_EINVAL, "bad mem flag");
    HIPC(hipSetDevice(ctx->opt.device));
    plan_drop(ctx);
    ctx->have_geom = false;
    // body tables are small: bring them to the host for validation
    std::vector<int32_t> np(n_bodies), sg(n_bodies), bg(n_bodies, 0);
    if (mem == CSBQ_DEVICE) {
        HIPC(hipMemcpy(np.data(), n_panels, n_bodies * 4, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(sg.data(), normal_sign, n_bodies * 4, hipMemcpyDeviceToHost));
        if (body_group) HIPC(hipMemcpy(bg.data(), body_group, n_bodies * 4, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(np.data(), n_panels, n_bodies * 4);
        std::memcpy(sg.data(), normal_sign, n_bodies * 4);
        if (body_group) std::memcpy(bg.data(), body_group, n_bodies * 4);
    }
    if (bg[0] != 0) return ctx->fail(CSBQ_EINVAL, "body_group must start at 0");
    for (int b = 1; b < n_bodies; ++b)
        if (bg[b] != bg[b - 1] && bg[b] != bg[b - 1] + 1)
            return ctx->fail(CSBQ_EINVAL, "body_group must be non-decreasing without gaps");
    const int G = bg[n_bodies - 1] + 1;
    int64_t E = 0, nsb = 0;
    for (int b = 0; b < n_bodies; ++b) {
        if (np[b] < 1) return ctx->fail(CSBQ_EINVAL, "a body has no panel");
        if (sg[b] != 1 && sg[b] != -1) return ctx->fail(CSBQ_EINVAL, "normal_sign must be +1 or -1");
        E += np[b];
        nsb += np[b] + 1;
    }
    if (E > (1 << 26)) return ctx->fail(CSBQ_EINVAL, "too many panels");
    std::vector<double> sb(nsb), h_eps((size_t)E * NS), h_xc((size_t)E * NS * 3), h_e1((size_t)E * NS * 3);
    if (mem == CSBQ_DEVICE) {
        HIPC(hipMemcpy(sb.data(), s_break, nsb * 8, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(h_eps.data(), eps, h_eps.size() * 8, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(h_xc.data(), xc, h_xc.size() * 8, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(h_e1.data(), e1, h_e1.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(sb.data(), s_break, nsb * 8);
        std::memcpy(h_eps.data(), eps, h_eps.size() * 8);
        std::memcpy(h_xc.data(), xc, h_xc.size() * 8);
        std::memcpy(h_e1.data(), e1, h_e1.size() * 8);
    }
    std::vector<double> sa(E), sc(E);
    std::vector<int> es(E), eb(E), eg(E), gel(G + 1, 0);
    int64_t k = 0, o = 0;
    for (int b = 0; b < n_bodies; ++b) {
        for (int p = 0; p < np[b]; ++p, ++k) {
            sa[k] = sb[o + p];
            sc[k] = sb[o + p + 1];
            if (!(sc[k] > sa[k]) || !std::isfinite(sa[k]) || !std::isfinite(sc[k]))
                return ctx->fail(CSBQ_EINVAL, "panel end points must increase");
            es[k] = sg[b];
            eb[k] = b;
            eg[k] = bg[b];
        }
        o += np[b] + 1;
        gel[bg[b] + 1] = (int)k;
    }
    for (double v : h_eps)
        if (!(v > 0) || !std::isfinite(v)) return ctx->fail(CSBQ_EINVAL, "eps must be positive and finite");
    ctx->E = (int)E;
    ctx->N = E * NPE;
    const int64_t N = ctx->N;
    int rc;
    if ((rc = to_device(ctx, ctx->g_xc, xc, (size_t)E * NS * 3, mem))) return rc;
    if ((rc = to_device(ctx, ctx->g_eps, eps, (size_t)E * NS, mem))) return rc;
    if ((rc = to_device(ctx, ctx->g_e1, e1, (size_t)E * NS * 3, mem))) return rc;
    if ((rc = to_device(ctx, ctx->g_sa, sa.data(), (size_t)E, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, ctx->g_sc, sc.data(), (size_t)E, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, ctx->g_sign, es.data(), (size_t)E, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, ctx->g_body, eb.data(), (size_t)E, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, ctx->g_group, eg.data(), (size_t)E, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, ctx->gel, gel.data(), (size_t)G + 1, CSBQ_HOST))) return rc;
    ctx->G = G;
    ctx->h_gel = gel;
    ctx->n_bodies = n_bodies;
    ctx->h_body_off.assign((size_t)n_bodies + 1, 0);
    for (int b = 0; b < n_bodies; ++b) ctx->h_body_off[b + 1] = ctx->h_body_off[b] + (int64_t)np[b] * NPE;
    ctx->tuned_key = 0;
    ctx->tiles_valid = false;
    ALLOC(ctx->clq, (size_t)E * CLQ * NS);
    ALLOC(ctx->circ, (size_t)E * NCIRC * CIRQ);
    ALLOC(ctx->info, (size_t)E);
    ALLOC(ctx->ny, (size_t)N * 3);
    ALLOC(ctx->nn, (size_t)N * 3);
    ALLOC(ctx->nw, (size_t)N);
    LCHK(launch_expand(ctx->stream, (int)E, ctx->g_xc.p, ctx->g_eps.p, ctx->g_e1.p, ctx->g_sa.p, ctx->g_sc.p,
                       ctx->g_sign.p, ctx->g_body.p, ctx->g_group.p, ctx->clq.p, ctx->circ.p, ctx->info.p, ctx->ny.p, ctx->nn.p,
                       ctx->nw.p, N, ctx->closed_fb));
    ALLOC(ctx->gridc, (size_t)E * NCIRC * CGRID * GRQ);
    LCHK(launch_grid_circles(ctx->stream, (int)E, ctx->clq.p, ctx->gridc.p));
    // upsampled whole-panel rules (Gauss-Legendre of up_ns points in s times
    // up_nt angles) and the Lagrange matrices from the NS panel nodes to them
    for (int ti = 0; ti < NUP; ++ti) {
        const int nsf = up_ns(ti), ntf = up_nt(ti);
        ctx->Mtot[ti] = E * up_pts(ti);
        ALLOC(ctx->cpy[ti], (size_t)ctx->Mtot[ti] * 3);
        ALLOC(ctx->cpn[ti], (size_t)ctx->Mtot[ti] * 3);
        ALLOC(ctx->cpw[ti], (size_t)ctx->Mtot[ti]);
        std::vector<double> gxf(nsf), gwf(nsf), lamf(nsf), Df((size_t)nsf * nsf), Tf((size_t)nsf * nsf);
        gl_tables(nsf, gxf.data(), gwf.data(), lamf.data(), Df.data(), Tf.data());
        std::vector<double> L((size_t)nsf * NS);
        for (int p = 0; p < nsf; ++p) lagrange_row(NS, ctx->gx, ctx->lam, gxf[p], &L[(size_t)p * NS]);
        ALLOC(ctx->Lup[ti], L.size());
        ALLOC(ctx->upx[ti], (size_t)nsf);
        ALLOC(ctx->upw[ti], (size_t)nsf);
        HIPC(hipMemcpy(ctx->Lup[ti].p, L.data(), L.size() * 8, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->upx[ti].p, gxf.data(), nsf * 8, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->upw[ti].p, gwf.data(), nsf * 8, hipMemcpyHostToDevice));
        LCHK(launch_expand_up(ctx->stream, (int)E, nsf, ntf, ctx->upx[ti].p, ctx->upw[ti].p, ctx->clq.p, ctx->info.p,
                              ctx->cpy[ti].p, ctx->cpn[ti].p, ctx->cpw[ti].p, ctx->Mtot[ti]));
    }
    // Gauss tables and Lagrange matrices of the coarser far-field rules
    for (int i = 0; i < NFS; ++i) {
        const int nsf = far_ns(i);
        std::vector<double> gxf(nsf), gwf(nsf), lamf(nsf), Df((size_t)nsf * nsf), Tf((size_t)nsf * nsf);
        gl_tables(nsf, gxf.data(), gwf.data(), lamf.data(), Df.data(), Tf.data());
        std::vector<double> L((size_t)nsf * NS);
        for (int p = 0; p < nsf; ++p) lagrange_row(NS, ctx->gx, ctx->lam, gxf[p], &L[(size_t)p * NS]);
        ALLOC(ctx->Lfar[i], L.size());
        ALLOC(ctx->farx[i], (size_t)nsf);
        ALLOC(ctx->farw[i], (size_t)nsf);
        HIPC(hipMemcpy(ctx->Lfar[i].p, L.data(), L.size() * 8, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->farx[i].p, gxf.data(), nsf * 8, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->farw[i].p, gwf.data(), nsf * 8, hipMemcpyHostToDevice));
    }
    // base (far-field) source set: own nodes, or the tier-0 rule for elements
    // whose cross-section closes at an end
    {
        std::vector<ElemInfo> hinf((size_t)E);
        HIPC(hipStreamSynchronize(ctx->stream));
        HIPC(hipMemcpy(hinf.data(), ctx->info.p, (size_t)E * sizeof(ElemInfo), hipMemcpyDeviceToHost));
        // shapes with tabulated whole-element singular s-rules
        int64_t nshape[3] = {0, 0, 0};
        std::vector<double> htor((size_t)E * TOR_Q);
        for (int64_t e = 0; e < E; ++e) {
            element_torus(&h_xc[(size_t)e * NS * 3], &h_eps[(size_t)e * NS], ctx->gx, &htor[(size_t)e * TOR_Q]);
            hinf[e].shape = element_shape(&h_xc[(size_t)e * NS * 3], &h_eps[(size_t)e * NS], &h_e1[(size_t)e * NS * 3],
                                          ctx->gx, ctx->Dgl);
            ++nshape[hinf[e].shape];
        }
        HIPC(hipMemcpy(ctx->info.p, hinf.data(), (size_t)E * sizeof(ElemInfo), hipMemcpyHostToDevice));
        ALLOC(ctx->tor, htor.size());
        HIPC(hipMemcpy(ctx->tor.p, htor.data(), htor.size() * sizeof(double), hipMemcpyHostToDevice));
        ctx->n_tor = 0;
        for (int64_t e = 0; e < E; ++e) ctx->n_tor += htor[(size_t)e * TOR_Q + TOR_Q - 1] != 0.0;
        ctx->n_cyl = nshape[SHAPE_CYLINDER];
        ctx->n_sph = nshape[SHAPE_SPHERE];
        // the base rules, then each element's coarser far-field rules (rule k
        // of element e at loff[k E + e], -1 where the element has none)
        std::vector<int64_t> bo((size_t)E + 1, 0);
        for (int64_t e = 0; e < E; ++e) bo[e + 1] = bo[e] + (hinf[e].fb == 2 ? up_pts(0) : NPE);
        ctx->Nb_rules = bo[E];
        std::vector<int64_t> lo((size_t)NFL * E, -1);
        int64_t nb = bo[E];
        for (int k = 0; k < NFL; ++k) ctx->far_used[k] = false;
        for (int64_t e = 0; e < E; ++e) {
            const int i0 = far_i0(hinf[e].fb == 2);
            for (int i = i0; i < i0 + FAR_NI; ++i)
                for (int j = 0; j < NFT; ++j) {
                    const int k = i * NFT + j;
                    if (hinf[e].fb != 2 && k == FAR_OPEN_BASE) continue;   // the base rule itself
                    lo[(size_t)k * E + e] = nb;
                    nb += far_pts(k);
                    ctx->far_used[k] = true;
                }
        }
        ctx->Nb = nb;
        ctx->h_boff = bo;
        ALLOC(ctx->boff, bo.size());
        ALLOC(ctx->loff, lo.size());
        ALLOC(ctx->by, (size_t)ctx->Nb * 3);
        ALLOC(ctx->bn, (size_t)ctx->Nb * 3);
        ALLOC(ctx->bw, (size_t)ctx->Nb);
        HIPC(hipMemcpy(ctx->boff.p, bo.data(), bo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(ctx->loff.p, lo.data(), lo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        LCHK(launch_base_build(ctx->stream, (int)E, ctx->info.p, ctx->boff.p, ctx->ny.p, ctx->nn.p, ctx->nw.p, N,
                               ctx->cpy[0].p, ctx->cpn[0].p, ctx->cpw[0].p, ctx->Mtot[0], ctx->by.p, ctx->bn.p,
                               ctx->bw.p, ctx->Nb));
        for (int k = 0; k < NFL; ++k)
            if (ctx->far_used[k])
                LCHK(launch_expand_up(ctx->stream, (int)E, far_ns(k / NFT), far_nt(k % NFT), ctx->farx[k / NFT].p,
                                      ctx->farw[k / NFT].p, ctx->clq.p, ctx->info.p, ctx->by.p, ctx->bn.p, ctx->bw.p,
                                      ctx->Nb, ctx->loff.p + (int64_t)k * E));
        // mixed precision: sources within sqrt(100 w_max) of a target are
        // summed in FP64, so no FP32 term exceeds ~1e-2 of the density scale
        // (w_max over the base rules: the coarser rules are summed only far
        // from their elements)
        std::vector<double> hbw((size_t)ctx->Nb_rules);
        HIPC(hipMemcpyAsync(hbw.data(), ctx->bw.p, hbw.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        double wmax = 0.0;
        for (double w : hbw) wmax = std::max(wmax, std::fabs(w));
        ctx->mix_near2 = 100.0 * wmax;
    }
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->have_geom = true;
    return CSBQ_OK;
}

int csbq_get_nodes(csbq_ctx* ctx, double* y, double* normal, double* weight, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    if (!ctx->have_geom) return ctx->fail(CSBQ_ESTATE, "no geometry");
    const int64_t N = ctx->N;
    std::vector<double> h((size_t)N * 3);
    auto kind = mem == CSBQ_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    // SoA on the device -> AoS for the caller
    DBuf<double> tmp;
    if (tmp.ensure((size_t)N * 3) != hipSuccess) return ctx->fail(CSBQ_ENOMEM, "alloc");
    const double* srcs[2] = {ctx->ny.p, ctx->nn.p};
    double* dsts[2] = {y, normal};
    for (int q = 0; q < 2; ++q) {
        if (!dsts[q]) continue;
        std::vector<double> soa((size_t)N * 3);
        HIPC(hipMemcpy(soa.data(), srcs[q], (size_t)N * 3 * 8, hipMemcpyDeviceToHost));
        for (int64_t n = 0; n < N; ++n)
            for (int d = 0; d < 3; ++d) h[n * 3 + d] = soa[d * N + n];
        HIPC(hipMemcpy(dsts[q], h.data(), (size_t)N * 3 * 8,
                       mem == CSBQ_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    }
    if (weight) HIPC(hipMemcpy(weight, ctx->nw.p, (size_t)N * 8, kind));
    tmp.release();
    return CSBQ_OK;
}

// common front part: inputs on the device, targets, density preparation
static int eval_front(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                      const int32_t* tgt_group, int mem, const double** sig_dev, const int64_t** tn_dev)
{
    if (!ctx->have_geom) return ctx->fail(CSBQ_ESTATE, "set_geometry must be called first");
    if (!sigma || T < 0) return ctx->fail(CSBQ_EINVAL, "missing density or negative target count");
    if (!x && !tgt_node && T > 0) return ctx->fail(CSBQ_EINVAL, "targets need x or tgt_node");
    if (mem != CSBQ_HOST && mem != CSBQ_DEVICE) return ctx->fail(CSBQ_EINVAL, "bad mem flag");
    if (T > (int64_t)INT32_MAX) return ctx->fail(CSBQ_EINVAL, "too many targets");
    const int64_t N = ctx->N;
    const int nc = ctx->nc();
    if (mem == CSBQ_HOST) {
        for (int64_t i = 0; i < N * nc; ++i)
            if (!std::isfinite(sigma[i])) return ctx->fail(CSBQ_EINVAL, "density has NaN/Inf");
        if (tgt_node)
            for (int64_t t = 0; t < T; ++t)
                if (tgt_node[t] >= N) return ctx->fail(CSBQ_EINVAL, "tgt_node out of range");
        if (x)
            for (int64_t t = 0; t < T; ++t)
                if ((!tgt_node || tgt_node[t] < 0) &&
                    !(std::isfinite(x[3 * t]) && std::isfinite(x[3 * t + 1]) && std::isfinite(x[3 * t + 2])))
                    return ctx->fail(CSBQ_EINVAL, "target has NaN/Inf");
        if (!x && tgt_node)
            for (int64_t t = 0; t < T; ++t)
                if (tgt_node[t] < 0) return ctx->fail(CSBQ_EINVAL, "free target without coordinates");
        int rc;
        if (nc == 3) {
            if ((rc = to_device(ctx, ctx->sig_d, sigma, (size_t)N * 3, CSBQ_HOST))) return rc;
        } else {
            // the scalar (Laplace) density into the first of three components
            if ((rc = to_device(ctx, ctx->sig1, sigma, (size_t)N, CSBQ_HOST))) return rc;
            ALLOC(ctx->sig_d, (size_t)N * 3);
            LCHK(launch_scalar_to_vec(ctx->stream, N, ctx->sig1.p, ctx->sig_d.p));
        }
        *sig_dev = ctx->sig_d.p;
        if (x) {
            if ((rc = to_device(ctx, ctx->x_d, x, (size_t)T * 3, CSBQ_HOST))) return rc;
            x = ctx->x_d.p;
        }
        if (tgt_node) {
            if ((rc = to_device(ctx, ctx->tn_d, tgt_node, (size_t)T, CSBQ_HOST))) return rc;
            tgt_node = ctx->tn_d.p;
        }
        if (tgt_group) {
            for (int64_t t = 0; t < T; ++t)
                if (tgt_group[t] < 0 || tgt_group[t] >= ctx->G) return ctx->fail(CSBQ_EINVAL, "tgt_group out of range");
            if ((rc = to_device(ctx, ctx->tgrp_d, tgt_group, (size_t)T, CSBQ_HOST))) return rc;
            tgt_group = ctx->tgrp_d.p;
        }
    } else if (nc == 3) {
        *sig_dev = sigma;
    } else {
        ALLOC(ctx->sig_d, (size_t)N * 3);
        LCHK(launch_scalar_to_vec(ctx->stream, N, sigma, ctx->sig_d.p));
        *sig_dev = ctx->sig_d.p;
    }
    *tn_dev = tgt_node;
    ALLOC(ctx->err_d, 1);
    HIPC(hipMemsetAsync(ctx->err_d.p, 0, sizeof(int), ctx->stream));
    ALLOC(ctx->xt, (size_t)T * 3 + 1);
    ALLOC(ctx->tgroup, (size_t)T + 1);
    ALLOC(ctx->gstart, (size_t)ctx->G);
    LCHK(launch_targets(ctx->stream, T, x, tgt_node, tgt_group, ctx->G, ctx->info.p, ctx->ny.p, N, ctx->xt.p,
                        ctx->tgroup.p, ctx->gstart.p, ctx->err_d.p));
    const int E = ctx->E;
    ALLOC(ctx->sw, (size_t)N * 3);
    ALLOC(ctx->sh, (size_t)E * NS * NSH);
    ALLOC(ctx->band, (size_t)E * 2);
    ALLOC(ctx->rnear, (size_t)E * (NFS + NFT));
    // (a negative threshold asks for the full band: see csbq_ctx::full_band)
    LCHK(launch_prep_sigma(ctx->stream, E, *sig_dev, ctx->nw.p, N, ctx->sw.p, ctx->sh.p, ctx->band.p,
                           ctx->full_band ? -1.0 : 0.1 * ctx->gc.tol, ctx->info.p, ctx->circ.p, ctx->gc,
                           ctx->rnear.p));
    return CSBQ_OK;
}

// Target range of every group, [tr[g], tr[g+1]), from the device's first-target
// table (after a stream synchronisation); fails on unordered targets.
static int group_ranges(csbq_ctx* ctx, int64_t T, int flags, std::vector<int64_t>& tr)
{
    if (flags & CSBQ_FLAG_GROUP_RANGE) return ctx->fail(CSBQ_EINVAL, "target group out of range");
    if (flags & CSBQ_FLAG_GROUP_ORDER) return ctx->fail(CSBQ_EINVAL, "targets must be ordered by group");
    const int G = ctx->G;
    tr.assign((size_t)G + 1, 0);
    tr[G] = T;
    if (G == 1) return CSBQ_OK;
    std::vector<int64_t> gs((size_t)G);
    HIPC(hipMemcpy(gs.data(), ctx->gstart.p, (size_t)G * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int g = G - 1; g >= 0; --g) tr[g] = gs[g] >= 0 ? gs[g] : tr[g + 1];
    return CSBQ_OK;
}

// Smooth-sum blocks: per group, blocks of 256*tpt consecutive targets times
// chunks of `chunk` sources, ordered by cost (largest first) so that one
// launch drains a batch of unequal geometries evenly.
// the context's upsampled rules of every tier, as the corrections kernel takes them
static UpRules up_rules(const csbq_ctx* ctx)
{
    UpRules ur{};
    for (int k = 0; k < NUP; ++k) {
        ur.y[k] = ctx->cpy[k].p;
        ur.n[k] = ctx->cpn[k].p;
        ur.sw[k] = ctx->swf[k].p;
        ur.Mf[k] = up_pts(k);
        ur.Mtot[k] = ctx->Mtot[k];
    }
    return ur;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2: block i runs on XCD i mod 8.  Within each run of equal-cost tiles
// (the cost order is kept for load balance), tiles are re-placed so that the
// blocks of one XCD take source chunks s0/chunk = XCD (mod 8), chunk by
// chunk: an XCD then streams one or two chunks (a few hundred KB) at a time
// from its L2 instead of every chunk of the sum from HBM.
static void xcd_order(std::vector<FarTile>& tiles, int64_t chunk)
{
    constexpr int NX = 8;
    std::vector<FarTile> q[NX];
    size_t i0 = 0;
    while (i0 < tiles.size()) {
        const int64_t cost = (int64_t)tiles[i0].tn * tiles[i0].sn;
        size_t i1 = i0;
        while (i1 < tiles.size() && (int64_t)tiles[i1].tn * tiles[i1].sn == cost) ++i1;
        for (auto& v : q) v.clear();
        for (size_t i = i0; i < i1; ++i) q[(tiles[i].s0 / chunk) % NX].push_back(tiles[i]);
        for (auto& v : q)
            std::stable_sort(v.begin(), v.end(), [](const FarTile& a, const FarTile& b) {
                return a.s0 != b.s0 ? a.s0 < b.s0 : a.t0 < b.t0;
            });
        size_t head[NX] = {};
        for (size_t i = i0; i < i1; ++i) {
            int x = (int)(i % NX);
            if (head[x] == q[x].size()) {   // this XCD's share is used up: take from the fullest
                size_t best = 0;
                for (int y = 0; y < NX; ++y)
                    if (q[y].size() - head[y] > best) {
                        best = q[y].size() - head[y];
                        x = y;
                    }
            }
            tiles[i] = q[x][head[x]++];
        }
        i0 = i1;
    }
}

static void far_tiles(const csbq_ctx* ctx, const std::vector<int64_t>& tr, bool native, int tpt, int64_t chunk,
                      int g_only, int64_t t_cap, std::vector<FarTile>& tiles, std::vector<int>& gnc, int* maxchunk)
{
    const int G = ctx->G;
    tiles.clear();
    gnc.assign((size_t)G, 0);
    *maxchunk = 0;
    const int64_t tb = 256LL * tpt;
    struct Chunk {
        int64_t s0, sn;
        int e0, e1;
    };
    std::vector<Chunk> ch;
    for (int g = 0; g < G; ++g) {
        if (g_only >= 0 && g != g_only) continue;
        const int64_t t0 = tr[g], tn = std::min(tr[g + 1] - tr[g], t_cap);
        const int e0 = ctx->h_gel[g], e1 = ctx->h_gel[g + 1];
        ch.clear();
        if (native) {   // plain source ranges of the element nodes
            const int64_t s0 = (int64_t)e0 * NPE, S = (int64_t)(e1 - e0) * NPE;
            for (int64_t a = 0; a < S; a += chunk) ch.push_back(Chunk{s0 + a, std::min(chunk, S - a), 0, 0});
        } else {        // whole elements, up to `chunk` base sources each (at least one element)
            int ea = e0;
            while (ea < e1) {
                int eb = ea + 1;
                while (eb < e1 && ctx->h_boff[eb + 1] - ctx->h_boff[ea] <= chunk) ++eb;
                ch.push_back(Chunk{ctx->h_boff[ea], ctx->h_boff[eb] - ctx->h_boff[ea], ea, eb});
                ea = eb;
            }
        }
        const int nch = (int)ch.size();
        gnc[g] = nch;
        *maxchunk = std::max(*maxchunk, nch);
        for (int64_t a = 0; a < tn; a += tb)
            for (int c = 0; c < nch; ++c)
                tiles.push_back(FarTile{t0 + a, ch[c].s0, (int32_t)std::min(tb, tn - a), (int32_t)ch[c].sn, c,
                                        ch[c].e0, ch[c].e1, 0});
    }
    std::stable_sort(tiles.begin(), tiles.end(), [](const FarTile& a, const FarTile& b) {
        return (int64_t)a.tn * a.sn > (int64_t)b.tn * b.sn;
    });
    xcd_order(tiles, chunk);
}

// the element chunks' choice of source set (closed elements' coarser rules
// beyond rc), with the per-block pair counts written to `pairs`
static FarSplit far_split(const csbq_ctx* ctx, int64_t* pairs)
{
    FarSplit f{};
    f.boff = ctx->boff.p;
    f.loff = ctx->loff.p;
    f.rc = ctx->far_split ? ctx->rnear.p + ctx->E : nullptr;
    f.info = ctx->info.p;
    f.pairs = pairs;
    f.E = ctx->E;
    return f;
}

// Launch shape of the smooth sum, chosen by timing: targets per thread 1/2/4
// times 8192/32768 sources per chunk, each timed once on the largest group
// (its first 4e10 / sources targets at most, so that a sample still fills
// the device with thousands of blocks); cached per (targets, sources,
// precision).  Small sums keep the default shape.
static int tune_far(csbq_ctx* ctx, int64_t T, const std::vector<int64_t>& tr, bool native, bool mixed)
{
    const uint64_t key = ((uint64_t)T * 1000003ULL) ^ ((uint64_t)(native ? ctx->N : ctx->Nb) << 20) ^
                         ((uint64_t)ctx->G << 50) ^ (mixed ? 7ULL : 3ULL) ^ (native ? 11ULL : 0ULL);
    if (ctx->tuned_key == key) return CSBQ_OK;
    ctx->tuned_key = key;
    ctx->tiles_valid = false;   // the timing passes reuse the block buffer
    int gbig = 0;
    double pbig = -1, ptot = 0;
    for (int g = 0; g < ctx->G; ++g) {
        const int e0 = ctx->h_gel[g], e1 = ctx->h_gel[g + 1];
        const double S = native ? (double)(e1 - e0) * NPE : (double)(ctx->h_boff[e1] - ctx->h_boff[e0]);
        const double pr = S * (double)(tr[g + 1] - tr[g]);
        ptot += pr;
        if (pr > pbig) {
            pbig = pr;
            gbig = g;
        }
    }
    ctx->far_tpt = 2;
    ctx->far_chunk = 16384;
    if (ptot < 2e8) return CSBQ_OK;
    const int e0 = ctx->h_gel[gbig], e1 = ctx->h_gel[gbig + 1];
    const int64_t S = native ? (int64_t)(e1 - e0) * NPE : ctx->h_boff[e1] - ctx->h_boff[e0];
    const int64_t t_cap = std::max<int64_t>(16384, (int64_t)(4e10 / std::max<int64_t>(S, 1))) / 1024 * 1024;
    const double* sy = native ? ctx->ny.p : ctx->by.p;
    const double* sn = native ? ctx->nn.p : ctx->bn.p;
    const double* ss = native ? ctx->sw.p : ctx->bsw.p;
    const int64_t Ns = native ? ctx->N : ctx->Nb;
    const int tpts[3] = {1, 2, 4};
    const int64_t chunks[2] = {8192, 32768};
    hipEvent_t a, b;
    HIPC(hipEventCreate(&a));
    HIPC(hipEventCreate(&b));
    float best = 1e30f;
    std::vector<FarTile> tl;
    std::vector<int> gnc;
    for (int pass = -1; pass < 6; ++pass) {
        const int tpt = tpts[pass < 0 ? 1 : pass / 2];
        const int64_t chunk = chunks[pass < 0 ? 0 : pass % 2];
        int maxch = 0;
        far_tiles(ctx, tr, native, tpt, chunk, gbig, t_cap, tl, gnc, &maxch);
        ALLOC(ctx->tiles, tl.size() + 1);
        HIPC(hipMemcpyAsync(ctx->tiles.p, tl.data(), tl.size() * sizeof(FarTile), hipMemcpyHostToDevice, ctx->stream));
        ALLOC(ctx->part, (size_t)std::max(maxch, 1) * 6 * T + 1);
        HIPC(hipEventRecord(a, ctx->stream));
        LCHK(launch_far(ctx->stream, T, ctx->xt.p, sy, sn, ss, Ns, ctx->tiles.p, (int)tl.size(), ctx->part.p, mixed,
                        ctx->mix_near2, tpt, ctx->ker, native ? FarSplit{} : far_split(ctx, nullptr)));
        HIPC(hipEventRecord(b, ctx->stream));
        HIPC(hipEventSynchronize(b));
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, a, b));
        if (pass < 0) continue;   // warm-up of the code object
        ctx->tune_ms[pass] = ms;
        if (ms < best) {
            best = ms;
            ctx->far_tpt = tpt;
            ctx->far_chunk = chunk;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return CSBQ_OK;
}

// smooth sum over a source set: the element nodes (native) or the base set
// The smooth sum over a source set, enqueued on `st` (tuned on the
// context's stream first): the element nodes (native, a diagnostic, always
// FP64) or the base set (the context's precision).
static int far_sum(csbq_ctx* ctx, int64_t T, bool native, const std::vector<int64_t>& tr, hipStream_t st,
                   hipEvent_t ev_start = nullptr)
{
    const bool mixed = !native && ctx->opt.precision == CSBQ_MIXED;
    int rc;
    if ((rc = tune_far(ctx, T, tr, native, mixed))) return rc;
    const int64_t Ns = native ? ctx->N : ctx->Nb;
    const double* sy = native ? ctx->ny.p : ctx->by.p;
    const double* sn = native ? ctx->nn.p : ctx->bn.p;
    const double* ss = native ? ctx->sw.p : ctx->bsw.p;
    // the blocks depend only on the geometry, the targets' group ranges and
    // the launch shape: built and uploaded again only when one changed
    const bool same = ctx->tiles_valid && ctx->tiles_native == native && ctx->tiles_tpt == ctx->far_tpt &&
                      ctx->tiles_chunk == ctx->far_chunk && ctx->tiles_T == T && ctx->tiles_tr == tr;
    if (!same) {
        ctx->tiles_valid = false;
        far_tiles(ctx, tr, native, ctx->far_tpt, ctx->far_chunk, -1, INT64_MAX, ctx->h_tiles, ctx->h_gnc,
                  &ctx->tiles_maxch);
        ALLOC(ctx->tiles, ctx->h_tiles.size() + 1);
        ALLOC(ctx->gnchunk, ctx->h_gnc.size());
        HIPC(hipMemcpyAsync(ctx->tiles.p, ctx->h_tiles.data(), ctx->h_tiles.size() * sizeof(FarTile),
                            hipMemcpyHostToDevice, st));
        HIPC(hipMemcpyAsync(ctx->gnchunk.p, ctx->h_gnc.data(), ctx->h_gnc.size() * sizeof(int), hipMemcpyHostToDevice,
                            st));
        ctx->tiles_valid = true;
        ctx->tiles_native = native;
        ctx->tiles_tpt = ctx->far_tpt;
        ctx->tiles_chunk = ctx->far_chunk;
        ctx->tiles_T = T;
        ctx->tiles_tr = tr;
        ctx->last_far_pairs = 0;
        for (const auto& t : ctx->h_tiles) ctx->last_far_pairs += (int64_t)t.tn * t.sn;
    }
    const auto& tl = ctx->h_tiles;
    ALLOC(ctx->part, (size_t)std::max(ctx->tiles_maxch, 1) * 6 * T + 1);
    ALLOC(ctx->fpairs, tl.size() + 1);
    if (ev_start) HIPC(hipEventRecord(ev_start, st));
    if (T > 0)
        LCHK(launch_far(st, T, ctx->xt.p, sy, sn, ss, Ns, ctx->tiles.p, (int)tl.size(), ctx->part.p, mixed,
                        ctx->mix_near2, ctx->far_tpt, ctx->ker, native ? FarSplit{} : far_split(ctx, ctx->fpairs.p)));
    ctx->fpairs_ok = !native && T > 0;
    ctx->last_ntiles = (int)tl.size();
    return CSBQ_OK;
}

// drop a frozen plan and its graph
static void plan_drop(csbq_ctx* ctx)
{
    auto& pl = ctx->plan;
    if (pl.exec) (void)hipGraphExecDestroy(pl.exec);
    if (pl.graph) (void)hipGraphDestroy(pl.graph);
    pl.exec = nullptr;
    pl.graph = nullptr;
    pl.valid = false;
}

static int outputs_back(csbq_ctx* ctx, int64_t T, double* u_sl, double* u_dl, int mem, double** usl_dev,
                        double** udl_dev)
{
    if (mem == CSBQ_DEVICE) {
        *usl_dev = u_sl;
        *udl_dev = u_dl;
        return CSBQ_OK;
    }
    ALLOC(ctx->usl_d, (size_t)T * 3 + 1);
    ALLOC(ctx->udl_d, (size_t)T * 3 + 1);
    *usl_dev = u_sl ? ctx->usl_d.p : nullptr;
    *udl_dev = u_dl ? ctx->udl_d.p : nullptr;
    return CSBQ_OK;
}

// Host mode: outputs and the final flag word back to the caller.  Device
// mode: nothing to wait for; the flags of the corrections (CSBQ_FLAG_SRULE_LIMIT,
// CSBQ_FLAG_THETA_CLAMP) stay on the device for csbq_eval_flags.
static int finish(csbq_ctx* ctx, int64_t T, double* u_sl, double* u_dl, int mem)
{
    int flags = 0;
    ctx->flags_pending = mem == CSBQ_DEVICE;
    ctx->flags_src = ctx->err_d.p;
    if (mem == CSBQ_HOST) {
        const size_t ob = (size_t)T * ctx->nc() * 8;
        if (u_sl && T) HIPC(hipMemcpyAsync(u_sl, ctx->usl_d.p, ob, hipMemcpyDeviceToHost, ctx->stream));
        if (u_dl && T) HIPC(hipMemcpyAsync(u_dl, ctx->udl_d.p, ob, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipMemcpyAsync(&flags, ctx->err_d.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        ctx->last_err_flags = flags;
        if (flags & CSBQ_FLAG_NODE_RANGE) return ctx->fail(CSBQ_EINVAL, "tgt_node out of range");
    }
    return CSBQ_OK;
}

int csbq_smooth_sum(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                    double* u_sl, double* u_dl, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    plan_drop(ctx);
    HIPC(hipSetDevice(ctx->opt.device));
    const double* sig;
    const int64_t* tn;
    int rc = eval_front(ctx, sigma, T, x, tgt_node, nullptr, mem, &sig, &tn);
    if (rc) return rc;
    if (T == 0) return finish(ctx, 0, u_sl, u_dl, mem);
    int flags = 0;
    HIPC(hipMemcpyAsync(&flags, ctx->err_d.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->last_err_flags = flags;
    if (flags & CSBQ_FLAG_NODE_RANGE) return ctx->fail(CSBQ_EINVAL, "tgt_node out of range");
    std::vector<int64_t> tr;
    if ((rc = group_ranges(ctx, T, flags, tr))) return rc;
    if ((rc = far_sum(ctx, T, true, tr, ctx->stream))) return rc;
    double *usl, *udl;
    if ((rc = outputs_back(ctx, T, u_sl, u_dl, mem, &usl, &udl))) return rc;
    LCHK(launch_reduce(ctx->stream, T, ctx->tgroup.p, ctx->gnchunk.p, ctx->part.p, nullptr, nullptr, nullptr, usl,
                       udl, ctx->ker));
    return finish(ctx, T, u_sl, u_dl, mem);
}

// csbq_smooth_sum without any allocation: every buffer beyond the caller's
// inputs and outputs lives in the device's static scratch array.  One fixed
// launch shape (two targets per thread, as many source chunks as the
// partial-sum space holds, at least 8192 sources each); no host wait, no
// memset (a fill kernel clears the flag word).  Calls on one device share the
// array, so overlapping calls race.
int csbq_smooth_sum_noalloc(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                            double* u_sl, double* u_dl)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!ctx->have_geom) return ctx->fail(CSBQ_ESTATE, "set_geometry must be called first");
    if (ctx->G != 1) return ctx->fail(CSBQ_EINVAL, "the allocation-free smooth sum takes a single geometry");
    if (!sigma || T < 0) return ctx->fail(CSBQ_EINVAL, "missing density or negative target count");
    if (!x && !tgt_node && T > 0) return ctx->fail(CSBQ_EINVAL, "targets need x or tgt_node");
    if (T > NOALLOC_MAX_TARGETS)
        return ctx->fail(CSBQ_ELIMIT, "allocation-free smooth sum: more than 262144 targets");
    if (ctx->N > NOALLOC_MAX_NODES)
        return ctx->fail(CSBQ_ELIMIT, "allocation-free smooth sum: more than 262144 surface nodes");
    if (!ctx->scratch) return ctx->fail(CSBQ_ESTATE, "no scratch array on this device");
    HIPC(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    unsigned char* sp = ctx->scratch;
    double* xt = (double*)(sp + NA_XT);
    double* sw = (double*)(sp + NA_SW);
    double* sh = (double*)(sp + NA_SH);
    double* part = (double*)(sp + NA_PART);
    int* tgroup = (int*)(sp + NA_TGROUP);
    int* band = (int*)(sp + NA_BAND);
    FarTile* tiles = (FarTile*)(sp + NA_TILES);
    int64_t* gstart = (int64_t*)(sp + NA_GSTART);
    int* gnchunk = (int*)(sp + NA_GNCHUNK);
    int* errf = (int*)(sp + NA_ERR);
    const int64_t N = ctx->N;
    const int tb = 256 * 2;   // targets per block (two per thread)
    const int64_t tblocks = std::max<int64_t>((T + tb - 1) / tb, 1);
    int64_t nch = std::min<int64_t>((N + 8191) / 8192, NOALLOC_PART_DOUBLES / std::max<int64_t>(6 * T, 1));
    nch = std::max<int64_t>(1, std::min<int64_t>(nch, NOALLOC_MAX_TILES / tblocks));
    const int64_t chunk = (N + nch - 1) / nch;
    const int ntiles = T > 0 ? (int)(tblocks * nch) : 0;
    LCHK(launch_noalloc_setup(st, ntiles, (int)nch, T, N, tb, chunk, tiles, gnchunk, errf));
    ctx->flags_src = errf;
    ctx->flags_pending = true;
    if (T == 0) return CSBQ_OK;
    LCHK(launch_targets(st, T, x, tgt_node, nullptr, 1, ctx->info.p, ctx->ny.p, N, xt, tgroup, gstart, errf));
    if (ctx->nc() == 1) {   // the scalar (Laplace) density into three components
        double* s3 = (double*)(sp + NA_SIG);
        LCHK(launch_scalar_to_vec(st, N, sigma, s3));
        sigma = s3;
    }
    LCHK(launch_prep_sigma(st, ctx->E, sigma, ctx->nw.p, N, sw, sh, band, 0.1 * ctx->gc.tol, ctx->info.p,
                           ctx->circ.p, ctx->gc, nullptr));
    LCHK(launch_far(st, T, xt, ctx->ny.p, ctx->nn.p, sw, N, tiles, ntiles, part, false, 0.0, 2, ctx->ker,
                    FarSplit{}));
    LCHK(launch_reduce(st, T, tgroup, gnchunk, part, nullptr, nullptr, nullptr, u_sl, u_dl, ctx->ker));
    return CSBQ_OK;
}

int csbq_eval(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node, double* u_sl,
              double* u_dl, int mem)
{
    return csbq_eval_batch(ctx, sigma, T, x, tgt_node, nullptr, u_sl, u_dl, mem);
}

int csbq_eval_batch(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                    const int32_t* tgt_group, double* u_sl, double* u_dl, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    plan_drop(ctx);
    HIPC(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    ctx->ph_ok = false;
    const double* sig;
    const int64_t* tn;
    HIPC(hipEventRecord(ctx->ph[0].a, st));
    int rc = eval_front(ctx, sigma, T, x, tgt_node, tgt_group, mem, &sig, &tn);
    if (rc) return rc;
    if (T == 0) return finish(ctx, 0, u_sl, u_dl, mem);
    HIPC(hipEventRecord(ctx->ph[0].b, st));
    const int E = ctx->E;
    const int64_t N = ctx->N;
    // density on the tier-0 rule and the base source set
    ALLOC(ctx->swf[0], (size_t)ctx->Mtot[0] * 3);
    LCHK(launch_sigma_up(st, E, up_ns(0), up_nt(0), ctx->sh.p, ctx->Lup[0].p, ctx->cpw[0].p, ctx->swf[0].p,
                         ctx->Mtot[0]));
    ALLOC(ctx->bsw, (size_t)ctx->Nb * 3);
    LCHK(launch_sigma_base(st, E, ctx->info.p, ctx->boff.p, ctx->sw.p, N, ctx->swf[0].p, ctx->Mtot[0], ctx->bsw.p,
                           ctx->Nb));
    LCHK(sigma_far(ctx, st));
    // candidate pairs: count, scan (the fill follows the synchronisation)
    HIPC(hipEventRecord(ctx->ph[2].a, st));
    ALLOC(ctx->cnt, (size_t)T + 1);
    ALLOC(ctx->off, (size_t)T + 1);
    HIPC(hipMemsetAsync(ctx->cnt.p, 0, ((size_t)T + 1) * sizeof(int), st));
    LCHK(launch_search(st, T, ctx->tgroup.p, ctx->gel.p, ctx->xt.p, tn, ctx->info.p, ctx->rnear.p, nullptr,
                       ctx->cnt.p, nullptr, nullptr));
    size_t tmpb = 0;
    HIPC(hipcub::DeviceScan::ExclusiveSum(nullptr, tmpb, ctx->cnt.p, ctx->off.p, (int)(T + 1), st));
    ALLOC(ctx->cub_tmp, tmpb);
    HIPC(hipcub::DeviceScan::ExclusiveSum(ctx->cub_tmp.p, tmpb, ctx->cnt.p, ctx->off.p, (int)(T + 1), st));
    int64_t P = 0;
    int flags = 0;
    HIPC(hipMemcpyAsync(&P, ctx->off.p + T, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(&flags, ctx->err_d.p, sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<int> hband((size_t)2 * E);
    HIPC(hipMemcpyAsync(hband.data(), ctx->band.p, hband.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    ctx->last_err_flags = flags;
    if (flags & CSBQ_FLAG_NODE_RANGE) return ctx->fail(CSBQ_EINVAL, "tgt_node out of range");
    // pair lists are sorted and scanned with 32-bit counts
    if (P < 0 || P >= (int64_t)INT32_MAX)
        return ctx->fail(CSBQ_ELIMIT, "more than 2^31 candidate pairs: evaluate the targets in slices");
    int mt_max = 0;
    for (int k = 0; k < E; ++k) mt_max = std::max(mt_max, hband[2 * k + 1]);
    std::vector<int64_t> tr;
    if ((rc = group_ranges(ctx, T, flags, tr))) return rc;
    ALLOC(ctx->pe, (size_t)P + 1);
    ALLOC(ctx->pt, (size_t)P + 1);
    ALLOC(ctx->tier, (size_t)P + 1);
    ALLOC(ctx->cls, (size_t)P * 4 + 1);
    ALLOC(ctx->corr, (size_t)P * 6 + 1);
    LCHK(launch_search(st, T, ctx->tgroup.p, ctx->gel.p, ctx->xt.p, tn, ctx->info.p, ctx->rnear.p, ctx->off.p,
                       nullptr, ctx->pe.p, ctx->pt.p));
    HIPC(hipEventRecord(ctx->ph[2].b, st));
    if ((rc = tune_far(ctx, T, tr, false, ctx->opt.precision == CSBQ_MIXED))) return rc;
    // classification into correction tiers, in element-major order
    HIPC(hipEventRecord(ctx->ph[3].a, st));
    int ebits = 1;
    while ((1LL << ebits) < (long long)E) ++ebits;
    int kbits = 1;
    while ((1LL << kbits) < (long long)(TIER_FULL + 1) * E) ++kbits;
    ALLOC(ctx->kin, (size_t)P + 1);
    ALLOC(ctx->kout, (size_t)P + 1);
    ALLOC(ctx->vin, (size_t)P + 1);
    ALLOC(ctx->perm, (size_t)P + 1);
    ALLOC(ctx->sorted, (size_t)P + 1);
    {
        size_t b1 = 0, b2 = 0, b3 = 0;
        HIPC(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, ctx->pe.p, ctx->kout.p, ctx->vin.p, ctx->perm.p,
                                                (int)P, 0, ebits, st));
        HIPC(hipcub::DeviceRadixSort::SortPairs(nullptr, b2, ctx->kin.p, ctx->kout.p, ctx->vin.p, ctx->sorted.p,
                                                (int)P, 0, kbits, st));
        HIPC(hipcub::DeviceRunLengthEncode::Encode(nullptr, b3, ctx->kout.p, ctx->runs_key.p, ctx->runs_cnt.p,
                                                   ctx->nruns.p, (int)P, st));
        size_t need = std::max(b1, std::max(b2, b3));
        if (need > tmpb) ALLOC(ctx->cub_tmp, need);
        tmpb = std::max(tmpb, need);
    }
    LCHK(launch_iota(st, P, ctx->vin.p));
    if (P > 0)
        HIPC(hipcub::DeviceRadixSort::SortPairs(ctx->cub_tmp.p, tmpb, ctx->pe.p, ctx->kout.p, ctx->vin.p,
                                                ctx->perm.p, (int)P, 0, ebits, st));
    if (ctx->opt.gate == CSBQ_GATE_MLP) {
        // learned gate: every pair's tier from the network; the pairs it is
        // not confident about (and every special-quadrature or own-element
        // pair, whose s-rule needs the singularity estimate) go to the
        // criterion
        if (!ctx->gate_ready) return ctx->fail(CSBQ_ESTATE, "the learned gate has no weights (csbq_gate_load)");
        ALLOC(ctx->gfeat, (size_t)P * GATE_NF + GATE_NF);
        ALLOC(ctx->gtier, (size_t)P + 1);
        ALLOC(ctx->gesc, (size_t)P + 1);
        ALLOC(ctx->gflag, (size_t)P + 1);
        ALLOC(ctx->gsel, (size_t)P + 1);
        ALLOC(ctx->gnsel, 1);
        LCHK(launch_gate_features(st, P, ctx->perm.p, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->circ.p,
                                  ctx->info.p, ctx->band.p, (float)std::log10(ctx->gc.tol), ctx->gfeat.p));
        LCHK(launch_gate_mlp(st, P, ctx->gfeat.p, ctx->gate_wfrag.p, ctx->gate_bias.p, ctx->gate_tau, ctx->gtier.p,
                             ctx->gesc.p, nullptr));
        LCHK(launch_gate_select(st, P, ctx->perm.p, ctx->pe.p, ctx->info.p, ctx->gesc.p, ctx->gtier.p, ctx->tier.p,
                                ctx->gflag.p));
        size_t sb = 0;
        HIPC(hipcub::DeviceSelect::Flagged(nullptr, sb, ctx->perm.p, ctx->gflag.p, ctx->gsel.p, ctx->gnsel.p, (int)P,
                                           st));
        if (sb > tmpb) {
            ALLOC(ctx->cub_tmp, sb);
            tmpb = sb;
        }
        int nsel = 0;
        if (P > 0) {
            HIPC(hipcub::DeviceSelect::Flagged(ctx->cub_tmp.p, tmpb, ctx->perm.p, ctx->gflag.p, ctx->gsel.p,
                                               ctx->gnsel.p, (int)P, st));
            HIPC(hipMemcpyAsync(&nsel, ctx->gnsel.p, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
        }
        ctx->last_esc = nsel;
        LCHK(launch_classify(st, nsel, ctx->gsel.p, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->clq.p,
                             ctx->circ.p, ctx->gridc.p, ctx->info.p, ctx->tor.p, ctx->band.p, ctx->gc, ctx->tier.p,
                             ctx->cls.p));
    } else {
        ctx->last_esc = -1;
        LCHK(launch_classify(st, P, ctx->perm.p, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->clq.p, ctx->circ.p,
                             ctx->gridc.p, ctx->info.p, ctx->tor.p, ctx->band.p, ctx->gc, ctx->tier.p,
                             ctx->cls.p));
    }
    HIPC(hipEventRecord(ctx->ph[3].b, st));
    // buckets: pairs sorted by (tier, element); runs give the per-element segments
    HIPC(hipEventRecord(ctx->ph[4].a, st));
    const size_t maxruns = (size_t)(TIER_FULL + 1) * E + 1;
    ALLOC(ctx->runs_key, maxruns);
    ALLOC(ctx->runs_cnt, maxruns);
    ALLOC(ctx->nruns, 1);
    int nr = 0;
    std::vector<int> rkey, rcnt;
    if (P > 0) {
        LCHK(launch_tier_keys(st, P, E, ctx->tier.p, ctx->pe.p, ctx->kin.p, ctx->vin.p));
        HIPC(hipcub::DeviceRadixSort::SortPairs(ctx->cub_tmp.p, tmpb, ctx->kin.p, ctx->kout.p, ctx->vin.p,
                                                ctx->sorted.p, (int)P, 0, kbits, st));
        HIPC(hipcub::DeviceRunLengthEncode::Encode(ctx->cub_tmp.p, tmpb, ctx->kout.p, ctx->runs_key.p,
                                                   ctx->runs_cnt.p, ctx->nruns.p, (int)P, st));
        HIPC(hipMemcpyAsync(&nr, ctx->nruns.p, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        rkey.resize(nr);
        rcnt.resize(nr);
        if (nr) {
            HIPC(hipMemcpy(rkey.data(), ctx->runs_key.p, nr * sizeof(int), hipMemcpyDeviceToHost));
            HIPC(hipMemcpy(rcnt.data(), ctx->runs_cnt.p, nr * sizeof(int), hipMemcpyDeviceToHost));
        }
    }
    std::vector<int> wd[NUP];
    int64_t npair[NUP] = {0, 0, 0};
    int nfull = 0, full_start = 0;
    {
        int pos = 0;
        for (int r = 0; r < nr; ++r) {
            int trr = rkey[r] / E, e = rkey[r] % E, c = rcnt[r];
            if (trr >= 1 && trr <= NUP) {
                for (int o = 0; o < c; o += UP_PAIRS) {
                    wd[trr - 1].push_back(pos + o);
                    wd[trr - 1].push_back(std::min(UP_PAIRS, c - o));
                    wd[trr - 1].push_back(e);
                    wd[trr - 1].push_back(trr - 1);
                }
                npair[trr - 1] += c;
            } else if (trr == TIER_FULL) {
                if (nfull == 0) full_start = pos;
                nfull += c;
            }
            pos += c;
        }
    }
    // one launch for every upsampled tier, the largest rules' wavefronts
    // first so that the short ones fill the device's tail
    int nwaves[NUP];
    std::vector<int> wall;
    for (int ti = NUP - 1; ti >= 0; --ti) {
        nwaves[ti] = (int)(wd[ti].size() / 4);
        wall.insert(wall.end(), wd[ti].begin(), wd[ti].end());
    }
    const int nw_up = (int)(wall.size() / 4);
    ALLOC(ctx->wdesc, wall.size() + 1);
    if (nw_up) HIPC(hipMemcpy(ctx->wdesc.p, wall.data(), wall.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipEventRecord(ctx->ph[4].b, st));
    // the smooth sum over every base source of the target's group (on the
    // same stream: it and the corrections are both VALU-bound, and running
    // them side by side gained 2 % while blurring every kernel's timing)
    // (the phase's start is recorded by far_sum just before the launch, so
    // that it does not count the host's block set-up)
    if ((rc = far_sum(ctx, T, false, tr, st, ctx->ph[1].a))) return rc;
    HIPC(hipEventRecord(ctx->ph[1].b, st));
    // upsampled-rule corrections
    HIPC(hipEventRecord(ctx->ph[5].a, st));
    for (int ti = 1; ti < NUP; ++ti) {
        if (!nwaves[ti]) continue;
        ALLOC(ctx->swf[ti], (size_t)ctx->Mtot[ti] * 3);
        LCHK(launch_sigma_up(st, E, up_ns(ti), up_nt(ti), ctx->sh.p, ctx->Lup[ti].p, ctx->cpw[ti].p, ctx->swf[ti].p,
                             ctx->Mtot[ti]));
    }
    LCHK(launch_corr_up(st, up_rules(ctx), nw_up, ctx->wdesc.p, ctx->sorted.p, ctx->pt.p, ctx->xt.p, T, ctx->info.p,
                        ctx->boff.p, ctx->by.p, ctx->bn.p, ctx->bsw.p, ctx->Nb, ctx->corr.p, ctx->ker));
    HIPC(hipEventRecord(ctx->ph[5].b, st));
    // special quadrature corrections
    HIPC(hipEventRecord(ctx->ph[6].a, st));
    ALLOC(ctx->work, (size_t)WORK_STRIDE * nfull + WORK_STRIDE);
    LCHK(launch_corr_full(st, nfull, ctx->sorted.p + full_start, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->clq.p, ctx->sh.p,
                          ctx->info.p, ctx->band.p, ctx->cls.p, ctx->boff.p, ctx->by.p, ctx->bn.p, ctx->bsw.p, ctx->Nb,
                          rule_args(ctx), ctx->gc, ctx->corr.p, ctx->err_d.p, ctx->work.p, mt_max, ctx->ker));
    HIPC(hipEventRecord(ctx->ph[6].b, st));
    // reduction
    HIPC(hipEventRecord(ctx->ph[7].a, st));
    double *usl, *udl;
    if ((rc = outputs_back(ctx, T, u_sl, u_dl, mem, &usl, &udl))) return rc;
    LCHK(launch_reduce(st, T, ctx->tgroup.p, ctx->gnchunk.p, ctx->part.p, ctx->off.p, ctx->tier.p, ctx->corr.p, usl,
                       udl, ctx->ker));
    HIPC(hipEventRecord(ctx->ph[7].b, st));
    ctx->last_T = T;
    ctx->last_P = P;
    for (int ti = 0; ti < NUP; ++ti) ctx->last_nup[ti] = npair[ti];
    ctx->last_nf = nfull;
    ctx->ph_ok = true;
    {
        auto& pl = ctx->plan;
        pl.T = T;
        for (int ti = 0; ti < NUP; ++ti) pl.nwaves[ti] = nwaves[ti];
        pl.nw_up = nw_up;
        pl.nfull = nfull;
        pl.full_start = full_start;
        pl.mt_max = mt_max;
        pl.ntiles = ctx->last_ntiles;
        pl.tpt = ctx->far_tpt;
        pl.mixed = ctx->opt.precision == CSBQ_MIXED;
        pl.tn = tn;
    }
    return finish(ctx, T, u_sl, u_dl, mem);
}

// The per-density part of an evaluation under a frozen plan: density
// coefficients (band checked against the plan's), the smooth sum over the
// plan's blocks, the corrections of the plan's tiers and rules, the
// reduction into the context's output buffers.  No allocation, no host
// synchronisation, no memset: the sequence is captured as a graph.
static int enqueue_apply(csbq_ctx* ctx, hipStream_t st)
{
    const auto& pl = ctx->plan;
    const int E = ctx->E;
    const int64_t N = ctx->N, T = pl.T;
    LCHK(launch_fill_i32(st, 1, ctx->err_d.p, 0));
    if (ctx->nc() == 1) LCHK(launch_scalar_to_vec(st, N, ctx->sig1.p, ctx->sig_d.p));
    LCHK(launch_prep_sigma(st, E, ctx->sig_d.p, ctx->nw.p, N, ctx->sw.p, ctx->sh.p, ctx->band_apply.p,
                           0.1 * ctx->gc.tol, ctx->info.p, ctx->circ.p, ctx->gc, nullptr));
    LCHK(launch_band_check(st, E, ctx->band_apply.p, ctx->band.p, ctx->err_d.p));
    LCHK(launch_sigma_up(st, E, up_ns(0), up_nt(0), ctx->sh.p, ctx->Lup[0].p, ctx->cpw[0].p, ctx->swf[0].p,
                         ctx->Mtot[0]));
    LCHK(launch_sigma_base(st, E, ctx->info.p, ctx->boff.p, ctx->sw.p, N, ctx->swf[0].p, ctx->Mtot[0], ctx->bsw.p,
                           ctx->Nb));
    LCHK(sigma_far(ctx, st));
    LCHK(launch_far(st, T, ctx->xt.p, ctx->by.p, ctx->bn.p, ctx->bsw.p, ctx->Nb, ctx->tiles.p, pl.ntiles, ctx->part.p,
                    pl.mixed, ctx->mix_near2, pl.tpt, ctx->ker, far_split(ctx, ctx->fpairs.p)));
    for (int ti = 1; ti < NUP; ++ti)
        if (pl.nwaves[ti])
            LCHK(launch_sigma_up(st, E, up_ns(ti), up_nt(ti), ctx->sh.p, ctx->Lup[ti].p, ctx->cpw[ti].p,
                                 ctx->swf[ti].p, ctx->Mtot[ti]));
    LCHK(launch_corr_up(st, up_rules(ctx), pl.nw_up, ctx->wdesc.p, ctx->sorted.p, ctx->pt.p, ctx->xt.p, T,
                        ctx->info.p, ctx->boff.p, ctx->by.p, ctx->bn.p, ctx->bsw.p, ctx->Nb, ctx->corr.p, ctx->ker));
    if (pl.matrix)
        LCHK(launch_emat_apply(st, pl.nfull, ctx->sorted.p + pl.full_start, ctx->pe.p, ctx->emat.p, ctx->sh.p,
                               ctx->corr.p));
    else
    LCHK(launch_corr_full(st, pl.nfull, ctx->sorted.p + pl.full_start, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, pl.tn,
                          ctx->clq.p, ctx->sh.p, ctx->info.p, ctx->band.p, ctx->cls.p, ctx->boff.p, ctx->by.p,
                          ctx->bn.p, ctx->bsw.p, ctx->Nb, rule_args(ctx), ctx->gc, ctx->corr.p, ctx->err_d.p,
                          ctx->work.p, pl.mt_max, ctx->ker));
    LCHK(launch_reduce(st, T, ctx->tgroup.p, ctx->gnchunk.p, ctx->part.p, ctx->off.p, ctx->tier.p, ctx->corr.p,
                       ctx->usl_d.p, ctx->udl_d.p, ctx->ker));
    return CSBQ_OK;
}

// The correction matrices of the plan's special-quadrature pairs (Section
// 3.2.1: the corrected rule's E for those pairs), in the density's
// coefficient basis: rows counted per pair, then built in chunks of pairs
// whose rows fit a bounded scratch, each chunk's rows assembled into the
// pairs' matrices.
static int build_matrix(csbq_ctx* ctx)
{
    auto& pl = ctx->plan;
    hipStream_t st = ctx->stream;
    const int nfull = pl.nfull;
    pl.matrix = false;
    if (ctx->ker != KER_STOKES) return ctx->fail(CSBQ_EINVAL, "the correction matrix is built for the Stokes layers");
    const double bytes = (double)nfull * EMAT_DOUBLES * 8.0;
    if (bytes > 160e9) return ctx->fail(CSBQ_ELIMIT, "correction matrices beyond 160 GB: plan fewer targets");
    hipEvent_t a, b;
    HIPC(hipEventCreate(&a));
    HIPC(hipEventCreate(&b));
    HIPC(hipEventRecord(a, st));
    ALLOC(ctx->emat, (size_t)nfull * EMAT_DOUBLES + 1);
    DBuf<int> cnt;
    DBuf<int64_t> roff;
    DBuf<double> V, L;
    if (nfull > 0) {
        const int* listf = ctx->sorted.p + pl.full_start;
        ALLOC(cnt, (size_t)nfull);
        ALLOC(ctx->work, (size_t)WORK_STRIDE * nfull + WORK_STRIDE);
        MatrixRows mr{nullptr, nullptr, nullptr, cnt.p, ctx->Lup[0].p, ctx->bw.p};
        auto corr_launch = [&](int n, const int* lf, int mode) {
            return launch_corr_full(st, n, lf, ctx->pe.p, ctx->pt.p, ctx->xt.p, pl.T, pl.tn, ctx->clq.p, ctx->sh.p,
                                    ctx->info.p, ctx->band.p, ctx->cls.p, ctx->boff.p, ctx->by.p, ctx->bn.p,
                                    ctx->bsw.p, ctx->Nb, rule_args(ctx), ctx->gc, ctx->corr.p,
                                    ctx->err_d.p, ctx->work.p, pl.mt_max, ctx->ker, mode, &mr);
        };
        LCHK(corr_launch(nfull, listf, MODE_COUNT));
        std::vector<int> hc((size_t)nfull);
        HIPC(hipMemcpyAsync(hc.data(), cnt.p, hc.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        // chunks of pairs whose rows fit ~3 GB of scratch (3 KB + 128 B a row)
        const int64_t budget = 3LL << 30, row_bytes = (int64_t)(12 * NT + NS) * 8;
        const int64_t max_rows = budget / row_bytes;
        int64_t rows_max_chunk = 0;
        std::vector<std::pair<int, int>> chunks;
        for (int p0 = 0; p0 < nfull;) {
            int64_t rows = 0;
            int p1 = p0;
            while (p1 < nfull && (p1 == p0 || rows + hc[p1] <= max_rows)) rows += hc[p1++];
            chunks.push_back({p0, p1});
            rows_max_chunk = std::max(rows_max_chunk, rows);
            p0 = p1;
        }
        ALLOC(V, (size_t)rows_max_chunk * 12 * NT);
        ALLOC(L, (size_t)rows_max_chunk * NS);
        int max_pairs = 0;
        for (auto& c : chunks) max_pairs = std::max(max_pairs, c.second - c.first);
        ALLOC(roff, (size_t)max_pairs + 1);
        std::vector<int64_t> ho((size_t)max_pairs + 1);
        for (auto& c : chunks) {
            const int n = c.second - c.first;
            ho[0] = 0;
            for (int k = 0; k < n; ++k) ho[k + 1] = ho[k] + hc[c.first + k];
            HIPC(hipMemcpyAsync(roff.p, ho.data(), ((size_t)n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
            mr = MatrixRows{roff.p, V.p, L.p, nullptr, ctx->Lup[0].p, ctx->bw.p};
            LCHK(corr_launch(n, listf + c.first, MODE_MATRIX));
            LCHK(launch_emat(st, n, roff.p, V.p, L.p, c.first, ctx->emat.p));
            HIPC(hipStreamSynchronize(st));   // ho is rewritten for the next chunk
        }
    }
    HIPC(hipEventRecord(b, st));
    HIPC(hipEventSynchronize(b));
    HIPC(hipEventElapsedTime(&pl.build_ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    pl.matrix = true;
    return CSBQ_OK;
}

int csbq_plan(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
              const int32_t* tgt_group, double* u_sl, double* u_dl, int mem)
{
    return csbq_plan_ex(ctx, sigma, T, x, tgt_node, tgt_group, 0, u_sl, u_dl, mem);
}

int csbq_plan_ex(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                 const int32_t* tgt_group, int32_t flags, double* u_sl, double* u_dl, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    if (T <= 0) return ctx->fail(CSBQ_EINVAL, "a plan needs targets");
    if (flags & ~(CSBQ_PLAN_MATRIX | CSBQ_PLAN_FULL_BAND)) return ctx->fail(CSBQ_EINVAL, "unknown plan flags");
    if ((flags & CSBQ_PLAN_MATRIX) && ctx->ker != KER_STOKES)
        return ctx->fail(CSBQ_EINVAL, "the correction matrix is built for the Stokes layers");
    const bool fb_prev = ctx->full_band;
    ctx->full_band = fb_prev || (flags & CSBQ_PLAN_FULL_BAND);
    int rc = csbq_eval_batch(ctx, sigma, T, x, tgt_node, tgt_group, u_sl, u_dl, mem);
    ctx->full_band = fb_prev;
    if (rc) return rc;
    auto& pl = ctx->plan;
    hipStream_t st = ctx->stream;
    pl.matrix = false;
    pl.build_ms = 0.f;
    // everything the graph reads must live in the context
    ALLOC(ctx->sig_d, (size_t)ctx->N * 3);
    ALLOC(ctx->sig1, (size_t)ctx->N);
    if (mem == CSBQ_DEVICE && tgt_node) {
        ALLOC(ctx->tn_d, (size_t)T);
        HIPC(hipMemcpyAsync(ctx->tn_d.p, tgt_node, (size_t)T * 8, hipMemcpyDeviceToDevice, st));
        pl.tn = ctx->tn_d.p;
    }
    ALLOC(ctx->usl_d, (size_t)T * 3 + 1);
    ALLOC(ctx->udl_d, (size_t)T * 3 + 1);
    ALLOC(ctx->band_apply, (size_t)ctx->E * 2);
    HIPC(hipStreamSynchronize(st));
    if (flags & CSBQ_PLAN_MATRIX)
        if ((rc = build_matrix(ctx))) return rc;
    if (!pl.gst) HIPC(hipStreamCreateWithFlags(&pl.gst, hipStreamNonBlocking));
    if (!pl.e0) HIPC(hipEventCreateWithFlags(&pl.e0, hipEventDisableTiming));
    if (!pl.e1) HIPC(hipEventCreateWithFlags(&pl.e1, hipEventDisableTiming));
    HIPC(hipStreamBeginCapture(pl.gst, hipStreamCaptureModeThreadLocal));
    rc = enqueue_apply(ctx, pl.gst);
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(pl.gst, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (he != hipSuccess) return ctx->fail(CSBQ_EHIP, std::string("graph capture failed: ") + hipGetErrorString(he));
    pl.graph = g;
    HIPC(hipGraphInstantiate(&pl.exec, g, nullptr, nullptr, 0));
    pl.valid = true;
    return CSBQ_OK;
}

int csbq_apply(csbq_ctx* ctx, const double* sigma, double* u_sl, double* u_dl, int mem)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    auto& pl = ctx->plan;
    if (!pl.valid) return ctx->fail(CSBQ_ESTATE, "no evaluation plan (csbq_plan)");
    if (!sigma) return ctx->fail(CSBQ_EINVAL, "missing density");
    if (mem != CSBQ_HOST && mem != CSBQ_DEVICE) return ctx->fail(CSBQ_EINVAL, "bad mem flag");
    HIPC(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->N, T = pl.T;
    const int nc = ctx->nc();
    if (mem == CSBQ_HOST)
        for (int64_t i = 0; i < N * nc; ++i)
            if (!std::isfinite(sigma[i])) return ctx->fail(CSBQ_EINVAL, "density has NaN/Inf");
    HIPC(hipMemcpyAsync(nc == 3 ? ctx->sig_d.p : ctx->sig1.p, sigma, (size_t)N * nc * 8,
                        mem == CSBQ_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    HIPC(hipEventRecord(pl.e0, st));
    HIPC(hipStreamWaitEvent(pl.gst, pl.e0, 0));
    HIPC(hipGraphLaunch(pl.exec, pl.gst));
    HIPC(hipEventRecord(pl.e1, pl.gst));
    HIPC(hipStreamWaitEvent(st, pl.e1, 0));
    const hipMemcpyKind k = mem == CSBQ_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (u_sl) HIPC(hipMemcpyAsync(u_sl, ctx->usl_d.p, (size_t)T * nc * 8, k, st));
    if (u_dl) HIPC(hipMemcpyAsync(u_dl, ctx->udl_d.p, (size_t)T * nc * 8, k, st));
    int flags = 0;
    HIPC(hipMemcpyAsync(&flags, ctx->err_d.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    ctx->last_err_flags = flags;
    ctx->flags_pending = false;
    if (flags & CSBQ_FLAG_BAND)
        return ctx->fail(CSBQ_ESTATE, "the density's band exceeds the one the plan was built for: plan again");
    return CSBQ_OK;
}

// ---------------------------------------------------------------------------
// learned gate
// ---------------------------------------------------------------------------
static_assert(GATE_NF == CSBQ_GATE_NF && GATE_NO == CSBQ_GATE_NO && GATE_NW == CSBQ_GATE_NW, "gate shape");

static uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

int csbq_gate_load(csbq_ctx* ctx, const float* W, float tau_esc)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!W) return ctx->fail(CSBQ_EINVAL, "missing weights");
    if (!(tau_esc > 0.f && tau_esc < 1.f)) return ctx->fail(CSBQ_EINVAL, "tau_esc must lie in (0, 1)");
    for (int i = 0; i < GATE_NW; ++i)
        if (!std::isfinite(W[i])) return ctx->fail(CSBQ_EINVAL, "weights have NaN/Inf");
    HIPC(hipSetDevice(ctx->opt.device));
    // B fragments of v_mfma_f32_16x16x16_bf16: lane l holds B[4 (l/16) + i][l % 16]
    std::vector<uint16_t> fr((size_t)GATE_NFRAG * GATE_FRAG_ELEMS, 0);
    int f = 0;
    auto put = [&](const float* M, int ncol, int kb, int nb, int ncol_used) {
        for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 4; ++i) {
                const int k = kb * 16 + 4 * (l / 16) + i, c = nb * 16 + (l % 16);
                const float v = c < ncol_used ? M[(size_t)k * ncol + c] : 0.f;
                fr[((size_t)f * 64 + l) * 4 + i] = host_bf16(v);
            }
        ++f;
    };
    for (int nb = 0; nb < 4; ++nb) put(W + GW1, GATE_H, 0, nb, GATE_H);
    for (int kb = 0; kb < 4; ++kb)
        for (int nb = 0; nb < 4; ++nb) put(W + GW2, GATE_H, kb, nb, GATE_H);
    for (int kb = 0; kb < 4; ++kb)
        for (int nb = 0; nb < 4; ++nb) put(W + GW3, GATE_H, kb, nb, GATE_H);
    for (int kb = 0; kb < 4; ++kb) put(W + GW4, GATE_NO, kb, 0, GATE_NO);
    std::vector<float> b((size_t)GATE_NBIAS, 0.f);
    for (int j = 0; j < GATE_H; ++j) {
        b[j] = W[GB1 + j];
        b[GATE_H + j] = W[GB2 + j];
        b[2 * GATE_H + j] = W[GB3 + j];
    }
    for (int c = 0; c < GATE_NO; ++c) b[3 * GATE_H + c] = W[GB4 + c];
    ALLOC(ctx->gate_wfrag, fr.size());
    ALLOC(ctx->gate_bias, b.size());
    HIPC(hipMemcpy(ctx->gate_wfrag.p, fr.data(), fr.size() * 2, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->gate_bias.p, b.data(), b.size() * 4, hipMemcpyHostToDevice));
    ctx->gate_tau = tau_esc;
    ctx->gate_ready = true;
    return CSBQ_OK;
}

int csbq_gate_infer(csbq_ctx* ctx, const float* feat, int64_t n, int8_t* tier, uint8_t* esc, float* logits)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!ctx->gate_ready) return ctx->fail(CSBQ_ESTATE, "no gate weights loaded");
    if (!feat || n < 0 || n > (int64_t)INT32_MAX) return ctx->fail(CSBQ_EINVAL, "bad features");
    HIPC(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    int rc;
    if ((rc = to_device(ctx, ctx->gfeat, feat, (size_t)n * GATE_NF, CSBQ_HOST))) return rc;
    ALLOC(ctx->gtier, (size_t)n + 1);
    ALLOC(ctx->gesc, (size_t)n + 1);
    DBuf<float> lg;
    ALLOC(lg, (size_t)n * GATE_NO + 1);
    LCHK(launch_gate_mlp(st, n, ctx->gfeat.p, ctx->gate_wfrag.p, ctx->gate_bias.p, ctx->gate_tau, ctx->gtier.p,
                         ctx->gesc.p, lg.p));
    if (n > 0) {
        if (tier) HIPC(hipMemcpyAsync(tier, ctx->gtier.p, (size_t)n, hipMemcpyDeviceToHost, st));
        if (esc) HIPC(hipMemcpyAsync(esc, ctx->gesc.p, (size_t)n, hipMemcpyDeviceToHost, st));
        if (logits) HIPC(hipMemcpyAsync(logits, lg.p, (size_t)n * GATE_NO * 4, hipMemcpyDeviceToHost, st));
    }
    HIPC(hipStreamSynchronize(st));
    return CSBQ_OK;
}

// one forward/backward pass over samples perm[0..n) of (feat, label) on the
// device buffers; grad (NW + 1 floats, the last the loss) averaged over n
static int gate_grad_dev(csbq_ctx* ctx, int64_t off, int64_t n, const int64_t* perm, const float* feat,
                         const int8_t* label, const float* W, const float* posw, DBuf<float>& partial,
                         float* grad)
{
    const int spb = 64;
    const int nblk = (int)((n + spb - 1) / spb);
    ALLOC(partial, (size_t)std::max(nblk, 1) * (GATE_NW + 1));
    LCHK(launch_gate_train_step(ctx->stream, nblk, spb, off, n, perm, feat, label, W, posw, partial.p));
    LCHK(launch_gate_reduce(ctx->stream, nblk, partial.p, 1.f / (float)std::max<int64_t>(n, 1), grad));
    return CSBQ_OK;
}

int csbq_gate_grad(csbq_ctx* ctx, const float* W, const float* feat, const int8_t* label, int64_t n,
                   const float* posw, float* grad_out, float* loss_out)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!W || !feat || !label || !posw || !grad_out || n <= 0) return ctx->fail(CSBQ_EINVAL, "bad arguments");
    HIPC(hipSetDevice(ctx->opt.device));
    DBuf<float> dW, df, dpw, part, grad;
    DBuf<int8_t> dl;
    DBuf<int64_t> dp;
    int rc;
    if ((rc = to_device(ctx, dW, W, GATE_NW, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, df, feat, (size_t)n * GATE_NF, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, dl, label, (size_t)n, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, dpw, posw, GATE_NO, CSBQ_HOST))) return rc;
    std::vector<int64_t> id((size_t)n);
    for (int64_t i = 0; i < n; ++i) id[i] = i;
    if ((rc = to_device(ctx, dp, id.data(), (size_t)n, CSBQ_HOST))) return rc;
    ALLOC(grad, GATE_NW + 1);
    if ((rc = gate_grad_dev(ctx, 0, n, dp.p, df.p, dl.p, dW.p, dpw.p, part, grad.p))) return rc;
    std::vector<float> g(GATE_NW + 1);
    HIPC(hipMemcpyAsync(g.data(), grad.p, g.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    std::memcpy(grad_out, g.data(), GATE_NW * 4);
    if (loss_out) *loss_out = g[GATE_NW];
    return CSBQ_OK;
}

int csbq_gate_train(csbq_ctx* ctx, const float* feat, const int8_t* label, int64_t n, const float* posw, int epochs,
                    int batch, float lr, uint64_t seed, float* W, float* loss_out)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!W || !feat || !label || !posw || n <= 0 || epochs <= 0 || batch <= 0 || !(lr > 0))
        return ctx->fail(CSBQ_EINVAL, "bad arguments");
    HIPC(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    DBuf<float> dW, df, dpw, part, grad, m, v;
    DBuf<int8_t> dl;
    DBuf<int64_t> dp;
    int rc;
    if ((rc = to_device(ctx, dW, W, GATE_NW, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, df, feat, (size_t)n * GATE_NF, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, dl, label, (size_t)n, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, dpw, posw, GATE_NO, CSBQ_HOST))) return rc;
    std::vector<float> zero(GATE_NW, 0.f);
    if ((rc = to_device(ctx, m, zero.data(), GATE_NW, CSBQ_HOST))) return rc;
    if ((rc = to_device(ctx, v, zero.data(), GATE_NW, CSBQ_HOST))) return rc;
    ALLOC(grad, GATE_NW + 1);
    ALLOC(dp, (size_t)n);
    std::vector<int64_t> id((size_t)n);
    for (int64_t i = 0; i < n; ++i) id[i] = i;
    std::mt19937_64 rng(seed);
    int step = 0;
    std::vector<float> g(GATE_NW + 1);
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(id.begin(), id.end(), rng);
        HIPC(hipMemcpyAsync(dp.p, id.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
        double lsum = 0.0;
        for (int64_t off = 0; off < n; off += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - off);
            if ((rc = gate_grad_dev(ctx, off, nb, dp.p, df.p, dl.p, dW.p, dpw.p, part, grad.p))) return rc;
            LCHK(launch_gate_adam(st, dW.p, grad.p, m.p, v.p, lr, 0.9f, 0.999f, 1e-8f, ++step));
            HIPC(hipMemcpyAsync(g.data() + GATE_NW, grad.p + GATE_NW, 4, hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            lsum += (double)g[GATE_NW] * (double)nb;
        }
        if (loss_out) loss_out[ep] = (float)(lsum / (double)n);
    }
    HIPC(hipMemcpyAsync(W, dW.p, GATE_NW * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return CSBQ_OK;
}

int csbq_gate_dataset(csbq_ctx* ctx, const double* sigma, int64_t T, const double* x, const int64_t* tgt_node,
                      double label_tol, int64_t cap, float* feat_out, int8_t* label_out, int8_t* crit_out,
                      int64_t* n_out)
{
    if (!ctx) return CSBQ_EINVAL;
    ctx->err.clear();
    if (!feat_out || !label_out || !n_out || cap <= 0 || !(label_tol > 0) || T <= 0)
        return ctx->fail(CSBQ_EINVAL, "bad arguments");
    if (ctx->ker != KER_STOKES) return ctx->fail(CSBQ_EINVAL, "gate training data are for the Stokes layers");
    if (ctx->opt.gate != CSBQ_GATE_CRITERION)
        return ctx->fail(CSBQ_ESTATE, "labels are generated with the criterion gate");
    plan_drop(ctx);
    // the evaluation leaves the candidate pairs, their classification
    // (singularity estimates for the special quadrature) and the element-major
    // order in the context
    std::vector<double> us((size_t)T * 3), ud((size_t)T * 3);
    int rc = csbq_eval(ctx, sigma, T, x, tgt_node, us.data(), ud.data(), CSBQ_HOST);
    if (rc) return rc;
    double ms = 0.0, md = 0.0;
    for (double v : us) ms = std::max(ms, std::fabs(v));
    for (double v : ud) md = std::max(md, std::fabs(v));
    const double PI_ = 3.14159265358979323846;
    const double thr_s = label_tol * ms * 8.0 * PI_, thr_d = label_tol * md * 4.0 * PI_ / 3.0;
    hipStream_t st = ctx->stream;
    const int64_t P = ctx->last_P;
    const int E = ctx->E;
    const int64_t* tn = tgt_node ? ctx->tn_d.p : nullptr;
    // features of every pair
    ALLOC(ctx->gfeat, (size_t)P * GATE_NF + GATE_NF);
    LCHK(launch_gate_features(st, P, ctx->perm.p, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->circ.p, ctx->info.p,
                              ctx->band.p, (float)std::log10(ctx->gc.tol), ctx->gfeat.p));
    // every pair through every tier: upsampled rules by element runs of the
    // element-major order, special quadrature on all
    std::vector<int> hperm((size_t)P), hpe((size_t)P);
    HIPC(hipMemcpyAsync(hperm.data(), ctx->perm.p, (size_t)P * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(hpe.data(), ctx->pe.p, (size_t)P * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    DBuf<int> dwd[NUP];
    DBuf<double> cup[NUP], cfull;
    for (int ti = 0; ti < NUP; ++ti) {
        std::vector<int> wd;
        for (int64_t i = 0; i < P;) {
            const int e = hpe[hperm[i]];
            int64_t j = i;
            while (j < P && hpe[hperm[j]] == e) ++j;
            for (int64_t o = i; o < j; o += UP_PAIRS) {
                wd.push_back((int)o);
                wd.push_back((int)std::min<int64_t>(UP_PAIRS, j - o));
                wd.push_back(e);
                wd.push_back(ti);
            }
            i = j;
        }
        const int nw = (int)(wd.size() / 4);
        if ((rc = to_device(ctx, dwd[ti], wd.data(), wd.size(), CSBQ_HOST))) return rc;
        ALLOC(cup[ti], (size_t)P * 6 + 1);
        ALLOC(ctx->swf[ti], (size_t)ctx->Mtot[ti] * 3);
        LCHK(launch_sigma_up(st, E, up_ns(ti), up_nt(ti), ctx->sh.p, ctx->Lup[ti].p, ctx->cpw[ti].p, ctx->swf[ti].p,
                             ctx->Mtot[ti]));
        LCHK(launch_corr_up(st, up_rules(ctx), nw, dwd[ti].p, ctx->perm.p, ctx->pt.p, ctx->xt.p, T, ctx->info.p,
                            ctx->boff.p, ctx->by.p, ctx->bn.p, ctx->bsw.p, ctx->Nb, cup[ti].p, ctx->ker));
    }
    ALLOC(cfull, (size_t)P * 6 + 1);
    std::vector<int> hband((size_t)2 * E);
    HIPC(hipMemcpy(hband.data(), ctx->band.p, hband.size() * 4, hipMemcpyDeviceToHost));
    int mt_max = 0;
    for (int k = 0; k < E; ++k) mt_max = std::max(mt_max, hband[2 * k + 1]);
    ALLOC(ctx->work, (size_t)WORK_STRIDE * P + WORK_STRIDE);
    LCHK(launch_corr_full(st, (int)P, ctx->perm.p, ctx->pe.p, ctx->pt.p, ctx->xt.p, T, tn, ctx->clq.p, ctx->sh.p,
                          ctx->info.p, ctx->band.p, ctx->cls.p, ctx->boff.p, ctx->by.p, ctx->bn.p, ctx->bsw.p,
                          ctx->Nb, rule_args(ctx), ctx->gc, cfull.p, ctx->err_d.p, ctx->work.p, mt_max, ctx->ker));
    DBuf<int8_t> lab;
    ALLOC(lab, (size_t)P + 1);
    LCHK(launch_gate_labels(st, P, cup[0].p, cup[1].p, cup[2].p, cfull.p, thr_s, thr_d, lab.p));
    ctx->ph_ok = false;   // the work counters now describe the label run
    // a strided sample of at most cap pairs
    const int64_t stride = (P + cap - 1) / cap;
    const int64_t nsel = stride > 0 ? (P + stride - 1) / stride : 0;
    if (nsel > 0) {
        HIPC(hipMemcpy2DAsync(feat_out, GATE_NF * 4, ctx->gfeat.p, (size_t)stride * GATE_NF * 4, GATE_NF * 4,
                              (size_t)nsel, hipMemcpyDeviceToHost, st));
        HIPC(hipMemcpy2DAsync(label_out, 1, lab.p, (size_t)stride, 1, (size_t)nsel, hipMemcpyDeviceToHost, st));
        if (crit_out)
            HIPC(hipMemcpy2DAsync(crit_out, 1, ctx->tier.p, (size_t)stride, 1, (size_t)nsel, hipMemcpyDeviceToHost,
                                  st));
    }
    HIPC(hipStreamSynchronize(st));
    *n_out = nsel;
    return CSBQ_OK;
}

int csbq_stats(const csbq_ctx* ctx, char* buf, int64_t cap)
{
    if (!ctx || !buf || cap <= 0) return CSBQ_EINVAL;
    // the work counters and phase events belong to work enqueued on the
    // context's stream, which need not be ordered with the copies below
    (void)hipSetDevice(ctx->opt.device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) (void)hipGetLastError();
    std::string s = "{";
    char tmp[256];
    std::snprintf(tmp, sizeof tmp,
                  "\"targets\": %lld, \"candidates\": %lld, \"pairs_up1\": %lld, \"pairs_up2\": %lld, "
                  "\"pairs_up3\": %lld, \"pairs_full\": %lld, \"flags\": %d, \"sources_base\": %lld",
                  (long long)ctx->last_T, (long long)ctx->last_P, (long long)ctx->last_nup[0],
                  (long long)ctx->last_nup[1], (long long)ctx->last_nup[2], (long long)ctx->last_nf,
                  ctx->last_err_flags, (long long)ctx->Nb_rules);
    s += tmp;
    if (ctx->last_esc >= 0) {
        std::snprintf(tmp, sizeof tmp, ", \"gate_escalated\": %lld", (long long)ctx->last_esc);
        s += tmp;
    }
    // pairs the last smooth sum summed (closed elements' coarser rules where
    // chosen), and what its base rules alone would have summed
    int64_t far_pairs = ctx->last_far_pairs;
    if (ctx->fpairs_ok && ctx->last_ntiles > 0) {
        std::vector<int64_t> fp((size_t)ctx->last_ntiles);
        if (hipMemcpy(fp.data(), ctx->fpairs.p, fp.size() * sizeof(int64_t), hipMemcpyDeviceToHost) == hipSuccess) {
            far_pairs = 0;
            for (int64_t v : fp) far_pairs += v;
        } else {
            (void)hipGetLastError();
        }
    }
    std::snprintf(tmp, sizeof tmp,
                  ", \"far_tpt\": %d, \"far_chunk\": %lld, \"far_pairs\": %lld, \"far_pairs_base\": %lld, "
                  "\"far_split\": %d",
                  ctx->far_tpt, (long long)ctx->far_chunk, (long long)far_pairs, (long long)ctx->last_far_pairs,
                  ctx->far_split ? 1 : 0);
    s += tmp;
    std::snprintf(tmp, sizeof tmp,
                  ", \"estimate\": {\"tol\": %.3e, \"cs\": %.1f, \"ct\": %.1f, \"hmin_fac\": %.3f, \"extra_modes\": %d}",
                  ctx->gc.tol, ctx->gc.cs, ctx->gc.ct, ctx->gc.hmin_fac, ctx->gc.extra_modes);
    s += tmp;
    {
        const size_t sl = ctx->table_path.find_last_of('/');
        s += ", \"theta_rules\": \"" + ctx->table_path.substr(sl == std::string::npos ? 0 : sl + 1) + "\"";
    }
    s += ctx->ker == KER_LAPLACE ? ", \"kernel\": \"laplace\"" : ", \"kernel\": \"stokes\"";
    if (!ctx->srule_path.empty()) {
        const size_t sl = ctx->srule_path.find_last_of('/');
        s += ", \"srule_table\": \"" + ctx->srule_path.substr(sl == std::string::npos ? 0 : sl + 1) + "\"";
    }
    s += ctx->opt.srule == CSBQ_SRULE_AUTO ? ", \"srule\": \"auto\""
         : ctx->opt.srule == CSBQ_SRULE_WHOLE ? ", \"srule\": \"whole\"" : ", \"srule\": \"general\"";
    if (ctx->have_geom) {
        std::snprintf(tmp, sizeof tmp,
                      ", \"elements_cylinder\": %lld, \"elements_sphere\": %lld, \"elements_torus_arc\": %lld",
                      (long long)ctx->n_cyl, (long long)ctx->n_sph, (long long)ctx->n_tor);
        s += tmp;
    }
    if (ctx->plan.valid) {
        std::snprintf(tmp, sizeof tmp, ", \"plan\": {\"matrix\": %s, \"build_ms\": %.3f, \"matrix_bytes\": %lld}",
                      ctx->plan.matrix ? "true" : "false", ctx->plan.build_ms,
                      (long long)(ctx->plan.matrix ? (int64_t)ctx->plan.nfull * EMAT_DOUBLES * 8 : 0));
        s += tmp;
    }
    if (ctx->ph_ok && ctx->last_nf > 0) {
        std::vector<int> wk((size_t)WORK_STRIDE * ctx->last_nf);
        if (hipMemcpy(wk.data(), ctx->work.p, wk.size() * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess) {
            long long nq = 0, nsn = 0, nqm = 0, nsm = 0, nwh = 0;
            for (size_t i = 0; i < wk.size(); i += WORK_STRIDE) {
                nq += wk[i];
                nsn += wk[i + 1];
                nqm += wk[i + 2];
                nsm += wk[i + 3];
                nwh += wk[i + 4];
            }
            std::snprintf(tmp, sizeof tmp,
                          ", \"theta_nodes\": %lld, \"s_nodes\": %lld, \"theta_modes\": %lld, \"s_modes\": %lld"
                          ", \"pairs_whole_rule\": %lld",
                          nq, nsn, nqm, nsm, nwh);
            s += tmp;
        }
    }
    if (ctx->ph_ok) {
        (void)hipEventSynchronize(ctx->ph[kNPhase - 1].b);
        s += ", \"ms\": {";
        for (int k = 0; k < kNPhase; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ctx->ph[k].a, ctx->ph[k].b) != hipSuccess) {
                (void)hipGetLastError();
                ms = -1.f;
            }
            std::snprintf(tmp, sizeof tmp, "%s\"%s\": %.4f", k ? ", " : "", ctx->ph[k].name, ms);
            s += tmp;
        }
        s += "}";
    }
    s += "}";
    std::snprintf(buf, (size_t)cap, "%s", s.c_str());
    return CSBQ_OK;
}

}  // extern "C"
