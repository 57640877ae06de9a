// csbq_math.hpp -- scalar geometry and estimate helpers shared by the kernels.
#pragma once
#include "csbq_common.hpp"

namespace csbq {

struct Frame {
    double X[3], Xp[3], E, Ep;   // centre, d/ds centre, radius, d/ds radius
    double t[3];                 // unit tangent
    double e1[3], e2[3];         // orthonormal cross-section frame, e2 = t x e1
    double e1p[3], e2p[3];       // d/ds of e1, e2
    double sp;                   // |x_c'|
};

__host__ __device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__host__ __device__ inline void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Frame at one s from the centerline quantities q[CLQ] (values and s-derivatives
// of x_c, eps, e1 there).  e1 is re-orthonormalised against the tangent
// (Section 3.1.1) and its derivative is that of the re-orthonormalised vector.
__host__ __device__ inline void frame_from_q(const double* q, Frame& f)
{
    for (int d = 0; d < 3; ++d) {
        f.X[d] = q[Q_X + d];
        f.Xp[d] = q[Q_XP + d];
    }
    f.E = q[Q_E];
    f.Ep = q[Q_EP];
    const double* Xpp = q + Q_XPP;
    const double* F = q + Q_F;
    const double* Fp = q + Q_FP;
    double sp = sqrt(dot3(f.Xp, f.Xp));
    f.sp = sp;
    double isp = 1.0 / sp;
    for (int d = 0; d < 3; ++d) f.t[d] = f.Xp[d] * isp;
    double tpp = dot3(Xpp, f.t);
    double tp[3];
    for (int d = 0; d < 3; ++d) tp[d] = (Xpp[d] - tpp * f.t[d]) * isp;
    double ft = dot3(F, f.t);
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = F[d] - ft * f.t[d];
    double un = sqrt(dot3(u, u));
    double iun = 1.0 / un;
    for (int d = 0; d < 3; ++d) f.e1[d] = u[d] * iun;
    cross3(f.t, f.e1, f.e2);
    double fpt = dot3(Fp, f.t), ftp = dot3(F, tp);
    double up[3];
    for (int d = 0; d < 3; ++d) up[d] = Fp[d] - (fpt + ftp) * f.t[d] - ft * tp[d];
    double upe = dot3(up, f.e1);
    for (int d = 0; d < 3; ++d) f.e1p[d] = (up[d] - upe * f.e1[d]) * iun;
    double c1[3], c2[3];
    cross3(tp, f.e1, c1);
    cross3(f.t, f.e1p, c2);
    for (int d = 0; d < 3; ++d) f.e2p[d] = c1[d] + c2[d];
}

// Surface point, dy/ds and dy/dt at angle (cos, sin) of a frame.
__host__ __device__ inline void surface_at(const Frame& f, double ct, double st, double* y, double* ys, double* yt)
{
    for (int d = 0; d < 3; ++d) {
        double b = f.e1[d] * ct + f.e2[d] * st;
        double bp = f.e1p[d] * ct + f.e2p[d] * st;
        y[d] = f.X[d] + f.E * b;
        ys[d] = f.Xp[d] + f.Ep * b + f.E * bp;
        yt[d] = f.E * (-f.e1[d] * st + f.e2[d] * ct);
    }
}

// Upper bound of |dy/ds| over the circle of a frame.
__host__ __device__ inline double speed_bound(const Frame& f)
{
    return f.sp + fabs(f.Ep) + f.E * (sqrt(dot3(f.e1p, f.e1p)) + sqrt(dot3(f.e2p, f.e2p)));
}

// Barycentric Lagrange weights at normalised point x in [-1,1] for the GL
// nodes gx with barycentric weights lam (second, "true" barycentric form).
__host__ __device__ inline void bary_weights(double x, const double* gx, const double* lam, double* l)
{
    double sum = 0.0;
    int hit = -1;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        double dx = x - gx[i];
        if (dx == 0.0) hit = i;
        l[i] = lam[i] / (hit == i ? 1.0 : dx);
        sum += l[i];
    }
    if (hit >= 0) {
        for (int i = 0; i < NS; ++i) l[i] = (i == hit) ? 1.0 : 0.0;
        return;
    }
    double is = 1.0 / sum;
#pragma unroll
    for (int i = 0; i < NS; ++i) l[i] *= is;
}

// Barycentric weights at x = gx[i0] + du (du small), forming every x - gx[i]
// without cancellation: used for points close to the GL node i0.
__host__ __device__ inline void bary_weights_rel(int i0, double du, const double* gx, const double* lam, double* l)
{
    if (du == 0.0) {
        for (int i = 0; i < NS; ++i) l[i] = (i == i0) ? 1.0 : 0.0;
        return;
    }
    double sum = 0.0;
    for (int i = 0; i < NS; ++i) {
        double dx = (i == i0) ? du : (gx[i0] - gx[i]) + du;
        l[i] = lam[i] / dx;
        sum += l[i];
    }
    double is = 1.0 / sum;
    for (int i = 0; i < NS; ++i) l[i] *= is;
}

// Bernstein-ellipse parameter of the complex point (zr + i zi) relative to the
// interval [lo, hi] (Trefethen, ATAP Thm 19.3): rho = |t + sqrt(t^2 - 1)| >= 1.
__host__ __device__ inline double bernstein_rho(double zr, double zi, double lo, double hi)
{
    double h = 0.5 * (hi - lo);
    double tr = (zr - 0.5 * (lo + hi)) / h, ti = zi / h;
    // w = t^2 - 1
    double wr = tr * tr - ti * ti - 1.0, wi = 2.0 * tr * ti;
    double m = sqrt(wr * wr + wi * wi);
    double sr = sqrt(fmax(0.0, 0.5 * (m + wr)));
    double si = sqrt(fmax(0.0, 0.5 * (m - wr)));
    if (wi < 0) si = -si;
    double p1 = (tr + sr) * (tr + sr) + (ti + si) * (ti + si);
    double p2 = (tr - sr) * (tr - sr) + (ti - si) * (ti - si);
    return sqrt(fmax(p1, p2));
}

// Target position relative to the circle of a frame: axial offset z, radial
// distance rho_t, and the unit radial direction b0 (e1 if on the axis).
struct CircleLocal {
    double z, rho, dr;   // dr = rho - eps
    double b0[3], b0p[3];  // radial direction and t x b0
    double d2;           // squared distance to the circle
    double cha;          // cosh(a) - 1 = d^2 / (2 rho eps)  (trapezoid decay rate a)
};

__host__ __device__ inline void circle_local(const Frame& f, const double* x, CircleLocal& c)
{
    double v[3] = {x[0] - f.X[0], x[1] - f.X[1], x[2] - f.X[2]};
    c.z = dot3(v, f.t);
    double w[3] = {v[0] - c.z * f.t[0], v[1] - c.z * f.t[1], v[2] - c.z * f.t[2]};
    double r2 = dot3(w, w);
    c.rho = sqrt(r2);
    if (c.rho > 0.0) {
        double ir = 1.0 / c.rho;
        for (int d = 0; d < 3; ++d) c.b0[d] = w[d] * ir;
    } else {
        for (int d = 0; d < 3; ++d) c.b0[d] = f.e1[d];
    }
    cross3(f.t, c.b0, c.b0p);
    c.dr = c.rho - f.E;
    c.d2 = c.dr * c.dr + c.z * c.z;
    // a vanishing (or rounding-negative) radius: constant angular integrand
    c.cha = (c.rho > 0.0 && f.E > 1e-300) ? c.d2 / (2.0 * c.rho * f.E) : 1e300;
}

// Local coordinates of an on-surface target relative to a nearby circle of
// the same element.  The target is the node at angle direction bn (unit) on
// the circle of frame f0 (s = s0); the circle has frame f at s = s0 + u and
// dq = q(s) - q(s0) holds the interpolated differences of the centerline
// quantities.  Every coordinate that vanishes with u (z, rho - eps) is formed
// from differences, so it keeps its relative accuracy as u -> 0; this is what
// keeps the r.n = O(|r|^2) factor of the double layer free of rounding noise.
__host__ __device__ inline void circle_local_rel(const Frame& f, const Frame& f0, const double* bn, const double* dq,
                                                 CircleLocal& c)
{
    const double* dX = dq + Q_X;
    const double* dXp = dq + Q_XP;
    const double dE = dq[Q_E];
    const double E0 = f0.E;
    double v[3];
    for (int d = 0; d < 3; ++d) v[d] = E0 * bn[d] - dX[d];
    double sm[3] = {f.Xp[0] + f0.Xp[0], f.Xp[1] + f0.Xp[1], f.Xp[2] + f0.Xp[2]};
    double dsp = dot3(dXp, sm) / (f.sp + f0.sp);
    double dt[3];
    for (int d = 0; d < 3; ++d) dt[d] = (dXp[d] - f0.t[d] * dsp) / f.sp;
    c.z = E0 * dot3(bn, dt) - dot3(dX, f.t);
    double w[3] = {v[0] - c.z * f.t[0], v[1] - c.z * f.t[1], v[2] - c.z * f.t[2]};
    c.rho = sqrt(dot3(w, w));
    double ir = 1.0 / c.rho;
    for (int d = 0; d < 3; ++d) c.b0[d] = w[d] * ir;
    cross3(f.t, c.b0, c.b0p);
    double r2mE2 = -dE * (2.0 * E0 + dE) - 2.0 * E0 * dot3(bn, dX) + dot3(dX, dX) - c.z * c.z;
    c.dr = r2mE2 / (c.rho + f.E);
    c.d2 = c.dr * c.dr + c.z * c.z;
    c.cha = (f.E > 1e-300) ? c.d2 / (2.0 * c.rho * f.E) : 1e300;
}

// Local coordinates of a free target relative to a circle of an element, in
// the same difference form: xr = x - x_c(s0) is the target's offset from the
// centerline at a reference node s0 of frame f0, z_ref = xr.t0 and
// k_ref = |xr|^2 - eps0^2 (both formed once per pair, so their rounding is the
// same for every circle), dq = q(s) - q(s0).  Then
//   z = z_ref + xr.(t - t0) - dX.t,
//   rho^2 - eps^2 = k_ref - 2 xr.dX + |dX|^2 - z^2 - deps (2 eps0 + deps),
// and the distance to the circle keeps its relative accuracy however close the
// target is (an on-surface target is xr = eps0 bn, z_ref = k_ref = 0).
__host__ __device__ inline void circle_local_off(const Frame& f, const Frame& f0, const double* xr, double z_ref,
                                                 double k_ref, const double* dq, CircleLocal& c)
{
    const double* dX = dq + Q_X;
    const double* dXp = dq + Q_XP;
    const double dE = dq[Q_E];
    const double E0 = f0.E;
    double v[3];
    for (int d = 0; d < 3; ++d) v[d] = xr[d] - dX[d];
    double sm[3] = {f.Xp[0] + f0.Xp[0], f.Xp[1] + f0.Xp[1], f.Xp[2] + f0.Xp[2]};
    double dsp = dot3(dXp, sm) / (f.sp + f0.sp);
    double dt[3];
    for (int d = 0; d < 3; ++d) dt[d] = (dXp[d] - f0.t[d] * dsp) / f.sp;
    c.z = z_ref + dot3(xr, dt) - dot3(dX, f.t);
    double w[3] = {v[0] - c.z * f.t[0], v[1] - c.z * f.t[1], v[2] - c.z * f.t[2]};
    c.rho = sqrt(dot3(w, w));
    if (c.rho > 0.0) {
        double ir = 1.0 / c.rho;
        for (int d = 0; d < 3; ++d) c.b0[d] = w[d] * ir;
    } else {
        for (int d = 0; d < 3; ++d) c.b0[d] = f.e1[d];
    }
    cross3(f.t, c.b0, c.b0p);
    double r2mE2 = k_ref - dE * (2.0 * E0 + dE) - 2.0 * dot3(xr, dX) + dot3(dX, dX) - c.z * c.z;
    c.dr = r2mE2 / (c.rho + f.E);
    c.d2 = c.dr * c.dr + c.z * c.z;
    c.cha = (c.rho > 0.0 && f.E > 1e-300) ? c.d2 / (2.0 * c.rho * f.E) : 1e300;
}

// a = acosh(1 + cha), stable for small cha
__host__ __device__ inline double acosh1p(double cha)
{
    return log1p(cha + sqrt(cha * (cha + 2.0)));
}

}  // namespace csbq
