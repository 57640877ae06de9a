// csbq_solve.hpp -- launchers of the solve kernels (csbq_solve.hip).  Every
// launcher enqueues on `st` and returns 0 or a hipError_t code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csbq {

// blocks of the first stage of launch_mdot (the partial buffer holds k x that)
int mdot_blocks(int64_t n);
// out[j] (+)= sum_i V[j*ld + i] w[i], j < k, in a fixed order
int launch_mdot(hipStream_t st, int64_t n, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, int accumulate);
// w += sgn * sum_j h[j] V[j*ld + .]   (h on the device)
int launch_maxpy(hipStream_t st, int64_t n, int k, const double* V, int64_t ld, const double* h, double sgn,
                 double* w);
// y = a x + b y
int launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y);
// y = tau/2 + dsign udl + eta usl (+ extra)
int launch_combine(hipStream_t st, int64_t n, const double* tau, const double* usl, const double* udl, double eta,
                   double dsign, const double* extra, double* y);
// per body: centroid, area, first and second moments (13 doubles)
int launch_body_geometry(hipStream_t st, int B, const int64_t* boff, const double* ny, const double* nw, int64_t N,
                         double* geo);
// per body: coef = Ginv (sum w sigma, sum w (y - c) x sigma)
int launch_body_project(hipStream_t st, int B, const int64_t* boff, const double* ny, const double* nw, int64_t N,
                        const double* geo, const double* Ginv, const double* sigma, double* coef);
// out = base + scale * (a + beta x (y - c)) per body (coef = a, beta)
int launch_rigid_field(hipStream_t st, int64_t N, int B, const int64_t* boff, const double* ny, const double* geo,
                       const double* coef, double scale, const double* base, double* out);
int launch_iota64(hipStream_t st, int64_t n, int64_t* v);

}  // namespace csbq
