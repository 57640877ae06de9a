// csbq_kernels.hpp -- host-callable launchers of the gfx950 kernels.
// Every launcher enqueues on `st` and returns 0 or a hipError_t code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csbq_common.hpp"

namespace csbq {

int upload_constants(const double* gx, const double* gw, const double* lam, const double* D, const double* T);

int launch_expand(hipStream_t st, int E, const double* xc, const double* eps, const double* e1, const double* sa,
                  const double* sc, const int* esign, const int* ebody, double* clq, double* circ, ElemInfo* info,
                  double* ny, double* nn, double* nw, int64_t N);
int launch_expand_up(hipStream_t st, int E, int f, const double* clq, const ElemInfo* info, const double* ny,
                     const double* nn, const double* nw, int64_t N, double* cpy, double* cpn, double* cpw,
                     int64_t Mtot);
int launch_prep_sigma(hipStream_t st, int E, const double* sigma, const double* nw, int64_t N, double* sw,
                      double* sh, int* band, double eta, const ElemInfo* info, GateConsts gc, double* rnear);
int launch_sigma_up(hipStream_t st, int E, int f, const double* sh, const double* Lup, const double* cpw,
                    const double* sw, int64_t N, double* swf, int64_t Mtot);
int launch_targets(hipStream_t st, int64_t T, const double* x, const int64_t* tnode, const double* ny, int64_t N,
                   double* xt, int* err);
int launch_far(hipStream_t st, int64_t T, const double* xt, const double* sy, const double* sn, const double* ssw,
               int64_t N, int64_t chunk, int nchunk, double* part);
int launch_search(hipStream_t st, int64_t T, int E, const double* xt, const int64_t* tnode, const ElemInfo* info,
                  const double* rnear, const int64_t* off, int* cnt, int* pe, int* pt);
int launch_classify(hipStream_t st, int64_t P, const int* pe, const int* pt, const double* xt, int64_t T,
                    const int64_t* tnode, const double* clq, const double* circ, const ElemInfo* info,
                    const int* band, GateConsts gc, int8_t* tier, double* cls);
int launch_bucket_count(hipStream_t st, int64_t P, const int8_t* tier, const int* pe, int* cnt2, int* cnt4,
                        int* nfull);
int launch_bucket_fill(hipStream_t st, int64_t P, const int8_t* tier, const int* pe, int* cur2, int* cur4,
                       int* curf, int64_t* list2, int64_t* list4, int64_t* listf);
int launch_corr_up(hipStream_t st, int f, int nwaves, const int* wave_elem, const int64_t* list, const int* pt,
                   const double* xt, int64_t T, const double* cpy, const double* cpn, const double* swf,
                   int64_t Mtot, double* corr);
int launch_corr_full(hipStream_t st, int nfull, const int64_t* listf, const int* pe, const int* pt, const double* xt,
                     int64_t T, const int64_t* tnode, const double* clq, const double* sh, const ElemInfo* info,
                     const int* band, const double* cls, const double* ny, const double* nn, const double* sw,
                     int64_t N, const int* roff, const double* rth, const double* rw, int nb, const double* lx,
                     const double* lw, int nl, GateConsts gc, double* corr, int* err, int* work);
int launch_reduce(hipStream_t st, int64_t T, int nchunk, const double* part, const int64_t* off, const int8_t* tier,
                  const double* corr, double* usl, double* udl);

}  // namespace csbq
