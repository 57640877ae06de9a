// csbq_kernels.hpp -- host-callable launchers of the gfx950 kernels.
// Every launcher enqueues on `st` and returns 0 or a hipError_t code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csbq_common.hpp"

namespace csbq {

int upload_constants(const double* gx, const double* gw, const double* lam, const double* D, const double* T);

int launch_expand(hipStream_t st, int E, const double* xc, const double* eps, const double* e1, const double* sa,
                  const double* sc, const int* esign, const int* ebody, const int* egroup, double* clq, double* circ,
                  ElemInfo* info, double* ny, double* nn, double* nw, int64_t N, int closed_fb);
// eoff (optional): element e's first output point (-1: skip the element)
// instead of e ns_f nt_f; Mtot is the arrays' leading dimension either way
int launch_expand_up(hipStream_t st, int E, int ns_f, int nt_f, const double* gx_f, const double* gw_f,
                     const double* clq, const ElemInfo* info, double* cpy, double* cpn, double* cpw, int64_t Mtot,
                     const int64_t* eoff = nullptr);
int launch_base_build(hipStream_t st, int E, const ElemInfo* info, const int64_t* boff, const double* ny,
                      const double* nn, const double* nw, int64_t N, const double* c0y, const double* c0n,
                      const double* c0w, int64_t M0, double* by, double* bn, double* bw, int64_t Nb);
// rnear (if not null, (NFS + NFT) E doubles): the candidate radius of each
// element in [0, E), then the distances from its centre beyond which the
// smooth sum may use far_ns(i) Gauss points in s (i < NFS) and far_nt(j)
// angles (0 < j < NFT) for it (+inf: never)
int launch_prep_sigma(hipStream_t st, int E, const double* sigma, const double* nw, int64_t N, double* sw,
                      double* sh, int* band, double eta, const ElemInfo* info, const double* circ, GateConsts gc,
                      double* rnear);
int launch_band_check(hipStream_t st, int E, const int* band_new, const int* band_plan, int* err);
int launch_fill_i32(hipStream_t st, int64_t n, int* v, int val);
int launch_sigma_up(hipStream_t st, int E, int ns_f, int nt_f, const double* sh, const double* Lup, const double* cpw,
                    double* swf, int64_t Mtot, const int64_t* eoff = nullptr);
int launch_sigma_base(hipStream_t st, int E, const ElemInfo* info, const int64_t* boff, const double* sw, int64_t N,
                      const double* swf0, int64_t M0, double* bsw, int64_t Nb);
int launch_targets(hipStream_t st, int64_t T, const double* x, const int64_t* tnode, const int* tgrp_in, int G,
                   const ElemInfo* info, const double* ny, int64_t N, double* xt, int* tgroup, int64_t* gstart,
                   int* err);
int launch_far(hipStream_t st, int64_t T, const double* xt, const double* sy, const double* sn, const double* ssw,
               int64_t N, const FarTile* tiles, int ntiles, double* part, bool mixed, double near2, int tpt, int ker,
               const FarSplit& spl);
int launch_search(hipStream_t st, int64_t T, const int* tgroup, const int* gel, const double* xt,
                  const int64_t* tnode, const ElemInfo* info, const double* rnear, const int64_t* off, int* cnt,
                  int* pe, int* pt);
// circles at the CGRID-point grid of every closest-circle bracket of every
// element: grid[((e NCIRC + k) CGRID + i) GRQ ..] (geometry only)
int launch_grid_circles(hipStream_t st, int E, const double* clq, double* grid);
int launch_classify(hipStream_t st, int64_t P, const int* perm, const int* pe, const int* pt, const double* xt,
                    int64_t T, const int64_t* tnode, const double* clq, const double* circ, const double* grid,
                    const ElemInfo* info, const double* tor,
                    const int* band, GateConsts gc, int8_t* tier, double* cls);
int launch_iota(hipStream_t st, int64_t P, int* v);
int launch_tier_keys(hipStream_t st, int64_t P, int E, const int8_t* tier, const int* pe, int* key, int* val);
// points (y, n, sigma w) of the upsampled rules of every element, per tier:
// element e's points of tier k are [e Mf[k], (e + 1) Mf[k]) of arrays with
// leading dimension Mtot[k]
struct UpRules {
    const double* y[NUP];
    const double* n[NUP];
    const double* sw[NUP];
    int64_t Mf[NUP];
    int64_t Mtot[NUP];
};
// ws: 4 ints per wavefront (first sorted position, pair count <= UP_PAIRS,
// element, tier index 0..NUP-1)
int launch_corr_up(hipStream_t st, const UpRules& ur, int nwaves, const int* ws, const int* sorted, const int* pt,
                   const double* xt, int64_t T, const ElemInfo* info, const int64_t* boff, const double* by,
                   const double* bn, const double* bsw, int64_t Nb, double* corr, int ker);
constexpr int FAR_BLOCK = 256;         // threads of a smooth-sum block (TPT targets each)

// Allocation-free smooth sum: limits of the one static scratch array per
// device (targets and nodes per call, partial-sum doubles) and its size.
constexpr int64_t NOALLOC_MAX_TARGETS = 262144;
constexpr int64_t NOALLOC_MAX_NODES = 262144;
constexpr int64_t NOALLOC_MAX_ELEMS = NOALLOC_MAX_NODES / NPE;
constexpr int64_t NOALLOC_PART_DOUBLES = 4LL << 20;       // 32 MiB of per-chunk partial sums
constexpr int64_t NOALLOC_MAX_TILES = 16384;
constexpr int NOALLOC_MAX_DEVICES = 64;
__host__ __device__ constexpr int64_t noalloc_align(int64_t b) { return (b + 255) / 256 * 256; }
// byte offsets of the scratch's buffers
constexpr int64_t NA_XT = 0;                                                                   // double [3][T]
constexpr int64_t NA_SW = NA_XT + noalloc_align(8 * 3 * NOALLOC_MAX_TARGETS);                  // double [3][N]
constexpr int64_t NA_SH = NA_SW + noalloc_align(8 * 3 * NOALLOC_MAX_NODES);                    // double [E][NS][NSH]
constexpr int64_t NA_PART = NA_SH + noalloc_align(8 * NOALLOC_MAX_ELEMS * NS * NSH);           // double [nch][6][T]
constexpr int64_t NA_TGROUP = NA_PART + noalloc_align(8 * NOALLOC_PART_DOUBLES);               // int [T]
constexpr int64_t NA_BAND = NA_TGROUP + noalloc_align(4 * NOALLOC_MAX_TARGETS);                // int [E][2]
constexpr int64_t NA_TILES = NA_BAND + noalloc_align(4 * 2 * NOALLOC_MAX_ELEMS);               // FarTile [ntiles]
constexpr int64_t NA_GSTART = NA_TILES + noalloc_align((int64_t)sizeof(FarTile) * NOALLOC_MAX_TILES);  // int64 [1]
constexpr int64_t NA_GNCHUNK = NA_GSTART + 256;                                                // int [1]
constexpr int64_t NA_ERR = NA_GNCHUNK + 256;                                                   // int [1]
constexpr int64_t NA_SIG = NA_ERR + 256;                                                       // double [N][3] (Laplace)
constexpr int64_t NOALLOC_SCRATCH_BYTES = NA_SIG + noalloc_align(8 * 3 * NOALLOC_MAX_NODES);

// Device address of this device's scratch array (the device must be
// current); looked up once per device with hipGetSymbolAddress.
int scratch_address(int device, void** out);
int launch_noalloc_setup(hipStream_t st, int ntiles, int nch, int64_t T, int64_t N, int tb, int64_t chunk,
                         FarTile* tiles, int* gnchunk, int* err);
// Correction-matrix form of the special quadrature (Section 3.2.1, the
// corrected rule's E): launch_corr_full in MODE_COUNT writes the rows of
// every pair (its s-nodes plus the far-field rule's rows) to count[]; in
// MODE_MATRIX the rows themselves (V: [rows][12][NT] kernel components times
// trigonometric basis functions summed over each row's angles; L: [rows][NS]
// interpolation weights), the pairs' rows starting at roff[]; launch_emat
// assembles E[p][12][NS][NT] = L^T V per pair; launch_emat_apply forms the
// pairs' corrections from E and the density's Fourier coefficients.
enum { MODE_DENSITY = 0, MODE_COUNT = 1, MODE_MATRIX = 2 };
constexpr int64_t EMAT_DOUBLES = 12 * NS * NT;
struct MatrixRows {
    const int64_t* roff;
    double* V;
    double* L;
    int* count;
    const double* lup0;
    const double* bw;
};
int launch_emat(hipStream_t st, int npairs, const int64_t* roff, const double* V, const double* L, int64_t p0,
                double* Em);
int launch_emat_apply(hipStream_t st, int npairs, const int* listf, const int* pe, const double* Em, const double* sh,
                      double* corr);
// the special quadrature's rule tables in device memory: theta-rules per
// distance bracket (offsets, nodes, weights, and cos, sin, 1 - cos of every
// node), the log rule, and the whole-element singular s-rules per (set,
// target GL index): wnb cylinder aspect brackets from 2^wb_lo, the sphere
// set wsph (-1: none), wany = 1 to apply the cylinder rules to every open
// element (wnb = 0 and wsph = -1: not used)
struct RuleArgs {
    const int* roff;
    const double* rth;
    const double* rw;
    int nb;
    const double* lx;
    const double* lw;
    int nl;
    const double* rcs;
    const double* rsn;
    const double* romc;
    const int* woff;
    const double* wd;
    const double* ww;
    int wb_lo, wnb, wl0, wsph, wany;
};
int launch_corr_full(hipStream_t st, int nfull, const int* listf, const int* pe, const int* pt, const double* xt,
                     int64_t T, const int64_t* tnode, const double* clq, const double* sh, const ElemInfo* info,
                     const int* band, const double* cls, const int64_t* boff, const double* by, const double* bn,
                     const double* bsw, int64_t Nb, const RuleArgs& ra, GateConsts gc, double* corr, int* err,
                     int* work, int mt_max, int ker, int mode = MODE_DENSITY, const MatrixRows* mr = nullptr);
int launch_reduce(hipStream_t st, int64_t T, const int* tgroup, const int* gnchunk, const double* part,
                  const int64_t* off, const int8_t* tier, const double* corr, double* usl, double* udl, int ker);
// scalar density into component 0 of a [N][3] array (the Laplace layers)
int launch_scalar_to_vec(hipStream_t st, int64_t N, const double* s, double* v);

}  // namespace csbq
