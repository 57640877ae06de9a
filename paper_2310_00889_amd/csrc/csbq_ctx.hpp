// csbq_ctx.hpp -- the library context shared by the C ABI translation units
// (evaluation in csbq_api.cpp, boundary-integral solves in csbq_solve.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/csbq.h"
#include "csbq_common.hpp"
#include "csbq_gate.hpp"
#include "csbq_kernels.hpp"

namespace csbq {

// grow-only device buffer
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t m)
    {
        if (m <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        size_t bytes = (m ? m : 1) * sizeof(T);
        hipError_t e = hipMalloc((void**)&p, bytes);
        if (e == hipSuccess) n = m;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
};

struct Phase {
    const char* name;
    hipEvent_t a, b;
};

constexpr int kNPhase = 8;

}  // namespace csbq

// private header of the library's own translation units
using namespace csbq;

struct csbq_ctx {
    csbq_options opt{};
    int ker = KER_STOKES;   // kernel pair (csbq_options.kernel)
    int nc() const { return ker == KER_LAPLACE ? 1 : 3; }   // density / output components
    DBuf<double> sig1;      // a scalar density before its expansion into three components
    std::string err;
    std::string table_dir, table_path, srule_path;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    GateConsts gc{};
    int closed_fb = 2;   // far-field rule of elements closed at an end: 2 = up_ns(0) x NT, 1 = their own nodes
    // quadrature tables
    DBuf<int> roff;
    DBuf<double> rth, rw, lx, lw, rcs, rsn, romc;
    int nb = 0, nl = 0;
    // whole-element singular s-rules (csbq_srule WHOLE): offsets per (aspect
    // bracket, target GL index), node offsets and weights; wnb = 0 when the
    // context uses the general rule
    DBuf<int> woff;
    DBuf<double> wd, ww;
    int wb_lo = 0, wnb = 0, wl0 = 0, wsph = -1;
    int64_t n_cyl = 0, n_sph = 0;   // elements of the geometry with those shapes
    double gx[NS], gw[NS], lam[NS];
    double Dgl[NS * NS];   // differentiation matrix at the GL nodes of [-1, 1]
    // geometry
    int E = 0;
    int64_t N = 0;
    bool have_geom = false;
    DBuf<double> g_xc, g_eps, g_e1, g_sa, g_sc;
    DBuf<int> g_sign, g_body, g_group;
    // batch of independent geometries: elements [h_gel[g], h_gel[g+1]) form group g
    int G = 1;
    std::vector<int> h_gel;
    std::vector<int64_t> h_boff;
    DBuf<int> gel;
    DBuf<double> clq, circ, gridc, ny, nn, nw;
    DBuf<ElemInfo> info;
    DBuf<double> cpy[NUP], cpn[NUP], cpw[NUP], Lup[NUP], upx[NUP], upw[NUP];
    int64_t Mtot[NUP] = {0, 0, 0};
    // coarser far-field rules: Lagrange matrices and Gauss tables per number
    // of points in s; each element's rules sit in the base source set
    // (rule k of element e at loff[k E + e], -1: none)
    DBuf<double> Lfar[NFS], farx[NFS], farw[NFS];
    DBuf<int64_t> loff;
    DBuf<double> tor;   // torus-arc parameters per element (TOR_Q), for the classification
    int64_t n_tor = 0;
    bool far_used[NFL] = {};
    // far-field (base) source set
    int64_t Nb = 0;         // base sources: the base rules, then the elements' coarser far-field rules
    int64_t Nb_rules = 0;   // the base rules alone
    double mix_near2 = 0.0;   // squared radius of the FP64 near part of the mixed-precision far sum
    DBuf<int64_t> boff;
    DBuf<double> by, bn, bw, bsw;
    // evaluation scratch
    DBuf<double> sig_d, x_d, usl_d, udl_d;
    DBuf<int64_t> tn_d;
    DBuf<double> sw, sh, rnear, xt, part, cls, corr, swf[NUP];
    DBuf<int> band, cnt, pe, pt, err_d, work, kin, kout, vin, perm, sorted, runs_key, runs_cnt, nruns, wdesc;
    DBuf<int64_t> off, gstart;
    DBuf<int> tgroup, tgrp_d, gnchunk;
    DBuf<FarTile> tiles;
    DBuf<int8_t> tier;
    // smooth-sum launch shape, chosen by timing (targets per thread, sources per chunk)
    int far_tpt = 2;
    int64_t far_chunk = 16384;
    uint64_t tuned_key = 0;
    float tune_ms[6] = {0, 0, 0, 0, 0, 0};
    // learned gate: inference weights (bf16 MFMA fragments, FP32 biases) and
    // per-pair scratch
    bool gate_ready = false;
    float gate_tau = 0.05f;
    DBuf<uint16_t> gate_wfrag;
    DBuf<float> gate_bias, gfeat;
    DBuf<int8_t> gtier;
    DBuf<uint8_t> gesc, gflag;
    DBuf<int> gsel, gnsel;
    int64_t last_esc = -1;
    // frozen evaluation plan (pairs, tiers, rules, smooth-sum blocks of the
    // last evaluation) and its apply sequence captured as a HIP graph
    struct Plan {
        bool valid = false;
        int64_t T = 0;
        int nwaves[NUP] = {0, 0, 0};   // upsampled-rule wavefronts per tier
        int nw_up = 0;                 // all of them, in the one launch
        int nfull = 0, full_start = 0, mt_max = 0, ntiles = 0, tpt = 2;
        bool mixed = false;
        bool matrix = false;           // special-quadrature corrections from the stored matrices
        float build_ms = 0.f;          // time to build them
        const int64_t* tn = nullptr;
        hipStream_t gst = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
    } plan;
    DBuf<int> band_apply;
    // correction matrices of the special-quadrature pairs (plan with
    // CSBQ_PLAN_MATRIX): EMAT_DOUBLES per pair, in the plan's pair order
    DBuf<double> emat;
    int last_ntiles = 0;
    int64_t last_far_pairs = 0;   // source-target pairs of the last smooth sum's base rules
    DBuf<int64_t> fpairs;         // per block of the last smooth sum: pairs summed (coarser rules where chosen)
    bool fpairs_ok = false;
    bool far_split = true;        // closed elements' coarser far-field rules where they suffice
    // host copies of the smooth-sum block list outlive the asynchronous uploads;
    // the device copy is reused while geometry, targets and shape stay
    std::vector<FarTile> h_tiles;
    std::vector<int> h_gnc;
    bool tiles_valid = false, tiles_native = false;
    int tiles_tpt = 0, tiles_maxch = 0;
    int64_t tiles_chunk = 0, tiles_T = -1;
    std::vector<int64_t> tiles_tr;
    DBuf<unsigned char> cub_tmp;
    // statistics of the last evaluation
    Phase ph[kNPhase];
    bool ph_ok = false;
    int64_t last_T = 0, last_P = 0, last_nup[NUP] = {0, 0, 0}, last_nf = 0;
    int last_err_flags = 0;
    bool flags_pending = false;   // device-mode call: the final flags are still on the device
    int* flags_src = nullptr;     // device flag word of the last call (err_d or the static scratch's)
    // boundary-integral solves: rules and tiers chosen for the widest band a
    // density can have (every Legendre degree and Fourier mode), so that one
    // frozen plan holds for any density (every Krylov vector)
    bool full_band = false;
    int n_bodies = 0;
    std::vector<int64_t> h_body_off;   // surface-node offsets of the bodies [n_bodies + 1]
    DBuf<int64_t> s_boff, s_tn;
    DBuf<double> s_geo, s_ginv, s_coef, s_V, s_w, s_h, s_part, s_b, s_x, s_tau, s_usl, s_udl, s_nu, s_lsig;
    unsigned char* scratch = nullptr;   // this device's static scratch (allocation-free smooth sum)

    int fail(int code, const std::string& msg)
    {
        err = msg;
        return code;
    }
};

#define HIPC(call)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ctx->fail(CSBQ_EHIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)
#define ALLOC(buf, n)                                                                 \
    do {                                                                              \
        if ((buf).ensure(n) != hipSuccess) {                                          \
            (void)hipGetLastError();                                                  \
            return ctx->fail(CSBQ_ENOMEM, "device allocation failed: " #buf);         \
        }                                                                             \
    } while (0)
#define LCHK(call)                                                                                  \
    do {                                                                                            \
        int r_ = (call);                                                                            \
        if (r_) return ctx->fail(CSBQ_EHIP, std::string(#call " failed: ") +                        \
                                                hipGetErrorString((hipError_t)r_));                \
    } while (0)
