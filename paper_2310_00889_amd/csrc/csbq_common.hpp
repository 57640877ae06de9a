// csbq_common.hpp -- shared definitions of the gfx950 layer-potential library.
//
// Fixed discretisation orders of the library: NS Gauss-Legendre nodes per panel
// in s and NT uniform angles (Section 3.1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csbq {

constexpr int NS = 16;
constexpr int NT = 32;
constexpr int NPE = NS * NT;           // nodes per element
constexpr int NMODE = NT / 2 + 1;      // Fourier modes 0..NT/2 of a real density
constexpr int NSH = NMODE * 6;         // per GL row: (a_x a_y a_z b_x b_y b_z) per mode
constexpr int CLQ = 17;                // centerline quantities per GL node
constexpr int NCIRC = NS + 2;          // GL circles + the two panel-end circles
constexpr int CIRQ = 9;                // per circle: X(3) t(3) eps smax s
constexpr int CGRID = 9;               // grid circles per closest-circle bracket
constexpr int GRQ = 8;                 // per grid circle: X(3) t(3) eps, padded
constexpr int MAXSUB = 96;             // s sub-panels of one special quadrature
constexpr int MAXRULE = 256;           // nodes of one theta rule
constexpr int MAXLOG = 64;             // nodes of the log rule
constexpr int MAXWHOLE = 160;          // nodes of one whole-element singular s-rule
constexpr int WORK_STRIDE = 5;         // per special-quadrature pair: theta nodes, s-nodes, their mode
                                       // counts, whole-element rule used (work counters)

// centerline quantity slots (clq[e][q][i], i = GL node)
enum { Q_X = 0, Q_XP = 3, Q_XPP = 6, Q_E = 9, Q_EP = 10, Q_F = 11, Q_FP = 14 };

// correction tiers of a (target, element) pair: skip, three upsampled
// whole-panel tensor rules (Gauss-Legendre of up_ns points in s times up_nt
// angles), and the special quadrature
enum : int8_t { TIER_SKIP = 0, TIER_UP1 = 1, TIER_UP2 = 2, TIER_UP3 = 3, TIER_FULL = 4 };
constexpr int NUP = 3;
constexpr int UP_TPT = 2;              // pairs per lane of the upsampled-rule corrections
constexpr int UP_PAIRS = 64 * UP_TPT;  // pairs per wavefront (one element)
constexpr int MAXUPNS = 64;
__host__ __device__ constexpr int up_ns(int k) { return k == 2 ? 64 : 32; }
__host__ __device__ constexpr int up_nt(int k) { return k == 0 ? 32 : (k == 1 ? 64 : 128); }
__host__ __device__ constexpr int64_t up_pts(int k) { return (int64_t)up_ns(k) * up_nt(k); }

// Far-field rules of the smooth sum coarser than an element's base rule:
// Gauss-Legendre of far_ns(i) points in s (i < NFS) times far_nt(j) angles
// (j < NFT), rule k = i NFT + j.  An element closed at an end (base rule
// up_ns(0) x NT) may take i in [0, 3): 24, 20 or 16 points; any other element
// (base rule: its own N_s x N_theta nodes) i in [2, 5): 16, 12 or 8 points,
// its base being the rule FAR_OPEN_BASE.  The rules follow the base rules in
// the base source set.
constexpr int NFS = 5, NFT = 3, NFL = NFS * NFT, FAR_NI = 3;
__host__ __device__ constexpr int far_ns(int i) { return i == 0 ? 24 : i == 1 ? 20 : i == 2 ? NS : i == 3 ? 12 : 8; }
__host__ __device__ constexpr int far_nt(int j) { return j == 0 ? NT : (j == 1 ? 24 : 16); }
__host__ __device__ constexpr int64_t far_pts(int k) { return (int64_t)far_ns(k / NFT) * far_nt(k % NFT); }
__host__ __device__ constexpr int far_i0(bool closed) { return closed ? 0 : 2; }
constexpr int FAR_OPEN_BASE = 2 * NFT;
static_assert(far_ns(2) == NS && far_nt(0) == NT, "rule FAR_OPEN_BASE is an element's own nodes");

// kernel pair of an evaluation: the Stokes single and double layers (Section
// 2) or the Laplace ones (Section 4.1)
enum : int { KER_STOKES = 0, KER_LAPLACE = 1 };

// bits of the evaluation's device flag word (the C ABI names them CSBQ_FLAG_*)
enum : int {
    FLAG_NODE_RANGE = 1,    // a target's node id is beyond the node count
    FLAG_SRULE_LIMIT = 2,   // an off-surface s-rule stopped bisecting at its limit
    FLAG_THETA_CLAMP = 4,   // a circle closer than the finest theta-rule bracket
    FLAG_GROUP_RANGE = 8,   // a free target's group is out of range
    FLAG_GROUP_ORDER = 16,  // targets not ordered by group
    FLAG_BAND = 32          // a density wider in band than a frozen plan's
};

// sub-panel kinds of an s-rule
// (log singularity at lo / at hi; SUB_WHOLE: one tabulated rule over the
// whole element for an on-surface target, Section 3.2.4)
enum : int { SUB_GL = 0, SUB_LOG_LO = 1, SUB_LOG_HI = 2, SUB_WHOLE = 3 };

struct ElemInfo {
    double a, c;       // panel interval in s
    double cen[3];     // bounding-ball centre
    double rad;        // bounding-ball radius
    double eps_max;    // largest cross-section radius
    double smax;       // largest surface speed |dy/ds| bound
    int32_t sign;      // normal orientation
    int32_t body;
    int32_t fb;        // far-field (base) rule: 1 = the element's own nodes, 2 = up_ns(0) x NT rule
    int32_t group;     // geometry of a batch: elements of different groups do not interact
    int32_t closed;    // the cross-section closes at a panel end
    int32_t shape;     // SHAPE_*: a shape a whole-element singular s-rule was built from
};

// element shapes with tabulated whole-element singular s-rules (Section
// 3.2.4): a straight cylinder of constant radius at constant speed with a
// constant e1, and a sphere as one element in its polar-angle
// parametrisation with a constant e1
enum : int { SHAPE_OTHER = 0, SHAPE_CYLINDER = 1, SHAPE_SPHERE = 2 };

// per element, the parameters of a torus-arc element (see the host's test):
// C(3), U(3), V(3), R, r, psi0, psi1, unused, flag (1: such an element)
constexpr int TOR_Q = 16;

// one block of the smooth sum: up to 256 x (targets per thread) consecutive
// targets of one group against a chunk of that group's sources.  A chunk is
// either a plain source range [s0, s0 + sn) or, when e1 > e0, the far-field
// rules of the whole elements [e0, e1) (sn then counts their base sources)
struct FarTile {
    int64_t t0, s0;    // first target, first source
    int32_t tn, sn;    // counts
    int32_t chunk;     // partial-sum slot
    int32_t e0, e1;    // element range (element chunks only)
    int32_t pad_;
};

// Element chunks of the smooth sum: an element is summed with the coarsest
// of its far_ns(i) x far_nt(j) rules whose radii from the element's centre
// (one for the points in s, one for the angles) the block's targets all lie
// beyond: the distances at which the same error estimates that choose the
// candidates let the rule meet the tolerance; else with its base rule.
struct FarSplit {
    const int64_t* boff;    // element e's base rule: sources [boff[e], boff[e + 1])
    const int64_t* loff;    // rule k of element e: sources loff[k E + e] .. + far_pts(k) (-1: none)
    const double* rc;       // radii (+inf: never), or null: base rules only: rc[i E + e] for far_ns(i) points
                            // in s (i < NFS), rc[(NFS + j - 1) E + e] for far_nt(j) angles (0 < j < NFT)
    const ElemInfo* info;   // element centres
    int64_t* pairs;         // per block: source-target pairs summed (or null)
    int E;
};

// constants of the error estimates (calibrated against the CPU oracle)
struct GateConsts {
    double tol;        // per-element quadrature tolerance
    double cs;         // Gauss-Legendre estimate prefactor
    double ct;         // trapezoid estimate prefactor
    double hmin_fac;   // dyadic refinement stops at hmin_fac * eps / speed
    int extra_modes;   // modes added to the density band for J and the normal
};

}  // namespace csbq
