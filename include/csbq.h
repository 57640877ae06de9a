/*
 * csbq.h -- C ABI of the MI355X (gfx950) Stokes layer-potential evaluator.
 *
 * Computes, at a set of targets x, the Stokes single-layer (stokeslet) and
 * double-layer (stresslet) velocity potentials of smooth densities given on
 * panel-discretised bodies (Malhotra & Barnett, "Efficient convergent boundary
 * integral methods for slender bodies"):
 *
 *   u_S(x) = int S(x - y) sigma(y) dS_y,  S(r) = (I/|r| + r r^T/|r|^3) / (8 pi)
 *   u_D(x) = int D(x - y; n_y) sigma(y) dS_y,  D(r; n) = -(3/(4 pi)) (r.n) r r^T / |r|^5
 *
 * (Section 2, single- and double-layer velocity kernels; viscosity 1).  The
 * two outputs are returned separately; a caller combines them as needed
 * (Section 3.2.1: the kernel may be any linear combination of S and D).
 *
 * Method (Section 3.2): the smooth Nystrom sum over every node (Eq. for the
 * Nystrom rule without corrections) plus local corrections for every
 * (target, element) pair inside the element's near region (Eq. for the
 * Nystrom rule with corrections): upsampled tensor rules, or the special
 * quadrature of Sections 3.2.2-3.2.4 (theta-integrals by generalised
 * Chebyshev rules per distance bracket, adaptive Gauss-Legendre panels in s
 * for near targets, dyadic + log-singular panels in s for on-surface targets).
 *
 * Geometry (Section 3.1): a body is a centerline x_c(s), s in its parameter
 * interval, cross-section radius eps(s) and orientation vector e1(s)
 * orthogonal to the centerline, all given by their values at the ns
 * Gauss-Legendre nodes (ascending) of each panel [s_break[k], s_break[k+1]].
 * The surface is y(s,t) = x_c + eps (e1 cos t + e2 sin t), e2 = t_c x e1 with
 * t_c the unit tangent and e1 re-orthonormalised against t_c wherever it is
 * evaluated (Section 3.1.1).  Surface nodes are the ns GL nodes of each panel
 * times nt angles t_j = 2 pi j / nt, numbered body-major, then panel, s-node,
 * angle.  The normal is normal_sign * (dy/dt x dy/ds) / J, J = |dy/ds x dy/dt|;
 * with normal_sign = +1 it points away from the centerline.  A density is
 * given by its values at the nodes and interpolated polynomially in s and
 * trigonometrically in t.
 *
 * Conventions for every entry point:
 *  - return value: CSBQ_OK (0) or a negative csbq_status; no C++ exception
 *    crosses the ABI; csbq_last_error() returns the message of the last error
 *    of that context (thread-unsafe; one context per thread).
 *  - mem = CSBQ_HOST: pointers are host memory; the call is synchronous.
 *    mem = CSBQ_DEVICE: pointers are device memory on the context's device;
 *    the work is enqueued on the context's stream.  The evaluation calls
 *    (csbq_eval, csbq_eval_batch, csbq_smooth_sum, csbq_plan) read sizes the
 *    device computes (candidate-pair counts, correction runs, group ranges)
 *    back to the host, so they wait for the stream part-way through; they
 *    return once their last kernels are enqueued, and the outputs may be read
 *    only after csbq_synchronize (or a synchronisation of the stream).
 *    csbq_apply returns with its outputs in place.
 *  - the caller owns every array passed in or out; the library copies what
 *    it keeps.
 *  - all floating point arrays are IEEE double, C order, contiguous.
 *  - the library supports ns = 16 and nt = 32 exactly (CSBQ_EINVAL otherwise).
 */
#ifndef CSBQ_H
#define CSBQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csbq_ctx csbq_ctx;

typedef enum {
    CSBQ_OK = 0,
    CSBQ_EINVAL = -1,   /* bad argument (sizes, NaN, unsupported orders, ...) */
    CSBQ_ENOMEM = -2,   /* device or host allocation failed */
    CSBQ_EHIP = -3,     /* a HIP runtime call failed */
    CSBQ_ETABLE = -4,   /* quadrature tables missing or malformed */
    CSBQ_ESTATE = -5,   /* call out of order (e.g. eval before set_geometry) */
    CSBQ_ELIMIT = -6    /* an internal work limit was exceeded */
} csbq_status;

/* Bits of an evaluation's flag word (csbq_eval_flags, and "flags" in
   csbq_stats).  NODE_RANGE, GROUP_RANGE and GROUP_ORDER make the call fail
   with CSBQ_EINVAL and BAND makes csbq_apply fail with CSBQ_ESTATE; SRULE_LIMIT
   and THETA_CLAMP are accuracy warnings of a completed evaluation: some
   special quadrature may have missed quad_tol. */
typedef enum {
    CSBQ_FLAG_NODE_RANGE = 1,   /* a tgt_node >= the node count */
    CSBQ_FLAG_SRULE_LIMIT = 2,  /* an off-surface s-rule (Section 3.2.3) stopped bisecting at its depth or
                                   sub-panel limit with the target still inside a sub-panel's near region */
    CSBQ_FLAG_THETA_CLAMP = 4,  /* a circle closer (relative to its radius) than the finest tabulated
                                   theta-rule bracket (Section 3.2.2, Appendix B) used that bracket's rule */
    CSBQ_FLAG_GROUP_RANGE = 8,  /* a free target's group is outside 0..G-1 */
    CSBQ_FLAG_GROUP_ORDER = 16, /* targets not ordered by group */
    CSBQ_FLAG_BAND = 32         /* csbq_apply: the density's band exceeds the plan's */
} csbq_flag;

typedef enum { CSBQ_HOST = 0, CSBQ_DEVICE = 1 } csbq_mem;
typedef enum { CSBQ_FP64 = 0, CSBQ_MIXED = 1 } csbq_precision;
typedef enum { CSBQ_GATE_CRITERION = 0, CSBQ_GATE_MLP = 1 } csbq_gate_mode;
/* Kernel pair.  CSBQ_KERNEL_LAPLACE evaluates the Laplace single and double
   layers of Section 4.1 instead of the Stokes ones, on a scalar density:
     u_S(x) = int G(x - y) sigma(y) dS_y,  u_D(x) = int dG(x - y)/dn_y sigma(y) dS_y,
     G(r) = 1 / (4 pi |r|),  dG/dn_y = (r.n) / (4 pi |r|^3),  r = x - y,
   so that u_D of a constant 1 is -1 inside a closed surface, -1/2 on it and
   0 outside.  Every density array then holds one value per node ([N]) and
   every output one value per target ([n_tgt]) where the Stokes layers have
   three; everything else (geometry, targets, tables, corrections) is shared. */
typedef enum { CSBQ_KERNEL_STOKES = 0, CSBQ_KERNEL_LAPLACE = 1 } csbq_kernel;

/* s-rule of an on-surface target's own element (Section 3.2.4).
   GENERAL: Gauss-Legendre panels refined dyadically toward the target plus
   the log-singular rule (p log + q) on its two sides.  The whole-element
   singular rules (the section's second part) are one generalised Chebyshev
   rule over the whole element per target GL index, built offline per
   Appendix B (tables/srules.bin): per aspect bracket [2^b, 2^(b+1)), b =
   2..30, from straight cylinders of constant radius, with the aspect at the
   target A = 2 hw |x_c'(s0)| / eps(s0) (hw the panel's half-length in s);
   and one set for a sphere given as one element in its polar-angle
   parametrisation (x_c = c + a cos(pi t) axis, eps = a sin(pi t), t the
   panel's normalised parameter, constant e1).
   AUTO (default): the sphere rules on such spheres; the cylinder rules on
   open elements whose aspect has a bracket and that are close enough to the
   rules' family to keep their accuracy (constant speed |x_c'| to 1e-9, bend
   = largest curvature x element length <= 0.06, radius varying by <= 10 %,
   e1 turning by <= 0.25 rad over the element); the general rule elsewhere.
   WHOLE: the cylinder rules on every open element whose aspect has a
   bracket (the paper's use; more bent or unevenly parametrised elements lie
   outside the rules' family, so their accuracy is not quad_tol's). */
typedef enum { CSBQ_SRULE_AUTO = 0, CSBQ_SRULE_WHOLE = 1, CSBQ_SRULE_GENERAL = 2 } csbq_srule;

/* Far-field rules of the smooth sum (Section 3.2.1's smooth rule).  Each
   element has a base rule: its own N_s x N_theta nodes, or for an element
   closed at an end (a sphere as one element in its polar angle, where
   Gauss-Legendre rules in that angle converge slowly nearby) a 32 x 32 rule
   (the first upsampled rule); the local corrections subtract the base rule.
   AUTO (default): a smooth-sum block of targets sums each element with n
   Gauss points in s times m angles (a sphere: n in {24, 20, 16}; any other
   element: n in {16, 12, 8}; m in {32, 24, 16}), each the smallest whose
   distance from the element's centre, at which the criterion's estimates let
   it meet quad_tol for the density's measured band, all the block's targets
   lie beyond; else the base rule.  Every candidate pair lies inside those
   distances, so the corrections are unchanged.  BASE: the base rules for
   every target. */
typedef enum { CSBQ_FAR_AUTO = 0, CSBQ_FAR_BASE = 1 } csbq_far_rule;

typedef struct {
    double quad_tol;       /* per-element quadrature tolerance (relative); <= 0 selects 1e-12 */
    int32_t precision;     /* csbq_precision: FP64, or mixed (FP32 far field, FP64 near corrections) */
    int32_t gate;          /* csbq_gate_mode: the error-estimate criterion, or the learned gate */
    int32_t device;        /* HIP device ordinal */
    void* stream;          /* hipStream_t to enqueue on; NULL = a stream owned by the context */
    const char* table_dir; /* directory holding rules.bin (and srules.bin); NULL = the package's tables/ */
    int32_t kernel;        /* csbq_kernel: the Stokes layers, or the Laplace layers (FP64, criterion gate only) */
    int32_t srule;         /* csbq_srule: the own element's s-rule for on-surface targets */
    int32_t far_rule;      /* csbq_far_rule: coarser far-field rules far from each element, or the base rules */
} csbq_options;

/* Fill *opt with defaults (quad_tol 1e-12, FP64, criterion gate, device 0,
   own stream, packaged tables, Stokes layers, CSBQ_SRULE_AUTO, CSBQ_FAR_AUTO). */
void csbq_default_options(csbq_options* opt);

/* Create a context: selects the device, creates/adopts the stream and loads
   the quadrature tables (theta-rules of Section 3.2.2, the log rule of
   Section 3.2.4 and, unless CSBQ_SRULE_GENERAL, its whole-element singular
   rules; generated offline per Appendix B): rules.bin and srules.bin (built
   to 1e-13 and 1e-12), or with quad_tol >= 1e-8 rules_t8.bin and
   srules_t8.bin (built to 1e-8, fewer nodes) where the table directory holds
   them.  *out receives the handle; CSBQ_ETABLE if a table is missing or
   malformed. */
int csbq_create(const csbq_options* opt, csbq_ctx** out);

/* Release every resource of the context (the adopted stream is not destroyed). */
int csbq_destroy(csbq_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* csbq_last_error(const csbq_ctx* ctx);

/* Define the geometry (Section 3.1) and expand it on the device: nodes,
   normals, smooth weights w_ij = J_ij w_i^GL 2 pi / nt (Section 3.2.1), and
   the per-element data used by the near-field corrections.
     n_bodies            number of bodies (>= 1)
     n_panels[b]         panels of body b (>= 1)
     normal_sign[b]      +1 or -1
     s_break             sum_b (n_panels[b] + 1) increasing panel end points, body-major
     xc, e1              [sum n_panels][ns][3] centerline and orientation samples
     eps                 [sum n_panels][ns] radius samples (> 0)
     ns, nt              16 and 32
   Arrays are in `mem` (host or device).  Replaces any previous geometry. */
int csbq_set_geometry(csbq_ctx* ctx, int32_t n_bodies, const int32_t* n_panels, const int32_t* normal_sign,
                      const double* s_break, const double* xc, const double* eps, const double* e1, int32_t ns,
                      int32_t nt, int mem);

/* Several independent geometries in one context (a batch): body_group[b] in
   0..G-1 names the geometry of body b (non-decreasing, every group present,
   starting at 0; NULL = one geometry).  Bodies of different groups never
   interact: each group's potential is the same sum as if it were alone (Eq.
   e:nystrom-no-correction and its local corrections, per geometry).  Every
   evaluation then runs as one pass over the whole batch: one smooth-sum
   launch over all groups' blocks ordered by cost (sources x targets), one
   near-pair search, one classification and one correction launch per tier.
   Other arguments as csbq_set_geometry; body_group lives in `mem`. */
int csbq_set_geometry_batch(csbq_ctx* ctx, int32_t n_bodies, const int32_t* body_group, const int32_t* n_panels,
                            const int32_t* normal_sign, const double* s_break, const double* xc, const double* eps,
                            const double* e1, int32_t ns, int32_t nt, int mem);

/* Number of surface nodes of the current geometry. */
int csbq_num_nodes(const csbq_ctx* ctx, int64_t* n_nodes);

/* Copy out node positions [N][3], unit normals [N][3] and smooth weights [N]
   (any pointer may be NULL). */
int csbq_get_nodes(csbq_ctx* ctx, double* y, double* normal, double* weight, int mem);

/* The layer potentials at n_tgt targets (the full hot path: near-pair search,
   gate, corrections, smooth sum, reduction).
     sigma     [N][3] nodal density
     x         [n_tgt][3] target points (may be NULL if every tgt_node >= 0)
     tgt_node  [n_tgt] node id of an on-surface target, any negative value
               for a free target; NULL means every target is free.  For an
               on-surface target the node's own position is used and x is
               ignored.  A node id >= the node count fails with CSBQ_EINVAL
               (in device mode too: the id is checked on the device before
               the call's first synchronisation).
     u_sl/u_dl [n_tgt][3] outputs (either may be NULL).
   Free targets must not lie on a surface (distance below ~1e-12 of the
   element size is undefined). */
int csbq_eval(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
              double* u_sl, double* u_dl, int mem);

/* The smooth Nystrom sum alone (Section 3.2.1, rule without corrections),
   self term zero; same arguments as csbq_eval.  Runs in the context's
   precision mode. */
int csbq_smooth_sum(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
                    double* u_sl, double* u_dl, int mem);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   csbq_smooth_sum with the same arguments and results (within rounding: the
   sum is split into a fixed number of source chunks), all pointers in device
   memory, and no allocation.  Every buffer beyond the caller's inputs and
   outputs lives in one static device array of the library (about 58 MiB per
   GPU, loaded with the library's code object and held until the process
   ends), whose address csbq_create looks up once per device.  Limits: a
   single geometry (csbq_set_geometry, not a batch of groups), at most
   CSBQ_NOALLOC_MAX_TARGETS targets and CSBQ_NOALLOC_MAX_NODES surface nodes;
   beyond them the call fails with CSBQ_ELIMIT.  The call only enqueues work
   on the context's stream (no host wait, no memset); a tgt_node beyond the
   node count sets CSBQ_FLAG_NODE_RANGE, read with csbq_eval_flags, and makes
   that target's outputs meaningless.  Calls on one GPU share the array,
   whose contents persist between calls: calls that overlap in time on one
   GPU (other streams, other threads or contexts) race and must be ordered by
   the caller. */
#define CSBQ_NOALLOC_MAX_TARGETS 262144
#define CSBQ_NOALLOC_MAX_NODES 262144
int csbq_smooth_sum_noalloc(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x,
                            const int64_t* tgt_node, double* u_sl, double* u_dl);

/* csbq_eval over a batch (csbq_set_geometry_batch): tgt_group[n_tgt] names
   the geometry of every free target (ignored for on-surface targets, whose
   node fixes it; NULL = group 0 for free targets).  Targets must be ordered by
   group (non-decreasing); an unordered list or a group out of range fails with
   CSBQ_EINVAL.  tgt_group lives in `mem`. */
int csbq_eval_batch(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
                    const int32_t* tgt_group, double* u_sl, double* u_dl, int mem);

/* ---- Setup / apply split (the paper's precomputed corrections, Section
   3.2.1 and Section 3.3, in density form).  csbq_plan evaluates like
   csbq_eval_batch and freezes what depends on the geometry and targets only:
   the candidate pairs, their tiers and special-quadrature rules, the
   smooth-sum blocks; the per-density part (density coefficients, smooth sum,
   corrections, reduction) is captured as a HIP graph.  csbq_apply replays it
   for a new density on the same geometry and targets, without a search,
   classification or host round trip inside, and returns once the outputs are
   in place.  Rules were chosen for the planning density's band limits: a
   density with a wider band (more Fourier or Legendre modes above the
   tolerance on some element) makes csbq_apply fail with CSBQ_ESTATE (plan
   again).  Any other evaluation call, set_geometry or destroy drops the plan.
   Arrays as in csbq_eval_batch; sigma, u_sl and u_dl of csbq_apply live in
   `mem`. */
int csbq_plan(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
              const int32_t* tgt_group, double* u_sl, double* u_dl, int mem);

/* csbq_plan with options (flags, a bitwise or):
   CSBQ_PLAN_FULL_BAND  tiers and rules for the widest band any density can
                        have (every Legendre degree and Fourier mode), so that
                        csbq_apply never refuses a density (the correction
                        pairs then do not depend on the planning density, as
                        the paper's E does not);
   CSBQ_PLAN_MATRIX     the paper's setup/evaluation split for the special
                        quadrature (Section 3.2.1, the sparse correction
                        matrix of Eq. e:nystrom-correction; Section 3.4 costs):
                        for every special-quadrature pair the 3 x 3 single- and
                        double-layer blocks (12 symmetric components) against
                        the element's density coefficients (16 GL rows x 32
                        trigonometric basis functions), 48 KB per pair,
                        built once; every csbq_apply then forms those
                        corrections by one bandwidth-bound pass over the
                        matrices instead of the special quadrature.  The
                        upsampled-rule tiers stay in density form.  Stokes
                        layers only (CSBQ_EINVAL otherwise); more than 160 GB
                        of matrices fails with CSBQ_ELIMIT. */
#define CSBQ_PLAN_MATRIX 1
#define CSBQ_PLAN_FULL_BAND 2
int csbq_plan_ex(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
                 const int32_t* tgt_group, int32_t flags, double* u_sl, double* u_dl, int mem);
int csbq_apply(csbq_ctx* ctx, const double* sigma, double* u_sl, double* u_dl, int mem);

/* ---- Boundary-integral solves (Section 4).  Both run on a single
   geometry (csbq_set_geometry), with the density at every surface node.
   Each freezes one evaluation plan over all surface nodes as on-surface
   targets, with tiers and rules chosen for the widest band a density can
   have (every Legendre degree and Fourier mode), and solves by restarted
   GMRES (classical Gram-Schmidt applied twice, fixed-order reductions: a
   solve is bitwise repeatable); every operator application replays the plan
   (csbq_apply).  The plan stays valid afterwards for csbq_apply.

   Double-layer orientation: the integral equations of Section 4 use the
   double layer D_4 = -D, D the potential u_dl of csbq_eval (whose stresslet
   gives c, c/2, 0 inside, on and outside a closed surface for a constant
   density c); with D_4 the rigid motions lie in the null space of I/2 + D_4
   (Proposition on the null space, Section 4.2).  The combined-field operator
   is K = I/2 + D_4 + eta S (Section 4.1; the slender choice of the weight is
   eta = 1 / (2 eps log(1/eps)), eps the cross-section radius). */
typedef struct {
    double eta;        /* weight of the single layer in K (> 0) */
    double tol;        /* GMRES stops at ||b - A sigma|| <= tol ||b|| (the Arnoldi estimate) */
    int32_t max_iter;  /* operator applications of the Krylov iterations, at most */
    int32_t restart;   /* Krylov basis size before a restart */
} csbq_solve_options;

typedef struct {
    int32_t iterations;   /* Krylov iterations taken */
    double rel_residual;  /* ||b - A sigma|| / ||b||, recomputed with one more application */
} csbq_solve_info;

/* eta 1, tol 1e-10, max_iter 200, restart 60 */
void csbq_default_solve_options(csbq_solve_options* opt);

/* Exterior Stokes Dirichlet problem, slender combined-field form (Section
   4.1): solves K sigma = u0 at the surface nodes.  The exterior velocity is
   then u = D_4[sigma] + eta S[sigma] = eta u_sl - u_dl of csbq_eval.  With
   the Laplace layers (CSBQ_KERNEL_LAPLACE) it is the Laplace problem of
   Section 4.1, K = I/2 + D + eta S with the evaluator's D itself (whose
   orientation is the one that equation uses), u0 and sigma of one value per
   node, and u = u_dl + eta u_sl off the surface.
     u0     [N][3] boundary velocity at the nodes (in `mem`)
     sigma  [N][3] solution (in `mem`)
     info   iterations and residual (host; may be NULL). */
int csbq_solve_dirichlet(csbq_ctx* ctx, const csbq_solve_options* opt, const double* u0, double* sigma,
                         csbq_solve_info* info, int mem);

/* Stokes mobility problem, slender mobility combined-field form (Section
   4.2): rigid bodies with given net force and torque and a slip velocity.
   Per body b the completion density nu = a_b + beta_b x (y - c_b) (c_b the
   surface centroid under the smooth weights) has sum w nu = F_b and
   sum w (y - c_b) x nu = T_b (the torque about c_b; the printed equation
   writes the cross product in the other order, which would flip the
   torque's sign).  L is the orthogonal projector onto the rigid motions of
   each body in the smooth-weight inner product.  Solves
   (K (I - L) + L) sigma = u_slip - S nu; the rigid motion is -L sigma.
     force, torque [n_bodies][3] (host)
     u_slip  [N][3] slip velocity (in `mem`; NULL = none)
     sigma   [N][3] out: the density (I - L) sigma of the representation
             u = (D_4 + eta S)[(I - L) sigma] + S[nu] = eta u_sl - u_dl of
             csbq_eval on this density, plus u_sl of csbq_eval on nu (in `mem`;
             may be NULL)
     nu      [N][3] out: the completion density (in `mem`; may be NULL)
     rigid   [n_bodies][6] out: translational velocity V_b and angular
             velocity Omega_b about c_b (host; may be NULL)
     centers [n_bodies][3] out: c_b (host; may be NULL)
   A body whose rigid-motion Gram matrix is singular fails with CSBQ_EINVAL. */
int csbq_solve_mobility(csbq_ctx* ctx, const csbq_solve_options* opt, const double* force, const double* torque,
                        const double* u_slip, double* sigma, double* nu, double* rigid, double* centers,
                        csbq_solve_info* info, int mem);

/* ---- Learned correction-tier gate (an extension beyond the paper; the
   criterion of Section 3.2's error estimates stays the fallback and decides
   every pair the network is unsure of).  A perceptron with three hidden layers of 64 ReLU units maps
   CSBQ_GATE_NF features of a (target, element) pair to CSBQ_GATE_NO ordinal
   outputs, output k estimating P(tier > k) for the tiers skip / three
   upsampled whole-panel rules / special quadrature.  With gate = MLP the
   evaluation takes the network's tier for the pairs it is confident about
   and sends the rest (P(tier above the prediction) > tau_esc, predicted
   special quadrature, own-element targets) to the criterion.  Inference runs
   on bf16 MFMA with FP32 accumulation; training is FP32.
   Weights: CSBQ_GATE_NW floats, W1[16][64] b1[64] W2[64][64] b2[64]
   W3[64][64] b3[64] W4[64][4] b4[4] (row-major, input index first). */
#define CSBQ_GATE_NF 16
#define CSBQ_GATE_NO 4
#define CSBQ_GATE_NW 9668

/* Install inference weights (host array) and the escalation threshold
   tau_esc in (0, 1). */
int csbq_gate_load(csbq_ctx* ctx, const float* weights, float tau_esc);

/* Run the installed network on n feature rows (host [n][16]); outputs (host,
   any may be NULL): tier [n] (0..4), esc [n] (1 = decided by the criterion),
   logits [n][4]. */
int csbq_gate_infer(csbq_ctx* ctx, const float* feat, int64_t n, int8_t* tier, uint8_t* esc, float* logits);

/* Mean loss and gradient (host [CSBQ_GATE_NW]) of the weighted ordinal
   cross-entropy  sum_k -(posw[k] y_k log s_k + (1 - y_k) log(1 - s_k)),
   y_k = [label > k], over n samples, at the given weights (host arrays). */
int csbq_gate_grad(csbq_ctx* ctx, const float* weights, const float* feat, const int8_t* label, int64_t n,
                   const float* posw, float* grad, float* loss);

/* Adam training (minibatches of `batch`, `epochs` passes, samples shuffled
   with `seed`): weights (host) hold the initial values on entry and the
   trained values on return; loss_out [epochs] (may be NULL) the mean loss of
   every pass. */
int csbq_gate_train(csbq_ctx* ctx, const float* feat, const int8_t* label, int64_t n, const float* posw, int epochs,
                    int batch, float lr, uint64_t seed, float* weights, float* loss_out);

/* Training data from one evaluation (criterion gate, host arrays): the
   features of every candidate pair and its label, the cheapest tier whose
   correction agrees with the special quadrature's to label_tol times the
   largest |u| of that kernel over the targets (4 if none does); crit (may be
   NULL) receives the criterion's tier.  At most cap pairs are returned (an
   even stride through the pair list); *n_out receives the count. */
int csbq_gate_dataset(csbq_ctx* ctx, const double* sigma, int64_t n_tgt, const double* x, const int64_t* tgt_node,
                      double label_tol, int64_t cap, float* feat, int8_t* label, int8_t* crit, int64_t* n_out);

/* Statistics of the last csbq_eval as a JSON object (phase times in ms from
   HIP events, pair counts per correction tier, s- and theta-node counts, the
   rule tables in use).  Blocks until the context's stream has drained.
   Writes at most cap bytes including the terminating zero. */
int csbq_stats(const csbq_ctx* ctx, char* buf, int64_t cap);

/* Block until the context's stream has drained. */
int csbq_synchronize(csbq_ctx* ctx);

/* Flag word (csbq_flag bits) of the last evaluation call.  After a
   device-mode call this waits for the context's stream, since the special
   quadrature sets its warnings on the device; call it before the next
   evaluation on the context. */
int csbq_eval_flags(csbq_ctx* ctx, int32_t* flags);

#ifdef __cplusplus
}
#endif
#endif /* CSBQ_H */
