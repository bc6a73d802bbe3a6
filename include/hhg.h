/*
 * hhg.h -- C ABI of the MI355X (gfx950) library for matrix-free stencil
 * scaling on hierarchical hybrid grids.
 *
 * Method: Drzisga, Ruede, Wohlmuth, "Stencil scaling for vector-valued PDEs on
 * hybrid grids with applications to generalized Newtonian fluids".  A macro
 * tetrahedral mesh is refined uniformly; inside every macro-tet the operator
 * of the vector-valued P1 form
 *
 *     a(u, v) = (2 mu(x) eps(u), eps(v)) + (lam(x) div u, div v)          (Sec. 2,
 *                                                   eq. bilinearformstd)
 *
 * with mu = mu0 + mu1 k, lam = lam0 + lam1 k for ONE nodal scalar field k is
 * applied by scaling constant reference stencils with nodal coefficient
 * averages plus the antisymmetric correction of the Lemma (eqs.
 * bilinearformscaling, patchmean, corrtermgeneral; 3-D form of Sec. 2.4),
 * instead of integrating the form element by element.
 *
 * Data layout (all vectors live in device memory, owned by the caller):
 *   * Nodes are stored per macro: macro m occupies slots
 *     [macro_offset[m], macro_offset[m+1]).  Inside a macro of level L
 *     (n = 2^L intervals per edge) node (i, j, k), i,j,k >= 0, i+j+k <= n, at
 *         x0 + (i/n)(x1-x0) + (j/n)(x2-x0) + (k/n)(x3-x0)
 *     sits at local slot  P(k) + (i+j)(i+j+1)/2 + i,  P(k) = nodes in planes
 *     below k.  Nodes on faces, edges and vertices shared by several macros
 *     appear once per macro ("copies"); a vector is CONSISTENT when all copies
 *     of a node hold the same value.  Every output of this library is
 *     consistent; inputs must be consistent.
 *   * A vector field is SoA [3][n_nodes] (component c of slot s at
 *     c*n_nodes + s); the coefficient k is [n_nodes].  Element type double
 *     (HHG_F64) or float (HHG_F32) as selected by `prec`.  Pointers must be
 *     16-byte aligned.
 *   * Homogeneous Dirichlet nodes (outer boundary of the macro mesh, Sec. 2):
 *     their entries of x are ignored (treated as 0) and their entries of every
 *     operator output are written as 0.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 * Apply/residual calls are asynchronous on that stream; solver calls
 * synchronize it before returning.
 *
 * Errors: every call returns HHG_OK (0) or a negative code; the text of the
 * last error of the calling thread is returned by hhg_last_error().  No C++
 * exception crosses this interface.  A handle must not be used by two host
 * threads at once.
 */
#ifndef HHG_H
#define HHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhg_ctx *hhg_handle;

enum hhg_status {
  HHG_OK = 0,
  HHG_EINVAL = -1,      /* bad argument: null/misaligned pointer, level out of
                           range, degenerate macro, unknown enum value        */
  HHG_EHIP = -2,        /* HIP runtime error (text in hhg_last_error)         */
  HHG_ENOCONV = -3,     /* solver reached maxit; x and info are still written */
  HHG_EBREAKDOWN = -4,  /* solver breakdown: NaN/Inf or p^T A p <= 0          */
  HHG_ENOMEM = -5       /* device or host allocation failed                   */
};

enum hhg_prec { HHG_F64 = 0, HHG_F32 = 1 };
enum hhg_coupling { HHG_CONFORMING = 0, HHG_INDEPENDENT = 1 };
enum hhg_dirichlet { HHG_DIRICHLET_OUTER = 0, HHG_DIRICHLET_NONE = 1 };
enum hhg_corr { HHG_CORR_PHYSICAL = 0, HHG_CORR_NONE = 1 };
enum hhg_khat { HHG_KHAT_PATCH = 0, HHG_KHAT_EDGE = 1 };
enum hhg_iface { HHG_IFACE_SYMMETRIC = 0, HHG_IFACE_ROWWISE = 1, HHG_IFACE_ZEROSUM = 2 };
enum hhg_method { HHG_METHOD_SCALED = 0, HHG_METHOD_ONTHEFLY = 1 };

/* Macro mesh (Sec. 2: macro triangulation T_H refined uniformly).
 *   verts     host, [n_macro][4][3] vertex coordinates; the vertex order fixes
 *             each macro's index space (see the layout above).
 *   level     host, [n_macro]; 2 <= level <= 8 (a macro needs an interior
 *             vertex, Sec. 2).  CONFORMING meshes need one common level.
 *   coupling  HHG_CONFORMING: macros sharing faces/edges/vertices (matched by
 *             coordinates) form one problem; HHG_INDEPENDENT: every macro is
 *             its own problem (batched use).
 *   dirichlet HHG_DIRICHLET_OUTER: homogeneous Dirichlet on every macro face
 *             owned by a single macro (and on its edges and vertices);
 *             HHG_DIRICHLET_NONE: pure Neumann operator.                     */
typedef struct {
  int32_t n_macro;
  const double *verts;
  const int32_t *level;
  int32_t coupling;
  int32_t dirichlet;
} hhg_mesh_desc;

/* Operator: 2 (mu0 + mu1 k) (eps, eps) + (lam0 + lam1 k) (div, div).
 *   corr   HHG_CORR_PHYSICAL: physical scaling (Lemma); HHG_CORR_NONE:
 *          unphysical scaling, R omitted (eq. stencilscalingwithoutcorr).
 *   khat   HHG_KHAT_PATCH: patch mean of the element means (eq. patchmean);
 *          HHG_KHAT_EDGE: (k_i + k_j)/2 (Remark after the Lemma).
 *   iface  rows of nodes on a macro boundary (Sec. 2.2):
 *          HHG_IFACE_SYMMETRIC: nodal-integration entries where both nodes lie
 *          on the macro boundary (and on the diagonal), scaled entries
 *          towards macro-interior nodes -- a symmetric matrix;
 *          HHG_IFACE_ROWWISE: the full nodal-integration row;
 *          HHG_IFACE_ZEROSUM (not in the paper): the entries of the symmetric
 *          rule off the diagonal and a centre block of minus the sum of the
 *          row's other blocks, as on macro-interior rows; still symmetric,
 *          and translations stay in the kernel of the interface rows.
 *          The on-the-fly method always uses the nodal row.                   */
typedef struct {
  double mu0, lam0;
  double mu1, lam1;
  int32_t corr;
  int32_t khat;
  int32_t iface;
} hhg_op_desc;

/* Host-side setup (Sec. 2.4: reference stencil and correction stencils are
 * precomputed once per macro).  Builds the per-macro constant tables in FP64
 * (and their FP32 copies), the interface-copy groups and the Dirichlet masks.
 * No device memory is touched here: the tables (a few KB per macro) are
 * uploaded to the current HIP device by the first device call, and the handle
 * may then only be used on that device.  On success *out owns host and device
 * memory until hhg_destroy.  Errors: HHG_EINVAL for null pointers,
 * n_macro < 1, a level outside 2..8, mixed levels in a conforming mesh, a
 * degenerate macro (|det| < 1e-12 |edges|^3) or unknown enum values;
 * HHG_EHIP / HHG_ENOMEM on device failures.                                  */
int hhg_setup_macro(const hhg_mesh_desc *mesh, const hhg_op_desc *op, hhg_handle *out);

/* Frees the handle's device and host memory.  NULL is accepted.            */
int hhg_destroy(hhg_handle h);

/* Sizes: *n_nodes total slots (copies included), *n_unknown number of
 * distinct non-Dirichlet nodes (3 unknowns each); macro_offset, if not NULL,
 * receives n_macro+1 slot offsets (host memory).                            */
int hhg_layout(hhg_handle h, int64_t *n_nodes, int64_t *n_unknown, int64_t *macro_offset);

/* Host output [3][n_nodes] of slot coordinates (caller-allocated).         */
int hhg_node_coords(hhg_handle h, double *xyz);

/* Host output [n_nodes] bit flags per slot: bit0 Dirichlet, bit1 owner copy
 * (exactly one copy of every distinct node), bit2 on a macro boundary, bit3
 * non-Dirichlet node with copies in other macros.                          */
int hhg_node_flags(hhg_handle h, uint8_t *flags);

/* y = A_s(k) x: physical (or unphysical) stencil scaling in macro interiors
 * (Lemma, Sec. 2.4) and the chosen interface rule on macro boundaries
 * (Sec. 2.2).  x [3][n], k [n], y [3][n] device pointers of type `prec`; x
 * and y must not overlap.  Asynchronous on `stream`.                        */
int hhg_apply_scaled(hhg_handle h, int32_t prec, const void *x, const void *k, void *y,
                     void *stream);

/* y = A_n(k) x: nodal integration computed element by element on the fly
 * (eq. nodalintegration with the vertex mean of eq. nodalquad) -- the
 * comparison method of Sec. 4 and Sec. 5.  Same arguments as above.        */
int hhg_apply_onthefly(hhg_handle h, int32_t prec, const void *x, const void *k, void *y,
                       void *stream);

/* r = f - A x with A = A_s (method HHG_METHOD_SCALED) or A_n
 * (HHG_METHOD_ONTHEFLY); the residual of Sec. 4 (eq. residuallinalg).
 * Dirichlet entries of r are 0.  r must not overlap x or f.                 */
int hhg_residual(hhg_handle h, int32_t prec, int32_t method, const void *f, const void *x,
                 const void *k, void *r, void *stream);

/* Solvers for A x = b on the unknowns (distinct non-Dirichlet nodes); the
 * paper solves these systems by multigrid (Sec. 5), this library provides
 * Krylov solvers over the same operators:
 *   HHG_CG_F64  preconditioned CG, all vectors, dots and applies in FP64.
 *   HHG_IR_F32  iterative refinement: the residual b - A x, its norm and the
 *               update x += e in FP64; the correction e from an inner
 *               preconditioned CG with FP32 vectors, FP32 coefficient and
 *               FP32 applies, inner dot products accumulated in FP64, run to
 *               inner_rtol relative reduction.
 *   HHG_FCG_F64 flexible CG in FP64: as HHG_CG_F64 with the Polak-Ribiere
 *               beta = (z+, r+ - r) / (z, r), computed from the (z, A p)
 *               product fused into the update; for a fixed symmetric positive
 *               definite preconditioner the iterates are those of CG.
 * Preconditioner: HHG_PRECOND_NONE, HHG_PRECOND_BLOCK_JACOBI (inverse of
 * the 3x3 diagonal block of the assembled operator at every node), or
 * HHG_PRECOND_LEARNED: P = (I + M)^T D^{-1} (I + M) with D that diagonal block
 * and M the output of the network attached by hhg_set_learned_model, fed the
 * node's coefficient neighbourhood and averaged over the node's copies
 * (computed once per solve; see the learned smoother section below).
 * Stopping rule: ||b - A x||_2 <= rtol ||b||_2 over the unknowns, with the
 * final residual recomputed in FP64 (reported in info->rel_residual). */
enum hhg_solver { HHG_CG_F64 = 0, HHG_IR_F32 = 1, HHG_FCG_F64 = 2 };
enum hhg_precond { HHG_PRECOND_NONE = 0, HHG_PRECOND_BLOCK_JACOBI = 1, HHG_PRECOND_LEARNED = 2 };

typedef struct {
  int32_t solver;        /* hhg_solver                                        */
  int32_t precond;       /* hhg_precond                                       */
  int32_t method;        /* HHG_METHOD_SCALED or HHG_METHOD_ONTHEFLY operator */
  int32_t maxit;         /* total CG iterations allowed (inner ones for IR)   */
  double rtol;           /* relative residual target, e.g. 1e-8               */
  double inner_rtol;     /* IR: relative reduction per inner solve, e.g. 1e-3 */
  int32_t check_every;   /* iterations between host convergence checks (>= 1) */
  int32_t pad;
} hhg_solve_opts;

typedef struct {
  int32_t iterations;        /* CG iterations until the recursive residual met
                                the tolerance (summed over the inner solves
                                for IR; all run if it never did)              */
  int32_t outer_iterations;  /* IR refinement steps (1 for CG_F64)            */
  int32_t status;            /* HHG_OK, HHG_ENOCONV or HHG_EBREAKDOWN         */
  int32_t iterations_run;    /* CG iterations executed: whole blocks of
                                check_every, so up to check_every - 1 more    */
  double rel_residual;       /* ||b - A x|| / ||b|| recomputed in FP64        */
  double seconds;            /* wall time of the solve                        */
} hhg_solve_info;

/* The preconditioner blocks a solve would use (symmetric 3x3 per slot,
 * P device FP64 [6][n_nodes] in the order xx yy zz xy xz yz; identity for
 * HHG_PRECOND_NONE, zero at Dirichlet slots), for operator `method` and
 * coefficient k.  Learned blocks need an attached model; they use a scratch
 * block of 68 n_nodes bytes that this call allocates and frees.
 * Synchronizes `stream`.  Errors: HHG_EINVAL, HHG_EHIP.                    */
int hhg_preconditioner(hhg_handle h, int32_t precond, int32_t method, const double *k, double *P,
                       void *stream);

/* The same blocks without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, results and errors as
 * hhg_preconditioner.  The learned blocks use a static scratch array of
 * 64 MiB on each device (held until the process ends; 68 bytes per slot,
 * so at most 986,895 slots: larger meshes get HHG_EINVAL).  The handle must
 * have made a device call already (its first one uploads its tables);
 * otherwise HHG_EINVAL.  Calls that overlap on one device share the scratch
 * and race: serialize them.  Synchronizes `stream`.                        */
int hhg_preconditioner_noalloc(hhg_handle h, int32_t precond, int32_t method, const double *k,
                               double *P, void *stream);

/* Device workspace needed by hhg_cg_solve for these options (bytes).      */
int hhg_workspace_bytes(hhg_handle h, const hhg_solve_opts *o, size_t *bytes);

/* Solve A x = b.  b, k, x: FP64 device vectors ([3][n], [n], [3][n]); x is
 * the start vector on input and the solution on output; b must be consistent
 * (its Dirichlet entries are ignored).  workspace: device memory of
 * hhg_workspace_bytes, 256-byte aligned, owned by the caller.  Runs on
 * `stream` and synchronizes it before returning.  Returns HHG_OK,
 * HHG_ENOCONV (maxit reached; x and info written), HHG_EBREAKDOWN (NaN/Inf
 * or p^T A p <= 0: indefinite operator or corrupt input), HHG_EINVAL. */
int hhg_cg_solve(hhg_handle h, const hhg_solve_opts *o, const double *b, const double *k,
                 double *x, void *workspace, hhg_solve_info *info, void *stream);

/* Generalized-Newtonian viscosity at the nodes from a velocity field
 * (Sec. 3: the strain rate |D(u)|^2 is evaluated from a local least-squares
 * fit of u; Carreau law eq. carreau of Sec. 5.2.2):
 *     mu_i = eta_inf + (eta0 - eta_inf) (1 + kappa |eps(u)_i|^2)^r,
 * |eps|^2 = eps : eps.  Macro-interior nodes: gradient of the affine
 * least-squares fit over the 15-node patch (exact for quadratic u there).
 * Nodes on macro boundaries (faces, edges, vertices), law->boundary =
 * HHG_STRAIN_LSQ: least squares over the node's patch in the whole mesh (the
 * node and all nodes sharing an element with it, in any macro) onto
 * quadratics (eq. minimization_problem, m = 2), the gradient taken at the
 * node; where the patch leaves that gradient undetermined (on the domain
 * boundary, a one-sided patch) the affine fit over the same patch.  Exact
 * for quadratic u at every node off the domain boundary.  The fit weights
 * are built on the host at the handle's first call (patches of equal shape
 * share them).  HHG_STRAIN_AVERAGE: volume-weighted mean of the gradients of
 * all elements at the node (the averaging Sec. 3 names as the alternative).
 * u: FP64 [3][n] consistent device vector, every node (Dirichlet ones
 * included) used as given; k: FP64 [n] device output, consistent.
 * workspace: hhg_viscosity_workspace_bytes bytes of device memory.  Errors:
 * HHG_EINVAL for null/misaligned pointers, parameters outside
 * eta0 >= eta_inf > 0, kappa >= 0, or an unknown boundary fit.
 * Asynchronous.                                                              */
enum hhg_strain_fit { HHG_STRAIN_LSQ = 0, HHG_STRAIN_AVERAGE = 1 };
typedef struct {
  double eta0, eta_inf, kappa, r;
  int32_t boundary;          /* hhg_strain_fit on macro-boundary nodes       */
  int32_t pad;
} hhg_carreau;

int hhg_viscosity_workspace_bytes(hhg_handle h, size_t *bytes);
int hhg_nodal_viscosity(hhg_handle h, const double *u, const hhg_carreau *law, double *k,
                        void *workspace, void *stream);

/* ---------------------------------------------------------------- batching
 * Many macros, or many independent problems of uneven level (coupling
 * HHG_INDEPENDENT), share one interior launch: the work list holds slabs of
 * 256 in-plane positions over a run of planes of one macro, ordered so that
 * item q runs on XCD q % 8.  (Not in the paper; its macro-interior sweep,
 * Sec. 4, is the unit of work here.)
 *
 * hhg_autotune: times the interior kernel of `method` in precision `prec` on
 * the caller's x and k (device, as for hhg_apply_scaled), `reps` launches per
 * candidate after one warm-up: per level, over balanced segments (-1: every
 * chunk's run of planes cut into segments of equal cost, about one per
 * resident workgroup) and slab depths 1, 2, 4, ... planes per item on that
 * level's macros alone; then over the whole list, over grids
 * of one workgroup per item or a persistent grid of 1..4 x (compute units)
 * resident workgroups striding the list.  The fastest choices are kept in
 * the handle for every later apply, residual and solve; results do not
 * depend on them (every row is computed by one thread the same way).  y is
 * scratch during tuning and holds A x on return.  Synchronizes `stream`.
 * Graphs from hhg_graph_create are dropped (their ids become invalid).
 * Errors: as hhg_apply_scaled, HHG_EINVAL for reps outside 1..1000 or a null
 * report, HHG_EHIP for a runtime failure (the previous configuration stays). */
typedef struct {
  int32_t n_levels;          /* distinct levels, ascending in level[]        */
  int32_t persist_blocks;    /* chosen grid: 0 = one workgroup per item      */
  int32_t level[8];
  int32_t slab[8];           /* chosen planes per work item (-1: balanced)   */
  int32_t macros[8];         /* macros of the level                          */
  int64_t rows[8];           /* macro-interior rows of the level             */
  double ms[8];              /* interior launch over the level's macros alone */
  double ms_total;           /* interior launch over all macros, chosen grid */
  int32_t candidates;        /* configurations timed                         */
  int32_t pad;
} hhg_tune_report;

int hhg_autotune(hhg_handle h, int32_t prec, int32_t method, const void *x, const void *k, void *y,
                 int32_t reps, hhg_tune_report *report, void *stream);

/* hhg_set_tuning: adopts a tuning record (as filled by hhg_autotune, or
 * written by the caller) without timing anything: slab[q] planes per work
 * item for macros of level[q] (-1: balanced segments; q < n_levels; 0 or an
 * absent level keeps the default depth: 5 planes from level 7 up, 3 below),
 * and the grid (persist_blocks 0: one workgroup per work
 * item; else a multiple of 8 up to 65536 resident workgroups striding the
 * list).  Other fields are ignored.  Waits for all queued device work, then
 * replaces the handle's work list; graphs from hhg_graph_create are dropped.
 * Results do not depend on the record.  Errors: HHG_EINVAL for a null record,
 * levels outside 2..8, slabs outside -1..1024 or an invalid grid; HHG_EHIP. */
int hhg_set_tuning(hhg_handle h, const hhg_tune_report *tuning);

/* hhg_graph_create: runs one checked apply y = A x (prec, method as in
 * hhg_residual) after all queued device work, then captures `count`
 * (1..1024) applies on the same device pointers into a HIP graph owned by
 * the handle and returns its id.  hhg_graph_launch replays it on `stream`
 * (asynchronous; the pointers must stay valid).  hhg_graph_destroy frees it;
 * hhg_destroy and hhg_autotune free all.  Errors: HHG_EINVAL for bad
 * arguments or an unknown id, HHG_EHIP for a capture or launch failure.     */
int hhg_graph_create(hhg_handle h, int32_t prec, int32_t method, const void *x, const void *k,
                     void *y, int32_t count, int32_t *graph_id);
int hhg_graph_launch(hhg_handle h, int32_t graph_id, void *stream);
int hhg_graph_destroy(hhg_handle h, int32_t graph_id);

/* ------------------------------------------------------ learned smoother
 * (Not in the paper, which smooths with Gauss-Seidel inside multigrid.)  A
 * small network maps the coefficient neighbourhood of a node to a 3x3 block
 * M; the preconditioner block is P = (I + M)^T D^{-1} (I + M), so M = 0 is
 * block Jacobi (the fallback) and P stays symmetric positive definite.
 *
 * Features of a node copy (16, BF16): the coefficient on the node's 15-point
 * patch (the node, then its neighbours in the order me mw mse mnw tc bc ts
 * bn mn ms tw be tse bnw of the stencil figure, Sec. 2.4), 0 for a
 * Dirichlet neighbour, the node's own value for a point outside the macro,
 * divided by the mean of the 15 values (summed left to right in that order,
 * then divided by 15); then level / 8.  Values are formed
 * in FP64, rounded to FP32 and then to BF16, both to nearest even.
 *
 * Network: h = relu(W1^T f + b1) with 64 units, h rounded to BF16, and
 * o = W2^T h + b2 (9 outputs, M row-major), BF16 weights W1 [16][64] and
 * W2 [64][9], FP32 biases, products on the matrix cores with FP32
 * accumulation.  Parameters as one FP32 vector of HHG_MLP_NPARAM entries:
 * W1 (row-major [16][64]), b1 [64], W2 (row-major [64][9]), b2 [9]; the
 * handle keeps FP32 master weights, their BF16 copies and Adam moments.
 *
 * Training record (HHG_SAMPLE_BYTES bytes, device): 16 BF16 features, then
 * 12 FP32 values r'0..2, e'0..2, S xx yy zz xy xz yz, then padding, where
 * for a node with residual r, error e and diagonal block D of a solver
 * iterate t = trace(D)/3, S = t D^{-1}, s = sqrt(|D^{-1} r|^2 + |e|^2),
 * r' = r / (t s), e' = e / s.  Loss of a record: |(I + M)^T S (I + M) r' -
 * e'|^2, the error left by one smoothing step z = P r relative to the sizes
 * of the error and of the block-Jacobi step; a batch's loss is the mean.  Gradients pass the BF16 roundings straight through.        */
enum {
  HHG_MLP_IN = 16,
  HHG_MLP_HIDDEN = 64,
  HHG_MLP_OUT = 9,
  HHG_MLP_NPARAM = 16 * 64 + 64 + 64 * 9 + 9,
  HHG_SAMPLE_BYTES = 128
};
typedef struct hhg_mlp_ctx *hhg_mlp;

/* Create a model with all parameters zero (block Jacobi) on the current
 * device / destroy it.  Errors: HHG_EINVAL (null), HHG_EHIP.               */
int hhg_mlp_create(hhg_mlp *out);
int hhg_mlp_destroy(hhg_mlp m);
/* Host FP32 parameter vector in / out (HHG_MLP_NPARAM entries); set also
 * resets the Adam moments and step count.  Synchronous.                    */
int hhg_mlp_set_weights(hhg_mlp m, const float *w);
int hhg_mlp_get_weights(hhg_mlp m, float *w);

/* Features of every slot: feat, device, [n_nodes][16] BF16 bit patterns
 * (uint16), from the FP64 coefficient k [n_nodes].  Asynchronous.          */
int hhg_learn_features(hhg_handle h, const double *k, uint16_t *feat, void *stream);

/* Network outputs of n feature records (device; record q starts at
 * feat + q * stride, stride >= 16 and a multiple of 4 uint16 entries, so
 * training records use stride HHG_SAMPLE_BYTES / 2): out, device,
 * [n][9] FP32.  Asynchronous.                                              */
int hhg_mlp_forward(hhg_mlp m, const uint16_t *feat, int64_t stride, int64_t n, float *out,
                    void *stream);

/* Training records of n nodes: for slots[q] (device int64, slots of
 * distinct non-Dirichlet nodes), its features and the record values above
 * from r and e (device FP64 [3][n_nodes]) and the operator's diagonal block
 * for `method` and coefficient k.  samples: device, n * HHG_SAMPLE_BYTES.
 * Allocates and frees a scratch block of 48 n_nodes bytes; synchronizes
 * `stream`.  Errors: HHG_EINVAL (null, n < 1, misaligned), HHG_EHIP.       */
int hhg_learn_collect(hhg_handle h, int32_t method, const double *k, const double *r,
                      const double *e, const int64_t *slots, int64_t n, void *samples,
                      void *stream);

/* Mean loss of n records and its gradient at the current weights (host
 * outputs: *loss, grad [HHG_MLP_NPARAM]).  Synchronizes `stream`.          */
int hhg_mlp_loss_grad(hhg_mlp m, const void *samples, int64_t n, double *loss, float *grad,
                      void *stream);

/* Adam training on the device: `epochs` passes over the n records in
 * consecutive mini-batches of `batch` (the last one may be shorter), one
 * Adam step per mini-batch (bias-corrected, step count kept by the model).
 * loss_hist (host, `epochs` entries, may be null): mean record loss of each
 * epoch, evaluated batch by batch before that batch's step.  Synchronizes
 * `stream`.  Errors: HHG_EINVAL for null pointers, n < 1, batch < 1,
 * epochs < 1, lr <= 0 or betas outside [0, 1); HHG_EHIP.                   */
typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr, beta1, beta2, eps;
} hhg_train_opts;
int hhg_mlp_train(hhg_mlp m, const void *samples, int64_t n, const hhg_train_opts *o,
                  float *loss_hist, void *stream);

/* Attach (or, with null, detach) the model used by HHG_PRECOND_LEARNED.  The
 * handle does not own it: keep it alive while solves use it.               */
int hhg_set_learned_model(hhg_handle h, hhg_mlp m);

/* Geometric multigrid on the hierarchy of uniform refinements (the paper's
 * solver, Sec. 5 and 6), for the scaled operator (interface rule of the
 * op descriptor, FP64):
 *   * one library handle per level coarse_level..L of the same conforming
 *     macro mesh (L = mesh->level[0]);
 *   * prolongation P: P1 interpolation from level l to l + 1 (a fine node
 *     that is a coarse node copies it, every other fine node is the midpoint
 *     of one coarse lattice edge and takes the mean of its end values);
 *     restriction R = P^T;
 *   * level operators rediscretised with the coefficient injected from the
 *     finest level (coarse node value = value at the same fine node);
 *   * smoother: damped block Jacobi x += omega D^-1 (b - A x), D the 3x3
 *     diagonal blocks (the paper smooths with a hybrid Gauss-Seidel);
 *   * coarsest level: exact solve with the inverse of the assembled operator
 *     (LU with partial pivoting; at most 512 unknown nodes, e.g. level 2);
 *   * hhg_mg_solve: CG preconditioned by one V(nu1, nu2) cycle per
 *     iteration (HHG_MG_CG; needs the symmetric interface rule), or the
 *     V-cycle iteration x += V(b - A x) the paper uses (HHG_MG_CYCLE; also
 *     for the row-wise interface rule, whose matrix is not symmetric).
 * Vectors are slot vectors of the level's handle ([3][n_nodes], FP64,
 * consistent, 16-byte aligned); Dirichlet entries are ignored on input and
 * written 0.  The caller owns every vector and the workspace
 * (hhg_mg_workspace_bytes, 256-byte aligned), which holds the per-level
 * coefficients, inverse blocks and vectors (FP64, and FP32 copies for FP32
 * cycles) and the coarse inverse between
 * hhg_mg_setup_coefficient and the cycles that use them (cycles and solves
 * accept only the workspace of the last coefficient setup).  Calls are
 * asynchronous on the stream except hhg_mg_create, hhg_mg_setup_coefficient
 * (synchronizes) and hhg_mg_solve (synchronizes once per iteration to test
 * convergence).  Errors: HHG_EINVAL (null or misaligned pointer, level out of
 * range, mixed levels, non-conforming mesh, a workspace without coefficient
 * setup, coarse level with more than 512 unknown nodes, nu1 + nu2 < 1,
 * omega outside (0, 2), nu_inc outside 0..8, unknown method or precision), HHG_EHIP,
 * HHG_EBREAKDOWN (singular coarse operator, or a breakdown of the solve),
 * HHG_ENOCONV (maxit reached; x and info are written).                     */
typedef struct hhg_mg_s *hhg_mg;
enum hhg_mg_method { HHG_MG_CG = 0, HHG_MG_CYCLE = 1 };
typedef struct {
  int32_t nu1, nu2;      /* pre- and post-smoothing steps (paper: 3, 3)      */
  double omega;          /* block-Jacobi damping, e.g. 0.7                    */
  double rtol;           /* hhg_mg_solve: ||b - A x|| <= rtol ||b||           */
  int32_t maxit;         /* hhg_mg_solve: iterations (CG steps or cycles)     */
  int32_t method;        /* hhg_mg_solve: hhg_mg_method                       */
  int32_t precision;     /* arithmetic of the cycle, hhg_prec: HHG_F64, or
                          * HHG_F32 (operator, smoother, transfers and vectors
                          * of every level in FP32, coarse inverse FP64; r is
                          * rounded to FP32 on entry and z widened on exit,
                          * while the solve's residuals, dot products and
                          * updates stay FP64)                                */
  int32_t nu_inc;        /* extra smoothing steps per level below the finest:
                          * level q of the finest F smooths nu1 + nu_inc (F - q)
                          * and nu2 + nu_inc (F - q) times (Sec. 5.2.1, the
                          * variable V-cycle: 2); 0: the fixed V(nu1, nu2)     */
} hhg_mg_opts;
int hhg_mg_create(const hhg_mesh_desc *mesh, const hhg_op_desc *op, int32_t coarse_level,
                  hhg_mg *out);
int hhg_mg_destroy(hhg_mg mg);
/* handle of one level (owned by mg: do not destroy it) */
int hhg_mg_level(hhg_mg mg, int32_t level, hhg_handle *out);
/* Blocks of the damped smoother x += omega P (b - A x) on the levels above
 * the coarsest (not in the paper): HHG_PRECOND_BLOCK_JACOBI (default,
 * P = D^-1) or HHG_PRECOND_LEARNED (P = (I + M)^T D^-1 (I + M) of
 * hhg_preconditioner, with the model attached to every one of those
 * levels' handles by hhg_set_learned_model).  Takes effect at the next
 * hhg_mg_setup_coefficient, which cycles and solves then require.  Errors:
 * HHG_EINVAL for another preconditioner or a level without a model.        */
int hhg_mg_set_smoother(hhg_mg mg, int32_t precond);
int hhg_mg_workspace_bytes(hhg_mg mg, size_t *bytes);
/* xf = P xc: xc on level fine_level - 1, xf on fine_level */
int hhg_mg_prolong(hhg_mg mg, int32_t fine_level, const double *xc, double *xf, void *stream);
/* rc = P^T rf (rc consistent over the copies; Dirichlet entries 0) */
int hhg_mg_restrict(hhg_mg mg, int32_t fine_level, const double *rf, double *rc, void *stream);
/* k: FP64 [n_nodes] coefficient of the finest level; injects it, builds the
 * inverse blocks of every level and the coarse inverse in the workspace.
 * method: the operator of every level from here on, HHG_METHOD_SCALED
 * (physical stencil scaling) or HHG_METHOD_ONTHEFLY (nodal integration) */
int hhg_mg_setup_coefficient(hhg_mg mg, int32_t method, const double *k, void *workspace,
                             void *stream);
/* z = V(r): one V(nu1, nu2) cycle on the finest level from z = 0 */
int hhg_mg_vcycle(hhg_mg mg, const hhg_mg_opts *o, const double *r, double *z, void *workspace,
                  void *stream);
/* x: start vector on input, solution on output (finest level) */
int hhg_mg_solve(hhg_mg mg, const hhg_mg_opts *o, const double *b, double *x, void *workspace,
                 hhg_solve_info *info, void *stream);

/* ------------------------------------------------ generalized Stokes
 * The incompressible generalized Stokes system of Sec. 5.2 (eqn.
 * generalizedstokes, stress 2 mu eps(u) - p I), equal-order P1 velocity and
 * pressure with the stabilization c_l(p, q) = -h_l^2/12 (grad p, grad q):
 *     [ A(mu)  B^T ] [u]   [f]
 *     [ B      C   ] [p] = [g],
 * A(mu) the velocity operator 2 (mu eps(u), eps(v)) of the handle (mu its
 * nodal coefficient), B[q, (j, l)] = -int d_l phi_j psi_q the divergence,
 * C = c_l.  Velocities are device FP64 [3][n_nodes], pressures device FP64
 * [n_nodes] (every node, all copies equal), 16-byte aligned.
 *
 * hhg_stokes_rows: one term on the handle's mesh, op
 *   HHG_STOKES_DIV   out[n]    = B in[3][n]   (Dirichlet velocities read as 0)
 *   HHG_STOKES_GRAD  out[3][n] = B^T in[n]    (Dirichlet rows 0)
 *   HHG_STOKES_STAB  out[n]    = C in[n], with mesh width hl (> 0)
 *   HHG_STOKES_MASS  out[n]    = int psi_q (lumped pressure mass; in unused)
 * Asynchronous on `stream`.  Errors: HHG_EINVAL, HHG_EHIP.                  */
enum hhg_stokes_op { HHG_STOKES_DIV = 0, HHG_STOKES_GRAD = 1, HHG_STOKES_STAB = 2,
                     HHG_STOKES_MASS = 3 };
int hhg_stokes_rows(hhg_handle h, int32_t op, double hl, const double *in, double *out,
                    void *stream);

/* Inexact Uzawa on the finest level of a multigrid handle (Sec. 5.2.1
 * names an inexact Uzawa method with V(3,3) cycles and pressure relaxation):
 *     u <- u + V(f - A u - B^T p)          (V: one cycle of hhg_mg_vcycle)
 *     p <- p + omega_p (B u + C p - g) / S,  S_q = mass_q / mu_q - C_qq
 *     p <- p - (mass . p) / (mass . 1)     (zero mean: the constant pressure
 *                                           lies in the kernel when every
 *                                           boundary node is Dirichlet)
 * until ||[f - A u - B^T p; g - B u - C p]|| <= rtol ||[f; g]|| (2-norms over
 * unknown velocity DoFs and all pressure nodes) or maxit steps.  The velocity
 * multigrid must hold A(mu): call hhg_mg_setup_coefficient(mg, method, mu,
 * mg_workspace) first.  u, p: start vectors on input, iterate on output.
 * g may be null (zero).  stokes_workspace: hhg_mg_stokes_workspace_bytes,
 * 256-byte aligned.  Synchronizes `stream` (every step reduces on the host).
 * info: iterations, rel_residual, status (HHG_OK / HHG_ENOCONV).            */
typedef struct {
  int32_t nu1, nu2;      /* velocity V-cycle smoothing steps (paper: 3, 3)   */
  double omega;          /* velocity block-Jacobi damping, e.g. 0.7          */
  double omega_p;        /* pressure relaxation                              */
  double h;              /* mesh width h_l of c_l; <= 0: 1 / 2^level (the
                          * unit-cube meshes, one macro edge of length 1)    */
  double rtol;           /* relative residual target                         */
  int32_t maxit;         /* Uzawa steps                                      */
  int32_t nu_inc;        /* velocity cycle: extra smoothing steps per coarser
                          * level, as hhg_mg_opts.nu_inc (the paper: 2)      */
} hhg_stokes_opts;
int hhg_mg_stokes_workspace_bytes(hhg_mg mg, size_t *bytes);
int hhg_mg_stokes_solve(hhg_mg mg, const hhg_stokes_opts *o, const double *f, const double *g,
                        const double *mu, double *u, double *p, void *mg_workspace,
                        void *stokes_workspace, hhg_solve_info *info, void *stream);

/* Fixed-point (Picard) iteration for the Carreau fluid (Sec. 5.2.2, eq.
 * fixpointsystem and Alg. fixedpoint_mg): from u = 0, p = 0 and
 * mu = mu(u) (hhg_nodal_viscosity, Sec. 3), repeat: one inexact Uzawa step
 * for the system with A(mu); mu = mu(u); until
 * max_i |u_i - u_i(previous)| < 1e-3 max_i |u_i| (node-wise 2-norms over
 * unknown nodes) or max_picard steps; then Uzawa steps with the last mu
 * until the relative residual is <= o->rtol (the paper: 1e-3) or o->maxit,
 * and a last mu = mu(u).  Uses the handle's operator (2 (mu eps, eps)) with
 * method HHG_METHOD_SCALED or HHG_METHOD_ONTHEFLY.  f: [3][n]; u, p, mu:
 * outputs.  Synchronizes `stream`.  info: picard steps, final Uzawa steps,
 * final relative residual, status.                                          */
typedef struct {
  int32_t picard;            /* fixed-point steps                           */
  int32_t final_iterations;  /* Uzawa steps of the final solve              */
  int32_t status;            /* HHG_OK, or HHG_ENOCONV if either loop hit
                                its limit                                    */
  int32_t pad;
  double rel_change;         /* last max |u - u_prev| / max |u|              */
  double rel_residual;       /* of the final solve                          */
  double seconds;
} hhg_picard_info;
int hhg_mg_stokes_picard(hhg_mg mg, const hhg_stokes_opts *o, const hhg_carreau *law,
                         int32_t method, int32_t max_picard, const double *f, double *u,
                         double *p, double *mu, void *mg_workspace, void *stokes_workspace,
                         hhg_picard_info *info, void *stream);

/* Kernel timing (tracing aid, not needed for results).  While enabled,
 * every kernel the library launches is bracketed by a pair of HIP events on
 * the launch stream.  hhg_profile_read synchronizes those events and returns,
 * per kernel id, the number of launches and the summed duration in ms since
 * enabling; ids: 0 interior scaled apply, 1 interior on-the-fly apply,
 * 2 macro-boundary rows, 3 copy-group sum, 4 solver vector kernels,
 * 5 learned smoother.
 * Enabling resets the counters.                                             */
enum hhg_kernel_id {
  HHG_K_INTERIOR_SCALED = 0,
  HHG_K_INTERIOR_ONTHEFLY = 1,
  HHG_K_BOUNDARY_ROWS = 2,
  HHG_K_GROUP_SUM = 3,
  HHG_K_SOLVER_VECTOR = 4,   /* all fused vector / reduction kernels of the solvers */
  HHG_K_LEARNED = 5,         /* features and network inference of the learned smoother */
  HHG_K_COUNT = 16
};
int hhg_profile_enable(hhg_handle h, int32_t on);
int hhg_profile_read(hhg_handle h, int32_t kernel_id, int64_t *launches, double *total_ms);

/* ---------------------------------------------------------------- 2-D
 * The method on macro triangles (Sec. 2, Sec. 2.3): each macro triangle
 * (vertices x0, x1, x2) is refined uniformly, 2^level intervals per edge;
 * node (i, j), i + j <= n, lies at x0 + (i/n)(x1 - x0) + (j/n)(x2 - x0) and
 * occupies slot off_m + j(n+1) - j(j-1)/2 + i, off_m = m (n+1)(n+2)/2.
 * Vectors are [2][n_slots] (x, y) and [n_slots] (k); nodes shared by macros
 * have one slot per macro, kept equal.  The operator is that of
 * hhg_op_desc in two dimensions.  Physical scaling (Lemma, eq.
 * correction2d): every edge of a macro-interior node has two elements, each
 * the reflection of the other, so the scaled stencil reproduces nodal
 * integration exactly (for any k) from the reference stencil, k at the
 * 7-point patch and one correction constant per direction.  Rows of nodes on
 * macro boundaries follow op->iface as in 3-D.
 * Flags per slot: bit 0 Dirichlet, bit 1 owner, bit 2 on a macro boundary,
 * bit 3 node with copies in other macros.                                  */
typedef struct hhg2d_ctx *hhg2d_handle;
typedef struct {
  int32_t n_macro;
  const double *verts;   /* host, [n_macro][3][2]                            */
  int32_t level;         /* 1..13, common to all macros                      */
  int32_t dirichlet;     /* HHG_DIRICHLET_OUTER: homogeneous on every macro
                            edge met by one macro; HHG_DIRICHLET_NONE         */
} hhg2d_mesh_desc;

/* Set up a 2-D mesh and operator (host only; tables go to the device at the
 * first apply).  Errors: HHG_EINVAL for a null argument, level outside
 * 1..13, unknown options or a degenerate macro.                            */
int hhg2d_setup(const hhg2d_mesh_desc *mesh, const hhg_op_desc *op, hhg2d_handle *out);
int hhg2d_destroy(hhg2d_handle h);
/* n_slots (vector length) and unknown nodes (distinct, non-Dirichlet).     */
int hhg2d_layout(hhg2d_handle h, int64_t *n_slots, int64_t *n_unknown);
/* Host outputs: coordinates [2][n_slots]; flags [n_slots] as above.        */
int hhg2d_node_coords(hhg2d_handle h, double *xy);
int hhg2d_node_flags(hhg2d_handle h, uint8_t *flags);
/* y = A x on the device: prec HHG_F64 or HHG_F32 (x, k, y of that type),
 * method HHG_METHOD_SCALED (scaled stencils on macro-interior rows) or
 * HHG_METHOD_ONTHEFLY (nodal integration, eq. nodalquad, on every row).
 * Dirichlet rows are zero and Dirichlet entries of x are read as 0; y is
 * consistent over copies.  Asynchronous on `stream`.  Errors: HHG_EINVAL
 * for null or misaligned pointers, y aliasing x or k, unknown options.      */
int hhg2d_apply(hhg2d_handle h, int32_t prec, int32_t method, const void *x, const void *k, void *y,
                void *stream);

/* Text of the calling thread's last error ("" if none).                    */
const char *hhg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HHG_H */
