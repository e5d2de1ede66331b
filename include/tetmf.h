/*
 * tetmf.h -- matrix-free finite-element operators on uniformly refined
 * macro-tetrahedra, for AMD Instinct MI355X (gfx950).
 *
 * The library computes y = A x for operators defined by a weak form on a
 * coarse (macro) tetrahedral mesh refined uniformly `level` times, without
 * assembling A.  Equation (4.1) of the paper's section "Matrix-Free Finite
 * Elements" defines the operation: A = sum_T P_T A_T R_T over all
 * micro-tetrahedra T, with A_T the local matrix of the integrand on T
 * (algorithm "LocalApply").  Section "Hybrid Tetrahedral Grids" defines the
 * mesh: each macro-tetrahedron is refined uniformly, every micro-tetrahedron
 * is a translate of one of six reference shapes, and DoFs are addressed by
 * implicit structured indices.  Operator kinds:
 *
 *   TMF_P1_LAPLACE   int grad(phi_i).grad(phi_j), linear Lagrange  (equation P1)
 *   TMF_P1_DIVKGRAD  int k grad(phi_i).grad(phi_j), k nodal linear
 *   TMF_P2_LAPLACE   int grad(phi_i).grad(phi_j), quadratic Lagrange
 *   TMF_P2_DIVKGRAD  int k grad(phi_i).grad(phi_j), k nodal quadratic (equation P2V)
 *   TMF_P2V_EPSILON  int 2 mu eps(u):eps(v), eps = sym grad, vector quadratic
 *                    Lagrange, mu nodal quadratic
 *   TMF_N1_CURLCURL  int alpha curl(phi_i).curl(phi_j) + beta phi_i.phi_j,
 *                    first-kind lowest-order Nedelec elements, alpha and beta
 *                    nodal linear (equation N1, section "Curl-Curl and Mass")
 *
 * N1 layout: the operator uses the quadratic lattice (N = 2n).  The DoF of a
 * micro-edge sits at the slot of its midpoint and is the tangential integral
 * along the edge oriented from the endpoint with the smaller canonical key
 * (the ordering of tmf_mesh_dof_info's keys, compared as 8 signed integers
 * in turn) to the larger; vertex slots carry no DoF (zero rows, their inputs
 * ignored).  Its coefficient vector holds 2 * n_local values: alpha, then
 * beta, each read at the vertex slots only.
 *
 * All are positive semi-definite stiffness matrices.  The affine forms are
 * integrated exactly (the integrand of P2V has degree 4; the kernels use the
 * exact closed form, which equals any degree-4-exact quadrature up to
 * rounding).  The epsilon operator on the radially blended shell map is
 * integrated with the quadrature rule given at operator creation.
 *
 * --- Vector layout ("macro-local") -----------------------------------------
 * The refinement lattice of macro tet (v0,v1,v2,v3) at level l, n = 2^l, is
 * the set of points (i,j,k), i,j,k >= 0, i+j+k <= N, at parameter position
 * v0 + (i(v1-v0) + j(v2-v0) + k(v3-v0))/N, integer barycentric coordinates
 * (N-i-j-k, i, j, k).  P1 DoFs use N = n; P2 DoFs use N = 2n (micro-vertex
 * p -> 2p, micro-edge (p,q) -> p+q).  Within a macro, point (i,j,k) is stored
 * at
 *     idx = C3(N) - C3(N-k) + j(2(N-k)+3-j)/2 + i,   C3(M) = (M+1)(M+2)(M+3)/6
 * (i fastest, then j, then k); macro m's block starts at m * C3(N).  A DoF on
 * a face, edge or vertex shared by several macros has one copy per macro.
 * Vector fields (epsilon operator) are stored component-major: [u_x | u_y | u_z],
 * each block of length n_local.  Coefficients use the layout of the space
 * they live in (P1 for TMF_P1_DIVKGRAD, P2 otherwise), one scalar per point.
 *
 * Inputs must be consistent (all copies of a DoF equal); outputs are
 * consistent (the partial sums of the copies are added and every copy gets
 * the total).  The canonical key of a point, which identifies the copies of
 * one DoF, is the list of (global vertex id, barycentric integer) pairs with
 * nonzero integer, sorted by vertex id, padded with (-1, 0): see
 * tmf_mesh_dof_info.
 *
 * --- Boundary condition ----------------------------------------------------
 * TMF_BC_DIRICHLET_ZERO applies D A D, D the 0/1 mask of DoFs not on the
 * domain boundary: boundary rows and columns are zero (y_b = 0, x_b ignored).
 * A DoF is on the domain boundary when one of its copies lies on a macro face
 * that belongs to a single macro tet.  TMF_BC_NONE applies A.
 *
 * --- Ownership, streams, errors --------------------------------------------
 * Every call returns TMF_OK (0) or a negative code; no exception crosses the
 * ABI and tmf_last_error() gives a thread-local message for the last failure.
 * Handles are owned by the library (create / destroy).  Device buffers passed
 * to apply calls are owned by the caller; they must be device memory of the
 * current HIP device, aligned to their element type, and must not alias
 * unless stated.  Apply calls enqueue work on `stream` (a hipStream_t; NULL
 * = the default stream) and return without synchronising; they allocate
 * nothing, so they can be captured into a HIP graph.  On an argument error
 * nothing is enqueued and outputs are untouched.
 */
#ifndef TETMF_H
#define TETMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tmf_status;
#define TMF_OK 0
#define TMF_EINVAL (-1)        /* invalid argument */
#define TMF_ENOMEM (-2)        /* host or device allocation failed */
#define TMF_EDEVICE (-3)       /* HIP runtime error (launch, copy) */
#define TMF_EUNSUPPORTED (-4)  /* valid but unsupported combination */
#define TMF_ENOTCONV (-5)      /* iterative solve did not reach its tolerance */

#define TMF_P1_LAPLACE 0
#define TMF_P1_DIVKGRAD 1
#define TMF_P2_LAPLACE 2
#define TMF_P2_DIVKGRAD 3
#define TMF_P2V_EPSILON 4
#define TMF_N1_CURLCURL 5

#define TMF_F64 0
#define TMF_F32 1

#define TMF_BC_NONE 0
#define TMF_BC_DIRICHLET_ZERO 1

/* Geometry map of the macro mesh.  AFFINE: physical = parametric position.
 * SHELL_RADIAL: physical x = Phi(xi) = xi |xi|_1 / |xi|_2, which maps the
 * flat faces |xi|_1 = r onto spheres of radius r (every macro tet must lie in
 * one closed coordinate octant).  Curved elements enter only through the
 * Jacobian at quadrature points (the curvilinear remark of the tabulation
 * section). */
#define TMF_MAP_AFFINE 0
#define TMF_MAP_SHELL_RADIAL 1

#define TMF_MAX_LEVEL_P1 9
#define TMF_MAX_LEVEL_P2 8
#define TMF_MAX_QUAD 64

typedef struct tmf_mesh tmf_mesh;
typedef struct tmf_op tmf_op;
typedef struct tmf_batch tmf_batch;
typedef void *tmf_stream; /* hipStream_t */

/* Library version string and the last error message of this thread. */
const char *tmf_version(void);
const char *tmf_last_error(void);
const char *tmf_status_string(tmf_status s);

/* Create a refined macro mesh.
 *   vertices  host, nv x 3 doubles (row-major)
 *   tets      host, nt x 4 vertex ids in [0, nv); the vertex order of a tet
 *             fixes its lattice (vertex 0 = lattice origin)
 *   level     refinement level, 0 <= level <= TMF_MAX_LEVEL_P1 (P2 operators
 *             further require level <= TMF_MAX_LEVEL_P2)
 *   map       TMF_MAP_AFFINE or TMF_MAP_SHELL_RADIAL
 * Errors: TMF_EINVAL for nv < 4, nt < 1, ids out of range, repeated ids in a
 * tet, zero-volume tets, a face shared by more than two tets, non-finite
 * coordinates, a bad level or map, or (SHELL_RADIAL) a tet not contained in
 * one octant or touching the origin. */
tmf_status tmf_mesh_create(const double *vertices, int64_t nv, const int64_t *tets, int64_t nt,
                           int level, int map, tmf_mesh **out);
void tmf_mesh_destroy(tmf_mesh *mesh);

/* Sizes of the macro-local layout of space 1 (P1) or 2 (P2): n_local scalar
 * slots per component (nt * C3(N)) and the number of distinct DoFs. */
tmf_status tmf_mesh_layout(const tmf_mesh *mesh, int space, int64_t *n_local, int64_t *n_unique);

/* Host-side description of every slot of the layout of `space`.  Each output
 * may be NULL; non-NULL outputs are caller-allocated host arrays:
 *   keys      n_local x 8 int64 canonical keys (pairs (vertex id, integer))
 *   xyz       n_local x 3 doubles, physical position (after the map)
 *   owner     n_local bytes, 1 on exactly one copy of each DoF
 *   boundary  n_local bytes, 1 if the DoF is on the domain boundary */
tmf_status tmf_mesh_dof_info(const tmf_mesh *mesh, int space, int64_t *keys, double *xyz,
                             uint8_t *owner, uint8_t *boundary);

/* Create an operator on `mesh` (the mesh must outlive the operator).
 *   kind   TMF_P1_LAPLACE .. TMF_N1_CURLCURL
 *   prec   TMF_F64 or TMF_F32: element type of coefficient, x and y; the
 *          geometry constants are computed in FP64 on the host and rounded
 *          once for TMF_F32
 *   bc     TMF_BC_NONE or TMF_BC_DIRICHLET_ZERO
 *   qbary, qw, nq   quadrature rule on the reference tet (host arrays: nq x 4
 *          barycentric coordinates, nq weights summing to 1/6).  Required
 *          (1 <= nq <= TMF_MAX_QUAD) for the blended shell map, which only the
 *          epsilon operator supports.  On affine meshes forms are integrated
 *          exactly and the rule must be NULL/NULL/0, except for
 *          TMF_P2_DIVKGRAD, where a rule selects its quadrature variant:
 *          weights 6 sum_q w_q k(q) lambda_c(q) lambda_e(q) in place of the
 *          exact ones (the under-integration option of section
 *          "Variable-Coefficient Diffusion" with a degree-2 rule; a rule of
 *          degree >= 4 gives the exact operator).  Diagonal, adjoint, stored
 *          matrices and batches are provided for the exact operator only.
 * Allocates the operator's device tables on the current HIP device.
 * Errors: TMF_EINVAL (bad enum, level above the space maximum, bad rule),
 * TMF_EUNSUPPORTED (blended map with a scalar kind), TMF_ENOMEM, TMF_EDEVICE. */
tmf_status tmf_op_create(const tmf_mesh *mesh, int kind, int prec, int bc, const double *qbary,
                         const double *qw, int nq, tmf_op **out);
void tmf_op_destroy(tmf_op *op);

/* n_local per component, n_unique scalar DoFs per component, components (1 or 3),
 * and whether the kind takes a coefficient field. */
tmf_status tmf_op_info(const tmf_op *op, int64_t *n_local, int64_t *n_unique, int *ncomp,
                       int *has_coeff);

/* y = A(coeff) x (device pointers, element type per the op's precision).
 * coeff: n_local values for the DIVKGRAD and EPSILON kinds, NULL otherwise.
 * x, y: ncomp * n_local values; y must not alias x or coeff. */
tmf_status tmf_apply(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream);

/* tmf_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * operation and arguments, with the seam partial sums of the P2 and epsilon
 * kinds (the apply's only device memory beyond x, coeff and y) in a static
 * device array of 64 MiB that every GPU the library is loaded on holds until
 * the process ends, instead of the operator's own buffer.  Allocates nothing
 * and never synchronises.  All calls on one GPU share that array: calls whose
 * executions overlap on a GPU (several streams, or a graph replayed
 * concurrently) race and give wrong results; calls ordered on one stream are
 * safe (no state carries over between calls).  P1 kinds use no scratch and
 * behave as tmf_apply.  Errors as tmf_apply, and TMF_EINVAL when the
 * operator's partial sums at its current tile shape exceed 64 MiB (the
 * message gives both sizes; e.g. the P2 FP64 cube of 6 macros at level 6
 * needs about 29 MB, at level 7 about 230 MB). */
tmf_status tmf_apply_noalloc(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream);

/* The macro-local part of the apply: y = sum over macros M of the sum over
 * micro-tets T of M of P_T A_T R_T x, i.e. tmf_apply without the final
 * interface sum.  On a DoF shared by several macros each copy holds only its
 * own macro's partial sum (x is read copy by copy).  tmf_apply is
 * tmf_apply_local followed by tmf_interface_sum. */
tmf_status tmf_apply_local(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream);

/* In place, v <- S v: every copy of a shared DoF receives the sum over its
 * copies (ncomp * n_local values of the op's precision; copies added in
 * ascending slot order).  No-op on single-macro meshes. */
tmf_status tmf_interface_sum(tmf_op *op, void *v, tmf_stream stream);

/* d = diag(A(coeff)): the diagonal of the operator that tmf_apply applies
 * (one of the operations the paper's generator provides besides the
 * matrix-vector product, section "Code Generation for FEM on Hybrid
 * Tetrahedral Grids"; its Conclusion names the inverse diagonal for
 * smoothers).  d_i = sum over the micro-tets T containing DoF i of
 * (A_T)_ii, summed over the copies of a shared DoF (every copy receives the
 * total); with TMF_BC_DIRICHLET_ZERO the rows of boundary DoFs are 0, as in
 * D A D.  coeff as for tmf_apply; d: ncomp * n_local values of the op's
 * precision (device; for TMF_P2V_EPSILON the diagonal of each component block,
 * component-major like x), must not alias coeff.  Asynchronous on `stream`.
 * Provided for the P1 kinds, the exactly integrated scalar P2 kinds and the
 * epsilon operator (affine or blended; on the blended shell each micro-tet's
 * 30 diagonal entries are formed by applying its element to unit vectors);
 * TMF_N1_CURLCURL and the quadrature variant of TMF_P2_DIVKGRAD return
 * TMF_EUNSUPPORTED. */
tmf_status tmf_diagonal(tmf_op *op, const void *coeff, void *d, tmf_stream stream);

/* The precomputed-matrix alternative to the matrix-free apply (the paper's
 * comparison of matrix-free kernels with stored local matrices, section
 * "Matrix-Free Finite Elements"): tmf_op_store_matrices evaluates every
 * micro-tet's symmetric 10 x 10 local matrix A_T(coeff) of TMF_P2_DIVKGRAD
 * once and keeps its 55 upper-triangle entries in device memory owned by the
 * op (about 55 * 8 bytes per micro-tet in FP64, allocated here; laid out per
 * tile, type and entry with the box's cubes contiguous, for the tile shape
 * current at this call); tmf_apply_stored then computes y = A x from them
 * (same result as tmf_apply with that coeff, up to rounding).  Both are
 * asynchronous on `stream`; tmf_apply_stored allocates nothing.  Errors:
 * TMF_EUNSUPPORTED for other kinds; TMF_EINVAL if nothing is stored. */
tmf_status tmf_op_store_matrices(tmf_op *op, const void *coeff, tmf_stream stream);
tmf_status tmf_apply_stored(tmf_op *op, const void *x, void *y, tmf_stream stream);

/* Reverse mode of the macro-local apply of TMF_P1_DIVKGRAD, TMF_P2_DIVKGRAD
 * and TMF_P2V_EPSILON (FP64 or FP32; for epsilon k is mu, and x, gy, gx hold
 * 3 * n_local values while coeff and gk hold n_local).
 * With y = L(k) x the local apply (boundary masking included), given gy:
 *   gx = L(k)^T gy = L(k) gy,
 *   gk_m = gy . (dL/dk_m) x   for every coefficient slot m (copy by copy;
 *          not zeroed on Dirichlet DoFs, whose k values act on interior rows),
 * gk written only if non-NULL.  The transpose of the full apply y = S L(k) x
 * is therefore: tmf_interface_sum on (a copy of) dL/dy, then this call.  For
 * a single macro S = I.  All pointers are device arrays; gx and gk must not
 * alias each other or any input.  P1: one fused launch.  P2
 * and epsilon: gx is the macro-local apply of gy, gk a second
 * element-kernel launch (L is linear in the nodal k, so gk_m = gy . L(e_m) x,
 * formed per micro-tet from the gradients or strains of x and gy; on the
 * blended shell per quadrature point).  Other kinds return TMF_EUNSUPPORTED. */
tmf_status tmf_apply_adjoint(tmf_op *op, const void *coeff, const void *x, const void *gy,
                             void *gx, void *gk, tmf_stream stream);

/* Same as tmf_apply, and additionally records the caller-created hipEvent_t
 * `ev_before` on `stream` immediately before the operator's main compute
 * kernel and `ev_after` immediately after it (fills and interface sums
 * outside), so that the kernel's own duration can be measured.  Either event
 * may be NULL. */
tmf_status tmf_apply_timed(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream,
                           void *ev_before, void *ev_after);

/* Tile shapes of the element-centric (P2, epsilon, N1) kernels.  Shapes 0-3
 * are boxes of micro-cubes staged in LDS by one workgroup (4x4x4, 8x4x2,
 * 8x4x4, 4x4x8); shapes 4-6 are column segments of 2, 4 and 8 sub-boxes of
 * 4x4x4 cubes (4x4x8, 4x4x16, 4x4x32) walked in z by a persistent workgroup,
 * for the exactly integrated scalar P2 applies (their other modes -- diagonal,
 * adjoint's coefficient gradient, stored matrices -- then run on the best box
 * shape).  tmf_op_num_tiles gives the number of shapes valid for the op's
 * kind (1 for P1 kinds, whose kernels are vertex-centric; 2 for epsilon: the
 * 64-cube boxes; 4 for N1 and the quadrature variant; 7 for the exact scalar
 * P2 kinds), tmf_op_tile_shape the cubes per tile edge. */
tmf_status tmf_op_num_tiles(const tmf_op *op, int *count);
tmf_status tmf_op_tile_shape(const tmf_op *op, int cfg, int *tx, int *ty, int *tz);
tmf_status tmf_op_set_tile(tmf_op *op, int cfg);
tmf_status tmf_op_get_tile(const tmf_op *op, int *cfg);

/* Autotuner: times `reps` applies of every valid tile shape on the given
 * (caller-owned, device) inputs with HIP events, keeps the fastest shape on
 * the op and returns it with its mean time per apply.  Synchronises the
 * stream; overwrites y.  Every shape computes the same operator (parity is
 * tested per shape); results differ only by floating-point summation order. */
tmf_status tmf_op_autotune(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream,
                           int reps, int *best_cfg, float *best_ms);

/* tmf_op_autotune with a result cache: a JSON file (host path) mapping a key
 * (operator kind, precision, boundary condition, rule size, map, level, macro
 * count, device architecture and compute units) to the chosen tile shape, the
 * box shape used by the modes marching shapes do not provide, and the time.
 * If the key is present, its shapes are set on the op without timing
 * (best_ms = the cached time); otherwise the shapes are timed as by
 * tmf_op_autotune and the result is added to the file (created if missing,
 * rewritten through a temporary file).  cache_json_path NULL: plain
 * autotune.  TMF_EINVAL if the file exists but is not such a cache or cannot
 * be written. */
tmf_status tmf_op_tune(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                       const char *cache_json_path, int *best_cfg, float *best_ms);

/* ---------------------------------------------------------------- batches
 * A batch applies `count` operator instances in one launch of the element
 * kernel (instances may have different meshes, levels and
 * coefficients).  All operators must be P2 kinds (TMF_P2_LAPLACE,
 * TMF_P2_DIVKGRAD or TMF_P2V_EPSILON) of one kind and one precision on affine
 * meshes; they must outlive the batch.  Vectors are concatenated: instance i
 * occupies [offsets[i], offsets[i+1]) with its own layout inside (components
 * of vector fields consecutive).  Errors: TMF_EINVAL (NULL, duplicate or
 * mismatched operators), TMF_EUNSUPPORTED (P1 kind, curved map), TMF_ENOMEM. */
tmf_status tmf_batch_create(tmf_op *const *ops, int count, tmf_batch **out);
void tmf_batch_destroy(tmf_batch *batch);
/* count and, if offsets != NULL, the count + 1 offsets (host array). */
tmf_status tmf_batch_info(const tmf_batch *batch, int *count, int64_t *offsets);
/* y = A_i(coeff_i) x_i for every instance i with active[i] != 0 (device byte
 * array, or NULL for all); y of inactive instances is set to 0.  Same rules as
 * tmf_apply (asynchronous on `stream`, no allocation, capturable). */
tmf_status tmf_batch_apply(tmf_batch *batch, const void *coeff, const void *x, void *y, const uint8_t *active,
                           tmf_stream stream);
/* tmf_batch_apply with events around the element kernel (see tmf_apply_timed). */
tmf_status tmf_batch_apply_timed(tmf_batch *batch, const void *coeff, const void *x, void *y,
                                 const uint8_t *active, tmf_stream stream, void *ev_before, void *ev_after);
/* d_i = diag(A_i(coeff_i)) for every instance (as tmf_diagonal), in one
 * launch; scalar P2 kinds only. */
tmf_status tmf_batch_diagonal(tmf_batch *batch, const void *coeff, void *d, tmf_stream stream);
tmf_status tmf_batch_set_tile(tmf_batch *batch, int cfg);
/* Autotuner over the tile shapes for the whole batch (as tmf_op_autotune). */
tmf_status tmf_batch_autotune(tmf_batch *batch, const void *coeff, const void *x, void *y, tmf_stream stream,
                              int reps, int *best_cfg, float *best_ms);
/* Batch autotuner with the result cache of tmf_op_tune (key: kind,
 * precision, each instance's level and macro count in order, device). */
tmf_status tmf_batch_tune(tmf_batch *batch, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                          const char *cache_json_path, int *best_cfg, float *best_ms);

/* ------------------------------------------------ mixed-precision solver
 * Iterative refinement for A_i x_i = b_i over a batch: outer iterations in
 * FP64 (r = b - A x with the FP64 batch, norms, x += |r| d), inner
 * conjugate-gradient corrections A d = r / |r| with the inner batch (FP32:
 * the mixed-precision solve; or FP64: plain FP64 CG, the comparison form)
 * and FP64-accumulated dot products, started from d = 0 and stopped per
 * instance when r.r (r.z with the Jacobi preconditioner) has fallen to
 * inner_rtol^2 times its start value, or after inner_maxit iterations.
 * Blocks of graph_iters inner iterations are captured once into a HIP graph
 * and replayed (use_graph = 0 runs the same kernels eagerly).  An instance
 * stops when |b - A x| <= tol |b| (2-norms over distinct DoFs).  With an FP64
 * inner batch and inner_rtol below tol, the first outer step is a plain
 * (Jacobi-preconditioned) FP64 CG solve to tol and the second confirms it. */
typedef struct tmf_ir tmf_ir;
/* Inner preconditioner: none, or Jacobi (z = D^-1 r with D = diag(A) of the
 * FP64 operators, assembled by tmf_batch_diagonal at the start of each solve;
 * Dirichlet rows, whose diagonal is 0, get 0).  With Jacobi the inner
 * iteration is preconditioned CG and its stopping test uses r.z. */
enum { TMF_PRECOND_NONE = 0, TMF_PRECOND_JACOBI = 1 };
typedef struct {
  double tol;         /* outer relative residual, e.g. 1e-10 */
  int max_outer;      /* outer steps */
  double inner_rtol;  /* inner relative residual, e.g. 1e-4 */
  int inner_maxit;    /* inner iterations per outer step */
  int graph_iters;    /* inner iterations per graph launch (even, >= 2) */
  int use_graph;      /* 1: replay a captured HIP graph */
  int precond;        /* TMF_PRECOND_NONE or TMF_PRECOND_JACOBI */
} tmf_ir_options;
typedef struct {
  int outer;           /* outer refinement steps taken */
  int inner_total;     /* inner iterations, summed over outer steps (max over instances) */
  int graph_launches;  /* graph replays */
  int converged;       /* 1 if every instance reached tol */
  double seconds;      /* wall time of the solve */
} tmf_ir_stats;
/* Both batches hold the same instances (same meshes and boundary conditions),
 * b64 in FP64 and the inner batch b32 in FP32 or FP64 (it may be b64 itself),
 * scalar kinds only; opt may be NULL for the defaults {1e-10, 30, 1e-4, 2000,
 * 16, 1, TMF_PRECOND_JACOBI}.  Allocates the device workspace (2 FP64 vectors
 * and 4 inner vectors of the batch length, 5 with Jacobi) and a private
 * stream.  Jacobi needs a scalar P2 kind (TMF_EUNSUPPORTED otherwise). */
tmf_status tmf_ir_create(tmf_batch *b64, tmf_batch *b32, const tmf_ir_options *opt, tmf_ir **out);
void tmf_ir_destroy(tmf_ir *solver);
/* Solve in place: x (device, FP64, initial guess on entry), b (device, FP64),
 * coefficients in FP64 and in the inner batch's precision (device; NULL for
 * constant-coefficient kinds).
 * Ordered after the work already queued on `stream`; blocks until done.
 * relres (host, count doubles, may be NULL) receives the final FP64 relative
 * residuals.  Returns TMF_ENOTCONV if max_outer steps were not enough. */
tmf_status tmf_ir_solve(tmf_ir *solver, const double *coeff64, const void *coeff_inner, const double *b, double *x,
                        tmf_ir_stats *stats, double *relres, tmf_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* TETMF_H */
