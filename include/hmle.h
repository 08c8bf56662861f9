/*
 * hmle.h -- C ABI of the MI355X hierarchical-matrix maximum-likelihood library.
 *
 * What it computes (Chen & Anitescu, "Scalable Physics-based Maximum Likelihood
 * Estimation using Hierarchical Matrices"):
 *   K(theta) = sigma2 * A^{-1} B^{-1} B^{-T} A^{-T} + tau2 * I           (Sec. 2.1, eq. "cov model")
 *   with B = kappa^2 I - Lap, A = I - alpha Lap on a Dirichlet grid (Sec. 5.1, eq. "SPDE"
 *   analogue), accessed only through products with blocks of vectors;
 *   K~(theta) ~ K(theta) in HODLR form built by randomized peeling            (Sec. 3.1-3.2, Alg. 1)
 *   K~_j = dK~/dtheta_j in the same format, by differentiating the peeling     (Sec. 3.3, Alg. 2)
 *   log|K~|, K~^{-1} y via the leaf-times-low-rank-updates factorisation       (Sec. 3.1, eq. "one way factor"; App. C)
 *   L~, grad(-L~), and I~_ij = 1/2 tr(K~^{-1} K~_i K~^{-1} K~_j)              (Sec. 4, eqs. "log-like approximated",
 *                                                                              "score approximated", "fisher info approximated")
 * with exact traces of HODLR products (Sec. 4.2, App. B) -- no stochastic estimator.
 *
 * Conventions
 *   * Every call returns hm_status; nothing throws across the ABI.  On failure
 *     hm_last_error() describes the cause.
 *   * Device buffers passed in (y, x, omega, X, Y) are plain device pointers
 *     owned by the caller; the library never frees them.  The library's own device
 *     memory comes from the context's allocator callbacks (hm_ctx_create).  Host
 *     buffers are plain host pointers owned by the caller.
 *   * All device work is enqueued on the stream given to hm_model_create; calls
 *     that return host scalars synchronise that stream once before returning.
 *   * Vectors y, x passed to solve / loglik are in natural grid order
 *     (row-major, x fastest).  Sketch draws are indexed by tree position.
 *   * The full parameter vector is theta_full[4] = (kappa, alpha, tau2, sigma2);
 *     the "free" parameters (gradient / Fisher order) are chosen by index.
 *   * Not thread-safe per handle: calls on one handle must not overlap.
 */
#ifndef HMLE_H
#define HMLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HM_OK = 0,
  HM_E_INVAL = 1,      /* bad sizes, unsupported shape, bad parameter (tau2 <= 0, ...) */
  HM_E_NOMEM = 2,      /* device allocation failed */
  HM_E_NOT_SPD = 3,    /* a leaf Cholesky pivot <= 0, or det(I + V^T U) <= 0 at a node */
  HM_E_RANK = 4,       /* every sketch block of a level has rank 0 */
  HM_E_NONFINITE = 5,  /* NaN/Inf in theta or detected on the device */
  HM_E_STATE = 6,      /* call out of order (e.g. fisher before factor) */
  HM_E_DEVICE = 7      /* HIP runtime error */
} hm_status;

typedef struct hm_ctx hm_ctx;       /* device, stream, device-memory allocator callbacks */
typedef struct hm_model hm_model;   /* grid, tree ordering, transform tables, stream */
typedef struct hm_sketch hm_sketch; /* fixed test matrices (drawn once, Sec. 3.3) + frozen compression */
typedef struct hm_H hm_H;           /* K~(theta), K~_j(theta), factorisation, per-iteration workspace */

/* Last error message of the calling thread (static storage, valid until the next call). */
const char* hm_last_error(void);

/* -------------------------------------------------------------- context ---
 * Device memory: every device buffer of a model, of its sketches and of its H
 * handles (panel sets, leaves, workspaces, setup temporaries) is obtained from
 * alloc(uctx, bytes) and returned with release(uctx, ptr) -- e.g. a framework's
 * caching allocator, so that the caller owns and accounts for the memory.  alloc
 * returns NULL on failure (the call then fails with HM_E_NOMEM); the memory must be
 * usable by work on `stream` in stream order.  With alloc = release = NULL the
 * library uses hipMalloc / hipFree.  Pinned host staging (a few KB per H) is not
 * device memory and is allocated by the library.  The context must outlive every
 * model created with it; it is not thread-safe. */
typedef void* (*hm_alloc_fn)(void* uctx, size_t bytes);
typedef void (*hm_free_fn)(void* uctx, void* ptr);
hm_status hm_ctx_create(int device, void* stream, hm_alloc_fn alloc, hm_free_fn release, void* uctx,
                        hm_ctx** out);
void hm_ctx_destroy(hm_ctx* c);

/* A caller-supplied covariance operator (the paper's black-box access to K, Sec. 3.2;
 * Sec. 2.1 eq. "general physical model"): Y = op_which(theta) X for c columns, where
 * which = 0 applies K_op(theta_full[0], theta_full[1]), 1 its derivative in
 * theta_full[0], 2 its derivative in theta_full[1].  X, Y: device, n x c column-major
 * (ld ldx, ldy) in the caller's point order; the work is enqueued on `stream` (the
 * model's) and must not synchronise with the host when it can be avoided.  Return 0,
 * or nonzero for failure (the library call then fails with HM_E_DEVICE).  K_op must be
 * symmetric (and its derivatives), positive semidefinite. */
typedef int (*hm_op_fn)(void* uctx, int which, const double* theta_full, const double* X, long long ldx,
                        long long c, double* Y, long long ldy, void* stream);

/* ---------------------------------------------------------------- model ---
 * hm_model_create: the stencil covariance model on a dim-D grid of side N
 * (n = N for dim 1, N*N for dim 2; h = 1/(N+1), Dirichlet boundary).
 * leaf: target leaf size; levels = floor(log2(n/leaf)) (Sec. 5.2 rule).
 * The tree is the recursive coordinate bisection of the grid (Sec. 5.2, KD-tree
 * ordering): split the longer side (x on ties), left child gets floor(side/2), so
 * leaves may differ in size (Sec. 3.2: block sizes need not divide); see hm_model_rows.
 * device: HIP device ordinal; stream: hipStream_t to enqueue on (NULL = default).
 */
hm_status hm_model_create(int device, void* stream, int dim, int N, int leaf, hm_model** out);
/* The same model with its device memory from a context (allocator callbacks, device and
 * stream of ctx) and the grid given in full (Sec. 2.1 eq. "cov model" with the stencil
 * operators of Sec. 5.1; observations Sec. 5.1 eq. "projection"):
 *   dim 1: nx points, ny = 1; dim 2: an nx x ny grid (row-major, x fastest);
 *   h: grid spacing (> 0) of the Dirichlet stencil (-Laplacian = (1/h^2) x 3-/5-point);
 *      hm_model_create uses h = 1/(N+1), the unit interval / square;
 *   nvars: variables per location.  1: the model above.  2: bivariate co-kriging (the
 *      2 x 2 block covariance of co-located variables, the analogue of Sec. 5.2's
 *      bivariate model, eq. "kphichi"): one latent noise w drives y1 = sigma B^{-1} w +
 *      tau1 eps1 and y2 = sigma A^{-1} B^{-1} w + tau2 eps2 at every node, so
 *      K = sigma2 [[C, C A^{-T}], [A^{-1} C, A^{-1} C A^{-T}]] + diag(tau2_1 I, tau2_2 I),
 *      C = B^{-1} B^{-T}; n = 2 x nodes, vectors stacked (y1; y2); theta_full has FIVE
 *      entries (kappa, alpha, tau2_1, sigma2, tau2_2) in every call on such a model
 *      (free_idx values 0..4); the tree bisects the nodes (KD rule of hm_model_create_op)
 *      with each node's two rows adjacent; levels = floor(log2(n / leaf)).  No selection.
 *      hm_iteration_batched takes univariate fields only;
 *   obs_idx, nobs: the observed grid points, or NULL / nobs = 0 for every point.  With a
 *      selection (host array of nobs distinct grid indices, read during the call; the
 *      observation operator Phi of eq. "projection" reads these nodes, Sec. 5.2.1 forms
 *      its smaller data sets this way) the model is K = sigma2 Phi A^{-1} B^{-1} B^{-T}
 *      A^{-T} Phi^T + tau2 I of dimension nobs: the physics on the full grid, the nugget
 *      on the observations.  Its tree is the KD-tree of the observed nodes' (x, y) grid
 *      positions (as hm_model_create_op), observation order = obs_idx order, leaves padded
 *      (hm_model_rows); each K-apply spreads its columns onto the full grid, applies the
 *      full-grid transforms and reads the observed nodes back.  Needs nobs >= 2 leaf and
 *      the full grid valid for leaf; out-of-range or repeated indices: HM_E_INVAL.
 * Currently nx = ny for dim 2; anything else returns HM_E_INVAL naming what is not
 * supported. */
hm_status hm_model_create_spde(hm_ctx* ctx, int dim, int nx, int ny, double h, int nvars, const int* obs_idx,
                               long long nobs, int leaf, hm_model** out);
/* A model on n scattered points with a caller-supplied operator: K(theta) =
 * sigma2 K_op(theta0, theta1) + tau2 I with theta_full = (theta0, theta1, tau2, sigma2)
 * (tau2 > 0, sigma2 > 0; theta0, theta1 as the operator defines them, finite).
 * coords: host, n x dim row-major (dim 1 or 2).  The tree is the KD-tree of the
 * points (Sec. 5.2): a node's points are split along the longer side of their bounding
 * box (x on ties), the floor(m/2) with the smallest coordinate (ties: the other
 * coordinate, then the point index) going left; points inside a leaf keep increasing
 * index; leaves are stored padded to the largest (hm_model_rows).  levels =
 * floor(log2(n / leaf)).  op and uctx must stay valid while the model lives.  Every
 * other call works on such a model as on the stencil model (sketches, H handles,
 * gradients -- the reverse sweep applies the operator's derivatives --, Fisher). */
hm_status hm_model_create_op(hm_ctx* ctx, int dim, const double* coords, int n, int leaf, hm_op_fn op, void* uctx,
                             hm_model** out);
/* The advection-diffusion-reaction model (Sec. 5.3, eqs. "ad1", "ad2"; latent Matern
 * source, Sec. 5.1 eq. "latent covariance" with the mass lumped) on an N x N grid of
 * the unit square (h = 1/(N+1), Dirichlet, central differences, constant coefficients):
 *   L u = -kd Lap u + (vx, vy) . grad u + c u,   B = kappa^2 I - Lap,
 *   K = sigma2 L^{-1} B^{-2} L^{-T} + tau2 I,   theta_full = (kappa, c, tau2, sigma2)
 * (kappa > 0, c >= 0).  L is not symmetric: the K-apply solves with L and with L^T.
 * The library applies K by direct transforms (a diagonal similarity makes each axis'
 * operator symmetric): accepted while the cell Peclet number |v| h / (2 kd) < 1 and
 * rho^(N-1) stays in [1e-3, 1e3], rho = sqrt((1 - P) / (1 + P)) per axis, P the cell
 * Peclet number with sign; else HM_E_INVAL.  2 <= N <= 1024.  An operator model in
 * every other respect (hm_model_create_op): the tree is the KD-tree of the grid points,
 * kappa and c are the two parameters with derivative matrices. */
hm_status hm_model_create_adr(hm_ctx* ctx, int N, double kd, double vx, double vy, int leaf, hm_model** out);
void hm_model_destroy(hm_model* m);
/* n (grid points), levels, leaf size of the stored layout (the largest leaf). Any pointer may be NULL. */
hm_status hm_model_info(const hm_model* m, int* n, int* levels, int* leaf);
/* Rows of the tree-ordered layout: 2^levels x leaf.  Equal to n when every bisection is
 * even and the leaves hold a multiple of four points; otherwise (odd sides: the left
 * child gets floor(side/2); scattered points) each leaf is stored padded to the largest
 * leaf rounded up to a multiple of four: padding rows are zero in every tree-ordered
 * vector, panel and sample the library writes, identity in the leaf blocks of K~ and
 * zero in those of its derivatives, and are ignored on input.  hm_kapply's X, Y,
 * hm_model_perm and hm_export use this row count. */
hm_status hm_model_rows(const hm_model* m, int* rows);
/* Move all later work of the model (and of its sketches and H handles) to another
 * stream; waits for the work already queued on the old one. */
hm_status hm_model_set_stream(hm_model* m, void* stream);
/* Kernel-variant autotuner (setup time; allocates and frees its own scratch):
 * times the variants of the panel products on launches of this model's shapes for
 * panel width kc (1..64, at most the leaf size): a coarser-level subtraction, the
 * leaf pass's subtraction (leaf-size width), the per-node products of every depth and
 * the Cholesky-QR products over one side of every node.  The variants are the expand's workgroup shape
 * (1: one 16-row block per wavefront, 4 wavefronts; 2: two row blocks, 4 wavefronts;
 * 3: one row block, 8 wavefronts) and the 2- or 4-wavefront row split of the reduce --
 * and keeps the fastest for all later work of the model.  report: host[8] or NULL:
 * expand ms for variants 1, 2, 3; reduce ms with the 4-wavefront split never / below
 * 1024 workgroups / always; the chosen expand variant; the chosen workgroup threshold.
 * HM_E_INVAL for a bad kc; HM_E_NOMEM if the scratch cannot be allocated. */
hm_status hm_model_autotune(hm_model* m, int kc, double* report);
/* Read (set = 0) or write (set = 1) the chosen variants, e.g. to copy one model's
 * tuning to others of the same shape.  expand_variant: 0 (built-in default, variant 1)
 * or 1..3 as above; reduce_split_below: workgroup count below which the reduce uses 4
 * wavefronts.  HM_E_INVAL for NULL pointers or values out of range. */
hm_status hm_model_tuning(hm_model* m, int* expand_variant, long long* reduce_split_below, int set);
/* Copy the tree->grid permutation (rows ints, perm[tree_pos] = grid index, -1 on padding
 * rows) to a host buffer. */
hm_status hm_model_perm(const hm_model* m, int* perm_host);

/* K-apply of the physics model (the only access to K the method uses, Sec. 3.2):
 * Y = op(theta) X with op = K (which=0), dK/dkappa (1), dK/dalpha (2).
 * X, Y: device, rows x c column-major in TREE order (hm_model_rows) with leading
 * dimensions ldx, ldy >= rows; padding rows of X are ignored and those of Y set to zero.
 * Exact direct solves of the Dirichlet stencils (orthonormal sine transforms along x and y). */
hm_status hm_kapply(hm_model* m, const double* theta_full, const double* X, int ldx, int c, double* Y,
                    int ldy, int which);

/* hm_kapply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same operator,
 * arguments, layout and errors as hm_kapply, with the transform scratch taken from
 * one fixed 64 MiB device array per GPU (held until the process ends) instead of the
 * model's workspace; the call allocates and frees nothing.  Columns are processed in
 * blocks of floor(64 MiB / (40 n)) (at most 4096), so n may be at most 1677721:
 * larger models get HM_E_INVAL.  All calls on one GPU share its array: calls that
 * overlap in time on one GPU (other streams or threads) race and must not be issued.
 * The model's stream and device are used; the caller's current device is restored. */
hm_status hm_kapply_noalloc(hm_model* m, const double* theta_full, const double* X, int ldx, int c, double* Y,
                            int ldy, int which);

/* --------------------------------------------------------------- sketch ---
 * hm_sketch_create: fix the test matrices for all later iterations (Sec. 3.3:
 * sampling matrices drawn once and kept fixed).  omega: device, levels x ell x n
 * doubles (omega[((l-1)*ell + j)*n + i] = draw for tree row i, column j, level l),
 * ell = rank + oversample, N(0,1) entries supplied by the caller; only rows of right
 * children at depth l are read; the buffer may be freed after the call.
 * At theta0 each block is sketched with ell columns; the right singular vectors of
 * that sample keep k = min(rank, #{s_i > 1e-10 s_1}) columns (each signed so that
 * its largest-magnitude entry is positive), and Omega_b V becomes the block's fixed
 * k-column test matrix (reading of Alg. 1 step 3 with oversampling).
 * Fails with HM_E_RANK if a whole level has rank 0. */
hm_status hm_sketch_create(hm_model* m, const double* omega, int rank, int oversample,
                           const double* theta0_full, hm_sketch** out);
/* As hm_sketch_create with the truncation tolerance given: each block keeps
 * k = min(rank, #{s_i > rank_tol s_1}) columns, so the ranks adapt per block to a
 * relative accuracy (a tolerance-driven rank, the adaptive strategy of Sec. 3.1 and
 * the paper's concluding remarks); rank stays the cap and sets the panel width when
 * some block reaches it.  hm_sketch_create is rank_tol = 1e-10.  rank_tol in [0, 1),
 * else HM_E_INVAL. */
hm_status hm_sketch_create_tol(hm_model* m, const double* omega, int rank, int oversample, double rank_tol,
                               const double* theta0_full, hm_sketch** out);
void hm_sketch_destroy(hm_sketch* s);
/* kept rank per block: k_host[2^levels - 1], heap order of the block's parent node
 * (root 0; children of node x are 2x+1, 2x+2); *kc = panel width (max kept rank). */
hm_status hm_sketch_ranks(const hm_sketch* s, int* k_host, int* kc);

/* ------------------------------------------------------------------ H ---
 * hm_H_create: allocate K~ and its p derivative matrices for the free parameters
 * free_idx[0..p-1] (indices into theta_full, distinct, p <= 4; p <= 5 for the bivariate model).  All device memory
 * of the iteration is allocated here; build/factor/... allocate nothing. */
hm_status hm_H_create(hm_sketch* s, int p, const int* free_idx, hm_H** out);
void hm_H_destroy(hm_H* H);

/* Build K~(theta) and K~_j(theta) by randomized peeling and its forward-mode
 * derivative (Sec. 3.2-3.3).  theta_full: host[4]; tau2 > 0, kappa > 0, alpha >= 0,
 * sigma2 > 0 required (else HM_E_INVAL). */
hm_status hm_build(hm_H* H, const double* theta_full);
/* Factor K~ = D (I + U^(tau) V^(tau)T) ... (I + U^(1) V^(1)T) (eq. "one way factor", App. C):
 * leaf Cholesky + per-node Woodbury factors.  HM_E_NOT_SPD if K~ is not SPD. */
hm_status hm_factor(hm_H* H);
/* log|K~| (Sylvester's identity over the factors, Sec. 3.1). Host scalar. */
hm_status hm_logdet(hm_H* H, double* out);
/* x = K~^{-1} y (Woodbury, Sec. 3.1) with one step of FP64 refinement against the
 * H-matvec (two under the mixed precision policy), for nrhs right-hand sides at once.
 * y, x: device, n x nrhs column-major with leading dimension ld >= n, natural grid
 * order; x may alias y.  nrhs = 0 does nothing.  Runs on the model's stream without
 * a host synchronisation; no allocation (up to 16 columns per sweep). */
hm_status hm_solve(hm_H* H, const double* y, double* x, long long nrhs, long long ld);
/* L~ (eq. "log-like approximated", including -n/2 log 2pi) and the NLL gradient
 * grad[j] = 1/2 tr(K~^{-1} K~_j) - 1/2 y^T K~^{-1} K~_j K~^{-1} y (= -S~_j,
 * eq. "score approximated").  y: device, grid order.  loglik, grad: host (grad may be NULL). */
hm_status hm_loglik_grad(hm_H* H, const double* y, double* loglik, double* grad);
/* Expected Fisher information I~_ij = 1/2 tr(K~^{-1}K~_i K~^{-1}K~_j)
 * (eq. "fisher info approximated"), exact for the HODLR matrices (App. B).
 * fim: host, p*p row-major (symmetric); each (i,j) is computed independently. */
hm_status hm_fisher(hm_H* H, double* fim);
/* One likelihood iteration: build + factor + logdet + loglik/grad + fisher. */
hm_status hm_iteration(hm_H* H, const double* theta_full, const double* y, double* loglik,
                       double* grad, double* fim);

/* Many independent fields in one call (batched H-MLE iteration): the same work as
 * hm_iteration for every handle hs[f] (each built on its own model), enqueued on
 * each model's stream without host synchronisation and collected at the end, so
 * fields on different streams run concurrently; results equal those of separate
 * hm_iteration calls.  thetas: host, nf x 4 row-major; ys[f]: device sample of
 * field f (grid order); loglik: host[nf]; grad: host, the fields' p_f entries
 * concatenated (or NULL); fim: host, the p_f x p_f blocks concatenated (or NULL).
 * A handle may appear once.  On failure the message names the first failing field. */
hm_status hm_iteration_batched(int nf, hm_H* const* hs, const double* thetas, const double* const* ys,
                               double* loglik, double* grad, double* fim);

/* Precision policy of H (the paper computes in double; this is a reading of where
 * lower precision may enter).  0 = FP64 throughout (default).  1 = mixed: the panel
 * products of the coarser-level subtraction, of the Woodbury panel updates, of the
 * solve sweep and of the trace / Fisher terms run as FP32 MFMA with FP32
 * accumulation (operands rounded from the FP64 storage); the K-apply, QR and Alg. 2,
 * leaf Cholesky and inverse, per-node factors, the log-determinant sum, the solve's
 * refinement residuals (FP64 H-matvec, two steps) and every scalar reduction stay
 * FP64.  2 = mixed with BF16 trace panels: as 1, and the panel products of the score
 * and Fisher traces (parameter preparation, tangent sweeps, panel products) take BF16
 * operands (rounded to nearest even) with FP32 accumulation; L~ is that of policy 1.
 * Invalidates the current factors (state returns to empty). */
hm_status hm_H_set_precision(hm_H* H, int precision);

/* L~ and the NLL gradient for the free parameters by reverse mode (adjoint):
 * builds K~(theta) only (no derivative matrices), factors it, and runs the
 * construction backwards with the sketches held fixed (Sec. 3.3), so grad is the
 * gradient of the same smooth L~(theta) that hm_loglik_grad differentiates
 * forward (eq. "score approximated") -- equal up to rounding -- at a cost that
 * does not grow with the number of parameters.  The test matrices of each level are
 * recomputed from the stored panels and the fixed sketch, not stored.
 * theta_full: host[4]; y: device, n doubles, grid order; loglik: host; grad: host[p]
 * or NULL (then only L~).  Leaves H factored at theta without derivative matrices:
 * hm_loglik_grad with grad and hm_fisher then return HM_E_STATE until hm_build. */
hm_status hm_loglik_grad_adjoint(hm_H* H, const double* theta_full, const double* y, double* loglik,
                                 double* grad);
/* The two halves of hm_loglik_grad_adjoint, for a forward / backward split (e.g. an
 * autograd function whose forward pass must not pay for the gradient):
 * hm_loglik builds K~(theta) only (no derivative matrices), factors it and returns L~
 * (eq. "log-like approximated"), keeping z = K~^{-1} y; hm_grad_reverse then runs the
 * reverse sweep for that construction and y and returns grad[p] (the NLL gradient of
 * the same L~).  hm_grad_reverse returns HM_E_STATE unless the last construction of H
 * was followed by an evaluation of L~ (hm_loglik, hm_loglik_grad or hm_iteration). */
hm_status hm_loglik(hm_H* H, const double* theta_full, const double* y, double* loglik);
hm_status hm_grad_reverse(hm_H* H, double* grad);

/* Export the representation for inspection (tests):
 * what=0: panel set of K~, n x (levels*kc), rows in tree order;
 * what=1+j: panel tangents of K~_j for the j-th free parameter that needs a
 *           derivative sketch (kappa, alpha), same shape;
 * what=10: leaf blocks of K~, leaves x nl x nl (leaf-major, column-major);
 * what=11+j: leaf blocks of K~_j (real parameters), same shape.
 * dst: device buffer of sufficient size. */
hm_status hm_export(hm_H* H, int what, double* dst);

/* ----------------------------------------------------------------- stats ---
 * Work counters and per-phase device time of one H handle since its creation or the
 * last hm_stats_reset (the instrumentation of the measured path): the K-apply column
 * counts are those of the handle's model (all its sketches and H handles); phase times
 * are HIP-event times of the enqueued work of each phase on the model's stream (build:
 * construction of K~ and K~_j; factor: factorisation and log-determinant; loglik: solve,
 * quadratic forms and the forward-mode traces of the gradient; fisher: the Fisher
 * terms; reverse: the adjoint sweep; solve: hm_solve).  hm_stats synchronises the
 * stream and copies min(bytes, sizeof(hm_stats_t)) bytes to out (host). */
typedef struct {
  long long kapply_calls;
  long long kapply_columns;        /* columns of K applied */
  long long kapply_deriv_columns;  /* columns of dK/dkappa and dK/dalpha applied */
  long long builds;                /* constructions of K~ */
  long long deriv_builds;          /*   of which with the derivative matrices K~_j */
  long long factors;
  long long loglik_evals;
  long long grad_evals;            /* forward-mode gradients */
  long long reverse_sweeps;        /* reverse-mode (adjoint) gradients */
  long long fisher_evals;
  long long solve_rhs;             /* right-hand sides solved by hm_solve */
  double ms_build, ms_factor, ms_loglik, ms_fisher, ms_reverse, ms_solve;
  long long device_bytes;          /* device memory held by the H handle */
} hm_stats_t;
hm_status hm_stats(hm_H* H, void* out, size_t bytes);
hm_status hm_stats_reset(hm_H* H);

/* ------------------------------------------------------------- profiling ---
 * Roofline instrumentation.  hm_profile_enable(m, family) brackets every later
 * launch of one kernel family with HIP events on the model's stream and records
 * the launch's algorithmic flop and byte counts (the useful work of the launch,
 * not tile padding).  family: 0 panel expand (Y += A T over the tree), 1 panel
 * reduce (A^T X per node), 2 sine-transform passes of the K-apply, 4 leaf-block
 * GEMM; -1 switches profiling off.  Enabling clears earlier records.
 * hm_profile_read synchronises the stream and returns the totals since enabling:
 * summed event time (ms), number of launches, flops and bytes (any pointer may be NULL). */
hm_status hm_profile_enable(hm_model* m, int family);
hm_status hm_profile_read(hm_model* m, double* ms, long long* launches, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* HMLE_H */
