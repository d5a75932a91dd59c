/*
 * fcm.h -- C-ABI of libfcm: multigrid-preconditioned CG for finite cell
 * method (FCM) systems on one AMD Instinct MI355X (gfx950).
 *
 * What is solved (Section 2.1, eq. weakform): find u_h in the span of an
 * integrated-Legendre tensor-product basis of order p on a uniform Cartesian
 * grid that embeds the physical domain, with
 *     a(u,v) = int alpha(x) (B v)^T C (B u) dOmega
 *     b(v)   = int alpha(x) (N v)^T f dOmega + int (N v)^T t dGamma_N
 * where alpha = 1 in the physical domain and alpha = eps << 1 in the
 * fictitious part.  Poisson (one field, C = kappa I) or isotropic linear
 * elasticity (dim fields).  Cut cells are integrated by recursive bisection
 * (quadtree/octree, Section 4.3.1) with a (p+1)^d Gauss rule per leaf.
 * Homogeneous Dirichlet conditions are imposed strongly on grid-aligned box
 * faces; elements entirely outside the physical domain are dropped.
 *
 * How it is solved (Section 3): hierarchical p-multigrid.  Level l holds the
 * basis functions of degree <= l+1 (eq. hierarchicalFunctions), so the level
 * vector is a prefix of the fine vector, restriction keeps the prefix and
 * prolongation zero-extends it (eq. restrictionoperation), and the level
 * matrix is the leading principal block of the fine one (eq.
 * hierarchicalMatrices).  Levels >= 1 are smoothed by additive Schwarz (eq.
 * AdditiveSchwarz) with relaxation omega, over element blocks or over patch
 * blocks (the basis functions nonzero on the kept elements around one grid
 * node, Section 3.3.1); level 0 (p = 1) is solved exactly.  One V-cycle
 * (Alg. 1) preconditions an FP64 CG (Section 4).
 *
 * Vectors.  All device vectors use the library's padded "plane" layout: the
 * vector of level l is nplanes(l) contiguous planes of G grid points each
 * (G = prod_ax (n_ax + 1), axis 0 fastest).  A plane holds one slot type
 * (vertex or bubble degree per axis) of one field component; planes are
 * sorted by polynomial degree, so level l is a prefix.  Entries that are not
 * DOFs (Dirichlet, padding, support only on dropped elements) are zero on
 * input and are written as zero.  fcm_dof_keys() maps every entry to a
 * canonical entity key (or -1) so results can be compared with any other
 * numbering.
 *
 * Memory ownership.  The handle owns every device allocation it makes (level
 * operators, Schwarz inverses, coarse factors, work vectors); they come from
 * the device's stream-ordered pool (see fcm_trim_pool).  Pointers passed
 * in (device vectors, host arrays) remain owned by the caller; the library
 * never frees or retains them beyond the call.  Device vectors must be
 * hipMalloc'ed (or torch-allocated) memory on the handle's device.
 *
 * Streams.  Every call that takes `stream` (a hipStream_t passed as void*,
 * NULL = default stream) enqueues its work on that stream.  Calls that return
 * host data synchronise that stream first.
 *
 * Errors.  A negative status means the call failed and produced no result;
 * fcm_last_error() returns a thread-local description.  Positive statuses are
 * warnings with a valid result (FCM_NOT_CONVERGED returns the last iterate).
 * Handles are not thread-safe; a server is safe for concurrent submit/poll.
 */
#ifndef FCM_H
#define FCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCM_OK = 0,
  FCM_NOT_CONVERGED = 1,
  FCM_ERR_ARG = -1,
  FCM_ERR_OOM = -2,
  FCM_ERR_HIP = -3,
  FCM_ERR_NOT_SPD = -4,
  FCM_ERR_BREAKDOWN = -5,
  FCM_ERR_NAN = -6,
  FCM_ERR_BUSY = -7
} fcm_status;

/* Physical domain: the box minus balls, the interior of one ball, (2D,
 * Section 4.1) the square of side ball_r[0] centred at ball_c[0] and rotated
 * by psi (counter-clockwise) about its centre, or (3D, Section 4.3) the
 * popcorn phi(x) = |x| - 0.6 - sum_k 3 exp(-|x - x_k|^2 / 0.04) <= 0 with the
 * paper's twelve centres x_k.  The popcorn problem carries its prescribed
 * solution u = x^3 + x y^2 + y^3 + z^4 + sin(3 (x^2 + y^2)): the source gets
 * -Lap u added, and with beta > 0 the penalty imposes u on phi = 0 with the
 * surface rule surf_n along rays from the origin.                          */
enum { FCM_GEOM_BOX_MINUS_BALLS = 0, FCM_GEOM_BALL_INTERIOR = 1, FCM_GEOM_SQUARE = 2,
       FCM_GEOM_POPCORN = 3 };
/* Element basis: the tensor-product integrated Legendre space, or its trunk
 * subspace (Table tab::upperbound, trunk column): the products whose bubble
 * factors' degrees sum to at most p; level q of the p-hierarchy holds the
 * modes whose sum (at least 1) is at most q.                               */
enum { FCM_SPACE_TENSOR = 0, FCM_SPACE_TRUNK = 1 };
/* V-cycle precision.  FCM_MIXED streams FP32 copies of the Schwarz inverses
 * (those whose Jacobi-scaled condition number is at most 1e5) and forms the
 * patch class products on the FP32 matrix cores; level vectors, residuals,
 * the coarse solve and the outer CG stay FP64.                              */
enum { FCM_FP64 = 0, FCM_MIXED = 1 };
enum { FCM_SMOOTH_ELEMENTWISE = 0, FCM_SMOOTH_PATCHWISE = 1 };  /* Schwarz blocks */
/* Solve on the p = 1 level: FCM_COARSE_BLOCKTRI factorises it exactly
 * (block LDL^T over layers of grid points); FCM_COARSE_HMG coarsens it
 * further by geometric h-levels (remark closing Section 3.2): d-linear
 * interpolation, Galerkin matrices P^T A P, patchwise additive Schwarz on
 * every h-level, a dense inverse on the coarsest.                          */
enum { FCM_COARSE_BLOCKTRI = 0, FCM_COARSE_HMG = 1 };

typedef struct fcm_handle fcm_handle;
typedef struct fcm_server fcm_server;

/* Problem statement (Section 2.1).  All pointers are host memory, read during
 * the call only.  Unused trailing axes of 3-vectors are ignored when dim = 2. */
typedef struct {
  int dim;                    /* 2 or 3                                          */
  int n[3];                   /* cells per axis, >= 1                            */
  double lo[3], hi[3];        /* embedding box                                   */
  int p;                      /* polynomial order, 1..6                          */
  int n_fields;               /* 1 (Poisson) or dim (linear elasticity)          */
  int refine_levels;          /* multi-level hp depth K (Section 2.2): elements cut
                                 by the sphere are bisected recursively K times;
                                 K > 0 needs Poisson, one ball and patchwise
                                 blocks (all functions on the base elements
                                 around a base node, Section 3.3.1)            */
  int geom;                   /* FCM_GEOM_*                                      */
  int n_balls;                /* holes (BOX_MINUS_BALLS) or 1 (BALL_INTERIOR)    */
  const double *ball_c;       /* [n_balls][dim] centres                          */
  const double *ball_r;       /* [n_balls] radii                                 */
  double alpha;               /* fictitious-domain scaling eps, 0 < eps <= 1     */
  int quad_depth;             /* sub-cell bisection depth for cut cells, 0..4    */
  double kappa;               /* Poisson conductivity                            */
  double E, nu;               /* elasticity                                      */
  unsigned dirichlet_faces;   /* bit 2*axis+side: u = 0 on that box face         */
  int n_traction;             /* Neumann tractions on box faces                  */
  const int *traction_face;   /* [n_traction] face bit index 2*axis+side         */
  const double *traction_vec; /* [n_traction][3] traction vector                 */
  int n_gauss;                /* Gaussian sources f += A exp(-|x-c|^2/w^2)       */
  const double *gauss;        /* [n_gauss][5]: A, w, c_x, c_y, c_z               */
  double f_const;             /* constant scalar source                          */
  double body_force[3];       /* constant body force (elasticity)                */
  double beta;                /* penalty of the Dirichlet condition on an immersed
                                 boundary (eq. weakform): u = 0 on the sphere
                                 (refine_levels > 0, BALL_INTERIOR) or u = g on
                                 the edges of the square (FCM_GEOM_SQUARE, g
                                 from trig_dir) or u = the prescribed solution
                                 on the popcorn surface; 0 = none              */
  int surf_n[2];              /* surface rule of the penalty (sphere, popcorn):
                                 Gauss-Legendre points in cos(theta) (<= 4096)
                                 and trapezoid points in phi (<= 8192; 2D: phi
                                 only); 0 = 256 x 512                            */
  int space;                  /* FCM_SPACE_TENSOR or FCM_SPACE_TRUNK (uniform
                                 grids only)                                   */
  double psi;                 /* FCM_GEOM_SQUARE: rotation in radians            */
  double trig_src[2];         /* source += A cos(a x') sin(a y') with (A, a) =
                                 trig_src, (x', y') the square's frame (origin
                                 at its centre, axes along its edges); A = 0:
                                 none; FCM_GEOM_SQUARE only                    */
  double trig_dir[2];         /* Dirichlet data g = A cos(a x') sin(a y') on the
                                 square's edges, (A, a) = trig_dir             */
} fcm_problem;

/* Solver options (Sections 3.3.2 and 4). */
typedef struct {
  int smoother;               /* FCM_SMOOTH_ELEMENTWISE: one block per kept element,
                                 all functions nonzero on it; FCM_SMOOTH_PATCHWISE:
                                 one block per grid node, all functions nonzero on
                                 the kept elements sharing it (Section 3.3.1); the
                                 patch size n_f (2p+1)^d must not exceed 2187     */
  double omega;               /* relaxation (Section 3.3.2): elementwise 1/3 (2D),
                                 2/15 (3D); patchwise 1/6 (2D), 1/18 (3D)         */
  int n_pre, n_post;          /* smoothing steps per level (5 and 5 in the paper) */
  int precision;              /* FCM_FP64 or FCM_MIXED (FP32 smoother matrices)  */
  double rtol;                /* ||r||/||b|| stopping tolerance                  */
  int max_iter;               /* CG iteration cap (500 in the paper)             */
  int use_graphs;             /* 1: replay each CG iteration as a captured HIP
                                 graph on a library-owned stream (0: eager)     */
  int autotune;               /* 1: at setup, time the launch variants of the
                                 patchwise smoother on this problem's data and
                                 keep the fastest (cached per problem shape in
                                 the process); 0: fixed heuristics            */
  int coarse;                 /* FCM_COARSE_BLOCKTRI or FCM_COARSE_HMG (uniform
                                 grids only)                                   */
  int coarse_dense_max;       /* HMG: an h-level with at most this many DOFs is
                                 the coarsest (solved by a dense inverse);
                                 0 = 2048, at most 8192                        */
} fcm_options;

typedef struct {
  int iterations;             /* CG iterations (x updates)                       */
  double rel_res;             /* recursive ||r||/||b|| at exit                   */
  double true_rel_res;        /* ||b - A x|| / ||b|| recomputed at exit (FP64)   */
  double t_setup_ms;          /* fcm_setup wall time                             */
  double t_solve_ms;          /* this solve's wall time                          */
  const double *res_history;  /* [n_history] relative residuals, owned by handle */
  int n_history;
} fcm_solve_info;

/* Build the discretisation and the whole multigrid hierarchy on the device:
 * cell classification, cut-cell integration, RHS, Schwarz block inverses
 * (elementwise or patchwise) for every level >= 1 and the exact factorisation
 * of level 0.
 * On success *out owns all device memory.  Errors: FCM_ERR_ARG (invalid
 * problem/options), FCM_ERR_OOM, FCM_ERR_HIP, FCM_ERR_NOT_SPD (a Schwarz block
 * or the coarse matrix lost positive definiteness in FP64).                 */
fcm_status fcm_setup(const fcm_problem *prob, const fcm_options *opts,
                     void *stream, fcm_handle **out);

/* Level count and sizes, coarse first: n_dofs[l] = number of unknowns,
 * n_padded[l] = length of the level vector in the padded plane layout.
 * Either array may be NULL; each must hold *n_levels entries (<= 8).        */
fcm_status fcm_sizes(const fcm_handle *h, int *n_levels, int64_t *n_dofs,
                     int64_t *n_padded);

/* Copy the assembled right-hand side b (fine level, FP64) to b_dev.         */
fcm_status fcm_rhs(fcm_handle *h, double *b_dev, void *stream);

/* y = A_l x (FP64) on level l (eq. hierarchicalMatrices); x, y level-l vectors.
 * With FCM_COARSE_HMG, level = -k (k >= 1) applies the Galerkin matrix of
 * h-level k to vectors of n_f (n_k+1)^d entries (fcm_hlevels).              */
fcm_status fcm_apply(fcm_handle *h, int level, const double *x, double *y,
                     void *stream);

/* z = M_l^{-1} r (FP64), the additive Schwarz operator of level l >= 1 (eq.
 * AdditiveSchwarz) with the handle's blocks (elementwise or patchwise), in
 * FP64 arithmetic from the FP64 inverses, without the relaxation factor.
 * With FCM_COARSE_HMG, level = 0 and level = -k give the patchwise operator
 * of h-level 0 (the p = 1 level) and h-level k (not the coarsest).          */
fcm_status fcm_smooth(fcm_handle *h, int level, const double *r, double *z,
                      void *stream);

/* Geometric h-levels of a handle set up with FCM_COARSE_HMG: *count = number
 * of h-levels J+1 (h-level 0 = the p = 1 level, J the coarsest), 0 without
 * them; cells (may be NULL, room for 3 * 12 ints) receives the cells per axis
 * of each (1 on unused axes).  A level-k vector holds n_f planes of
 * (n_0+1)(n_1+1)(n_2+1) grid points, axis 0 fastest, zero where no DOF is. */
fcm_status fcm_hlevels(const fcm_handle *h, int *count, int *cells);

/* Test hook for the batched SPD inversion used by the Schwarz blocks and the
 * coarse factorisation: A_dev (device, `batch` row-major n x n FP64 SPD
 * matrices, contiguous) is overwritten by the inverses, computed on `stream`
 * by the Jacobi-scaled Gauss-Jordan sweep.  The matrices must be exactly
 * symmetric: for n > 384 and batch >= 8 the sweep works on the upper
 * triangle only (the inverse is returned in full).  kappa_dev (device, may
 * be NULL) receives ||A_s||_1 ||A_s^{-1}||_1 of each Jacobi-scaled matrix.
 * Returns FCM_ERR_NOT_SPD if a pivot was not positive.  Synchronises the
 * stream.                                                                   */
fcm_status fcm_spd_inverse(double *A_dev, int n, int batch, double *kappa_dev,
                           void *stream);

/* fcm_spd_inverse for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results, but the sweep's scratch and pivot flag
 * live in a static device buffer of 4 Mi doubles (32 MiB) that each GPU the
 * library runs on holds until the process ends; no hipMalloc, hipFree or
 * allocating library call is made.  Needs 385*n + 2 doubles per matrix
 * (at most 4,194,272 in total); larger requests return FCM_ERR_ARG with
 * nothing launched.  Calls on one GPU share its buffer: calls that overlap on
 * one GPU (several streams or threads) race and must be serialised by the
 * caller.  Synchronises the stream; FCM_ERR_NOT_SPD as fcm_spd_inverse.    */
fcm_status fcm_spd_inverse_noalloc(double *A_dev, int n, int batch, double *kappa_dev,
                                   void *stream);

/* x = A_0^{-1} b on the coarsest level (exact FP64 solve); with
 * FCM_COARSE_HMG, x = one h-cycle applied to b (its approximation).         */
fcm_status fcm_coarse_solve(fcm_handle *h, const double *b, double *x,
                            void *stream);

/* z = V(0, r): one V-cycle of Alg. 1 on the fine level with zero initial
 * guess, in the handle's precision (FCM_MIXED: FP32 smoother matrices).
 * r and z are fine-level FP64 vectors.                                      */
fcm_status fcm_vcycle(fcm_handle *h, const double *r_dev, double *z_dev,
                      void *stream);

/* CG preconditioned by one V-cycle (Section 4).  b_dev = NULL uses the
 * assembled right-hand side.  x_dev receives the solution (x0 = 0).  Stops
 * when ||r||/||b|| < rtol or after max_iter iterations (FCM_NOT_CONVERGED).
 * info may be NULL.  Synchronises the stream before returning.             */
fcm_status fcm_pcg_solve(fcm_handle *h, const double *b_dev, double *x_dev,
                         fcm_solve_info *info, void *stream);

/* Batched MG-PCG (systems batching, not in the paper): solves the n problems
 * of the handles hs[0..n-1] (sizes, orders and dimensions may differ;
 * uniform grids only), each with its assembled right-hand side, into x_dev[i]
 * (caller-owned device vectors of the handle's fine-level padded length).
 * After every problem's first iteration, each CG step of all unfinished
 * problems is ONE hipGraphLaunch of a graph holding their iterations as
 * independent branches (captured with each problem on its own stream); the
 * graph is captured again when a problem finishes.  Per problem the
 * arithmetic is that of fcm_pcg_solve (same kernels in the same order:
 * identical iterates).  infos[i] (may be NULL) as fcm_pcg_solve with
 * t_solve_ms = the batch's wall time; status[i] (may be NULL) each problem's
 * status.  Returns the worst status (a negative one, else FCM_NOT_CONVERGED
 * if any, else FCM_OK); a handle that is null, multi-level or repeated is
 * FCM_ERR_ARG with nothing launched.  Synchronises the handles' streams.   */
fcm_status fcm_pcg_solve_batched(fcm_handle *const *hs, int n, double *const *x_dev,
                                 fcm_solve_info *infos, fcm_status *status, void *stream);

/* The V-cycle as a stand-alone solver: x <- x + V(b - A x) (Section 4,
 * eq. contraction).  *rho_max receives the largest contraction number.     */
fcm_status fcm_mg_solve(fcm_handle *h, const double *b_dev, double *x_dev,
                        fcm_solve_info *info, double *rho_max, void *stream);

/* Canonical entity key of every fine-level padded entry (host array of
 * n_padded[fine] int64), -1 for entries that are not DOFs.  Key:
 *   code_ax = i*p (vertex at node i) or i*p + j - 1 (degree-j bubble, cell i)
 *   key = code_0 + S_0*(code_1 + S_1*(code_2 + S_2*component)),
 *   S_ax = (n_ax + 1)*p.                                                    */
fcm_status fcm_dof_keys(const fcm_handle *h, int64_t *keys);

/* Local mode table of the element matrices: for each of the m local modes
 * (degree-sorted), 4 ints: a_0, a_1, a_2, component, where a_ax = 0 (left
 * vertex), 1 (right vertex) or j >= 2 (degree-j bubble).  *m receives m.    */
fcm_status fcm_local_modes(const fcm_handle *h, int *m, int *modes);

/* Element data for element linear index e (axis 0 fastest): *state = 0 void,
 * 1 uncut, 2 cut; K (host, m*m, row-major, may be NULL) and be (host, m, may
 * be NULL) receive the element stiffness and load in the local mode order.  */
fcm_status fcm_element(const fcm_handle *h, int64_t e, int *state, double *K,
                       double *be);

/* Counts for reporting: number of cut elements, kept elements, unique
 * Schwarz blocks per level >= 1, shared classes, bytes of device memory.   */
typedef struct {
  int64_t n_elements, n_kept, n_cut, n_unique_blocks, n_shared_classes;
  int64_t device_bytes;
  int coarse_blocks, coarse_block_size;  /* layer blocks of the exact coarse
                                 factorisation and their size; with
                                 FCM_COARSE_HMG: h-levels below p = 1 and the
                                 DOFs of the coarsest                         */
  int64_t n_fp64_blocks;      /* unique Schwarz blocks applied in FP64 (mixed)   */
} fcm_stats;
fcm_status fcm_get_stats(const fcm_handle *h, fcm_stats *s);

/* Launch variants of the patchwise smoother of level l >= 1 (set at setup by
 * the autotuner, or by the heuristics when options.autotune = 0):
 * class_rows = rows of the class inverse per workgroup of the class-product
 * kernel divided by 128 (1, 2 or 3; mixed form, blocks above 32), gemv_band =
 * 1 when the unique-patch inverses are streamed by band pairs, 0 one
 * workgroup per patch.  fcm_set_tuning overrides them (0 < class_rows <= 3,
 * gemv_band 0 or 1; band pairs are the only kernel above 384 unknowns; -1
 * keeps a value); every variant computes the same products (class rows:
 * identical bits; band pairs: the row sums in another order).               */
fcm_status fcm_get_tuning(const fcm_handle *h, int level, int *class_rows, int *gemv_band,
                          double *tune_ms);
fcm_status fcm_set_tuning(fcm_handle *h, int level, int class_rows, int gemv_band);

/* Benchmark hook: launch one operator of the solve `reps` times between two
 * HIP events recorded on `stream` and report the average time per launch and
 * the algorithmic bytes one launch must move (inputs read once, outputs
 * written once, matrices streamed once).
 * op: FCM_OP_SMOOTH (Schwarz smoother of `level`, handle precision),
 *     FCM_OP_RESIDUAL (residual update r -= omega A delta of `level`),
 *     FCM_OP_COARSE (one coarse solve or h-cycle), FCM_OP_VCYCLE (one V-cycle,
 *     bytes = sum over its launches), FCM_OP_SMOOTH_STORED (patchwise only:
 *     the kernel that streams the unique patch inverses of `level`, alone).  Work vectors of the handle are used;
 * their contents are overwritten.                                          */
enum { FCM_OP_SMOOTH = 0, FCM_OP_RESIDUAL = 1, FCM_OP_COARSE = 2, FCM_OP_VCYCLE = 3,
       FCM_OP_SMOOTH_STORED = 4 };
fcm_status fcm_time_op(fcm_handle *h, int op, int level, int reps, void *stream,
                       double *ms_per_launch, double *bytes_per_launch);

/* Releases every device allocation of the handle.  The memory is returned
 * to the device's stream-ordered pool in stream order after the work queued
 * on the stream given to fcm_setup(); work the caller queued with this
 * handle on any other stream must have completed (synchronise it first).
 * A handle that held more than an eighth of the device's memory waits for
 * its stream and then trims the current device's pool (as fcm_trim_pool),
 * since the next large setup could not reuse blocks cut to its sizes.
 * NULL is ignored.                                                          */
void fcm_destroy(fcm_handle *h);

/* The library allocates device memory from the current device's default
 * stream-ordered memory pool (hipMallocAsync), which keeps released memory
 * cached for the next setup instead of returning it, so that setups and
 * teardowns never synchronise the whole device.  This call returns the
 * cached, unused memory of the current device's pool to the system.        */
fcm_status fcm_trim_pool(void);

/* ---------------------------------------------------------------------------
 * Serving: a request loop that admits solves of different grids and orders
 * by device-memory footprint, keeps their hierarchies resident and advances
 * all admitted solves together, one CG iteration per tick (continuous
 * batching: requests join and leave between ticks).                        */
typedef struct {
  int64_t memory_budget_bytes;  /* admit while resident footprint fits        */
  int max_active;               /* batch slots                                */
  int n_streams;                /* device streams the ticks spread over       */
} fcm_server_opts;

fcm_status fcm_server_create(const fcm_server_opts *o, fcm_server **out);
/* Copies *prob and *opts; returns a request id.                            */
fcm_status fcm_serve_submit(fcm_server *s, const fcm_problem *prob,
                            const fcm_options *opts, uint64_t *req_id);
/* *done = 1 when finished.  x_host (may be NULL) receives the fine-level
 * padded solution (n_padded doubles); info receives the solve record with
 * t_setup_ms/t_solve_ms, and latency_ms (submit to done).  Returns the
 * request's own status once done.                                          */
fcm_status fcm_serve_poll(fcm_server *s, uint64_t req_id, int *done,
                          double *x_host, int64_t x_len, fcm_solve_info *info,
                          double *latency_ms);
fcm_status fcm_server_destroy(fcm_server *s);

const char *fcm_status_string(fcm_status s);
const char *fcm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FCM_H */
