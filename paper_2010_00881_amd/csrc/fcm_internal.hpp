// Internal declarations of libfcm (not part of the C-ABI).
//
// Data layout in device memory (gfx950, HBM3E):
//  * Grid: G = prod (n_ax + 1) points, axis 0 fastest.  Element e has the
//    same multi-index as its lowest grid point.
//  * Vectors: padded planes.  A plane is one slot type T = (t_0..t_{d-1})
//    (t = 0 vertex, t = j-1 for the degree-j bubble) and one component; plane
//    P occupies [P*G, (P+1)*G).  Planes are sorted by max degree, so the
//    level-q vector (degree <= q) is the prefix of nf*q^d planes.
//  * Element matrices: m_p x m_p row-major in a degree-sorted local mode
//    order; the level-q matrix is the leading m_q x m_q block (ld = m_p).
//  * Schwarz inverses of level q: m_q x m_q row-major, shared classes first
//    (translation-invariant blocks away from cuts), then unique blocks.
//  * Coarse level (q = 1, vertex planes): split along the slowest axis into
//    blocks of w grid layers; dense inverses of the block Schur complements.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fcm.h"

namespace fcm {

constexpr int kMaxP = 6;
constexpr int kMaxLevels = 8;
constexpr int kMaxDepth = 4;
constexpr double kKappa64 = 1e5; // scaled kappa_1 above which a Schwarz block stays FP64
constexpr int kSmallInv = 88;
// Schwarz blocks up to kSmallInv are formed and inverted in LDS (<= 64 KB).
constexpr int kMaxStoredIn = 1029; // largest element matrix (p = 6 elasticity: 3*7^3)
constexpr int kMaxPatchM = 2187;   // largest patchwise Schwarz block (n_f (2p+1)^d: 3D
                                   // elasticity at p = 4)
constexpr int kSmallPatchM = 384;  // blocks up to this size: one workgroup per unique patch

enum : uint8_t { kVoid = 0, kPhys = 1, kCut = 2 };

// Geometry and discretisation constants, passed to kernels by value.
struct Geo {
  int d, nf, p;
  int n[3];      // cells per axis (1 for unused axes)
  int gn[3];     // grid points per axis (1 for unused axes)
  int G;         // grid points
  int E;         // elements
  double lo[3], h[3];
  unsigned dir;  // Dirichlet face bits
  int geom, nballs;
  double alpha;
  int depth;
  int trunk;     // 1: trunk-space basis (FCM_SPACE_TRUNK)
  double sq[5];  // FCM_GEOM_SQUARE: centre x, y, half side, cos psi, sin psi
  double trig[2];  // source A cos(a x') sin(a y'): A, a (A = 0: none)
};

// Per-level Schwarz data and work vectors.
struct Level {
  int q = 0, m = 0, nP = 0;
  int mpatch = 0;              // patchwise block size n_f (2q+1)^d
  int64_t npad = 0, ndofs = 0;
  double *invS64 = nullptr, *invU64 = nullptr;
  float *invS32 = nullptr, *invU32 = nullptr;
  uint8_t *hi64 = nullptr;     // unique blocks applied from FP64 copies in the mixed form
  int n_hi64 = 0;
  int ldp = 0;                 // patchwise: leading dimension of the stored inverses
  int class_rows = 0;          // patchwise launch variants (autotuner): class-product rows
  int gemv_band = 0;           //   per workgroup / 128, unique GEMV by band pairs
  double tune_ms = 0.0;        //   (time the autotuner spent on this level)
  int *units = nullptr;        // owner-kernel work units of this level
  int nunits = 0;
  double *x64 = nullptr, *r64 = nullptr, *d64 = nullptr;
};

struct Coarse {
  int w = 1;          // grid layers per block
  int nblk = 0;       // number of blocks
  int layer0 = 0;     // first grid layer of block 0
  int PP = 0;         // points per layer
  int nb = 0;         // block size = nf * w * PP
  int no = 0;         // in-layer stencil offsets (3^{d-1})
  double *Sinv = nullptr;           // [nblk][nb][nb] inverted Schur complements S_k^{-1}
  double *Gm = nullptr;             // [nblk][nb][nb] G_k = S_k^{-1} B_k   (k >= 1)
  double *Fm = nullptr;             // [nblk][nb][nb] F_k = S_k^{-1} B_{k+1}^T (k < nblk-1)
  double *Dst = nullptr;            // [nblk*nb][3][no][nf] stencil rows (slow offsets -1, 0, +1)
  double *xb = nullptr, *bb = nullptr;  // FP64 coarse vectors (used by the FP32 V-cycle)
  double *xblk = nullptr, *bblk = nullptr;  // [nblk][nb] block-layout sweep vectors
};

// Geometric h-levels below the p = 1 level (hlevels.hip).  h-level 0 is the
// p = 1 level itself (its vectors are the level-0 vectors of the p-hierarchy:
// n_f vertex planes of G points); h-level k+1 has ceil(n_k / 2) cells per
// axis and the Galerkin matrix P^T A_k P of the d-linear interpolation P.
// Every h-level's matrix is held as a 3^d-point stencil per row, vectors as
// n_f planes of its grid points (axis 0 fastest), absent DOFs zero.
constexpr int kMaxH = 12;
struct HLev {
  int n[3] = {1, 1, 1}, gn[3] = {1, 1, 1};   // cells and grid points per axis
  int64_t G = 1, len = 0;                    // points, vector length n_f G
  int ndof = 0;                              // DOFs (present entries)
  int *pres = nullptr;                       // [len] 1 = DOF
  double *S = nullptr;                       // [len][3^d][n_f] stencil rows
  int np = 0;                                // Schwarz patches (nodes with a kept cell)
  int *pidx = nullptr;                       // [G] patch of a node, -1 none
  int *pmem = nullptr;                       // [np][m] vector index of patch slot, -1 none
  double *Binv = nullptr;                    // [np][m][m] patch inverses
  double *Y = nullptr;                       // [np][m] patch products
  double *x = nullptr, *b = nullptr;         // level vectors (level 0: the p-level's)
  double *r = nullptr, *dl = nullptr, *e = nullptr;
};
struct HMG {
  int J = 0;                                 // coarsest h-level (exact dense solve)
  int m = 0;                                 // patch slots n_f 3^d
  HLev lev[kMaxH];
  int nd = 0;                                // DOFs of the coarsest level
  int *didx = nullptr;                       // [nd] their vector indices
  double *Ainv = nullptr;                    // [nd][nd] inverse of the coarsest matrix
  double *scr = nullptr;                     // setup scratch (SPD inverse)
  size_t scr_doubles = 0;
};

struct Problem {
  fcm_problem pr;
  std::vector<double> ball;    // [nballs][4]: cx, cy, cz, r
  std::vector<double> gsrc;    // [ngauss][5]
  std::vector<int> tface;
  std::vector<double> tvec;
};

// Device tables shared by the kernels.
struct Tables {
  int m = 0, ms = 0, nP = 0;
  int *lm = nullptr;        // [m][4] local modes a0,a1,a2,c (degree-sorted)
  int *xoff = nullptr;      // [m] plane(b)*G + grid offset of mode b
  int *rows = nullptr;      // [nP][8] local row of plane P in element g - delta(s), or -1
  int *pinfo = nullptr;     // [nP] bit0..2 vertex axes, bits 8..10 bubble axes
  int *smap = nullptr;      // [ms*nf] local index of (scalar tuple s, comp c)
  double *tab1d = nullptr;  // [nint][3][(p+1)^2] 1D sub-interval matrices M1, K1, D1
  double *gxw = nullptr;    // [2][p+1] Gauss nodes and weights on [-1,1]
  double *vgauss = nullptr; // [p+1][p+1] mode values at the Gauss nodes
  double *ball = nullptr;   // [nballs][4]
  double *gsrc = nullptr;   // [ngauss][5]
};

// Patchwise Schwarz tables (order p, see kernels_patch.hip).
struct PatchTables {
  int m = 0;                // patch modes at order p: n_f (2p+1)^d
  int *pm = nullptr;        // [m][4] per-axis slot 0..2p and component (degree-sorted)
  int *pxoff = nullptr;     // [m] plane * G + grid offset relative to the node
  int *pinfo = nullptr;     // [m] element mask, hat axes and offsets (kernels_patch.hip)
  int *prow = nullptr;      // [nP][27] local mode of plane P in the patch of node g - delta
};

struct MlhpState;   // multi-level hp path (mlhp.hip)

}  // namespace fcm

struct fcm_handle {
  fcm::Problem prob;
  fcm_options opt{};
  fcm::Geo geo{};
  hipStream_t stream = nullptr;
  int device = 0;
  int L = 0;                                  // fine level index (= p-1)
  fcm::Level lev[fcm::kMaxLevels];
  fcm::Tables tab;
  std::vector<int> h_lm;                      // host copy of the local modes
  std::vector<uint8_t> h_state;               // element states
  std::vector<int> h_kmat, h_blk;             // per element matrix ids
  std::vector<int> h_cut;                     // element ids of cut elements
  int n_shared = 0, n_unique = 0;
  std::vector<int> h_block_elems;             // representative element per block
  uint8_t *state = nullptr;
  int *kmat = nullptr;                        // -1 void, 0 uncut (K_ref), 1+c cut c
  int *blk = nullptr;                         // -1 void, <n_shared class, else n_shared+u
  int *cut_elems = nullptr;                   // element of each cut matrix
  int *uniq_elems = nullptr;                  // element of each unique Schwarz block
  int *uncut_list = nullptr;                  // kept uncut elements (K_ref)
  int *class_list = nullptr;                  // elements with a shared Schwarz class, by class
  int n_uncut = 0, n_classed = 0;
  int *uncut_chk = nullptr, *class_chk = nullptr;   // same-matrix chunks of the two lists
  int n_uncut_chk = 0, n_class_chk = 0;
  // patchwise smoother: patches (grid nodes with a kept element) ordered
  // class-sorted shared patches first, then unique patches
  fcm::PatchTables ptab;
  int np_shared = 0, np_unique = 0, np_classes = 0;
  int *pnode = nullptr, *pkm = nullptr, *pid = nullptr;
  int *pchk = nullptr, np_chunks = 0;         // class chunks of <= 256 patches
  unsigned *pcpres = nullptr;                 // class mode-presence bits
  int p_words = 0;
  std::vector<int> h_pnode, h_pkm;            // host copies (patch order)
  std::vector<int> h_ppinfo;                  // host copy of the patch mode info
  double *pYs = nullptr, *pYu = nullptr;      // patch products (scratch)
  double *pband = nullptr;                    // band-pair partials of large unique blocks
  double *Yscr = nullptr;                     // stored-matrix products (scratch)
  double *Yshr = nullptr;                     // shared-matrix element products (scratch)
  double *Kref64 = nullptr, *Kcut64 = nullptr, *be = nullptr, *b = nullptr;
  fcm::Coarse co;
  fcm::HMG *hmg = nullptr;                    // set when options.coarse = FCM_COARSE_HMG
  // CG work vectors (fine level, FP64) and reduction scratch
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
  double *red = nullptr;                      // partial sums
  double *scal = nullptr;                     // device scalars
  double *hscal = nullptr;                    // pinned host mirror
  int *dflag = nullptr;                       // device error flag
  int *dflag_co = nullptr;                    // device error flag of the coarse factorisation
  std::vector<double> history;
  hipStream_t own = nullptr;                  // stream of captured CG iterations (and of
                                              // the coarse factorisation during setup)
  hipEvent_t co_ready = nullptr;              // element matrices ready for the coarse setup
  double *co_scr = nullptr;                   // coarse factorisation scratch (setup only)
  hipGraphExec_t cg_exec = nullptr;           // captured steady-state CG iteration
  hipGraph_t cg_graph = nullptr;
  const double *graph_b = nullptr;
  double *graph_x = nullptr;
  double t_setup_ms = 0.0;
  int64_t bytes = 0;
  std::vector<void *> allocs;
  fcm::MlhpState *ml = nullptr;               // set when refine_levels > 0
};

namespace fcm {

// ----------------------------------------------------------------- helpers
void set_error(const char *fmt, ...);
#define FCM_HIP(call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      fcm::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,               \
                     hipGetErrorString(e_));                                  \
      return FCM_ERR_HIP;                                                     \
    }                                                                         \
  } while (0)

// Stream-ordered device memory from the device's default pool, and recycled
// pinned host blocks of 16 doubles (fcm_host.hip).
fcm_status pool_alloc(void **p, size_t bytes, hipStream_t s);
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// Multi-level hp path (mlhp.hip): setup, operators and solvers of a handle
// whose problem has refine_levels > 0.
fcm_status mlhp_setup(fcm_handle *h);
void mlhp_free(fcm_handle *h);
fcm_status mlhp_sizes(const fcm_handle *h, int *n_levels, int64_t *n_dofs, int64_t *n_padded);
fcm_status mlhp_dof_keys(const fcm_handle *h, int64_t *keys);
fcm_status mlhp_rhs(fcm_handle *h, double *b, hipStream_t s);
fcm_status mlhp_apply(fcm_handle *h, int level, const double *x, double *y, hipStream_t s);
fcm_status mlhp_smooth(fcm_handle *h, int level, const double *r, double *z, hipStream_t s);
fcm_status mlhp_coarse_solve(fcm_handle *h, const double *b, double *x, hipStream_t s);
fcm_status mlhp_vcycle(fcm_handle *h, const double *r, double *z, hipStream_t s);
fcm_status mlhp_pcg(fcm_handle *h, const double *b, double *x, fcm_solve_info *info,
                    hipStream_t s);
fcm_status mlhp_stats(const fcm_handle *h, fcm_stats *st);
void pool_free(void *p, hipStream_t s);
double *pinned_get();
void pinned_put(double *b);

// Zero-filled device memory owned by the handle (freed by fcm_destroy), and
// a host vector copied into such memory (the copy is complete on return).
template <typename T>
fcm_status device_alloc(fcm_handle *h, T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  fcm_status st = pool_alloc((void **)p, n * sizeof(T), h->stream);
  if (st != FCM_OK) return st;
  h->allocs.push_back(*p);
  h->bytes += (int64_t)(n * sizeof(T));
  FCM_HIP(hipMemsetAsync(*p, 0, n * sizeof(T), h->stream));
  return FCM_OK;
}

template <typename T>
fcm_status device_upload(fcm_handle *h, T **p, const std::vector<T> &v) {
  fcm_status st = device_alloc(h, p, v.size());
  if (st != FCM_OK) return st;
  if (!v.empty()) {
    FCM_HIP(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    FCM_HIP(hipStreamSynchronize(h->stream));
  }
  return FCM_OK;
}

// Geometric h-levels (hlevels.hip).  hmg_alloc builds the host tables and
// allocates everything on the handle's stream (after the element matrices
// exist); hmg_launch enqueues the level-0 stencil, the Galerkin products, the
// patch blocks and all inverses on stream cs; hmg_cycle applies one h-cycle
// (Alg. 1 over the h-levels, x = 0 on entry) to the level-0 right-hand side.
fcm_status hmg_alloc(fcm_handle *h);
fcm_status hmg_launch(fcm_handle *h, hipStream_t cs);
void hmg_cycle(fcm_handle *h, const double *b, double *x, hipStream_t s);
// Test hooks: y = A_k x (k >= 1) and z = M_k^{-1} r (k >= 0) on h-level k.
fcm_status hmg_apply(fcm_handle *h, int k, const double *x, double *y, hipStream_t s);
fcm_status hmg_smooth(fcm_handle *h, int k, const double *r, double *z, hipStream_t s);
double hmg_cycle_bytes(const fcm_handle *h);

// ------------------------------------------------------- kernel launchers
// Setup (kernels_setup.hip).
void launch_classify(const Geo &g, const double *ball, uint8_t *state, hipStream_t s);
void launch_integrate(const Geo &g, const Tables &t, const fcm_problem &pr, const int *elist,
                      int nlist, int ref_mode, double *Kout, double *be_all, int *flag,
                      hipStream_t s);
void launch_phys_rhs(const Geo &g, const Tables &t, const fcm_problem &pr, const uint8_t *state,
                     double *be_all, hipStream_t s);
// Penalty of the Dirichlet data on an immersed boundary (square edges,
// popcorn surface): for the elements pel[0..nel) with points ptr[k]..ptr[k+1]
// of pts ([x, y, z, w, g]), K_e += beta sum w N N^T and b_e += beta sum w g N,
// in point order.
void launch_edge_penalty(const Geo &g, const Tables &t, const int *pel, int nel, const int *ptr,
                         const double *pts, double beta, const int *kmat, double *Kcut,
                         double *be_all, hipStream_t s);
void launch_traction_rhs(const Geo &g, const Tables &t, int face, const double *tvec,
                         const uint8_t *state, double *be_all, hipStream_t s);
void launch_assemble_rhs(const Geo &g, const Tables &t, const int *kmat, const double *be_all,
                         double *b, hipStream_t s);
void launch_hstencil0(const Geo &g, const Tables &t, const int *kmat, const double *Kref,
                      const double *Kcut, const int *pres, double *S, hipStream_t s);
void launch_form_invert_small(const Geo &g, const Tables &t, int q, int m, const int *belems,
                              int nblocks, const int *kmat, const double *Kref,
                              const double *Kcut, double *inv64, float *inv32, int *flag,
                              double *kappa, hipStream_t s);
void launch_form_blocks(const Geo &g, const Tables &t, int q, int m, const int *belems,
                        int nblocks, const int *kmat, const double *Kref, const double *Kcut,
                        double *out, hipStream_t s);
// Batched in-place SPD inverse of `batch` n x n matrices (row-major, stride n*n).
// kappa (may be null): per matrix ||A_s||_1 ||A_s^{-1}||_1 of the Jacobi-scaled matrix A_s.
int spd_inverse_batched(double *A, int n, int batch, double *scratch, int *flag, double *kappa,
                        hipStream_t s);
size_t spd_inverse_scratch_doubles(int n, int batch);
void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void launch_coarse_stencils(const Geo &g, const Tables &t, const Coarse &c, const int *kmat,
                            const double *Kref, const double *Kcut, hipStream_t s);
void launch_coarse_first(const Geo &g, const Coarse &c, int k, double *S, hipStream_t s);
void launch_coarse_schur(const Geo &g, const Coarse &c, int k, double *S, double *T,
                         hipStream_t s);
void launch_coarse_G(const Geo &g, const Coarse &c, int k, hipStream_t s);

// Solve (kernels_solve.hip).
template <typename T>
struct OpArgs {
  const T *x = nullptr;       // input vector (level q or q-1 planes)
  int m_in = 0;               // local input modes used
  int nP_out = 0;             // output planes
  int ld = 0;                 // matrix leading dimension
  const int *mid = nullptr;   // per element matrix id (-1 skip)
  const T *matS = nullptr;    // shared matrices
  const double *matS64 = nullptr;  // FP64 shared matrices and FP64 accumulation (optional)
  int nS = 0;
  const T *matU = nullptr;    // stored matrices (id - nS)
  const float *matU32 = nullptr;    // mixed-form smoother: FP32 copies of the stored
  const uint8_t *u64flag = nullptr; //   matrices, used where u64flag is null or 0
  int m_out = 0;              // rows of the operator (local modes of the output level)
  const int *units = nullptr; // [nunits][12]: vmask, comp, count, planes[8], pad
  int nunits = 0;
  const int *selem = nullptr; // element of each stored matrix
  int nstored = 0;
  double *Y = nullptr;        // [nstored][m_out] stored-matrix products (scratch)
  void *Yshared = nullptr;    // [m_out][E] shared-matrix products (scratch, TM)
  const int *shlist = nullptr; // elements with a shared matrix, sorted by matrix id
  int nsh = 0;
  const int *chk = nullptr;   // [nchunks][3]: matrix id, first list entry, count (<= 256)
  int nchunks = 0;
  T *out = nullptr;           // out = cvec + scale*acc  (cvec may be null)
  const T *cvec = nullptr;
  T scale = 1;
  T *xs = nullptr;            // smoother: xs = (first ? 0 : xs) + omega*acc
  T omega = 0;
  int first = 0;
  T *xp = nullptr;            // prolongation: xp[P] += ep[P] for P < nP_e
  const T *ep = nullptr;
  int nP_e = 0;
};
template <typename T>
void launch_elem_op(const Geo &g, const Tables &t, const OpArgs<T> &a, hipStream_t s);

// Patchwise smoother apply: out = M^-1 x (delta); xs = (first ? 0 : xs) + omega * delta.
template <typename T>
struct PatchArgs {
  const T *x = nullptr;
  int xlen = 0;                   // length of x (a level vector in the padded plane layout)
  int m = 0, ld = 0;              // level block size, matrix leading dimension (ld % 4 == 0)
  int nP_out = 0;
  const int *pnode = nullptr, *pkm = nullptr, *pid = nullptr;
  int nsh = 0, npu = 0;           // class patches, unique patches
  const int *chk = nullptr;       // [nchunks][3]: class, first patch, count (<= 256)
  int nchunks = 0;
  const unsigned *cpres = nullptr; // [classes][pwords] mode presence bits per class
  int pwords = 0;
  const double *matS64 = nullptr; // [classes][m][ld]
  const float *matS32 = nullptr;  // mixed form: FP32 class inverses (FP32 matrix-core path)
  const double *matU = nullptr;   // [npu][tiles][16][16]: symmetric unique inverses, the 16 x 16
                                  // tiles on and above the diagonal, I-major
  const float *matU32 = nullptr;  // mixed form: FP32 copies of the unique inverses, used where
  const uint8_t *u64flag = nullptr; //   u64flag is null or 0 (matU otherwise)
  int ntile = 0;                  // tiles per row of a unique inverse: ceil(m / 16)
  double *Ys = nullptr;           // [m][nsh]
  double *Yu = nullptr;           // [npu][m]
  double *Pband = nullptr;        // m > kSmallPatchM: [npu][band pairs][512] partial products
  T *out = nullptr;
  T *xs = nullptr;
  T omega = 0;
  int first = 0;
  int stored_only = 0;            // timing hook: launch only the unique-patch GEMV
  int class_rows = 0;             // class-product rows per workgroup / 128 (0: by m)
  int gemv_band = 0;              // 1: unique GEMV by band pairs (always for m > kSmallPatchM)
};
template <typename T>
void launch_patch_op(const Geo &g, const Tables &t, const PatchTables &pt, const PatchArgs<T> &a,
                     hipStream_t s);
void launch_form_patch_blocks(const Geo &g, const Tables &t, const PatchTables &pt, int m,
                              const int *bnode, const int *bkm, int nblocks, const int *kmat,
                              const double *Kref, const double *Kcut, double *out,
                              hipStream_t s);
// Symmetric m x m blocks -> tiles on and above the diagonal (see PatchArgs::matU)
void launch_pack_tiles(const double *src, int m, int nb, double *d64, float *d32, hipStream_t s);
inline int patch_tiles(int m) {
  const int nt = (m + 15) / 16;
  return nt * (nt + 1) / 2;
}
void launch_pack_blocks(const double *src, int m, int ld, int nb, double *d64, float *d32,
                        hipStream_t s);

void launch_dot_partial(const double *x, const double *y, int64_t n, double *partial, int nblk,
                        hipStream_t s);
int dot_blocks(int64_t n);
void launch_dot_final(const double *partial, int nblk, double *dst, hipStream_t s);
void launch_cg_alpha(double *scal, hipStream_t s);
void launch_cg_update_xr(double *x, double *r, const double *p, const double *q,
                         const double *scal, int64_t n, double *partial, int nblk, hipStream_t s);
void launch_cg_beta(double *scal, int flexible, hipStream_t s);
void launch_cg_update_p(double *p, const double *z, const double *scal, int64_t n, int first,
                        hipStream_t s);
void launch_axpby(double *y, const double *x, double a, double b, int64_t n, hipStream_t s);
// y = x (x null: y = 0); a kernel, so that it may sit inside a captured graph
template <typename T>
void launch_copy(T *y, const T *x, int64_t n, hipStream_t s);

// Resumable PCG used by fcm_pcg_solve and the server (fcm_host.hip).
struct CGState {
  const double *b = nullptr;
  double *x = nullptr;
  double nb = 0.0, rel = 1.0;
  int it = 0, status = 0;
  bool first = true, done = false;
};
fcm_status cg_begin(fcm_handle *h, CGState &cg, const double *b_dev, double *x, hipStream_t s);
void cg_issue(fcm_handle *h, CGState &cg, hipStream_t s);
fcm_status cg_capture(fcm_handle *h, const CGState &cg, hipStream_t s);
void cg_finish(fcm_handle *h, CGState &cg);
fcm_status cg_report(fcm_handle *h, CGState &cg, fcm_solve_info *info, hipStream_t s);
int64_t footprint_estimate(const fcm_problem &p, const fcm_options &o);

// Coarse solve.  b, x: level-0 vectors (FP64, padded planes).
void coarse_solve_launch(const Geo &g, const Coarse &c, const double *b, double *x,
                         hipStream_t s);

}  // namespace fcm
