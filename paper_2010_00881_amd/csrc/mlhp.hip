// Multi-level hp overlay path (Section 2.2) with its hp-multigrid (Section
// 3.2): the refinement tree, the active basis, leaf matrices with ancestor
// functions, the patchwise additive Schwarz smoother (Section 3.3.1), the
// V-cycle (Alg. 1) and FP64 CG (Section 4) for the Poisson problem.
//
// Discretisation (host index work, device arithmetic):
//  * base grid n^d; an element whose box is cut by a sphere is bisected into
//    2^d children, recursively to depth K; children are kept even where void
//    (fictitious, alpha-scaled leaves), void base elements are dropped;
//  * every element of every level k carries the integrated Legendre modes of
//    order p on its level's grid; a component (per axis: vertex at node i or
//    degree-j bubble of cell i) is switched off when
//      R1 k >= 1 and a grid cell containing it is not a level-k element but
//         lies in a kept coarser leaf (compatibility),
//      R2 it has a bubble factor and every kept level-k element containing it
//         is refined (linear independence),
//      R3 k >= 1 and it is a vertex that is also a level-(k-1) vertex;
//    it exists when an element containing it carries a kept leaf;
//  * a leaf's functions are its own active modes and those of its ancestors;
//    K_L = int alpha grad N . grad N over the leaf (recursive bisection of cut
//    leaves, (p+1)^d Gauss points per sub-cell) plus beta int_Gamma N N with a
//    fixed surface rule (Gauss-Legendre in cos(theta) x trapezoid in phi),
//    each surface point belonging to the leaf whose half-open box holds it;
//  * DOF order: hats of level 0..K, then modes of degree 2..p, so the
//    multigrid levels (1,0), (1,1), .., (1,K), (2,K), .., (p,K) are prefixes;
//  * Schwarz block of base node v: every function of the multigrid level that
//    is nonzero on a kept leaf inside the base elements around v.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "fcm_internal.hpp"

namespace fcm {

constexpr int kMlMaxM = 256;      // functions per leaf (p = 3, K = 3 in 3D: <= 4 x 64)
constexpr int kMlMaxPatch = 8192; // functions per Schwarz patch (LDS gather)
constexpr int kMlMaxK = 4;        // refinement depth
constexpr int kMlBatch = 4;       // quadrature points per LDS batch

struct MlPatches {                // Schwarz blocks of one multigrid level
  int npatch = 0, max_mb = 0;
  int *pidx = nullptr;            // per patch, padded size mb: block row -> dof (-1 pad)
  int64_t *poff = nullptr;        // per patch offset into pidx
  int *pm = nullptr;              // per patch: padded size, real size
  int64_t *pinv = nullptr;        // per patch offset into inv
  int *plf = nullptr;             // per patch: first (patch, leaf) pair, count
  int *pair_leaf = nullptr;       // per pair: leaf
  int64_t *pair_map = nullptr;    // per pair: offset into map
  int *map = nullptr;             // per pair and leaf function: block row or -1
  int *pg_ptr = nullptr, *pg_slot = nullptr;  // per DOF: its patch rows (slots into pidx)
  double *pc = nullptr;           // per patch row: the smoother product (gathered per DOF)
  double *inv = nullptr;
  int64_t inv_doubles = 0;
  // mixed form: FP32 copies of the inverses whose Jacobi-scaled kappa_1 is small
  // enough (ml_lowprec_kernel)
  double *scal = nullptr;         // per patch row: Jacobi scaling 1/sqrt(B_ii)
  double *norm1 = nullptr;        // per patch: ||S B S||_1
  float *inv32 = nullptr;
  uint8_t *lo32 = nullptr;        // per patch: 1 = applied from inv32
  int n32 = 0;
  int64_t nrows = 0;              // patch rows (padded), the length of pidx
  std::vector<std::pair<int64_t, std::pair<int, int>>> buckets;  // (inv offset, (count, mb))
};

struct MlhpState {
  int d = 3, p = 1, K = 0, nlev = 1;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, h0[3] = {1, 1, 1};
  double ball[4] = {0, 0, 0, 0};
  int geom = 0;
  int nleaf = 0, m_max = 0, n_cut_leaves = 0;
  int64_t ndof = 0;
  std::vector<int64_t> level_size;       // per multigrid level
  std::vector<int64_t> keys;             // DOF order
  std::vector<int> h_leaf;               // k, e0, e1, e2, foff, m, state per leaf
  // device
  int *leaf = nullptr;
  int64_t *koff = nullptr;
  int *fdof = nullptr, *fdesc = nullptr;
  int *lg_ptr = nullptr, *lg_slot = nullptr;  // per DOF: its leaf-function slots (into fdof)
  double *lc = nullptr;                       // per leaf function: load / product contribution
  int64_t *ce_tgt = nullptr, *ce_src = nullptr;  // coarse matrix: entries and Kl sources
  int *ce_ptr = nullptr;
  int n_ce = 0;
  double *Kl = nullptr, *b = nullptr;
  double *surf = nullptr;
  int nsurf = 0;
  double *gx = nullptr;                  // Gauss nodes and weights, p + 1 each
  std::vector<MlPatches> pl;             // multigrid levels 1 .. nlev-1
  double *A0 = nullptr;                  // inverse of the level-0 matrix (n0p x n0p)
  int n0 = 0, n0p = 0;
  std::vector<double *> vx, vr, vy, vz;  // per level work vectors
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
  double *red = nullptr;
  int *flag = nullptr;
  std::vector<double> hist;
};

#define ML_TRY(x)                \
  do {                           \
    fcm_status s_ = (x);         \
    if (s_ != FCM_OK) return s_; \
  } while (0)

// Gather table: for every target t < nt, the slots s with tgt[s] == t in
// increasing s (targets outside [0, nt) are skipped).
static void gather_csr(const std::vector<int> &tgt, int64_t nt, std::vector<int> &ptr,
                       std::vector<int> &slot) {
  ptr.assign(nt + 1, 0);
  for (int t : tgt)
    if (t >= 0 && t < nt) ptr[t + 1]++;
  for (int64_t t = 0; t < nt; ++t) ptr[t + 1] += ptr[t];
  slot.assign(ptr[nt], 0);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (size_t s = 0; s < tgt.size(); ++s)
    if (tgt[s] >= 0 && tgt[s] < nt) slot[fill[tgt[s]]++] = (int)s;
}

// ------------------------------------------------------------ device helpers
struct MlGeo {
  int d, p, K, geom, nballs;
  double lo[3], h0[3];
  const double *ball;              // (cx, cy, cz, r) per ball
  double alpha, kappa, beta, f_const;
  int ngauss;
  const double *gauss;             // (A, w, cx, cy, cz) per source
  int depth;
};

enum { kMlVoid = 0, kMlPhys = 1, kMlCut = 2 };

__device__ int ml_classify(const MlGeo &g, const double *lo, const double *hi) {
  bool any_surface = false;
  for (int j = 0; j < g.nballs; ++j) {
    const double *c = g.ball + 4 * j;
    double s0 = 0.0, s1 = 0.0;
    for (int ax = 0; ax < g.d; ++ax) {
      const double nearest = fmin(fmax(c[ax], lo[ax]), hi[ax]);
      const double far = fabs(lo[ax] - c[ax]) > fabs(hi[ax] - c[ax]) ? lo[ax] : hi[ax];
      s0 += (nearest - c[ax]) * (nearest - c[ax]);
      s1 += (far - c[ax]) * (far - c[ax]);
    }
    const double dmin = sqrt(s0), dmax = sqrt(s1), r = c[3];
    if (g.geom == FCM_GEOM_BALL_INTERIOR) {
      if (dmin >= r) return kMlVoid;
      if (dmax <= r) return kMlPhys;
      return kMlCut;
    }
    if (dmax < r) return kMlVoid;
    if (dmin < r) any_surface = true;
  }
  return any_surface ? kMlCut : kMlPhys;
}

__device__ double ml_alpha(const MlGeo &g, const double *x) {
  if (g.geom == FCM_GEOM_BALL_INTERIOR) {
    const double *c = g.ball;
    double s = 0.0;
    for (int ax = 0; ax < g.d; ++ax) s += (x[ax] - c[ax]) * (x[ax] - c[ax]);
    return s <= c[3] * c[3] ? 1.0 : g.alpha;
  }
  for (int j = 0; j < g.nballs; ++j) {
    const double *c = g.ball + 4 * j;
    double s = 0.0;
    for (int ax = 0; ax < g.d; ++ax) s += (x[ax] - c[ax]) * (x[ax] - c[ax]);
    if (!(s >= c[3] * c[3])) return g.alpha;
  }
  return 1.0;
}

__device__ double ml_source(const MlGeo &g, const double *x) {
  double f = g.f_const;
  for (int k = 0; k < g.ngauss; ++k) {
    const double *s = g.gauss + 5 * k;
    double d2 = 0.0;
    for (int ax = 0; ax < g.d; ++ax) d2 += (x[ax] - s[2 + ax]) * (x[ax] - s[2 + ax]);
    f += s[0] * exp(-d2 / (s[1] * s[1]));
  }
  return f;
}

// value and d/dxi of 1D mode a (0, 1 vertex; j >= 2 integrated Legendre) at xi
__device__ void ml_mode(int a, double xi, double &v, double &dv) {
  if (a == 0) { v = 0.5 * (1.0 - xi); dv = -0.5; return; }
  if (a == 1) { v = 0.5 * (1.0 + xi); dv = 0.5; return; }
  double Lm2 = 1.0, Lm1 = xi;   // L_{a-2}, L_{a-1} after the loop
  for (int k = 1; k < a - 1; ++k) {
    const double Ln = ((2 * k + 1) * xi * Lm1 - k * Lm2) / (k + 1);
    Lm2 = Lm1;
    Lm1 = Ln;
  }
  const double La = ((2 * a - 1) * xi * Lm1 - (a - 1) * Lm2) / a;
  const double s = 1.0 / sqrt(2.0 * (2 * a - 1));
  v = (La - Lm2) * s;
  dv = (2 * a - 1) * Lm1 * s;
}

// ------------------------------------------------------------ classification
__global__ void ml_classify_kernel(MlGeo g, int k, const int *cells, int ncell, uint8_t *state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  double lo[3], hi[3];
  for (int ax = 0; ax < 3; ++ax) {
    const double hk = g.h0[ax] / (double)(1 << k);
    lo[ax] = g.lo[ax] + (double)cells[3 * i + ax] * hk;
    hi[ax] = lo[ax] + hk;
  }
  state[i] = (uint8_t)ml_classify(g, lo, hi);
}

// ------------------------------------------------------------ leaf integration
// Slot of this thread's item among the items that the 256 threads of the
// workgroup take in this call, in thread order (a deterministic list order,
// so the quadrature sums over it are reproducible); *total receives their
// number.  Every thread of the workgroup must call it.
__device__ inline int ml_ordered_slot(bool take, int *wcnt, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long mask = __ballot(take);
  if (lane == 0) wcnt[w] = __popcll(mask);
  __syncthreads();
  int base = 0, tot = 0;
  for (int j = 0; j < 4; ++j) {
    if (j < w) base += wcnt[j];
    tot += wcnt[j];
  }
  __syncthreads();
  *total = tot;
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// One workgroup per leaf.  Integration cells (the leaf, or the sub-cells of
// its recursive bisection) are listed in LDS; points are processed in batches
// whose function values and gradients are staged in LDS; every thread adds
// the batch contribution to 2 x 2 entry blocks of K_L in global memory.
struct MlLeafArgs {
  MlGeo g;
  const int *leaf;        // k, e0, e1, e2, foff, m, state
  const int64_t *koff;
  const int *fdesc;
  const double *gx;       // nodes[p+1], weights[p+1]
  const double *surf;     // x, y, z, w
  int nsurf;
  double *Kl, *lc;        // leaf matrices, per leaf-function load contributions
};

__global__ __launch_bounds__(256) void ml_integrate_kernel(MlLeafArgs a) {
  const MlGeo &g = a.g;
  const int L = blockIdx.x, tid = threadIdx.x;
  const int *lf = a.leaf + 7 * L;
  const int k = lf[0], foff = lf[4], m = lf[5], st = lf[6];
  const int d = g.d, np1 = g.p + 1;
  __shared__ double alo[kMlMaxK + 1][3], ah[kMlMaxK + 1][3];
  __shared__ int fd[kMlMaxM];
  __shared__ double cells[512][6];
  __shared__ int ncells;
  __shared__ double bx[kMlBatch][3], bwg[kMlBatch], bwv[kMlBatch], bwf[kMlBatch];
  __shared__ double V[kMlBatch][kMlMaxM], G[kMlBatch][kMlMaxM][3];
  double *K = a.Kl + a.koff[L];
  for (int i = tid; i < m; i += 256) fd[i] = a.fdesc[foff + i];
  if (tid <= k) {
    for (int ax = 0; ax < 3; ++ax) {
      const double hj = g.h0[ax] / (double)(1 << tid);
      ah[tid][ax] = hj;
      alo[tid][ax] = g.lo[ax] + (double)(lf[1 + ax] >> (k - tid)) * hj;
    }
  }
  for (int i = tid; i < m * m; i += 256) K[i] = 0.0;
  if (tid == 0) ncells = 0;
  __syncthreads();
  double llo[3], lhi[3];
  for (int ax = 0; ax < 3; ++ax) {
    llo[ax] = alo[k][ax];
    lhi[ax] = llo[ax] + ah[k][ax];
  }
  // integration cells: recursive bisection of a cut leaf to depth D, as the
  // set of sub-boxes at which the recursion stops
  const int D = st == kMlCut ? g.depth : 0;
  const int nfine = 1 << (d * D);
  __shared__ int wcnt[4];
  int nc = 0;
  for (int f0 = 0; f0 < nfine; f0 += 256) {
    const int f = f0 + tid;
    int sdepth = D;
    double slo[3], shi[3];
    for (int s = 0; s <= D && f < nfine; ++s) {
      // sub-box of depth s containing fine cell f
      for (int ax = 0; ax < 3; ++ax) {
        if (ax >= d) { slo[ax] = llo[ax]; shi[ax] = lhi[ax]; continue; }
        int idx = 0;
        for (int t = 0; t < s; ++t) idx = 2 * idx + ((f >> (d * (D - 1 - t) + ax)) & 1);
        double blo = llo[ax], bhi = lhi[ax];
        for (int t = 0; t < s; ++t) {
          const double mid = 0.5 * (blo + bhi);
          if ((idx >> (s - 1 - t)) & 1) blo = mid; else bhi = mid;
        }
        slo[ax] = blo;
        shi[ax] = bhi;
      }
      if (s == D || ml_classify(g, slo, shi) != kMlCut) {
        sdepth = s;
        break;
      }
    }
    // f is the representative of its stopping box when its lower bits are 0
    bool first = f < nfine;
    for (int t = sdepth; t < D; ++t)
      for (int ax = 0; ax < d; ++ax) first = first && (((f >> (d * (D - 1 - t) + ax)) & 1) == 0);
    int cnt;
    const int c = nc + ml_ordered_slot(first, wcnt, &cnt);
    if (first) {
      for (int ax = 0; ax < 3; ++ax) {
        cells[c][ax] = slo[ax];
        cells[c][3 + ax] = shi[ax];
      }
    }
    nc += cnt;
  }
  if (tid == 0) ncells = nc;
  __syncthreads();
  int npq = 1;
  for (int ax = 0; ax < d; ++ax) npq *= np1;
  const int nvol = ncells * npq;
  // surface points of this leaf (penalty), only if its closed box meets a sphere
  bool scan = false;
  if (g.beta != 0.0) {
    for (int j = 0; j < g.nballs; ++j) {
      const double *c = g.ball + 4 * j;
      double s0 = 0.0, s1 = 0.0;
      for (int ax = 0; ax < d; ++ax) {
        const double nearest = fmin(fmax(c[ax], llo[ax]), lhi[ax]);
        const double far = fabs(llo[ax] - c[ax]) > fabs(lhi[ax] - c[ax]) ? llo[ax] : lhi[ax];
        s0 += (nearest - c[ax]) * (nearest - c[ax]);
        s1 += (far - c[ax]) * (far - c[ax]);
      }
      if (sqrt(s0) <= c[3] && sqrt(s1) >= c[3]) scan = true;
    }
  }
  const int nsurf = scan ? a.nsurf : 0;
  __shared__ int sel[256];
  double bacc[2] = {0.0, 0.0};
  // one batch of cnt staged points: values/gradients, then K and b updates
  auto process = [&](int cnt) {
    for (int it = tid; it < cnt * m; it += 256) {
      const int q = it / m, i = it % m;
      const int desc = fd[i], j = desc & 15;
      double v = 1.0, gr[3] = {1.0, 1.0, 1.0};
      for (int ax = 0; ax < d; ++ax) {
        const int md = (desc >> (4 + 4 * ax)) & 15;
        const double xi = 2.0 * (bx[q][ax] - alo[j][ax]) / ah[j][ax] - 1.0;
        double mv, mdv;
        ml_mode(md, xi, mv, mdv);
        mdv *= 2.0 / ah[j][ax];
        v *= mv;
        for (int gg = 0; gg < d; ++gg) gr[gg] *= gg == ax ? mdv : mv;
      }
      V[q][i] = v;
      for (int gg = 0; gg < 3; ++gg) G[q][i][gg] = gg < d ? gr[gg] : 0.0;
    }
    __syncthreads();
    // K += sum_q wg G G^T + wv V V^T over 2 x 2 blocks of entries
    const int mh = (m + 1) / 2;
    for (int blk = tid; blk < mh * mh; blk += 256) {
      const int i0 = 2 * (blk / mh), j0 = 2 * (blk % mh);
      double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
      for (int q = 0; q < cnt; ++q) {
        const double wg = bwg[q], wv = bwv[q];
        for (int u = 0; u < 2; ++u) {
          const int i = min(i0 + u, m - 1);
          for (int v2 = 0; v2 < 2; ++v2) {
            const int j = min(j0 + v2, m - 1);
            double sg = 0.0;
            for (int gg = 0; gg < d; ++gg) sg += G[q][i][gg] * G[q][j][gg];
            acc[u][v2] += wg * sg + wv * (V[q][i] * V[q][j]);
          }
        }
      }
      for (int u = 0; u < 2; ++u)
        for (int v2 = 0; v2 < 2; ++v2) {
          const int i = i0 + u, j = j0 + v2;
          if (i < m && j < m) K[(size_t)i * m + j] += acc[u][v2];
        }
    }
    for (int u = 0; u < 2; ++u) {
      const int i = tid + 256 * u;
      if (i < m)
        for (int q = 0; q < cnt; ++q) bacc[u] += bwf[q] * V[q][i];
    }
    __syncthreads();
  };
  // volume points: Gauss points of the integration cells
  for (int base = 0; base < nvol; base += kMlBatch) {
    const int cnt = min(kMlBatch, nvol - base);
    if (tid < cnt) {
      const int q = base + tid, c = q / npq;
      int r = q % npq;
      double x[3] = {0, 0, 0}, w = 1.0;
      for (int ax = 0; ax < d; ++ax) {
        const int qi = r % np1;
        r /= np1;
        const double half = 0.5 * (cells[c][3 + ax] - cells[c][ax]);
        const double mid = 0.5 * (cells[c][3 + ax] + cells[c][ax]);
        x[ax] = mid + half * a.gx[qi];
        w *= half * a.gx[np1 + qi];
      }
      const double al = ml_alpha(g, x);
      for (int ax = 0; ax < 3; ++ax) bx[tid][ax] = x[ax];
      bwg[tid] = w * al * g.kappa;
      bwv[tid] = 0.0;
      bwf[tid] = w * al * ml_source(g, x);
    }
    __syncthreads();
    process(cnt);
  }
  // surface points of the penalty term inside the half-open leaf box
  for (int s0 = 0; s0 < nsurf; s0 += 256) {
    bool in = s0 + tid < nsurf;
    if (in) {
      const double *sp = a.surf + 4 * (size_t)(s0 + tid);
      for (int ax = 0; ax < d; ++ax) in = in && floor((sp[ax] - g.lo[ax]) / ah[k][ax]) == (double)lf[1 + ax];
    }
    int ns;
    const int slot = ml_ordered_slot(in, wcnt, &ns);
    if (in) sel[slot] = s0 + tid;
    __syncthreads();
    for (int b0 = 0; b0 < ns; b0 += kMlBatch) {
      const int cnt = min(kMlBatch, ns - b0);
      if (tid < cnt) {
        const double *sp = a.surf + 4 * (size_t)sel[b0 + tid];
        for (int ax = 0; ax < 3; ++ax) bx[tid][ax] = sp[ax];
        bwg[tid] = 0.0;
        bwv[tid] = g.beta * sp[3];
        bwf[tid] = 0.0;
      }
      __syncthreads();
      process(cnt);
    }
  }
  for (int u = 0; u < 2; ++u) {
    const int i = tid + 256 * u;
    if (i < m) a.lc[foff + i] = bacc[u];
  }
}

// sum_j M[j] v[j] over j = lane, lane + 64, ... < n with four independent
// accumulators (four loads in flight per lane), fixed order
template <typename TM>
__device__ inline double ml_row_dot(const TM *M, const double *v, int n, int lane) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int j = lane;
  for (; j + 192 < n; j += 256) {
    a0 += M[j] * v[j];
    a1 += M[j + 64] * v[j + 64];
    a2 += M[j + 128] * v[j + 128];
    a3 += M[j + 192] * v[j + 192];
  }
  for (; j < n; j += 64) a0 += M[j] * v[j];
  return (a0 + a1) + (a2 + a3);
}

// ------------------------------------------------------------ operators
// y += A_l x over the leaves (functions with DOF index >= n_l are absent)
__global__ __launch_bounds__(256) void ml_apply_kernel(const int *leaf, const int64_t *koff,
                                                       const int *fdof, const double *Kl,
                                                       int64_t nl, const double *x, double *lc) {
  const int L = blockIdx.x, tid = threadIdx.x;
  const int foff = leaf[7 * L + 4], m = leaf[7 * L + 5];
  __shared__ double xs[kMlMaxM];
  __shared__ int ds[kMlMaxM];
  for (int i = tid; i < m; i += 256) {
    const int dof = fdof[foff + i];
    ds[i] = dof;
    xs[i] = dof < nl ? x[dof] : 0.0;
  }
  __syncthreads();
  const double *K = Kl + koff[L];
  const int wave = tid >> 6, lane = tid & 63;
  for (int i = wave; i < m; i += 4) {
    if (ds[i] >= nl) continue;
    double s = ml_row_dot(K + (size_t)i * m, xs, m, lane);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) lc[foff + i] = s;
  }
}

// Owner gather: y[t] = sum of c[slot[k]], ptr[t] <= k < ptr[t + 1], in that
// (fixed) order, for every t < n.  Replaces atomic scatters: the leaves' and
// patches' contributions land in per-slot buffers and every DOF adds its own,
// so the sums are the same on every run.
__global__ void ml_gather_kernel(int64_t n, const int *ptr, const int *slot, const double *c,
                                 double *y) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int k = ptr[t]; k < ptr[t + 1]; ++k) v += c[slot[k]];
    y[t] = v;
  }
}

// dense level-0 matrix from the leaf matrices (functions with DOF < n0): entry
// tgt[e] = the sum of Kl[src[k]], ptr[e] <= k < ptr[e + 1], in leaf order
__global__ void ml_coarse_assemble_kernel(int ne, const int64_t *tgt, const int *ptr,
                                          const int64_t *src, const double *Kl, double *A0) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double v = 0.0;
  for (int k = ptr[e]; k < ptr[e + 1]; ++k) v += Kl[src[k]];
  A0[tgt[e]] = v;
}

// x = M b for the leading n x n block of a matrix with leading dimension ld
// (one wave per row)
__global__ void ml_gemv_kernel(const double *M, int n, int ld, const double *b, double *x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = ml_row_dot(M + (size_t)row * ld, b, n, lane);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = s;
}

// Schwarz block of each patch from the leaf matrices: B = P^T A_l P, with
// identity rows and columns in the padding
__global__ __launch_bounds__(256) void ml_form_blocks_kernel(
    const int *pm, const int64_t *pinv, const int *plf, const int *pair_leaf,
    const int64_t *pair_map, const int *map, const int *leaf, const int64_t *koff,
    const double *Kl, double *inv) {
  const int P = blockIdx.x, tid = threadIdx.x;
  const int mb = pm[2 * P], mreal = pm[2 * P + 1];
  double *B = inv + pinv[P];
  for (int e = tid; e < mb * mb; e += 256) {
    const int r = e / mb, c = e % mb;
    B[e] = (r == c && r >= mreal) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int first = plf[2 * P], count = plf[2 * P + 1];
  for (int t = 0; t < count; ++t) {
    const int L = pair_leaf[first + t];
    const int m = leaf[7 * L + 5];
    const int *mp = map + pair_map[first + t];
    const double *K = Kl + koff[L];
    for (int e = tid; e < m * m; e += 256) {
      const int ia = mp[e / m], ib = mp[e % m];
      if (ia >= 0 && ib >= 0) B[(size_t)ia * mb + ib] += K[e];
    }
    __syncthreads();
  }
}

// z += sum_patches P_i A_i^{-1} P_i^T r; workgroup (P, c) takes rows
// [64 c, 64 c + 64) of patch P (grid.y = max rows / 64)
__global__ __launch_bounds__(256) void ml_smooth_kernel(const int *pm, const int64_t *pinv,
                                                        const int64_t *poff, const int *pidx,
                                                        const double *inv, const float *inv32,
                                                        const uint8_t *lo32, const double *r,
                                                        double *pc) {
  const int P = blockIdx.x, tid = threadIdx.x;
  const int mb = pm[2 * P], mreal = pm[2 * P + 1];
  const int row0 = 64 * blockIdx.y;
  if (row0 >= mreal) return;
  const int *idx = pidx + poff[P];
  __shared__ double rs[kMlMaxPatch];
  for (int i = tid; i < mb; i += 256) rs[i] = i < mreal ? r[idx[i]] : 0.0;
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int row1 = min(mreal, row0 + 64);
  const bool lo = inv32 && lo32[P];
  for (int i = row0 + wave; i < row1; i += 4) {
    double s = lo ? ml_row_dot(inv32 + pinv[P] + (size_t)i * mb, rs, mreal, lane)
                  : ml_row_dot(inv + pinv[P] + (size_t)i * mb, rs, mreal, lane);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) pc[poff[P] + i] = s;
  }
}

// Inverses of SPD blocks in Gram form, blocked and batched over a bucket of
// equal-size blocks (n a multiple of 32, count = gridDim.y):
//   S = diag(B)^{-1/2},  S B S = U^T U  (upper Cholesky factor, in place),
//   X = U^{-1}  (upper triangular, into a scratch copy),
//   B^{-1} = S X X^T S,
// in blocks of kCB = 64 pivots: the diagonal block of each step is factored
// (or solved against) in LDS, the O(n^3) parts -- the block-row updates of
// the left-looking factorisation, the block products of the triangular
// inverse and the Gram product -- run on v_mfma_f64_16x16x4f64 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4j + l/16][l%16] of a 16 x 16 tile).  Unlike an
// elimination inverse, the Gram form stays positive definite when the scaled
// condition reaches 1e13 and more (patch blocks with fictitious leaves).
// Every reduction has a fixed order: the result is bitwise reproducible.
constexpr int kCB = 64;
typedef double ml_d4 __attribute__((ext_vector_type(4)));

__global__ void mlc_zero_kernel(double *x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// s_i = 1 / sqrt(B_ii) (1 and the flag where B_ii <= 0)
__global__ void mlc_diag_kernel(const double *Ball, int n, double *sc, int *flag) {
  const int b = blockIdx.y;
  const double *B = Ball + (size_t)b * n * n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double dg = B[(size_t)i * n + i];
    if (!(dg > 0.0)) atomicOr(flag, 1);
    sc[(size_t)b * n + i] = dg > 0.0 ? 1.0 / sqrt(dg) : 1.0;
  }
}

// B <- S B S, one wave per row; with norm1, ||S B S||_1 (the largest absolute
// row sum of the symmetric scaled block) by atomicMax on the bit pattern
// (order-preserving for non-negative doubles, so the result does not depend
// on the order of the rows)
__global__ void mlc_scale_kernel(double *Ball, int n, const double *sc, double *norm1) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= n) return;
  double *row = Ball + (size_t)b * n * n + (size_t)r * n;
  const double *s = sc + (size_t)b * n;
  const double sr = s[r];
  double sum = 0.0;
  for (int c = lane; c < n; c += 64) {
    const double v = row[c] * sr * s[c];
    row[c] = v;
    sum += fabs(v);
  }
  if (!norm1) return;
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  if (lane == 0)
    atomicMax((unsigned long long *)(norm1 + b), (unsigned long long)__double_as_longlong(sum));
}

// Step k0 of the factorisation, diagonal block (one workgroup per block of
// the bucket): A11 = U11^T U11 in LDS, row by row (left-looking, as the
// block-row update: each entry of row j is formed once from the rows above
// it), U11 written over A11.  The diagonal entries are left untouched by the
// block-row updates: each pivot is formed here from the scaled diagonal
// entry minus the compensated (Kahan) sum of the squares of its whole column
// of U above it, since the smallest pivots (scaled conditions of 1e13 and
// more) are the last bits of that cancellation.  Only upper triangles are
// read and written; the lower one is never used again.
__global__ __launch_bounds__(256) void mlc_potrf_kernel(double *Ball, int n, int k0, int *flag) {
  __shared__ double a[kCB][kCB + 1];
  __shared__ double part[4][kCB];
  __shared__ double piv_s;
  const int b = blockIdx.x, tid = threadIdx.x;
  double *B = Ball + (size_t)b * n * n;
  const int kb = min(kCB, n - k0);
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int i = e >> 6, j = e & 63;
    a[i][j] = (i < kb && j < kb && i <= j) ? B[(size_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  {
    // sum_{k < k0} U[k][k0 + j]^2 in four interleaved compensated chains
    const int j = tid & 63, r = tid >> 6;
    const int jc = min(j, kb - 1);
    double s = 0.0, c = 0.0;
    for (int k = r; k < k0; k += 4) {
      const double u = B[(size_t)k * n + k0 + jc];
      const double y = fma(u, u, -c);
      const double t2 = s + y;
      c = (t2 - s) - y;
      s = t2;
    }
    part[r][j] = s;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      double s = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j], c = 0.0;
      for (int k = 0; k < j; ++k) {
        const double y = fma(a[k][j], a[k][j], -c);
        const double t2 = s + y;
        c = (t2 - s) - y;
        s = t2;
      }
      const double dj = a[j][j] - s;
      if (!(dj > 0.0)) atomicOr(flag, 1);
      piv_s = dj > 0.0 ? sqrt(dj) : 1.0;
    }
    __syncthreads();
    const double piv = piv_s;
    if (tid > j && tid < kb) {
      double v = a[j][tid];
      for (int k = 0; k < j; ++k) v -= a[k][j] * a[k][tid];
      a[j][tid] = v / piv;
    }
    if (tid == j) a[j][j] = piv;
    __syncthreads();
  }
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int i = e >> 6, j = e & 63;
    if (i < kb && j < kb && i <= j) B[(size_t)(k0 + i) * n + k0 + j] = a[i][j];
  }
}

// Step k0, panel: workgroup (x, b) forms the columns [k0 + 64 (x + 1), + 64)
// of U12 = U11^{-T} A12 by forward substitution (U11 in LDS, one column per
// lane).  A separate launch from mlc_potrf_kernel, which writes U11 over A11.
__global__ __launch_bounds__(256) void mlc_trsm_kernel(double *Ball, int n, int k0) {
  __shared__ double a[kCB][kCB + 1];
  __shared__ double xs[kCB][kCB + 1];
  const int b = blockIdx.y, tid = threadIdx.x;
  double *B = Ball + (size_t)b * n * n;
  const int c0 = k0 + kCB * ((int)blockIdx.x + 1), w = min(kCB, n - c0);
  // columns past k0 + 64 exist only when the step is 64 wide
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int i = e >> 6, j = e & 63;
    a[i][j] = i <= j ? B[(size_t)(k0 + i) * n + k0 + j] : 0.0;
    xs[i][j] = j < w ? B[(size_t)(k0 + i) * n + c0 + j] : 0.0;
  }
  __syncthreads();
  if (tid < w) {
    const int c = tid;
    for (int t = 0; t < kCB; ++t) {
      double v = xs[t][c];
      for (int s = 0; s < t; ++s) v -= a[s][t] * xs[s][c];
      xs[t][c] = v / a[t][t];
    }
  }
  __syncthreads();
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int t = e >> 6, c = e & 63;
    if (c < w) B[(size_t)(k0 + t) * n + c0 + c] = xs[t][c];
  }
}

// Block row q of the factorisation (left-looking): before its diagonal block
// is factored, every entry of rows [k0, k0 + 64) above the diagonal (the
// pivots are formed in mlc_potrf_kernel) takes all its updates at once, A[i][j] - sum_{k < k0} U[k][i] U[k][j], the
// sum in one matrix-core accumulator over the final rows of U above it, and
// the entry is rounded once (a right-looking update would store and round it
// after every earlier block; with scaled conditions of 1e13 and more the
// small pivots come out of a cancellation that those roundings spoil).
// Workgroup (x, b): the 64 x 64 tile of columns [k0 + 64 x, + 64), wave w
// its 32 x 32 quarter (w / 2, w % 2) as 2 x 2 MFMA tiles.  n and k0 are
// multiples of 32 and 64, so a quarter that starts inside the matrix lies
// inside it.
__global__ __launch_bounds__(256) void mlc_rowupdate_kernel(double *Ball, int n, int k0) {
  const int b = blockIdx.y;
  double *B = Ball + (size_t)b * n * n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 15, lq = lane >> 4;
  const int i0 = k0 + (wave >> 1) * 32, j0 = k0 + kCB * (int)blockIdx.x + (wave & 1) * 32;
  if (i0 >= n || j0 >= n || i0 > j0 + 31) return;
  ml_d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = ml_d4{0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < k0; k += 16) {
    double av[4][2], bv[4][2];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[s][u] = B[(size_t)(k + 4 * s + lq) * n + i0 + 16 * u + ln];
        bv[s][u] = B[(size_t)(k + 4 * s + lq) * n + j0 + 16 * u + ln];
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][u], bv[s][v], acc[u][v], 0, 0, 0);
  }
  double old[2][2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        old[u][v][jj] = B[(size_t)(i0 + 16 * u + 4 * jj + lq) * n + j0 + 16 * v + ln];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + 16 * u + 4 * jj + lq, j = j0 + 16 * v + ln;
        if (i < j) B[(size_t)i * n + j] = old[u][v][jj] - acc[u][v][jj];
      }
}

// Block column J of X = U^{-1}, solved from the right as in the classic
// blocked triangular inverse: every block X_rJ satisfies X_rJ U_JJ = R with
// R = I (r = J) or R = -(sum_{K=r}^{J-1} X_rK U_KJ) (r < J, the sum on the
// matrix cores from the earlier block columns of X), solved row by row by
// forward substitution against U_JJ in LDS (one row per lane), so that every
// block has a small right residual X U - I (as the row-by-row forward
// substitution U^T x_c = e_c has); multiplying by an explicit inverse of
// U_JJ instead lets an ill-conditioned U_JJ amplify that residual.  r = J
// stores the zeros below the diagonal of X_JJ too.
__global__ __launch_bounds__(256) void mlc_trtri_kernel(const double *Ball, double *Xall, int n,
                                                        int J) {
  __shared__ double ua[kCB][kCB + 1];   // U_JJ (identity past the matrix)
  __shared__ double rs[kCB][kCB + 1];   // right-hand sides, then X_rJ
  const int r = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const double *B = Ball + (size_t)b * n * n;
  double *X = Xall + (size_t)b * n * n;
  const int c0 = kCB * J, w = min(kCB, n - c0);
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int i = e >> 6, j = e & 63;
    ua[i][j] = (i < w && j < w) ? (i <= j ? B[(size_t)(c0 + i) * n + c0 + j] : 0.0)
                                : (i == j ? 1.0 : 0.0);
  }
  const int wave = tid >> 6, lane = tid & 63;
  if (r == J) {
    for (int e = tid; e < kCB * kCB; e += 256) rs[e >> 6][e & 63] = (e >> 6) == (e & 63) ? 1.0 : 0.0;
  } else {
    // R = -sum_{k in [64 r, 64 J)} X[i][k] U[k][c] for the 64 rows of block r
    const int ln = lane & 15, lq = lane >> 4;
    const int i0 = kCB * r + (wave >> 1) * 32, j0 = c0 + (wave & 1) * 32;
    ml_d4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[u][v] = ml_d4{0.0, 0.0, 0.0, 0.0};
    if (j0 < n) {   // wave-uniform: the right half of a 32-wide last block column is empty
      for (int k = kCB * r; k < c0; k += 16) {
        double av[4][2], bv[4][2];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            av[s][u] = X[(size_t)(i0 + 16 * u + ln) * n + k + 4 * s + lq];
            bv[s][u] = B[(size_t)(k + 4 * s + lq) * n + j0 + 16 * u + ln];
          }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
              acc[u][v] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][u], bv[s][v], acc[u][v], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          rs[(wave >> 1) * 32 + 16 * u + 4 * jj + lq][(wave & 1) * 32 + 16 * v + ln] =
              -acc[u][v][jj];
  }
  __syncthreads();
  if (wave == 0) {
    // row `lane`: x[c] = (R[c] - sum_{t < c} x[t] U[t][c]) / U[c][c], in place
    for (int c = 0; c < w; ++c) {
      double v = rs[lane][c];
      for (int t = 0; t < c; ++t) v -= rs[lane][t] * ua[t][c];
      rs[lane][c] = v / ua[c][c];
    }
  }
  __syncthreads();
  const int rows = r == J ? w : kCB;
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int i = e >> 6, c = e & 63;
    if (i < rows && c < w) X[(size_t)(kCB * r + i) * n + c0 + c] = rs[i][c];
  }
}

// B^{-1} = S X X^T S: entry (i, j) = s_i s_j sum_{k >= max(i, j)} X[i][k] X[j][k]
// (X upper triangular, zero below the diagonal inside its diagonal blocks);
// 64 x 64 tiles ti <= tj, each value stored at (i, j) and (j, i), so the
// inverse is exactly symmetric.
__global__ __launch_bounds__(256) void mlc_gram_kernel(const double *Xall, const double *scall,
                                                       double *Call, int n, int ntile) {
  const int b = blockIdx.y;
  int ti = 0, rem = blockIdx.x;
  while (rem >= ntile - ti) {
    rem -= ntile - ti;
    ++ti;
  }
  const int tj = ti + rem;
  const double *X = Xall + (size_t)b * n * n;
  const double *sc = scall + (size_t)b * n;
  double *C = Call + (size_t)b * n * n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 15, lq = lane >> 4;
  const int i0 = ti * 64 + (wave >> 1) * 32, j0 = tj * 64 + (wave & 1) * 32;
  if (i0 >= n || j0 >= n || i0 > j0 + 31) return;
  ml_d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = ml_d4{0.0, 0.0, 0.0, 0.0};
  for (int k = tj * 64; k < n; k += 32) {
    double av[8][2], bv[8][2];
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[s][u] = X[(size_t)(i0 + 16 * u + ln) * n + k + 4 * s + lq];
        bv[s][u] = X[(size_t)(j0 + 16 * u + ln) * n + k + 4 * s + lq];
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][u], bv[s][v], acc[u][v], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + 16 * u + 4 * jj + lq, j = j0 + 16 * v + ln;
        if (i > j) continue;
        const double val = sc[i] * sc[j] * acc[u][v][jj];
        C[(size_t)i * n + j] = val;
        C[(size_t)j * n + i] = val;
      }
}

// Mixed form: ||(S B S)^{-1}||_1 = max_i sum_j |inv_ij| / (s_i s_j) of each
// patch inverse (one workgroup per patch, fixed reduction order).  Rounding
// the entries of an m x m inverse to FP32 moves its smallest eigenvalue by up
// to about u32 sqrt(m) kappa relative (u32 = 2^-24), so a patch gets an FP32
// copy, and is applied from it, only where u32 sqrt(m) kappa_1 <= 1e-2 (with
// blocks of up to 1858 rows the uniform-grid rule kappa_1 <= 1e5 allowed
// perturbations of 25 % and one seeded solve stalled).
__global__ __launch_bounds__(256) void ml_lowprec_kernel(const int *pm, const int64_t *pinv,
                                                         const int64_t *poff, const double *scal,
                                                         const double *norm1, const double *inv,
                                                         float *inv32, uint8_t *lo32) {
  const int P = blockIdx.x, tid = threadIdx.x;
  const int n = pm[2 * P];
  const double *M = inv + pinv[P];
  const double *sc = scal + poff[P];
  __shared__ double red[256];
  double mx = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double *row = M + (size_t)i * n;
    double rs = 0.0;
    for (int j = 0; j < n; ++j) rs += fabs(row[j]) / (sc[i] * sc[j]);
    mx = fmax(mx, rs);
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const bool lo = 0x1p-24 * sqrt((double)n) * norm1[P] * red[0] <= 1e-2;
  if (tid == 0) lo32[P] = lo ? 1 : 0;
  if (!lo) return;
  float *M32 = inv32 + pinv[P];
  for (size_t e = tid; e < (size_t)n * n; e += 256) M32[e] = (float)M[e];
}

// ------------------------------------------------------------ vectors
__global__ void ml_axpby_kernel(int64_t n, double a, const double *x, double b, double *y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void ml_sub_kernel(int64_t n, const double *b, const double *y, double *r) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - y[i];
}

// per-block partial sums (fixed tree order), added in block order by ml_sum_kernel
__global__ void ml_dot_kernel(int64_t n, const double *x, const double *y, double *partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void ml_sum_kernel(int nb, const double *partial, double *out) {
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += partial[b];
    *out = v;
  }
}

static int ml_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

// Inverses of the SPD blocks of a level in place, in Gram form (see the
// mlc_ kernels above), one launch sequence per bucket (inv offset, (count,
// size)) of equal-size blocks.  The patches of a bucket are consecutive, so
// their scalings (scal, by patch row) and norms (norm1, by patch) are
// consecutive too.  wt: scratch for X (the size of inv); w: scratch for the
// scalings where scal is null.
static fcm_status ml_spd_inverse(double *inv,
                                 const std::vector<std::pair<int64_t, std::pair<int, int>>> &bk,
                                 double *wt, double *w, int *flag, hipStream_t s,
                                 double *scal = nullptr, double *norm1 = nullptr) {
  int64_t soff = 0;
  int p0 = 0;
  for (const auto &bkt : bk) {
    const int cnt = bkt.second.first, n = bkt.second.second;
    if (n % 32 != 0) {
      set_error("multi-level hp: block size %d is not a multiple of 32", n);
      return FCM_ERR_ARG;
    }
    double *B = inv + bkt.first, *X = wt + bkt.first;
    double *sc = scal ? scal + soff : w + bkt.first;
    double *nrm = norm1 ? norm1 + p0 : nullptr;
    if (nrm) mlc_zero_kernel<<<(cnt + 255) / 256, 256, 0, s>>>(nrm, cnt);
    mlc_diag_kernel<<<dim3((n + 255) / 256, cnt), 256, 0, s>>>(B, n, sc, flag);
    mlc_scale_kernel<<<dim3((n + 3) / 4, cnt), 256, 0, s>>>(B, n, sc, nrm);
    const int nb = (n + kCB - 1) / kCB;
    for (int q = 0; q < nb; ++q) {
      const int k0 = q * kCB, kb = std::min(kCB, n - k0), k1 = k0 + kb;
      if (q > 0) mlc_rowupdate_kernel<<<dim3(nb - q, cnt), 256, 0, s>>>(B, n, k0);
      mlc_potrf_kernel<<<cnt, 256, 0, s>>>(B, n, k0, flag);
      // only the last block row can be 32 high, and it has nothing to its right
      if (k1 < n) mlc_trsm_kernel<<<dim3(nb - q - 1, cnt), 256, 0, s>>>(B, n, k0);
    }
    for (int J = 0; J < nb; ++J)
      mlc_trtri_kernel<<<dim3(J + 1, cnt), 256, 0, s>>>(B, X, n, J);
    mlc_gram_kernel<<<dim3(nb * (nb + 1) / 2, cnt), 256, 0, s>>>(X, sc, B, n, nb);
    soff += (int64_t)cnt * n;
    p0 += cnt;
  }
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

// ------------------------------------------------------------ host: tree and basis
namespace {

struct LevelGrid {                // dense per-level arrays over the level-k grid
  int N[3] = {1, 1, 1};
  std::vector<uint8_t> inE, refined, state, carries;
  int64_t lin(const int *c) const { return c[0] + (int64_t)N[0] * (c[1] + (int64_t)N[1] * c[2]); }
  bool in_box(const int *c, int d) const {
    for (int ax = 0; ax < d; ++ax)
      if (c[ax] < 0 || c[ax] >= N[ax]) return false;
    return true;
  }
};

struct Builder {
  fcm_handle *h;
  MlhpState *S;
  MlGeo g;
  std::vector<LevelGrid> lv;
  std::vector<std::vector<int>> modes;      // mode tuples (a0, a1, a2), axis 0 fastest
  int64_t S_ax[kMlMaxK + 1][3];
  int64_t key_off[kMlMaxK + 2];

  void mode_codes(int k, const int *e, const std::vector<int> &t, int64_t *codes) const {
    const int p = S->p;
    for (int ax = 0; ax < 3; ++ax) {
      if (ax >= S->d) { codes[ax] = 0; continue; }
      const int a = t[ax];
      codes[ax] = a <= 1 ? (int64_t)(e[ax] + a) * p : (int64_t)e[ax] * p + (a - 1);
    }
    (void)k;
  }
  int64_t key_of(int k, const int64_t *codes) const {
    int64_t key = 0;
    for (int ax = S->d - 1; ax >= 0; --ax) key = key * S_ax[k][ax] + codes[ax];
    return key + key_off[k];
  }
  bool dropped_base(int k, const int *c) const {
    int b[3] = {0, 0, 0};
    for (int ax = 0; ax < S->d; ++ax) b[ax] = c[ax] >> k;
    return lv[0].state[lv[0].lin(b)] == kMlVoid;
  }
};

}  // namespace

static fcm_status ml_build_tree(Builder &B) {
  MlhpState *S = B.S;
  fcm_handle *h = B.h;
  const int d = S->d;
  B.lv.resize(S->K + 1);
  std::vector<int> cells;
  for (int k = 0; k <= S->K; ++k) {
    LevelGrid &G = B.lv[k];
    for (int ax = 0; ax < 3; ++ax) G.N[ax] = ax < d ? S->n[ax] << k : 1;
    const int64_t tot = (int64_t)G.N[0] * G.N[1] * G.N[2];
    G.inE.assign(tot, 0);
    G.refined.assign(tot, 0);
    G.state.assign(tot, kMlVoid);
    cells.clear();
    if (k == 0) {
      for (int64_t i = 0; i < tot; ++i) G.inE[i] = 1;
    } else {
      const LevelGrid &P = B.lv[k - 1];
      for (int c2 = 0; c2 < G.N[2]; ++c2)
        for (int c1 = 0; c1 < G.N[1]; ++c1)
          for (int c0 = 0; c0 < G.N[0]; ++c0) {
            int c[3] = {c0, c1, c2}, pc[3] = {c0 >> 1, c1 >> 1, d == 3 ? c2 >> 1 : 0};
            if (P.refined[P.lin(pc)]) G.inE[G.lin(c)] = 1;
          }
    }
    for (int c2 = 0; c2 < G.N[2]; ++c2)
      for (int c1 = 0; c1 < G.N[1]; ++c1)
        for (int c0 = 0; c0 < G.N[0]; ++c0) {
          int c[3] = {c0, c1, c2};
          if (G.inE[G.lin(c)]) cells.insert(cells.end(), c, c + 3);
        }
    const int nc = (int)cells.size() / 3;
    if (nc > 0) {
      int *dc = nullptr;
      uint8_t *ds = nullptr;
      ML_TRY(pool_alloc((void **)&dc, cells.size() * sizeof(int), h->stream));
      ML_TRY(pool_alloc((void **)&ds, nc, h->stream));
      FCM_HIP(hipMemcpyAsync(dc, cells.data(), cells.size() * sizeof(int), hipMemcpyHostToDevice,
                             h->stream));
      ml_classify_kernel<<<(nc + 255) / 256, 256, 0, h->stream>>>(B.g, k, dc, nc, ds);
      std::vector<uint8_t> st(nc);
      FCM_HIP(hipMemcpyAsync(st.data(), ds, nc, hipMemcpyDeviceToHost, h->stream));
      FCM_HIP(hipStreamSynchronize(h->stream));
      pool_free(dc, h->stream);
      pool_free(ds, h->stream);
      for (int i = 0; i < nc; ++i) {
        const int64_t li = G.lin(&cells[3 * i]);
        G.state[li] = st[i];
        if (k < S->K && st[i] == kMlCut) G.refined[li] = 1;
      }
    }
  }
  // elements carrying kept leaves (bottom-up); leaves
  for (int k = S->K; k >= 0; --k) {
    LevelGrid &G = B.lv[k];
    const int64_t tot = (int64_t)G.N[0] * G.N[1] * G.N[2];
    G.carries.assign(tot, 0);
    for (int c2 = 0; c2 < G.N[2]; ++c2)
      for (int c1 = 0; c1 < G.N[1]; ++c1)
        for (int c0 = 0; c0 < G.N[0]; ++c0) {
          int c[3] = {c0, c1, c2};
          const int64_t li = G.lin(c);
          if (!G.inE[li]) continue;
          if (!G.refined[li]) {
            G.carries[li] = (k > 0 || G.state[li] != kMlVoid) ? 1 : 0;
            if (G.carries[li]) {
              S->h_leaf.insert(S->h_leaf.end(), {k, c0, c1, c2, 0, 0, (int)G.state[li]});
            }
          } else {
            const LevelGrid &C = B.lv[k + 1];
            uint8_t any = 0;
            for (int s = 0; s < (1 << d); ++s) {
              int cc[3] = {2 * c0 + (s & 1), 2 * c1 + ((s >> 1) & 1), d == 3 ? 2 * c2 + ((s >> 2) & 1) : 0};
              any |= C.carries[C.lin(cc)];
            }
            G.carries[li] = any;
          }
        }
  }
  S->nleaf = (int)S->h_leaf.size() / 7;
  return FCM_OK;
}

// (active, exists) of the level-k component with per-axis codes
static void ml_status(const Builder &B, int k, const int64_t *codes, bool &active, bool &exists) {
  const MlhpState *S = B.S;
  const int d = S->d, p = S->p;
  const LevelGrid &G = B.lv[k];
  int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  bool vertex = true, even = true;
  for (int ax = 0; ax < d; ++ax) {
    const int64_t i = codes[ax] / p, r = codes[ax] % p;
    if (r == 0) {
      lo[ax] = (int)i - 1;
      cnt[ax] = 2;
      if (i % 2 != 0) even = false;
    } else {
      lo[ax] = (int)i;
      cnt[ax] = 1;
      vertex = false;
    }
  }
  bool boundary = false, any_existing = false, all_refined = true;
  exists = false;
  for (int s2 = 0; s2 < cnt[2]; ++s2)
    for (int s1 = 0; s1 < cnt[1]; ++s1)
      for (int s0 = 0; s0 < cnt[0]; ++s0) {
        int c[3] = {lo[0] + s0, lo[1] + s1, lo[2] + s2};
        if (!G.in_box(c, d)) continue;
        const int64_t li = G.lin(c);
        if (G.inE[li]) {
          if (k == 0 && B.dropped_base(0, c)) continue;
          any_existing = true;
          if (!G.refined[li]) all_refined = false;
          if (G.carries[li]) exists = true;
        } else {
          // the coarser leaf containing c: kept unless a dropped base element
          for (int j = k - 1; j >= 0; --j) {
            int a[3] = {c[0] >> (k - j), c[1] >> (k - j), c[2] >> (k - j)};
            if (d == 2) a[2] = 0;
            if (B.lv[j].inE[B.lv[j].lin(a)]) {
              if (!(j == 0 && B.dropped_base(0, a))) boundary = true;
              break;
            }
          }
        }
      }
  active = true;
  if (k >= 1 && boundary) active = false;                         // R1
  if (!vertex && any_existing && all_refined) active = false;     // R2
  if (k >= 1 && vertex && even) active = false;                   // R3
  const unsigned faces = B.h->prob.pr.dirichlet_faces;
  for (int ax = 0; ax < d; ++ax) {
    const int64_t i = codes[ax] / p, r = codes[ax] % p;
    if (r == 0 && ((faces >> (2 * ax)) & 1) && i == 0) exists = false;
    if (r == 0 && ((faces >> (2 * ax + 1)) & 1) && i == G.N[ax]) exists = false;
  }
}

static fcm_status ml_number(Builder &B, std::unordered_map<int64_t, int> &dof_of) {
  MlhpState *S = B.S;
  const int d = S->d, p = S->p, K = S->K;
  struct Rec { int64_t key; int group, level, deg; };
  std::vector<Rec> recs;
  std::unordered_map<int64_t, char> seen;
  for (int k = 0; k <= K; ++k) {
    const LevelGrid &G = B.lv[k];
    for (int c2 = 0; c2 < G.N[2]; ++c2)
      for (int c1 = 0; c1 < G.N[1]; ++c1)
        for (int c0 = 0; c0 < G.N[0]; ++c0) {
          int c[3] = {c0, c1, c2};
          if (!G.inE[G.lin(c)]) continue;
          for (const auto &t : B.modes) {
            int64_t codes[3];
            B.mode_codes(k, c, t, codes);
            const int64_t key = B.key_of(k, codes);
            if (seen.count(key)) continue;
            seen[key] = 1;
            bool active, exists;
            ml_status(B, k, codes, active, exists);
            if (!(active && exists)) continue;
            int deg = 1;
            for (int ax = 0; ax < d; ++ax) deg = std::max(deg, t[ax] < 2 ? 1 : t[ax]);
            recs.push_back({key, deg == 1 ? k : K + deg - 1, k, deg});
          }
        }
  }
  std::sort(recs.begin(), recs.end(), [](const Rec &a, const Rec &b) {
    return a.group != b.group ? a.group < b.group : a.key < b.key;
  });
  S->ndof = (int64_t)recs.size();
  S->keys.resize(recs.size());
  dof_of.reserve(recs.size() * 2);
  for (size_t i = 0; i < recs.size(); ++i) {
    S->keys[i] = recs[i].key;
    dof_of[recs[i].key] = (int)i;
  }
  S->nlev = K + p;
  S->level_size.assign(S->nlev, 0);
  for (int l = 0; l < S->nlev; ++l) {
    int64_t c = 0;
    for (const Rec &r : recs) c += r.group <= l;
    S->level_size[l] = c;
  }
  (void)p;
  return FCM_OK;
}

// per leaf: functions (own and ancestors' active modes)
static fcm_status ml_leaf_functions(Builder &B, const std::unordered_map<int64_t, int> &dof_of,
                                    std::vector<int> &fdof, std::vector<int> &fdesc,
                                    std::vector<int64_t> &koff) {
  MlhpState *S = B.S;
  koff.assign(S->nleaf + 1, 0);
  for (int L = 0; L < S->nleaf; ++L) {
    int *lf = &S->h_leaf[7 * L];
    const int k = lf[0];
    lf[4] = (int)fdof.size();
    for (int j = 0; j <= k; ++j) {
      int ej[3] = {lf[1] >> (k - j), lf[2] >> (k - j), lf[3] >> (k - j)};
      for (const auto &t : B.modes) {
        int64_t codes[3];
        B.mode_codes(j, ej, t, codes);
        auto it = dof_of.find(B.key_of(j, codes));
        if (it == dof_of.end()) continue;
        fdof.push_back(it->second);
        fdesc.push_back(j | (t[0] << 4) | (t[1] << 8) | (t[2] << 12));
      }
    }
    lf[5] = (int)fdof.size() - lf[4];
    if (lf[5] > kMlMaxM) {
      set_error("multi-level hp: a leaf has %d functions (limit %d)", lf[5], kMlMaxM);
      return FCM_ERR_ARG;
    }
    S->m_max = std::max(S->m_max, lf[5]);
    if (lf[6] == kMlCut) S->n_cut_leaves++;
    koff[L + 1] = koff[L] + (int64_t)lf[5] * lf[5];
  }
  return FCM_OK;
}

// Schwarz patches of multigrid level l (base-node patches)
static fcm_status ml_patches(Builder &B, int l, const std::vector<int> &fdof,
                             const std::vector<std::vector<int>> &leaves_of_base,
                             const std::vector<std::vector<int>> &leaves_of_dof, MlPatches &P) {
  MlhpState *S = B.S;
  fcm_handle *h = B.h;
  const int d = S->d;
  const int64_t nl = S->level_size[l];
  const LevelGrid &G0 = B.lv[0];
  struct Patch { std::vector<int> idx; std::vector<int> leaves; };
  std::vector<Patch> patches;
  std::vector<int> mark(S->ndof, -1), lmark(S->nleaf, -1);
  int pid = 0;
  for (int v2 = 0; v2 <= (d == 3 ? S->n[2] : 0); ++v2)
    for (int v1 = 0; v1 <= S->n[1]; ++v1)
      for (int v0 = 0; v0 <= S->n[0]; ++v0) {
        Patch pt;
        for (int s = 0; s < (1 << d); ++s) {
          int c[3] = {v0 - (s & 1), v1 - ((s >> 1) & 1), d == 3 ? v2 - ((s >> 2) & 1) : 0};
          if (!G0.in_box(c, d)) continue;
          for (int L : leaves_of_base[G0.lin(c)]) {
            const int *lf = &S->h_leaf[7 * L];
            for (int i = 0; i < lf[5]; ++i) {
              const int dof = fdof[lf[4] + i];
              if (dof < nl && mark[dof] != pid) {
                mark[dof] = pid;
                pt.idx.push_back(dof);
              }
            }
          }
        }
        if (!pt.idx.empty()) {
          std::sort(pt.idx.begin(), pt.idx.end());
          for (int dof : pt.idx)
            for (int L : leaves_of_dof[dof])
              if (lmark[L] != pid) {
                lmark[L] = pid;
                pt.leaves.push_back(L);
              }
          std::sort(pt.leaves.begin(), pt.leaves.end());
          if ((int)pt.idx.size() > kMlMaxPatch) {
            set_error("multi-level hp: a Schwarz patch has %zu functions (limit %d)",
                      pt.idx.size(), kMlMaxPatch);
            return FCM_ERR_ARG;
          }
          patches.push_back(std::move(pt));
        }
        ++pid;
      }
  // order by size, buckets of up to 64 patches padded to a multiple of 32
  std::vector<int> order(patches.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return patches[a].idx.size() < patches[b].idx.size(); });
  P.npatch = (int)patches.size();
  std::vector<int> pidx, pm, plf, pair_leaf, map;
  std::vector<int64_t> poff, pinv, pair_map;
  int64_t inv_off = 0;
  for (size_t b0 = 0; b0 < order.size(); b0 += 64) {
    const size_t b1 = std::min(order.size(), b0 + 64);
    int mb = 0;
    for (size_t t = b0; t < b1; ++t) mb = std::max(mb, (int)patches[order[t]].idx.size());
    mb = (mb + 31) / 32 * 32;
    P.buckets.push_back({inv_off, {(int)(b1 - b0), mb}});
    for (size_t t = b0; t < b1; ++t) {
      const Patch &pt = patches[order[t]];
      poff.push_back((int64_t)pidx.size());
      for (int i = 0; i < mb; ++i) pidx.push_back(i < (int)pt.idx.size() ? pt.idx[i] : -1);
      pm.push_back(mb);
      pm.push_back((int)pt.idx.size());
      pinv.push_back(inv_off);
      inv_off += (int64_t)mb * mb;
      plf.push_back((int)pair_leaf.size());
      plf.push_back((int)pt.leaves.size());
      std::unordered_map<int, int> row;
      row.reserve(pt.idx.size() * 2);
      for (size_t i = 0; i < pt.idx.size(); ++i) row[pt.idx[i]] = (int)i;
      for (int L : pt.leaves) {
        pair_leaf.push_back(L);
        pair_map.push_back((int64_t)map.size());
        const int *lf = &S->h_leaf[7 * L];
        for (int i = 0; i < lf[5]; ++i) {
          auto it = row.find(fdof[lf[4] + i]);
          map.push_back(it == row.end() ? -1 : it->second);
        }
      }
      P.max_mb = std::max(P.max_mb, mb);
    }
  }
  P.inv_doubles = inv_off;
  {
    // per DOF of the level: its patch rows (padding rows carry -1)
    std::vector<int> gptr, gslot;
    gather_csr(pidx, S->level_size[l], gptr, gslot);
    ML_TRY(device_upload(h, &P.pg_ptr, gptr));
    ML_TRY(device_upload(h, &P.pg_slot, gslot));
    ML_TRY(device_alloc(h, &P.pc, pidx.size()));
    P.nrows = (int64_t)pidx.size();
  }
  ML_TRY(device_upload(h, &P.pidx, pidx));
  ML_TRY(device_upload(h, &P.poff, poff));
  ML_TRY(device_upload(h, &P.pm, pm));
  ML_TRY(device_upload(h, &P.pinv, pinv));
  ML_TRY(device_upload(h, &P.plf, plf));
  ML_TRY(device_upload(h, &P.pair_leaf, pair_leaf));
  ML_TRY(device_upload(h, &P.pair_map, pair_map));
  ML_TRY(device_upload(h, &P.map, map));
  ML_TRY(device_alloc(h, &P.inv, (size_t)std::max<int64_t>(1, inv_off)));
  return FCM_OK;
}

fcm_status mlhp_setup(fcm_handle *h) {
  const fcm_problem &pr = h->prob.pr;
  MlhpState *S = new MlhpState();
  h->ml = S;
  S->d = pr.dim;
  S->p = pr.p;
  S->K = pr.refine_levels;
  S->geom = pr.geom;
  Builder B;
  B.h = h;
  B.S = S;
  MlGeo &g = B.g;
  g.d = pr.dim;
  g.p = pr.p;
  g.K = pr.refine_levels;
  g.geom = pr.geom;
  g.nballs = pr.n_balls;
  g.alpha = pr.alpha;
  g.kappa = pr.kappa;
  g.beta = pr.beta;
  g.f_const = pr.f_const;
  g.ngauss = pr.n_gauss;
  g.depth = pr.quad_depth;
  for (int ax = 0; ax < 3; ++ax) {
    S->n[ax] = ax < pr.dim ? pr.n[ax] : 1;
    S->lo[ax] = ax < pr.dim ? pr.lo[ax] : 0.0;
    S->h0[ax] = ax < pr.dim ? (pr.hi[ax] - pr.lo[ax]) / pr.n[ax] : 1.0;
    g.lo[ax] = S->lo[ax];
    g.h0[ax] = S->h0[ax];
  }
  double *dball = nullptr, *dgauss = nullptr;
  ML_TRY(device_upload(h, &dball, h->prob.ball));
  ML_TRY(device_upload(h, &dgauss, h->prob.gsrc));
  g.ball = dball;
  g.gauss = dgauss;
  // modes of an element, axis 0 fastest
  const int np1 = S->p + 1;
  for (int t2 = 0; t2 < (S->d == 3 ? np1 : 1); ++t2)
    for (int t1 = 0; t1 < np1; ++t1)
      for (int t0 = 0; t0 < np1; ++t0) B.modes.push_back({t0, t1, t2});
  B.key_off[0] = 0;
  for (int k = 0; k <= S->K; ++k) {
    int64_t prod = 1;
    for (int ax = 0; ax < 3; ++ax) {
      B.S_ax[k][ax] = ax < S->d ? ((int64_t)(S->n[ax] << k) + 1) * S->p : 1;
      prod *= B.S_ax[k][ax];
    }
    B.key_off[k + 1] = B.key_off[k] + prod;
  }
  ML_TRY(ml_build_tree(B));
  std::unordered_map<int64_t, int> dof_of;
  ML_TRY(ml_number(B, dof_of));
  std::vector<int> fdof, fdesc;
  std::vector<int64_t> koff;
  ML_TRY(ml_leaf_functions(B, dof_of, fdof, fdesc, koff));
  ML_TRY(device_upload(h, &S->leaf, S->h_leaf));
  {
    std::vector<int> gptr, gslot;
    gather_csr(fdof, S->ndof, gptr, gslot);
    ML_TRY(device_upload(h, &S->lg_ptr, gptr));
    ML_TRY(device_upload(h, &S->lg_slot, gslot));
    ML_TRY(device_alloc(h, &S->lc, fdof.size()));
    // level-0 matrix entries: per (i, j) with i, j < n0 the leaf-matrix entries
    // that add to it, in leaf order
    const int n0 = (int)S->level_size[0], n0p = (n0 + 31) / 32 * 32;
    std::vector<std::pair<int64_t, int64_t>> ent;
    for (int L = 0; L < S->nleaf; ++L) {
      const int foff = S->h_leaf[7 * L + 4], m = S->h_leaf[7 * L + 5];
      for (int a = 0; a < m; ++a) {
        const int i = fdof[foff + a];
        if (i >= n0) continue;
        for (int b = 0; b < m; ++b) {
          const int j = fdof[foff + b];
          if (j < n0) ent.push_back({(int64_t)i * n0p + j, koff[L] + (int64_t)a * m + b});
        }
      }
    }
    std::stable_sort(ent.begin(), ent.end(),
                     [](const std::pair<int64_t, int64_t> &x, const std::pair<int64_t, int64_t> &y) {
                       return x.first < y.first;
                     });
    std::vector<int64_t> tgt, src;
    std::vector<int> ptr;
    for (size_t k = 0; k < ent.size(); ++k) {
      if (k == 0 || ent[k].first != ent[k - 1].first) {
        tgt.push_back(ent[k].first);
        ptr.push_back((int)k);
      }
      src.push_back(ent[k].second);
    }
    ptr.push_back((int)ent.size());
    S->n_ce = (int)tgt.size();
    ML_TRY(device_upload(h, &S->ce_tgt, tgt));
    ML_TRY(device_upload(h, &S->ce_ptr, ptr));
    ML_TRY(device_upload(h, &S->ce_src, src));
  }
  ML_TRY(device_upload(h, &S->fdof, fdof));
  ML_TRY(device_upload(h, &S->fdesc, fdesc));
  ML_TRY(device_upload(h, &S->koff, koff));
  ML_TRY(device_alloc(h, &S->Kl, (size_t)koff[S->nleaf]));
  ML_TRY(device_alloc(h, &S->b, (size_t)S->ndof));
  ML_TRY(device_alloc(h, &S->flag, 1));
  // Gauss rule and surface rule
  {
    std::vector<double> x, w, gw;
    gauss_legendre(np1, x, w);
    gw = x;
    gw.insert(gw.end(), w.begin(), w.end());
    ML_TRY(device_upload(h, &S->gx, gw));
    std::vector<double> sp;
    if (pr.beta != 0.0) {
      const int nt = pr.surf_n[0] > 0 ? pr.surf_n[0] : 256;
      const int nph = pr.surf_n[1] > 0 ? pr.surf_n[1] : 512;
      const double *c = h->prob.ball.data();
      const double r = c[3];
      if (S->d == 2) {
        for (int j = 0; j < nph; ++j) {
          const double phi = 2.0 * M_PI * j / nph;
          sp.insert(sp.end(), {c[0] + r * std::cos(phi), c[1] + r * std::sin(phi), 0.0,
                               2.0 * M_PI * r / nph});
        }
      } else {
        std::vector<double> mu, wmu;
        gauss_legendre(nt, mu, wmu);
        for (int i = 0; i < nt; ++i)
          for (int j = 0; j < nph; ++j) {
            const double phi = 2.0 * M_PI * j / nph;
            const double s = std::sqrt(1.0 - mu[i] * mu[i]);
            sp.insert(sp.end(), {s * std::cos(phi) * r + c[0], s * std::sin(phi) * r + c[1],
                                 mu[i] * r + c[2], r * r * wmu[i] * (2.0 * M_PI / nph)});
          }
      }
    }
    S->nsurf = (int)sp.size() / 4;
    ML_TRY(device_upload(h, &S->surf, sp));
  }
  // leaf matrices and load
  if (S->nleaf > 0) {
    MlLeafArgs a;
    a.g = g;
    a.leaf = S->leaf;
    a.koff = S->koff;
    a.fdesc = S->fdesc;
    a.gx = S->gx;
    a.surf = S->surf;
    a.nsurf = S->nsurf;
    a.Kl = S->Kl;
    a.lc = S->lc;
    ml_integrate_kernel<<<S->nleaf, 256, 0, h->stream>>>(a);
    ml_gather_kernel<<<ml_grid(S->ndof), 256, 0, h->stream>>>(S->ndof, S->lg_ptr, S->lg_slot,
                                                              S->lc, S->b);
    FCM_HIP(hipGetLastError());
  }
  // coarse level: dense inverse of A_0
  S->n0 = (int)S->level_size[0];
  S->n0p = (S->n0 + 31) / 32 * 32;
  {
    const size_t nn = (size_t)S->n0p * S->n0p;
    ML_TRY(device_alloc(h, &S->A0, nn));
    std::vector<double> eye(nn, 0.0);
    for (int i = S->n0; i < S->n0p; ++i) eye[(size_t)i * S->n0p + i] = 1.0;
    FCM_HIP(hipMemcpyAsync(S->A0, eye.data(), nn * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
    if (S->n_ce > 0)
      ml_coarse_assemble_kernel<<<(S->n_ce + 255) / 256, 256, 0, h->stream>>>(
          S->n_ce, S->ce_tgt, S->ce_ptr, S->ce_src, S->Kl, S->A0);
    if (S->n0p > kMlMaxPatch) {
      set_error("multi-level hp: %d coarse unknowns (limit %d)", S->n0, kMlMaxPatch);
      return FCM_ERR_ARG;
    }
    double *s1 = nullptr, *s2 = nullptr;
    ML_TRY(pool_alloc((void **)&s1, nn * sizeof(double), h->stream));
    ML_TRY(pool_alloc((void **)&s2, nn * sizeof(double), h->stream));
    ML_TRY(ml_spd_inverse(S->A0, {{0, {1, S->n0p}}}, s1, s2, S->flag, h->stream));
    FCM_HIP(hipStreamSynchronize(h->stream));
    pool_free(s1, h->stream);
    pool_free(s2, h->stream);
  }
  // Schwarz patches of every level >= 1
  std::vector<std::vector<int>> leaves_of_base((size_t)B.lv[0].N[0] * B.lv[0].N[1] * B.lv[0].N[2]);
  std::vector<std::vector<int>> leaves_of_dof(S->ndof);
  for (int L = 0; L < S->nleaf; ++L) {
    const int *lf = &S->h_leaf[7 * L];
    int b[3] = {lf[1] >> lf[0], lf[2] >> lf[0], lf[3] >> lf[0]};
    leaves_of_base[B.lv[0].lin(b)].push_back(L);
    for (int i = 0; i < lf[5]; ++i) leaves_of_dof[fdof[lf[4] + i]].push_back(L);
  }
  S->pl.resize(S->nlev);
  size_t scr_need = 1;
  for (int l = 1; l < S->nlev; ++l) {
    ML_TRY(ml_patches(B, l, fdof, leaves_of_base, leaves_of_dof, S->pl[l]));
    scr_need = std::max(scr_need, (size_t)S->pl[l].inv_doubles);
  }
  double *s1 = nullptr, *s2 = nullptr;
  ML_TRY(pool_alloc((void **)&s1, scr_need * sizeof(double), h->stream));
  ML_TRY(pool_alloc((void **)&s2, scr_need * sizeof(double), h->stream));
  const bool mixed = h->opt.precision == FCM_MIXED;
  for (int l = 1; l < S->nlev; ++l) {
    MlPatches &P = S->pl[l];
    if (P.npatch == 0) continue;
    if (mixed) {
      ML_TRY(device_alloc(h, &P.scal, (size_t)P.nrows));
      ML_TRY(device_alloc(h, &P.norm1, (size_t)P.npatch));
      ML_TRY(device_alloc(h, &P.inv32, (size_t)std::max<int64_t>(1, P.inv_doubles)));
      ML_TRY(device_alloc(h, &P.lo32, (size_t)P.npatch));
    }
    ml_form_blocks_kernel<<<P.npatch, 256, 0, h->stream>>>(P.pm, P.pinv, P.plf, P.pair_leaf,
                                                           P.pair_map, P.map, S->leaf, S->koff,
                                                           S->Kl, P.inv);
    ML_TRY(ml_spd_inverse(P.inv, P.buckets, s1, s2, S->flag, h->stream, P.scal, P.norm1));
    if (mixed) {
      ml_lowprec_kernel<<<P.npatch, 256, 0, h->stream>>>(P.pm, P.pinv, P.poff, P.scal, P.norm1,
                                                         P.inv, P.inv32, P.lo32);
      std::vector<uint8_t> lo(P.npatch);
      FCM_HIP(hipMemcpyAsync(lo.data(), P.lo32, P.npatch, hipMemcpyDeviceToHost, h->stream));
      FCM_HIP(hipStreamSynchronize(h->stream));
      P.n32 = 0;
      for (uint8_t v : lo) P.n32 += v;
    }
  }
  FCM_HIP(hipStreamSynchronize(h->stream));
  pool_free(s1, h->stream);
  pool_free(s2, h->stream);
  FCM_HIP(hipGetLastError());
  // work vectors
  S->vx.assign(S->nlev, nullptr);
  S->vr.assign(S->nlev, nullptr);
  S->vy.assign(S->nlev, nullptr);
  S->vz.assign(S->nlev, nullptr);
  for (int l = 0; l < S->nlev; ++l) {
    const size_t n = (size_t)S->level_size[l];
    ML_TRY(device_alloc(h, &S->vx[l], n));
    ML_TRY(device_alloc(h, &S->vr[l], n));
    ML_TRY(device_alloc(h, &S->vy[l], n));
    ML_TRY(device_alloc(h, &S->vz[l], n));
  }
  ML_TRY(device_alloc(h, &S->cg_r, (size_t)S->ndof));
  ML_TRY(device_alloc(h, &S->cg_z, (size_t)S->ndof));
  ML_TRY(device_alloc(h, &S->cg_p, (size_t)S->ndof));
  ML_TRY(device_alloc(h, &S->cg_q, (size_t)S->ndof));
  ML_TRY(device_alloc(h, &S->red, 2049));   // result, then up to 2048 block partials
  int f = 0;
  FCM_HIP(hipMemcpyAsync(&f, S->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  FCM_HIP(hipStreamSynchronize(h->stream));
  if (f) {
    set_error("multi-level hp: a Schwarz block or the coarse matrix is not positive definite");
    return FCM_ERR_NOT_SPD;
  }
  return FCM_OK;
}

void mlhp_free(fcm_handle *h) {
  delete h->ml;
  h->ml = nullptr;
}

// ------------------------------------------------------------ operators
static void ml_apply(MlhpState *S, int l, const double *x, double *y, hipStream_t s) {
  const int64_t n = S->level_size[l];
  if (S->nleaf > 0)
    ml_apply_kernel<<<S->nleaf, 256, 0, s>>>(S->leaf, S->koff, S->fdof, S->Kl, n, x, S->lc);
  ml_gather_kernel<<<ml_grid(n), 256, 0, s>>>(n, S->lg_ptr, S->lg_slot, S->lc, y);
}

// z = M_l^{-1} r; mixed: patches flagged at setup are applied from FP32 copies
static void ml_smooth(MlhpState *S, int l, const double *r, double *z, hipStream_t s,
                      bool mixed = false) {
  const int64_t n = S->level_size[l];
  const MlPatches &P = S->pl[l];
  const bool lo = mixed && P.inv32;
  if (P.npatch > 0)
    ml_smooth_kernel<<<dim3(P.npatch, (P.max_mb + 63) / 64), 256, 0, s>>>(
        P.pm, P.pinv, P.poff, P.pidx, P.inv, lo ? P.inv32 : nullptr, lo ? P.lo32 : nullptr, r,
        P.pc);
  ml_gather_kernel<<<ml_grid(n), 256, 0, s>>>(n, P.pg_ptr, P.pg_slot, P.pc, z);
}

static void ml_coarse(MlhpState *S, const double *b, double *x, hipStream_t s) {
  if (S->n0 > 0) ml_gemv_kernel<<<(S->n0 + 3) / 4, 256, 0, s>>>(S->A0, S->n0, S->n0p, b, x);
}

// Alg. 1 with the residual recomputed after every smoothing step
static void ml_vcycle(fcm_handle *h, int l, const double *b, double *x, hipStream_t s) {
  MlhpState *S = h->ml;
  if (l == 0) {
    ml_coarse(S, b, x, s);
    return;
  }
  const int64_t n = S->level_size[l], nc = S->level_size[l - 1];
  const double w = h->opt.omega;
  double *r = S->vr[l], *y = S->vy[l], *z = S->vz[l];
  (void)hipMemsetAsync(x, 0, n * sizeof(double), s);
  hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  auto steps = [&](int count) {
    for (int it = 0; it < count; ++it) {
      ml_smooth(S, l, r, z, s, h->opt.precision == FCM_MIXED);
      ml_axpby_kernel<<<ml_grid(n), 256, 0, s>>>(n, w, z, 1.0, x);
      ml_apply(S, l, x, y, s);
      ml_sub_kernel<<<ml_grid(n), 256, 0, s>>>(n, b, y, r);
    }
  };
  steps(h->opt.n_pre);
  ml_vcycle(h, l - 1, r, S->vx[l - 1], s);
  ml_axpby_kernel<<<ml_grid(nc), 256, 0, s>>>(nc, 1.0, S->vx[l - 1], 1.0, x);
  ml_apply(S, l, x, y, s);
  ml_sub_kernel<<<ml_grid(n), 256, 0, s>>>(n, b, y, r);
  steps(h->opt.n_post);
}

static double ml_dot(MlhpState *S, int64_t n, const double *x, const double *y, hipStream_t s) {
  const int nb = ml_grid(n);
  ml_dot_kernel<<<nb, 256, 0, s>>>(n, x, y, S->red + 1);
  ml_sum_kernel<<<1, 64, 0, s>>>(nb, S->red + 1, S->red);
  double v = 0.0;
  hipMemcpyAsync(&v, S->red, sizeof(double), hipMemcpyDeviceToHost, s);
  hipStreamSynchronize(s);
  return v;
}

fcm_status mlhp_sizes(const fcm_handle *h, int *n_levels, int64_t *n_dofs, int64_t *n_padded) {
  const MlhpState *S = h->ml;
  *n_levels = S->nlev;
  for (int l = 0; l < S->nlev; ++l) {
    if (n_dofs) n_dofs[l] = S->level_size[l];
    if (n_padded) n_padded[l] = S->level_size[l];
  }
  return FCM_OK;
}

fcm_status mlhp_dof_keys(const fcm_handle *h, int64_t *keys) {
  const MlhpState *S = h->ml;
  std::memcpy(keys, S->keys.data(), S->keys.size() * sizeof(int64_t));
  return FCM_OK;
}

fcm_status mlhp_rhs(fcm_handle *h, double *b, hipStream_t s) {
  FCM_HIP(hipMemcpyAsync(b, h->ml->b, h->ml->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  return FCM_OK;
}

fcm_status mlhp_apply(fcm_handle *h, int level, const double *x, double *y, hipStream_t s) {
  if (level < 0 || level >= h->ml->nlev) {
    set_error("invalid level");
    return FCM_ERR_ARG;
  }
  ml_apply(h->ml, level, x, y, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status mlhp_smooth(fcm_handle *h, int level, const double *r, double *z, hipStream_t s) {
  if (level < 1 || level >= h->ml->nlev) {
    set_error("invalid level");
    return FCM_ERR_ARG;
  }
  ml_smooth(h->ml, level, r, z, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status mlhp_coarse_solve(fcm_handle *h, const double *b, double *x, hipStream_t s) {
  ml_coarse(h->ml, b, x, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status mlhp_vcycle(fcm_handle *h, const double *r, double *z, hipStream_t s) {
  ml_vcycle(h, h->ml->nlev - 1, r, z, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

// FP64 CG preconditioned by one V-cycle (Section 4), x0 = 0, flexible beta
fcm_status mlhp_pcg(fcm_handle *h, const double *b_in, double *x, fcm_solve_info *info,
                    hipStream_t s) {
  MlhpState *S = h->ml;
  const int64_t n = S->ndof;
  const int top = S->nlev - 1;
  auto t0 = std::chrono::steady_clock::now();
  const double *b = b_in ? b_in : S->b;
  double *r = S->cg_r, *z = S->cg_z, *p = S->cg_p, *q = S->cg_q;
  FCM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  FCM_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  const double nb = std::sqrt(ml_dot(S, n, b, b, s));
  S->hist.assign(1, 1.0);
  int it = 0, status = FCM_OK;
  double rel = nb == 0.0 ? 0.0 : 1.0;
  if (nb > 0.0) {
    ml_vcycle(h, top, r, z, s);
    FCM_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double rz = ml_dot(S, n, r, z, s);
    status = FCM_NOT_CONVERGED;
    while (it < h->opt.max_iter) {
      ml_apply(S, top, p, q, s);
      const double pq = ml_dot(S, n, p, q, s);
      if (!(pq > 0.0) || !std::isfinite(rz)) {
        status = std::isfinite(pq) ? FCM_ERR_BREAKDOWN : FCM_ERR_NAN;
        break;
      }
      const double al = rz / pq;
      ml_axpby_kernel<<<ml_grid(n), 256, 0, s>>>(n, al, p, 1.0, x);
      ml_axpby_kernel<<<ml_grid(n), 256, 0, s>>>(n, -al, q, 1.0, r);
      ++it;
      rel = std::sqrt(ml_dot(S, n, r, r, s)) / nb;
      S->hist.push_back(rel);
      if (!std::isfinite(rel)) {
        status = FCM_ERR_NAN;
        break;
      }
      if (rel < h->opt.rtol) {
        status = FCM_OK;
        break;
      }
      // flexible (Polak-Ribiere) beta: with patch blocks of scaled condition
      // ~1e13 the V-cycle applied in floating point is symmetric only to about
      // 1e-4 relative, and the plain beta then loses the conjugacy it assumes
      const double rzo = ml_dot(S, n, r, z, s);
      ml_vcycle(h, top, r, z, s);
      const double rz2 = ml_dot(S, n, r, z, s);
      ml_axpby_kernel<<<ml_grid(n), 256, 0, s>>>(n, 1.0, z, (rz2 - rzo) / rz, p);
      rz = rz2;
    }
  }
  FCM_HIP(hipGetLastError());
  if (info) {
    info->iterations = it;
    info->rel_res = rel;
    // true residual || b - A x || / || b ||
    ml_apply(S, top, x, q, s);
    ml_sub_kernel<<<ml_grid(n), 256, 0, s>>>(n, b, q, z);
    info->true_rel_res = nb > 0.0 ? std::sqrt(ml_dot(S, n, z, z, s)) / nb : 0.0;
    info->t_setup_ms = h->t_setup_ms;
    info->t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->res_history = S->hist.data();
    info->n_history = (int)S->hist.size();
  }
  return (fcm_status)status;
}

fcm_status mlhp_stats(const fcm_handle *h, fcm_stats *st) {
  const MlhpState *S = h->ml;
  std::memset(st, 0, sizeof(*st));
  st->n_elements = S->nleaf;
  st->n_kept = S->nleaf;
  st->n_cut = S->n_cut_leaves;
  int64_t np = 0, n32 = 0;
  for (int l = 1; l < S->nlev; ++l) {
    np += S->pl[l].npatch;
    n32 += S->pl[l].n32;
  }
  st->n_unique_blocks = np;
  st->n_fp64_blocks = np - n32;
  st->device_bytes = h->bytes;
  st->coarse_blocks = 1;
  st->coarse_block_size = S->n0;
  return FCM_OK;
}

}  // namespace fcm
