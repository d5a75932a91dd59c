// Geometric h-levels below the p = 1 level of libfcm (gfx950).
//
// The hierarchy of Section 3.2 ends at p = 1 on the finite cell grid, solved
// exactly; the remark closing Section 3.2 notes that this level can itself be
// coarsened by a standard geometric multigrid.  Here:
//   * h-level 0 is the p = 1 level (vertex functions); its matrix is taken
//     from the element matrices as a 3^d-point stencil per row;
//   * h-level k+1 has ceil(n_k / 2) cells per axis, a cell being kept when
//     one of its 2^d children is; the prolongation P_k is d-linear
//     interpolation (weight prod_ax w(i_ax - 2 V_ax), w(0) = 1, w(+-1) = 1/2,
//     between fine node i and coarse node V), restricted to existing DOFs; a
//     coarse node is a DOF unless it lies on a Dirichlet face or touches no
//     fine DOF; A_{k+1} = P_k^T A_k P_k (Galerkin), again a 3^d-point stencil;
//   * every h-level but the coarsest is smoothed by additive Schwarz with
//     the patchwise blocks of Section 3.3.1 at p = 1 (block v = the DOFs of
//     the vertices of the kept cells around node v, n_f 3^d slots), damped
//     by omega_h = 1 / (c 3^(d-1)) (c = 2 scalar, 3 vector: 1/6, 1/9 in 2D,
//     1/18, 1/27 in 3D; omega_h lambda_max(M^-1 A) is 1.4-1.9) with the
//     residual recomputed (Alg. 1);
//   * the coarsest h-level (at most options.coarse_dense_max DOFs) is solved
//     by a dense inverse.
// Layout: h-level vectors are n_f planes of the level's grid points (axis 0
// fastest), entries of absent DOFs zero; stencil row r holds 3^d x n_f
// entries, offset o = (dx+1) + 3 (dy+1) + 9 (dz+1) major, component minor.
// Every sum is taken in a fixed order (no atomics): results are bitwise
// reproducible.
#include <algorithm>
#include <vector>

#include "fcm_internal.hpp"

namespace fcm {

#define HTRY(x)                  \
  do {                           \
    fcm_status s_ = (x);         \
    if (s_ != FCM_OK) return s_; \
  } while (0)

namespace {

constexpr int kHThreads = 256;
constexpr int kHMaxM = 81;                       // patch slots n_f 3^d (3D elasticity)
constexpr size_t kHScratchDoubles = size_t(48) << 20;  // SPD-inverse scratch budget (384 MiB)

// Grid of one h-level, by value.
struct HG {
  int d, nf, no;      // dimension, fields, stencil offsets 3^d
  int gn[3];
  int64_t G;
};

HG hg_of(const Geo &g, const HLev &L) {
  HG q;
  q.d = g.d;
  q.nf = g.nf;
  q.no = g.d == 3 ? 27 : 9;
  for (int ax = 0; ax < 3; ++ax) q.gn[ax] = L.gn[ax];
  q.G = L.G;
  return q;
}

__host__ __device__ inline int hoff(int o, int ax) {
  return ax == 0 ? o % 3 - 1 : (ax == 1 ? (o / 3) % 3 - 1 : o / 9 - 1);
}

__host__ __device__ inline void hcoords(const HG &q, int64_t pt, int *c) {
  c[0] = (int)(pt % q.gn[0]);
  c[1] = (int)((pt / q.gn[0]) % q.gn[1]);
  c[2] = (int)(pt / ((int64_t)q.gn[0] * q.gn[1]));
}

__host__ __device__ inline int64_t hlin(const HG &q, const int *c) {
  return c[0] + (int64_t)q.gn[0] * (c[1] + (int64_t)q.gn[1] * c[2]);
}

__host__ __device__ inline bool hin(const HG &q, const int *c) {
  bool in = true;
  for (int ax = 0; ax < 3; ++ax) in = in && c[ax] >= 0 && c[ax] < q.gn[ax];
  return in;
}

// -------------------------------------------------------------- kernels
// Galerkin stencil of h-level k+1: row (ci, V), column (cj, U = V + off):
//   sum over fine i near 2V and fine j near both i and 2U of
//   w(i - 2V) S_f[(ci, i)][j - i][cj] w(j - 2U).
__global__ void hgalerkin_kernel(HG f, const int *__restrict__ presf,
                                 const double *__restrict__ Sf, HG c,
                                 const int *__restrict__ presc, double *__restrict__ Sc) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= c.nf * c.G) return;
  const int ci = (int)(row / c.G);
  int V[3];
  hcoords(c, row % c.G, V);
  const int per = c.no * c.nf;
  double *out = Sc + row * per;
  const bool ok = presc[row] != 0;
  for (int K = 0; K < c.no; ++K) {
    int U[3] = {V[0] + hoff(K, 0), V[1] + hoff(K, 1), V[2] + (c.d == 3 ? hoff(K, 2) : 0)};
    const bool inU = hin(c, U);
    for (int cj = 0; cj < c.nf; ++cj) {
      double sum = 0.0;
      if (ok && inU && presc[cj * c.G + hlin(c, U)]) {
        for (int io = 0; io < f.no; ++io) {
          int i[3] = {2 * V[0] + hoff(io, 0), 2 * V[1] + hoff(io, 1),
                      2 * V[2] + (f.d == 3 ? hoff(io, 2) : 0)};
          if (!hin(f, i)) continue;
          const int64_t fr = ci * f.G + hlin(f, i);
          if (!presf[fr]) continue;
          double wi = 1.0;
          for (int ax = 0; ax < f.d; ++ax) wi *= hoff(io, ax) == 0 ? 1.0 : 0.5;
          const double *Srow = Sf + fr * (f.no * f.nf);
          for (int jo = 0; jo < f.no; ++jo) {
            double wj = 1.0;
            bool near = true;
            for (int ax = 0; ax < f.d; ++ax) {
              const int rel = i[ax] + hoff(jo, ax) - 2 * U[ax];
              near = near && rel >= -1 && rel <= 1;
              wj *= rel == 0 ? 1.0 : 0.5;
            }
            if (near) sum += wi * Srow[jo * f.nf + cj] * wj;
          }
        }
      }
      out[K * c.nf + cj] = sum;
    }
  }
}

// out = cvec + scale * A x on one h-level (out may be cvec, not x); rows of
// absent DOFs are set to zero.
__global__ void happly_kernel(HG q, const double *__restrict__ S, const int *__restrict__ pres,
                              const double *__restrict__ x, const double *cvec, double scale,
                              double *out) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= q.nf * q.G) return;
  if (!pres[row]) {
    out[row] = 0.0;
    return;
  }
  int u[3];
  hcoords(q, row % q.G, u);
  const double *Srow = S + row * (q.no * q.nf);
  double y = 0.0;
  for (int o = 0; o < q.no; ++o) {
    int v[3] = {u[0] + hoff(o, 0), u[1] + hoff(o, 1), u[2] + (q.d == 3 ? hoff(o, 2) : 0)};
    if (!hin(q, v)) continue;
    const int64_t pv = hlin(q, v);
    for (int cj = 0; cj < q.nf; ++cj) y += Srow[o * q.nf + cj] * x[cj * q.G + pv];
  }
  out[row] = (cvec ? cvec[row] : 0.0) + scale * y;
}

// b_c = P^T r_f.
__global__ void hrestrict_kernel(HG f, const double *__restrict__ rf, HG c,
                                 const int *__restrict__ presc, double *__restrict__ bc) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= c.nf * c.G) return;
  double sum = 0.0;
  if (presc[row]) {
    const int ci = (int)(row / c.G);
    int V[3];
    hcoords(c, row % c.G, V);
    for (int io = 0; io < f.no; ++io) {
      int i[3] = {2 * V[0] + hoff(io, 0), 2 * V[1] + hoff(io, 1),
                  2 * V[2] + (f.d == 3 ? hoff(io, 2) : 0)};
      if (!hin(f, i)) continue;
      double w = 1.0;
      for (int ax = 0; ax < f.d; ++ax) w *= hoff(io, ax) == 0 ? 1.0 : 0.5;
      sum += w * rf[ci * f.G + hlin(f, i)];
    }
  }
  bc[row] = sum;
}

// e_f = P x_c (zero at absent fine DOFs), x_f += e_f.
__global__ void hprolong_kernel(HG c, const double *__restrict__ xc, HG f,
                                const int *__restrict__ presf, double *__restrict__ xf,
                                double *__restrict__ ef) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= f.nf * f.G) return;
  if (!presf[row]) {
    ef[row] = 0.0;
    return;
  }
  const int cc = (int)(row / f.G);
  int i[3];
  hcoords(f, row % f.G, i);
  // per axis: one coarse node (weight 1) for even i, two (1/2 each) for odd i
  int lo[3], cnt[3];
  for (int ax = 0; ax < 3; ++ax) {
    const bool odd = ax < f.d && (i[ax] & 1);
    lo[ax] = odd ? (i[ax] - 1) / 2 : i[ax] / 2;
    cnt[ax] = odd ? 2 : 1;
  }
  double e = 0.0;
  for (int b2 = 0; b2 < cnt[2]; ++b2)
    for (int b1 = 0; b1 < cnt[1]; ++b1)
      for (int b0 = 0; b0 < cnt[0]; ++b0) {
        int V[3] = {lo[0] + b0, lo[1] + b1, lo[2] + b2};
        if (!hin(c, V)) continue;
        const double w = (cnt[0] == 2 ? 0.5 : 1.0) * (cnt[1] == 2 ? 0.5 : 1.0) *
                         (cnt[2] == 2 ? 0.5 : 1.0);
        e += w * xc[cc * c.G + hlin(c, V)];
      }
  xf[row] += e;
  ef[row] = e;
}

// Patch blocks: B[p][a][b] = A entry of slots a, b (identity on absent slots).
// Slot s = c 3^d + o is component c of the node v + off(o).
__global__ void hform_kernel(HG q, const double *__restrict__ S, const int *__restrict__ pmem,
                             int np, int m, double *__restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)np * m) return;
  const int p = (int)(t / m), a = (int)(t % m);
  const int ia = pmem[(int64_t)p * m + a];
  const int ca = a / q.no, oa = a % q.no;
  double *Brow = B + ((int64_t)p * m + a) * m;
  for (int b = 0; b < m; ++b) {
    const int ib = pmem[(int64_t)p * m + b];
    double v = a == b ? 1.0 : 0.0;
    if (ia >= 0 && ib >= 0) {
      const int cb = b / q.no, ob = b % q.no;
      int o = 0, stride = 1;
      bool near = true;
      for (int ax = 0; ax < q.d; ++ax) {
        const int rel = hoff(ob, ax) - hoff(oa, ax);
        near = near && rel >= -1 && rel <= 1;
        o += (rel + 1) * stride;
        stride *= 3;
      }
      v = near ? S[(int64_t)ia * (q.no * q.nf) + o * q.nf + cb] : 0.0;
    }
    Brow[b] = v;
  }
}

// Y[p] = B[p] x[slots of p]: one wave per patch; B is symmetric, so lane j
// forms y_j = sum_i B[i][j] x_i from coalesced rows.
__global__ __launch_bounds__(64) void hpatch_kernel(const double *__restrict__ in,
                                                    const int *__restrict__ pmem,
                                                    const double *__restrict__ B, int m,
                                                    double *__restrict__ Y) {
  __shared__ double xs[kHMaxM];
  const int p = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < m; i += 64) {
    const int idx = pmem[(int64_t)p * m + i];
    xs[i] = idx >= 0 ? in[idx] : 0.0;
  }
  __syncthreads();
  const double *Bp = B + (int64_t)p * m * m;
  for (int j = lane; j < m; j += 64) {
    double y = 0.0;
    for (int i = 0; i < m; ++i) y += Bp[(int64_t)i * m + j] * xs[i];
    Y[(int64_t)p * m + j] = y;
  }
}

// Owner gather of the patch products with the smoother epilogue:
// dl = sum over the patches v = u - off(o) of slot (c, o); x = (first ? 0 :
// x) + omega dl.  A slot that is not a member of its patch holds an exact 0.
__global__ void hgather_kernel(HG q, const double *__restrict__ Y, const int *__restrict__ pidx,
                               const int *__restrict__ pres, int m, double omega, int first,
                               double *__restrict__ dl, double *__restrict__ x) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= q.nf * q.G) return;
  double delta = 0.0;
  if (pres[row]) {
    const int c = (int)(row / q.G);
    int u[3];
    hcoords(q, row % q.G, u);
    for (int o = 0; o < q.no; ++o) {
      int v[3] = {u[0] - hoff(o, 0), u[1] - hoff(o, 1), u[2] - (q.d == 3 ? hoff(o, 2) : 0)};
      if (!hin(q, v)) continue;
      const int pv = pidx[hlin(q, v)];
      if (pv >= 0) delta += Y[(int64_t)pv * m + c * q.no + o];
    }
  }
  dl[row] = delta;
  x[row] = (first ? 0.0 : x[row]) + omega * delta;
}

// Dense matrix of the coarsest h-level over its DOFs didx.
__global__ void hdense_form_kernel(HG q, const double *__restrict__ S,
                                   const int *__restrict__ didx, int nd, double *__restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nd * nd) return;
  const int a = (int)(t / nd), b = (int)(t % nd);
  const int ia = didx[a], ib = didx[b];
  const int cb = (int)(ib / q.G);
  int na[3], nb[3];
  hcoords(q, ia % q.G, na);
  hcoords(q, ib % q.G, nb);
  int o = 0, stride = 1;
  bool near = true;
  for (int ax = 0; ax < q.d; ++ax) {
    const int rel = nb[ax] - na[ax];
    near = near && rel >= -1 && rel <= 1;
    o += (rel + 1) * stride;
    stride *= 3;
  }
  A[t] = near ? S[(int64_t)ia * (q.no * q.nf) + o * q.nf + cb] : 0.0;
}

// x[didx[i]] = sum_j Ainv[i][j] b[didx[j]]: one wave per row, lanes over j,
// a fixed-order wave reduction.
__global__ __launch_bounds__(256) void hdense_solve_kernel(const double *__restrict__ Ainv,
                                                           const int *__restrict__ didx, int nd,
                                                           const double *__restrict__ b,
                                                           double *__restrict__ x) {
  const int row = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (row >= nd) return;
  const double *Ar = Ainv + (int64_t)row * nd;
  double s = 0.0;
  for (int j = lane; j < nd; j += 64) s += Ar[j] * b[didx[j]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[didx[row]] = s;
}

inline unsigned nblocks(int64_t n, int t = kHThreads) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------ host tables
int64_t lin3(const int *gn, const int *c) {
  return c[0] + (int64_t)gn[0] * (c[1] + (int64_t)gn[1] * c[2]);
}

}  // namespace

fcm_status hmg_alloc(fcm_handle *h) {
  const Geo &g = h->geo;
  const int d = g.d, nf = g.nf, no = d == 3 ? 27 : 9, m = nf * no;
  HMG *H = new HMG;
  h->hmg = H;
  H->m = m;
  const int dense_max = h->opt.coarse_dense_max > 0 ? h->opt.coarse_dense_max : 2048;
  // kept cells and DOF presence of every h-level, on the host
  std::vector<std::vector<uint8_t>> kept;
  std::vector<std::vector<int>> pres;
  std::vector<int> n0(3, 1);
  for (int ax = 0; ax < d; ++ax) n0[ax] = g.n[ax];
  {
    std::vector<uint8_t> k0(g.E);
    for (int e = 0; e < g.E; ++e) k0[e] = h->h_state[e] != kVoid;
    kept.push_back(k0);
  }
  auto fill_geom = [&](HLev &L, const int *n) {
    L.G = 1;
    for (int ax = 0; ax < 3; ++ax) {
      L.n[ax] = ax < d ? n[ax] : 1;
      L.gn[ax] = ax < d ? n[ax] + 1 : 1;
      L.G *= L.gn[ax];
    }
    L.len = nf * L.G;
  };
  fill_geom(H->lev[0], n0.data());
  {
    // a vertex DOF exists unless on a Dirichlet face, if one of its cells is kept
    const HLev &L = H->lev[0];
    std::vector<int> p0(L.len, 0);
    for (int64_t pt = 0; pt < L.G; ++pt) {
      int c[3] = {(int)(pt % L.gn[0]), (int)((pt / L.gn[0]) % L.gn[1]),
                  (int)(pt / ((int64_t)L.gn[0] * L.gn[1]))};
      bool ok = true;
      for (int ax = 0; ax < d; ++ax) {
        if (c[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) ok = false;
        if (c[ax] == L.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) ok = false;
      }
      bool any = false;
      for (int s = 0; ok && s < (1 << d); ++s) {
        int e[3] = {c[0] - (s & 1), c[1] - ((s >> 1) & 1), c[2] - ((s >> 2) & 1)};
        bool in = true;
        for (int ax = 0; ax < 3; ++ax) in = in && e[ax] >= 0 && e[ax] < L.n[ax];
        if (in && kept[0][lin3(L.n, e)]) any = true;
      }
      if (ok && any)
        for (int cc = 0; cc < nf; ++cc) p0[cc * L.G + pt] = 1;
    }
    pres.push_back(p0);
  }
  // coarsen while the level has more than dense_max DOFs and an axis to halve
  int J = 0;
  while (true) {
    HLev &F = H->lev[J];
    int64_t nd = 0;
    for (int v : pres[J]) nd += v;
    F.ndof = (int)nd;
    bool halvable = false;
    for (int ax = 0; ax < d; ++ax) halvable = halvable || F.n[ax] > 1;
    if (nd <= dense_max || !halvable || J + 1 >= kMaxH) break;
    HLev &C = H->lev[J + 1];
    int nc[3] = {1, 1, 1};
    for (int ax = 0; ax < d; ++ax) nc[ax] = (F.n[ax] + 1) / 2;
    fill_geom(C, nc);
    std::vector<uint8_t> kc((size_t)C.n[0] * C.n[1] * C.n[2], 0);
    for (int e2 = 0; e2 < F.n[2]; ++e2)
      for (int e1 = 0; e1 < F.n[1]; ++e1)
        for (int e0 = 0; e0 < F.n[0]; ++e0) {
          const int e[3] = {e0, e1, e2}, ec[3] = {e0 / 2, e1 / 2, e2 / 2};
          if (kept[J][lin3(F.n, e)]) kc[lin3(C.n, ec)] = 1;
        }
    kept.push_back(kc);
    std::vector<int> pc(C.len, 0);
    for (int64_t pt = 0; pt < C.G; ++pt) {
      int V[3] = {(int)(pt % C.gn[0]), (int)((pt / C.gn[0]) % C.gn[1]),
                  (int)(pt / ((int64_t)C.gn[0] * C.gn[1]))};
      bool face = false;
      for (int ax = 0; ax < d; ++ax) {
        if (V[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) face = true;
        if (2 * V[ax] == F.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) face = true;
      }
      if (face) continue;
      for (int cc = 0; cc < nf; ++cc) {
        bool any = false;
        for (int io = 0; io < no && !any; ++io) {
          int i[3] = {2 * V[0] + hoff(io, 0), 2 * V[1] + hoff(io, 1),
                      2 * V[2] + (d == 3 ? hoff(io, 2) : 0)};
          bool in = true;
          for (int ax = 0; ax < 3; ++ax) in = in && i[ax] >= 0 && i[ax] < F.gn[ax];
          if (in && pres[J][cc * F.G + lin3(F.gn, i)]) any = true;
        }
        if (any) pc[cc * C.G + pt] = 1;
      }
    }
    pres.push_back(pc);
    ++J;
  }
  H->J = J;
  // device tables and buffers
  size_t max_chunk = 1;
  for (int k = 0; k <= J; ++k) {
    HLev &L = H->lev[k];
    HTRY(device_upload(h, &L.pres, pres[k]));
    HTRY(device_alloc(h, &L.S, (size_t)L.len * no * nf));
    if (k >= 1) {
      HTRY(device_alloc(h, &L.x, (size_t)L.len));
      HTRY(device_alloc(h, &L.b, (size_t)L.len));
    }
    if (k == J) break;
    HTRY(device_alloc(h, &L.r, (size_t)L.len));
    HTRY(device_alloc(h, &L.dl, (size_t)L.len));
    HTRY(device_alloc(h, &L.e, (size_t)L.len));
    // patches: nodes with a kept cell around them and a DOF among the slots
    std::vector<int> pidx(L.G, -1), pmem;
    for (int64_t pt = 0; pt < L.G; ++pt) {
      int v[3] = {(int)(pt % L.gn[0]), (int)((pt / L.gn[0]) % L.gn[1]),
                  (int)(pt / ((int64_t)L.gn[0] * L.gn[1]))};
      std::vector<int> mem(m, -1);
      bool any = false;
      for (int s = 0; s < (1 << d); ++s) {
        int e[3] = {v[0] - (s & 1), v[1] - ((s >> 1) & 1), v[2] - ((s >> 2) & 1)};
        bool in = true;
        for (int ax = 0; ax < 3; ++ax) in = in && e[ax] >= 0 && e[ax] < L.n[ax];
        if (!in || !kept[k][lin3(L.n, e)]) continue;
        for (int t = 0; t < (1 << d); ++t) {
          int u[3] = {e[0] + (t & 1), e[1] + ((t >> 1) & 1), e[2] + ((t >> 2) & 1)};
          int o = 0, stride = 1;
          for (int ax = 0; ax < d; ++ax) {
            o += (u[ax] - v[ax] + 1) * stride;
            stride *= 3;
          }
          const int64_t ul = lin3(L.gn, u);
          for (int cc = 0; cc < nf; ++cc)
            if (pres[k][cc * L.G + ul]) {
              mem[cc * no + o] = (int)(cc * L.G + ul);
              any = true;
            }
        }
      }
      if (!any) continue;
      pidx[pt] = L.np++;
      pmem.insert(pmem.end(), mem.begin(), mem.end());
    }
    HTRY(device_upload(h, &L.pidx, pidx));
    HTRY(device_upload(h, &L.pmem, pmem));
    HTRY(device_alloc(h, &L.Binv, (size_t)std::max(1, L.np) * m * m));
    HTRY(device_alloc(h, &L.Y, (size_t)std::max(1, L.np) * m));
    max_chunk = std::max(max_chunk, (size_t)L.np);
  }
  // coarsest level: dense inverse over its DOFs
  {
    const HLev &L = H->lev[J];
    std::vector<int> didx;
    for (int64_t r = 0; r < L.len; ++r)
      if (pres[J][r]) didx.push_back((int)r);
    H->nd = (int)didx.size();
    HTRY(device_upload(h, &H->didx, didx));
    HTRY(device_alloc(h, &H->Ainv, (size_t)std::max(1, H->nd) * std::max(1, H->nd)));
  }
  // scratch of the batched SPD inverse: patches in chunks within the budget
  const size_t per = spd_inverse_scratch_doubles(m, 1);
  const size_t chunk = std::max<size_t>(1, std::min(max_chunk, kHScratchDoubles / per));
  H->scr_doubles = std::max(spd_inverse_scratch_doubles(m, (int)chunk),
                            spd_inverse_scratch_doubles(std::max(1, H->nd), 1));
  fcm_status st = pool_alloc((void **)&h->co_scr, H->scr_doubles * sizeof(double), h->stream);
  if (st != FCM_OK) return st;
  return FCM_OK;
}

fcm_status hmg_launch(fcm_handle *h, hipStream_t cs) {
  const Geo &g = h->geo;
  HMG *H = h->hmg;
  const int m = H->m;
  const HLev &L0 = H->lev[0];
  launch_hstencil0(g, h->tab, h->kmat, h->Kref64, h->Kcut64, L0.pres, L0.S, cs);
  for (int k = 0; k < H->J; ++k) {
    const HLev &F = H->lev[k], &C = H->lev[k + 1];
    hgalerkin_kernel<<<nblocks(C.len, 128), 128, 0, cs>>>(hg_of(g, F), F.pres, F.S,
                                                           hg_of(g, C), C.pres, C.S);
  }
  const size_t per = spd_inverse_scratch_doubles(m, 1);
  for (int k = 0; k < H->J; ++k) {
    const HLev &L = H->lev[k];
    if (L.np == 0) continue;
    hform_kernel<<<nblocks((int64_t)L.np * m), kHThreads, 0, cs>>>(hg_of(g, L), L.S, L.pmem, L.np,
                                                                  m, L.Binv);
    int chunk = (int)std::max<size_t>(1, std::min<size_t>(L.np, H->scr_doubles / per));
    while (chunk > 1 && spd_inverse_scratch_doubles(m, chunk) > H->scr_doubles) --chunk;
    for (int p0 = 0; p0 < L.np; p0 += chunk) {
      const int cnt = std::min(chunk, L.np - p0);
      spd_inverse_batched(L.Binv + (size_t)p0 * m * m, m, cnt, h->co_scr, h->dflag_co, nullptr,
                          cs);
    }
  }
  if (H->nd > 0) {
    const HLev &L = H->lev[H->J];
    hdense_form_kernel<<<nblocks((int64_t)H->nd * H->nd), kHThreads, 0, cs>>>(
        hg_of(g, L), L.S, H->didx, H->nd, H->Ainv);
    spd_inverse_batched(H->Ainv, H->nd, 1, h->co_scr, h->dflag_co, nullptr, cs);
  }
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

namespace {

void hsmooth_launch(const fcm_handle *h, int k, const double *in, double *dl, double *x,
                    double omega, int first, hipStream_t s) {
  const HMG *H = h->hmg;
  const HLev &L = H->lev[k];
  const HG q = hg_of(h->geo, L);
  if (L.np > 0) hpatch_kernel<<<L.np, 64, 0, s>>>(in, L.pmem, L.Binv, H->m, L.Y);
  hgather_kernel<<<nblocks(L.len), kHThreads, 0, s>>>(q, L.Y, L.pidx, L.pres, H->m, omega, first,
                                                      dl, x);
}

void happly_launch(const fcm_handle *h, int k, const double *x, const double *cvec,
                   double scale, double *out, hipStream_t s) {
  const HLev &L = h->hmg->lev[k];
  happly_kernel<<<nblocks(L.len), kHThreads, 0, s>>>(hg_of(h->geo, L), L.S, L.pres, x, cvec,
                                                     scale, out);
}

void hcycle(const fcm_handle *h, int k, const double *b, double *x, hipStream_t s) {
  const HMG *H = h->hmg;
  const HLev &L = H->lev[k];
  if (k == H->J) {
    if (H->nd > 0)
      hdense_solve_kernel<<<(H->nd + 3) / 4, 256, 0, s>>>(H->Ainv, H->didx, H->nd, b, x);
    return;
  }
  const double w = 1.0 / ((h->geo.nf == 1 ? 2.0 : 3.0) * (h->geo.d == 3 ? 9.0 : 3.0));
  const int npre = h->opt.n_pre, npost = h->opt.n_post;
  // pre-smoothing: x = 0 + w M^-1 b, r = b - w A dl, then x += w M^-1 r, ...
  if (npre == 0) {
    launch_copy<double>(L.r, b, L.len, s);
    launch_copy<double>(x, nullptr, L.len, s);
  }
  for (int it = 0; it < npre; ++it) {
    const double *in = it == 0 ? b : L.r;
    hsmooth_launch(h, k, in, L.dl, x, w, it == 0, s);
    happly_launch(h, k, L.dl, in, -w, L.r, s);
  }
  // coarse-grid correction
  const HLev &C = H->lev[k + 1];
  const HG f = hg_of(h->geo, L), c = hg_of(h->geo, C);
  hrestrict_kernel<<<nblocks(C.len), kHThreads, 0, s>>>(f, L.r, c, C.pres, C.b);
  hcycle(h, k + 1, C.b, C.x, s);
  hprolong_kernel<<<nblocks(L.len), kHThreads, 0, s>>>(c, C.x, f, L.pres, x, L.e);
  happly_launch(h, k, L.e, L.r, -1.0, L.r, s);
  for (int it = 0; it < npost; ++it) {
    hsmooth_launch(h, k, L.r, L.dl, x, w, 0, s);
    if (it + 1 < npost) happly_launch(h, k, L.dl, L.r, -w, L.r, s);
  }
}

}  // namespace

void hmg_cycle(fcm_handle *h, const double *b, double *x, hipStream_t s) { hcycle(h, 0, b, x, s); }

fcm_status hmg_apply(fcm_handle *h, int k, const double *x, double *y, hipStream_t s) {
  if (!h->hmg || k < 0 || k > h->hmg->J) {
    set_error("h-level %d does not exist", k);
    return FCM_ERR_ARG;
  }
  happly_launch(h, k, x, nullptr, 1.0, y, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status hmg_smooth(fcm_handle *h, int k, const double *r, double *z, hipStream_t s) {
  if (!h->hmg || k < 0 || k >= h->hmg->J) {
    set_error("h-level %d has no smoother", k);
    return FCM_ERR_ARG;
  }
  hsmooth_launch(h, k, r, z, h->hmg->lev[k].e, 1.0, 1, s);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

double hmg_cycle_bytes(const fcm_handle *h) {
  const HMG *H = h->hmg;
  if (!H) return 0.0;
  const int no = h->geo.d == 3 ? 27 : 9, nf = h->geo.nf;
  const double steps = h->opt.n_pre + h->opt.n_post;
  double bytes = 8.0 * H->nd * (H->nd + 2.0);
  for (int k = 0; k < H->J; ++k) {
    const HLev &L = H->lev[k];
    const double stencil = 8.0 * L.len * no * nf + 24.0 * L.len;
    const double patches = 8.0 * L.np * H->m * (H->m + 2.0) + 24.0 * L.len;
    bytes += steps * (patches + stencil) + stencil;   // smoothing, correction residual
  }
  return bytes;
}

}  // namespace fcm
