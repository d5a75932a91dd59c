// Solve-phase kernels of libfcm (gfx950).
//
// elem_op: y = sum_e P_e M_e P_e^T x for element-structured operators.  It
// serves both the level stiffness apply (M_e = K_e, eq. hierarchicalMatrices:
// level-q rows/columns are the leading block of the order-p element matrix)
// and the elementwise additive Schwarz smoother (M_e = (P_e^T A_q P_e)^{-1},
// eq. AdditiveSchwarz).  Owner computes: one thread per output entry
// (grid point g, plane P) sums the matching rows of the 2^k element
// matrices that touch that DOF, so no atomics or colouring are needed and the
// result is deterministic.  Epilogues fuse the damped update of Section 3.1
// (x += omega * delta), the residual update r -= omega A delta, and the
// prolongation of eq. restrictionoperation (x[:n_{l-1}] += e).
//
// CG: fused vector updates and deterministic two-stage dot products (fixed
// per-block order, then one block sums the partials in a fixed tree).
//
// Coarse: forward/backward block sweeps of the layer-block-tridiagonal p = 1
// system with dense inverted Schur complements.
#include "fcm_internal.hpp"

namespace fcm {

template <typename T>
__global__ __launch_bounds__(256) void elem_op_kernel(Geo g, const int *__restrict__ xoff,
                                                      const int *__restrict__ rows,
                                                      const int *__restrict__ pinfo,
                                                      OpArgs<T> a) {
  const int P = blockIdx.y;
  const int gi = blockIdx.x * 256 + threadIdx.x;
  if (gi >= g.G) return;
  const int gx = gi % g.gn[0];
  const int rest = gi / g.gn[0];
  const int gy = rest % g.gn[1];
  const int gz = rest / g.gn[1];
  const int gc[3] = {gx, gy, gz};
  const int info = pinfo[P], vmask = info & 7, bmask = (info >> 8) & 7;
  bool valid = true;
  for (int ax = 0; ax < g.d; ++ax) {
    if (((bmask >> ax) & 1) && gc[ax] == g.n[ax]) valid = false;
    if ((vmask >> ax) & 1) {
      if (gc[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) valid = false;
      if (gc[ax] == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) valid = false;
    }
  }
  T acc = 0;
  double acc64 = 0.0;
  bool any = false;
  const int ld = a.ld;
  const int nsub = 1 << g.d;
  if (valid) {
    for (int s = 0; s < nsub; ++s) {
      if (s & ~vmask) continue;
      const int ex = gx - (s & 1), ey = gy - ((s >> 1) & 1), ez = gz - ((s >> 2) & 1);
      if (ex < 0 || ey < 0 || ez < 0 || ex >= g.n[0] || ey >= g.n[1] || ez >= g.n[2]) continue;
      const int e = ex + g.n[0] * (ey + g.n[1] * ez);
      const int id = a.mid[e];
      if (id < 0) continue;
      any = true;
      const int row = rows[P * 8 + s];
      const int base = ex + g.gn[0] * (ey + g.gn[1] * ez);
      const T *xb = a.x + base;
      if (a.matU64 && id >= a.nS && (!a.u64flag || a.u64flag[id - a.nS])) {
        // ill-conditioned stored matrix inside the FP32 operator: FP64 entries, FP64 sum
        const double *M = a.matU64 + (size_t)(id - a.nS) * ld * ld + (size_t)row * ld;
        double d0 = 0.0, d1 = 0.0;
        int b = 0;
        for (; b + 1 < a.m_in; b += 2) {
          d0 += M[b] * (double)xb[xoff[b]];
          d1 += M[b + 1] * (double)xb[xoff[b + 1]];
        }
        if (b < a.m_in) d0 += M[b] * (double)xb[xoff[b]];
        acc64 += d0 + d1;
        continue;
      }
      const T *M = (id < a.nS) ? a.matS + (size_t)id * ld * ld
                               : a.matU + (size_t)(id - a.nS) * ld * ld;
      M += (size_t)row * ld;
      T s0 = 0, s1 = 0;
      int b = 0;
      for (; b + 1 < a.m_in; b += 2) {
        s0 += M[b] * xb[xoff[b]];
        s1 += M[b + 1] * xb[xoff[b + 1]];
      }
      if (b < a.m_in) s0 += M[b] * xb[xoff[b]];
      acc += s0 + s1;
    }
  }
  const bool live = valid && any;
  const T val = live ? (T)((double)acc + acc64) : T(0);
  const size_t oi = (size_t)P * g.G + gi;
  if (a.xs) {
    a.out[oi] = val;
    const T xo = a.first ? T(0) : a.xs[oi];
    a.xs[oi] = xo + a.omega * val;
  } else {
    T o = a.scale * val;
    if (a.cvec) o += a.cvec[oi];
    if (!live) o = 0;
    a.out[oi] = o;
  }
  if (a.xp && P < a.nP_e) a.xp[oi] += a.ep[oi];
}

template <typename T>
void launch_elem_op(const Geo &g, const Tables &t, const OpArgs<T> &a, hipStream_t s) {
  dim3 grid((g.G + 255) / 256, a.nP_out);
  elem_op_kernel<T><<<grid, 256, 0, s>>>(g, t.xoff, t.rows, t.pinfo, a);
}
template void launch_elem_op<double>(const Geo &, const Tables &, const OpArgs<double> &,
                                     hipStream_t);
template void launch_elem_op<float>(const Geo &, const Tables &, const OpArgs<float> &,
                                    hipStream_t);

// ------------------------------------------------------------------ vectors
constexpr int kRedThreads = 256;

int dot_blocks(int64_t n) {
  int64_t b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

__device__ inline double block_sum(double v, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kRedThreads) void dot_partial_kernel(const double *x,
                                                                  const double *y, int64_t n,
                                                                  double *partial) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += x[i] * y[i];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

void launch_dot_partial(const double *x, const double *y, int64_t n, double *partial, int nblk,
                        hipStream_t s) {
  dot_partial_kernel<<<nblk, kRedThreads, 0, s>>>(x, y, n, partial);
}

__global__ __launch_bounds__(kRedThreads) void dot_final_kernel(const double *partial, int nblk,
                                                                double *dst) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kRedThreads) s += partial[i];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) *dst = t;
}

void launch_dot_final(const double *partial, int nblk, double *dst, hipStream_t s) {
  dot_final_kernel<<<1, kRedThreads, 0, s>>>(partial, nblk, dst);
}

// Device scalars: 0 rz, 1 pq, 2 alpha, 3 rr, 4 rz_new, 5 beta
__global__ void cg_alpha_kernel(double *sc) { sc[2] = sc[0] / sc[1]; }
void launch_cg_alpha(double *scal, hipStream_t s) { cg_alpha_kernel<<<1, 1, 0, s>>>(scal); }

__global__ __launch_bounds__(kRedThreads) void cg_update_xr_kernel(double *x, double *r,
                                                                   const double *p,
                                                                   const double *q,
                                                                   const double *sc, int64_t n,
                                                                   double *partial) {
  __shared__ double sh[kRedThreads];
  const double al = sc[2];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    x[i] += al * p[i];
    double ri = r[i] - al * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

void launch_cg_update_xr(double *x, double *r, const double *p, const double *q,
                         const double *scal, int64_t n, double *partial, int nblk,
                         hipStream_t s) {
  cg_update_xr_kernel<<<nblk, kRedThreads, 0, s>>>(x, r, p, q, scal, n, partial);
}

__global__ void cg_beta_kernel(double *sc) {
  sc[5] = sc[4] / sc[0];
  sc[0] = sc[4];
}
void launch_cg_beta(double *scal, hipStream_t s) { cg_beta_kernel<<<1, 1, 0, s>>>(scal); }

__global__ void cg_update_p_kernel(double *p, const double *z, const double *sc, int64_t n,
                                   int first) {
  const double be = first ? 0.0 : sc[5];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = first ? z[i] : z[i] + be * p[i];
}

void launch_cg_update_p(double *p, const double *z, const double *scal, int64_t n, int first,
                        hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  cg_update_p_kernel<<<blocks, 256, 0, s>>>(p, z, scal, n, first);
}

__global__ void axpby_kernel(double *y, const double *x, double a, double b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

void launch_axpby(double *y, const double *x, double a, double b, int64_t n, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  axpby_kernel<<<blocks, 256, 0, s>>>(y, x, a, b, n);
}

__global__ void f64_to_f32_kernel(const double *x, float *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void f32_to_f64_kernel(const float *x, double *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}
void launch_f64_to_f32(const double *x, float *y, int64_t n, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  f64_to_f32_kernel<<<blocks, 256, 0, s>>>(x, y, n);
}
void launch_f32_to_f64(const float *x, double *y, int64_t n, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  f32_to_f64_kernel<<<blocks, 256, 0, s>>>(x, y, n);
}

// ------------------------------------------------------------------ coarse
// Block-local row i of block k -> index in the level-0 padded vector, or -1.
__device__ inline int64_t coarse_vec_index(const Geo &g, const Coarse &c, int k, int i) {
  const int lay = c.w * c.PP;
  const int comp = i / lay, rem = i % lay;
  const int lam = rem / c.PP, pt = rem % c.PP;
  const int layer = c.layer0 + k * c.w + lam;
  if (layer >= g.gn[g.d - 1]) return -1;
  return (int64_t)comp * g.G + (int64_t)layer * c.PP + pt;
}

__device__ inline int coarse_nbr_s(const Geo &g, const Coarse &c, int i, int so, int o, int cb,
                                   int *dblk) {
  const int lay = c.w * c.PP;
  int rem = i % lay;
  int lam = rem / c.PP, pt = rem % c.PP;
  int px, py = 0;
  if (g.d == 3) {
    px = pt % g.gn[0];
    py = pt / g.gn[0];
  } else {
    px = pt;
  }
  px += o % 3 - 1;
  if (g.d == 3) py += o / 3 - 1;
  if (px < 0 || px >= g.gn[0]) return -1;
  if (g.d == 3 && (py < 0 || py >= g.gn[1])) return -1;
  int npt = (g.d == 3) ? px + g.gn[0] * py : px;
  int nl = lam + so;
  *dblk = 0;
  if (nl < 0) {
    nl += c.w;
    *dblk = -1;
  } else if (nl >= c.w) {
    nl -= c.w;
    *dblk = 1;
  }
  return cb * lay + nl * c.PP + npt;
}

// Sum of the JS partial products of entry l of the previous step's result.
__device__ inline double red_partials(const double *Pp, int JS, int nb, int l) {
  double s = 0.0;
  for (int t = 0; t < JS; ++t) s += Pp[(size_t)t * nb + l];
  return s;
}

// One sweep step.  mode 0 (forward, block k): v = b_k - B_k u_{k-1}
// (u_{k-1} = sum of previous partials), W_k = v.  mode 1 (backward, block k):
// v = W_k - B_{k+1}^T x_{k+1}, x_{k+1} from `xlast` (block k+1 is the last
// block) or from the partials, which are also written to x.  Then the
// partial products Pcur[js][i] = sum_{j in chunk js} Sinv_k[j][i] v_j.
__global__ __launch_bounds__(256) void coarse_step_kernel(Geo g, Coarse c, int k, int mode,
                                                          const double *b, double *x,
                                                          const double *Pprev, double *Pcur,
                                                          int have_prev, int next_is_last) {
  extern __shared__ double v[];
  const int nb = c.nb, JS = c.JS, CJ = c.CJ;
  const int rt = blockIdx.x, js = blockIdx.y;
  const int j0 = js * CJ, j1 = min(nb, j0 + CJ);
  const int per = 3 * c.no * g.nf;
  const int tid = threadIdx.x;
  for (int j = j0 + tid; j < j1; j += 256) {
    double val;
    const double *st = c.Dst + (size_t)(k * nb + j) * per;
    if (mode == 0) {
      int64_t gi = coarse_vec_index(g, c, k, j);
      val = gi >= 0 ? b[gi] : 0.0;
      if (have_prev) {
        for (int t = 0; t < c.no * g.nf; ++t) {
          double cf = st[t];
          if (cf == 0.0) continue;
          int o = t / g.nf, cb = t % g.nf, db;
          int l = coarse_nbr_s(g, c, j, -1, o, cb, &db);
          if (l < 0 || db != -1) continue;
          val -= cf * red_partials(Pprev, JS, nb, l);
        }
      }
      if (rt == 0) c.W[(size_t)k * nb + j] = val;
    } else {
      val = c.W[(size_t)k * nb + j];
      const double *su = st + 2 * c.no * g.nf;
      for (int t = 0; t < c.no * g.nf; ++t) {
        double cf = su[t];
        if (cf == 0.0) continue;
        int o = t / g.nf, cb = t % g.nf, db;
        int l = coarse_nbr_s(g, c, j, 1, o, cb, &db);
        if (l < 0 || db != 1) continue;
        double xv;
        if (next_is_last) {
          int64_t gi = coarse_vec_index(g, c, k + 1, l);
          xv = gi >= 0 ? x[gi] : 0.0;
        } else {
          xv = red_partials(Pprev, JS, nb, l);
        }
        val -= cf * xv;
      }
      if (rt == 0 && !next_is_last) {
        int64_t gi = coarse_vec_index(g, c, k + 1, j);
        if (gi >= 0) x[gi] = red_partials(Pprev, JS, nb, j);
      }
    }
    v[j - j0] = val;
  }
  __syncthreads();
  // partial GEMV: 64 rows x 4 column groups per workgroup
  __shared__ double red[4][64];
  const int lane = tid & 63, grp = tid >> 6;
  const int i = rt * 64 + lane;
  double acc = 0.0;
  if (i < nb) {
    const double *S = c.Sinv + (size_t)k * nb * nb;
    for (int j = j0 + grp; j < j1; j += 4) acc += S[(size_t)j * nb + i] * v[j - j0];
  }
  red[grp][lane] = acc;
  __syncthreads();
  if (grp == 0 && i < nb) Pcur[(size_t)js * nb + i] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

__global__ void coarse_finish_kernel(Geo g, Coarse c, int k, const double *Pp, double *x) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c.nb) return;
  int64_t gi = coarse_vec_index(g, c, k, j);
  if (gi >= 0) x[gi] = red_partials(Pp, c.JS, c.nb, j);
}

__global__ void fill_zero_kernel(double *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

void coarse_solve_launch(const Geo &g, const Coarse &c, const double *b, double *x,
                         hipStream_t s) {
  const int nb = c.nb;
  // entries outside the blocked system (Dirichlet layers) are zero
  {
    const int64_t n = (int64_t)g.nf * g.G;
    fill_zero_kernel<<<(int)std::min<int64_t>((n + 255) / 256, 1024), 256, 0, s>>>(x, n);
  }
  dim3 grid((nb + 63) / 64, c.JS);
  const size_t shm = (size_t)c.CJ * sizeof(double);
  double *P[2] = {c.P0, c.P1};
  int cur = 0;
  for (int k = 0; k < c.nblk; ++k) {
    coarse_step_kernel<<<grid, 256, shm, s>>>(g, c, k, 0, b, x, P[cur ^ 1], P[cur], k > 0, 0);
    cur ^= 1;
  }
  // last block: x_K = u_K
  coarse_finish_kernel<<<(nb + 255) / 256, 256, 0, s>>>(g, c, c.nblk - 1, P[cur ^ 1], x);
  for (int k = c.nblk - 2; k >= 0; --k) {
    const int next_is_last = (k + 1 == c.nblk - 1);
    coarse_step_kernel<<<grid, 256, shm, s>>>(g, c, k, 1, b, x, P[cur ^ 1], P[cur], 1,
                                              next_is_last);
    cur ^= 1;
  }
  if (c.nblk > 1) coarse_finish_kernel<<<(nb + 255) / 256, 256, 0, s>>>(g, c, 0, P[cur ^ 1], x);
}

}  // namespace fcm
