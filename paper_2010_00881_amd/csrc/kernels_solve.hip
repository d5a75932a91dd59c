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
#include <type_traits>

#include "fcm_internal.hpp"

namespace fcm {

// Phase A: stored matrices (cut stiffness, unique Schwarz inverses).  One wave
// per matrix streams it row by row with lanes over the output index (the
// matrices are symmetric, so row b holds column b contiguously) and writes
// Y[sid][a] = sum_b M[a][b] x_e[b] in FP64.  In the mixed form the smoother
// streams FP32 copies of the well-conditioned inverses (matU32).
template <typename M>
__device__ inline void stored_rows(const M *Mb, int ld, int m_in, const double *xw, int row,
                                   double &out) {
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  const M *Mr = Mb + row;
  int b = 0;
  // 16 independent coalesced loads in flight per lane (lanes = rows)
#pragma unroll 4
  for (; b + 3 < m_in; b += 4) {
    c0 += (double)Mr[(size_t)b * ld] * xw[b];
    c1 += (double)Mr[(size_t)(b + 1) * ld] * xw[b + 1];
    c2 += (double)Mr[(size_t)(b + 2) * ld] * xw[b + 2];
    c3 += (double)Mr[(size_t)(b + 3) * ld] * xw[b + 3];
  }
  for (; b < m_in; ++b) c0 += (double)Mr[(size_t)b * ld] * xw[b];
  out = (c0 + c1) + (c2 + c3);
}

template <typename T>
__device__ void stored_gemv_wg(Geo g, const int *__restrict__ xoff, OpArgs<T> a, int wg,
                               double *scratch) {
  double(*xs)[kMaxStoredIn] = reinterpret_cast<double(*)[kMaxStoredIn]>(scratch);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sid = wg * 4 + wave;
  const bool active = sid < a.nstored;
  if (active) {
    const int e = a.selem[sid];
    const int ex = e % g.n[0], r = e / g.n[0];
    const int base = ex + g.gn[0] * ((r % g.n[1]) + g.gn[1] * (r / g.n[1]));
    for (int b = lane; b < a.m_in; b += 64) xs[wave][b] = (double)a.x[base + xoff[b]];
  }
  __syncthreads();
  if (!active) return;
  const int ld = a.ld;
  const bool lo = a.matU32 && !(a.u64flag && a.u64flag[sid]);
  const size_t off = (size_t)sid * ld * ld;
  const double *xw = xs[wave];
  for (int a0 = 0; a0 < a.m_out; a0 += 64) {
    const int row = a0 + lane;
    if (row >= a.m_out) break;
    double y;
    if (lo)
      stored_rows<float>(a.matU32 + off, ld, a.m_in, xw, row, y);
    else
      stored_rows<T>(a.matU + off, ld, a.m_in, xw, row, y);
    a.Y[(size_t)sid * a.m_out + row] = y;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void stored_gemv_kernel(Geo g, const int *__restrict__ xoff,
                                                          OpArgs<T> a) {
  __shared__ double xs[4 * kMaxStoredIn];
  stored_gemv_wg<T>(g, xoff, a, blockIdx.x, xs);
}

// Phase B: elements with a shared matrix (K_ref, Schwarz classes).  One thread
// per element computes Ys[a][e] = sum_b M[a][b] x_e[b] for all output rows;
// the matrix is wave-uniform (one pass per distinct class present in the
// wave), so its rows come through scalar loads and every gathered x value
// feeds kRows FMAs.  TM is the matrix / accumulation type (FP64 for the
// residual of the FP32 V-cycle, where the sum over elements must cancel).
constexpr int kRows = 32;
constexpr int kCols = 32;

template <typename T, typename TM>
__global__ __launch_bounds__(256) void shared_elem_kernel(Geo g, const int *__restrict__ xoff,
                                                          const TM *__restrict__ matS,
                                                          OpArgs<T> a, TM *__restrict__ Ys) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const bool in = e < g.E;
  const int id = in ? a.mid[e] : -1;
  bool todo = id >= 0 && id < a.nS;
  const int ex = e % g.n[0], r = e / g.n[0];
  const int base = ex + g.gn[0] * ((r % g.n[1]) + g.gn[1] * (r / g.n[1]));
  const T *xb = a.x + base;
  const int ld = a.ld;
  for (;;) {
    const unsigned long long msk = __ballot(todo);
    if (msk == 0ull) break;
    const int first = __ffsll((long long)msk) - 1;
    const int id0 = __builtin_amdgcn_readfirstlane(__shfl(id, first));
    const bool mine = todo && id == id0;
    todo = todo && !mine;
    const TM *M0 = matS + (size_t)id0 * ld * ld;
    for (int a0 = 0; a0 < a.m_out; a0 += kRows) {
      TM acc[kRows];
#pragma unroll
      for (int rr = 0; rr < kRows; ++rr) acc[rr] = 0;
      for (int b0 = 0; b0 < a.m_in; b0 += kCols) {
        TM xv[kCols];
#pragma unroll
        for (int bb = 0; bb < kCols; ++bb)
          xv[bb] = (mine && b0 + bb < a.m_in) ? (TM)xb[xoff[b0 + bb]] : TM(0);
#pragma unroll
        for (int rr = 0; rr < kRows; ++rr) {
          if (a0 + rr >= a.m_out) break;
          const TM *Mr = M0 + (size_t)(a0 + rr) * ld + b0;
          TM sum = 0;
#pragma unroll
          for (int bb = 0; bb < kCols; ++bb)
            if (b0 + bb < a.m_in) sum += Mr[bb] * xv[bb];
          acc[rr] += sum;
        }
      }
      if (mine) {
#pragma unroll
        for (int rr = 0; rr < kRows; ++rr)
          if (a0 + rr < a.m_out) Ys[(size_t)(a0 + rr) * g.E + e] = acc[rr];
      }
    }
  }
}

// Phase B on the matrix cores (element matrices up to 64 x 64).  A wave takes
// 32 (FP32) or 16 (FP64) consecutive elements and computes Y = M X with
// v_mfma_f32_32x32x2f32 / v_mfma_f64_16x16x4f64: A = M read column-wise
// (M is symmetric, so column k is row k and the read is coalesced over the
// lanes' row index), B = the gathered element vectors x_e.  Lane layouts
// (gfx950): 32x32x2 f32 -- lane l supplies A[l%32][l/32] and B[l/32][l%32],
// holds D[8(j/4) + 4(l/32) + j%4][l%32] in register j; 16x16x4 f64 -- lane l
// supplies A[l%16][l/16] and B[l/16][l%16], holds D[4j + l/16][l%16].
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// FP64 matrix-core variant.  A workgroup takes 16 elements of the class-sorted
// list; wave w computes rows [16w, 16w+16) of Y = M X for them with
// v_mfma_f64_16x16x4f64 (one wave per row tile keeps enough waves in flight
// to hide the gather latency).  A operands are read straight from the
// (L1/L2-resident) shared matrix, one pass per distinct class in the wave.
template <typename T>
__global__ __launch_bounds__(256) void shared_mfma64_kernel(Geo g, const int *__restrict__ xoff,
                                                            const double *__restrict__ matS,
                                                            OpArgs<T> a, double *__restrict__ Ys) {
  constexpr int KS = 16;   // k-steps of 4 (m_in <= 64)
  const int rt = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, kq = lane >> 4;
  const int ld = a.ld, mi = a.m_in, mo = a.m_out;
  if (16 * rt >= mo) return;   // whole wave
  const int li = blockIdx.x * 16 + n;
  const bool in = li < a.nsh;
  const int e = in ? a.shlist[li] : 0;
  const int id = in ? a.mid[e] : -1;
  const bool shared = id >= 0 && id < a.nS;
  bool todo = shared;
  const int ee = shared ? e : 0;
  const int ex = ee % g.n[0], r = ee / g.n[0];
  const int base = ex + g.gn[0] * ((r % g.n[1]) + g.gn[1] * (r / g.n[1]));
  double bv[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = min(4 * ks + kq, mi - 1);
    const double v = (double)a.x[base + xoff[k]];
    bv[ks] = (shared && 4 * ks + kq < mi) ? v : 0.0;
  }
  const int nks = (mi + 3) / 4;
  const int row = min(16 * rt + n, mo - 1);
  const bool rowv = 16 * rt + n < mo;
  for (;;) {
    const unsigned long long msk = __ballot(todo);
    if (msk == 0ull) break;
    const int first = __ffsll((long long)msk) - 1;
    const int id0 = __builtin_amdgcn_readfirstlane(__shfl(id, first));
    const bool mine = todo && id == id0;
    todo = todo && !mine;
    const double *M0 = matS + (size_t)id0 * ld * ld;
    double av[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = min(4 * ks + kq, mi - 1);
      const double v = M0[(size_t)k * ld + row];   // M[row][k] = M[k][row]
      av[ks] = (4 * ks + kq < mi && rowv) ? v : 0.0;
    }
    doublex4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      if (ks < nks) c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], mine ? bv[ks] : 0.0, c, 0, 0, 0);
    if (mine) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = 16 * rt + 4 * j + kq;
        if (rr < mo) Ys[(size_t)rr * g.E + e] = c[j];
      }
    }
  }
}

// Phase B for wide element matrices (64 < m <= 384, e.g. elasticity at p = 4):
// work item = (8 row tiles of 16, chunk of <= 256 elements with the same
// shared matrix).  Wave w keeps rows [16 rt, 16 rt + 16) of the shared matrix
// in registers as v_mfma_f64_16x16x4f64 A operands (the matrix is symmetric,
// so row r is read as column r, coalesced), 16-element groups of gathered
// inputs stream through LDS as B operands (lane l supplies A[l%16][l/16] and
// B[l/16][l%16], holds D[4j+l/16][l%16]).
typedef double doublex4e __attribute__((ext_vector_type(4)));

template <typename T, int NKS>
__global__ __launch_bounds__(512) void elem_class_mfma_kernel(Geo g, const int *__restrict__ xoff,
                                                              const double *__restrict__ matS,
                                                              OpArgs<T> a,
                                                              double *__restrict__ Ys) {
  extern __shared__ double X[];   // [NKS * 4][16]
  constexpr int KP = NKS * 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, kq = lane >> 4;
  const int *ch = a.chk + 3 * blockIdx.y;
  const int c = ch[0], p0 = ch[1], cnt = ch[2];
  const int mi = a.m_in, mo = a.m_out, ld = a.ld;
  const int rt = blockIdx.x * 8 + wave;
  const bool rtv = 16 * rt < mo;
  double av[NKS];
  {
    const double *A0 = matS + (size_t)c * ld * ld;
    const int r = 16 * rt + n;
    const bool rv = rtv && r < mo;
    const int rc = min(r, mo - 1);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k = 4 * ks + kq;
      const double v = A0[(size_t)min(k, mi - 1) * ld + rc];   // M[r][k] = M[k][r]
      av[ks] = (rv && k < mi) ? v : 0.0;
    }
  }
  const int ngroups = (cnt + 15) >> 4;
  for (int gi = 0; gi < ngroups; ++gi) {
    const int q0 = p0 + 16 * gi, qn = min(16, cnt - 16 * gi);
    for (int i = threadIdx.x; i < 16 * KP; i += 512) {
      const int nn = i & 15, k = i >> 4;
      double v = 0.0;
      if (nn < qn && k < mi) {
        const int e = a.shlist[q0 + nn];
        const int ex = e % g.n[0], r = e / g.n[0];
        const int base = ex + g.gn[0] * ((r % g.n[1]) + g.gn[1] * (r / g.n[1]));
        v = (double)a.x[base + xoff[k]];
      }
      X[i] = v;
    }
    __syncthreads();
    if (rtv) {
      doublex4e acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], X[(4 * ks + kq) * 16 + n], acc, 0, 0, 0);
      if (n < qn) {
        const int e = a.shlist[q0 + n];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = 16 * rt + 4 * j + kq;
          if (rr < mo) Ys[(size_t)rr * g.E + e] = acc[j];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int NKS>
static void launch_elem_class_nks(const Geo &g, const Tables &t, const OpArgs<T> &a,
                                  const double *matS, double *Ys, hipStream_t s) {
  const int nrt = (a.m_out + 15) / 16;
  dim3 grid((nrt + 7) / 8, a.nchunks);
  elem_class_mfma_kernel<T, NKS><<<grid, 512, (size_t)NKS * 4 * 16 * sizeof(double), s>>>(
      g, t.xoff, matS, a, Ys);
}

template <typename T>
static bool launch_elem_class(const Geo &g, const Tables &t, const OpArgs<T> &a,
                              const double *matS, double *Ys, hipStream_t s) {
  const int nks = (a.m_in + 3) / 4;
  if (!a.chk || a.nchunks <= 0 || nks > 96) return false;
  if (nks <= 24) launch_elem_class_nks<T, 24>(g, t, a, matS, Ys, s);
  else if (nks <= 48) launch_elem_class_nks<T, 48>(g, t, a, matS, Ys, s);
  else if (nks <= 64) launch_elem_class_nks<T, 64>(g, t, a, matS, Ys, s);
  else if (nks <= 88) launch_elem_class_nks<T, 88>(g, t, a, matS, Ys, s);
  else launch_elem_class_nks<T, 96>(g, t, a, matS, Ys, s);
  return true;
}

// Phase C: owner gather.  One thread per output entry (grid point g, plane P)
// sums the 2^k element results that belong to this DOF and applies the fused
// epilogue (damped update, residual update, prolongation).
template <typename T, typename TM>
__global__ __launch_bounds__(256) void gather_kernel(Geo g, const int *__restrict__ rows,
                                                     const int *__restrict__ pinfo, OpArgs<T> a,
                                                     const TM *__restrict__ Ys) {
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
  TM acc = 0;
  double acc64 = 0.0;
  bool any = false;
  if (valid) {
    for (int s = 0; s < (1 << g.d); ++s) {
      if (s & ~vmask) continue;
      const int ex = gx - (s & 1), ey = gy - ((s >> 1) & 1), ez = gz - ((s >> 2) & 1);
      if (ex < 0 || ey < 0 || ez < 0 || ex >= g.n[0] || ey >= g.n[1] || ez >= g.n[2]) continue;
      const int e = ex + g.n[0] * (ey + g.n[1] * ez);
      const int id = a.mid[e];
      if (id < 0) continue;
      any = true;
      const int row = rows[P * 8 + s];
      if (id < a.nS) acc += Ys[(size_t)row * g.E + e];
      else acc64 += a.Y[(size_t)(id - a.nS) * a.m_out + row];
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

template <typename T, typename TM>
static void launch_shared(const Geo &g, const Tables &t, const OpArgs<T> &a, const TM *matS,
                          TM *Ys, hipStream_t s) {
  shared_elem_kernel<T, TM><<<(g.E + 255) / 256, 256, 0, s>>>(g, t.xoff, matS, a, Ys);
}

template <typename T, typename TM>
static void launch_op3(const Geo &g, const Tables &t, const OpArgs<T> &a, const TM *matS,
                       hipStream_t s) {
  TM *Ys = reinterpret_cast<TM *>(a.Yshared);
  launch_shared<T, TM>(g, t, a, matS, Ys, s);
  dim3 grid((g.G + 255) / 256, a.nP_out);
  gather_kernel<T, TM><<<grid, 256, 0, s>>>(g, t.rows, t.pinfo, a, Ys);
}

template <typename T>
void launch_elem_op(const Geo &g, const Tables &t, const OpArgs<T> &a, hipStream_t s) {
  const double *mS64 = a.matS64 ? a.matS64
                                 : (std::is_same<T, double>::value
                                        ? reinterpret_cast<const double *>(a.matS)
                                        : nullptr);
  if (mS64 && a.m_out <= 64) {
    // stored-matrix GEMV (HBM stream) and FP64 matrix-core work on shared matrices
    double *Ys = reinterpret_cast<double *>(a.Yshared);
    if (a.nstored > 0)
      stored_gemv_kernel<T><<<(a.nstored + 3) / 4, 256, 0, s>>>(g, t.xoff, a);
    if (a.nsh > 0)
      shared_mfma64_kernel<T><<<(a.nsh + 15) / 16, 256, 0, s>>>(g, t.xoff, mS64, a, Ys);
    dim3 grid((g.G + 255) / 256, a.nP_out);
    gather_kernel<T, double><<<grid, 256, 0, s>>>(g, t.rows, t.pinfo, a, Ys);
    return;
  }
  if (a.nstored > 0)
    stored_gemv_kernel<T><<<(a.nstored + 3) / 4, 256, 0, s>>>(g, t.xoff, a);
  if (mS64 && a.nsh > 0) {
    double *Ys = reinterpret_cast<double *>(a.Yshared);
    if (launch_elem_class<T>(g, t, a, mS64, Ys, s)) {
      dim3 grid((g.G + 255) / 256, a.nP_out);
      gather_kernel<T, double><<<grid, 256, 0, s>>>(g, t.rows, t.pinfo, a, Ys);
      return;
    }
  }
  if (a.matS64)
    launch_op3<T, double>(g, t, a, a.matS64, s);
  else
    launch_op3<T, T>(g, t, a, a.matS, s);
}
template void launch_elem_op<double>(const Geo &, const Tables &, const OpArgs<double> &,
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

// beta = r_new.z_new / r.z (flexible: (r_new.z_new - r_new.z_old) / r.z, scal[8])
__global__ void cg_beta_kernel(double *sc, int flexible) {
  sc[5] = (sc[4] - (flexible ? sc[8] : 0.0)) / sc[0];
  sc[0] = sc[4];
}
void launch_cg_beta(double *scal, int flexible, hipStream_t s) {
  cg_beta_kernel<<<1, 1, 0, s>>>(scal, flexible);
}

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

template <typename T>
__global__ void copy_kernel(T *y, const T *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x ? x[i] : T(0);
}
template <typename T>
void launch_copy(T *y, const T *x, int64_t n, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  copy_kernel<T><<<blocks, 256, 0, s>>>(y, x, n);
}
template void launch_copy<double>(double *, const double *, int64_t, hipStream_t);


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

// Block sweeps of the layer-block-tridiagonal p = 1 system (block LDL^T):
//   u_k = c_k - G_k u_{k-1},  c_k = S_k^{-1} b_k       (forward, k = 1..K-1)
//   x_k = u_k - F_k x_{k+1}                           (backward, k = K-2..0)
// with G_k = S_k^{-1} B_k and F_k = S_k^{-1} B_{k+1}^T precomputed at setup.
// Every step is a dense FP64 GEMV, one wave per row (coalesced row reads,
// shuffle reduction); the c_k of all blocks are one batched launch.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  return v;
}

// The sweeps work on contiguous block-layout copies of the coarse vectors.
__global__ void coarse_to_block_kernel(Geo g, Coarse c, const double *src, double *dst) {
  const int k = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.nb; i += gridDim.x * blockDim.x) {
    const int64_t gi = coarse_vec_index(g, c, k, i);
    dst[(size_t)k * c.nb + i] = gi >= 0 ? src[gi] : 0.0;
  }
}

__global__ void coarse_from_block_kernel(Geo g, Coarse c, const double *src, double *dst) {
  const int k = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.nb; i += gridDim.x * blockDim.x) {
    const int64_t gi = coarse_vec_index(g, c, k, i);
    if (gi >= 0) dst[gi] = src[(size_t)k * c.nb + i];
  }
}

// mode 0: xb_k = Sinv_k bb_k for all k (batched over blockIdx.y)
// mode 1: xb_k -= G_k xb_{k-1}        mode 2: xb_k -= F_k xb_{k+1}
__global__ __launch_bounds__(256) void coarse_gemv_kernel(int nb, int k, int mode,
                                                          const double *__restrict__ M,
                                                          const double *__restrict__ bb,
                                                          double *xb) {
  const int kk = mode == 0 ? (int)blockIdx.y : k;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nb) return;
  const int kin = mode == 0 ? kk : (mode == 1 ? kk - 1 : kk + 1);
  const double *row = M + ((size_t)(mode == 0 ? kk : 0) * nb + i) * nb;
  const double *vin = (mode == 0 ? bb : xb) + (size_t)kin * nb;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int j = lane;
  for (; j + 192 < nb; j += 256) {
    a0 += row[j] * vin[j];
    a1 += row[j + 64] * vin[j + 64];
    a2 += row[j + 128] * vin[j + 128];
    a3 += row[j + 192] * vin[j + 192];
  }
  for (; j < nb; j += 64) a0 += row[j] * vin[j];
  const double acc = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) {
    double *o = xb + (size_t)kk * nb + i;
    *o = (mode == 0) ? acc : *o - acc;
  }
}

__global__ void fill_zero_kernel(double *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

void coarse_solve_launch(const Geo &g, const Coarse &c, const double *b, double *x,
                         hipStream_t s) {
  const int nb = c.nb;
  const size_t nb2 = (size_t)nb * nb;
  const dim3 vgrid((nb + 255) / 256, c.nblk);
  coarse_to_block_kernel<<<vgrid, 256, 0, s>>>(g, c, b, c.bblk);
  const int rows_blocks = (nb + 3) / 4;
  coarse_gemv_kernel<<<dim3(rows_blocks, c.nblk), 256, 0, s>>>(nb, 0, 0, c.Sinv, c.bblk, c.xblk);
  for (int k = 1; k < c.nblk; ++k)
    coarse_gemv_kernel<<<rows_blocks, 256, 0, s>>>(nb, k, 1, c.Gm + k * nb2, c.bblk, c.xblk);
  for (int k = c.nblk - 2; k >= 0; --k)
    coarse_gemv_kernel<<<rows_blocks, 256, 0, s>>>(nb, k, 2, c.Fm + k * nb2, c.bblk, c.xblk);
  // entries outside the blocked system (Dirichlet layers) are zero
  const int64_t n = (int64_t)g.nf * g.G;
  fill_zero_kernel<<<(int)std::min<int64_t>((n + 255) / 256, 1024), 256, 0, s>>>(x, n);
  coarse_from_block_kernel<<<vgrid, 256, 0, s>>>(g, c, c.xblk, x);
}

}  // namespace fcm
