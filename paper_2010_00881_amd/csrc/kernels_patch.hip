// Patchwise additive Schwarz smoother of libfcm (gfx950).
//
// One block per grid node v (Section 3.3.1, patchwise groups on a uniform
// grid): every level-q function that is nonzero on a kept element among the
// 2^d elements sharing v.  Per axis the patch sees 2q+1 one-dimensional
// functions -- the hats at nodes v-1, v, v+1 and the bubbles of elements v-1
// and v -- so m_q = n_f (2q+1)^d (Table tab::upperbound with n = 2).
//
// Patch-local modes are sorted by degree, so the level-q block is the leading
// m_q x m_q block of the order-p patch (eq. hierarchicalMatrices).  A local
// mode is one per-axis slot (0..2p) per axis plus a component:
//   slot 0        hat at node v-1           (delta -1)
//   slot 1..p-1   bubble of element v-1     (type t = slot, degree t+1)
//   slot p        hat at node v             (delta  0)
//   slot p+1..2p-1 bubble of element v      (type t = slot-p)
//   slot 2p       hat at node v+1           (delta +1)
// A mode is absent from patch v when it is Dirichlet-constrained or nonzero
// on no kept element of the patch; absent modes get identity rows in the
// block and a zero input, so their outputs are exactly zero.
//
// Application M^-1 r = sum_v P_v A_v^{-1} P_v^T r (eq. AdditiveSchwarz):
//  * unique patches (a cut or void element within the 4^d elements that their
//    functions touch): stored inverses streamed from HBM, one workgroup per
//    patch, 4 rows per lane (128-bit loads of the symmetric matrix);
//  * class patches (translation-invariant blocks): A_v^{-1} shared per class,
//    Y = A^{-1} X on the FP64 matrix cores with the inverse held in registers;
//  * owner gather: each DOF sums its rows of the <= 3^d patches containing
//    it in a fixed order (deterministic) and applies the smoother epilogue.
#include <algorithm>
#include <type_traits>

#include "fcm_internal.hpp"

namespace fcm {

__device__ __host__ inline void patch_slot(int sl, int p, int &t, int &dl) {
  if (sl == 0) { t = 0; dl = -1; }
  else if (sl < p) { t = sl; dl = -1; }
  else if (sl == p) { t = 0; dl = 0; }
  else if (sl < 2 * p) { t = sl - p; dl = 0; }
  else { t = 0; dl = 1; }
}

__device__ inline void node_coords(const Geo &g, int node, int *vc) {
  vc[0] = node % g.gn[0];
  const int r = node / g.gn[0];
  vc[1] = r % g.gn[1];
  vc[2] = r / g.gn[1];
}

// pinfo bits: 0..7 element mask (bit s: element v - s, s_a = 1 meaning
// element index v_a - 1), 8..10 hat axes, 12+2a..13+2a delta_a + 1.
__device__ inline bool patch_present(const Geo &g, int info, int kmask, const int *vc) {
  if (!(info & kmask & 0xff)) return false;
  for (int ax = 0; ax < g.d; ++ax) {
    if (!((info >> (8 + ax)) & 1)) continue;
    const int node = vc[ax] + ((info >> (12 + 2 * ax)) & 3) - 1;
    if (node == 0 && ((g.dir >> (2 * ax)) & 1)) return false;
    if (node == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) return false;
  }
  return true;
}

// Entry (i, j) of the patch block at node vc: sum over the kept elements in
// the common support of the two functions of the element-matrix entries.
__device__ double patch_entry(const Geo &g, const PatchTables &pt, const int *smap, int mp,
                              const int *kmat, const double *Kref, const double *Kcut,
                              const int *vc, int kmask, int i, int j) {
  const int ii = pt.pinfo[i], ij = pt.pinfo[j];
  const bool pi = patch_present(g, ii, kmask, vc), pj = patch_present(g, ij, kmask, vc);
  if (!pi || !pj) return i == j ? 1.0 : 0.0;
  const int *mi = pt.pm + 4 * i, *mj = pt.pm + 4 * j;
  const int p = g.p, np = p + 1;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int ti[3] = {0, 0, 0}, di[3] = {0, 0, 0}, tj[3] = {0, 0, 0}, dj[3] = {0, 0, 0};
  for (int ax = 0; ax < g.d; ++ax) {
    patch_slot(mi[ax], p, ti[ax], di[ax]);
    patch_slot(mj[ax], p, tj[ax], dj[ax]);
    // element index ranges of the two supports (hat at node c: elements
    // c-1, c; bubble of element c: element c), relative to v
    const int li = ti[ax] == 0 ? di[ax] - 1 : di[ax], hi_ = di[ax];
    const int lj = tj[ax] == 0 ? dj[ax] - 1 : dj[ax], hj = dj[ax];
    lo[ax] = max(li, lj);
    hi[ax] = min(hi_, hj);
    if (lo[ax] > hi[ax]) return 0.0;
  }
  // the (at most 2 per axis) common elements, axis 0 fastest: all element
  // ids, then all matrix entries, summed in that order.  Each pass issues
  // its loads unconditionally from clamped addresses (a load under a
  // condition is waited for before the next is issued) and masks afterwards.
  int kid[8], la[8], lb[8];
  bool in[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int ec[3] = {0, 0, 0}, ai[3] = {0, 0, 0}, aj[3] = {0, 0, 0};
    bool ok = true;
    for (int ax = 0; ax < 3; ++ax) {
      const int rel = lo[ax] + ((c >> ax) & 1);
      if (ax >= g.d) {
        ok = ok && ((c >> ax) & 1) == 0;
        continue;
      }
      ec[ax] = vc[ax] + rel;
      ok = ok && rel <= hi[ax] && ec[ax] >= 0 && ec[ax] < g.n[ax];
      ec[ax] = min(max(ec[ax], 0), g.n[ax] - 1);
      // element-local 1D mode: 0 / 1 = hat at the element's left / right
      // node, t + 1 = bubble of type t
      ai[ax] = min(max(ti[ax] == 0 ? di[ax] - rel : ti[ax] + 1, 0), p);
      aj[ax] = min(max(tj[ax] == 0 ? dj[ax] - rel : tj[ax] + 1, 0), p);
    }
    in[c] = ok;
    kid[c] = kmat[ec[0] + g.n[0] * (ec[1] + g.n[1] * ec[2])];
    la[c] = smap[(ai[0] + np * (ai[1] + np * ai[2])) * g.nf + mi[3]];
    lb[c] = smap[(aj[0] + np * (aj[1] + np * aj[2])) * g.nf + mj[3]];
  }
  double v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int k = in[c] ? kid[c] : -1;
    in[c] = k >= 0;
    const double *K = k <= 0 ? Kref : Kcut + (size_t)(k - 1) * mp * mp;
    v[c] = K[(size_t)la[c] * mp + lb[c]];
  }
  double sum = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) sum += (in[c] ? 1.0 : 0.0) * v[c];
  return sum;
}

__global__ __launch_bounds__(256) void form_patch_blocks_kernel(Geo g, PatchTables pt,
                                                                const int *smap, int mp, int m,
                                                                const int *bnode,
                                                                const int *bkm, const int *kmat,
                                                                const double *Kref,
                                                                const double *Kcut,
                                                                double *out) {
  const int blk = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int i = e / m, j = e % m;
  if (j < i) return;
  int vc[3];
  node_coords(g, bnode[blk], vc);
  // the element matrices are symmetric and the element sum runs in the same
  // order for (i, j) and (j, i): the upper entry is stored at both places
  const double v = patch_entry(g, pt, smap, mp, kmat, Kref, Kcut, vc, bkm[blk], i, j);
  out[(size_t)blk * m * m + e] = v;
  out[(size_t)blk * m * m + (size_t)j * m + i] = v;
}

void launch_form_patch_blocks(const Geo &g, const Tables &t, const PatchTables &pt, int m,
                              const int *bnode, const int *bkm, int nblocks, const int *kmat,
                              const double *Kref, const double *Kcut, double *out,
                              hipStream_t s) {
  if (nblocks <= 0) return;
  dim3 grid((m * m + 255) / 256, nblocks);
  form_patch_blocks_kernel<<<grid, 256, 0, s>>>(g, pt, t.smap, t.m, m, bnode, bkm, kmat, Kref,
                                                Kcut, out);
}

// dst[b] (m x ld, zero-padded columns) <- src[b] (m x m), FP64 and/or FP32
__global__ void pack_blocks_kernel(const double *src, int m, int ld, int nb, double *d64,
                                   float *d32) {
  const size_t tot = (size_t)nb * m * ld;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / ((size_t)m * ld);
    const int r = (int)((i / ld) % m), c = (int)(i % ld);
    const double v = c < m ? src[b * m * m + (size_t)r * m + c] : 0.0;
    if (d64) d64[i] = v;
    if (d32) d32[i] = (float)v;
  }
}

void launch_pack_blocks(const double *src, int m, int ld, int nb, double *d64, float *d32,
                        hipStream_t s) {
  if (nb <= 0) return;
  const size_t tot = (size_t)nb * m * ld;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 8192);
  pack_blocks_kernel<<<blocks, 256, 0, s>>>(src, m, ld, nb, d64, d32);
}

// Tile (I, J), I <= J, at index t of the I-major enumeration
__device__ __host__ inline void tile_ij(int t, int nt, int &I, int &J) {
  I = 0;
  while (t >= nt - I) {
    t -= nt - I;
    ++I;
  }
  J = I + t;
}

// One workgroup per (tile, block): 256 threads copy the 16 x 16 tile.
__global__ __launch_bounds__(256) void pack_tiles_kernel(const double *src, int m, double *d64,
                                                         float *d32) {
  const int nt = (m + 15) / 16, tiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x, e = threadIdx.x;
  const size_t b = blockIdx.y;
  int I, J;
  tile_ij(t, nt, I, J);
  const int r = 16 * I + e / 16, c = 16 * J + e % 16;
  const double v = (r < m && c < m) ? src[b * m * m + (size_t)r * m + c] : 0.0;
  const size_t i = (b * tiles + t) * 256 + e;
  if (d64) d64[i] = v;
  if (d32) d32[i] = (float)v;
}

void launch_pack_tiles(const double *src, int m, int nb, double *d64, float *d32, hipStream_t s) {
  if (nb <= 0) return;
  pack_tiles_kernel<<<dim3(patch_tiles(m), nb), 256, 0, s>>>(src, m, d64, d32);
}

// ---------------------------------------------------------------- apply
// Unique patches: workgroup u computes Yu[u] = A_u^{-1} x_v from the stored
// tiles on and above the diagonal of the symmetric inverse: tile (I, J) adds
// M_IJ x_J to the rows of I and, for I < J, M_IJ^T x_I to the rows of J, so
// every stored entry is read once and used twice.  Wave w takes the tiles
// t = w, w + 4, ...; a tile is read contiguously (lane l: row l / 4, columns
// 4 (l % 4) .. + 3, one 128-bit FP32 or two FP64 loads) and staged in LDS.
// Every wave adds into its own LDS copy of y, its two half-waves one after
// the other, and the four copies are added in a fixed order, so the result
// is the same on every run (one copy per wave rather than per half-wave
// halves the LDS and doubles the workgroups a CU holds).
// A lane's 4 consecutive entries of a stored tile, kept in the storage type
// while the load is in flight (converted to FP64 when staged in LDS).
template <typename T> struct TileRaw;
template <> struct TileRaw<float> {
  float4 q;
  __device__ void load(const float *p) { q = *reinterpret_cast<const float4 *>(p); }
  __device__ double get(int k) const {
    return k == 0 ? q.x : k == 1 ? q.y : k == 2 ? q.z : q.w;
  }
};
template <> struct TileRaw<double> {
  double2 q0, q1;
  __device__ void load(const double *p) {
    q0 = *reinterpret_cast<const double2 *>(p);
    q1 = *reinterpret_cast<const double2 *>(p + 2);
  }
  __device__ double get(int k) const {
    return k == 0 ? q0.x : k == 1 ? q0.y : k == 2 ? q1.x : q1.y;
  }
};

// One wave's share of the tiles, two at a time (t and t + 4 of the wave's
// sequence t = w, w + 8, ...): each lane loads 4 entries of both tiles and
// stages them in the wave's LDS buffer (rows padded to 17 doubles); then in
// each half-wave 16 lanes form the row sums M_IJ x_J and 16 lanes the column
// sums M_IJ^T x_I of one tile, adding them to that half-wave's copy of y.
// Each trip issues the loads of kGemvPairs pairs together (unconditionally:
// a tile index past the end is replaced by the trip's first tile, an L1
// hit), then stages and computes the pairs in order, waiting only for the
// pair it needs: kGemvPairs pairs per wave are in flight (the bound is HBM)
// and no load is pending across trips.
constexpr int kGemvPairs = 3;

// toff (LDS, may be null): storage index of the t-th tile of the list
// (consecutive tiles when null).
template <typename M>
__device__ inline void tile_sweep(const M *base, int ntiles, const unsigned char *tI,
                                  const unsigned char *tJ, const int *toff, const double *xs,
                                  double (*tb)[16][17], double *yh, int wave, int lane) {
  const int r = lane >> 2, c0 = (lane & 3) * 4;
  const int half = lane >> 5, i = lane & 15;
  const bool rowpart = (lane & 16) == 0;
  const M *lp = base + r * 16 + c0;
  for (int t0 = wave; t0 < ntiles; t0 += 8 * kGemvPairs) {
    TileRaw<M> ta[kGemvPairs], tb2[kGemvPairs];
#pragma unroll
    for (int q = 0; q < kGemvPairs; ++q) {
      const int ta_i = t0 + 8 * q, tb_i = ta_i + 4;
      const int ia = ta_i < ntiles ? ta_i : t0, ib = tb_i < ntiles ? tb_i : t0;
      ta[q].load(lp + (size_t)(toff ? toff[ia] : ia) * 256);
      tb2[q].load(lp + (size_t)(toff ? toff[ib] : ib) * 256);
    }
#pragma unroll
    for (int q = 0; q < kGemvPairs; ++q) {
      const int tp = t0 + 8 * q;
      if (tp >= ntiles) break;   // wave-uniform
      const bool hasb = tp + 4 < ntiles;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        tb[0][r][c0 + e] = ta[q].get(e);
        tb[1][r][c0 + e] = hasb ? tb2[q].get(e) : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      const int t = tp + 4 * half;
      int dst = -1;
      double acc = 0.0;
      if (t < ntiles) {
        const int I = tI[t], J = tJ[t];
        if (rowpart) {
          const double *xJ = xs + 16 * J;
#pragma unroll
          for (int k = 0; k < 16; ++k) acc += tb[half][i][k] * xJ[k];
          dst = 16 * I + i;
        } else if (I != J) {
          const double *xI = xs + 16 * I;
#pragma unroll
          for (int k = 0; k < 16; ++k) acc += tb[half][k][i] * xI[k];
          dst = 16 * J + i;
        }
      }
      // the wave's copy of y: the first half-wave adds, then the second (the
      // two tiles may share rows), so the order is fixed
      if (half == 0 && dst >= 0) yh[dst] += acc;
      __builtin_amdgcn_wave_barrier();
      if (half == 1 && dst >= 0) yh[dst] += acc;
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void patch_gemv_kernel(Geo g, const int *__restrict__ pxoff,
                                                         const int *__restrict__ pinfo,
                                                         PatchArgs<T> a) {
  constexpr int kPad = (kSmallPatchM + 15) / 16 * 16;
  constexpr int kMaxTiles = (kPad / 16) * (kPad / 16 + 1) / 2;
  __shared__ double xs[kPad];
  __shared__ double yw[4][kPad];
  __shared__ double tbuf[4][2][16][17];
  __shared__ unsigned char tI[kMaxTiles], tJ[kMaxTiles];
  const int u = blockIdx.x;
  const int pi = a.nsh + u;
  const int node = a.pnode[pi], kmask = a.pkm[pi];
  int vc[3];
  node_coords(g, node, vc);
  const int m = a.m, nt = a.ntile, mp = 16 * nt;
  const int ntiles = nt * (nt + 1) / 2;
  for (int k = threadIdx.x; k < mp; k += 256) {
    xs[k] = k < m && patch_present(g, pinfo[k], kmask, vc) ? (double)a.x[node + pxoff[k]] : 0.0;
    for (int w = 0; w < 4; ++w) yw[w][k] = 0.0;
  }
  for (int t = threadIdx.x; t < ntiles; t += 256) {
    int I, J;
    tile_ij(t, nt, I, J);
    tI[t] = (unsigned char)I;
    tJ[t] = (unsigned char)J;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t base = (size_t)u * ntiles * 256;
  const bool lo = a.matU32 && !(a.u64flag && a.u64flag[u]);
  if (lo)
    tile_sweep<float>(a.matU32 + base, ntiles, tI, tJ, nullptr, xs, tbuf[wave], yw[wave], wave,
                      lane);
  else
    tile_sweep<double>(a.matU + base, ntiles, tI, tJ, nullptr, xs, tbuf[wave], yw[wave], wave,
                       lane);
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += 256) {
    double y = 0.0;
    for (int w = 0; w < 4; ++w) y += yw[w][k];
    a.Yu[(size_t)u * m + k] = y;
  }
}

// Unique patches with large blocks (m > kSmallPatchM, e.g. elasticity at
// p = 3, 4: m = 1029, 2187), whose per-wave copies of y would not fit in
// LDS.  The tile rows are cut into bands of kBandT tiles (256 rows); work item
// (patch u, band pair a <= b) takes the stored tiles (I, J) with I in band a,
// J in band b and J >= I, so every stored tile is read by exactly one work
// item.  Its row sums land in band a and its column sums in band b; the
// work item keeps both bands of x and one copy per wave of both bands of
// y in LDS (local tile index i for band a, 16 + j for band b, or j when
// a = b) and writes the two partial bands to P[u][pair][0..511].
// patch_band_reduce_kernel then adds, for every row of band c, the partials
// of the pairs (a, c), a < c, then (c, c), then (c, b), b > c -- a fixed
// order, so the result is the same on every run.
constexpr int kBandT = 16;

__device__ inline void band_pair(int pr, int nbands, int &A, int &B) {
  A = 0;
  while (pr >= nbands - A) {
    pr -= nbands - A;
    ++A;
  }
  B = A + pr;
}

template <typename T>
__global__ __launch_bounds__(256) void patch_gemv_band_kernel(Geo g, const int *__restrict__ pxoff,
                                                              const int *__restrict__ pinfo,
                                                              PatchArgs<T> a, int nbands,
                                                              int npairs, double *P) {
  constexpr int R = 16 * kBandT;           // rows per band
  __shared__ double xs[2 * R];
  __shared__ double yw[4][2 * R];
  __shared__ double tbuf[4][2][16][17];
  __shared__ unsigned char tI[kBandT * kBandT], tJ[kBandT * kBandT];
  __shared__ int toff[kBandT * kBandT];
  const int u = blockIdx.x / npairs, pr = blockIdx.x - u * npairs;
  int A, B;
  band_pair(pr, nbands, A, B);
  const bool same = A == B;
  const int pi = a.nsh + u;
  const int node = a.pnode[pi], kmask = a.pkm[pi];
  int vc[3];
  node_coords(g, node, vc);
  const int m = a.m, nt = a.ntile;
  for (int k = threadIdx.x; k < 2 * R; k += 256) {
    const int row = (k < R ? A : B) * R + (k & (R - 1));
    const int rc = min(row, m - 1);
    double v = 0.0;
    if (row < m && patch_present(g, pinfo[rc], kmask, vc)) v = (double)a.x[node + pxoff[rc]];
    xs[k] = v;
#pragma unroll
    for (int w = 0; w < 4; ++w) yw[w][k] = 0.0;
  }
  // the work item's tiles, I-major: a < b all (i, j) of the two bands, a = b
  // the triangle j >= i
  const int ni = min(kBandT, nt - kBandT * A), nj = min(kBandT, nt - kBandT * B);
  const int ntl = same ? ni * (ni + 1) / 2 : ni * nj;
  for (int t = threadIdx.x; t < ntl; t += 256) {
    int i, j;
    if (same) {
      tile_ij(t, ni, i, j);
    } else {
      i = t / nj;
      j = t - i * nj;
    }
    const int I = kBandT * A + i, J = kBandT * B + j;
    tI[t] = (unsigned char)i;
    tJ[t] = (unsigned char)(same ? j : kBandT + j);
    toff[t] = I * nt - I * (I - 1) / 2 + (J - I);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t base = (size_t)u * (nt * (nt + 1) / 2) * 256;
  const bool lo = a.matU32 && !(a.u64flag && a.u64flag[u]);
  if (lo)
    tile_sweep<float>(a.matU32 + base, ntl, tI, tJ, toff, xs, tbuf[wave], yw[wave], wave, lane);
  else
    tile_sweep<double>(a.matU + base, ntl, tI, tJ, toff, xs, tbuf[wave], yw[wave], wave, lane);
  __syncthreads();
  double *Pw = P + ((size_t)u * npairs + pr) * (2 * R);
  for (int k = threadIdx.x; k < 2 * R; k += 256) {
    double y = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) y += yw[w][k];
    Pw[k] = y;
  }
}

__global__ __launch_bounds__(256) void patch_band_reduce_kernel(const double *__restrict__ P,
                                                                int m, int nbands, int npairs,
                                                                int npu, double *Yu) {
  constexpr int R = 16 * kBandT;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)npu * m) return;
  const int u = (int)(idx / m), row = (int)(idx - (size_t)u * m);
  const int c = row / R, k = row - c * R;
  const double *Pu = P + (size_t)u * npairs * (2 * R);
  auto pair = [&](int x, int y) { return x * nbands - x * (x - 1) / 2 + (y - x); };
  double y = 0.0;
  for (int aa = 0; aa < c; ++aa) y += Pu[(size_t)pair(aa, c) * (2 * R) + R + k];
  for (int bb = c; bb < nbands; ++bb) y += Pu[(size_t)pair(c, bb) * (2 * R) + k];
  Yu[idx] = y;
}

// Class patches on the FP64 matrix cores.  Work item = (8 row tiles of 16,
// chunk of <= 256 patches of one class).  Wave w keeps rows [16 rt, 16 rt + 16)
// of the class inverse in registers (A operands, loaded once per chunk) and
// streams the chunk in groups of 16 patches: the workgroup gathers X (m x 16)
// into LDS, then each wave runs NKS back-to-back v_mfma_f64_16x16x4f64 with
// B from LDS.  Lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[4j+l/16][l%16].  Mode presence of a class patch depends only on its
// class (bit k of cpres[class]).
typedef double doublex4p __attribute__((ext_vector_type(4)));

template <typename T, int NKS>
__global__ __launch_bounds__(512) void patch_class_mfma_kernel(Geo g,
                                                               const int *__restrict__ pxoff,
                                                               PatchArgs<T> a) {
  extern __shared__ double X[];   // [NKS * 4][16]
  constexpr int KP = NKS * 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, kq = lane >> 4;
  const int *ch = a.chk + 3 * blockIdx.y;
  const int c = ch[0], p0 = ch[1], cnt = ch[2];
  const int m = a.m, ld = a.ld;
  const int rt = blockIdx.x * 8 + wave;
  const bool rtv = 16 * rt < m;
  const unsigned *pres = a.cpres + (size_t)c * a.pwords;
  double av[NKS];
  {
    const double *A0 = a.matS64 + (size_t)c * m * ld;
    const int r = 16 * rt + n;
    const bool rv = rtv && r < m;
    const int rc = min(r, m - 1);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k = 4 * ks + kq;
      const double v = A0[(size_t)min(k, m - 1) * ld + rc];   // A[r][k] = A[k][r]
      av[ks] = (rv && k < m) ? v : 0.0;
    }
  }
  const int ngroups = (cnt + 15) >> 4;
  // gathered inputs of the next group are prefetched into registers while the
  // current group runs on the matrix cores (element i = tid + 512 j of X);
  // the widest tiles have no registers to spare and gather in place
  constexpr int PER = NKS / 8;
  constexpr bool kPrefetch = NKS <= 64;
  T pf[PER];
  auto fetch = [&](int gi) {
    const int q0 = p0 + 16 * gi, qn = min(16, cnt - 16 * gi);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = threadIdx.x + 512 * j;
      const int nn = i & 15, k = i >> 4;
      T v = T(0);
      if (nn < qn && k < m && ((pres[k >> 5] >> (k & 31)) & 1u))
        v = a.x[a.pnode[q0 + nn] + pxoff[k]];
      pf[j] = v;
    }
  };
  if (kPrefetch) fetch(0);
  for (int gi = 0; gi < ngroups; ++gi) {
    const int q0 = p0 + 16 * gi, qn = min(16, cnt - 16 * gi);
    if (kPrefetch) {
#pragma unroll
      for (int j = 0; j < PER; ++j) X[threadIdx.x + 512 * j] = (double)pf[j];
    } else {
      for (int i = threadIdx.x; i < 16 * KP; i += 512) {
        const int nn = i & 15, k = i >> 4;
        double v = 0.0;
        if (nn < qn && k < m && ((pres[k >> 5] >> (k & 31)) & 1u))
          v = (double)a.x[a.pnode[q0 + nn] + pxoff[k]];
        X[i] = v;
      }
    }
    __syncthreads();
    if (kPrefetch && gi + 1 < ngroups) fetch(gi + 1);
    if (rtv) {
      doublex4p acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], X[(4 * ks + kq) * 16 + n], acc, 0, 0, 0);
      if (n < qn) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = 16 * rt + 4 * j + kq;
          if (rr < m) a.Ys[(size_t)rr * a.nsh + q0 + n] = acc[j];
        }
      }
    }
    __syncthreads();
  }
}

// FP32 variant for the mixed form, used for small blocks (m <= 32; larger
// ones go to patch_class_tile_kernel): class inverses are well conditioned
// (uncut patches), so their products use v_mfma_f32_16x16x4f32 (inputs
// rounded to FP32, FP32 accumulation; lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4(l/16)+j][l%16]).  Half-width registers leave
// room for the next group's prefetch and two accumulation chains.
typedef float floatx4p __attribute__((ext_vector_type(4)));

template <typename T, int NKS>
__global__ __launch_bounds__(512) void patch_class_mfma32_kernel(Geo g,
                                                                 const int *__restrict__ pxoff,
                                                                 PatchArgs<T> a) {
  extern __shared__ float Xf[];   // [NKS * 4][16]
  constexpr int KP = NKS * 4;
  constexpr int PER = NKS / 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, kq = lane >> 4;
  const int *ch = a.chk + 3 * blockIdx.y;
  const int c = ch[0], p0 = ch[1], cnt = ch[2];
  const int m = a.m, ld = a.ld;
  const int rt = blockIdx.x * 8 + wave;
  const bool rtv = 16 * rt < m;
  const unsigned *pres = a.cpres + (size_t)c * a.pwords;
  float av[NKS];
  {
    const float *A0 = a.matS32 + (size_t)c * m * ld;
    const int r = 16 * rt + n;
    const bool rv = rtv && r < m;
    const int rc = min(r, m - 1);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k = 4 * ks + kq;
      const float v = A0[(size_t)min(k, m - 1) * ld + rc];   // A[r][k] = A[k][r]
      av[ks] = (rv && k < m) ? v : 0.f;
    }
  }
  const int ngroups = (cnt + 15) >> 4;
  float pf[PER];
  auto fetch = [&](int gi) {
    const int q0 = p0 + 16 * gi, qn = min(16, cnt - 16 * gi);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = threadIdx.x + 512 * j;
      const int nn = i & 15, k = i >> 4;
      float v = 0.f;
      if (nn < qn && k < m && ((pres[k >> 5] >> (k & 31)) & 1u))
        v = (float)a.x[a.pnode[q0 + nn] + pxoff[k]];
      pf[j] = v;
    }
  };
  fetch(0);
  for (int gi = 0; gi < ngroups; ++gi) {
    const int q0 = p0 + 16 * gi, qn = min(16, cnt - 16 * gi);
#pragma unroll
    for (int j = 0; j < PER; ++j) Xf[threadIdx.x + 512 * j] = pf[j];
    __syncthreads();
    if (gi + 1 < ngroups) fetch(gi + 1);
    if (rtv) {
      floatx4p acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < NKS; ks += 2) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], Xf[(4 * ks + kq) * 16 + n], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks + 1], Xf[(4 * ks + 4 + kq) * 16 + n], acc1,
                                                    0, 0, 0);
      }
      if (n < qn) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = 16 * rt + 4 * kq + j;
          if (rr < m) a.Ys[(size_t)rr * a.nsh + q0 + n] = (double)(acc0[j] + acc1[j]);
        }
      }
    }
    __syncthreads();
  }
}

// Class products with both operands streamed through LDS: a workgroup
// computes ROWS = 128 NRT rows (row block blockIdx.y) for 64 patches of one
// class, Y[r0:r0+ROWS, q0:q0+64] = A_c[r0:r0+ROWS, :] X, in slices of 32 k
// (A_c from L2, X gathered once per patch and row block), prefetching the
// next slice into registers while the matrix cores work on the current one.
// C is the arithmetic type: float (mixed form, v_mfma_f32_16x16x4f32, lane l
// holds D[4(l/16) + j][l%16]) or double (v_mfma_f64_16x16x4f64, D[4j +
// l/16][l%16]); both take A[l%16][l/16] and B[l/16][l%16].  Every thread
// fetches an equal share of both slices: rows tid % 128 + 128 i and k rows
// tid / 128 + 4 j of the A slice (coalesced over rows; the class inverses are
// allocated with a tail of 32 ld + 512 entries, so the reads past row or
// column m need no clamp and are masked when stored) and X rows wave + 8 j
// (lane = patch).  X stays in its storage type (FP64 level vectors) while
// the load is in flight.  Wave w owns row tiles w, w + 8, .., w + 8 (NRT -
// 1) and all four 16-patch column tiles.  LDS rows are padded so that the
// four k rows an MFMA operand read touches fall in distinct banks.
constexpr int kKTab = ((kMaxPatchM + 31) / 32) * 32;   // mode tables of the class kernel

template <typename C> struct ClassMfma;
template <> struct ClassMfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static constexpr int kPadA = 16, kPadX = 16;
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int j, int kq) { return 4 * kq + j; }
  template <typename A> __device__ static const float *mat(const A &a) { return a.matS32; }
};
template <> struct ClassMfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static constexpr int kPadA = 8, kPadX = 8;
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int j, int kq) { return 4 * j + kq; }
  template <typename A> __device__ static const double *mat(const A &a) { return a.matS64; }
};

template <typename T, typename C, int NRT, int KTAB>
__global__ __launch_bounds__(512, 4) void patch_class_tile_kernel(const int *__restrict__ pxoff,
                                                                  PatchArgs<T> a) {
  typedef ClassMfma<C> MM;
  typedef typename MM::v4 v4;
  constexpr int ROWS = 128 * NRT, RS = ROWS + MM::kPadA, XS = 64 + MM::kPadX;
  __shared__ C As[32 * RS];
  __shared__ C Xs[32 * XS];
  __shared__ int koff[KTAB];           // offset of mode k from the patch node in x
  __shared__ C kmask[KTAB];            // 1 if mode k is present in the class, else 0
  // Workgroups are dealt to the 8 XCDs round-robin by id; the four quarters
  // of a chunk get ids of one residue mod 8 (gridDim.x is a multiple of 32),
  // so its class inverse is read from HBM once into that XCD's L2 and the
  // other quarters hit there.
  const int L = blockIdx.x, slot = L >> 3;
  const int chunk = (slot >> 2) * 8 + (L & 7), quarter = slot & 3;
  if (chunk >= a.nchunks) return;
  const int *ch = a.chk + 3 * chunk;
  const int c = ch[0], q0 = ch[1] + 64 * quarter, qn = min(64, ch[2] - 64 * quarter);
  if (qn <= 0) return;
  const int m = a.m, ld = a.ld, r0 = ROWS * blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kq = lane >> 4;
  const int ar = tid & 127, ak = tid >> 7;
  const C *Ab = MM::mat(a) + (size_t)c * m * ld + (size_t)ak * ld + r0 + ar;
  const unsigned *pres = a.cpres + (size_t)c * a.pwords;
  const int pn = a.pnode[q0 + min(lane, qn - 1)];
  // Every load below is issued unconditionally from a clamped, valid address
  // (a load under a branch makes the compiler wait for it before the
  // branches join, one memory latency per element), and the raw values are
  // masked only when the slice is stored to LDS, one trip later: masking
  // right after the loads would wait for them before the matrix-core work.
  C pa[8 * NRT];
  T px[4];
  auto fetch = [&](int k0) {
    const C *Ak = Ab + (size_t)k0 * ld;   // A[r][k] = A[k][r]: row k of the slice
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < NRT; ++i) pa[j * NRT + i] = Ak[(size_t)(4 * j) * ld + 128 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      px[j] = a.x[min(max(pn + koff[k0 + wave + 8 * j], 0), a.xlen - 1)];
  };
  v4 acc[NRT][4];
#pragma unroll
  for (int i = 0; i < NRT; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[i][t] = v4{0, 0, 0, 0};
  for (int k = tid; k < KTAB; k += 512) {
    koff[k] = k < m ? pxoff[k] : 0;
    kmask[k] = k < m && ((pres[k >> 5] >> (k & 31)) & 1u) ? C(1) : C(0);
  }
  __syncthreads();
  const int nslice = (m + 31) >> 5;
  fetch(0);
  for (int sl = 0; sl < nslice; ++sl) {
    const int k0 = 32 * sl;
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < NRT; ++i) {
        const int k = ak + 4 * j, r = ar + 128 * i;
        As[k * RS + r] = ((r0 + r < m) & (k0 + k < m)) ? pa[j * NRT + i] : C(0);
      }
    // absent modes and missing patches are scaled by 0 (not selected: a
    // select on a loaded value would be turned back into a branch)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kr = wave + 8 * j, k = k0 + kr;
      const C mk = lane < qn ? kmask[k] : C(0);
      Xs[kr * XS + lane] = (C)px[j] * mk;
    }
    __syncthreads();
    if (sl + 1 < nslice) fetch(32 * (sl + 1));
#pragma unroll
    for (int k4 = 0; k4 < 8; ++k4) {
      const int kr = 4 * k4 + kq;
      C bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = Xs[kr * XS + 16 * t + n];
#pragma unroll
      for (int i = 0; i < NRT; ++i) {
        const C av = As[kr * RS + 16 * (wave + 8 * i) + n];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[i][t] = MM::mma(av, bv[t], acc[i][t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NRT; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = 16 * t + n;
      if (q < qn)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = r0 + 16 * (wave + 8 * i) + MM::row(j, kq);
          if (rr < m) a.Ys[(size_t)rr * a.nsh + q0 + q] = (double)acc[i][t][j];
        }
    }
}

template <typename T, int NKS>
static void launch_class32_nks(const Geo &g, const PatchTables &pt, const PatchArgs<T> &a,
                               hipStream_t s) {
  const int nrt = (a.m + 15) / 16;
  dim3 grid((nrt + 7) / 8, a.nchunks);
  patch_class_mfma32_kernel<T, NKS><<<grid, 512, (size_t)NKS * 4 * 16 * sizeof(float), s>>>(
      g, pt.pxoff, a);
}

template <typename T, typename C, int NRT>
static void launch_class_tile(const Geo &g, const PatchTables &pt, const PatchArgs<T> &a,
                              hipStream_t s) {
  (void)g;
  // chunks hold <= 256 patches (four quarters of 64)
  const dim3 grid(4 * ((a.nchunks + 7) / 8 * 8), (a.m + 128 * NRT - 1) / (128 * NRT));
  if (a.m <= kSmallPatchM)
    patch_class_tile_kernel<T, C, NRT, 384><<<grid, 512, 0, s>>>(pt.pxoff, a);
  else
    patch_class_tile_kernel<T, C, NRT, kKTab><<<grid, 512, 0, s>>>(pt.pxoff, a);
}

// Mixed form: FP32 class products (m <= 32 on the register-tile kernel).
// FP64 form: register-resident inverse rows for m <= kSmallPatchM, the
// LDS-streamed FP64 kernel above that.
template <typename T>
static bool launch_class32(const Geo &g, const PatchTables &pt, const PatchArgs<T> &a,
                           hipStream_t s) {
  if (!a.matS32) {
    if (a.m <= kSmallPatchM) return false;
    launch_class_tile<T, double, 1>(g, pt, a, s);
    return true;
  }
  if (a.m <= 32) {
    launch_class32_nks<T, 8>(g, pt, a, s);   // nks <= 8
    return true;
  }
  const int rows = a.class_rows > 0 ? a.class_rows : a.m > 256 ? 3 : a.m > 128 ? 2 : 1;
  if (rows >= 3) launch_class_tile<T, float, 3>(g, pt, a, s);
  else if (rows == 2) launch_class_tile<T, float, 2>(g, pt, a, s);
  else launch_class_tile<T, float, 1>(g, pt, a, s);
  return true;
}

template <typename T, int NKS>
static void launch_class_nks(const Geo &g, const PatchTables &pt, const PatchArgs<T> &a,
                             hipStream_t s) {
  const int nrt = (a.m + 15) / 16;
  dim3 grid((nrt + 7) / 8, a.nchunks);
  patch_class_mfma_kernel<T, NKS><<<grid, 512, (size_t)NKS * 4 * 16 * sizeof(double), s>>>(
      g, pt.pxoff, a);
}

template <typename T>
static void launch_class(const Geo &g, const PatchTables &pt, const PatchArgs<T> &a,
                         hipStream_t s) {
  const int nks = (a.m + 3) / 4;
  if (nks <= 8) launch_class_nks<T, 8>(g, pt, a, s);
  else if (nks <= 16) launch_class_nks<T, 16>(g, pt, a, s);
  else if (nks <= 24) launch_class_nks<T, 24>(g, pt, a, s);
  else if (nks <= 32) launch_class_nks<T, 32>(g, pt, a, s);
  else if (nks <= 48) launch_class_nks<T, 48>(g, pt, a, s);
  else if (nks <= 64) launch_class_nks<T, 64>(g, pt, a, s);
  else if (nks <= 88) launch_class_nks<T, 88>(g, pt, a, s);
  else launch_class_nks<T, 96>(g, pt, a, s);
}

// Owner gather with the smoother epilogue: out = delta, xs = (first ? 0 :
// xs) + omega * delta.  One thread per (grid point, plane).
template <typename T>
__global__ __launch_bounds__(256) void patch_gather_kernel(Geo g, const int *__restrict__ prow,
                                                           const int *__restrict__ pinfoP,
                                                           PatchArgs<T> a) {
  const int P = blockIdx.y;
  const int gi = blockIdx.x * 256 + threadIdx.x;
  if (gi >= g.G) return;
  int gc[3];
  node_coords(g, gi, gc);
  const int info = pinfoP[P], vmask = info & 7, bmask = (info >> 8) & 7;
  bool valid = true;
  for (int ax = 0; ax < g.d; ++ax) {
    if (((bmask >> ax) & 1) && gc[ax] == g.n[ax]) valid = false;
    if ((vmask >> ax) & 1) {
      if (gc[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) valid = false;
      if (gc[ax] == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) valid = false;
    }
  }
  double acc = 0.0;
  if (valid) {
    // all patch ids first, then all products (the loads of each pass are
    // independent and in flight together); summed in the fixed order cb
    const int nc = g.d == 3 ? 27 : 9;
    int pis[27];
#pragma unroll
    for (int cb = 0; cb < 27; ++cb) {
      pis[cb] = -1;
      if (cb >= nc) continue;
      const int dl[3] = {cb % 3 - 1, (cb / 3) % 3 - 1, g.d == 3 ? cb / 9 - 1 : 0};
      int vcn[3] = {0, 0, 0};
      bool ok = true;
      for (int ax = 0; ax < g.d; ++ax) {
        // a bubble of element c sits in the patches of nodes c and c+1
        if (((bmask >> ax) & 1) && dl[ax] == 1) ok = false;
        vcn[ax] = gc[ax] - dl[ax];
        ok = ok && vcn[ax] >= 0 && vcn[ax] <= g.n[ax];
      }
      if (ok) pis[cb] = a.pid[vcn[0] + g.gn[0] * (vcn[1] + g.gn[1] * vcn[2])];
    }
    double vals[27];
#pragma unroll
    for (int cb = 0; cb < 27; ++cb) {
      const int pi = pis[cb];
      vals[cb] = 0.0;
      if (pi < 0) continue;
      const int row = prow[P * 27 + cb];
      vals[cb] = pi < a.nsh ? a.Ys[(size_t)row * a.nsh + pi]
                            : a.Yu[(size_t)(pi - a.nsh) * a.m + row];
    }
#pragma unroll
    for (int cb = 0; cb < 27; ++cb)
      if (pis[cb] >= 0) acc += vals[cb];
  }
  const T val = valid ? (T)acc : T(0);
  const size_t oi = (size_t)P * g.G + gi;
  a.out[oi] = val;
  if (a.xs) {
    const T xo = a.first ? T(0) : a.xs[oi];
    a.xs[oi] = xo + a.omega * val;
  }
}

template <typename T>
void launch_patch_op(const Geo &g, const Tables &t, const PatchTables &pt, const PatchArgs<T> &a,
                     hipStream_t s) {
  if (a.npu > 0) {
    if (a.m <= kSmallPatchM && !a.gemv_band) {
      patch_gemv_kernel<T><<<a.npu, 256, 0, s>>>(g, pt.pxoff, pt.pinfo, a);
    } else {
      const int nbands = (a.ntile + kBandT - 1) / kBandT, npairs = nbands * (nbands + 1) / 2;
      patch_gemv_band_kernel<T><<<a.npu * npairs, 256, 0, s>>>(g, pt.pxoff, pt.pinfo, a, nbands,
                                                               npairs, a.Pband);
      if (a.stored_only) return;   // timing hook: the band kernel alone
      const size_t rows = (size_t)a.npu * a.m;
      patch_band_reduce_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(
          a.Pband, a.m, nbands, npairs, a.npu, a.Yu);
    }
  }
  if (a.stored_only) return;
  if (a.nsh > 0 && a.nchunks > 0) {
    if (!launch_class32<T>(g, pt, a, s)) launch_class<T>(g, pt, a, s);
  }
  dim3 grid((g.G + 255) / 256, a.nP_out);
  patch_gather_kernel<T><<<grid, 256, 0, s>>>(g, pt.prow, t.pinfo, a);
}
template void launch_patch_op<double>(const Geo &, const Tables &, const PatchTables &,
                                      const PatchArgs<double> &, hipStream_t);

}  // namespace fcm
