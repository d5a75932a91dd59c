// Setup kernels of libfcm (gfx950): everything that builds the hierarchy.
//
//  classify        element state from ball/box tests (Section 2.1)
//  integrate       cut-cell stiffness and load by recursive bisection of cut
//                  cells (Section 4.3.1); uncut sub-cells use separable closed
//                  forms, cut leaf sub-cells a (p+1)^d Gauss rule with alpha
//                  per point (eq. weakform)
//  phys/traction   loads of uncut elements and of box-face tractions
//  form/invert     elementwise additive Schwarz blocks P_i^T A_l P_i (eq.
//                  AdditiveSchwarz) and their inverses (Jacobi-scaled
//                  Gauss-Jordan sweeps in FP64)
//  coarse          stencil of the p = 1 matrix and the block Schur
//                  complements of its layer-block-tridiagonal form
//
// All arithmetic is FP64; the setup is bound by FP64 VALU throughput.
#include <cstdio>

#include "fcm_internal.hpp"

namespace fcm {

// ------------------------------------------------------------ device helpers
// Square of FCM_GEOM_SQUARE: point in its frame.
__device__ inline void square_frame_dev(const Geo &g, const double *x, double *xr) {
  const double rx = x[0] - g.sq[0], ry = x[1] - g.sq[1];
  xr[0] = g.sq[3] * rx + g.sq[4] * ry;
  xr[1] = -g.sq[4] * rx + g.sq[3] * ry;
}

__device__ inline bool inside_square_dev(const Geo &g, const double *x) {
  double xr[2];
  square_frame_dev(g, x, xr);
  return fabs(xr[0]) <= g.sq[2] && fabs(xr[1]) <= g.sq[2];
}

// Box against the (convex) square: kPhys if all four corners are inside,
// kVoid if an axis of the box or of the square separates the two (touching
// counts as separated), kCut otherwise.
__device__ inline int classify_square_dev(const Geo &g, const double *lo, const double *hi) {
  const double bx[4] = {lo[0], hi[0], hi[0], lo[0]}, by[4] = {lo[1], lo[1], hi[1], hi[1]};
  bool all = true;
  for (int i = 0; i < 4; ++i) {
    const double x[2] = {bx[i], by[i]};
    all = all && inside_square_dev(g, x);
  }
  if (all) return kPhys;
  const double cx = g.sq[0], cy = g.sq[1], hs = g.sq[2], cs = g.sq[3], sn = g.sq[4];
  const double ux = cs, uy = sn, vx = -sn, vy = cs;
  double sx[4], sy[4];
  const int sgn[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
  for (int i = 0; i < 4; ++i) {
    sx[i] = cx + hs * (sgn[i][0] * ux + sgn[i][1] * vx);
    sy[i] = cy + hs * (sgn[i][0] * uy + sgn[i][1] * vy);
  }
  const double ax[4] = {1.0, 0.0, ux, vx}, ay[4] = {0.0, 1.0, uy, vy};
  for (int k = 0; k < 4; ++k) {
    double bmin = 1e300, bmax = -1e300, smin = 1e300, smax = -1e300;
    for (int i = 0; i < 4; ++i) {
      const double pb = bx[i] * ax[k] + by[i] * ay[k], ps = sx[i] * ax[k] + sy[i] * ay[k];
      bmin = fmin(bmin, pb);
      bmax = fmax(bmax, pb);
      smin = fmin(smin, ps);
      smax = fmax(smax, ps);
    }
    if (bmax <= smin || smax <= bmin) return kVoid;
  }
  return kCut;
}

// Popcorn level set (FCM_GEOM_POPCORN); ball holds the twelve bump centres
// (x, y, z, unused).
constexpr double kPopR0 = 0.6, kPopA = 3.0, kPopSigma = 0.2;
__device__ inline double popcorn_phi_dev(const double *ball, const double *x) {
  double f = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - kPopR0;
  for (int k = 0; k < 12; ++k) {
    const double *c = ball + 4 * k;
    const double d2 = (x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) +
                      (x[2] - c[2]) * (x[2] - c[2]);
    f -= kPopA * exp(-d2 / (kPopSigma * kPopSigma));
  }
  return f;
}

// phi at the box centre against a bound of its change over the box: |grad|x||
// = 1 plus, per bump, the largest (2A/sigma^2) d exp(-d^2/sigma^2) over the
// box's distances d to the centre (rising up to sigma/sqrt(2), then falling).
// kVoid if phi > 0 on the whole box, kPhys if phi <= 0 on it, else kCut.
__device__ inline int classify_popcorn_dev(const double *ball, const double *lo,
                                           const double *hi) {
  double c[3], r2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    c[ax] = 0.5 * (lo[ax] + hi[ax]);
    r2 += (hi[ax] - lo[ax]) * (hi[ax] - lo[ax]);
  }
  const double rad = 0.5 * sqrt(r2);
  const double s2 = kPopSigma * kPopSigma, dpk = kPopSigma / sqrt(2.0);
  double L = 1.0;
  for (int k = 0; k < 12; ++k) {
    const double *b = ball + 4 * k;
    double dmin2 = 0.0, dmax2 = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
      const double nr = fmin(fmax(b[ax], lo[ax]), hi[ax]) - b[ax];
      dmin2 += nr * nr;
      const double fa = fmax(fabs(lo[ax] - b[ax]), fabs(hi[ax] - b[ax]));
      dmax2 += fa * fa;
    }
    const double dmin = sqrt(dmin2), dmax = sqrt(dmax2);
    const double d = dmax <= dpk ? dmax : (dmin >= dpk ? dmin : dpk);
    L += 2.0 * kPopA / s2 * d * exp(-d * d / s2);
  }
  const double f = popcorn_phi_dev(ball, c), slack = L * rad;
  if (f - slack > 0.0) return kVoid;
  if (f + slack <= 0.0) return kPhys;
  return kCut;
}

__device__ inline int classify_box_dev(const Geo &g, const double *ball, const double *lo,
                                       const double *hi) {
  if (g.geom == FCM_GEOM_SQUARE) return classify_square_dev(g, lo, hi);
  if (g.geom == FCM_GEOM_POPCORN) return classify_popcorn_dev(ball, lo, hi);
  if (g.geom == FCM_GEOM_BOX_MINUS_BALLS) {
    bool any = false;
    for (int j = 0; j < g.nballs; ++j) {
      const double *b = ball + 4 * j;
      double dmin2 = 0.0, dmax2 = 0.0;
      for (int ax = 0; ax < g.d; ++ax) {
        double c = b[ax];
        double nr = fmin(fmax(c, lo[ax]), hi[ax]) - c;
        dmin2 += nr * nr;
        double fa = fmax(fabs(lo[ax] - c), fabs(hi[ax] - c));
        dmax2 += fa * fa;
      }
      double r = b[3];
      if (sqrt(dmax2) < r) return kVoid;
      if (sqrt(dmin2) < r) any = true;
    }
    return any ? kCut : kPhys;
  }
  const double *b = ball;
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int ax = 0; ax < g.d; ++ax) {
    double c = b[ax];
    double nr = fmin(fmax(c, lo[ax]), hi[ax]) - c;
    dmin2 += nr * nr;
    double fa = fmax(fabs(lo[ax] - c), fabs(hi[ax] - c));
    dmax2 += fa * fa;
  }
  double r = b[3];
  if (sqrt(dmin2) >= r) return kVoid;
  if (sqrt(dmax2) <= r) return kPhys;
  return kCut;
}

__device__ inline bool inside_phys_dev(const Geo &g, const double *ball, const double *x) {
  if (g.geom == FCM_GEOM_SQUARE) return inside_square_dev(g, x);
  if (g.geom == FCM_GEOM_POPCORN) return popcorn_phi_dev(ball, x) <= 0.0;
  if (g.geom == FCM_GEOM_BOX_MINUS_BALLS) {
    for (int j = 0; j < g.nballs; ++j) {
      const double *b = ball + 4 * j;
      double d2 = 0.0;
      for (int ax = 0; ax < g.d; ++ax) {
        double t = x[ax] - b[ax];
        d2 += t * t;
      }
      if (d2 < b[3] * b[3]) return false;
    }
    return true;
  }
  double d2 = 0.0;
  for (int ax = 0; ax < g.d; ++ax) {
    double t = x[ax] - ball[ax];
    d2 += t * t;
  }
  return d2 <= ball[3] * ball[3];
}

// Integrated Legendre modes on [-1,1]: vertex modes (1 -+ xi)/2 and
// (L_j - L_{j-2}) / sqrt(2(2j-1)); Legendre values by the three-term recurrence.
__device__ inline void modes1d_dev(int p, double xi, double *v, double *dv) {
  double L[kMaxP + 1];
  L[0] = 1.0;
  if (p >= 1) L[1] = xi;
  for (int n = 1; n < p; ++n) L[n + 1] = ((2 * n + 1) * xi * L[n] - n * L[n - 1]) / (n + 1);
  v[0] = 0.5 * (1.0 - xi);
  v[1] = 0.5 * (1.0 + xi);
  dv[0] = -0.5;
  dv[1] = 0.5;
  for (int j = 2; j <= p; ++j) {
    double s = rsqrt(2.0 * (2 * j - 1));
    v[j] = (L[j] - L[j - 2]) * s;
    dv[j] = (2 * j - 1) * L[j - 1] * s;
  }
}

__device__ inline double source_dev(const Geo &g, const double *gsrc, int ngauss, double fconst,
                                    const double *x, int d) {
  double f = fconst;
  if (g.trig[0] != 0.0) {
    double xr[2];
    square_frame_dev(g, x, xr);
    f += g.trig[0] * cos(g.trig[1] * xr[0]) * sin(g.trig[1] * xr[1]);
  }
  if (g.geom == FCM_GEOM_POPCORN) {
    // -Lap of the prescribed solution x^3 + x y^2 + y^3 + z^4 + sin(3 (x^2 + y^2))
    const double s = x[0] * x[0] + x[1] * x[1];
    f -= 8.0 * x[0] + 6.0 * x[1] + 12.0 * x[2] * x[2] + 12.0 * cos(3.0 * s) -
         36.0 * s * sin(3.0 * s);
  }
  for (int k = 0; k < ngauss; ++k) {
    const double *s = gsrc + 5 * k;
    double d2 = 0.0;
    for (int ax = 0; ax < d; ++ax) {
      double t = x[ax] - s[2 + ax];
      d2 += t * t;
    }
    f += s[0] * exp(-d2 / (s[1] * s[1]));
  }
  return f;
}

__device__ inline void elem_coords(const Geo &g, int e, int *c) {
  c[0] = e % g.n[0];
  int r = e / g.n[0];
  c[1] = r % g.n[1];
  c[2] = r / g.n[1];
}

// ------------------------------------------------------------------ classify
__global__ void classify_kernel(Geo g, const double *ball, uint8_t *state) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  int c[3];
  elem_coords(g, e, c);
  double lo[3], hi[3];
  for (int ax = 0; ax < 3; ++ax) {
    lo[ax] = g.lo[ax] + c[ax] * g.h[ax];
    hi[ax] = lo[ax] + g.h[ax];
  }
  state[e] = (uint8_t)classify_box_dev(g, ball, lo, hi);
}

void launch_classify(const Geo &g, const double *ball, uint8_t *state, hipStream_t s) {
  classify_kernel<<<(g.E + 255) / 256, 256, 0, s>>>(g, ball, state);
}

// ----------------------------------------------------------------- integrate
// One workgroup per cut element (or the reference element).  Leaves of the
// sub-cell tree (bisection of cut sub-cells to the given depth) are
// enumerated breadth first in a fixed order; every leaf gets the tensor Gauss
// rule with NP = p+1 points per axis and alpha evaluated per point (constant
// on uncut leaves), as in Section 4.3.1.  The stiffness moments
//   G^{kl}_{ab} = sum_q w_q alpha_q (dN_a/dx_k)(dN_b/dx_l)
// over scalar tensor modes a = (a0,a1,a2), b = (b0,b1,b2) are evaluated by sum
// factorisation over the leaf's tensor points (F = value V or derivative D of
// the 1D modes per axis, chosen by the moment):
//   T1[q0 q1][a2 b2] = sum_q2 F2_a2(q2) F2_b2(q2) W[q0 q1 q2]     (LDS)
//   t2[q0]           = sum_q1 F1_a1(q1) F1_b1(q1) T1[q0 q1][a2 b2] (thread)
//   G[a0 b0; r]     += sum_q0 F0_a0(q0) F0_b0(q0) t2[q0]           (registers)
// Each thread owns one rest index r = (a1,b1,a2,b2) and all NP^2 pairs
// (a0,b0), so the element matrix accumulates in registers in a fixed order.
// Poisson: K = kappa sum_k G^{kk}; elasticity: K_{(a,i),(b,j)} = lambda G^{ij}
// + mu G^{ji} + mu delta_ij sum_k G^{kk} (eq. weakform with isotropic C).
constexpr int kIntThreads = 256;

struct IntegArgs {
  Geo g;
  const double *ball, *gsrc, *gxw;
  const int *smap;
  int ngauss, ms, m, elastic;
  double fconst, kappa, lam, mu;
  double bf[3];
  const int *elist;
  int ref_mode;
  double *Kout, *be_all;
  int max_leaves, max_cur, max_child;
};

__device__ inline int leaf_pack(int lvl, int kind, int ix, int iy, int iz) {
  return lvl | (kind << 3) | (ix << 5) | (iy << 10) | (iz << 15);
}

template <int NP>
__global__ __launch_bounds__(kIntThreads) void integrate_kernel(IntegArgs A) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
  extern __shared__ double smem[];
  const Geo &g = A.g;
  const int d = g.d, nf = g.nf, ms = A.ms, m = A.m;
  double *Fv = smem;                     // [3][NP q][NP a] mode values
  double *Fd = Fv + 3 * NP2;             // [3][NP][NP] physical derivatives
  double *W = Fd + 3 * NP2;              // [NP^3] w * alpha
  double *Wf = W + NP3;                  // [NP^3] w * alpha * f
  double *P = Wf + NP3;                  // [2 axes][4 types][NP q][NP a][NP b]
  double *T1 = P + 8 * NP3;              // [2][NP^2 (q0,q1)][NP^2 (a2,b2)]
  int *leaves = (int *)(T1 + 2 * NP2 * NP2);
  int *curA = leaves + A.max_leaves;
  int *curB = curA + A.max_cur;
  uint8_t *chst = (uint8_t *)(curB + A.max_cur);
  __shared__ int s_nleaf, s_ncur;

  const int tid = threadIdx.x;
  const int e = A.ref_mode ? 0 : A.elist[blockIdx.x];
  int ec[3];
  elem_coords(g, e, ec);
  double elo[3], ehi[3];
  for (int ax = 0; ax < 3; ++ax) elo[ax] = g.lo[ax] + ec[ax] * g.h[ax];
  if (A.ref_mode) elo[0] = elo[1] = elo[2] = 0.0;
  for (int ax = 0; ax < 3; ++ax) ehi[ax] = elo[ax] + g.h[ax];

  // ---- enumerate leaves
  if (tid == 0) {
    if (A.ref_mode) {
      leaves[0] = leaf_pack(0, kPhys, 0, 0, 0);
      s_nleaf = 1;
      s_ncur = 0;
    } else if (g.depth == 0) {
      leaves[0] = leaf_pack(0, kCut, 0, 0, 0);
      s_nleaf = 1;
      s_ncur = 0;
    } else if (classify_box_dev(g, A.ball, elo, ehi) == kPhys) {
      // an uncut element with a stored matrix (an immersed edge's penalty
      // lies on it): one Gauss rule over the element, as for K_ref
      leaves[0] = leaf_pack(0, kPhys, 0, 0, 0);
      s_nleaf = 1;
      s_ncur = 0;
    } else {
      curA[0] = leaf_pack(0, kCut, 0, 0, 0);
      s_nleaf = 0;
      s_ncur = 1;
    }
  }
  __syncthreads();
  for (int lvl = 0; lvl < g.depth && !A.ref_mode; ++lvl) {
    int *cur = (lvl & 1) ? curB : curA;
    int *nxt = (lvl & 1) ? curA : curB;
    const int ncur = s_ncur;
    const int nch = ncur << d;
    const double sub = 1.0 / (double)(1 << (lvl + 1));
    for (int c = tid; c < nch; c += kIntThreads) {
      int par = cur[c >> d];
      int bits = c & ((1 << d) - 1);
      int idx[3] = {(par >> 5) & 31, (par >> 10) & 31, (par >> 15) & 31};
      double lo[3], hi[3];
      for (int ax = 0; ax < 3; ++ax) {
        int ci = ax < d ? 2 * idx[ax] + ((bits >> ax) & 1) : 0;
        lo[ax] = elo[ax] + ci * sub * g.h[ax];
        hi[ax] = lo[ax] + sub * g.h[ax];
      }
      chst[c] = (uint8_t)classify_box_dev(g, A.ball, lo, hi);
    }
    __syncthreads();
    if (tid == 0) {
      int nl = s_nleaf, nn = 0;
      for (int c = 0; c < nch; ++c) {
        int par = cur[c >> d];
        int bits = c & ((1 << d) - 1);
        int idx[3] = {(par >> 5) & 31, (par >> 10) & 31, (par >> 15) & 31};
        int ci[3];
        for (int ax = 0; ax < 3; ++ax) ci[ax] = ax < d ? 2 * idx[ax] + ((bits >> ax) & 1) : 0;
        int st = chst[c];
        if (st != kCut) leaves[nl++] = leaf_pack(lvl + 1, st, ci[0], ci[1], ci[2]);
        else if (lvl + 1 < g.depth) nxt[nn++] = leaf_pack(lvl + 1, kCut, ci[0], ci[1], ci[2]);
        else leaves[nl++] = leaf_pack(lvl + 1, kCut, ci[0], ci[1], ci[2]);
      }
      s_nleaf = nl;
      s_ncur = nn;
    }
    __syncthreads();
  }
  const int nleaf = s_nleaf;
  const int nq2 = d == 3 ? NP : 1;
  const int Q = NP2 * nq2;
  const double *gx = A.gxw, *gw = A.gxw + NP;
  const int R = d == 3 ? NP2 * NP2 : NP2;           // rest indices (a1,b1[,a2,b2])
  const int ngroups = A.elastic ? d * d : 1;        // moment groups
  double bacc[2] = {0.0, 0.0};
  const bool want_load = !A.ref_mode;
  double *Kel = A.ref_mode ? A.Kout : A.Kout + (size_t)blockIdx.x * m * m;

  for (int r0 = 0; r0 < R; r0 += kIntThreads) {
    const int r = r0 + tid;
    const bool ractive = r < R;
    const int rr = ractive ? r : 0;
    const int a1 = (rr % NP2) / NP, b1 = rr % NP;
    const int a2 = d == 3 ? (rr / NP2) / NP : 0, b2 = d == 3 ? (rr / NP2) % NP : 0;
    if (A.elastic && ractive) {
      // this thread owns the K entries of its (a, b) pairs for all components
      for (int a0 = 0; a0 < NP; ++a0)
        for (int b0 = 0; b0 < NP; ++b0) {
          const int sa = a0 + NP * (a1 + NP * a2), sb = b0 + NP * (b1 + NP * b2);
          if (A.smap[sa * nf] < 0 || A.smap[sb * nf] < 0) continue;   // not a trunk mode
          for (int ci = 0; ci < nf; ++ci)
            for (int cj = 0; cj < nf; ++cj)
              Kel[(size_t)A.smap[sa * nf + ci] * m + A.smap[sb * nf + cj]] = 0.0;
        }
    }
    for (int grp = 0; grp < ngroups; ++grp) {
      const int mk = grp / d, ml = grp % d;   // elasticity moment (k, l)
      double acc[NP2];
#pragma unroll
      for (int i = 0; i < NP2; ++i) acc[i] = 0.0;
      const bool do_load = want_load && r0 == 0 && grp == 0;
      for (int lf = 0; lf < nleaf; ++lf) {
        const int pk = leaves[lf];
        const int lvl = pk & 7, kind = (pk >> 3) & 3;
        const int li[3] = {(pk >> 5) & 31, (pk >> 10) & 31, (pk >> 15) & 31};
        const double half = 1.0 / (1 << lvl);
        __syncthreads();
        // phase A: 1D tables at the leaf's Gauss points, point weights
        if (tid < d * NP) {
          const int ax = tid / NP, q = tid % NP;
          const double xi = -1.0 + (2.0 * li[ax] + 1.0) * half + half * gx[q];
          double v[kMaxP + 1], dv[kMaxP + 1];
          modes1d_dev(NP - 1, xi, v, dv);
          const double sc = 2.0 / g.h[ax];
          for (int a = 0; a < NP; ++a) {
            Fv[(ax * NP + q) * NP + a] = v[a];
            Fd[(ax * NP + q) * NP + a] = sc * dv[a];
          }
        }
        for (int q = tid; q < Q; q += kIntThreads) {
          const int qc[3] = {q % NP, (q / NP) % NP, q / NP2};
          double x[3] = {0.0, 0.0, 0.0};
          double w = 1.0;
          for (int ax = 0; ax < d; ++ax) {
            const double xi = -1.0 + (2.0 * li[ax] + 1.0) * half + half * gx[qc[ax]];
            x[ax] = elo[ax] + 0.5 * (xi + 1.0) * g.h[ax];
            w *= gw[qc[ax]] * half * 0.5 * g.h[ax];
          }
          double al;
          if (kind == kPhys) al = 1.0;
          else if (kind == kVoid) al = g.alpha;
          else al = inside_phys_dev(g, A.ball, x) ? 1.0 : g.alpha;
          W[q] = w * al;
          if (do_load)
            Wf[q] = w * al * (A.elastic ? 1.0 : source_dev(g, A.gsrc, A.ngauss, A.fconst, x, d));
        }
        __syncthreads();
        // phase B: pair tables of axes 0, 1 and the q2-contraction T1
        for (int i = tid; i < 8 * NP3; i += kIntThreads) {
          const int ax = i / (4 * NP3), t = (i / NP3) & 3, q = (i / NP2) % NP;
          const int a = (i / NP) % NP, b = i % NP;
          const double fa = ((t >> 1) ? Fd : Fv)[(ax * NP + q) * NP + a];
          const double fb = ((t & 1) ? Fd : Fv)[(ax * NP + q) * NP + b];
          P[i] = fa * fb;
        }
        if (d == 3) {
          // T1[0]: axis-2 pair type of the group (Poisson: VV), T1[1]: DD (Poisson k = 2)
          const int t0 = A.elastic ? 2 * (mk == 2) + (ml == 2) : 0;
          const int nt = A.elastic ? 1 : 2;
          for (int i = tid; i < nt * NP2 * NP2; i += kIntThreads) {
            const int which = i / (NP2 * NP2), j = i % (NP2 * NP2);
            const int t = which ? 3 : t0;
            const int q01 = j / NP2, a2i = (j % NP2) / NP, b2i = j % NP;
            const double *Fa = (t >> 1) ? Fd : Fv, *Fb = (t & 1) ? Fd : Fv;
            double sum = 0.0;
            for (int q2 = 0; q2 < NP; ++q2)
              sum += Fa[(2 * NP + q2) * NP + a2i] * Fb[(2 * NP + q2) * NP + b2i] * W[q01 + NP2 * q2];
            T1[i] = sum;
          }
        } else {
          for (int i = tid; i < NP2; i += kIntThreads) T1[i] = W[i];
        }
        if (do_load) {
          for (int k = 0; k < 2; ++k) {
            const int sidx = tid + k * kIntThreads;
            if (sidx >= ms) continue;
            const int sc[3] = {sidx % NP, (sidx / NP) % NP, sidx / NP2};
            double sum = 0.0;
            for (int q = 0; q < Q; ++q) {
              const int qc[3] = {q % NP, (q / NP) % NP, q / NP2};
              double v = Wf[q] * Fv[qc[0] * NP + sc[0]] * Fv[(NP + qc[1]) * NP + sc[1]];
              if (d == 3) v *= Fv[(2 * NP + qc[2]) * NP + sc[2]];
              sum += v;
            }
            bacc[k] += sum;
          }
        }
        __syncthreads();
        // phase C: per-thread contraction over q1 and q0
        if (ractive) {
          const int ncombo = A.elastic ? 1 : d;
#pragma unroll 1
          for (int cb = 0; cb < ncombo; ++cb) {
            int t0, t1, tT;
            if (A.elastic) {
              t0 = 2 * (mk == 0) + (ml == 0);
              t1 = 2 * (mk == 1) + (ml == 1);
              tT = 0;
            } else {
              // Poisson moment k = cb: DD on axis k, VV elsewhere
              t0 = cb == 0 ? 3 : 0;
              t1 = cb == 1 ? 3 : 0;
              tT = (d == 3 && cb == 2) ? 1 : 0;
            }
            const double *P0 = P + t0 * NP3;
            const double *P1 = P + (4 + t1) * NP3 + a1 * NP + b1;
            const double *Tb = T1 + tT * NP2 * NP2 + a2 * NP + b2;
            const int tstride = d == 3 ? NP2 : 1;
#pragma unroll 1
            for (int q0 = 0; q0 < NP; ++q0) {
              double s2 = 0.0;
#pragma unroll
              for (int q1 = 0; q1 < NP; ++q1) s2 += P1[q1 * NP2] * Tb[(q0 + NP * q1) * tstride];
              const double *p0 = P0 + q0 * NP2;
#pragma unroll
              for (int ab = 0; ab < NP2; ++ab) acc[ab] += p0[ab] * s2;
            }
          }
        }
      }
      // ---- write this group's contribution
      if (ractive) {
#pragma unroll
        for (int a0 = 0; a0 < NP; ++a0)
#pragma unroll
          for (int b0 = 0; b0 < NP; ++b0) {
            const double G = acc[a0 * NP + b0];
            const int sa = a0 + NP * (a1 + NP * a2), sb = b0 + NP * (b1 + NP * b2);
            // tuples outside the trunk space have no local index
            if (A.smap[sa * nf] < 0 || A.smap[sb * nf] < 0) continue;
            if (!A.elastic) {
              Kel[(size_t)A.smap[sa] * m + A.smap[sb]] = A.kappa * G;
            } else {
              Kel[(size_t)A.smap[sa * nf + mk] * m + A.smap[sb * nf + ml]] += A.lam * G;
              Kel[(size_t)A.smap[sa * nf + ml] * m + A.smap[sb * nf + mk]] += A.mu * G;
              if (mk == ml)
                for (int c = 0; c < nf; ++c)
                  Kel[(size_t)A.smap[sa * nf + c] * m + A.smap[sb * nf + c]] += A.mu * G;
            }
          }
      }
    }
  }
  if (!want_load) return;
  for (int k = 0; k < 2; ++k) {
    const int sidx = tid + k * kIntThreads;
    if (sidx >= ms || A.smap[sidx * nf] < 0) continue;
    double *be = A.be_all + (size_t)e * m;
    if (!A.elastic) be[A.smap[sidx]] = bacc[k];
    else
      for (int c = 0; c < nf; ++c) be[A.smap[sidx * nf + c]] = A.bf[c] * bacc[k];
  }
}

void launch_integrate(const Geo &g, const Tables &t, const fcm_problem &pr, const int *elist,
                      int nlist, int ref_mode, double *Kout, double *be_all, int *flag,
                      hipStream_t s) {
  (void)flag;
  if (nlist <= 0) return;
  IntegArgs A;
  A.g = g;
  A.ball = t.ball;
  A.gsrc = t.gsrc;
  A.gxw = t.gxw;
  A.smap = t.smap;
  A.ngauss = pr.n_gauss;
  A.ms = t.ms;
  A.m = t.m;
  A.elastic = g.nf > 1;
  A.fconst = pr.f_const;
  A.kappa = pr.kappa;
  A.lam = pr.E * pr.nu / ((1.0 + pr.nu) * (1.0 - 2.0 * pr.nu));
  A.mu = pr.E / (2.0 * (1.0 + pr.nu));
  for (int i = 0; i < 3; ++i) A.bf[i] = pr.body_force[i];
  A.elist = elist;
  A.ref_mode = ref_mode;
  A.Kout = Kout;
  A.be_all = be_all;
  int maxl = 1, cur = 1, maxc = 1;
  for (int l = 1; l <= g.depth; ++l) {
    int c = 1 << (g.d * l);
    maxl += c;
    maxc = std::max(maxc, c);
    cur = std::max(cur, 1 << (g.d * (l - 1)));
  }
  A.max_leaves = maxl;
  A.max_cur = cur;
  A.max_child = maxc;
  const int np = g.p + 1, np2 = np * np, np3 = np2 * np;
  const size_t shm = (size_t)(6 * np2 + 2 * np3 + 8 * np3 + 2 * np2 * np2) * sizeof(double) +
                     (size_t)(maxl + 2 * cur) * sizeof(int) + maxc + 16;
  dim3 grid(ref_mode ? 1 : nlist);
  switch (np) {
    case 2: integrate_kernel<2><<<grid, kIntThreads, shm, s>>>(A); break;
    case 3: integrate_kernel<3><<<grid, kIntThreads, shm, s>>>(A); break;
    case 4: integrate_kernel<4><<<grid, kIntThreads, shm, s>>>(A); break;
    case 5: integrate_kernel<5><<<grid, kIntThreads, shm, s>>>(A); break;
    case 6: integrate_kernel<6><<<grid, kIntThreads, shm, s>>>(A); break;
    default: integrate_kernel<7><<<grid, kIntThreads, shm, s>>>(A); break;
  }
}

__global__ __launch_bounds__(64) void phys_rhs_kernel(Geo g, const double *gxw,
                                                      const double *vgauss, const int *smap,
                                                      const double *gsrc, int ngauss,
                                                      double fconst, double bf0, double bf1,
                                                      double bf2, int ms, int m,
                                                      const uint8_t *state, double *be_all) {
  __shared__ double fw[343];
  const int e = blockIdx.x;
  if (state[e] != kPhys) return;
  const int d = g.d, np = g.p + 1, np2 = np * np;
  const int Q = (d == 2) ? np2 : np2 * np;
  int ec[3];
  elem_coords(g, e, ec);
  const double *gx = gxw, *gw = gxw + np;
  const bool elastic = g.nf > 1;
  for (int q = threadIdx.x; q < Q; q += 64) {
    int qc[3] = {q % np, (q / np) % np, q / np2};
    double x[3] = {0, 0, 0}, w = 1.0;
    for (int ax = 0; ax < d; ++ax) {
      x[ax] = g.lo[ax] + ec[ax] * g.h[ax] + 0.5 * (gx[qc[ax]] + 1.0) * g.h[ax];
      w *= gw[qc[ax]] * 0.5 * g.h[ax];
    }
    fw[q] = w * (elastic ? 1.0 : source_dev(g, gsrc, ngauss, fconst, x, d));
  }
  __syncthreads();
  double *be = be_all + (size_t)e * m;
  for (int s = threadIdx.x; s < ms; s += 64) {
    if (smap[s * g.nf] < 0) continue;    // not a trunk mode
    int sc[3] = {s % np, (s / np) % np, s / np2};
    double sum = 0.0;
    for (int q = 0; q < Q; ++q) {
      int qc[3] = {q % np, (q / np) % np, q / np2};
      double v = fw[q];
      for (int ax = 0; ax < d; ++ax) v *= vgauss[qc[ax] * np + sc[ax]];
      sum += v;
    }
    if (!elastic) {
      be[smap[s]] = sum;
    } else {
      const double bfv[3] = {bf0, bf1, bf2};
      for (int c = 0; c < g.nf; ++c) be[smap[s * g.nf + c]] = bfv[c] * sum;
    }
  }
}

void launch_phys_rhs(const Geo &g, const Tables &t, const fcm_problem &pr, const uint8_t *state,
                     double *be_all, hipStream_t s) {
  phys_rhs_kernel<<<g.E, 64, 0, s>>>(g, t.gxw, t.vgauss, t.smap, t.gsrc, pr.n_gauss, pr.f_const,
                                     pr.body_force[0], pr.body_force[1], pr.body_force[2], t.ms,
                                     t.m, state, be_all);
}

// Box-face traction t on face (axis, side): int_face N_a t dA, closed form per mode.
// Penalty of the Dirichlet data on an immersed boundary (eq. weakform): one
// workgroup per element with boundary points; the mode values of up to 32
// points at a time are staged in LDS, then thread (a, b) adds
// beta sum_q w_q N_a N_b to K_e and thread a adds beta sum_q w_q g_q N_a to
// b_e, points in their stored order.
constexpr int kPenPts = 32;
__global__ __launch_bounds__(256) void edge_penalty_kernel(Geo g, const int *lm, int m,
                                                           const int *pel, const int *ptr,
                                                           const double *pts, double beta,
                                                           const int *kmat, double *Kcut,
                                                           double *be_all) {
  __shared__ double N[kPenPts * 64];
  __shared__ double W[kPenPts], Gv[kPenPts];
  const int e = pel[blockIdx.x];
  const int kid = kmat[e];
  if (kid <= 0) return;   // the host gives every penalty element a stored matrix
  int ec[3];
  elem_coords(g, e, ec);
  double *K = Kcut + (size_t)(kid - 1) * m * m;
  double *be = be_all + (size_t)e * m;
  const int np = g.p + 1;
  for (int q0 = ptr[blockIdx.x]; q0 < ptr[blockIdx.x + 1]; q0 += kPenPts) {
    const int nq = min(kPenPts, ptr[blockIdx.x + 1] - q0);
    __syncthreads();
    for (int i = threadIdx.x; i < nq * m; i += blockDim.x) {
      const int q = i / m, a = i % m;
      const double *pt = pts + 5 * (size_t)(q0 + q);
      double val = 1.0;
      for (int ax = 0; ax < g.d; ++ax) {
        const double xi = 2.0 * (pt[ax] - (g.lo[ax] + ec[ax] * g.h[ax])) / g.h[ax] - 1.0;
        double v[kMaxP + 1], dv[kMaxP + 1];
        modes1d_dev(np - 1, xi, v, dv);
        val *= v[lm[4 * a + ax]];
      }
      N[q * 64 + a] = val;
      if (a == 0) {
        W[q] = pt[3];
        Gv[q] = pt[4];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
      const int a = i / m, b = i % m;
      double s = 0.0;
      for (int q = 0; q < nq; ++q) s += W[q] * N[q * 64 + a] * N[q * 64 + b];
      K[i] += beta * s;
    }
    for (int a = threadIdx.x; a < m; a += blockDim.x) {
      double s = 0.0;
      for (int q = 0; q < nq; ++q) s += W[q] * Gv[q] * N[q * 64 + a];
      be[a] += beta * s;
    }
  }
}

void launch_edge_penalty(const Geo &g, const Tables &t, const int *pel, int nel, const int *ptr,
                         const double *pts, double beta, const int *kmat, double *Kcut,
                         double *be_all, hipStream_t s) {
  if (nel <= 0) return;
  edge_penalty_kernel<<<nel, 256, 0, s>>>(g, t.lm, t.m, pel, ptr, pts, beta, kmat, Kcut, be_all);
}

__global__ void traction_kernel(Geo g, const double *gxw, const double *vgauss, const int *smap,
                                int ms, int m, int face, double t0, double t1, double t2,
                                const uint8_t *state, double *be_all) {
  const int ax = face / 2, side = face % 2;
  const int np = g.p + 1;
  // enumerate elements on the face: index over the other axes
  int nface = 1;
  for (int k = 0; k < g.d; ++k)
    if (k != ax) nface *= g.n[k];
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nface * ms) return;
  int s = id % ms, fe = id / ms;
  int ec[3] = {0, 0, 0};
  for (int k = 0; k < g.d; ++k) {
    if (k == ax) continue;
    ec[k] = fe % g.n[k];
    fe /= g.n[k];
  }
  ec[ax] = side ? g.n[ax] - 1 : 0;
  int e = ec[0] + g.n[0] * (ec[1] + g.n[1] * ec[2]);
  if (state[e] == kVoid) return;
  int sc[3] = {s % np, (s / np) % np, s / (np * np)};
  if (sc[ax] != side) return;
  const double *gw = gxw + np;
  double val = 1.0;
  for (int k = 0; k < g.d; ++k) {
    if (k == ax) continue;
    double integ = 0.0;
    for (int q = 0; q < np; ++q) integ += gw[q] * vgauss[q * np + sc[k]];
    val *= integ * 0.5 * g.h[k];
  }
  const double tv[3] = {t0, t1, t2};
  double *be = be_all + (size_t)e * m;
  if (smap[s * g.nf] < 0) return;        // not a trunk mode
  for (int c = 0; c < g.nf; ++c) be[smap[s * g.nf + c]] += tv[c] * val;
}

void launch_traction_rhs(const Geo &g, const Tables &t, int face, const double *tvec,
                         const uint8_t *state, double *be_all, hipStream_t s) {
  int ax = face / 2;
  int nface = 1;
  for (int k = 0; k < g.d; ++k)
    if (k != ax) nface *= g.n[k];
  int tot = nface * t.ms;
  traction_kernel<<<(tot + 255) / 256, 256, 0, s>>>(g, t.gxw, t.vgauss, t.smap, t.ms, t.m, face,
                                                    tvec[0], tvec[1], tvec[2], state, be_all);
}

// Gather of element loads into the padded fine vector (owner computes).
__global__ void assemble_rhs_kernel(Geo g, const int *rows, const int *pinfo, const int *kmat,
                                    const double *be_all, int m, double *b) {
  const int P = blockIdx.y;
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= g.G) return;
  int gc[3] = {gi % g.gn[0], (gi / g.gn[0]) % g.gn[1], gi / (g.gn[0] * g.gn[1])};
  const int info = pinfo[P], vmask = info & 7, bmask = (info >> 8) & 7;
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
    for (int s = 0; s < (1 << g.d); ++s) {
      if (s & ~vmask) continue;
      int ec[3] = {gc[0] - (s & 1), gc[1] - ((s >> 1) & 1), gc[2] - ((s >> 2) & 1)};
      bool in = true;
      for (int ax = 0; ax < 3; ++ax) in = in && ec[ax] >= 0 && ec[ax] < g.n[ax];
      if (!in) continue;
      int e = ec[0] + g.n[0] * (ec[1] + g.n[1] * ec[2]);
      if (kmat[e] < 0) continue;
      acc += be_all[(size_t)e * m + rows[P * 8 + s]];
    }
  }
  b[(size_t)P * g.G + gi] = acc;
}

void launch_assemble_rhs(const Geo &g, const Tables &t, const int *kmat, const double *be_all,
                         double *b, hipStream_t s) {
  dim3 grid((g.G + 255) / 256, t.nP);
  assemble_rhs_kernel<<<grid, 256, 0, s>>>(g, t.rows, t.pinfo, kmat, be_all, t.m, b);
}

// ----------------------------------------------------- Schwarz block entries
// Entry (a,b) of P_i^T A_q P_i for the block of element e (local modes of e,
// level q): sum over the 3^d neighbours e' of the entries of K_{e'} that
// couple the same two global DOFs.  A vertex mode of e is shared with the
// neighbour on that side; bubble modes only with e itself along their axis.
__device__ inline bool local_dirichlet(const Geo &g, const int *lm4, const int *ec) {
  for (int ax = 0; ax < g.d; ++ax) {
    int a = lm4[ax];
    if (a > 1) continue;
    int node = ec[ax] + a;
    if (node == 0 && ((g.dir >> (2 * ax)) & 1)) return true;
    if (node == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) return true;
  }
  return false;
}

__device__ inline double block_entry(const Geo &g, const int *lm, const int *smap, int mp,
                                     const int *kmat, const double *Kref, const double *Kcut,
                                     const int *ec, int a, int b) {
  const int *la = lm + 4 * a, *lb = lm + 4 * b;
  const bool da = local_dirichlet(g, la, ec), db = local_dirichlet(g, lb, ec);
  if (da || db) return (a == b) ? 1.0 : 0.0;
  const int np = g.p + 1;
  double sum = 0.0;
  const int nofs = (g.d == 2) ? 9 : 27;
  for (int o = 0; o < nofs; ++o) {
    int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
    int ne[3];
    bool ok = true;
    for (int ax = 0; ax < 3; ++ax) {
      ne[ax] = ec[ax] + (ax < g.d ? off[ax] : 0);
      ok = ok && ne[ax] >= 0 && ne[ax] < g.n[ax];
    }
    if (!ok) continue;
    int kid = kmat[ne[0] + g.n[0] * (ne[1] + g.n[1] * ne[2])];
    if (kid < 0) continue;
    int ta[3] = {0, 0, 0}, tb[3] = {0, 0, 0};
    for (int ax = 0; ax < g.d && ok; ++ax) {
      int x = la[ax], y = lb[ax];
      if (off[ax] == -1) {
        ok = (x == 0) && (y == 0);
        x = 1;
        y = 1;
      } else if (off[ax] == 1) {
        ok = (x == 1) && (y == 1);
        x = 0;
        y = 0;
      }
      ta[ax] = x;
      tb[ax] = y;
    }
    if (!ok) continue;
    int sa = ta[0] + np * (ta[1] + np * ta[2]);
    int sb = tb[0] + np * (tb[1] + np * tb[2]);
    int ia = smap[sa * g.nf + la[3]], ib = smap[sb * g.nf + lb[3]];
    const double *K = kid == 0 ? Kref : Kcut + (size_t)(kid - 1) * mp * mp;
    sum += K[(size_t)ia * mp + ib];
  }
  return sum;
}

// Form and invert one block per workgroup entirely in LDS (m <= kSmallInv).
// Jacobi scaling, then an in-place Gauss-Jordan sweep over all pivots, which
// leaves -A^{-1}; SPD guarantees positive pivots (checked).
__global__ __launch_bounds__(256) void form_invert_small_kernel(Geo g, const int *lm,
                                                                const int *smap, int mp, int m,
                                                                const int *belems,
                                                                const int *kmat,
                                                                const double *Kref,
                                                                const double *Kcut,
                                                                double *inv64, float *inv32,
                                                                int *flag, double *kappa) {
  extern __shared__ double sm[];
  const int ldA = m + 1;
  double *Am = sm;               // m x (m+1)
  double *sc = Am + m * ldA;     // scale
  double *ck = sc + m;           // pivot column
  double *rk = ck + m;           // pivot row
  const int e = belems[blockIdx.x];
  int ec[3];
  elem_coords(g, e, ec);
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
    int a = i / m, b = i % m;
    Am[a * ldA + b] = block_entry(g, lm, smap, mp, kmat, Kref, Kcut, ec, a, b);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    double dg = Am[i * ldA + i];
    if (!(dg > 0.0)) atomicOr(flag, 1);
    sc[i] = dg > 0.0 ? rsqrt(dg) : 1.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
    int a = i / m, b = i % m;
    Am[a * ldA + b] *= sc[a] * sc[b];
  }
  __syncthreads();
  __shared__ double s_norm[2];
  if (threadIdx.x == 0) {
    // 1-norm of the scaled block (max absolute column sum; symmetric)
    double nm = 0.0;
    for (int b = 0; b < m; ++b) {
      double cs = 0.0;
      for (int a = 0; a < m; ++a) cs += fabs(Am[a * ldA + b]);
      nm = fmax(nm, cs);
    }
    s_norm[0] = nm;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      ck[i] = Am[i * ldA + k];
      rk[i] = Am[k * ldA + i];
    }
    __syncthreads();
    const double piv = ck[k];
    if (threadIdx.x == 0 && !(piv > 0.0)) atomicOr(flag, 1);
    const double P = 1.0 / piv;
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
      int a = i / m, b = i % m;
      double v;
      if (a != k && b != k) v = Am[a * ldA + b] - ck[a] * rk[b] * P;
      else if (a != k) v = ck[a] * P;
      else if (b != k) v = rk[b] * P;
      else v = -P;
      Am[a * ldA + b] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double nm = 0.0;
    for (int b = 0; b < m; ++b) {
      double cs = 0.0;
      for (int a = 0; a < m; ++a) cs += fabs(Am[a * ldA + b]);
      nm = fmax(nm, cs);
    }
    if (kappa) kappa[blockIdx.x] = s_norm[0] * nm;
  }
  double *o64 = inv64 + (size_t)blockIdx.x * m * m;
  float *o32 = inv32 + (size_t)blockIdx.x * m * m;
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
    int a = i / m, b = i % m;
    double v = -Am[a * ldA + b] * sc[a] * sc[b];
    o64[i] = v;
    o32[i] = (float)v;
  }
}

void launch_form_invert_small(const Geo &g, const Tables &t, int q, int m, const int *belems,
                              int nblocks, const int *kmat, const double *Kref,
                              const double *Kcut, double *inv64, float *inv32, int *flag,
                              double *kappa, hipStream_t s) {
  (void)q;
  if (nblocks <= 0) return;
  size_t shm = ((size_t)m * (m + 1) + 3 * m) * sizeof(double);
  form_invert_small_kernel<<<nblocks, 256, shm, s>>>(g, t.lm, t.smap, t.m, m, belems, kmat,
                                                     Kref, Kcut, inv64, inv32, flag, kappa);
}

__global__ void form_blocks_kernel(Geo g, const int *lm, const int *smap, int mp, int m,
                                   const int *belems, const int *kmat, const double *Kref,
                                   const double *Kcut, double *out) {
  const int blk = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  int ec[3];
  elem_coords(g, belems[blk], ec);
  out[(size_t)blk * m * m + i] =
      block_entry(g, lm, smap, mp, kmat, Kref, Kcut, ec, i / m, i % m);
}

void launch_form_blocks(const Geo &g, const Tables &t, int q, int m, const int *belems,
                        int nblocks, const int *kmat, const double *Kref, const double *Kcut,
                        double *out, hipStream_t s) {
  (void)q;
  if (nblocks <= 0) return;
  dim3 grid((m * m + 255) / 256, nblocks);
  form_blocks_kernel<<<grid, 256, 0, s>>>(g, t.lm, t.smap, t.m, m, belems, kmat, Kref, Kcut, out);
}

// --------------------------------------------- batched blocked SPD inverse
// In-place symmetric Gauss-Jordan sweep: sweeping pivot block K maps
// [[A_KK, A_KJ],[A_IK, A_IJ]] to [[-P, P A_KJ],[A_IK P, A_IJ - A_IK P A_KJ]]
// with P = A_KK^{-1}; after all K the matrix holds -A^{-1}.  Two levels of
// pivot blocks: the rows of an outer block of kPB = 128 pivots (the panel,
// copied to scratch) are swept in four steps of kTB = 32 pivots -- the pivot
// rows pivot by pivot in registers (product form), then the other panel
// rows by the same rank-32 step -- and the rest of the matrix then takes the
// four rank-32 updates of those steps at once, as one symmetric rank-128
// update on the FP64 matrix cores: sum_s R_s^T W_s with R_s and W_s the rows
// of step s as they were before and after that step (stacked, kPB rows).
// This is the step-by-step sweep with the updates of the rows outside the
// panel deferred and summed; only the order of the additions changes.  (The
// Schur-complement form R_K^T W_K with the panel before and after all four
// steps is equal in exact arithmetic but amounts to an explicit inverse of
// the 128 x 128 pivot block: on cut-cell patch blocks of scaled condition
// 1e12 and more it loses positivity.)  The matrix is Jacobi-scaled first.
constexpr int kTB = 32;
constexpr int kPB = 128;
// Batches of at least kTwoLevelBatch matrices larger than kTwoLevelN take the
// 128-pivot panels; the rest one trailing update per 32 pivots (fewer
// dependent launches for single coarse blocks, and no gain below ~400: the
// 343 x 343 patch blocks of the p = 3 Poisson cube set up 15 % faster that way).
constexpr int kTwoLevelBatch = 8;
constexpr int kTwoLevelN = 384;

__global__ void jacobi_scale_kernel(double *A, int n, double *scale, int *flag) {
  const int b = blockIdx.y;
  double *M = A + (size_t)b * n * n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double dg = M[(size_t)i * n + i];
    if (!(dg > 0.0)) atomicOr(flag, 1);
    scale[(size_t)b * n + i] = dg > 0.0 ? rsqrt(dg) : 1.0;
  }
}

// M <- sign * S M S, one wave per row; with nrm, also the largest absolute
// row sum (= 1-norm, the matrices are symmetric) of the result (sign > 0:
// the scaled matrix) or of the input (sign < 0: the swept matrix -B_s^{-1}),
// combined over rows by atomicMax on the bit pattern (order-preserving for
// non-negative doubles).
__global__ void apply_scale_kernel(double *A, int n, const double *scale, double sign,
                                   double *nrm) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= n) return;
  double *M = A + (size_t)b * n * n + (size_t)r * n;
  const double *s = scale + (size_t)b * n;
  const double sr = s[r];
  double sum_in = 0.0, sum_out = 0.0;
  for (int c = lane; c < n; c += 64) {
    const double v = M[c];
    const double w = sign * v * sr * s[c];
    M[c] = w;
    sum_in += fabs(v);
    sum_out += fabs(w);
  }
  if (!nrm) return;
  double rs = sign > 0.0 ? sum_out : sum_in;
  for (int off = 32; off > 0; off >>= 1) rs += __shfl_down(rs, off, 64);
  if (lane == 0)
    atomicMax((unsigned long long *)(nrm + b), (unsigned long long)__double_as_longlong(rs));
}

__global__ void kappa_product_kernel(const double *nrm, int batch, double *kappa) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) kappa[b] = nrm[b] * nrm[batch + b];
}

// Panel of outer block [k0, k0 + kb): Wp = rows k0.. of the matrix (kPB x n
// per matrix, rows past kb zero), read from the upper triangle, the only one
// kept during the two-level sweep: entry (k0 + t, c) is M[k0 + t][c] for c >= k0 + t and
// M[c][k0 + t] below the diagonal.  Workgroup (x, b) takes the columns
// [64 x, + 64): the transposed block M[c][k0 .. k0 + 128) of its columns is
// read along rows into LDS, so that both reads and the panel's writes run
// along rows.
__global__ __launch_bounds__(256) void panel_copy_upper_kernel(const double *A, int n, int k0,
                                                               int kb, double *Wp) {
  __shared__ double tr[64][kPB + 1];
  const int b = blockIdx.y, c0 = 64 * blockIdx.x, tid = threadIdx.x;
  const double *M = A + (size_t)b * n * n;
  double *W = Wp + (size_t)b * kPB * n;
  if (c0 >= k0 + kb - 1) {
    // every column on or right of the panel's diagonal: rows read directly
    for (int e = tid; e < kPB * 64; e += 256) {
      const int tt = e >> 6, c = c0 + (e & 63);
      if (c < n) W[(size_t)tt * n + c] = tt < kb ? M[(size_t)(k0 + tt) * n + c] : 0.0;
    }
    return;
  }
  for (int e = tid; e < 64 * kPB; e += 256) {
    const int cl = e >> 7, tt = e & (kPB - 1);
    const int c = c0 + cl;
    tr[cl][tt] = (c < n && tt < kb) ? M[(size_t)c * n + k0 + tt] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kPB * 64; e += 256) {
    const int tt = e >> 6, cl = e & 63;
    const int c = c0 + cl;
    if (c >= n) continue;
    double v = 0.0;
    if (tt < kb) v = c >= k0 + tt ? M[(size_t)(k0 + tt) * n + c] : tr[cl][tt];
    W[(size_t)tt * n + c] = v;
  }
}

// Lower triangle <- upper triangle after the two-level sweep: workgroup
// (pair, b) copies the 64 x 64 tile (ti, tj), ti <= tj, to (tj, ti) through
// LDS (both along rows); on diagonal tiles only the entries below the diagonal.
__global__ __launch_bounds__(256) void mirror_upper_kernel(double *A, int n, int ntile) {
  __shared__ double tl[64][65];
  const int b = blockIdx.y, tid = threadIdx.x;
  int ti = 0, rem = blockIdx.x;
  while (rem >= ntile - ti) {
    rem -= ntile - ti;
    ++ti;
  }
  const int tj = ti + rem;
  double *M = A + (size_t)b * n * n;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int il = e >> 6, jl = e & 63;
    const int i = 64 * ti + il, j = 64 * tj + jl;
    tl[il][jl] = (i < n && j < n) ? M[(size_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int jl = e >> 6, il = e & 63;
    const int i = 64 * ti + il, j = 64 * tj + jl;
    if (i < j && j < n) M[(size_t)j * n + i] = tl[il][jl];
  }
}

// Pivot rows of one inner block (kTB pivots, global index k0 of the first):
// one wave per workgroup (J, b).  P points at the block's rows (row r at P +
// b pstride + r n); W and R receive them at + b wstride + r n.  Lanes 0..31 hold the columns of the 32 x 32 pivot tile
// (a private copy, needed for the pivot columns), lanes 32..63 the panel
// columns [32 J, 32 J + 32), each a column of 32 rows in registers; the wave
// sweeps them pivot by pivot (product form), the pivot column being
// broadcast from its lane's registers (readlane).  Rows past n of a partial last block
// are identity rows.  It writes the swept rows W and the rows before the
// sweep R of its panel columns.
constexpr int kTJ = 32;

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(64) void sweep_rows_kernel(const double *P, size_t pstride, int n,
                                                        int k0, double *W, double *Rg,
                                                        size_t wstride, int *flag) {
  const int J = blockIdx.x, b = blockIdx.y, l = threadIdx.x;
  const double *M = P + (size_t)b * pstride;
  double *Wb = W + (size_t)b * wstride;
  double *Rb = Rg + (size_t)b * wstride;
  const bool panel = l >= kTB;
  const int col = panel ? J * kTJ + (l - kTB) : k0 + l;
  double x[kTB];
  // unconditional loads from clamped addresses, then a select: a load under a
  // condition is issued and waited for one row at a time
  const int cc = min(col, n - 1);
#pragma unroll
  for (int r = 0; r < kTB; ++r) x[r] = M[(size_t)min(r, n - 1 - k0) * n + cc];
#pragma unroll
  for (int r = 0; r < kTB; ++r) {
    const int gr = k0 + r;
    const double v = (gr < n && col < n) ? x[r] : (gr == col ? 1.0 : 0.0);
    x[r] = v;
    if (panel && col < n) Rb[(size_t)r * n + col] = v;
  }
#pragma unroll
  for (int kk = 0; kk < kTB; ++kk) {
    const int kc = k0 + kk;   // pivot column; lane kk holds it
    // broadcast of lane kk's column straight from its registers (kk is a
    // constant of the unrolled loop), no LDS round trip and no barrier
    double ck[kTB];
#pragma unroll
    for (int r = 0; r < kTB; ++r) ck[r] = readlane_f64(x[r], kk);
    const double piv = ck[kk];
    if (l == 0 && J == 0 && kc < n && !(piv > 0.0)) atomicOr(flag, 1);
    const double ip = 1.0 / piv;
    if (col == kc) {
#pragma unroll
      for (int r = 0; r < kTB; ++r) x[r] = r == kk ? -ip : ck[r] * ip;
    } else {
      const double xk = x[kk] * ip;
#pragma unroll
      for (int r = 0; r < kTB; ++r) x[r] = r == kk ? xk : x[r] - ck[r] * xk;
    }
  }
  if (panel && col < n) {
#pragma unroll
    for (int r = 0; r < kTB; ++r) Wb[(size_t)r * n + col] = x[r];
  }
}

// The inner step [s0, s0 + kTB) applied to the other rows of the panel
// (global rows k0p + t, t < kb): entries in the inner block's columns <- the
// swept rows' transposes, the rest -= R_S^T W_S; the inner block's own rows
// <- W_S.  Workgroup (column group, row group, matrix): 64 columns x 16
// panel rows, the step's W_S columns and the R_S entries of the 16 rows
// staged in LDS, wave w takes rows 16 g + w, + 4, + 8, + 12.  Within the panel's own columns (the K x K block, the pivot tiles
// of the next steps) only the upper triangle is computed and each value is
// also stored at its mirror position, so that block stays exactly symmetric
// (the row sweeps of the next steps read whole panel rows); the mirror
// targets are entries no thread computes.  Ws, Rs: the step's rows in the stacks
// (matrix stride kPB n).
__global__ __launch_bounds__(256) void sweep_panel_kernel(double *Wp, int n, int k0p, int kb,
                                                          int s0, const double *Ws,
                                                          const double *Rs) {
  __shared__ double wt[kTB][64];
  __shared__ double rt[kTB][16];
  const int b = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 64 + lane;
  double *Wb = Wp + (size_t)b * kPB * n;
  const double *Wsb = Ws + (size_t)b * kPB * n;
  const double *Rsb = Rs + (size_t)b * kPB * n;
  const int jc = min(j, n - 1);
  for (int k = wave; k < kTB; k += 4) wt[k][lane] = Wsb[(size_t)k * n + jc];
  for (int e = threadIdx.x; e < kTB * 16; e += 256) {
    const int k = e >> 4, r = e & 15;
    rt[k][r] = Rsb[(size_t)k * n + min(k0p + 16 * (int)blockIdx.y + r, n - 1)];
  }
  __syncthreads();
  if (j >= n) return;
  const bool jin = j >= s0 && j < s0 + kTB;
  const int jl = j - k0p, sl = s0 - k0p;
  const bool jK = jl >= 0 && jl < kb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = 16 * blockIdx.y + wave + 4 * q;
    if (t >= kb || (jK && t > jl)) continue;   // K block: rows on and above the diagonal
    const int tg = k0p + t;
    double v;
    if (t >= sl && t < sl + kTB) {
      v = wt[t - sl][lane];
    } else if (jin) {
      v = Wsb[(size_t)(j - s0) * n + tg];
    } else {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < kTB; ++k) acc += rt[k][t - 16 * blockIdx.y] * wt[k][lane];
      v = Wb[(size_t)t * n + j] - acc;
    }
    Wb[(size_t)t * n + j] = v;
    if (jK && t < jl) Wb[(size_t)jl * n + tg] = v;
  }
}

// M_IJ -= sum_s R_s,I^T W_s,J = Rst_KI^T Wst_KJ (the stacked rows of the
// four steps) for I, J outside the outer block K = [k0, k0 + kb); rows of K
// <- Wp (the swept panel); columns of K <- Wp^T.  Only the upper triangle is
// computed and every value is stored at (i, j) and (j, i) (the mirror through
// LDS, row by row): the swept matrix is
// symmetric in exact arithmetic, and keeping it exactly symmetric matters for
// cut-cell blocks whose scaled condition reaches 1e12 or more, where R^T (P R)
// and its mirror image differ by the pivot-block solve error.  64 x 64 output
// tile (ti <= tj) per workgroup, wave w owns the 32 x 32 quarter (w / 2, w %
// 2) as 2 x 2 v_mfma_f64_16x16x4f64 tiles (lane l supplies A[l%16][l/16] and
// B[l/16][l%16], holds D[4j + l/16][l%16]); the kPB-deep sum runs in chunks of
// 16 k, the loads of the next chunk in flight while the current one is on the
// matrix cores.
typedef double doublex4s __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void sweep_update_mfma_kernel(double *A, int n, int k0, int kb,
                                                                const double *Wp,
                                                                const double *Wst,
                                                                const double *Rst, int ntile,
                                                                int batch) {
  // Workgroups are dealt to the 8 XCDs round-robin by linear id; in batches
  // of 8 and more all tiles of a matrix get ids of one residue mod 8, so that
  // the matrix's row stacks are fetched from HBM into one XCD's L2 (and
  // reused there by its other tiles) instead of into all eight.  Smaller
  // batches (single coarse blocks) take the plain order.
  const int npair = ntile * (ntile + 1) / 2;
  const int L = blockIdx.x;
  int b, rem;
  if (batch >= 8) {
    const int slot = L >> 3;
    b = 8 * (slot / npair) + (L & 7);
    rem = slot % npair;
  } else {
    b = L / npair;
    rem = L % npair;
  }
  if (b >= batch) return;
  int ti = 0;
  while (rem >= ntile - ti) {
    rem -= ntile - ti;
    ++ti;
  }
  const int tj = ti + rem;
  double *M = A + (size_t)b * n * n;
  const double *Wb = Wp + (size_t)b * kPB * n;
  const double *Sw = Wst + (size_t)b * kPB * n;
  const double *Sr = Rst + (size_t)b * kPB * n;
  const int k1 = k0 + kb;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 15, lq = lane >> 4;
  const int i0 = ti * 64 + (wave >> 1) * 32, j0 = tj * 64 + (wave & 1) * 32;
  __shared__ double tile[64][65];   // the tile's results, for the mirrored store
  // a wave with nothing on or above the diagonal (or outside the matrix)
  // skips the products but joins the barrier before the mirrored store
  const bool active = !(i0 >= n || j0 >= n || i0 > j0 + 31);
  if (active) {
  doublex4s acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = doublex4s{0.0, 0.0, 0.0, 0.0};
  const int ic[2] = {min(i0 + ln, n - 1), min(i0 + 16 + ln, n - 1)};
  const int jc[2] = {min(j0 + ln, n - 1), min(j0 + 16 + ln, n - 1)};
  const double mi[2] = {i0 + ln < n ? 1.0 : 0.0, i0 + 16 + ln < n ? 1.0 : 0.0};
  const double mj[2] = {j0 + ln < n ? 1.0 : 0.0, j0 + 16 + ln < n ? 1.0 : 0.0};
  // operand loads from clamped addresses (stack rows kb.. up to the next
  // multiple of 32 are the zero rows of a partial last step), masked by a
  // multiply once they have arrived
  double av[2][4][2], bv[2][4][2];
  auto load = [&](int c, int buf) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const size_t kk = (size_t)(c + 4 * ks + lq) * n;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[buf][ks][u] = Sr[kk + ic[u]];   // A[i][k] = R[k][i]
        bv[buf][ks][u] = Sw[kk + jc[u]];   // B[k][j] = W[k][j]
      }
    }
  };
  const int nk = (kb + 15) & ~15;
  load(0, 0);
#pragma unroll
  for (int c = 0; c < kPB; c += 16) {
    if (c >= nk) break;   // wave-uniform
    const int cur = (c >> 4) & 1;
    if (c + 16 < nk) load(c + 16, cur ^ 1);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a[2], bb[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = av[cur][ks][u] * mi[u];
        bb[u] = bv[cur][ks][u] * mj[u];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[v], acc[u][v], 0, 0, 0);
    }
  }
  // all loads of the write phase are issued before any store (the output
  // entries are distinct and Wp is not written here)
  double old[2][2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + 16 * u + 4 * jj + lq, j = j0 + 16 * v + ln;
        const bool ok = i < n && j < n && i <= j;
        const bool ik = i >= k0 && i < k1, jk = j >= k0 && j < k1;
        const double *src = !ok ? M : ik ? Wb + (size_t)(i - k0) * n + j
                                      : jk ? Wb + (size_t)(j - k0) * n + i
                                           : M + (size_t)i * n + j;
        old[u][v][jj] = *src;
      }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + 16 * u + 4 * jj + lq, j = j0 + 16 * v + ln;
        if (i >= n || j >= n || i > j) continue;
        const bool inK = (i >= k0 && i < k1) || (j >= k0 && j < k1);
        const double val = inK ? old[u][v][jj] : old[u][v][jj] - acc[u][v][jj];
        M[(size_t)i * n + j] = val;
        tile[i - ti * 64][j - tj * 64] = val;
      }
  }
  __syncthreads();
  // the mirror (j, i) of every entry i < j, written along rows of the
  // transposed tile (a store straight from the MFMA layout would touch 16
  // rows 32 bytes each)
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int jl = e >> 6, il = e & 63;
    const int i = ti * 64 + il, j = tj * 64 + jl;
    if (i < j && j < n) M[(size_t)j * n + i] = tile[il][jl];
  }
}

// Two-level path, the same update from 128 x 128 tiles (ti <= tj): the
// stacks' 16-deep chunks of the tile's 128 rows and 128 columns are staged in
// LDS (double-buffered: the next chunk's loads are in flight while the
// matrix cores work on the current one) and each wave takes a 64 x 64
// quadrant as 4 x 4 v_mfma_f64_16x16x4f64 tiles, so that the L2 delivers
// each operand once per workgroup, with four times the products per byte of
// the 64 x 64 tiles, whose waves each load their own operands.  Entries and
// the K rows and columns are as above, the XCD mapping too; only the upper
// triangle is stored (the two-level sweep reads its panels from it).
constexpr int kUT = 128, kUK = 16, kUS = kUT + 4;
typedef double doublex4w __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 2) void sweep_update_wide_kernel(double *A, int n, int k0,
                                                                   int kb, const double *Wp,
                                                                   const double *Wst,
                                                                   const double *Rst, int ntile,
                                                                   int batch) {
  __shared__ double lds[2 * 2 * kUK * kUS];   // [buffer][R | W][k][column]
  const int npair = ntile * (ntile + 1) / 2;
  const int L = blockIdx.x;
  int b, rem;
  if (batch >= 8) {
    const int slot = L >> 3;
    b = 8 * (slot / npair) + (L & 7);
    rem = slot % npair;
  } else {
    b = L / npair;
    rem = L % npair;
  }
  if (b >= batch) return;   // the whole workgroup
  int ti = 0;
  while (rem >= ntile - ti) {
    rem -= ntile - ti;
    ++ti;
  }
  const int tj = ti + rem;
  double *M = A + (size_t)b * n * n;
  const double *Wb = Wp + (size_t)b * kPB * n;
  const double *Sw = Wst + (size_t)b * kPB * n;
  const double *Sr = Rst + (size_t)b * kPB * n;
  const int k1 = k0 + kb;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ln = lane & 15, lq = lane >> 4;
  const int I0 = ti * kUT, J0 = tj * kUT;
  const int qi0 = I0 + (wave >> 1) * 64, qj0 = J0 + (wave & 1) * 64;
  // a quadrant with nothing on or above the diagonal (or outside the matrix)
  // skips the products but joins the loads and the barriers
  const bool active = qi0 < n && qj0 < n && qi0 <= qj0 + 63;
  // each thread stages one column (tid % 128) of rows tid / 128 + 2 r
  const int lc = tid & 127, lk = tid >> 7;
  const int ci = min(I0 + lc, n - 1), cj = min(J0 + lc, n - 1);
  const double mi = I0 + lc < n ? 1.0 : 0.0, mj = J0 + lc < n ? 1.0 : 0.0;
  double pr[8], pw[8];
  // stack rows kb.. up to the next multiple of 32 are the zero rows of a
  // partial last step
  auto fetch = [&](int c) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const size_t row = (size_t)(c + lk + 2 * r) * n;
      pr[r] = Sr[row + ci];
      pw[r] = Sw[row + cj];
    }
  };
  auto stage = [&](int buf) {
    double *a = lds + buf * 2 * kUK * kUS, *w = a + kUK * kUS;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      a[(lk + 2 * r) * kUS + lc] = pr[r] * mi;
      w[(lk + 2 * r) * kUS + lc] = pw[r] * mj;
    }
  };
  doublex4w acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = doublex4w{0.0, 0.0, 0.0, 0.0};
  const int nk = (kb + 15) & ~15;
  const int ai = (wave >> 1) * 64 + ln, aj = (wave & 1) * 64 + ln;
  fetch(0);
  for (int c = 0; c < nk; c += kUK) {
    const int buf = (c / kUK) & 1;
    stage(buf);
    __syncthreads();
    if (c + kUK < nk) fetch(c + kUK);
    if (active) {
      const double *a = lds + buf * 2 * kUK * kUS, *w = a + kUK * kUS;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kr = (4 * ks + lq) * kUS;
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = a[kr + ai + 16 * u];
          bv[u] = w[kr + aj + 16 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
      }
    }
  }
  // store of the upper entries (the two-level sweep keeps the upper
  // triangle only; its lower one is filled once at the end)
  if (active) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double old[4][4];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = qi0 + 16 * u + 4 * jj + lq, j = qj0 + 16 * v + ln;
          const bool ok = i < n && j < n && i <= j;
          const bool ik = i >= k0 && i < k1, jk = j >= k0 && j < k1;
          const double *src = !ok ? M : ik ? Wb + (size_t)(i - k0) * n + j
                                        : jk ? Wb + (size_t)(j - k0) * n + i
                                             : M + (size_t)i * n + j;
          old[v][jj] = *src;
        }
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = qi0 + 16 * u + 4 * jj + lq, j = qj0 + 16 * v + ln;
          if (i >= n || j >= n || i > j) continue;
          const bool inK = (i >= k0 && i < k1) || (j >= k0 && j < k1);
          const double val = inK ? old[v][jj] : old[v][jj] - acc[u][v][jj];
          M[(size_t)i * n + j] = val;
        }
    }
  }
}

size_t spd_inverse_scratch_doubles(int n, int batch) {
  // the panel (Wp) and the stacked rows after (Wst) and before (Rst) each
  // step, kPB x n each; scale; two norms per matrix
  return (size_t)batch * n * (3 * kPB + 1) + 2 * (size_t)batch;
}

__global__ void zero_doubles_kernel(double *x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

int spd_inverse_batched(double *A, int n, int batch, double *scratch, int *flag, double *kappa,
                        hipStream_t s) {
  if (batch <= 0 || n <= 0) return 0;
  const size_t bn = (size_t)batch * n;
  double *Wp = scratch, *Wst = Wp + bn * kPB, *Rst = Wst + bn * kPB;
  double *scale = Rst + bn * kPB;
  double *nrm = scale + bn;
  // norm accumulators start at zero (a kernel, not a memset node, so that the
  // sequence may sit inside a captured graph)
  if (kappa) zero_doubles_kernel<<<(2 * batch + 255) / 256, 256, 0, s>>>(nrm, 2 * (size_t)batch);
  jacobi_scale_kernel<<<dim3((n + 255) / 256, batch), 256, 0, s>>>(A, n, scale, flag);
  const dim3 sgrid((n + 3) / 4, batch);
  apply_scale_kernel<<<sgrid, 256, 0, s>>>(A, n, scale, 1.0, kappa ? nrm : nullptr);
  const int nt = (n + 63) / 64;
  // one-dimensional: tile pairs x batch, the batch rounded up to a multiple
  // of 8 from 8 on (the update kernel maps ids to (matrix, tile) XCD by XCD)
  const unsigned bgrid = (unsigned)(batch >= 8 ? (batch + 7) / 8 * 8 : batch);
  const dim3 ugrid((unsigned)(nt * (nt + 1) / 2) * bgrid);
  const int ntw = (n + kUT - 1) / kUT;
  const dim3 wgrid((unsigned)(ntw * (ntw + 1) / 2) * bgrid);
  if (batch < kTwoLevelBatch || n <= kTwoLevelN) {
    // one trailing update per 32 pivots, straight from the matrix rows
    for (int k0 = 0; k0 < n; k0 += kTB) {
      const int kb = std::min(kTB, n - k0);
      sweep_rows_kernel<<<dim3((n + kTJ - 1) / kTJ, batch), 64, 0, s>>>(
          A + (size_t)k0 * n, (size_t)n * n, n, k0, Wst, Rst, (size_t)kPB * n, flag);
      sweep_update_mfma_kernel<<<ugrid, 256, 0, s>>>(A, n, k0, kb, Wst, Wst, Rst, nt, batch);
    }
  } else {
    // only the upper triangle is kept during the sweep (the panel is read
    // from it, the update writes it), the lower one is filled at the end
    for (int k0 = 0; k0 < n; k0 += kPB) {
      const int kb = std::min(kPB, n - k0);
      panel_copy_upper_kernel<<<dim3((n + 63) / 64, batch), 256, 0, s>>>(A, n, k0, kb, Wp);
      for (int t0 = 0; t0 < kb; t0 += kTB) {
        const size_t off = (size_t)t0 * n;
        sweep_rows_kernel<<<dim3((n + kTJ - 1) / kTJ, batch), 64, 0, s>>>(
            Wp + off, (size_t)kPB * n, n, k0 + t0, Wst + off, Rst + off, (size_t)kPB * n, flag);
        sweep_panel_kernel<<<dim3((n + 63) / 64, (kb + 15) / 16, batch), 256, 0, s>>>(
            Wp, n, k0, kb, k0 + t0, Wst + off, Rst + off);
      }
      sweep_update_wide_kernel<<<wgrid, 256, 0, s>>>(A, n, k0, kb, Wp, Wst, Rst, ntw, batch);
    }
    mirror_upper_kernel<<<dim3(nt * (nt + 1) / 2, batch), 256, 0, s>>>(A, n, nt);
  }
  apply_scale_kernel<<<sgrid, 256, 0, s>>>(A, n, scale, -1.0, kappa ? nrm + batch : nullptr);
  if (kappa) kappa_product_kernel<<<(batch + 255) / 256, 256, 0, s>>>(nrm, batch, kappa);
  return 0;
}

__global__ void to_f32_kernel(const double *src, float *dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  to_f32_kernel<<<blocks, 256, 0, s>>>(src, dst, n);
}

// ----------------------------------------------------------- coarse level
// Coarse DOF (vertex at grid point g, component c) exists iff a kept element
// touches g and g is not on a Dirichlet face.
__device__ inline bool coarse_exists(const Geo &g, const int *kmat, const int *gc) {
  for (int ax = 0; ax < g.d; ++ax) {
    if (gc[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) return false;
    if (gc[ax] == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) return false;
  }
  for (int s = 0; s < (1 << g.d); ++s) {
    int ec[3] = {gc[0] - (s & 1), gc[1] - ((s >> 1) & 1), gc[2] - ((s >> 2) & 1)};
    bool in = true;
    for (int ax = 0; ax < 3; ++ax) in = in && ec[ax] >= 0 && ec[ax] < g.n[ax];
    if (in && kmat[ec[0] + g.n[0] * (ec[1] + g.n[1] * ec[2])] >= 0) return true;
  }
  return false;
}

// Row r of the blocked coarse system -> grid point; false for padding rows.
__device__ inline bool coarse_row_point(const Geo &g, const Coarse &c, int blk, int i, int *gc,
                                        int *comp) {
  const int lay = c.w * c.PP;
  *comp = i / lay;
  int rem = i % lay;
  int lam = rem / c.PP, pt = rem % c.PP;
  const int sl = g.d - 1;
  int layer = c.layer0 + blk * c.w + lam;
  if (layer >= g.gn[sl]) return false;
  gc[0] = gc[1] = gc[2] = 0;
  if (g.d == 3) {
    gc[0] = pt % g.gn[0];
    gc[1] = pt / g.gn[0];
  } else {
    gc[0] = pt;
  }
  gc[sl] = layer;
  return true;
}

__device__ inline double coarse_entry(const Geo &g, const int *smap, int mp, const int *kmat,
                                      const double *Kref, const double *Kcut, const int *ga,
                                      int ca, const int *gb, int cb) {
  // elements containing both vertices
  double sum = 0.0;
  for (int s = 0; s < (1 << g.d); ++s) {
    int ec[3] = {ga[0] - (s & 1), ga[1] - ((s >> 1) & 1), ga[2] - ((s >> 2) & 1)};
    bool ok = true;
    int ta[3] = {0, 0, 0}, tb[3] = {0, 0, 0};
    for (int ax = 0; ax < 3; ++ax) {
      ok = ok && ec[ax] >= 0 && ec[ax] < g.n[ax];
      int db = gb[ax] - ec[ax];
      ok = ok && db >= 0 && db <= 1;
      ta[ax] = ga[ax] - ec[ax];
      tb[ax] = db;
    }
    if (!ok) continue;
    int kid = kmat[ec[0] + g.n[0] * (ec[1] + g.n[1] * ec[2])];
    if (kid < 0) continue;
    const int np = g.p + 1;
    int ia = smap[(ta[0] + np * (ta[1] + np * ta[2])) * g.nf + ca];
    int ib = smap[(tb[0] + np * (tb[1] + np * tb[2])) * g.nf + cb];
    const double *K = kid == 0 ? Kref : Kcut + (size_t)(kid - 1) * mp * mp;
    sum += K[(size_t)ia * mp + ib];
  }
  return sum;
}

// Full 27-point (9-point in 2D) stencil per coarse row, for slow offsets
// -1, 0, +1: St[row][(so+1)*no*nf + o*nf + c'].
__global__ void coarse_stencil_kernel(Geo g, Coarse c, const int *smap, int mp,
                                      const int *kmat, const double *Kref, const double *Kcut,
                                      double *St) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int nrows = c.nblk * c.nb;
  if (row >= nrows) return;
  const int blk = row / c.nb, i = row % c.nb;
  const int per = 3 * c.no * g.nf;
  double *out = St + (size_t)row * per;
  int ga[3], ca;
  bool inrange = coarse_row_point(g, c, blk, i, ga, &ca);
  bool ex = inrange && coarse_exists(g, kmat, ga);
  const int sl = g.d - 1;
  for (int so = -1; so <= 1; ++so)
    for (int o = 0; o < c.no; ++o)
      for (int cb = 0; cb < g.nf; ++cb) {
        double v = 0.0;
        if (ex) {
          int gb[3] = {ga[0], ga[1], ga[2]};
          gb[0] += o % 3 - 1;
          if (g.d == 3) gb[1] += o / 3 - 1;
          gb[sl] += so;
          bool in = true;
          for (int ax = 0; ax < g.d; ++ax) in = in && gb[ax] >= 0 && gb[ax] < g.gn[ax];
          if (in && coarse_exists(g, kmat, gb))
            v = coarse_entry(g, smap, mp, kmat, Kref, Kcut, ga, ca, gb, cb);
        }
        out[((so + 1) * c.no + o) * g.nf + cb] = v;
      }
}

void launch_coarse_stencils(const Geo &g, const Tables &t, const Coarse &c, const int *kmat,
                            const double *Kref, const double *Kcut, hipStream_t s) {
  int nrows = c.nblk * c.nb;
  coarse_stencil_kernel<<<(nrows + 127) / 128, 128, 0, s>>>(g, c, t.smap, t.m, kmat, Kref, Kcut,
                                                            c.Dst);
}

// 3^d-point stencil of the p = 1 matrix for the geometric h-levels: row
// (c, node) holds, for offset o = (dx+1) + 3 (dy+1) + 9 (dz+1) and component
// c', the entry of the vertex DOF (c', node + off(o)); rows and columns of
// absent DOFs (pres = 0) are zero.
__global__ void hstencil0_kernel(Geo g, const int *smap, int mp, const int *kmat,
                                 const double *Kref, const double *Kcut, const int *pres,
                                 double *S) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int64_t)g.nf * g.G) return;
  const int no = g.d == 3 ? 27 : 9;
  const int ca = (int)(row / g.G);
  const int pt = (int)(row % g.G);
  int ga[3] = {pt % g.gn[0], (pt / g.gn[0]) % g.gn[1], pt / (g.gn[0] * g.gn[1])};
  double *out = S + row * (no * g.nf);
  const bool ok = pres[row] != 0;
  for (int o = 0; o < no; ++o) {
    int gb[3] = {ga[0] + o % 3 - 1, ga[1] + (o / 3) % 3 - 1, ga[2] + (g.d == 3 ? o / 9 - 1 : 0)};
    bool in = true;
    for (int ax = 0; ax < 3; ++ax) in = in && gb[ax] >= 0 && gb[ax] < g.gn[ax];
    const int pb = in ? gb[0] + g.gn[0] * (gb[1] + g.gn[1] * gb[2]) : 0;
    for (int cb = 0; cb < g.nf; ++cb) {
      double v = 0.0;
      if (ok && in && pres[(int64_t)cb * g.G + pb])
        v = coarse_entry(g, smap, mp, kmat, Kref, Kcut, ga, ca, gb, cb);
      out[o * g.nf + cb] = v;
    }
  }
}

void launch_hstencil0(const Geo &g, const Tables &t, const int *kmat, const double *Kref,
                      const double *Kcut, const int *pres, double *S, hipStream_t s) {
  const int64_t rows = (int64_t)g.nf * g.G;
  hstencil0_kernel<<<(unsigned)((rows + 127) / 128), 128, 0, s>>>(g, t.smap, t.m, kmat, Kref,
                                                                   Kcut, pres, S);
}

// Neighbour of block-local row i at (so, o, c') -> block-local index in the
// block of that layer, and which block (-1, 0, +1 relative), or -1 if none.
__device__ inline int coarse_nbr(const Geo &g, const Coarse &c, int i, int so, int o, int cb,
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

// Dense diagonal block D_k from the stencil (identity rows for non-DOFs).
__global__ void coarse_fill_kernel(Geo g, Coarse c, int k, double *S) {
  const int i = blockIdx.y;
  const int nb = c.nb;
  double *row = S + (size_t)i * nb;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += gridDim.x * blockDim.x)
    row[j] = 0.0;
  __syncthreads();
  if (blockIdx.x != 0) return;
  int ga[3], ca;
  bool inrange = coarse_row_point(g, c, k, i, ga, &ca);
  const double *st = c.Dst + (size_t)(k * nb + i) * 3 * c.no * g.nf;
  bool any = false;
  if (inrange) {
    for (int t = threadIdx.x; t < 3 * c.no * g.nf; t += blockDim.x) {
      int so = t / (c.no * g.nf) - 1;
      int o = (t / g.nf) % c.no, cb = t % g.nf;
      double v = st[t];
      if (v == 0.0) continue;
      int db;
      int j = coarse_nbr(g, c, i, so, o, cb, &db);
      if (j < 0 || db != 0) continue;
      row[j] = v;
    }
    any = st[(c.no + c.no / 2) * g.nf + ca] != 0.0;   // diagonal entry present
  }
  __syncthreads();
  if (threadIdx.x == 0 && !any) row[i] = 1.0;
}

void launch_coarse_first(const Geo &g, const Coarse &c, int k, double *S, hipStream_t s) {
  dim3 grid(1, c.nb);
  coarse_fill_kernel<<<grid, 256, 0, s>>>(g, c, k, S);
}

// T = Sinv_{k-1} B_k^T  (only columns j of the first layer of block k couple)
__global__ void coarse_T_kernel(Geo g, Coarse c, int k, const double *Sprev, double *T) {
  const int nb = c.nb;
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += gridDim.x * blockDim.x) {
    const double *st = c.Dst + (size_t)(k * nb + j) * 3 * c.no * g.nf;   // so = -1 part
    double s = 0.0;
    for (int t = 0; t < c.no * g.nf; ++t) {
      double v = st[t];
      if (v == 0.0) continue;
      int o = t / g.nf, cb = t % g.nf, db;
      int l = coarse_nbr(g, c, j, -1, o, cb, &db);
      if (l < 0 || db != -1) continue;
      s += Sprev[(size_t)i * nb + l] * v;
    }
    T[(size_t)i * nb + j] = s;
  }
}

// S_k = D_k - B_k T
__global__ void coarse_S_kernel(Geo g, Coarse c, int k, const double *T, double *S) {
  const int nb = c.nb;
  const int i = blockIdx.y;
  const double *st = c.Dst + (size_t)(k * nb + i) * 3 * c.no * g.nf;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < c.no * g.nf; ++t) {
      double v = st[t];
      if (v == 0.0) continue;
      int o = t / g.nf, cb = t % g.nf, db;
      int l = coarse_nbr(g, c, i, -1, o, cb, &db);
      if (l < 0 || db != -1) continue;
      s += v * T[(size_t)l * nb + j];
    }
    S[(size_t)i * nb + j] -= s;
  }
}

// G_k = S_k^{-1} B_k: column j (block k-1) couples through the upper stencil
// of row j, B_k[l][j] = A[(k-1,j),(k,l)].
__global__ void coarse_G_kernel(Geo g, Coarse c, int k, const double *Sk, double *Gk) {
  const int nb = c.nb;
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nb; j += gridDim.x * blockDim.x) {
    const double *st = c.Dst + (size_t)((k - 1) * nb + j) * 3 * c.no * g.nf + 2 * c.no * g.nf;
    double s = 0.0;
    for (int t = 0; t < c.no * g.nf; ++t) {
      double v = st[t];
      if (v == 0.0) continue;
      int o = t / g.nf, cb = t % g.nf, db;
      int l = coarse_nbr(g, c, j, 1, o, cb, &db);
      if (l < 0 || db != 1) continue;
      s += Sk[(size_t)i * nb + l] * v;
    }
    Gk[(size_t)i * nb + j] = s;
  }
}

void launch_coarse_G(const Geo &g, const Coarse &c, int k, hipStream_t s) {
  const int nb = c.nb;
  dim3 grid((nb + 255) / 256, nb);
  coarse_G_kernel<<<grid, 256, 0, s>>>(g, c, k, c.Sinv + (size_t)k * nb * nb,
                                       c.Gm + (size_t)k * nb * nb);
}

void launch_coarse_schur(const Geo &g, const Coarse &c, int k, double *S, double *T,
                         hipStream_t s) {
  const int nb = c.nb;
  const double *Sprev = c.Sinv + (size_t)(k - 1) * nb * nb;
  dim3 grid((nb + 255) / 256, nb);
  coarse_T_kernel<<<grid, 256, 0, s>>>(g, c, k, Sprev, T);
  coarse_S_kernel<<<grid, 256, 0, s>>>(g, c, k, T, S);
}

}  // namespace fcm
