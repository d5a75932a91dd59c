// Host side of libfcm: C-ABI entry points, hierarchy setup, V-cycle (Alg. 1)
// and CG driver (Section 4).  All numerical work runs in the kernels of
// kernels_setup.hip and kernels_solve.hip; the host only builds index tables
// (local mode order, plane order, Schwarz block classes) and sequences
// launches on the caller's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "fcm_internal.hpp"

namespace fcm {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

// ------------------------------------------------------------ host basis
// Gauss-Legendre nodes by Newton iteration on L_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (n == 1) {
    x[0] = 0.0;
    w[0] = 2.0;
  }
}

static void modes1d_host(int p, double xi, double *v, double *dv) {
  double L[kMaxP + 1];
  L[0] = 1.0;
  if (p >= 1) L[1] = xi;
  for (int n = 1; n < p; ++n) L[n + 1] = ((2 * n + 1) * xi * L[n] - n * L[n - 1]) / (n + 1);
  v[0] = 0.5 * (1.0 - xi);
  v[1] = 0.5 * (1.0 + xi);
  dv[0] = -0.5;
  dv[1] = 0.5;
  for (int j = 2; j <= p; ++j) {
    double s = 1.0 / std::sqrt(2.0 * (2 * j - 1));
    v[j] = (L[j] - L[j - 2]) * s;
    dv[j] = (2 * j - 1) * L[j - 1] * s;
  }
}

static int deg1(int a) { return a < 2 ? 1 : a; }      // local 1D mode -> degree
static int tdeg(int t) { return t == 0 ? 1 : t + 1; }  // slot type -> degree

// Level order q of a product of 1D functions of degrees dg[0..d-1] (1 for a
// linear factor): the largest degree in the tensor-product space; in the
// trunk space the sum of the degrees above 1, at least 1.
static int prod_degree(bool trunk, int d, const int *dg) {
  int mx = 1, sum = 0;
  for (int ax = 0; ax < d; ++ax) {
    mx = std::max(mx, dg[ax]);
    if (dg[ax] > 1) sum += dg[ax];
  }
  return trunk ? std::max(1, sum) : mx;
}
static int mode_degree(const Geo &g, int a0, int a1, int a2) {
  const int dg[3] = {deg1(a0), deg1(a1), deg1(a2)};
  return prod_degree(g.trunk, g.d, dg);
}
static int plane_degree(const Geo &g, int t0, int t1, int t2) {
  const int dg[3] = {tdeg(t0), tdeg(t1), tdeg(t2)};
  return prod_degree(g.trunk, g.d, dg);
}
// Patch-local functions of level q (per-axis slots 0..2p: hats at 0, p, 2p,
// bubbles of degree t+1 at slots t and p+t), times n_f.
static int patch_size(bool trunk, int d, int nf, int p, int q) {
  int cnt = 0;
  const int S = 2 * p + 1;
  for (int s2 = 0; s2 < (d == 3 ? S : 1); ++s2)
    for (int s1 = 0; s1 < S; ++s1)
      for (int s0 = 0; s0 < S; ++s0) {
        const int sl[3] = {s0, s1, s2};
        int dg[3];
        for (int ax = 0; ax < 3; ++ax) {
          const int t = sl[ax] % p;          // 0 for the hats, else the bubble type
          dg[ax] = tdeg(t);
        }
        if (prod_degree(trunk, d, dg) <= q) ++cnt;
      }
  return cnt * nf;
}

#define TRY(x)                         \
  do {                                 \
    fcm_status s_ = (x);               \
    if (s_ != FCM_OK) return s_;       \
  } while (0)

// ------------------------------------------------------- device memory
// Device memory comes from the device's default stream-ordered pool.  An
// allocation or release is an operation on a stream and, unlike hipMalloc /
// hipFree, never synchronises the whole device, so setups and teardowns of
// independent solves (the request server) do not serialise each other.  The
// pool keeps released memory for reuse (release threshold raised once per
// device) until fcm_trim_pool().
static std::mutex g_pool_mu;
static std::vector<char> g_pool_ready;

static fcm_status pool_prepare() {
  int dev = 0;
  FCM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pool_ready.size() <= dev) g_pool_ready.resize(dev + 1, 0);
  if (g_pool_ready[dev]) return FCM_OK;
  hipMemPool_t pool;
  FCM_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t thr = UINT64_MAX;
  FCM_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
  g_pool_ready[dev] = 1;
  return FCM_OK;
}

fcm_status pool_alloc(void **p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  TRY(pool_prepare());
  hipError_t e = hipMallocAsync(p, std::max<size_t>(bytes, 1), s);
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("hipMallocAsync of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? FCM_ERR_OOM : FCM_ERR_HIP;
  }
  return FCM_OK;
}

void pool_free(void *p, hipStream_t s) {
  if (p) hipFreeAsync(p, s);
}

// Pinned host blocks of 16 doubles for scalar read-back, recycled across
// handles (freeing pinned memory synchronises the device as hipFree does).
static std::vector<double *> g_pinned_free;

double *pinned_get() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pinned_free.empty()) {
    const int per = 64;
    double *slab = nullptr;
    if (hipHostMalloc((void **)&slab, per * 16 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess)
      return nullptr;
    for (int k = per - 1; k >= 0; --k) g_pinned_free.push_back(slab + 16 * k);
  }
  double *b = g_pinned_free.back();
  g_pinned_free.pop_back();
  return b;
}

void pinned_put(double *b) {
  if (!b) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pinned_free.push_back(b);
}

// ------------------------------------------------------------ validation
static fcm_status validate(const fcm_problem *p, const fcm_options *o) {
  if (!p || !o) { set_error("null problem or options"); return FCM_ERR_ARG; }
  if (p->dim != 2 && p->dim != 3) { set_error("dim must be 2 or 3"); return FCM_ERR_ARG; }
  if (p->p < 1 || p->p > kMaxP) { set_error("p must be in 1..%d", kMaxP); return FCM_ERR_ARG; }
  if (p->n_fields != 1 && p->n_fields != p->dim) {
    set_error("n_fields must be 1 or dim");
    return FCM_ERR_ARG;
  }
  if (p->refine_levels < 0 || p->refine_levels > 4) {
    set_error("refine_levels must be in 0..4");
    return FCM_ERR_ARG;
  }
  if (o->coarse != FCM_COARSE_BLOCKTRI && o->coarse != FCM_COARSE_HMG) {
    set_error("coarse must be FCM_COARSE_BLOCKTRI or FCM_COARSE_HMG");
    return FCM_ERR_ARG;
  }
  if (o->coarse_dense_max < 0 || o->coarse_dense_max > 8192) {
    set_error("coarse_dense_max must be in 0..8192");
    return FCM_ERR_ARG;
  }
  if (p->refine_levels > 0) {
    if (p->n_fields != 1) { set_error("multi-level hp: Poisson only"); return FCM_ERR_ARG; }
    if (o->coarse != FCM_COARSE_BLOCKTRI) {
      set_error("multi-level hp: the coarse level is solved exactly");
      return FCM_ERR_ARG;
    }
    if (o->smoother != FCM_SMOOTH_PATCHWISE) {
      set_error("multi-level hp: patchwise Schwarz blocks only");
      return FCM_ERR_ARG;
    }
    if (p->quad_depth > (p->dim == 3 ? 3 : 4)) {
      set_error("multi-level hp: quad_depth must be <= %d", p->dim == 3 ? 3 : 4);
      return FCM_ERR_ARG;
    }
    if (p->p > 3) { set_error("multi-level hp: p must be <= 3"); return FCM_ERR_ARG; }
  } else if (p->beta != 0.0 && p->geom != FCM_GEOM_SQUARE && p->geom != FCM_GEOM_POPCORN) {
    set_error("beta (sphere penalty) needs refine_levels > 0");
    return FCM_ERR_ARG;
  }
  if (!std::isfinite(p->beta) || p->beta < 0.0) { set_error("invalid beta"); return FCM_ERR_ARG; }
  if (p->beta > 0.0 && p->geom != FCM_GEOM_BALL_INTERIOR && p->geom != FCM_GEOM_SQUARE &&
      p->geom != FCM_GEOM_POPCORN) {
    set_error("beta (sphere penalty) needs the ball-interior geometry");
    return FCM_ERR_ARG;
  }
  if (p->geom == FCM_GEOM_SQUARE) {
    if (p->dim != 2 || p->n_fields != 1 || p->refine_levels != 0 || p->n_balls != 1) {
      set_error("the square geometry needs a 2D Poisson problem on a uniform grid with one "
                "centre (ball_c) and side (ball_r)");
      return FCM_ERR_ARG;
    }
    if (!std::isfinite(p->psi) || !std::isfinite(p->trig_src[0]) ||
        !std::isfinite(p->trig_src[1]) || !std::isfinite(p->trig_dir[0]) ||
        !std::isfinite(p->trig_dir[1])) {
      set_error("invalid square rotation or trigonometric data");
      return FCM_ERR_ARG;
    }
  } else if (p->geom == FCM_GEOM_POPCORN) {
    if (p->dim != 3 || p->n_fields != 1 || p->refine_levels != 0 || p->n_balls != 0) {
      set_error("the popcorn geometry needs a 3D Poisson problem on a uniform grid and no balls");
      return FCM_ERR_ARG;
    }
  }
  if (p->geom != FCM_GEOM_SQUARE && (p->trig_src[0] != 0.0 || p->trig_dir[0] != 0.0)) {
    set_error("trigonometric source and Dirichlet data need the square geometry");
    return FCM_ERR_ARG;
  }
  if (p->surf_n[0] < 0 || p->surf_n[1] < 0 || p->surf_n[0] > 4096 || p->surf_n[1] > 8192) {
    set_error("surface rule sizes out of range");
    return FCM_ERR_ARG;
  }
  for (int ax = 0; ax < p->dim; ++ax) {
    if (p->n[ax] < 1 || p->n[ax] > 4096) { set_error("n[%d] out of range", ax); return FCM_ERR_ARG; }
    if (!(p->hi[ax] > p->lo[ax])) { set_error("empty box on axis %d", ax); return FCM_ERR_ARG; }
  }
  if (!(p->alpha > 0.0) || p->alpha > 1.0) { set_error("alpha must be in (0,1]"); return FCM_ERR_ARG; }
  if (p->quad_depth < 0 || p->quad_depth > kMaxDepth) {
    set_error("quad_depth must be in 0..%d", kMaxDepth);
    return FCM_ERR_ARG;
  }
  if (p->geom != FCM_GEOM_BOX_MINUS_BALLS && p->geom != FCM_GEOM_BALL_INTERIOR &&
      p->geom != FCM_GEOM_SQUARE && p->geom != FCM_GEOM_POPCORN) {
    set_error("unknown geometry");
    return FCM_ERR_ARG;
  }
  if (p->n_balls < 0 || (p->n_balls > 0 && (!p->ball_c || !p->ball_r))) {
    set_error("invalid balls");
    return FCM_ERR_ARG;
  }
  if (p->geom == FCM_GEOM_BALL_INTERIOR && p->n_balls != 1) {
    set_error("ball interior needs exactly one ball");
    return FCM_ERR_ARG;
  }
  for (int j = 0; j < p->n_balls; ++j)
    if (!(p->ball_r[j] >= 0.0) || !std::isfinite(p->ball_r[j])) {
      set_error("invalid radius");
      return FCM_ERR_ARG;
    }
  if (p->n_gauss < 0 || (p->n_gauss > 0 && !p->gauss)) { set_error("invalid sources"); return FCM_ERR_ARG; }
  for (int k = 0; k < 5 * p->n_gauss; ++k)
    if (!std::isfinite(p->gauss[k])) { set_error("non-finite source parameter"); return FCM_ERR_NAN; }
  if (!std::isfinite(p->f_const)) { set_error("non-finite source"); return FCM_ERR_NAN; }
  if (p->n_traction < 0 || (p->n_traction > 0 && (!p->traction_face || !p->traction_vec))) {
    set_error("invalid tractions");
    return FCM_ERR_ARG;
  }
  for (int k = 0; k < p->n_traction; ++k)
    if (p->traction_face[k] < 0 || p->traction_face[k] >= 2 * p->dim) {
      set_error("invalid traction face");
      return FCM_ERR_ARG;
    }
  if (p->n_fields > 1) {
    if (!(p->E > 0.0) || !(p->nu > -1.0 && p->nu < 0.5)) { set_error("invalid E/nu"); return FCM_ERR_ARG; }
  } else if (!(p->kappa > 0.0)) {
    set_error("kappa must be positive");
    return FCM_ERR_ARG;
  }
  if (!(o->omega > 0.0) || o->n_pre < 0 || o->n_post < 0 || o->max_iter < 0 ||
      !(o->rtol >= 0.0) || (o->precision != FCM_FP64 && o->precision != FCM_MIXED) ||
      (o->smoother != FCM_SMOOTH_ELEMENTWISE && o->smoother != FCM_SMOOTH_PATCHWISE)) {
    set_error("invalid options");
    return FCM_ERR_ARG;
  }
  if (p->space != FCM_SPACE_TENSOR && p->space != FCM_SPACE_TRUNK) {
    set_error("space must be FCM_SPACE_TENSOR or FCM_SPACE_TRUNK");
    return FCM_ERR_ARG;
  }
  if (p->space == FCM_SPACE_TRUNK && p->refine_levels > 0) {
    set_error("multi-level hp: tensor-product space only");
    return FCM_ERR_ARG;
  }
  if (o->smoother == FCM_SMOOTH_PATCHWISE) {
    const int mpatch =
        patch_size(p->space == FCM_SPACE_TRUNK, p->dim, p->n_fields, p->p, p->p);
    if (mpatch > kMaxPatchM) {
      set_error("patchwise blocks of size %d exceed the supported %d", mpatch, kMaxPatchM);
      return FCM_ERR_ARG;
    }
  }
  return FCM_OK;
}

// --------------------------------------------------------------- tables
static void plane_types(const fcm_handle *h, std::vector<int> &pt) {
  const Geo &g = h->geo;
  const int p = g.p, d = g.d, nf = g.nf;
  pt.clear();
  for (int s = 1; s <= p; ++s)
    for (int t2 = 0; t2 < (d == 3 ? p : 1); ++t2)
      for (int t1 = 0; t1 < p; ++t1)
        for (int t0 = 0; t0 < p; ++t0) {
          const int dg = plane_degree(g, t0, t1, t2);
          if (dg != s) continue;
          for (int c = 0; c < nf; ++c) {
            pt.push_back(t0);
            pt.push_back(t1);
            pt.push_back(t2);
            pt.push_back(c);
          }
        }
}


// Per-axis slot of a patch-local mode (see kernels_patch.hip): slot 0 / p / 2p
// are the hats at nodes v-1 / v / v+1, slots 1..p-1 and p+1..2p-1 the bubbles
// of elements v-1 and v.
static void patch_slot_host(int sl, int p, int &t, int &dl) {
  if (sl == 0) { t = 0; dl = -1; }
  else if (sl < p) { t = sl; dl = -1; }
  else if (sl == p) { t = 0; dl = 0; }
  else if (sl < 2 * p) { t = sl - p; dl = 0; }
  else { t = 0; dl = 1; }
}

static fcm_status build_tables(fcm_handle *h) {
  const Geo &g = h->geo;
  const int d = g.d, nf = g.nf, p = g.p, np = p + 1;
  Tables &t = h->tab;
  // scalar tuples (axis 0 fastest), local modes degree-sorted
  int ms = 1;
  for (int ax = 0; ax < d; ++ax) ms *= np;
  t.ms = ms;
  std::vector<int> lm;
  std::vector<int> smap(ms * nf, -1);
  for (int s = 1; s <= p; ++s)
    for (int a2 = 0; a2 < (d == 3 ? np : 1); ++a2)
      for (int a1 = 0; a1 < np; ++a1)
        for (int a0 = 0; a0 < np; ++a0) {
          const int dg = mode_degree(g, a0, a1, a2);
          if (dg != s) continue;
          for (int c = 0; c < nf; ++c) {
            int idx = (int)lm.size() / 4;
            smap[(a0 + np * (a1 + np * a2)) * nf + c] = idx;
            lm.push_back(a0);
            lm.push_back(a1);
            lm.push_back(a2);
            lm.push_back(c);
          }
        }
  t.m = (int)lm.size() / 4;
  h->h_lm = lm;
  // planes: slot types t_ax in 0..p-1, degree-sorted
  std::vector<int> pidx(std::max(1, p * p * p) * nf, -1);
  std::vector<int> ptype;
  for (int s = 1; s <= p; ++s)
    for (int t2 = 0; t2 < (d == 3 ? p : 1); ++t2)
      for (int t1 = 0; t1 < p; ++t1)
        for (int t0 = 0; t0 < p; ++t0) {
          const int dg = plane_degree(g, t0, t1, t2);
          if (dg != s) continue;
          for (int c = 0; c < nf; ++c) {
            pidx[(t0 + p * (t1 + p * t2)) * nf + c] = (int)ptype.size() / 4;
            ptype.push_back(t0);
            ptype.push_back(t1);
            ptype.push_back(t2);
            ptype.push_back(c);
          }
        }
  t.nP = (int)ptype.size() / 4;
  std::vector<int> xoff(t.m), rows(t.nP * 8, -1), pinfo(t.nP);
  for (int b = 0; b < t.m; ++b) {
    int tt[3], off[3];
    for (int ax = 0; ax < 3; ++ax) {
      int a = lm[4 * b + ax];
      tt[ax] = a <= 1 ? 0 : a - 1;
      off[ax] = (a == 1) ? 1 : 0;
    }
    int plane = pidx[(tt[0] + p * (tt[1] + p * tt[2])) * nf + lm[4 * b + 3]];
    xoff[b] = plane * g.G + off[0] + g.gn[0] * (off[1] + g.gn[1] * off[2]);
  }
  for (int P = 0; P < t.nP; ++P) {
    int vmask = 0, bmask = 0;
    for (int ax = 0; ax < d; ++ax) {
      if (ptype[4 * P + ax] == 0) vmask |= 1 << ax;
      else bmask |= 1 << ax;
    }
    pinfo[P] = vmask | (bmask << 8);
    for (int s = 0; s < (1 << d); ++s) {
      if (s & ~vmask) continue;
      int a[3] = {0, 0, 0};
      for (int ax = 0; ax < d; ++ax) {
        int tt = ptype[4 * P + ax];
        a[ax] = ((s >> ax) & 1) ? 1 : (tt == 0 ? 0 : tt + 1);
      }
      rows[P * 8 + s] = smap[(a[0] + np * (a[1] + np * a[2])) * nf + ptype[4 * P + 3]];
    }
  }
  // Gauss rule, basis at the nodes, 1D sub-interval matrices for levels 0..depth
  std::vector<double> gx, gw;
  gauss_legendre(np, gx, gw);
  std::vector<double> gxw(2 * np), vg(np * np);
  for (int i = 0; i < np; ++i) {
    gxw[i] = gx[i];
    gxw[np + i] = gw[i];
    double v[kMaxP + 1], dv[kMaxP + 1];
    modes1d_host(p, gx[i], v, dv);
    for (int a = 0; a < np; ++a) vg[i * np + a] = v[a];
  }
  const int nint = (2 << g.depth) - 1;
  std::vector<double> tab1d((size_t)nint * 3 * np * np, 0.0);
  for (int l = 0; l <= g.depth; ++l) {
    int nsub = 1 << l;
    for (int i = 0; i < nsub; ++i) {
      double half = 1.0 / nsub, mid = -1.0 + (2.0 * i + 1.0) * half;
      double *T = &tab1d[(size_t)((nsub - 1) + i) * 3 * np * np];
      for (int q = 0; q < np; ++q) {
        double v[kMaxP + 1], dv[kMaxP + 1];
        modes1d_host(p, mid + half * gx[q], v, dv);
        double w = gw[q] * half;
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b) {
            T[a * np + b] += w * v[a] * v[b];
            T[np * np + a * np + b] += w * dv[a] * dv[b];
            T[2 * np * np + a * np + b] += w * dv[a] * v[b];
          }
      }
    }
  }
  TRY(device_upload(h, &t.lm, lm));
  TRY(device_upload(h, &t.xoff, xoff));
  TRY(device_upload(h, &t.rows, rows));
  TRY(device_upload(h, &t.pinfo, pinfo));
  TRY(device_upload(h, &t.smap, smap));
  TRY(device_upload(h, &t.tab1d, tab1d));
  TRY(device_upload(h, &t.gxw, gxw));
  TRY(device_upload(h, &t.vgauss, vg));
  std::vector<double> ball = h->prob.ball, gs = h->prob.gsrc;
  if (ball.empty()) ball.assign(4, 0.0);
  if (gs.empty()) gs.assign(5, 0.0);
  TRY(device_upload(h, &t.ball, ball));
  TRY(device_upload(h, &t.gsrc, gs));
  return FCM_OK;
}

static inline int elin(const Geo &g, int x, int y, int z) { return x + g.n[0] * (y + g.n[1] * z); }

// Schwarz block classes: an element whose whole 3^d neighbourhood is uncut
// has a block that depends only on its position relative to the box faces.
static void build_blocks(fcm_handle *h) {
  const Geo &g = h->geo;
  h->h_blk.assign(g.E, -1);
  std::map<int, int> cls;
  std::vector<int> reps, uniq;
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x) {
        int e = elin(g, x, y, z);
        if (h->h_state[e] == kVoid) continue;
        // uncut = shares K_ref (an uncut element with an edge penalty does not)
        bool unique = h->h_kmat[e] != 0;
        int c[3] = {x, y, z};
        for (int o = 0; o < 27 && !unique; ++o) {
          int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
          if (g.d == 2 && off[2] != 0) continue;
          int nc[3];
          bool in = true;
          for (int ax = 0; ax < 3; ++ax) {
            nc[ax] = c[ax] + off[ax];
            in = in && nc[ax] >= 0 && nc[ax] < g.n[ax];
          }
          if (in && h->h_kmat[elin(g, nc[0], nc[1], nc[2])] != 0) unique = true;
        }
        if (unique) {
          uniq.push_back(e);
          h->h_blk[e] = -2;
          continue;
        }
        int key = 0;
        for (int ax = 0; ax < g.d; ++ax) {
          int cat = (c[ax] == 0 ? 1 : 0) | (c[ax] == g.n[ax] - 1 ? 2 : 0);
          key |= cat << (2 * ax);
        }
        auto it = cls.find(key);
        if (it == cls.end()) {
          int id = (int)reps.size();
          cls[key] = id;
          reps.push_back(e);
          h->h_blk[e] = id;
        } else {
          h->h_blk[e] = it->second;
        }
      }
  h->n_shared = (int)reps.size();
  h->n_unique = (int)uniq.size();
  for (size_t u = 0; u < uniq.size(); ++u) h->h_blk[uniq[u]] = h->n_shared + (int)u;
  h->h_block_elems = reps;
  h->h_block_elems.insert(h->h_block_elems.end(), uniq.begin(), uniq.end());
}

// Kept elements whose component (elements sharing a grid node) touches no
// Dirichlet face are dropped like void ones: constants on such an island have
// zero energy and would make the system singular.  Only overlapping holes
// that enclose cells produce them; without Dirichlet faces nothing changes.
// Returns whether an element was dropped.
static bool drop_floating(const Geo &g, std::vector<uint8_t> &state) {
  if (g.dir == 0) return false;
  std::vector<uint8_t> reach(g.E, 0);
  std::vector<int> stack;
  for (int e = 0; e < g.E; ++e) {
    if (state[e] == kVoid) continue;
    const int c[3] = {e % g.n[0], (e / g.n[0]) % g.n[1], e / (g.n[0] * g.n[1])};
    bool face = false;
    for (int ax = 0; ax < g.d; ++ax) {
      if (c[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) face = true;
      if (c[ax] == g.n[ax] - 1 && ((g.dir >> (2 * ax + 1)) & 1)) face = true;
    }
    if (face) {
      reach[e] = 1;
      stack.push_back(e);
    }
  }
  while (!stack.empty()) {
    const int e = stack.back();
    stack.pop_back();
    const int c[3] = {e % g.n[0], (e / g.n[0]) % g.n[1], e / (g.n[0] * g.n[1])};
    for (int dz = (g.d == 3 ? -1 : 0); dz <= (g.d == 3 ? 1 : 0); ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= g.n[0] || y >= g.n[1] || z >= g.n[2]) continue;
          const int f = x + g.n[0] * (y + g.n[1] * z);
          if (state[f] == kVoid || reach[f]) continue;
          reach[f] = 1;
          stack.push_back(f);
        }
  }
  bool dropped = false;
  for (int e = 0; e < g.E; ++e)
    if (state[e] != kVoid && !reach[e]) {
      state[e] = kVoid;
      dropped = true;
    }
  return dropped;
}

static fcm_status check_flag(fcm_handle *h, const char *what) {
  int f = 0;
  FCM_HIP(hipMemcpyAsync(&f, h->dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  FCM_HIP(hipStreamSynchronize(h->stream));
  if (f) {
    set_error("%s: a pivot was not positive (matrix not SPD in FP64)", what);
    return FCM_ERR_NOT_SPD;
  }
  return FCM_OK;
}

// Coarse level: layer-block-tridiagonal factorisation (exact solve on level
// 0).  Allocation happens on the handle's stream; the factorisation chain is
// issued on a second stream `cs` (it depends only on the element matrices)
// so that it overlaps the Schwarz block setup; coarse_join waits for it.
static fcm_status setup_coarse_alloc(fcm_handle *h) {
  const Geo &g = h->geo;
  Coarse &c = h->co;
  const int sl = g.d - 1;
  int first = ((g.dir >> (2 * sl)) & 1) ? 1 : 0;
  int last = ((g.dir >> (2 * sl + 1)) & 1) ? g.n[sl] - 1 : g.n[sl];
  if (last < first) last = first;
  const int nl = last - first + 1;
  c.PP = 1;
  for (int ax = 0; ax < sl; ++ax) c.PP *= g.gn[ax];
  const int per_layer = g.nf * c.PP;
  int w = std::max(1, (int)std::lround(1024.0 / per_layer));
  w = std::min(w, nl);
  c.w = w;
  c.layer0 = first;
  c.nblk = (nl + w - 1) / w;
  c.nb = g.nf * w * c.PP;
  c.no = g.d == 3 ? 9 : 3;
  const size_t nb2 = (size_t)c.nb * c.nb;
  TRY(device_alloc(h, &c.Sinv, nb2 * c.nblk));
  TRY(device_alloc(h, &c.Gm, nb2 * c.nblk));
  TRY(device_alloc(h, &c.Fm, nb2 * c.nblk));
  TRY(device_alloc(h, &c.Dst, (size_t)c.nblk * c.nb * 3 * c.no * g.nf));
  TRY(device_alloc(h, &c.xblk, (size_t)c.nblk * c.nb));
  TRY(device_alloc(h, &c.bblk, (size_t)c.nblk * c.nb));
  TRY(pool_alloc((void **)&h->co_scr, spd_inverse_scratch_doubles(c.nb, 1) * sizeof(double),
                 h->stream));
  return FCM_OK;
}

// Make stream cs wait for the work enqueued so far on the handle's stream.
static fcm_status coarse_fork(fcm_handle *h, hipStream_t cs) {
  FCM_HIP(hipEventRecord(h->co_ready, h->stream));
  FCM_HIP(hipStreamWaitEvent(cs, h->co_ready, 0));
  return FCM_OK;
}

// Enqueues the block-tridiagonal coarse factorisation (or the h-level setup)
// on cs (after coarse_fork).
static fcm_status setup_coarse_launch(fcm_handle *h, hipStream_t cs) {
  if (h->hmg) return hmg_launch(h, cs);
  const Geo &g = h->geo;
  Coarse &c = h->co;
  const size_t nb2 = (size_t)c.nb * c.nb;
  launch_coarse_stencils(g, h->tab, c, h->kmat, h->Kref64, h->Kcut64, cs);
  for (int k = 0; k < c.nblk; ++k) {
    double *S = c.Sinv + (size_t)k * nb2;
    launch_coarse_first(g, c, k, S, cs);
    // S_k = D_k - B_k F_{k-1},  F_{k-1} = S_{k-1}^{-1} B_k^T is kept for the back sweep
    if (k > 0) launch_coarse_schur(g, c, k, S, c.Fm + (size_t)(k - 1) * nb2, cs);
    spd_inverse_batched(S, c.nb, 1, h->co_scr, h->dflag_co, nullptr, cs);
    if (k > 0) launch_coarse_G(g, c, k, cs);
  }
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

static fcm_status coarse_join(fcm_handle *h, hipStream_t cs) {
  pool_free(h->co_scr, cs);
  h->co_scr = nullptr;
  FCM_HIP(hipStreamSynchronize(cs));
  int f = 0;
  FCM_HIP(hipMemcpyAsync(&f, h->dflag_co, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  FCM_HIP(hipStreamSynchronize(h->stream));
  if (f) {
    set_error("coarse factorisation: a pivot was not positive (matrix not SPD in FP64)");
    return FCM_ERR_NOT_SPD;
  }
  return FCM_OK;
}

// Owner-kernel work units of level l: planes grouped by (vertex mask, comp),
// at most kUnit = 8 planes per unit.
static fcm_status build_units(fcm_handle *h, int l) {
  const Geo &g = h->geo;
  const int p = g.p, d = g.d, nf = g.nf;
  std::vector<int> pt;
  pt.clear();
  for (int s = 1; s <= p; ++s)
    for (int t2 = 0; t2 < (d == 3 ? p : 1); ++t2)
      for (int t1 = 0; t1 < p; ++t1)
        for (int t0 = 0; t0 < p; ++t0) {
          const int dg = plane_degree(g, t0, t1, t2);
          if (dg != s) continue;
          for (int c = 0; c < nf; ++c) {
            pt.push_back(t0);
            pt.push_back(t1);
            pt.push_back(t2);
            pt.push_back(c);
          }
        }
  const int nP = h->lev[l].nP;
  std::vector<int> units;
  for (int V = 0; V < (1 << d); ++V)
    for (int c = 0; c < nf; ++c) {
      std::vector<int> planes;
      for (int P = 0; P < nP; ++P) {
        int vm = 0;
        for (int ax = 0; ax < d; ++ax)
          if (pt[4 * P + ax] == 0) vm |= 1 << ax;
        if (vm == V && pt[4 * P + 3] == c) planes.push_back(P);
      }
      for (size_t k0 = 0; k0 < planes.size(); k0 += 8) {
        int cnt = (int)std::min<size_t>(8, planes.size() - k0);
        int rec[12] = {V, c, cnt, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < cnt; ++k) rec[3 + k] = planes[k0 + k];
        for (int k = cnt; k < 8; ++k) rec[3 + k] = planes[k0];
        units.insert(units.end(), rec, rec + 12);
      }
    }
  h->lev[l].nunits = (int)units.size() / 12;
  return device_upload(h, &h->lev[l].units, units);
}

static fcm_status autotune_levels(fcm_handle *h);

static fcm_status setup_levels(fcm_handle *h) {
  const Geo &g = h->geo;
  int *belems = nullptr;
  TRY(device_upload(h, &belems, h->h_block_elems));
  const int nblocks = (int)h->h_block_elems.size();
  double *kappa = nullptr;
  TRY(pool_alloc((void **)&kappa, std::max(1, nblocks) * sizeof(double), h->stream));
  std::vector<double> hk(nblocks);
  for (int l = 1; l <= h->L; ++l) {
    Level &L = h->lev[l];
    const int m = L.m;
    const size_t mm = (size_t)m * m;
    TRY(device_alloc(h, &L.invS64, mm * nblocks));
    TRY(device_alloc(h, &L.invS32, mm * nblocks));
    L.invU64 = L.invS64 + mm * h->n_shared;
    L.invU32 = L.invS32 + mm * h->n_shared;
    if (m <= kSmallInv) {
      launch_form_invert_small(g, h->tab, L.q, m, belems, nblocks, h->kmat, h->Kref64, h->Kcut64,
                               L.invS64, L.invS32, h->dflag, kappa, h->stream);
    } else {
      const int chunk = 512;
      double *scr = nullptr;
      const int cb = std::min(chunk, nblocks);
      TRY(pool_alloc((void **)&scr, spd_inverse_scratch_doubles(m, cb) * sizeof(double), h->stream));
      launch_form_blocks(g, h->tab, L.q, m, belems, nblocks, h->kmat, h->Kref64, h->Kcut64,
                         L.invS64, h->stream);
      for (int b0 = 0; b0 < nblocks; b0 += chunk) {
        int nbat = std::min(chunk, nblocks - b0);
        spd_inverse_batched(L.invS64 + mm * b0, m, nbat, scr, h->dflag, kappa + b0, h->stream);
      }
      launch_to_f32(L.invS64, L.invS32, (int64_t)(mm * nblocks), h->stream);
      pool_free(scr, h->stream);
    }
    // unique blocks whose Jacobi-scaled condition number exceeds kKappa64 are
    // applied from their FP64 inverse inside the FP32 V-cycle
    FCM_HIP(hipMemcpyAsync(hk.data(), kappa, nblocks * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    FCM_HIP(hipStreamSynchronize(h->stream));
    std::vector<uint8_t> fl(std::max(1, h->n_unique), 0);
    L.n_hi64 = 0;
    for (int u = 0; u < h->n_unique; ++u)
      if (!(hk[h->n_shared + u] <= kKappa64)) {
        fl[u] = 1;
        L.n_hi64++;
      }
    TRY(device_upload(h, &L.hi64, fl));
  }
  pool_free(kappa, h->stream);
  return check_flag(h, "Schwarz block inversion");
}

// ------------------------------------------------------- patchwise blocks
// Patch-local modes at order p, degree-sorted (level q = prefix), with their
// vector offsets, element masks and the owner-gather row table.
static fcm_status build_patch_tables(fcm_handle *h) {
  const Geo &g = h->geo;
  const int d = g.d, nf = g.nf, p = g.p, S = 2 * p + 1;
  std::vector<int> pt;
  plane_types(h, pt);
  const int nP = (int)pt.size() / 4;
  std::map<int, int> pidx;
  for (int P = 0; P < nP; ++P)
    pidx[((pt[4 * P] + p * (pt[4 * P + 1] + p * pt[4 * P + 2])) * nf) + pt[4 * P + 3]] = P;
  auto sdeg = [&](int sl) {
    int t, dl;
    patch_slot_host(sl, p, t, dl);
    return t == 0 ? 1 : t + 1;
  };
  auto pdeg = [&](int s0, int s1, int s2) {
    const int dg[3] = {sdeg(s0), sdeg(s1), sdeg(s2)};
    return prod_degree(g.trunk, d, dg);
  };
  std::vector<int> pm;
  std::map<int, int> kmap;
  for (int q = 1; q <= p; ++q)
    for (int s2 = (d == 3 ? 0 : p); s2 <= (d == 3 ? 2 * p : p); ++s2)
      for (int s1 = 0; s1 < S; ++s1)
        for (int s0 = 0; s0 < S; ++s0) {
          if (pdeg(s0, s1, s2) != q) continue;
          for (int c = 0; c < nf; ++c) {
            kmap[((s0 + S * (s1 + S * s2)) * nf) + c] = (int)pm.size() / 4;
            pm.push_back(s0);
            pm.push_back(s1);
            pm.push_back(s2);
            pm.push_back(c);
          }
        }
  const int m = (int)pm.size() / 4;
  h->ptab.m = m;
  std::vector<int> pxoff(m), pinfo(m);
  for (int k = 0; k < m; ++k) {
    int t[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
    for (int ax = 0; ax < d; ++ax) patch_slot_host(pm[4 * k + ax], p, t[ax], dl[ax]);
    const int P = pidx.at(((t[0] + p * (t[1] + p * t[2])) * nf) + pm[4 * k + 3]);
    pxoff[k] = P * g.G + dl[0] + g.gn[0] * (dl[1] + g.gn[1] * dl[2]);
    int info = 0;
    for (int sm = 0; sm < (1 << d); ++sm) {
      bool ok = true;
      for (int ax = 0; ax < d; ++ax) {
        const int rel = -((sm >> ax) & 1);
        const int lo = t[ax] == 0 ? dl[ax] - 1 : dl[ax], hi = dl[ax];
        ok = ok && rel >= lo && rel <= hi;
      }
      if (ok) info |= 1 << sm;
    }
    for (int ax = 0; ax < d; ++ax) {
      if (t[ax] == 0) info |= 1 << (8 + ax);
      info |= (dl[ax] + 1) << (12 + 2 * ax);
    }
    pinfo[k] = info;
  }
  h->h_ppinfo = pinfo;
  std::vector<int> prow((size_t)nP * 27, -1);
  const int ncb = d == 3 ? 27 : 9;
  for (int P = 0; P < nP; ++P)
    for (int cb = 0; cb < ncb; ++cb) {
      const int dl[3] = {cb % 3 - 1, (cb / 3) % 3 - 1, d == 3 ? cb / 9 - 1 : 0};
      int sl[3] = {p, p, p};
      bool ok = true;
      for (int ax = 0; ax < d; ++ax) {
        const int t = pt[4 * P + ax];
        if (t == 0) sl[ax] = dl[ax] == -1 ? 0 : (dl[ax] == 0 ? p : 2 * p);
        else if (dl[ax] == 1) ok = false;
        else sl[ax] = dl[ax] == -1 ? t : p + t;
      }
      if (!ok) continue;
      prow[(size_t)P * 27 + cb] = kmap.at(((sl[0] + S * (sl[1] + S * sl[2])) * nf) + pt[4 * P + 3]);
    }
  TRY(device_upload(h, &h->ptab.pm, pm));
  TRY(device_upload(h, &h->ptab.pxoff, pxoff));
  TRY(device_upload(h, &h->ptab.pinfo, pinfo));
  TRY(device_upload(h, &h->ptab.prow, prow));
  return FCM_OK;
}

// Patches: grid nodes with at least one kept element around them.  A patch
// whose functions touch only uncut elements (the 4^d elements v-2..v+1 per
// axis) has a block that depends only on its position relative to the box
// faces and shares one inverse per class; all others are unique.
static fcm_status build_patches(fcm_handle *h, std::vector<int> &bnode, std::vector<int> &bkm) {
  const Geo &g = h->geo;
  const int d = g.d;
  std::vector<int> km(g.G, 0), key(g.G, -1);
  for (int z = 0; z < g.gn[2]; ++z)
    for (int y = 0; y < g.gn[1]; ++y)
      for (int x = 0; x < g.gn[0]; ++x) {
        const int v[3] = {x, y, z};
        const int node = x + g.gn[0] * (y + g.gn[1] * z);
        int mask = 0;
        for (int sm = 0; sm < (1 << d); ++sm) {
          int ec[3] = {0, 0, 0};
          bool in = true;
          for (int ax = 0; ax < d; ++ax) {
            ec[ax] = v[ax] - ((sm >> ax) & 1);
            in = in && ec[ax] >= 0 && ec[ax] < g.n[ax];
          }
          if (in && h->h_state[elin(g, ec[0], ec[1], ec[2])] != kVoid) mask |= 1 << sm;
        }
        km[node] = mask;
        if (!mask) continue;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int ax = 0; ax < d; ++ax) {
          lo[ax] = std::max(0, v[ax] - 2);
          hi[ax] = std::min(g.n[ax] - 1, v[ax] + 1);
        }
        bool shared = true;
        for (int ez = lo[2]; ez <= hi[2] && shared; ++ez)
          for (int ey = lo[1]; ey <= hi[1] && shared; ++ey)
            for (int ex = lo[0]; ex <= hi[0] && shared; ++ex)
              if (h->h_kmat[elin(g, ex, ey, ez)] != 0) shared = false;
        if (!shared) continue;
        int k = 0;
        for (int ax = d - 1; ax >= 0; --ax)
          k = 9 * k + 3 * std::min(v[ax], 2) + std::min(g.n[ax] - v[ax], 2);
        key[node] = k;
      }
  std::map<int, int> cls;
  std::vector<std::vector<int>> members;
  std::vector<int> uniq;
  for (int node = 0; node < g.G; ++node) {
    if (!km[node]) continue;
    if (key[node] < 0) {
      uniq.push_back(node);
      continue;
    }
    auto it = cls.find(key[node]);
    if (it == cls.end()) {
      cls[key[node]] = (int)members.size();
      members.emplace_back();
      members.back().push_back(node);
    } else {
      members[it->second].push_back(node);
    }
  }
  std::vector<int> pnode, pkm, pid(g.G, -1), chk;
  const int mp = h->ptab.m, W = (mp + 31) / 32;
  std::vector<unsigned> cpres(std::max<size_t>(1, members.size()) * W, 0u);
  for (size_t c = 0; c < members.size(); ++c) {
    const int first = (int)pnode.size(), cnt = (int)members[c].size();
    for (int q = 0; q < cnt; q += 256) {
      chk.push_back((int)c);
      chk.push_back(first + q);
      chk.push_back(std::min(256, cnt - q));
    }
    for (int node : members[c]) {
      pid[node] = (int)pnode.size();
      pnode.push_back(node);
      pkm.push_back(km[node]);
    }
    // modes present in every patch of the class (same box-face position)
    const int v0 = members[c][0];
    const int vc[3] = {v0 % g.gn[0], (v0 / g.gn[0]) % g.gn[1], v0 / (g.gn[0] * g.gn[1])};
    for (int k = 0; k < mp; ++k) {
      const int info = h->h_ppinfo[k];
      bool pres = (info & km[v0] & 0xff) != 0;
      for (int ax = 0; ax < d && pres; ++ax) {
        if (!((info >> (8 + ax)) & 1)) continue;
        const int nd = vc[ax] + ((info >> (12 + 2 * ax)) & 3) - 1;
        if (nd == 0 && ((g.dir >> (2 * ax)) & 1)) pres = false;
        if (nd == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) pres = false;
      }
      if (pres) cpres[c * W + k / 32] |= 1u << (k % 32);
    }
  }
  h->np_chunks = (int)chk.size() / 3;
  h->p_words = W;
  h->np_shared = (int)pnode.size();
  h->np_classes = (int)members.size();
  for (int node : uniq) {
    pid[node] = (int)pnode.size();
    pnode.push_back(node);
    pkm.push_back(km[node]);
  }
  h->np_unique = (int)uniq.size();
  bnode.clear();
  bkm.clear();
  for (auto &mem : members) {
    bnode.push_back(mem[0]);
    bkm.push_back(km[mem[0]]);
  }
  for (int node : uniq) {
    bnode.push_back(node);
    bkm.push_back(km[node]);
  }
  h->h_pnode = pnode;
  h->h_pkm = pkm;
  if (pnode.empty()) {
    pnode.push_back(0);
    pkm.push_back(0);
  }
  if (chk.empty()) chk.assign(3, 0);
  TRY(device_upload(h, &h->pnode, pnode));
  TRY(device_upload(h, &h->pkm, pkm));
  TRY(device_upload(h, &h->pchk, chk));
  TRY(device_upload(h, &h->pcpres, cpres));
  TRY(device_upload(h, &h->pid, pid));
  return FCM_OK;
}

// Scratch of the patch-block setup, sized for the largest level and
// allocated before the coarse factorisation is launched (freeing memory
// synchronises the device, which would serialise the two).
struct PatchScratch {
  double *blk = nullptr, *scr = nullptr, *kappa = nullptr;
  int chunk = 0;
  size_t nblk = 0, nscr = 0;          // capacities in doubles
};

static int patch_chunk(int m, int nblocks) {
  const size_t per = (size_t)m * m * sizeof(double);
  // up to 1024 blocks (1 GiB of FP64 scratch; 4 GiB for blocks above
  // kSmallPatchM): large batches keep the sweep launches of the SPD inverse
  // wide enough to fill the device
  const size_t budget = (size_t)(m > kSmallPatchM ? 4096 : 1024) << 20;
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(1024, budget / per));
  return std::max(1, std::min(chunk, nblocks));
}

static fcm_status patch_scratch_alloc(fcm_handle *h, int nblocks, PatchScratch &ps) {
  const Geo &g = h->geo;
  size_t nblk = 1, nscr = 1;
  for (int l = 1; l <= h->L; ++l) {
    // the same block size and chunk as setup_patch_levels uses
    const int m = patch_size(g.trunk, g.d, g.nf, g.p, h->lev[l].q);
    const int cb = patch_chunk(m, std::max(1, nblocks));
    nblk = std::max(nblk, (size_t)cb * m * m);
    nscr = std::max(nscr, spd_inverse_scratch_doubles(m, cb));
  }
  TRY(pool_alloc((void **)&ps.blk, nblk * sizeof(double), h->stream));
  TRY(pool_alloc((void **)&ps.scr, nscr * sizeof(double), h->stream));
  ps.nblk = nblk;
  ps.nscr = nscr;
  TRY(pool_alloc((void **)&ps.kappa, std::max(1, nblocks) * sizeof(double), h->stream));
  return FCM_OK;
}

static void patch_scratch_free(fcm_handle *h, PatchScratch &ps) {
  pool_free(ps.blk, h->stream);
  pool_free(ps.scr, h->stream);
  pool_free(ps.kappa, h->stream);
  ps = PatchScratch();
}

// Form and invert the patch blocks of every level >= 1 (FP64, Jacobi-scaled
// Gauss-Jordan sweep) in chunks.  Class inverses are stored as m x ld (ld = m
// rounded up to 4, the layout of the class-product kernels), unique inverses
// as their 16 x 16 tiles on and above the diagonal (symmetric GEMV).
// dbn, dbk: the nblocks base nodes of the patch blocks and their kinds (device).
static fcm_status setup_patch_levels(fcm_handle *h, const int *dbn, const int *dbk, int nblocks,
                                     const PatchScratch &ps) {
  const Geo &g = h->geo;
  const bool mixed = h->opt.precision == FCM_MIXED;
  const int ncls = h->np_classes;
  std::vector<double> hk(std::max(1, nblocks));
  for (int l = 1; l <= h->L; ++l) {
    Level &L = h->lev[l];
    const int m = patch_size(g.trunk, g.d, g.nf, g.p, L.q);
    const int ld = (m + 3) & ~3;
    L.mpatch = m;
    L.ldp = ld;
    const size_t mm = (size_t)m * ld;
    const size_t tp = (size_t)patch_tiles(m) * 256;
    // class inverses carry a tail that the class-product kernels may read past
    // the last row and column (values masked there)
    const size_t tail = 32 * (size_t)ld + 512;
    TRY(device_alloc(h, &L.invS64, mm * std::max(1, ncls) + tail));
    if (mixed) TRY(device_alloc(h, &L.invS32, mm * std::max(1, ncls) + tail));
    TRY(device_alloc(h, &L.invU64, tp * std::max(1, h->np_unique)));
    if (mixed) TRY(device_alloc(h, &L.invU32, tp * std::max(1, h->np_unique)));
    if (nblocks > 0) {
      const int cb = patch_chunk(m, nblocks);
      if ((size_t)cb * m * m > ps.nblk || spd_inverse_scratch_doubles(m, cb) > ps.nscr) {
        set_error("internal: patch block scratch too small for %d blocks of %d", cb, m);
        return FCM_ERR_ARG;
      }
      for (int b0 = 0; b0 < nblocks; b0 += cb) {
        const int nb = std::min(cb, nblocks - b0);
        launch_form_patch_blocks(g, h->tab, h->ptab, m, dbn + b0, dbk + b0, nb, h->kmat,
                                 h->Kref64, h->Kcut64, ps.blk, h->stream);
        spd_inverse_batched(ps.blk, m, nb, ps.scr, h->dflag, ps.kappa + b0, h->stream);
        const int ce = std::min(b0 + nb, ncls);
        if (b0 < ce)
          launch_pack_blocks(ps.blk, m, ld, ce - b0, L.invS64 + mm * b0,
                             mixed ? L.invS32 + mm * b0 : nullptr, h->stream);
        const int ub = std::max(b0, ncls);
        if (ub < b0 + nb)
          launch_pack_tiles(ps.blk + (size_t)(ub - b0) * m * m, m, b0 + nb - ub,
                            L.invU64 + tp * (ub - ncls),
                            mixed ? L.invU32 + tp * (ub - ncls) : nullptr, h->stream);
      }
      FCM_HIP(hipMemcpyAsync(hk.data(), ps.kappa, nblocks * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
      FCM_HIP(hipStreamSynchronize(h->stream));
    }
    std::vector<uint8_t> fl(std::max(1, h->np_unique), 0);
    L.n_hi64 = 0;
    for (int u = 0; u < h->np_unique; ++u)
      if (!(hk[ncls + u] <= kKappa64)) {
        fl[u] = 1;
        L.n_hi64++;
      }
    TRY(device_upload(h, &L.hi64, fl));
  }
  const int mtop = h->lev[h->L].mpatch;
  TRY(device_alloc(h, &h->pYs, (size_t)std::max(1, h->np_shared) * mtop));
  TRY(device_alloc(h, &h->pYu, (size_t)std::max(1, h->np_unique) * mtop));
  // band-pair partial products of the unique GEMV (every level: the
  // autotuner may pick band pairs below kSmallPatchM too)
  size_t nband = 0;
  for (int l = 1; l <= h->L; ++l) {
    const int m = h->lev[l].mpatch;
    const int nb = ((m + 15) / 16 + 15) / 16;
    nband = std::max(nband, (size_t)nb * (nb + 1) / 2 * 512);
  }
  if (nband > 0) TRY(device_alloc(h, &h->pband, nband * std::max(1, h->np_unique)));
  return check_flag(h, "patch Schwarz block inversion");
}

// Quadrature of the penalty on the square's edges (FCM_GEOM_SQUARE, beta >
// 0): each edge, corner to corner counter-clockwise, is cut at every
// crossing with a grid line; a piece gets the (2p+2)-point Gauss rule and
// belongs to the element containing its midpoint (floor((x - lo) / h),
// clamped to the grid).  Output per element with points (increasing element
// index): pel, ptr (CSR) and pts [x, y, weight, Dirichlet data g].
static void edge_penalty_points(const fcm_handle *h, std::vector<int> &pel,
                                std::vector<int> &ptr, std::vector<double> &pts) {
  const Geo &g = h->geo;
  const fcm_problem &pr = h->prob.pr;
  std::vector<double> gx, gw;
  gauss_legendre(2 * g.p + 2, gx, gw);
  const double hs = g.sq[2], cs = g.sq[3], sn = g.sq[4];
  const int sgn[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
  double cx[4], cy[4];
  for (int i = 0; i < 4; ++i) {
    cx[i] = g.sq[0] + hs * (sgn[i][0] * cs - sgn[i][1] * sn);
    cy[i] = g.sq[1] + hs * (sgn[i][0] * sn + sgn[i][1] * cs);
  }
  std::map<int, std::vector<double>> per;   // element -> points
  for (int i = 0; i < 4; ++i) {
    const double a[2] = {cx[i], cy[i]}, b[2] = {cx[(i + 1) % 4], cy[(i + 1) % 4]};
    std::set<double> ts = {0.0, 1.0};
    for (int ax = 0; ax < 2; ++ax) {
      if (b[ax] == a[ax]) continue;
      for (int k = 0; k <= g.n[ax]; ++k) {
        const double t = (g.lo[ax] + k * g.h[ax] - a[ax]) / (b[ax] - a[ax]);
        if (t > 0.0 && t < 1.0) ts.insert(t);
      }
    }
    const double len = std::hypot(b[0] - a[0], b[1] - a[1]);
    std::vector<double> tv(ts.begin(), ts.end());
    for (size_t j = 0; j + 1 < tv.size(); ++j) {
      const double t0 = tv[j], t1 = tv[j + 1];
      if (!(t1 > t0)) continue;
      int cell[2];
      for (int ax = 0; ax < 2; ++ax) {
        const double mid = a[ax] + 0.5 * (t0 + t1) * (b[ax] - a[ax]);
        const double f = std::floor((mid - g.lo[ax]) / g.h[ax]);
        cell[ax] = (int)std::min(std::max(f, 0.0), (double)(g.n[ax] - 1));
      }
      std::vector<double> &out = per[cell[0] + g.n[0] * cell[1]];
      for (size_t q = 0; q < gx.size(); ++q) {
        const double tq = t0 + 0.5 * (gx[q] + 1.0) * (t1 - t0);
        const double x = a[0] + tq * (b[0] - a[0]), y = a[1] + tq * (b[1] - a[1]);
        const double rx = x - g.sq[0], ry = y - g.sq[1];
        const double xr = cs * rx + sn * ry, yr = -sn * rx + cs * ry;
        out.push_back(x);
        out.push_back(y);
        out.push_back(0.0);
        out.push_back(0.5 * gw[q] * (t1 - t0) * len);
        out.push_back(pr.trig_dir[0] * std::cos(pr.trig_dir[1] * xr) *
                      std::sin(pr.trig_dir[1] * yr));
      }
    }
  }
  pel.clear();
  ptr.assign(1, 0);
  pts.clear();
  for (auto &kv : per) {
    pel.push_back(kv.first);
    pts.insert(pts.end(), kv.second.begin(), kv.second.end());
    ptr.push_back((int)(pts.size() / 5));
  }
}

// Penalty quadrature on the popcorn surface phi = 0 (FCM_GEOM_POPCORN, beta >
// 0), the domain read as star-shaped about the origin: directions from a
// Gauss-Legendre rule in cos(theta) (surf_n[0]) times a trapezoid rule in the
// azimuth (surf_n[1]); the radius rho of the surface point by 60 bisection
// steps of phi(rho omega) on [0, 1.5]; weight w_mu (2 pi / n) rho^2 |grad phi|
// / |omega . grad phi|; a point belongs to the element containing it (floor
// rule, clamped); Dirichlet data = the prescribed solution.  Same CSR output
// as edge_penalty_points.
static void popcorn_penalty_points(const fcm_handle *h, std::vector<int> &pel,
                                   std::vector<int> &ptr, std::vector<double> &pts) {
  const Geo &g = h->geo;
  const fcm_problem &pr = h->prob.pr;
  const std::vector<double> &cen = h->prob.ball;
  const int nmu = pr.surf_n[0] > 0 ? pr.surf_n[0] : 256;
  const int naz = pr.surf_n[1] > 0 ? pr.surf_n[1] : 512;
  const double s2 = 0.2 * 0.2, pi = 3.14159265358979323846;
  auto phi = [&](const double *x) {
    double f = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - 0.6;
    for (int k = 0; k < 12; ++k) {
      const double *c = &cen[4 * k];
      const double d2 = (x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) +
                        (x[2] - c[2]) * (x[2] - c[2]);
      f -= 3.0 * std::exp(-d2 / s2);
    }
    return f;
  };
  std::vector<double> mu, wmu;
  gauss_legendre(nmu, mu, wmu);
  std::map<int, std::vector<double>> per;
  for (int i = 0; i < nmu; ++i)
    for (int j = 0; j < naz; ++j) {
      const double az = 2.0 * pi * j / naz, st = std::sqrt(1.0 - mu[i] * mu[i]);
      const double om[3] = {st * std::cos(az), st * std::sin(az), mu[i]};
      double lo = 0.0, hi = 1.5;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double x[3] = {mid * om[0], mid * om[1], mid * om[2]};
        if (phi(x) <= 0.0) lo = mid;
        else hi = mid;
      }
      const double rho = 0.5 * (lo + hi);
      const double x[3] = {rho * om[0], rho * om[1], rho * om[2]};
      const double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      double gr[3] = {x[0] / nx, x[1] / nx, x[2] / nx};
      for (int k = 0; k < 12; ++k) {
        const double *c = &cen[4 * k];
        const double d2 = (x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) +
                          (x[2] - c[2]) * (x[2] - c[2]);
        const double e = 3.0 * std::exp(-d2 / s2);
        for (int ax = 0; ax < 3; ++ax) gr[ax] += 2.0 / s2 * e * (x[ax] - c[ax]);
      }
      const double gn = std::sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
      const double w = wmu[i] * (2.0 * pi / naz) * rho * rho * gn /
                       std::fabs(om[0] * gr[0] + om[1] * gr[1] + om[2] * gr[2]);
      int cell[3];
      for (int ax = 0; ax < 3; ++ax) {
        const double f = std::floor((x[ax] - g.lo[ax]) / g.h[ax]);
        cell[ax] = (int)std::min(std::max(f, 0.0), (double)(g.n[ax] - 1));
      }
      const double sxy = x[0] * x[0] + x[1] * x[1];
      const double u = x[0] * x[0] * x[0] + x[0] * x[1] * x[1] + x[1] * x[1] * x[1] +
                       x[2] * x[2] * x[2] * x[2] + std::sin(3.0 * sxy);
      std::vector<double> &out = per[cell[0] + g.n[0] * (cell[1] + g.n[1] * cell[2])];
      out.insert(out.end(), {x[0], x[1], x[2], w, u});
    }
  pel.clear();
  ptr.assign(1, 0);
  pts.clear();
  for (auto &kv : per) {
    pel.push_back(kv.first);
    pts.insert(pts.end(), kv.second.begin(), kv.second.end());
    ptr.push_back((int)(pts.size() / 5));
  }
}

static fcm_status do_setup(fcm_handle *h) {
  Geo &g = h->geo;
  const fcm_problem &pr = h->prob.pr;
  TRY(build_tables(h));
  const int m = h->tab.m;
  TRY(device_alloc(h, &h->dflag, 1));
  TRY(device_alloc(h, &h->dflag_co, 1));
  // classification
  TRY(device_alloc(h, &h->state, (size_t)g.E));
  launch_classify(g, h->tab.ball, h->state, h->stream);
  h->h_state.resize(g.E);
  FCM_HIP(hipMemcpyAsync(h->h_state.data(), h->state, g.E, hipMemcpyDeviceToHost, h->stream));
  FCM_HIP(hipStreamSynchronize(h->stream));
  if (drop_floating(g, h->h_state))
    FCM_HIP(hipMemcpyAsync(h->state, h->h_state.data(), g.E, hipMemcpyHostToDevice, h->stream));
  // penalty of immersed edges: those elements get stored matrices
  std::vector<int> pen_el, pen_ptr;
  std::vector<double> pen_pts;
  std::vector<uint8_t> pen(g.E, 0);
  if ((g.geom == FCM_GEOM_SQUARE || g.geom == FCM_GEOM_POPCORN) && pr.beta > 0.0) {
    if (g.geom == FCM_GEOM_SQUARE) edge_penalty_points(h, pen_el, pen_ptr, pen_pts);
    else popcorn_penalty_points(h, pen_el, pen_ptr, pen_pts);
    for (int e : pen_el) {
      if (h->h_state[e] == kVoid) {
        set_error("boundary penalty points in a void element");
        return FCM_ERR_ARG;
      }
      pen[e] = 1;
    }
  }
  h->h_kmat.assign(g.E, -1);
  h->h_cut.clear();
  for (int e = 0; e < g.E; ++e) {
    if (h->h_state[e] == kPhys && !pen[e]) h->h_kmat[e] = 0;
    else if (h->h_state[e] != kVoid) {
      h->h_kmat[e] = 1 + (int)h->h_cut.size();
      h->h_cut.push_back(e);
    }
  }
  int *dpel = nullptr, *dpptr = nullptr;
  double *dppts = nullptr;
  if (!pen_el.empty()) {
    TRY(device_upload(h, &dpel, pen_el));
    TRY(device_upload(h, &dpptr, pen_ptr));
    TRY(device_upload(h, &dppts, pen_pts));
  }
  build_blocks(h);
  TRY(device_upload(h, &h->kmat, h->h_kmat));
  TRY(device_upload(h, &h->blk, h->h_blk));
  // element matrices and loads
  const size_t mm = (size_t)m * m;
  const int ncut = (int)h->h_cut.size();
  TRY(device_alloc(h, &h->Kref64, mm));
  TRY(device_alloc(h, &h->Kcut64, mm * std::max(1, ncut)));
  TRY(device_alloc(h, &h->be, (size_t)g.E * m));
  FCM_HIP(hipMemsetAsync(h->be, 0, (size_t)g.E * m * sizeof(double), h->stream));
  int *dcut = nullptr;
  if (ncut > 0) TRY(device_upload(h, &dcut, h->h_cut));
  const int L = h->L;
  TRY(device_alloc(h, &h->b, (size_t)h->lev[L].npad));
  // Element matrices, loads and the assembled right-hand side.  Enqueued after
  // every host-built table is uploaded: an upload drains the stream, so one
  // issued behind these kernels would leave the host waiting for them.
  auto element_work = [&] {
    launch_integrate(g, h->tab, pr, nullptr, 1, 1, h->Kref64, h->be, h->dflag, h->stream);
    if (ncut > 0)
      launch_integrate(g, h->tab, pr, dcut, ncut, 0, h->Kcut64, h->be, h->dflag, h->stream);
    launch_phys_rhs(g, h->tab, pr, h->state, h->be, h->stream);
    launch_edge_penalty(g, h->tab, dpel, (int)pen_el.size(), dpptr, dppts, pr.beta, h->kmat,
                        h->Kcut64, h->be, h->stream);
    for (int k = 0; k < pr.n_traction; ++k)
      launch_traction_rhs(g, h->tab, pr.traction_face[k], &h->prob.tvec[3 * k], h->state, h->be,
                          h->stream);
    launch_assemble_rhs(g, h->tab, h->kmat, h->be, h->b, h->stream);
  };
  // Schwarz inverses per level >= 1, coarse factorisation
  for (int l = 0; l <= L; ++l) TRY(build_units(h, l));
  {
    std::vector<int> ue(h->h_block_elems.begin() + h->n_shared, h->h_block_elems.end());
    if (ue.empty()) ue.push_back(0);
    TRY(device_upload(h, &h->uniq_elems, ue));
    std::vector<int> ce = h->h_cut;
    if (ce.empty()) ce.push_back(0);
    TRY(device_upload(h, &h->cut_elems, ce));
    TRY(device_alloc(h, &h->Yscr, (size_t)std::max(1, std::max(ncut, h->n_unique)) * m));
    TRY(device_alloc(h, &h->Yshr, (size_t)g.E * m));
    std::vector<int> ul, cl;
    for (int e = 0; e < g.E; ++e)
      if (h->h_kmat[e] == 0) ul.push_back(e);
    for (int c = 0; c < h->n_shared; ++c)
      for (int e = 0; e < g.E; ++e)
        if (h->h_blk[e] == c) cl.push_back(e);
    h->n_uncut = (int)ul.size();
    h->n_classed = (int)cl.size();
    // chunks of <= 256 consecutive list entries with the same shared matrix
    auto chunks = [](const std::vector<int> &list, const std::vector<int> &id) {
      std::vector<int> ch;
      size_t i = 0;
      while (i < list.size()) {
        const int c = id[list[i]];
        size_t j = i;
        while (j < list.size() && id[list[j]] == c && j - i < 256) ++j;
        ch.push_back(c);
        ch.push_back((int)i);
        ch.push_back((int)(j - i));
        i = j;
      }
      if (ch.empty()) ch.assign(3, 0);
      return ch;
    };
    std::vector<int> uck = chunks(ul, h->h_kmat), cck = chunks(cl, h->h_blk);
    h->n_uncut_chk = ul.empty() ? 0 : (int)uck.size() / 3;
    h->n_class_chk = cl.empty() ? 0 : (int)cck.size() / 3;
    if (ul.empty()) ul.push_back(0);
    if (cl.empty()) cl.push_back(0);
    TRY(device_upload(h, &h->uncut_list, ul));
    TRY(device_upload(h, &h->class_list, cl));
    TRY(device_upload(h, &h->uncut_chk, uck));
    TRY(device_upload(h, &h->class_chk, cck));
  }
  if (h->opt.coarse == FCM_COARSE_HMG) TRY(hmg_alloc(h));
  else TRY(setup_coarse_alloc(h));
  FCM_HIP(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
  FCM_HIP(hipEventCreateWithFlags(&h->co_ready, hipEventDisableTiming));
  if (h->opt.smoother == FCM_SMOOTH_PATCHWISE) {
    // patch tables and scratch first; the block setup then overlaps the
    // coarse factorisation running on the second stream
    std::vector<int> bnode, bkm;
    PatchScratch ps;
    TRY(build_patch_tables(h));
    TRY(build_patches(h, bnode, bkm));
    int *dbn = nullptr, *dbk = nullptr;
    TRY(device_upload(h, &dbn, bnode.empty() ? std::vector<int>{0} : bnode));
    TRY(device_upload(h, &dbk, bkm.empty() ? std::vector<int>{0} : bkm));
    element_work();
    fcm_status sst = patch_scratch_alloc(h, (int)bnode.size(), ps);
    if (sst == FCM_OK) sst = coarse_fork(h, h->own);
    // The coarse chain is thousands of small serial launches (every block's
    // inverse is a sweep per 32 pivots); a host thread of its own enqueues
    // them while this thread enqueues the patch setup on the handle's stream.
    fcm_status lst = FCM_OK;
    std::string lerr;
    std::thread co;
    if (sst == FCM_OK) {
      try {
        co = std::thread([h, &lst, &lerr] {
          if (hipSetDevice(h->device) != hipSuccess) {
            lst = FCM_ERR_HIP;
            lerr = "coarse launch thread: hipSetDevice failed";
            return;
          }
          lst = setup_coarse_launch(h, h->own);
          if (lst != FCM_OK) lerr = g_err;
        });
      } catch (...) {
        lst = setup_coarse_launch(h, h->own);
        if (lst != FCM_OK) lerr = g_err;
      }
    }
    if (sst == FCM_OK) sst = setup_patch_levels(h, dbn, dbk, (int)bnode.size(), ps);
    if (co.joinable()) co.join();
    fcm_status cst = coarse_join(h, h->own);
    if (lst != FCM_OK && sst == FCM_OK) {
      sst = lst;
      set_error("%s", lerr.c_str());
    }
    patch_scratch_free(h, ps);
    if (sst != FCM_OK) return sst;
    TRY(cst);
  } else {
    element_work();
    TRY(setup_levels(h));
    TRY(coarse_fork(h, h->own));
    TRY(setup_coarse_launch(h, h->own));
    TRY(coarse_join(h, h->own));
  }
  // work vectors
  for (int l = 0; l <= L; ++l) {
    Level &lv = h->lev[l];
    TRY(device_alloc(h, &lv.x64, lv.npad));
    if (l >= 1) {
      TRY(device_alloc(h, &lv.r64, lv.npad));
      TRY(device_alloc(h, &lv.d64, lv.npad));
    }
  }
  const int64_t nf = h->lev[L].npad;
  TRY(device_alloc(h, &h->cg_r, nf));
  TRY(device_alloc(h, &h->cg_z, nf));
  TRY(device_alloc(h, &h->cg_p, nf));
  TRY(device_alloc(h, &h->cg_q, nf));
  TRY(device_alloc(h, &h->red, 1024));
  TRY(device_alloc(h, &h->scal, 16));
  h->hscal = pinned_get();
  if (!h->hscal) {
    set_error("pinned host allocation failed");
    return FCM_ERR_OOM;
  }
  if (h->opt.smoother == FCM_SMOOTH_PATCHWISE) TRY(autotune_levels(h));
  FCM_HIP(hipStreamSynchronize(h->stream));
  return FCM_OK;
}

// ------------------------------------------------------------- V-cycle
static void coarse_solve_t(fcm_handle *h, const double *b, double *x, hipStream_t s) {
  if (h->hmg) hmg_cycle(h, b, x, s);
  else coarse_solve_launch(h->geo, h->co, b, x, s);
}

template <typename T>
static OpArgs<T> stiffness_args(fcm_handle *h, int l) {
  OpArgs<T> a;
  a.m_in = h->lev[l].m;
  a.nP_out = h->lev[l].nP;
  a.ld = h->tab.m;
  a.mid = h->kmat;
  a.matS = h->Kref64;
  a.nS = 1;
  a.matU = h->Kcut64;
  a.m_out = h->lev[l].m;
  a.units = h->lev[l].units;
  a.nunits = h->lev[l].nunits;
  a.selem = h->cut_elems;
  a.nstored = (int)h->h_cut.size();
  a.Y = h->Yscr;
  a.Yshared = h->Yshr;
  a.shlist = h->uncut_list;
  a.nsh = h->n_uncut;
  a.chk = h->uncut_chk;
  a.nchunks = h->n_uncut_chk;
  return a;
}

// mixed: use the FP32 copies of the inverses (FCM_MIXED handles in the V-cycle)
template <typename T>
static OpArgs<T> smoother_args(fcm_handle *h, int l, bool mixed) {
  Level &L = h->lev[l];
  OpArgs<T> a;
  a.m_in = L.m;
  a.nP_out = L.nP;
  a.ld = L.m;
  a.mid = h->blk;
  a.matS = L.invS64;
  a.nS = h->n_shared;
  a.matU = L.invU64;
  a.m_out = L.m;
  a.units = L.units;
  a.nunits = L.nunits;
  a.selem = h->uniq_elems;
  a.nstored = h->n_unique;
  a.Y = h->Yscr;
  a.Yshared = h->Yshr;
  a.shlist = h->class_list;
  a.nsh = h->n_classed;
  a.chk = h->class_chk;
  a.nchunks = h->n_class_chk;
  if (mixed) {
    // FP32 copies of the well-conditioned unique inverses; class inverses and
    // all arithmetic in FP64
    a.matU32 = L.invU32;
    a.u64flag = L.hi64;
  }
  return a;
}

template <typename T>
static PatchArgs<T> patch_args(fcm_handle *h, int l, bool mixed) {
  Level &L = h->lev[l];
  PatchArgs<T> a;
  a.m = L.mpatch;
  a.ld = L.ldp;
  a.ntile = (L.mpatch + 15) / 16;
  a.xlen = (int)L.npad;
  a.nP_out = L.nP;
  a.pnode = h->pnode;
  a.pkm = h->pkm;
  a.chk = h->pchk;
  a.nchunks = h->np_chunks;
  a.cpres = h->pcpres;
  a.pwords = h->p_words;
  a.pid = h->pid;
  a.nsh = h->np_shared;
  a.npu = h->np_unique;
  a.matS64 = L.invS64;
  a.matU = L.invU64;
  if (mixed) {
    // FP32 storage where the block is well conditioned, FP64 otherwise; class
    // (uncut) inverses in FP32 on the FP32 matrix cores
    a.matU32 = L.invU32;
    a.u64flag = L.hi64;
    a.matS32 = L.invS32;
  }
  a.Ys = h->pYs;
  a.Yu = h->pYu;
  a.Pband = h->pband;
  a.class_rows = L.class_rows;
  a.gemv_band = L.gemv_band;
  return a;
}

// out = M_l^{-1} x; if xs: xs = (first ? 0 : xs) + omega * out.  fp64: use
// the FP64 inverses even in a mixed-form handle.
template <typename T>
static void smooth_launch(fcm_handle *h, int l, const T *x, T *out, T *xs, T omega, int first,
                          hipStream_t s, bool stored_only = false, bool fp64 = false) {
  const bool mixed = h->opt.precision == FCM_MIXED && !fp64;
  if (h->opt.smoother == FCM_SMOOTH_PATCHWISE) {
    PatchArgs<T> a = patch_args<T>(h, l, mixed);
    a.stored_only = stored_only;
    a.x = x;
    a.out = out;
    a.xs = xs;
    a.omega = omega;
    a.first = first;
    launch_patch_op<T>(h->geo, h->tab, h->ptab, a, s);
    return;
  }
  OpArgs<T> a = smoother_args<T>(h, l, mixed);
  a.x = x;
  a.out = out;
  a.xs = xs;
  a.omega = omega;
  a.first = first;
  launch_elem_op<T>(h->geo, h->tab, a, s);
}

// Alg. 1 on level l with zero initial guess: x = V(l, b).  The residual is
// updated after every smoothing step (r -= omega A delta == b - A x).
template <typename T>
static void vcycle_level(fcm_handle *h, int l, const T *b, T *x, hipStream_t s) {
  if (l == 0) {
    coarse_solve_t(h, b, x, s);
    return;
  }
  const Geo &g = h->geo;
  Level &L = h->lev[l];
  T *r = L.r64, *dl = L.d64;
  const T w = (T)h->opt.omega;
  OpArgs<T> ap = stiffness_args<T>(h, l);
  ap.x = dl;
  ap.out = r;
  ap.scale = -w;
  const int npre = h->opt.n_pre, npost = h->opt.n_post;
  if (npre == 0) {
    launch_copy<T>(r, b, L.npad, s);
    launch_copy<T>(x, nullptr, L.npad, s);
  }
  for (int it = 0; it < npre; ++it) {
    smooth_launch<T>(h, l, it == 0 ? b : r, dl, x, w, it == 0, s);
    ap.cvec = it == 0 ? b : r;
    launch_elem_op<T>(g, h->tab, ap, s);
  }
  // coarse-grid correction: b_{l-1} = R r (prefix), x += R^T e, r -= A R^T e
  Level &Lc = h->lev[l - 1];
  T *e = Lc.x64;
  vcycle_level<T>(h, l - 1, r, e, s);
  OpArgs<T> pr = stiffness_args<T>(h, l);
  pr.x = e;
  pr.m_in = Lc.m;
  pr.out = r;
  pr.cvec = r;
  pr.scale = (T)-1;
  pr.xp = x;
  pr.ep = e;
  pr.nP_e = Lc.nP;
  launch_elem_op<T>(g, h->tab, pr, s);
  for (int it = 0; it < npost; ++it) {
    smooth_launch<T>(h, l, (const T *)r, dl, x, w, 0, s);
    if (it + 1 < npost) {
      ap.cvec = r;
      launch_elem_op<T>(g, h->tab, ap, s);
    }
  }
}

// ----------------------------------------------------------- autotuner
// Launch variants of the patchwise smoother per level: the rows of the class
// inverse per class-product workgroup (128, 256 or 384; mixed form, blocks
// above 32) and, for blocks up to kSmallPatchM, the unique-patch GEMV by one
// workgroup per patch or by band pairs.  With options.autotune the first
// handle of a problem shape times every candidate on its own data (three
// event-timed smoother launches after one warm-up, on the handle's stream,
// class rows first, then the GEMV kind with the best class rows) and keeps
// the fastest; the choice is cached per shape (dimension, fields, level
// order, form, and the numbers of class and unique patches to a factor of
// two) for the rest of the process.
namespace {
struct TuneKey {
  int d, nf, q, mixed, lsh, lsu;
  bool operator<(const TuneKey &o) const {
    return std::tie(d, nf, q, mixed, lsh, lsu) < std::tie(o.d, o.nf, o.q, o.mixed, o.lsh, o.lsu);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

int ilog2(int v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}
}  // namespace

static fcm_status autotune_levels(fcm_handle *h) {
  const bool mixed = h->opt.precision == FCM_MIXED;
  hipStream_t s = h->stream;
  for (int l = 1; l <= h->L; ++l) {
    Level &L = h->lev[l];
    const int m = L.mpatch;
    L.class_rows = m > 256 ? 3 : m > 128 ? 2 : 1;
    L.gemv_band = m > kSmallPatchM ? 1 : 0;
    L.tune_ms = 0.0;
    if (!h->opt.autotune) continue;
    const TuneKey key{h->geo.d, h->geo.nf, L.q, mixed ? 1 : 0, ilog2(h->np_shared + 1),
                      ilog2(h->np_unique + 1)};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        L.class_rows = it->second.first;
        L.gemv_band = it->second.second;
        continue;
      }
    }
    auto t_start = std::chrono::steady_clock::now();
    launch_copy<double>(L.r64, nullptr, L.npad, s);
    launch_copy<double>(L.x64, nullptr, L.npad, s);
    hipEvent_t e0, e1;
    FCM_HIP(hipEventCreate(&e0));
    FCM_HIP(hipEventCreate(&e1));
    auto time_smoother = [&]() {
      smooth_launch<double>(h, l, L.r64, L.d64, L.x64, h->opt.omega, 0, s);
      hipEventRecord(e0, s);
      for (int i = 0; i < 3; ++i) smooth_launch<double>(h, l, L.r64, L.d64, L.x64, h->opt.omega, 0, s);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      return ms;
    };
    if (mixed && m > 32 && h->np_shared > 0) {
      int best = L.class_rows;
      float tbest = 1e30f;
      for (int c = 1; c <= 3; ++c) {
        L.class_rows = c;
        const float t = time_smoother();
        if (t < tbest) {
          tbest = t;
          best = c;
        }
      }
      L.class_rows = best;
    }
    if (m <= kSmallPatchM && h->np_unique > 0) {
      int best = L.gemv_band;
      float tbest = 1e30f;
      for (int b = 0; b <= 1; ++b) {
        L.gemv_band = b;
        const float t = time_smoother();
        if (t < tbest) {
          tbest = t;
          best = b;
        }
      }
      L.gemv_band = best;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    FCM_HIP(hipGetLastError());
    L.tune_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
            .count();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {L.class_rows, L.gemv_band};
  }
  return FCM_OK;
}

static void vcycle_top(fcm_handle *h, const double *r, double *z, hipStream_t s) {
  const int L = h->L;
  if (L == 0) {
    coarse_solve_t(h, r, z, s);
    return;
  }
  // both forms keep the level vectors in FP64; the mixed form streams FP32
  // copies of the smoother's inverses (smoother_args, patch_args)
  vcycle_level<double>(h, L, r, z, s);
}

static void apply_fine64(fcm_handle *h, int l, const double *x, double *y, hipStream_t s) {
  OpArgs<double> a = stiffness_args<double>(h, l);
  a.x = x;
  a.out = y;
  launch_elem_op<double>(h->geo, h->tab, a, s);
}

static double dot_sync(fcm_handle *h, const double *x, const double *y, int64_t n,
                       hipStream_t s, int slot) {
  int nb = dot_blocks(n);
  launch_dot_partial(x, y, n, h->red, nb, s);
  launch_dot_final(h->red, nb, h->scal + slot, s);
  hipMemcpyAsync(h->hscal + slot, h->scal + slot, sizeof(double), hipMemcpyDeviceToHost, s);
  hipStreamSynchronize(s);
  return h->hscal[slot];
}


// ------------------------------------------------ resumable PCG (Section 4)
// cg_issue enqueues one CG iteration without synchronising: the V-cycle of
// the previous residual (if due), q = A p, alpha, x += alpha p, r -= alpha q
// and ||r||^2, whose scalars are copied to pinned host memory.  cg_finish
// reads them after the stream has drained and decides convergence.  Solves
// driven this way can be interleaved on several streams (serving).
fcm_status cg_begin(fcm_handle *h, CGState &cg, const double *b_dev, double *x, hipStream_t s) {
  const int L = h->L;
  const int64_t n = h->lev[L].npad;
  cg = CGState();
  cg.b = b_dev ? b_dev : h->b;
  cg.x = x;
  FCM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  FCM_HIP(hipMemcpyAsync(h->cg_r, cg.b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  h->history.assign(1, 1.0);
  double bb = dot_sync(h, cg.b, cg.b, n, s, 6);
  if (!std::isfinite(bb)) {
    set_error("non-finite right-hand side");
    cg.done = true;
    cg.status = FCM_ERR_NAN;
    return FCM_ERR_NAN;
  }
  cg.nb = std::sqrt(bb);
  cg.first = true;
  cg.status = FCM_NOT_CONVERGED;
  if (cg.nb == 0.0) {
    cg.rel = 0.0;
    cg.done = true;
    cg.status = FCM_OK;
  } else if (h->opt.max_iter == 0) {
    cg.done = true;
  }
  return FCM_OK;
}

static void cg_issue_body(fcm_handle *h, CGState &cg, hipStream_t s) {
  const int L = h->L;
  const int64_t n = h->lev[L].npad;
  double *r = h->cg_r, *z = h->cg_z, *p = h->cg_p, *q = h->cg_q;
  const int nblk = dot_blocks(n);
  // The FP32 V-cycle is an inexact preconditioner: its CG uses the flexible
  // (Polak-Ribiere) beta, which needs r_new . z_old before z is overwritten.
  const int flexible = h->opt.precision == FCM_MIXED;
  if (flexible && !cg.first) {
    launch_dot_partial(r, z, n, h->red, nblk, s);
    launch_dot_final(h->red, nblk, h->scal + 8, s);
  }
  vcycle_top(h, r, z, s);
  launch_dot_partial(r, z, n, h->red, nblk, s);
  if (cg.first) {
    launch_dot_final(h->red, nblk, h->scal + 0, s);
    launch_cg_update_p(p, z, h->scal, n, 1, s);
  } else {
    launch_dot_final(h->red, nblk, h->scal + 4, s);
    launch_cg_beta(h->scal, flexible, s);
    launch_cg_update_p(p, z, h->scal, n, 0, s);
  }
  apply_fine64(h, L, p, q, s);
  launch_dot_partial(p, q, n, h->red, nblk, s);
  launch_dot_final(h->red, nblk, h->scal + 1, s);
  launch_cg_alpha(h->scal, s);
  launch_cg_update_xr(cg.x, r, p, q, h->scal, n, h->red, nblk, s);
  launch_dot_final(h->red, nblk, h->scal + 3, s);
  hipMemcpyAsync(h->hscal, h->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s);
}

// Capture the steady-state CG iteration for (cg.b, cg.x) as a HIP graph on
// stream s (not the legacy default stream).  Nothing is executed.  Callers
// capture from the thread that owns the handle, before iterating.
fcm_status cg_capture(fcm_handle *h, const CGState &cg, hipStream_t s) {
  if (!h->opt.use_graphs || s == nullptr) return FCM_OK;
  if (h->cg_exec && h->graph_x == cg.x && h->graph_b == cg.b) return FCM_OK;
  if (h->cg_exec) {
    hipGraphExecDestroy(h->cg_exec);
    hipGraphDestroy(h->cg_graph);
    h->cg_exec = nullptr;
    h->cg_graph = nullptr;
  }
  CGState steady = cg;
  steady.first = false;
  FCM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  cg_issue_body(h, steady, s);
  hipGraph_t gph = nullptr;
  FCM_HIP(hipStreamEndCapture(s, &gph));
  if (hipGraphInstantiate(&h->cg_exec, gph, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(gph);
    h->cg_exec = nullptr;
    set_error("graph instantiation failed");
    return FCM_ERR_HIP;
  }
  h->cg_graph = gph;
  h->graph_x = cg.x;
  h->graph_b = cg.b;
  return FCM_OK;
}

// One CG iteration: the captured graph after the first iteration when one
// exists for (b, x) (same launches as the eager body, no memset nodes).
void cg_issue(fcm_handle *h, CGState &cg, hipStream_t s) {
  if (h->opt.use_graphs && !cg.first && h->cg_exec && h->graph_x == cg.x &&
      h->graph_b == cg.b && s != nullptr) {
    hipGraphLaunch(h->cg_exec, s);
    return;
  }
  cg_issue_body(h, cg, s);
}

void cg_finish(fcm_handle *h, CGState &cg) {
  cg.first = false;
  ++cg.it;
  const double pq = h->hscal[1], rr = h->hscal[3];
  if (!(pq > 0.0) || !std::isfinite(rr)) {
    set_error("CG breakdown (p^T A p = %g, r^T r = %g)", pq, rr);
    cg.status = std::isfinite(rr) ? FCM_ERR_BREAKDOWN : FCM_ERR_NAN;
    cg.done = true;
    return;
  }
  cg.rel = std::sqrt(rr) / cg.nb;
  h->history.push_back(cg.rel);
  if (cg.rel < h->opt.rtol) {
    cg.status = FCM_OK;
    cg.done = true;
  } else if (cg.it >= h->opt.max_iter) {
    cg.status = FCM_NOT_CONVERGED;
    cg.done = true;
  }
}

fcm_status cg_report(fcm_handle *h, CGState &cg, fcm_solve_info *info, hipStream_t s) {
  const int64_t n = h->lev[h->L].npad;
  double *q = h->cg_q;
  apply_fine64(h, h->L, cg.x, q, s);
  launch_axpby(q, cg.b, 1.0, -1.0, n, s);   // q = b - A x
  double rr = dot_sync(h, q, q, n, s, 7);
  info->iterations = cg.it;
  info->rel_res = cg.rel;
  info->true_rel_res = cg.nb > 0 ? std::sqrt(rr) / cg.nb : 0.0;
  info->t_setup_ms = h->t_setup_ms;
  info->t_solve_ms = 0.0;
  info->res_history = h->history.data();
  info->n_history = (int)h->history.size();
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

}  // namespace fcm

using namespace fcm;

// ================================================================= C-ABI
extern "C" {

const char *fcm_last_error(void) { return g_err.c_str(); }

const char *fcm_status_string(fcm_status s) {
  switch (s) {
    case FCM_OK: return "ok";
    case FCM_NOT_CONVERGED: return "not converged";
    case FCM_ERR_ARG: return "invalid argument";
    case FCM_ERR_OOM: return "out of device memory";
    case FCM_ERR_HIP: return "HIP runtime error";
    case FCM_ERR_NOT_SPD: return "matrix not positive definite";
    case FCM_ERR_BREAKDOWN: return "CG breakdown";
    case FCM_ERR_NAN: return "non-finite value";
    case FCM_ERR_BUSY: return "busy";
  }
  return "unknown status";
}

void fcm_destroy(fcm_handle *h) {
  if (!h) return;
  if (h->ml) mlhp_free(h);
  if (h->own) hipStreamSynchronize(h->own);   // a failed setup may leave coarse work in flight
  if (h->cg_exec) hipGraphExecDestroy(h->cg_exec);
  if (h->cg_graph) hipGraphDestroy(h->cg_graph);
  // release the memory in stream order after the work queued on the handle's
  // stream (on the library's own stream when it exists, so that a caller's
  // legacy default stream never hosts the release)
  hipStream_t fs = h->stream;
  if (h->own && h->co_ready && hipEventRecord(h->co_ready, h->stream) == hipSuccess &&
      hipStreamWaitEvent(h->own, h->co_ready, 0) == hipSuccess)
    fs = h->own;
  pool_free(h->co_scr, fs);
  for (void *p : h->allocs) pool_free(p, fs);
  if (h->own) hipStreamSynchronize(h->own);
  if (h->co_ready) hipEventDestroy(h->co_ready);
  if (h->own) hipStreamDestroy(h->own);
  pinned_put(h->hscal);
  // A problem that held more than an eighth of the device leaves the pool
  // cut into blocks of its own sizes, which the next large setup mostly
  // cannot use: it would wait while the runtime trims and re-maps the pool
  // on a failed allocation (seconds at 150 GB).  Such memory goes back now.
  size_t free_b = 0, total_b = 0;
  if (h->bytes > ((int64_t)8 << 30) && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
      (size_t)h->bytes > total_b / 8) {
    int dev = 0;
    hipMemPool_t pool;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
      hipMemPoolTrimTo(pool, 0);
  }
  delete h->hmg;
  delete h;
}

fcm_status fcm_hlevels(const fcm_handle *h, int *count, int *cells) {
  if (!h || !count) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  *count = h->hmg ? h->hmg->J + 1 : 0;
  if (cells)
    for (int k = 0; k < *count; ++k)
      for (int ax = 0; ax < 3; ++ax) cells[3 * k + ax] = h->hmg->lev[k].n[ax];
  return FCM_OK;
}

fcm_status fcm_trim_pool(void) {
  int dev = 0;
  FCM_HIP(hipGetDevice(&dev));
  hipMemPool_t pool;
  FCM_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  FCM_HIP(hipMemPoolTrimTo(pool, 0));
  return FCM_OK;
}

fcm_status fcm_setup(const fcm_problem *pr, const fcm_options *op, void *stream,
                     fcm_handle **out) {
  if (!out) {
    set_error("null output handle");
    return FCM_ERR_ARG;
  }
  *out = nullptr;
  fcm_status st = validate(pr, op);
  if (st != FCM_OK) return st;
  auto t0 = std::chrono::steady_clock::now();
  fcm_handle *h = new fcm_handle();
  h->stream = (hipStream_t)stream;
  hipGetDevice(&h->device);
  h->opt = *op;
  Problem &P = h->prob;
  P.pr = *pr;
  for (int j = 0; j < pr->n_balls; ++j) {
    for (int ax = 0; ax < 3; ++ax) P.ball.push_back(ax < pr->dim ? pr->ball_c[j * pr->dim + ax] : 0.0);
    P.ball.push_back(pr->ball_r[j]);
  }
  if (pr->geom == FCM_GEOM_POPCORN) {
    // the twelve bump centres of the popcorn level set (Section 4.3)
    const double r0 = 0.6, s5 = r0 / std::sqrt(5.0), pi = 3.14159265358979323846;
    for (int k = 0; k < 12; ++k) {
      double c[3];
      if (k < 10) {
        const double t = k < 5 ? 2.0 * k * pi / 5.0 : (2.0 * (k - 5) - 1.0) * pi / 5.0;
        c[0] = s5 * 2.0 * std::cos(t);
        c[1] = s5 * std::sin(t);
        c[2] = s5;
      } else {
        c[0] = c[1] = 0.0;
        c[2] = k == 10 ? r0 : -r0;
      }
      P.ball.insert(P.ball.end(), {c[0], c[1], c[2], 0.0});
    }
  }
  P.gsrc.assign(pr->gauss, pr->gauss + 5 * pr->n_gauss);
  P.tface.assign(pr->traction_face, pr->traction_face + pr->n_traction);
  P.tvec.assign(pr->traction_vec, pr->traction_vec + 3 * pr->n_traction);
  P.pr.ball_c = nullptr;
  P.pr.ball_r = nullptr;
  P.pr.gauss = P.gsrc.data();
  P.pr.traction_face = P.tface.data();
  P.pr.traction_vec = P.tvec.data();
  Geo &g = h->geo;
  g.d = pr->dim;
  g.nf = pr->n_fields;
  g.p = pr->p;
  g.G = 1;
  g.E = 1;
  for (int ax = 0; ax < 3; ++ax) {
    g.n[ax] = ax < g.d ? pr->n[ax] : 1;
    g.gn[ax] = ax < g.d ? pr->n[ax] + 1 : 1;
    g.lo[ax] = ax < g.d ? pr->lo[ax] : 0.0;
    g.h[ax] = ax < g.d ? (pr->hi[ax] - pr->lo[ax]) / pr->n[ax] : 1.0;
    g.G *= g.gn[ax];
    g.E *= g.n[ax];
  }
  g.dir = pr->dirichlet_faces;
  g.geom = pr->geom;
  g.nballs = pr->geom == FCM_GEOM_POPCORN ? 12 : pr->n_balls;
  for (int k = 0; k < 5; ++k) g.sq[k] = 0.0;
  if (g.geom == FCM_GEOM_SQUARE) {
    g.sq[0] = pr->ball_c[0];
    g.sq[1] = pr->ball_c[1];
    g.sq[2] = 0.5 * pr->ball_r[0];
    g.sq[3] = std::cos(pr->psi);
    g.sq[4] = std::sin(pr->psi);
  }
  g.trig[0] = pr->trig_src[0];
  g.trig[1] = pr->trig_src[1];
  g.alpha = pr->alpha;
  g.depth = pr->quad_depth;
  g.trunk = pr->space == FCM_SPACE_TRUNK;
  h->L = pr->p - 1;
  for (int l = 0; l <= h->L; ++l) {
    Level &lv = h->lev[l];
    lv.q = l + 1;
    // local modes (per-axis 1D modes 0..p) and planes (per-axis slot types
    // 0..p-1) of level order <= q, times n_f
    int nm = 0, np = 0;
    for (int a2 = 0; a2 < (g.d == 3 ? g.p + 1 : 1); ++a2)
      for (int a1 = 0; a1 <= g.p; ++a1)
        for (int a0 = 0; a0 <= g.p; ++a0) {
          if (mode_degree(g, a0, a1, a2) <= lv.q) ++nm;
          if (a0 < g.p && a1 < g.p && a2 < g.p && plane_degree(g, a0, a1, a2) <= lv.q) ++np;
        }
    lv.m = g.nf * nm;
    lv.nP = g.nf * np;
    lv.npad = (int64_t)lv.nP * g.G;
  }
  if ((int64_t)h->lev[h->L].npad >= (1ll << 31) - 1) {
    delete h;
    set_error("problem too large for 32-bit plane offsets");
    return FCM_ERR_ARG;
  }
  st = pr->refine_levels > 0 ? mlhp_setup(h) : do_setup(h);
  if (st != FCM_OK) {
    fcm_destroy(h);
    return st;
  }
  // DOF counts per level (host, from the states)
  {
    std::vector<int64_t> keys;
    // counted in fcm_sizes on demand
  }
  h->t_setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return FCM_OK;
}

// Existence of DOF (grid point gc, plane slot types tt) on the host.
static bool dof_exists(const fcm_handle *h, const int *gc, const int *tt) {
  const Geo &g = h->geo;
  int vmask = 0;
  for (int ax = 0; ax < g.d; ++ax) {
    if (tt[ax] == 0) {
      vmask |= 1 << ax;
      if (gc[ax] == 0 && ((g.dir >> (2 * ax)) & 1)) return false;
      if (gc[ax] == g.n[ax] && ((g.dir >> (2 * ax + 1)) & 1)) return false;
    } else if (gc[ax] == g.n[ax]) {
      return false;
    }
  }
  for (int s = 0; s < (1 << g.d); ++s) {
    if (s & ~vmask) continue;
    int ec[3] = {gc[0] - (s & 1), gc[1] - ((s >> 1) & 1), gc[2] - ((s >> 2) & 1)};
    bool in = true;
    for (int ax = 0; ax < 3; ++ax) in = in && ec[ax] >= 0 && ec[ax] < g.n[ax];
    if (in && h->h_state[elin(g, ec[0], ec[1], ec[2])] != kVoid) return true;
  }
  return false;
}

fcm_status fcm_sizes(const fcm_handle *h, int *n_levels, int64_t *n_dofs, int64_t *n_padded) {
  if (!h || !n_levels) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_sizes(h, n_levels, n_dofs, n_padded);
  *n_levels = h->L + 1;
  if (n_padded)
    for (int l = 0; l <= h->L; ++l) n_padded[l] = h->lev[l].npad;
  if (n_dofs) {
    const Geo &g = h->geo;
    std::vector<int> pt;
    plane_types(h, pt);
    std::vector<int64_t> per_plane(pt.size() / 4, 0);
    for (size_t P = 0; P < per_plane.size(); ++P)
      for (int gi = 0; gi < g.G; ++gi) {
        int gc[3] = {gi % g.gn[0], (gi / g.gn[0]) % g.gn[1], gi / (g.gn[0] * g.gn[1])};
        if (dof_exists(h, gc, &pt[4 * P])) per_plane[P]++;
      }
    for (int l = 0; l <= h->L; ++l) {
      int64_t s = 0;
      for (int P = 0; P < h->lev[l].nP; ++P) s += per_plane[P];
      n_dofs[l] = s;
    }
  }
  return FCM_OK;
}

fcm_status fcm_dof_keys(const fcm_handle *h, int64_t *keys) {
  if (!h || !keys) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_dof_keys(h, keys);
  const Geo &g = h->geo;
  std::vector<int> pt;
  plane_types(h, pt);
  const int p = g.p;
  int64_t S[3];
  for (int ax = 0; ax < 3; ++ax) S[ax] = (int64_t)(g.n[ax] + 1) * p;
  for (size_t P = 0; P < pt.size() / 4; ++P)
    for (int gi = 0; gi < g.G; ++gi) {
      int gc[3] = {gi % g.gn[0], (gi / g.gn[0]) % g.gn[1], gi / (g.gn[0] * g.gn[1])};
      int64_t &k = keys[(int64_t)P * g.G + gi];
      if (!dof_exists(h, gc, &pt[4 * P])) {
        k = -1;
        continue;
      }
      int64_t key = pt[4 * P + 3];
      for (int ax = g.d - 1; ax >= 0; --ax) {
        int64_t code = (int64_t)gc[ax] * p + pt[4 * P + ax];
        key = key * S[ax] + code;
      }
      k = key;
    }
  return FCM_OK;
}

fcm_status fcm_local_modes(const fcm_handle *h, int *m, int *modes) {
  if (!h || !m) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) {
    set_error("multi-level hp handles have no uniform element layout");
    return FCM_ERR_ARG;
  }
  *m = h->tab.m;
  if (modes) std::memcpy(modes, h->h_lm.data(), h->h_lm.size() * sizeof(int));
  return FCM_OK;
}

fcm_status fcm_element(const fcm_handle *h, int64_t e, int *state, double *K, double *be) {
  if (h && h->ml) {
    set_error("multi-level hp handles have no uniform element layout");
    return FCM_ERR_ARG;
  }
  if (!h || e < 0 || e >= h->geo.E) {
    set_error("element index out of range");
    return FCM_ERR_ARG;
  }
  const int m = h->tab.m;
  if (state) *state = h->h_state[e];
  int kid = h->h_kmat[e];
  if (K && kid >= 0) {
    const double *src = kid == 0 ? h->Kref64 : h->Kcut64 + (size_t)(kid - 1) * m * m;
    FCM_HIP(hipMemcpyAsync(K, src, (size_t)m * m * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  }
  if (be && kid >= 0)
    FCM_HIP(hipMemcpyAsync(be, h->be + (size_t)e * m, (size_t)m * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
  FCM_HIP(hipStreamSynchronize(h->stream));
  return FCM_OK;
}

fcm_status fcm_get_stats(const fcm_handle *h, fcm_stats *s) {
  if (!h || !s) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_stats(h, s);
  s->n_elements = h->geo.E;
  int64_t kept = 0;
  for (auto v : h->h_state) kept += v != kVoid;
  s->n_kept = kept;
  s->n_cut = 0;   // cut elements (stored matrices also serve uncut penalty elements)
  for (uint8_t st : h->h_state) s->n_cut += st == kCut;
  const bool patch = h->opt.smoother == FCM_SMOOTH_PATCHWISE;
  s->n_unique_blocks = patch ? h->np_unique : h->n_unique;
  s->n_shared_classes = patch ? h->np_classes : h->n_shared;
  s->device_bytes = h->bytes;
  s->coarse_blocks = h->hmg ? h->hmg->J : h->co.nblk;
  s->coarse_block_size = h->hmg ? h->hmg->nd : h->co.nb;
  s->n_fp64_blocks = 0;
  for (int l = 1; l <= h->L; ++l) s->n_fp64_blocks += h->lev[l].n_hi64;
  return FCM_OK;
}

fcm_status fcm_get_tuning(const fcm_handle *h, int level, int *class_rows, int *gemv_band,
                          double *tune_ms) {
  if (!h || h->ml || h->opt.smoother != FCM_SMOOTH_PATCHWISE || level < 1 || level > h->L) {
    set_error("fcm_get_tuning: needs a uniform-grid patchwise handle and 1 <= level <= %d",
              h ? h->L : 0);
    return FCM_ERR_ARG;
  }
  const fcm::Level &L = h->lev[level];
  if (class_rows) *class_rows = L.class_rows;
  if (gemv_band) *gemv_band = L.gemv_band;
  if (tune_ms) *tune_ms = L.tune_ms;
  return FCM_OK;
}

fcm_status fcm_set_tuning(fcm_handle *h, int level, int class_rows, int gemv_band) {
  if (!h || h->ml || h->opt.smoother != FCM_SMOOTH_PATCHWISE || level < 1 || level > h->L ||
      class_rows == 0 || class_rows > 3 || class_rows < -1 || gemv_band < -1 || gemv_band > 1) {
    set_error("fcm_set_tuning: invalid handle, level or variant");
    return FCM_ERR_ARG;
  }
  fcm::Level &L = h->lev[level];
  if (gemv_band == 0 && L.mpatch > kSmallPatchM) {
    set_error("fcm_set_tuning: blocks of %d unknowns take band pairs only", L.mpatch);
    return FCM_ERR_ARG;
  }
  if (class_rows > 0) L.class_rows = class_rows;
  if (gemv_band >= 0) L.gemv_band = gemv_band;
  if (h->cg_exec) {   // a captured iteration holds the old launch parameters
    hipGraphExecDestroy(h->cg_exec);
    hipGraphDestroy(h->cg_graph);
    h->cg_exec = nullptr;
    h->cg_graph = nullptr;
  }
  return FCM_OK;
}

fcm_status fcm_rhs(fcm_handle *h, double *b_dev, void *stream) {
  if (!h || !b_dev) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_rhs(h, b_dev, (hipStream_t)stream);
  FCM_HIP(hipMemcpyAsync(b_dev, h->b, h->lev[h->L].npad * sizeof(double),
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return FCM_OK;
}

fcm_status fcm_apply(fcm_handle *h, int level, const double *x, double *y, void *stream) {
  if (h && h->ml && x && y) return mlhp_apply(h, level, x, y, (hipStream_t)stream);
  if (h && h->hmg && x && y && level < 0) return hmg_apply(h, -level, x, y, (hipStream_t)stream);
  if (!h || !x || !y || level < 0 || level > h->L) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  apply_fine64(h, level, x, y, (hipStream_t)stream);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status fcm_smooth(fcm_handle *h, int level, const double *r, double *z, void *stream) {
  if (h && h->ml && r && z) return mlhp_smooth(h, level, r, z, (hipStream_t)stream);
  if (h && h->hmg && r && z && level <= 0)
    return hmg_smooth(h, -level, r, z, (hipStream_t)stream);
  if (!h || !r || !z || level < 1 || level > h->L) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  smooth_launch<double>(h, level, r, z, nullptr, 1.0, 0, (hipStream_t)stream, false, true);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status fcm_spd_inverse(double *A, int n, int batch, double *kappa, void *stream) {
  if (!A || n < 1 || batch < 1) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  double *scr = nullptr;
  int *flag = nullptr;
  FCM_HIP(hipMalloc((void **)&scr, spd_inverse_scratch_doubles(n, batch) * sizeof(double)));
  FCM_HIP(hipMalloc((void **)&flag, sizeof(int)));
  FCM_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  spd_inverse_batched(A, n, batch, scr, flag, kappa, s);
  int f = 0;
  FCM_HIP(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  FCM_HIP(hipStreamSynchronize(s));
  FCM_HIP(hipFree(scr));
  FCM_HIP(hipFree(flag));
  FCM_HIP(hipGetLastError());
  if (f) {
    set_error("a pivot was not positive (matrix not SPD in FP64)");
    return FCM_ERR_NOT_SPD;
  }
  return FCM_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free SPD inverse
// Scratch of fcm_spd_inverse_noalloc: one file-scope device array, so every
// GPU the library runs on holds its own copy (kNoAllocDoubles doubles,
// 32 MiB) until the process ends.  Its last 32 doubles hold the pivot flag.
// Host code never passes the array's name to a kernel (in host code it is a
// host-side stand-in, not a device address): the device address of each
// GPU's copy is looked up once per device with hipGetSymbolAddress.
constexpr size_t kNoAllocDoubles = size_t(4) << 20;
constexpr size_t kNoAllocFlagOff = kNoAllocDoubles - 32;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kNoAllocDevices] = {};

__global__ void clear_flag_kernel(int *flag) { *flag = 0; }

// Device address of the current device's scratch array (nullptr on error).
double *noalloc_scratch(int &dev) {
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_noalloc_ptr[dev] = static_cast<double *>(p);
  }
  return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" {

fcm_status fcm_spd_inverse_noalloc(double *A, int n, int batch, double *kappa, void *stream) {
  if (!A || n < 1 || batch < 1) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  const size_t need = spd_inverse_scratch_doubles(n, batch);
  if (need > kNoAllocFlagOff) {
    set_error("fcm_spd_inverse_noalloc: n = %d, batch = %d need %zu scratch doubles, more than "
              "the %zu of the static device buffer (385 n + 2 doubles per matrix)",
              n, batch, need, kNoAllocFlagOff);
    return FCM_ERR_ARG;
  }
  int dev = -1;
  double *scr = noalloc_scratch(dev);
  if (!scr) {
    if (dev < 0 || dev >= kNoAllocDevices) set_error("no usable current HIP device (%d)", dev);
    return FCM_ERR_HIP;
  }
  hipStream_t s = (hipStream_t)stream;
  int *flag = reinterpret_cast<int *>(scr + kNoAllocFlagOff);
  clear_flag_kernel<<<1, 1, 0, s>>>(flag);
  spd_inverse_batched(A, n, batch, scr, flag, kappa, s);
  int f = 0;
  FCM_HIP(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  FCM_HIP(hipStreamSynchronize(s));
  FCM_HIP(hipGetLastError());
  if (f) {
    set_error("a pivot was not positive (matrix not SPD in FP64)");
    return FCM_ERR_NOT_SPD;
  }
  return FCM_OK;
}

fcm_status fcm_coarse_solve(fcm_handle *h, const double *b, double *x, void *stream) {
  if (!h || !b || !x) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_coarse_solve(h, b, x, (hipStream_t)stream);
  coarse_solve_t(h, b, x, (hipStream_t)stream);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status fcm_vcycle(fcm_handle *h, const double *r, double *z, void *stream) {
  if (!h || !r || !z) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) return mlhp_vcycle(h, r, z, (hipStream_t)stream);
  vcycle_top(h, r, z, (hipStream_t)stream);
  FCM_HIP(hipGetLastError());
  return FCM_OK;
}

fcm_status fcm_pcg_solve(fcm_handle *h, const double *b_dev, double *x_dev, fcm_solve_info *info,
                         void *stream) {
  if (!h || !x_dev) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if (h->ml) return mlhp_pcg(h, b_dev, x_dev, info, s);
  auto t0 = std::chrono::steady_clock::now();
  if (h->opt.use_graphs) {
    // captured iterations run on the library's own stream (capture is not
    // possible on the legacy default stream); order it after the caller's work
    FCM_HIP(hipStreamSynchronize(s));
    s = h->own;
  }
  CGState cg;
  fcm_status st = cg_begin(h, cg, b_dev, x_dev, s);
  if (st < 0) return st;
  if (h->opt.use_graphs && !cg.done) {
    st = cg_capture(h, cg, s);
    if (st < 0) return st;
  }
  while (!cg.done) {
    cg_issue(h, cg, s);
    FCM_HIP(hipStreamSynchronize(s));
    cg_finish(h, cg);
  }
  FCM_HIP(hipGetLastError());
  if (info) {
    st = cg_report(h, cg, info, s);
    if (st < 0) return st;
    info->t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return (fcm_status)cg.status;
}

fcm_status fcm_pcg_solve_batched(fcm_handle *const *hs, int n, double *const *x_dev,
                                 fcm_solve_info *infos, fcm_status *status, void *stream) {
  if (!hs || n < 1 || !x_dev) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !x_dev[i] || hs[i]->ml || !hs[i]->own) {
      set_error("batched solve: handle %d is null or multi-level hp", i);
      return FCM_ERR_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) {
        set_error("batched solve: handle %d appears twice", i);
        return FCM_ERR_ARG;
      }
  }
  auto t0 = std::chrono::steady_clock::now();
  FCM_HIP(hipStreamSynchronize((hipStream_t)stream));   // after the caller's work
  std::vector<CGState> cg(n);
  std::vector<fcm_status> st(n, FCM_OK);
  for (int i = 0; i < n; ++i) {
    st[i] = cg_begin(hs[i], cg[i], nullptr, x_dev[i], hs[i]->own);
    if (st[i] < 0) cg[i].done = true;
  }
  // the first iteration (no beta) of every problem, each on its own stream
  for (int i = 0; i < n; ++i)
    if (!cg[i].done) cg_issue(hs[i], cg[i], hs[i]->own);
  for (int i = 0; i < n; ++i)
    if (!cg[i].done) {
      FCM_HIP(hipStreamSynchronize(hs[i]->own));
      cg_finish(hs[i], cg[i]);
    }
  // steady iterations: one graph holds the iterations of all unfinished
  // problems as independent branches (captured from the launch stream, each
  // problem forked onto its own stream and joined back), launched once per
  // step; it is captured again whenever a problem finishes
  hipStream_t ls = hs[0]->own;
  hipGraph_t pg = nullptr;
  hipGraphExec_t pexec = nullptr;
  std::vector<int> act, built;
  std::vector<hipEvent_t> ev(n + 1, nullptr);
  for (auto &e : ev) FCM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  fcm_status gst = FCM_OK;
  for (;;) {
    act.clear();
    for (int i = 0; i < n; ++i)
      if (!cg[i].done) act.push_back(i);
    if (act.empty()) break;
    if (act != built) {
      if (pexec) hipGraphExecDestroy(pexec);
      if (pg) hipGraphDestroy(pg);
      pexec = nullptr;
      pg = nullptr;
      // the launch stream is hs[0]->own: problem 0 runs on it directly
      hipError_t e = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) e = hipEventRecord(ev[n], ls);
      for (size_t k = 0; e == hipSuccess && k < act.size(); ++k) {
        const int i = act[k];
        hipStream_t si = hs[i]->own;
        if (si != ls) e = hipStreamWaitEvent(si, ev[n], 0);
        if (e != hipSuccess) break;
        CGState steady = cg[i];
        steady.first = false;
        cg_issue_body(hs[i], steady, si);
        if (si != ls) {
          e = hipEventRecord(ev[i], si);
          if (e == hipSuccess) e = hipStreamWaitEvent(ls, ev[i], 0);
        }
      }
      hipError_t e2 = hipStreamEndCapture(ls, &pg);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&pexec, pg, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        set_error("batched solve: building the step graph failed: %s", hipGetErrorString(e));
        gst = FCM_ERR_HIP;
        break;
      }
      built = act;
    }
    hipError_t e = hipGraphLaunch(pexec, ls);
    if (e == hipSuccess) e = hipStreamSynchronize(ls);
    if (e != hipSuccess) {
      set_error("batched solve: step graph failed: %s", hipGetErrorString(e));
      gst = FCM_ERR_HIP;
      break;
    }
    for (int i : act) cg_finish(hs[i], cg[i]);
  }
  for (auto &e : ev) hipEventDestroy(e);
  if (pexec) hipGraphExecDestroy(pexec);
  if (pg) hipGraphDestroy(pg);
  if (gst < 0) return gst;
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  fcm_status worst = FCM_OK;
  for (int i = 0; i < n; ++i) {
    if (st[i] >= 0) st[i] = (fcm_status)cg[i].status;
    if (infos && st[i] >= 0) {
      fcm_status rs = cg_report(hs[i], cg[i], &infos[i], hs[i]->own);
      if (rs < 0) st[i] = rs;
      infos[i].t_solve_ms = ms;
    }
    if (status) status[i] = st[i];
    if (st[i] < 0 && (worst >= 0 || st[i] < worst)) worst = st[i];
    else if (worst >= 0 && st[i] == FCM_NOT_CONVERGED) worst = FCM_NOT_CONVERGED;
  }
  for (int i = 0; i < n; ++i) FCM_HIP(hipStreamSynchronize(hs[i]->own));
  return worst;
}

fcm_status fcm_mg_solve(fcm_handle *h, const double *b_dev, double *x_dev, fcm_solve_info *info,
                        double *rho_max, void *stream) {
  if (!h || !x_dev) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  if (h->ml) {
    set_error("multi-level hp: use fcm_pcg_solve");
    return FCM_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  const int L = h->L;
  const int64_t n = h->lev[L].npad;
  const double *b = b_dev ? b_dev : h->b;
  double *x = x_dev, *r = h->cg_r, *z = h->cg_z, *q = h->cg_p;
  FCM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  FCM_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  h->history.assign(1, 1.0);
  const double nb = std::sqrt(dot_sync(h, b, b, n, s, 6));
  int it = 0;
  double rel = 1.0, rmax = 0.0;
  fcm_status st = FCM_NOT_CONVERGED;
  while (nb > 0 && it < h->opt.max_iter) {
    vcycle_top(h, r, z, s);
    launch_axpby(x, z, 1.0, 1.0, n, s);
    apply_fine64(h, L, x, q, s);
    FCM_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_axpby(r, q, -1.0, 1.0, n, s);
    double rr = dot_sync(h, r, r, n, s, 3);
    ++it;
    double nrel = std::sqrt(rr) / nb;
    if (!std::isfinite(nrel)) {
      st = FCM_ERR_NAN;
      break;
    }
    rmax = std::max(rmax, nrel / rel);
    rel = nrel;
    h->history.push_back(rel);
    if (rel < h->opt.rtol) {
      st = FCM_OK;
      break;
    }
  }
  if (rho_max) *rho_max = rmax;
  if (info) {
    info->iterations = it;
    info->rel_res = rel;
    info->true_rel_res = rel;
    info->t_setup_ms = h->t_setup_ms;
    info->t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->res_history = h->history.data();
    info->n_history = (int)h->history.size();
  }
  return st;
}

// Algorithmic bytes of one smoother / residual launch on level l.  Level
// vectors are FP64 in both forms; the mixed form streams FP32 copies of the
// well-conditioned unique inverses (and of the patch class inverses).
static double op_bytes(const fcm_handle *h, int op, int l) {
  const bool mixed = h->opt.precision == FCM_MIXED;
  const double sm = mixed ? 4.0 : 8.0;
  const fcm::Level &L = h->lev[l];
  const double mm = (double)L.m * L.m;
  const double E = h->geo.E;
  if (op == FCM_OP_SMOOTH && h->opt.smoother == FCM_SMOOTH_PATCHWISE) {
    // unique inverses streamed once, class inverses once, x read, delta and
    // the iterate written, the iterate read
    // (a symmetric unique inverse carries m (m + 1) / 2 numbers)
    const double pm2 = (double)L.mpatch * L.mpatch;
    const double ps2 = 0.5 * L.mpatch * (L.mpatch + 1.0);
    const double nhi = mixed ? L.n_hi64 : 0;
    const double mats = (h->np_unique - nhi) * ps2 * sm + nhi * ps2 * 8.0 +
                        (double)h->np_classes * pm2 * sm;
    return 4.0 * L.npad * 8.0 + mats;
  }
  if (op == FCM_OP_SMOOTH) {
    // class inverses FP64 in both forms
    const double nhi = mixed ? L.n_hi64 : 0;
    const double mats = (h->n_unique - nhi) * mm * sm + nhi * mm * 8.0 + h->n_shared * mm * 8.0;
    return 4.0 * L.npad * 8.0 + mats + 4.0 * E;
  }
  // residual update: delta, r read, r written; FP64 element matrices
  const double mats = ((double)h->h_cut.size() + 1.0) * mm * 8.0;
  return 3.0 * L.npad * 8.0 + mats + 4.0 * E;
}

// Unique-patch GEMV: every symmetric inverse (m (m + 1) / 2 numbers) streamed
// once (FP64 where flagged), the gathered FP64 inputs read once, the FP64
// products written once.
static double stored_bytes(const fcm_handle *h, int l) {
  const bool mixed = h->opt.precision == FCM_MIXED;
  const fcm::Level &L = h->lev[l];
  const double ps2 = 0.5 * L.mpatch * (L.mpatch + 1.0);
  const double nhi = mixed ? L.n_hi64 : h->np_unique;
  const double mats = (h->np_unique - nhi) * ps2 * 4.0 + nhi * ps2 * 8.0;
  return mats + (double)h->np_unique * L.mpatch * 16.0;
}

static double coarse_bytes(const fcm_handle *h) {
  if (h->hmg) return hmg_cycle_bytes(h);
  const fcm::Coarse &c = h->co;
  // S_k^{-1} (all blocks), G_k (k >= 1) and F_k (k < K-1) are each read once
  return (3.0 * c.nblk - 2.0) * c.nb * c.nb * 8.0 + 3.0 * (double)c.nblk * c.nb * 8.0;
}

fcm_status fcm_time_op(fcm_handle *h, int op, int level, int reps, void *stream,
                       double *ms_per_launch, double *bytes_per_launch) {
  if (h && h->ml) {
    set_error("multi-level hp: no timing hook");
    return FCM_ERR_ARG;
  }
  if (!h || reps < 1 || op < FCM_OP_SMOOTH || op > FCM_OP_SMOOTH_STORED ||
      (op != FCM_OP_COARSE && op != FCM_OP_VCYCLE && (level < 1 || level > h->L))) {
    set_error("invalid argument");
    return FCM_ERR_ARG;
  }
  if (op == FCM_OP_SMOOTH_STORED && h->opt.smoother != FCM_SMOOTH_PATCHWISE) {
    set_error("FCM_OP_SMOOTH_STORED needs the patchwise smoother");
    return FCM_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  FCM_HIP(hipEventCreate(&e0));
  FCM_HIP(hipEventCreate(&e1));
  double bytes = 0.0;
  auto launch = [&]() {
    if (op == FCM_OP_SMOOTH || op == FCM_OP_RESIDUAL || op == FCM_OP_SMOOTH_STORED) {
      fcm::Level &L = h->lev[level];
      if (op == FCM_OP_SMOOTH) {
        smooth_launch<double>(h, level, L.r64, L.d64, L.x64, h->opt.omega, 0, s);
      } else if (op == FCM_OP_SMOOTH_STORED) {
        smooth_launch<double>(h, level, L.r64, L.d64, L.x64, h->opt.omega, 0, s, true);
      } else {
        OpArgs<double> a = op == FCM_OP_SMOOTH
                               ? smoother_args<double>(h, level,
                                                       h->opt.precision == FCM_MIXED)
                               : stiffness_args<double>(h, level);
        a.x = op == FCM_OP_SMOOTH ? L.r64 : L.d64;
        a.out = op == FCM_OP_SMOOTH ? L.d64 : L.r64;
        if (op == FCM_OP_SMOOTH) {
          a.xs = L.x64;
          a.omega = h->opt.omega;
        } else {
          a.cvec = L.r64;
          a.scale = -h->opt.omega;
        }
        launch_elem_op<double>(h->geo, h->tab, a, s);
      }
    } else if (op == FCM_OP_COARSE) {
      coarse_solve_t(h, h->b, h->lev[0].x64, s);
    } else {
      vcycle_top(h, h->b, h->cg_z, s);
    }
  };
  if (op == FCM_OP_SMOOTH || op == FCM_OP_RESIDUAL) bytes = op_bytes(h, op, level);
  else if (op == FCM_OP_SMOOTH_STORED) bytes = stored_bytes(h, level);
  else if (op == FCM_OP_COARSE) bytes = coarse_bytes(h);
  else {
    for (int l = 1; l <= h->L; ++l)
      bytes += (h->opt.n_pre + h->opt.n_post) * op_bytes(h, FCM_OP_SMOOTH, l) +
               (h->opt.n_pre + h->opt.n_post) * op_bytes(h, FCM_OP_RESIDUAL, l);
    bytes += coarse_bytes(h);
  }
  launch();  // warm-up
  FCM_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) launch();
  FCM_HIP(hipEventRecord(e1, s));
  FCM_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  FCM_HIP(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (ms_per_launch) *ms_per_launch = ms / reps;
  if (bytes_per_launch) *bytes_per_launch = bytes;
  return FCM_OK;
}

}  // extern "C"
