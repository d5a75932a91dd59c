// Serving loop of libfcm: continuous batching of MG-PCG solves on one GPU.
//
// Host threads share the device:
//  * admission (two threads): take pending requests in arrival order and,
//    while a batch slot is free and the estimated device footprint of the
//    request fits the memory budget next to the hierarchies already resident,
//    build its hierarchy (fcm_setup) on their own admission stream;
//  * ticks: each active solve has one CG iteration (V-cycle, apply, fused
//    updates; a captured graph after the first) in flight on one of several
//    streams; when its completion event fires, the iteration is finished on
//    the host and the next one issued.  Requests join and leave at any time,
//    so solves of different grids and orders overlap on the device.
// Results are copied to host memory when a solve retires and its hierarchy is
// freed at once, returning its footprint to the budget.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "fcm_internal.hpp"

namespace fcm {

// Device footprint estimate of a problem before setup (bytes): padded vectors,
// element matrices of the cells within one cell of a hole surface, Schwarz
// inverses (elementwise: of the cut-affected elements; patchwise: of the
// cut-affected grid nodes, about 4-5 per cut cell, plus the class inverses and
// the transient block scratch), and the dense coarse S^-1, G, F blocks.
int64_t footprint_estimate(const fcm_problem &p, const fcm_options &o) {
  const int d = p.dim, nf = p.n_fields;
  const bool mixed = o.precision == FCM_MIXED;
  int64_t G = 1, E = 1;
  double h = 1.0;
  for (int ax = 0; ax < d; ++ax) {
    G *= p.n[ax] + 1;
    E *= p.n[ax];
    h = std::min(h, (p.hi[ax] - p.lo[ax]) / p.n[ax]);
  }
  int64_t mp = nf, nP = nf;
  for (int ax = 0; ax < d; ++ax) {
    mp *= p.p + 1;
    nP *= p.p;
  }
  // cells touched by the ball surfaces
  double surf = 0.0;
  for (int j = 0; j < p.n_balls; ++j) {
    double r = p.ball_r[j];
    surf += (d == 3) ? 4.0 * M_PI * r * r / (h * h) : 2.0 * M_PI * r / h;
  }
  int64_t ncut = std::min<int64_t>(E, (int64_t)(3.0 * surf) + 1);
  int64_t bytes = 0;
  bytes += ncut * mp * mp * 12;               // cut matrices FP64 + FP32
  bytes += E * mp * 8;                        // element loads
  const int64_t per = mixed ? 12 : 8;         // FP64 (+ FP32) copy per inverse entry
  int64_t inv = 0;
  if (o.smoother == FCM_SMOOTH_PATCHWISE) {
    const int64_t nuniq = std::min<int64_t>(G, ncut * (d == 3 ? 5 : 4));
    int64_t mtop = 0;
    for (int q = 2; q <= p.p; ++q) {
      int64_t m = nf;    // tensor-space block size (an upper bound for the trunk space)
      for (int ax = 0; ax < d; ++ax) m *= 2 * q + 1;
      const int64_t ld = (m + 3) & ~3, nt = (m + 15) / 16;
      inv += 128 * m * ld * per + nuniq * (nt * (nt + 1) / 2) * 256 * per;
      mtop = m;
    }
    inv += G * mtop * 8 + ((int64_t)1100 << 20);  // patch products, block scratch (setup)
  } else {
    const int64_t nuniq = std::min<int64_t>(E, ncut * (d == 3 ? 4 : 3));
    for (int q = 2; q <= p.p; ++q) {
      int64_t m = nf;
      for (int ax = 0; ax < d; ++ax) m *= q + 1;
      inv += (nuniq + 64) * m * m * per;
    }
    inv += E * mp * 8;                         // element products
  }
  bytes += inv;
  // vectors: ~10 FP64 + 6 FP32 fine-level vectors
  bytes += nP * G * (10 * 8 + 6 * 4);
  // coarse: layers of ~1024 unknowns, S^-1, G and F blocks
  int64_t per_layer = nf;
  for (int ax = 0; ax < d - 1; ++ax) per_layer *= p.n[ax] + 1;
  int64_t w = std::max<int64_t>(1, (int64_t)(1024.0 / per_layer + 0.5));
  int64_t nb = per_layer * w;
  int64_t nblk = (p.n[d - 1] + w) / w;
  bytes += 3 * nblk * nb * nb * 8 + nblk * nb * 27 * nf * 8;
  return bytes + (16 << 20);
}

}  // namespace fcm

using namespace fcm;

namespace {

struct Request {
  uint64_t id = 0;
  fcm_problem pr{};
  fcm_options opt{};
  std::vector<double> ball_c, ball_r, gauss, tvec;
  std::vector<int> tface;
  std::chrono::steady_clock::time_point t_submit, t_done;
  fcm_handle *h = nullptr;
  double *x = nullptr;
  CGState cg;
  int stream = 0;
  bool done = false;
  fcm_status status = FCM_OK;
  std::vector<double> x_host;
  fcm_solve_info info{};
  std::vector<double> hist;
  int64_t footprint = 0;
  double t_solve_start_ms = 0.0;
  hipEvent_t ev = nullptr;     // completion of the iteration in flight
  bool inflight = false;
  std::string err;             // error text of a failed request
};

// Setups of admitted requests run on this many threads, each with its own
// stream: the coarse factorisation of a small request is a chain of launches
// that fills a few compute units, so several setups share the device.
constexpr int kAdmitThreads = 4;

}  // namespace

struct fcm_server {
  fcm_server_opts opt{};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> pending;
  std::vector<std::shared_ptr<Request>> active;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> next_id{1};
  int64_t resident = 0;          // bytes of admitted hierarchies (estimates until set up)
  int n_admitting = 0;
  std::vector<hipStream_t> streams;
  hipStream_t setup_stream[kAdmitThreads] = {};
  std::thread admit_thr[kAdmitThreads], tick_thr;
  // Graph captures run alone: setup work and ticks hold this lock shared,
  // a capture holds it exclusively (capture must not overlap synchronous
  // allocation or copy calls of other threads).
  std::shared_mutex hip_mu;
  int device = 0;
};

static void finish_request(fcm_server *s, std::shared_ptr<Request> &r, hipStream_t st) {
  if (r->h && r->status >= 0) {
    fcm_solve_info info{};
    cg_report(r->h, r->cg, &info, st);
    r->hist.assign(info.res_history, info.res_history + info.n_history);
    r->info = info;
    r->info.res_history = nullptr;
    r->info.n_history = (int)r->hist.size();
    const int64_t n = r->h->lev[r->h->L].npad;
    r->x_host.resize(n);
    hipMemcpyAsync(r->x_host.data(), r->x, n * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
  }
  r->t_done = std::chrono::steady_clock::now();
  r->info.t_solve_ms =
      std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count() -
      r->t_solve_start_ms;
  fcm::pool_free(r->x, st);
  r->x = nullptr;
  if (r->h) fcm_destroy(r->h);
  r->h = nullptr;
}

static void admission_loop(fcm_server *s, int which) {
  hipSetDevice(s->device);
  hipStream_t setup_stream = s->setup_stream[which];
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] {
        if (s->stop) return true;
        if (s->pending.empty()) return false;
        const int64_t need = s->pending.front()->footprint;
        const bool slot = (int)s->active.size() + s->n_admitting < s->opt.max_active;
        const bool mem = s->resident + need <= s->opt.memory_budget_bytes || s->resident == 0;
        return slot && mem;
      });
      if (s->stop) return;
      r = s->pending.front();
      s->pending.pop_front();
      s->resident += r->footprint;
      s->n_admitting++;
    }
    fcm_handle *h = nullptr;
    std::shared_lock<std::shared_mutex> hl(s->hip_mu);
    fcm_status st = fcm_setup(&r->pr, &r->opt, setup_stream, &h);
    if (st < 0) r->err = fcm_last_error();
    double *x = nullptr;
    if (st == FCM_OK) {
      const int64_t n = h->lev[h->L].npad;
      st = fcm::pool_alloc((void **)&x, n * sizeof(double), setup_stream);
    }
    if (st == FCM_OK) {
      h->stream = nullptr;
      // pick the stream this solve ticks on
      r->h = h;
      r->x = x;
      r->stream = (int)(r->id % s->streams.size());
      // the first CG steps run on the admission stream (never on a tick stream,
      // which the tick thread may be capturing a graph on)
      st = cg_begin(h, r->cg, nullptr, x, setup_stream);
      hl.unlock();
      if (st >= 0 && !r->cg.done) {
        std::unique_lock<std::shared_mutex> xl(s->hip_mu);
        st = cg_capture(h, r->cg, setup_stream);
      }
      hl.lock();
      if (st < 0) r->err = fcm_last_error();
      if (st >= 0 && hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess)
        st = FCM_ERR_HIP;
      r->t_solve_start_ms = std::chrono::duration<double, std::milli>(
                                std::chrono::steady_clock::now() - r->t_submit)
                                .count();
    } else if (h) {
      fcm_destroy(h);
    }
    hl.unlock();
    std::lock_guard<std::mutex> lk(s->mu);
    s->n_admitting--;
    if (st < 0) {
      r->status = st;
      r->done = true;
      r->t_done = std::chrono::steady_clock::now();
      fcm::pool_free(r->x, setup_stream);
      if (r->h) fcm_destroy(r->h);
      r->h = nullptr;
      r->x = nullptr;
      s->resident -= r->footprint;
    } else {
      // replace the estimate by the measured footprint
      s->resident += h->bytes - r->footprint;
      r->footprint = h->bytes;
      s->active.push_back(r);
    }
    s->cv.notify_all();
  }
}

// Ticks: each active solve has at most one CG iteration in flight, followed
// by an event.  As soon as a solve's event has completed its iteration is
// finished on the host and the next one issued, so small and large solves
// progress at their own pace while sharing the device.
static void tick_loop(fcm_server *s) {
  hipSetDevice(s->device);
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->active.empty(); });
      if (s->stop) return;
      batch = s->active;
    }
    bool progressed = false;
    std::vector<std::shared_ptr<Request>> retired;
    std::shared_lock<std::shared_mutex> hl(s->hip_mu);
    for (auto &r : batch) {
      hipStream_t st = s->streams[r->stream];
      if (r->inflight) {
        const hipError_t q = hipEventQuery(r->ev);
        if (q == hipErrorNotReady) continue;
        r->inflight = false;
        progressed = true;
        if (q != hipSuccess) {
          r->cg.done = true;
          r->cg.status = FCM_ERR_HIP;
          set_error("device error in a CG iteration: %s", hipGetErrorString(q));
        } else {
          cg_finish(r->h, r->cg);
        }
      }
      if (r->cg.done) {
        retired.push_back(r);
        continue;
      }
      cg_issue(r->h, r->cg, st);
      hipEventRecord(r->ev, st);
      r->inflight = true;
      progressed = true;
    }
    for (auto &r : retired) {
      r->status = (fcm_status)r->cg.status;
      if (r->status < 0) r->err = fcm_last_error();
      int64_t fp = r->footprint;
      finish_request(s, r, s->streams[r->stream]);
      if (r->ev) hipEventDestroy(r->ev);
      r->ev = nullptr;
      std::lock_guard<std::mutex> lk(s->mu);
      r->done = true;
      s->resident -= fp;
      for (size_t i = 0; i < s->active.size(); ++i)
        if (s->active[i] == r) {
          s->active.erase(s->active.begin() + i);
          break;
        }
      s->cv.notify_all();
    }
    hl.unlock();
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

extern "C" {

fcm_status fcm_server_create(const fcm_server_opts *o, fcm_server **out) {
  if (!o || !out || o->max_active < 1 || o->n_streams < 1 || o->memory_budget_bytes <= 0) {
    set_error("invalid server options");
    return FCM_ERR_ARG;
  }
  auto *s = new fcm_server();
  s->opt = *o;
  hipGetDevice(&s->device);
  s->streams.resize(std::min(o->n_streams, 16));
  for (auto &st : s->streams)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      set_error("stream creation failed");
      return FCM_ERR_HIP;
    }
  for (int k = 0; k < kAdmitThreads; ++k)
    if (hipStreamCreateWithFlags(&s->setup_stream[k], hipStreamNonBlocking) != hipSuccess) {
      set_error("stream creation failed");
      return FCM_ERR_HIP;
    }
  for (int k = 0; k < kAdmitThreads; ++k) s->admit_thr[k] = std::thread(admission_loop, s, k);
  s->tick_thr = std::thread(tick_loop, s);
  *out = s;
  return FCM_OK;
}

fcm_status fcm_serve_submit(fcm_server *s, const fcm_problem *prob, const fcm_options *opts,
                            uint64_t *req_id) {
  if (!s || !prob || !opts || !req_id) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  auto r = std::make_shared<Request>();
  r->id = s->next_id++;
  r->pr = *prob;
  r->opt = *opts;
  r->ball_c.assign(prob->ball_c, prob->ball_c + prob->n_balls * prob->dim);
  r->ball_r.assign(prob->ball_r, prob->ball_r + prob->n_balls);
  r->gauss.assign(prob->gauss, prob->gauss + 5 * prob->n_gauss);
  r->tface.assign(prob->traction_face, prob->traction_face + prob->n_traction);
  r->tvec.assign(prob->traction_vec, prob->traction_vec + 3 * prob->n_traction);
  r->pr.ball_c = r->ball_c.data();
  r->pr.ball_r = r->ball_r.data();
  r->pr.gauss = r->gauss.data();
  r->pr.traction_face = r->tface.data();
  r->pr.traction_vec = r->tvec.data();
  r->footprint = footprint_estimate(r->pr, r->opt);
  r->t_submit = std::chrono::steady_clock::now();
  *req_id = r->id;
  std::lock_guard<std::mutex> lk(s->mu);
  s->all[r->id] = r;
  s->pending.push_back(r);
  s->cv.notify_all();
  return FCM_OK;
}

fcm_status fcm_serve_poll(fcm_server *s, uint64_t req_id, int *done, double *x_host,
                          int64_t x_len, fcm_solve_info *info, double *latency_ms) {
  if (!s || !done) {
    set_error("null argument");
    return FCM_ERR_ARG;
  }
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end()) {
      set_error("unknown request id");
      return FCM_ERR_ARG;
    }
    r = it->second;
    *done = r->done ? 1 : 0;
  }
  if (!*done) return FCM_OK;
  if (x_host && !r->x_host.empty()) {
    int64_t n = std::min<int64_t>(x_len, (int64_t)r->x_host.size());
    std::memcpy(x_host, r->x_host.data(), n * sizeof(double));
  }
  if (info) {
    *info = r->info;
    info->res_history = r->hist.data();
    info->n_history = (int)r->hist.size();
  }
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (r->status < 0) set_error("request %llu: %s", (unsigned long long)req_id, r->err.c_str());
  return r->status;
}

fcm_status fcm_server_destroy(fcm_server *s) {
  if (!s) return FCM_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (int k = 0; k < kAdmitThreads; ++k)
    if (s->admit_thr[k].joinable()) s->admit_thr[k].join();
  if (s->tick_thr.joinable()) s->tick_thr.join();
  hipSetDevice(s->device);
  for (auto st : s->streams) hipStreamSynchronize(st);
  for (int k = 0; k < kAdmitThreads; ++k)
    if (s->setup_stream[k]) hipStreamSynchronize(s->setup_stream[k]);
  for (auto &r : s->active) {
    if (r->ev) hipEventDestroy(r->ev);
    fcm::pool_free(r->x, s->setup_stream[0]);
    if (r->h) fcm_destroy(r->h);
  }
  for (auto st : s->streams) hipStreamDestroy(st);
  for (int k = 0; k < kAdmitThreads; ++k)
    if (s->setup_stream[k]) hipStreamDestroy(s->setup_stream[k]);
  fcm_trim_pool();
  delete s;
  return FCM_OK;
}

}  // extern "C"
