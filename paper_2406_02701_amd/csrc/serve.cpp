// Serving engine: continuous batching of Gaussian log-likelihood requests.
//
// Worker slots each own a context (its own HIP stream and workspace) whose
// device allocations come from one arena sized by the HBM budget.  A request
// is admitted from the FIFO queue when a slot is free and its estimated
// footprint fits in the unreserved part of the budget; requests on different
// slots overlap on the device.  The arithmetic of a request never depends on
// its co-runners (no shared buffers, no atomics, fixed reduction orders), so a
// result is bitwise the same alone and in a mix.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "mpcr_internal.h"

using namespace mpcr;

namespace {

struct Request {
  uint64_t id;
  int64_t n;
  std::vector<double> locs, z;
  mpcr_theta_t theta;
  double t_submit;
  size_t footprint;
  int retries = 0;
};

struct Done {
  uint64_t id;
  double loglik;
  mpcr_diag_t diag;
  double t_submit, t_done;
  int status;
  int fallback;
};

}  // namespace

struct mpcr_server {
  int device = 0;
  mpcr_serve_opts_t opts{};
  std::unique_ptr<Arena> arena;
  size_t budget = 0, reserved = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::deque<Done> done;
  int64_t running = 0, rejected = 0, finished_total = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Band map, then (guard > 0) promotion by the norm guard on the sorted sites.
int request_map(mpcr_ctx* ctx, const mpcr_serve_opts_t& o, int64_t n, const double* d_sorted_locs,
                const mpcr_theta_t& th, std::vector<uint8_t>& map) {
  const int64_t nt = (n + o.nb - 1) / o.nb;
  const int dmax[3] = {o.band_fp64, o.band_fp32, -1};
  const int precs[3] = {MPCR_FP64, MPCR_FP32, o.far_prec};
  std::vector<uint8_t> band(nt * nt);
  int rc = mpcr_tilemap_banded(n, o.nb, dmax, precs, 3, band.data());
  if (rc) return rc;
  if (!(o.guard > 0)) {
    map = band;
    return MPCR_OK;
  }
  std::vector<double> amax(nt * nt);
  if ((rc = mpcr_covariance_tile_amax(ctx, n, o.nb, d_sorted_locs, &th, amax.data()))) return rc;
  map.resize(nt * nt);
  return mpcr_tilemap_guarded(n, o.nb, band.data(), amax.data(), o.guard * th.nugget, map.data());
}

// One request on the worker's context: Morton order, map, log-likelihood.
void run_request(mpcr_server* srv, mpcr_ctx* ctx, Request& r, Done& d) {
  TraceRange tr("serve request");
  const mpcr_serve_opts_t& o = srv->opts;
  hipStream_t s = ctx_stream(ctx);
  const int64_t n = r.n;
  d.status = MPCR_OK;
  d.fallback = 0;
  d.loglik = 0;
  memset(&d.diag, 0, sizeof d.diag);
  double *dl = nullptr, *dz = nullptr, *dls = nullptr, *dzs = nullptr;
  int64_t* perm = nullptr;
  Arena* A = srv->arena.get();
  auto cleanup = [&] {
    (void)hipStreamSynchronize(s);
    for (void* p : {(void*)dl, (void*)dz, (void*)dls, (void*)dzs, (void*)perm}) A->free(p);
  };
  dl = (double*)A->alloc(n * 16);
  dz = (double*)A->alloc(n * 8);
  dls = (double*)A->alloc(n * 16);
  dzs = (double*)A->alloc(n * 8);
  perm = (int64_t*)A->alloc(n * 8);
  if (!dl || !dz || !dls || !dzs || !perm) {
    d.status = MPCR_ERR_NOMEM;
    cleanup();
    return;
  }
  hipError_t e = hipMemcpyAsync(dl, r.locs.data(), n * 16, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dz, r.z.data(), n * 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    d.status = MPCR_ERR_DEVICE;
    cleanup();
    return;
  }
  int rc = mpcr_morton_order(ctx, n, dl, perm);
  if (rc == MPCR_OK) {
    e = launch_gather_rows((int)n, 2, dl, n, perm, dls, n, s);
    if (e == hipSuccess) e = launch_gather_rows((int)n, 1, dz, n, perm, dzs, n, s);
    if (e != hipSuccess) rc = MPCR_ERR_DEVICE;
  }
  std::vector<uint8_t> map;
  if (rc == MPCR_OK) rc = request_map(ctx, o, n, dls, r.theta, map);
  if (rc == MPCR_OK) {
    mpcr_tilemap_t tm{n, o.nb, (n + o.nb - 1) / o.nb, map.data()};
    rc = mpcr_gauss_loglik(ctx, n, dls, dzs, 1, &r.theta, &tm, 0, &o.refine, &d.loglik, &d.diag);
    if (rc == MPCR_ERR_NOT_SPD && o.fallback_fp64) {  // last resort after any promotions
      for (auto& v : map)
        if (v != 255) v = MPCR_FP64;
      d.fallback = 1;
      rc = mpcr_gauss_loglik(ctx, n, dls, dzs, 1, &r.theta, &tm, 0, &o.refine, &d.loglik, &d.diag);
    }
  }
  d.status = rc;
  cleanup();
  ctx_release_workspace(ctx);
}

void worker_main(mpcr_server* srv) {
  (void)hipSetDevice(srv->device);
  mpcr_ctx* ctx = nullptr;
  if (ctx_create_with_arena(srv->device, srv->arena.get(), &ctx) != MPCR_OK) return;
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      // FIFO admission: the head of the queue runs when its footprint fits
      srv->cv.wait(lk, [&] {
        return srv->stop || (!srv->queue.empty() && srv->reserved + srv->queue.front().footprint <= srv->budget);
      });
      if (srv->stop) break;
      r = std::move(srv->queue.front());
      srv->queue.pop_front();
      srv->reserved += r.footprint;
      srv->running += 1;
    }
    Done d;
    d.id = r.id;
    d.t_submit = r.t_submit;
    run_request(srv, ctx, r, d);
    d.t_done = srv->now();
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->reserved -= r.footprint;
      srv->running -= 1;
      // the arena can be fragmented although the reservation fitted: retry once
      // another request has finished
      if (d.status == MPCR_ERR_NOMEM && srv->running > 0 && r.retries < 8 && !srv->stop) {
        r.retries += 1;
        const int64_t finished_before = srv->finished_total;
        srv->cv.wait(lk, [&] { return srv->stop || srv->finished_total != finished_before || srv->running == 0; });
        srv->queue.push_front(std::move(r));
      } else {
        srv->done.push_back(d);
        srv->finished_total += 1;
      }
    }
    srv->cv.notify_all();
  }
  mpcr_ctx_destroy(ctx);
}

}  // namespace

extern "C" {

size_t mpcr_serve_footprint(int64_t n, int64_t nb) {
  if (n <= 0 || nb <= 0) return 0;
  return loglik_footprint(n, nb, 1) + (size_t)n * 64 + 4096;
}

int mpcr_serve_create(int device, size_t hbm_budget, int max_slots, const mpcr_serve_opts_t* opts,
                      mpcr_server** out) {
  if (!out || !opts || max_slots < 1 || max_slots > 64 || hbm_budget < (1u << 20)) return MPCR_ERR_ARG;
  if (opts->nb < 128 || opts->nb % 128 || opts->band_fp64 < 0 || opts->band_fp32 < opts->band_fp64 ||
      !(opts->far_prec == MPCR_FP16 || opts->far_prec == MPCR_BF16 || opts->far_prec == MPCR_FP32 ||
        opts->far_prec == MPCR_FP64) ||
      !(opts->refine.tol > 0) || opts->refine.max_iter < 0 || opts->refine.solver < 0 || opts->refine.solver > 1 ||
      opts->refine.recompute < 0 || (opts->refine.promote_on_breakdown != 0 && opts->refine.promote_on_breakdown != 1) ||
      (opts->refine.direct_eta != 0 && opts->refine.direct_eta != 1))
    return MPCR_ERR_ARG;
  // the stored FP64 residual doubles a request's device footprint, which the
  // admission estimate does not cover: requests regenerate Sigma from the sites
  if (opts->refine.residual != 0) return MPCR_ERR_ARG;
  *out = nullptr;
  auto* srv = new mpcr_server();
  srv->device = device;
  srv->opts = *opts;
  srv->budget = hbm_budget;
  srv->arena.reset(new Arena());
  (void)hipSetDevice(device);
  if (srv->arena->init(hbm_budget) != hipSuccess) {
    delete srv;
    return MPCR_ERR_NOMEM;
  }
  for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back(worker_main, srv);
  *out = srv;
  return MPCR_OK;
}

int mpcr_serve_destroy(mpcr_server* srv) {
  if (!srv) return MPCR_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->queue.clear();
  }
  srv->cv.notify_all();
  for (auto& t : srv->workers) t.join();
  delete srv;
  return MPCR_OK;
}

int mpcr_serve_submit(mpcr_server* srv, uint64_t req_id, int64_t n, const double* h_locs, const double* h_z,
                      const mpcr_theta_t* theta) {
  if (!srv || n <= 0 || n >= (1ll << 31) || !h_locs || !h_z || !theta) return MPCR_ERR_ARG;
  if (!(theta->nu == 0.5 || theta->nu == 1.5 || theta->nu == 2.5) || !(theta->sigma2 > 0) || !(theta->range > 0) ||
      !(theta->nugget >= 0))
    return MPCR_ERR_ARG;
  Request r;
  r.id = req_id;
  r.n = n;
  r.locs.assign(h_locs, h_locs + 2 * n);
  r.z.assign(h_z, h_z + n);
  r.theta = *theta;
  r.footprint = mpcr_serve_footprint(n, srv->opts.nb);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (r.footprint > srv->budget) {
      srv->rejected += 1;
      return MPCR_ERR_REJECTED;
    }
    r.t_submit = srv->now();
    srv->queue.push_back(std::move(r));
  }
  srv->cv.notify_all();
  return MPCR_OK;
}

int mpcr_serve_poll(mpcr_server* srv, uint64_t* req_id, double* loglik, mpcr_diag_t* diag, double* t_submit,
                    double* t_done, int* status, int* used_fallback) {
  if (!srv) return MPCR_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->done.empty()) return 0;
  Done d = srv->done.front();
  srv->done.pop_front();
  if (req_id) *req_id = d.id;
  if (loglik) *loglik = d.loglik;
  if (diag) *diag = d.diag;
  if (t_submit) *t_submit = d.t_submit;
  if (t_done) *t_done = d.t_done;
  if (status) *status = d.status;
  if (used_fallback) *used_fallback = d.fallback;
  return 1;
}

double mpcr_serve_clock(const mpcr_server* srv) { return srv ? srv->now() : 0.0; }

int mpcr_serve_stats(mpcr_server* srv, int64_t* queued, int64_t* running, int64_t* finished, int64_t* rejected,
                     size_t* bytes_reserved) {
  if (!srv) return MPCR_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (queued) *queued = (int64_t)srv->queue.size();
  if (running) *running = srv->running;
  if (finished) *finished = (int64_t)srv->done.size();
  if (rejected) *rejected = srv->rejected;
  if (bytes_reserved) *bytes_reserved = srv->reserved;
  return MPCR_OK;
}

}  // extern "C"
