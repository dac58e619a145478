// Serving: a request loop that keeps several E_c solves on the device at
// once.  Requests wait in arrival order; a dispatcher thread admits the
// first waiting request whose memory footprint (the valence-block model of
// ssrpa_footprint) fits what is not yet reserved, up to max_running at once,
// and hands it to a worker thread with its own HIP stream.  Device work of
// the admitted requests overlaps; every solve uses only its own system, and
// kernel configurations depend only on the request's sizes, so each result
// is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

using clock_type = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  std::vector<int32_t> miller;
  std::vector<double> coeff;
  std::vector<double> energy;
  ssrpa_system_desc desc{};
  int n_eig = 0, n_freq = 0, vb = 0;
  std::vector<double> omega, weight;
  ssrpa_precision prec = SSRPA_FP64;
  size_t footprint = 0;
  int state = SSRPA_REQ_QUEUED;
  ssrpa_status status = SSRPA_OK;
  double ec = 0.0;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
};

}  // namespace

struct ssrpa_server {
  ssrpa::Context *ctx = nullptr;
  int max_running = 1;
  double max_bypass = 0.0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> queue;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<std::thread> workers;
  size_t reserved = 0, reserved_peak = 0;
  int running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  clock_type::time_point t0 = clock_type::now();
  std::thread dispatcher;

  double now() const {
    return std::chrono::duration<double>(clock_type::now() - t0).count();
  }
  size_t capacity() const { return ctx->budget; }
  void dispatch_loop();
  void run(Request *r);
};

void ssrpa_server::run(Request *r) {
  hipStream_t st = nullptr;
  ssrpa_status s = hipSetDevice(ctx->device) == hipSuccess ? SSRPA_OK : SSRPA_ERR_HIP;
  if (s == SSRPA_OK && hipStreamCreate(&st) != hipSuccess) s = SSRPA_ERR_HIP;
  ssrpa_system *sys = nullptr;
  double ec = 0.0;
  auto *cctx = static_cast<ssrpa_context *>(ctx);
  if (s == SSRPA_OK) s = ssrpa_system_create(cctx, &r->desc, st, &sys);
  if (s == SSRPA_OK) s = ssrpa_chi0_static(sys, r->prec, r->vb, nullptr, 1, st);
  int n_g = 0;
  if (s == SSRPA_OK) s = ssrpa_chi_gvectors(sys, &n_g, nullptr);
  if (s == SSRPA_OK && r->n_eig < n_g)
    s = ssrpa_subspace(sys, r->n_eig, nullptr, nullptr, st);
  if (s == SSRPA_OK)
    s = ssrpa_correlation_energy(sys, r->n_eig, r->n_freq, r->omega.data(),
                                 r->weight.data(), r->prec, r->vb, 1.0, &ec,
                                 nullptr, nullptr, st);
  if (sys) ssrpa_system_destroy(sys);
  if (st) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> g(mu);
  r->status = s;
  r->ec = ec;
  r->t_done = now();
  r->state = s == SSRPA_OK ? SSRPA_REQ_DONE : SSRPA_REQ_FAILED;
  reserved -= r->footprint;
  running -= 1;
  // the host copies of the inputs are no longer needed
  std::vector<double>().swap(r->coeff);
  cv.notify_all();
}

void ssrpa_server::dispatch_loop() {
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    bool admitted = false;
    if (!queue.empty() && running < max_running) {
      const double t = now();
      for (auto it = queue.begin(); it != queue.end(); ++it) {
        Request *r = *it;
        if (reserved + r->footprint <= capacity()) {
          queue.erase(it);
          reserved += r->footprint;
          reserved_peak = std::max(reserved_peak, reserved);
          running += 1;
          r->state = SSRPA_REQ_RUNNING;
          r->t_start = t;
          workers.emplace_back([this, r] { run(r); });
          admitted = true;
          break;
        }
        // an old request keeps its place: nothing behind it may pass
        if (t - r->t_submit > max_bypass) break;
      }
    }
    if (admitted) continue;
    if (stop && queue.empty()) break;
    cv.wait(lk);
  }
}

extern "C" {

ssrpa_status ssrpa_server_create(ssrpa_context *ctx, int max_running,
                                 double max_bypass_s, ssrpa_server **out) {
  if (!ctx || !out || max_running < 1 || !(max_bypass_s >= 0.0))
    return SSRPA_ERR_ARG;
  auto *s = new (std::nothrow) ssrpa_server();
  if (!s) return SSRPA_ERR_NOMEM;
  s->ctx = ctx;
  s->max_running = max_running;
  s->max_bypass = max_bypass_s;
  s->dispatcher = std::thread([s] { s->dispatch_loop(); });
  *out = s;
  return SSRPA_OK;
}

ssrpa_status ssrpa_server_submit(ssrpa_server *srv, const ssrpa_system_desc *desc,
                                 int n_eig, int n_freq, const double *omega,
                                 const double *weight, ssrpa_precision precision,
                                 uint64_t *request_id) {
  if (!srv || !desc || !omega || !weight || !request_id || n_freq < 1 ||
      n_eig < 1 || desc->coeff_on_device || !desc->coeff || !desc->miller ||
      !desc->energy || desc->n_pw < 1 || desc->n_v < 1 || desc->n_c < 1)
    return SSRPA_ERR_ARG;
  auto r = std::make_unique<Request>();
  const int nb = desc->n_v + desc->n_c;
  r->miller.assign(desc->miller, desc->miller + 3 * (size_t)desc->n_pw);
  r->coeff.assign(desc->coeff, desc->coeff + 2 * (size_t)desc->n_pw * nb);
  r->energy.assign(desc->energy, desc->energy + nb);
  r->desc = *desc;
  r->desc.miller = r->miller.data();
  r->desc.coeff = r->coeff.data();
  r->desc.energy = r->energy.data();
  r->n_eig = n_eig;
  r->n_freq = n_freq;
  r->omega.assign(omega, omega + n_freq);
  r->weight.assign(weight, weight + n_freq);
  r->prec = precision;
  // Block size: the largest whose footprint leaves room for a second request
  // of the same size; otherwise the largest that fits at all.
  const size_t cap = srv->capacity();
  int vb = 0;
  ssrpa_status st = ssrpa_plan_valence_block(&r->desc, n_eig, n_freq, precision,
                                             cap / 2, &vb);
  if (st != SSRPA_OK)
    st = ssrpa_plan_valence_block(&r->desc, n_eig, n_freq, precision, cap, &vb);
  if (st != SSRPA_OK) return st;
  size_t fp = 0;
  st = ssrpa_footprint(&r->desc, n_eig, n_freq, precision, vb, &fp);
  if (st != SSRPA_OK) return st;
  if (fp > cap) return SSRPA_ERR_NOMEM;
  r->vb = vb;
  r->footprint = fp;
  std::lock_guard<std::mutex> g(srv->mu);
  r->id = srv->next_id++;
  r->t_submit = srv->now();
  *request_id = r->id;
  srv->queue.push_back(r.get());
  srv->all[r->id] = std::move(r);
  srv->cv.notify_all();
  return SSRPA_OK;
}

ssrpa_status ssrpa_server_poll(ssrpa_server *srv, uint64_t request_id, int *state,
                               ssrpa_status *status, double *ec, double *t_submit,
                               double *t_start, double *t_done) {
  if (!srv) return SSRPA_ERR_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end()) return SSRPA_ERR_ARG;
  const Request &r = *it->second;
  if (state) *state = r.state;
  if (status) *status = r.status;
  if (ec) *ec = r.ec;
  if (t_submit) *t_submit = r.t_submit;
  if (t_start) *t_start = r.t_start;
  if (t_done) *t_done = r.t_done;
  return SSRPA_OK;
}

ssrpa_status ssrpa_server_drain(ssrpa_server *srv) {
  if (!srv) return SSRPA_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv.wait(lk, [srv] { return srv->queue.empty() && srv->running == 0; });
  return SSRPA_OK;
}

ssrpa_status ssrpa_server_memory(ssrpa_server *srv, size_t *reserved_peak,
                                 size_t *high_water) {
  if (!srv) return SSRPA_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (reserved_peak) *reserved_peak = srv->reserved_peak;
  }
  return ssrpa_context_memory(static_cast<ssrpa_context *>(srv->ctx), nullptr,
                              high_water);
}

ssrpa_status ssrpa_server_destroy(ssrpa_server *srv) {
  if (!srv) return SSRPA_ERR_ARG;
  ssrpa_server_drain(srv);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv.notify_all();
  }
  srv->dispatcher.join();
  for (auto &t : srv->workers)
    if (t.joinable()) t.join();
  delete srv;
  return SSRPA_OK;
}

}  // extern "C"
