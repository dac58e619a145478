// Serving: a request loop that keeps several E_c solves on the device at
// once.  Requests wait in arrival order.  The server owns a fixed pool of
// max_running worker threads, each with one HIP stream created with the
// server and destroyed only after every worker has been joined, so no HIP
// state is created or torn down while requests run.  A free worker admits
// the first waiting request whose memory footprint (the valence-block model
// of ssrpa_footprint) fits what is not yet reserved and runs the whole solve
// on its own stream.  Device work of the admitted requests overlaps; every
// solve uses only its own system, and kernel configurations depend only on
// the request's sizes, so each result is the same alone and in the mix.
//
// Each solve also records two HIP events on its stream (before the first
// and after the last of its device work); their times relative to an event
// recorded when the server started show whether solves shared the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
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
  std::vector<double> occupation;
  ssrpa_system_desc desc{};
  int n_eig = 0, n_freq = 0, vb = 0;
  std::vector<double> omega, weight;
  ssrpa_precision prec = SSRPA_FP64;
  size_t footprint = 0;
  int state = SSRPA_REQ_QUEUED;
  ssrpa_status status = SSRPA_OK;
  double ec = 0.0;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  double dev_start_ms = -1.0, dev_end_ms = -1.0;  // device clock, vs t0 event
  std::string error;  // the failed call's message
};

struct Worker {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  std::thread th;
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
  std::vector<Worker> workers;
  hipEvent_t ev_t0 = nullptr;   // device time origin of the event times
  size_t reserved = 0, reserved_peak = 0;
  int running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  clock_type::time_point t0 = clock_type::now();

  double now() const {
    return std::chrono::duration<double>(clock_type::now() - t0).count();
  }
  size_t capacity() const { return ctx->budget; }
  // First waiting request that may start now (locked); nullptr if none.
  Request *admit_locked();
  void worker_loop(Worker *w);
  void run(Request *r, Worker *w, bool dev_ok);
};

Request *ssrpa_server::admit_locked() {
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
      return r;
    }
    // an old request keeps its place: nothing behind it may pass
    if (t - r->t_submit > max_bypass) break;
  }
  return nullptr;
}

void ssrpa_server::run(Request *r, Worker *w, bool dev_ok) {
  hipStream_t st = w->stream;
  ssrpa_system *sys = nullptr;
  double ec = 0.0;
  auto *cctx = static_cast<ssrpa_context *>(ctx);
  ssrpa_status s = dev_ok && hipEventRecord(w->ev_start, st) == hipSuccess
                       ? SSRPA_OK
                       : SSRPA_ERR_HIP;
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
  // the worker's own error text (error text is kept per thread)
  std::string err = s == SSRPA_OK ? std::string() : ssrpa_last_error(cctx);
  // every call has finished its device work when it returns (failed calls
  // included), so the system's memory goes back to the cache idle
  if (sys) ssrpa_system_destroy(sys);
  float ms0 = -1.f, ms1 = -1.f;
  if (dev_ok && hipEventRecord(w->ev_end, st) == hipSuccess &&
      hipEventSynchronize(w->ev_end) == hipSuccess) {
    if (hipEventElapsedTime(&ms0, ev_t0, w->ev_start) != hipSuccess) ms0 = -1.f;
    if (hipEventElapsedTime(&ms1, ev_t0, w->ev_end) != hipSuccess) ms1 = -1.f;
  }
  std::lock_guard<std::mutex> g(mu);
  r->status = s;
  r->error = std::move(err);
  r->ec = ec;
  r->t_done = now();
  r->dev_start_ms = ms0;
  r->dev_end_ms = ms1;
  r->state = s == SSRPA_OK ? SSRPA_REQ_DONE : SSRPA_REQ_FAILED;
  reserved -= r->footprint;
  running -= 1;
  // the host copies of the inputs are no longer needed
  std::vector<double>().swap(r->coeff);
  cv.notify_all();
}

void ssrpa_server::worker_loop(Worker *w) {
  // the thread's device is set once; the stream lives as long as the server
  const bool dev_ok = hipSetDevice(ctx->device) == hipSuccess;
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    Request *r = admit_locked();
    if (r) {
      lk.unlock();
      run(r, w, dev_ok);
      lk.lock();
      continue;
    }
    if (stop && queue.empty()) break;
    cv.wait(lk);
  }
}

namespace {

void destroy_server(ssrpa_server *s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto &w : s->workers)
    if (w.th.joinable()) w.th.join();
  // every worker has exited: the streams are idle and no thread uses them
  for (auto &w : s->workers) {
    if (w.ev_start) (void)hipEventDestroy(w.ev_start);
    if (w.ev_end) (void)hipEventDestroy(w.ev_end);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  if (s->ev_t0) (void)hipEventDestroy(s->ev_t0);
  delete s;
}

}  // namespace

extern "C" {

ssrpa_status ssrpa_server_create(ssrpa_context *ctx, int max_running,
                                 double max_bypass_s, ssrpa_server **out) {
  if (!ctx || !out || max_running < 1 || max_running > 64 ||
      !(max_bypass_s >= 0.0))
    return SSRPA_ERR_ARG;
  *out = nullptr;
  auto *s = new (std::nothrow) ssrpa_server();
  if (!s) return SSRPA_ERR_NOMEM;
  s->ctx = ctx;
  s->max_running = max_running;
  s->max_bypass = max_bypass_s;
  // all HIP objects of the server are made here, on the calling thread
  bool ok = hipSetDevice(ctx->device) == hipSuccess &&
            hipEventCreate(&s->ev_t0) == hipSuccess;
  s->workers.resize(max_running);
  for (auto &w : s->workers) {
    if (!ok) break;
    ok = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&w.ev_start) == hipSuccess &&
         hipEventCreate(&w.ev_end) == hipSuccess;
  }
  ok = ok && hipEventRecord(s->ev_t0, s->workers[0].stream) == hipSuccess &&
       hipEventSynchronize(s->ev_t0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    destroy_server(s);
    return SSRPA_ERR_HIP;
  }
  s->t0 = clock_type::now();
  for (auto &w : s->workers) {
    Worker *wp = &w;
    w.th = std::thread([s, wp] { s->worker_loop(wp); });
  }
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
  if (desc->occupation) {
    r->occupation.assign(desc->occupation, desc->occupation + nb);
    r->desc.occupation = r->occupation.data();
  }
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

ssrpa_status ssrpa_server_device_times(ssrpa_server *srv, uint64_t request_id,
                                       double *start_ms, double *end_ms) {
  if (!srv || !start_ms || !end_ms) return SSRPA_ERR_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end()) return SSRPA_ERR_ARG;
  const Request &r = *it->second;
  if (r.state != SSRPA_REQ_DONE && r.state != SSRPA_REQ_FAILED)
    return SSRPA_ERR_STATE;
  *start_ms = r.dev_start_ms;
  *end_ms = r.dev_end_ms;
  return SSRPA_OK;
}

const char *ssrpa_server_error(ssrpa_server *srv, uint64_t request_id) {
  if (!srv) return "";
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end()) return "";
  const Request &r = *it->second;
  if (r.state != SSRPA_REQ_FAILED) return "";
  return r.error.c_str();
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
  destroy_server(srv);
  return SSRPA_OK;
}

}  // extern "C"
