// Host stand-in of the HIP runtime calls used by the library's host code
// (see mock/hip/hip_runtime.h): streams are FIFOs run by executor threads.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <set>
#include <thread>

struct MockStream {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool busy = false, stop = false;
  std::thread th;
  MockStream() { th = std::thread([this] { run(); }); }
  void run() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv.wait(lk, [&] { return stop || !q.empty(); });
      if (q.empty()) break;  // stop requested and nothing left
      auto t = std::move(q.front());
      q.pop_front();
      busy = true;
      lk.unlock();
      t();
      lk.lock();
      busy = false;
      cv.notify_all();
    }
  }
  void push(std::function<void()> f) {
    std::lock_guard<std::mutex> g(mu);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return q.empty() && !busy; });
  }
  ~MockStream() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
      cv.notify_all();
    }
    th.join();
  }
};

struct MockEvent {
  std::mutex mu;
  std::condition_variable cv;
  bool done = true;
  std::chrono::steady_clock::time_point t;
};

namespace {
std::mutex g_mu;                 // guards g_streams
std::set<MockStream *> g_streams;
MockStream *null_stream() {
  static MockStream *s = [] {
    auto *m = new MockStream();
    std::lock_guard<std::mutex> g(g_mu);
    g_streams.insert(m);
    return m;
  }();
  return s;
}
MockStream *S(hipStream_t s) { return s ? s : null_stream(); }
}  // namespace

void mock_enqueue(hipStream_t s, std::function<void()> task) {
  S(s)->push(std::move(task));
}

hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipMemGetInfo(size_t *f, size_t *t) {
  *f = size_t(16) << 30;
  *t = size_t(16) << 30;
  return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t bytes) {
  *p = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
  // like the device runtime, freeing waits for all queued work first
  std::set<MockStream *> all;
  {
    std::lock_guard<std::mutex> g(g_mu);
    all = g_streams;
  }
  for (auto *s : all) s->sync();
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes,
                          hipMemcpyKind, hipStream_t s) {
  S(s)->push([dst, src, bytes] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = new MockStream();
  std::lock_guard<std::mutex> g(g_mu);
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_streams.erase(s);
  }
  delete s;  // drains the queue, joins the executor
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  S(s)->sync();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  if (e) {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&] { return e->done; });
  }
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  {
    std::lock_guard<std::mutex> g(e->mu);
    e->done = false;
  }
  S(s)->push([e] {
    std::lock_guard<std::mutex> g(e->mu);
    e->t = std::chrono::steady_clock::now();
    e->done = true;
    e->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] { return e->done; });
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  std::chrono::steady_clock::time_point ta, tb;
  {
    std::lock_guard<std::mutex> g(a->mu);
    if (!a->done) return hipErrorInvalidValue;
    ta = a->t;
  }
  {
    std::lock_guard<std::mutex> g(b->mu);
    if (!b->done) return hipErrorInvalidValue;
    tb = b->t;
  }
  *ms = std::chrono::duration<float, std::milli>(tb - ta).count();
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "mock HIP error"; }
