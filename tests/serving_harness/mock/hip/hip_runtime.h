// Host-only stand-in for the part of the HIP runtime API that the library's
// host code (capi.cpp, serve.cpp) calls, used to run that code under
// ThreadSanitizer on a machine without a GPU.  Test infrastructure only: it
// is never part of the library build.
//
// It keeps the ordering rules the host code relies on instead of stubbing
// them away: every stream is a FIFO of tasks run by its own executor thread
// (so "device" work runs concurrently with the host and with other streams),
// hipMemcpyAsync copies when its task runs (not when it is called), events
// complete when the stream reaches them, hipStreamSynchronize waits for the
// stream's queue to drain, and device memory is host memory from malloc, so
// any access that is not ordered by these rules is a data race that
// ThreadSanitizer reports.
#pragma once

#include <cstddef>
#include <functional>

enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3
};
constexpr unsigned hipStreamNonBlocking = 1;

struct MockStream;
struct MockEvent;
typedef MockStream *hipStream_t;
typedef MockEvent *hipEvent_t;

hipError_t hipSetDevice(int);
hipError_t hipGetDeviceCount(int *);
hipError_t hipMemGetInfo(size_t *free_b, size_t *total_b);
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes,
                          hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t);

// Harness hook: run `task` on stream `s` in order (a "kernel").
void mock_enqueue(hipStream_t s, std::function<void()> task);
