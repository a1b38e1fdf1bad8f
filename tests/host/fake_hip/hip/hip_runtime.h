// A host-only stand-in for the HIP runtime, just large enough to compile the fit
// server (sb_server.cpp) for CPU tests under the thread and address sanitizers.
// Streams execute every operation immediately in the calling thread; memory is
// host memory.  Not a HIP implementation: only what the server calls.
#pragma once

#include <cstddef>
#include <cstdlib>
#include <cstring>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidDevice = 101 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };

struct FakeStream {};
struct FakeEvent {};
typedef FakeStream* hipStream_t;
typedef FakeEvent* hipEvent_t;

struct float2 {
  float x, y;
};
inline float2 make_float2(float x, float y) { return float2{x, y}; }

inline const char* hipGetErrorString(hipError_t) { return "fake hip error"; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new FakeStream;
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new FakeEvent;
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) {
  *p = (T*)std::calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned) {
  *p = (T*)std::calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
