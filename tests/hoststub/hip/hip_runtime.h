// Host-only stand-in for the subset of the HIP runtime API the library's host
// runtime calls, for building that runtime as plain C++ under AddressSanitizer /
// UndefinedBehaviorSanitizer on a machine without a GPU (tests/host_check.cpp).
// "Device" memory is host memory, copies are synchronous memcpy, streams and
// events are tokens; the kernels are replaced by the launchers host_check.cpp
// registers.  Test infrastructure only: never part of the library.
#pragma once
#include <cstddef>
#include <cstdlib>
#include <cstring>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotReady = 600 };
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
struct ihipStream_t { int id; };
struct ihipEvent_t { int id; };
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
constexpr unsigned hipHostMallocDefault = 0;
constexpr unsigned hipStreamNonBlocking = 1;
constexpr unsigned hipEventDisableTiming = 2;

namespace hipstub {
// Live allocations (device and pinned), events and streams: a test checks that a
// context's teardown returns every one of them.
inline long &live_allocs() { static long n = 0; return n; }
inline long &live_streams() { static long n = 0; return n; }
inline size_t &alloc_limit() { static size_t n = (size_t)1 << 34; return n; }   // larger requests fail
}  // namespace hipstub

inline const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stub error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }

inline hipError_t hipMalloc(void **p, size_t n) {
    if (n > hipstub::alloc_limit()) { *p = nullptr; return hipErrorOutOfMemory; }
    *p = std::calloc(1, n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    ++hipstub::live_allocs();
    return hipSuccess;
}
inline hipError_t hipFree(void *p) {
    if (p) { std::free(p); --hipstub::live_allocs(); }
    return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    if (n) std::memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(d, s, n, k);
}
inline hipError_t hipMemset(void *d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { return hipMemset(d, v, n); }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new ihipStream_t{0};
    ++hipstub::live_streams();
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; --hipstub::live_streams(); return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new ihipEvent_t{0}; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
// Work is done when it is enqueued; a query still reports "not ready" two times in
// three, so that callers' waiting paths run.
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) {
    static unsigned n = 0;
    return (n++ % 3 == 2) ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
