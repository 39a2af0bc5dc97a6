// Host-only stand-in for the few HIP runtime declarations that the library's
// host headers and its request server (serve.cpp) use, so that the server's
// queueing, admission, batching and slot threads can be built with g++ under
// ThreadSanitizer / AddressSanitizer and run without a GPU
// (tests/native/serve_check.cpp, tests/test_native_sanitizers.py).  "Device"
// memory is host memory and every copy is synchronous; nothing here is used by
// the library build itself.
#pragma once
#include <cstddef>

typedef enum hipError_t { hipSuccess = 0, hipErrorOutOfMemory = 2 } hipError_t;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3
} hipMemcpyKind;

struct ihipStream_t;
struct ihipEvent_t;
struct hipGraphExec;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef hipGraphExec* hipGraphExec_t;

enum { hipStreamNonBlocking = 1, hipHostMallocDefault = 0 };

hipError_t hipSetDevice(int device);
hipError_t hipGetLastError();
hipError_t hipMalloc(void** ptr, size_t bytes);
hipError_t hipFree(void* ptr);
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* ptr);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t stream);
hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
