// Host-only stand-in for the few HIP runtime calls the serving loop makes,
// so that jefi_server.cpp can be built with the host compiler and run under
// ThreadSanitizer on a machine without a GPU.  Streams are worker threads
// that run their operations in order; events complete when their stream
// reaches them.  Test infrastructure only.
#pragma once

#include <cstddef>
#include <cstdint>

typedef enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorNotReady = 600,
  hipErrorUnknown = 999
} hipError_t;

typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3
} hipMemcpyKind;

struct MockStream;
struct MockEvent;
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;

#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

struct int2 {
  int x, y;
};

hipError_t hipSetDevice(int device);
hipError_t hipGetDevice(int* device);
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetLastError(void);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
