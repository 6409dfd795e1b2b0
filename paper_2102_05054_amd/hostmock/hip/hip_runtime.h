// Host-only stand-in for <hip/hip_runtime.h>, used to compile the
// Krylov-Schur driver sources (krylov.cpp, block.cpp, dense.cpp) with a plain
// host compiler against the mock operator of hostmock.cpp.  "Device" memory
// is host memory, streams are ignored and every copy is synchronous.  Only
// the part of the runtime API that the driver calls is declared; the
// definitions live in hostmock.cpp (which can also cap the reported free
// memory to drive the out-of-memory paths).
#pragma once

#include <cstddef>

#define __host__
#define __device__
#define __forceinline__ inline

struct double2 {
  double x, y;
};

typedef enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 } hipError_t;

typedef struct ihipStream_t* hipStream_t;

typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

enum { hipHostMallocDefault = 0 };

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes);
const char* hipGetErrorString(hipError_t e);

template <typename T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t bytes, unsigned flags) {
  return hipHostMalloc(reinterpret_cast<void**>(p), bytes, flags);
}
