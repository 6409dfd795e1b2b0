// Shared device/host helpers of the gfx950 Floquet library: complex types,
// error plumbing and the internal (non-ABI) launcher declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/floquet.h"

namespace fq {

// ---------------------------------------------------------------------------
// Complex amplitudes: interleaved {re, im}; 8-byte (c64) or 16-byte (c128)
// aligned so that one amplitude is one vector memory access.
// ---------------------------------------------------------------------------
template <typename Real>
struct alignas(2 * sizeof(Real)) cpx {
  Real x, y;
};
using c64 = cpx<float>;
using c128 = cpx<double>;

template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> mk(Real a, Real b) {
  cpx<Real> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> cadd(cpx<Real> a, cpx<Real> b) {
  return mk<Real>(a.x + b.x, a.y + b.y);
}
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> csub(cpx<Real> a, cpx<Real> b) {
  return mk<Real>(a.x - b.x, a.y - b.y);
}
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> cmul(cpx<Real> a, cpx<Real> b) {
  return mk<Real>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> cmulc(cpx<Real> a, cpx<Real> b) {
  return mk<Real>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// a + b * c (complex multiply-add)
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> cfma(cpx<Real> b, cpx<Real> c, cpx<Real> a) {
  return mk<Real>(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}
// x + i*w*y for real w (two fused multiply-adds)
template <typename Real>
__host__ __device__ __forceinline__ cpx<Real> xpiwy(cpx<Real> x, Real w, cpx<Real> y) {
  return mk<Real>(x.x - w * y.y, x.y + w * y.x);
}

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

#define FQ_HIP_CHECK(expr)                                                              \
  do {                                                                                  \
    hipError_t e__ = (expr);                                                            \
    if (e__ != hipSuccess) {                                                            \
      ::fq::set_error(std::string(#expr) + " failed: " + hipGetErrorString(e__));       \
      return FQ_EDEVICE;                                                                \
    }                                                                                   \
  } while (0)

}  // namespace fq
