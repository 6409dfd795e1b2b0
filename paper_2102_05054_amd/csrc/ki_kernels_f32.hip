// complex64 instances of the kicked-Ising kernels, and the precision casts.
#include <algorithm>

#include "ki_kernels_impl.h"

namespace fq {

template hipError_t ki_launch_pass<float>(const KiPassArgs<float>&, int, int, bool, unsigned, hipStream_t,
                                          unsigned);
template hipError_t ki_launch_pass3<float>(const KiPassArgs<float>&, int, unsigned, hipStream_t, unsigned);
template hipError_t ki_launch_pipe<float>(const KiPassArgs<float>&, int, int, bool, unsigned, unsigned, unsigned,
                                          hipStream_t);
template hipError_t ki_launch_single<float>(const KiSingleArgs<float>&, int, int, bool, bool, unsigned,
                                            hipStream_t, bool);

// ---------------------------------------------------------------------------
// Casts between complex128 and complex64 (mixed-precision filter).
// ---------------------------------------------------------------------------
__global__ void cast_c128_to_c64(const c128* __restrict__ in, c64* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = mk<float>(static_cast<float>(in[i].x), static_cast<float>(in[i].y));
}
__global__ void cast_c64_to_c128(const c64* __restrict__ in, c128* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = mk<double>(in[i].x, in[i].y);
}

hipError_t launch_cast_c128_to_c64(const void* in, void* out, size_t n, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(cast_c128_to_c64, dim3(blocks ? blocks : 1), dim3(256), 0, s,
                     static_cast<const c128*>(in), static_cast<c64*>(out), n);
  return hipGetLastError();
}
hipError_t launch_cast_c64_to_c128(const void* in, void* out, size_t n, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(cast_c64_to_c128, dim3(blocks ? blocks : 1), dim3(256), 0, s,
                     static_cast<const c64*>(in), static_cast<c128*>(out), n);
  return hipGetLastError();
}

}  // namespace fq
