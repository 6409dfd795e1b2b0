// apply_filter_many_noalloc: the block filter of apply_filter_many for
// kicked-Ising ops without any device allocation.
//
// apply_filter_many keeps per-op device state that it allocates on demand:
// the launch descriptors of the vectors, the phase tables of each target
// rotation and (complex128, four vectors) the kicked copies of psi of the
// folded passes.  This variant puts the descriptors and the phase tables in a
// fixed file-scope device array instead, fills both with two small kernels on
// the caller's stream, and runs the plain (unfolded) batched passes with the
// tile shape the autotuner cached for this case, or the default shape, without
// timing anything.  One array per GPU holds the last call's contents; calls
// that overlap on one GPU (several streams or host threads) race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "ki_batched.h"
#include "op.h"

namespace fq {
namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;  // 4 MiB per GPU
constexpr int kMaxVec = 64;
constexpr int kMaxDevices = 64;
constexpr size_t kDescBytes = 256 * ((kMaxVec * sizeof(KiDesc<double>) + kMaxVec * sizeof(int) + 255) / 256);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// device address of `scratch` on device dev (the current device), resolved
// once per device
fq_status scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress of the filter scratch failed: ") + hipGetErrorString(e));
      return FQ_EDEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return FQ_OK;
}

// The kicked-Ising diagonal as two tables (see ki_kernels_impl.h): entry s of
// the low table is pre * e^{-i E_lo(s)} over the low m bits, entry idx of the
// high table e^{-i E_hi} over the high bits, with the two low boundary bits
// b_0 = bit 1 of idx and b_{m-1} = bit 0 of idx for the bonds that cross the
// split.  pre holds the per-U scale of the factored kicks and e^{-i phi}.
struct TableArgs {
  int L, m, nb;
  int bu[32], bv[32];
  double bJ[32];
  double hbit[32];  // field on bit b (site L - b)
  double pre_re, pre_im;
};

template <typename Real>
__global__ void __launch_bounds__(256) tables_kernel(TableArgs a, cpx<Real>* tlo, cpx<Real>* thi) {
  const uint32_t nlo = 1u << a.m;
  const uint32_t nhi = 4u << (a.L - a.m);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlo + nhi) return;
  double E = 0.0;
  double re = 1.0, im = 0.0;
  if (i < nlo) {
    for (int q = 0; q < a.nb; ++q)
      if (a.bu[q] < a.m && a.bv[q] < a.m)
        E += a.bJ[q] * (1 - 2 * int((i >> a.bu[q]) & 1u)) * (1 - 2 * int((i >> a.bv[q]) & 1u));
    for (int b = 0; b < a.m; ++b) E += a.hbit[b] * (1 - 2 * int((i >> b) & 1u));
    re = a.pre_re;
    im = a.pre_im;
  } else {
    const uint32_t idx = i - nlo;
    const uint32_t shi = idx >> 2;
    const int b0 = int((idx >> 1) & 1u), bm1 = int(idx & 1u);
    auto z = [&](int bit) -> int {
      if (bit >= a.m) return 1 - 2 * int((shi >> (bit - a.m)) & 1u);
      if (bit == 0) return 1 - 2 * b0;
      if (bit == a.m - 1) return 1 - 2 * bm1;
      return 0;
    };
    for (int q = 0; q < a.nb; ++q)
      if (!(a.bu[q] < a.m && a.bv[q] < a.m)) E += a.bJ[q] * z(a.bu[q]) * z(a.bv[q]);
    for (int b = a.m; b < a.L; ++b) E += a.hbit[b] * z(b);
  }
  double sn, cs;
  sincos(-E, &sn, &cs);
  const double vr = re * cs - im * sn, vi = re * sn + im * cs;
  cpx<Real> v;
  v.x = static_cast<Real>(vr);
  v.y = static_cast<Real>(vi);
  if (i < nlo)
    tlo[i] = v;
  else
    thi[i - nlo] = v;
}

template <typename Real>
__global__ void __launch_bounds__(64) desc_kernel(KiDesc<Real>* desc, int* list, const cpx<Real>* psi,
                                                  cpx<Real>* out, size_t d, const cpx<Real>* tlo,
                                                  const cpx<Real>* thi, double w, int n) {
  const int j = threadIdx.x;
  if (j >= n) return;
  KiDesc<Real> q;
  q.psi = psi + size_t(j) * d;
  q.x = out + size_t(j) * d;
  q.tlo = tlo;
  q.thi = thi;
  q.w = w;
  q.pad = 0.0;
  q.chi[0] = nullptr;
  q.chi[1] = nullptr;
  desc[j] = q;
  list[j] = j;
}

template <typename Real>
fq_status filter_noalloc(floquet_op* op, int k, double phi, int n, const void* psi, void* out, hipStream_t s) {
  int dev = 0;
  FQ_HIP_CHECK(hipGetDevice(&dev));
  if (dev != op->device || dev < 0 || dev >= kMaxDevices) {
    set_error("apply_filter_many_noalloc: the op's device must be the current device");
    return FQ_EINVAL;
  }
  unsigned char* base = nullptr;
  fq_status st = scratch_address(dev, &base);
  if (st != FQ_OK) return st;
  const int L = op->L, m = op->m;
  const size_t nlo = size_t(1) << m, nhi = size_t(4) << (L - m);
  const size_t need = kDescBytes + (nlo + nhi) * sizeof(cpx<Real>);
  if (need > kScratchBytes) {
    set_error("apply_filter_many_noalloc: the phase tables need " + std::to_string(need) + " bytes, more than the " +
              std::to_string(kScratchBytes) + "-byte scratch");
    return FQ_EINVAL;
  }
  KiDesc<Real>* desc = reinterpret_cast<KiDesc<Real>*>(base);
  int* list = reinterpret_cast<int*>(base + kMaxVec * sizeof(KiDesc<Real>));
  cpx<Real>* tlo = reinterpret_cast<cpx<Real>*>(base + kDescBytes);
  cpx<Real>* thi = tlo + nlo;

  TableArgs ta{};
  ta.L = L;
  ta.m = m;
  for (int i = 1; i <= L - 1; ++i) {  // bond (i, i+1): bits L-i, L-i-1
    ta.bu[ta.nb] = L - i;
    ta.bv[ta.nb] = L - i - 1;
    ta.bJ[ta.nb] = op->J[i - 1];
    ++ta.nb;
  }
  if (op->periodic) {  // bond (L, 1): bits 0, L-1
    ta.bu[ta.nb] = 0;
    ta.bv[ta.nb] = L - 1;
    ta.bJ[ta.nb] = op->J[L - 1];
    ++ta.nb;
  }
  for (int i = 1; i <= L; ++i) ta.hbit[L - i] = op->h[i - 1];
  const zd pre = std::pow(op->site_scale, L) * std::polar(1.0, -phi);
  ta.pre_re = pre.real();
  ta.pre_im = pre.imag();
  const unsigned nt = static_cast<unsigned>(nlo + nhi);
  hipLaunchKernelGGL(tables_kernel<Real>, dim3((nt + 255) / 256), dim3(256), 0, s, ta, tlo, thi);
  FQ_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(desc_kernel<Real>, dim3(1), dim3(64), 0, s, desc, list, static_cast<const cpx<Real>*>(psi),
                     static_cast<cpx<Real>*>(out), op->dim(), static_cast<const cpx<Real>*>(tlo),
                     static_cast<const cpx<Real>*>(thi), op->w, n);
  FQ_HIP_CHECK(hipGetLastError());
  KiBatchShape sh;
  st = ki_batch_shape_untimed<Real>(L, op->sw, k, static_cast<unsigned>(n), &sh);
  if (st != FQ_OK) return st;
  return ki_batch_filter<Real>(sh, k, desc, list, static_cast<unsigned>(n), s);
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" fq_status apply_filter_many_noalloc(floquet_op* op, int k, double phi, fq_dtype dtype, int n_vec,
                                               const void* psi_dev, void* out_dev, void* hip_stream) {
  clear_error();
  if (!op || !psi_dev || !out_dev) {
    set_error("apply_filter_many_noalloc: op and device pointers must not be NULL");
    return FQ_EINVAL;
  }
  if (op->model != FQ_KICKED_ISING || op->L < 4) {
    set_error("apply_filter_many_noalloc: kicked-Ising ops with L >= 4 only");
    return FQ_EINVAL;
  }
  if (k < 0 || !std::isfinite(phi) || (dtype != FQ_C64 && dtype != FQ_C128) || n_vec < 1 || n_vec > kMaxVec) {
    set_error("apply_filter_many_noalloc: need k >= 0, finite phi, a valid dtype and 1 <= n_vec <= 64");
    return FQ_EINVAL;
  }
  const size_t bytes = op->dim() * size_t(n_vec) * (dtype == FQ_C64 ? sizeof(c64) : sizeof(c128));
  const char* a = static_cast<const char*>(psi_dev);
  const char* b = static_cast<const char*>(out_dev);
  if (a < b + bytes && b < a + bytes) {
    set_error("apply_filter_many_noalloc: out must not overlap psi");
    return FQ_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (k == 0) {
    FQ_HIP_CHECK(hipMemcpyAsync(out_dev, psi_dev, bytes, hipMemcpyDeviceToDevice, s));
    return FQ_OK;
  }
  return dtype == FQ_C64 ? filter_noalloc<float>(op, k, phi, n_vec, psi_dev, out_dev, s)
                         : filter_noalloc<double>(op, k, phi, n_vec, psi_dev, out_dev, s);
}
