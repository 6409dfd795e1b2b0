// Host mock of the device layer under the Krylov-Schur driver.
//
// Test infrastructure: the driver sources (krylov.cpp, block.cpp, dense.cpp)
// are compiled unchanged with a host compiler against this file, so that the
// restart logic, the convergence and stall rules, the mixed-precision
// hand-over, non-convergence, NaN detection, the out-of-memory checks and the
// invariant-subspace path run on the CPU without a GPU (and under the address
// and undefined-behaviour sanitizers).  The operator is a diagonal unitary
// U = diag(e^{i theta_s}) with caller-given phases, so the exact eigenpairs
// are known; the "complex64" filter does its arithmetic in single precision.
// Nothing here is linked into libfloquet.so.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../csrc/blas.h"
#include "../csrc/ki_batched.h"
#include "../csrc/krylov.h"
#include "../csrc/op.h"

// ---------------------------------------------------------------------------
// Runtime stand-in: device memory is host memory.
// ---------------------------------------------------------------------------
namespace {
size_t g_free_bytes = size_t(64) << 30;  // reported free device memory
long long g_nan_at = -1;                 // filter application that returns NaN (-1: never)
long long g_filter_apps = 0;             // filter applications so far
thread_local std::string g_err;
}  // namespace

hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes) {
  *free_bytes = g_free_bytes;
  *total_bytes = g_free_bytes;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "mock error"; }

namespace fq {

void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

namespace {
using zf = std::complex<float>;

inline zd Z(const c128& a) { return zd(a.x, a.y); }
inline c128 C(const zd& a) { return mk<double>(a.real(), a.imag()); }

// diagonal of U, stored in op->gates
const std::vector<zd>& diag(const floquet_op* op) { return op->gates; }

// out = g(U) psi (geometric sum with rotation phi, or the polynomial coefs)
template <typename R, typename IO>
void filter_one(const floquet_op* op, int k, double phi, const zd* coefs, const IO* in, IO* out) {
  using Cx = std::complex<R>;
  const size_t d = op->dim();
  const auto& u = diag(op);
  const Cx rot(static_cast<R>(std::cos(-phi)), static_cast<R>(std::sin(-phi)));
  for (size_t s = 0; s < d; ++s) {
    const Cx us(static_cast<R>(u[s].real()), static_cast<R>(u[s].imag()));
    const Cx x(static_cast<R>(in[s].x), static_cast<R>(in[s].y));
    Cx w;
    if (coefs) {
      w = Cx(static_cast<R>(coefs[k].real()), static_cast<R>(coefs[k].imag())) * x;
      for (int m = k - 1; m >= 0; --m)
        w = Cx(static_cast<R>(coefs[m].real()), static_cast<R>(coefs[m].imag())) * x + us * w;
    } else {
      w = x;
      for (int m = 0; m < k; ++m) w = x + rot * (us * w);
    }
    out[s].x = static_cast<decltype(out[s].x)>(w.real());
    out[s].y = static_cast<decltype(out[s].y)>(w.imag());
  }
  ++g_filter_apps;
  if (g_nan_at >= 0 && g_filter_apps == g_nan_at) out[0].x = std::numeric_limits<decltype(out[0].x)>::quiet_NaN();
}

}  // namespace

fq_status apply_U_internal(floquet_op* op, fq_dtype dt, const void* psi, void* out, hipStream_t) {
  const size_t d = op->dim();
  const auto& u = diag(op);
  if (dt == FQ_C128) {
    const c128* x = static_cast<const c128*>(psi);
    c128* y = static_cast<c128*>(out);
    for (size_t s = 0; s < d; ++s) y[s] = C(u[s] * Z(x[s]));
  } else {
    const c64* x = static_cast<const c64*>(psi);
    c64* y = static_cast<c64*>(out);
    for (size_t s = 0; s < d; ++s) {
      const zf v = zf(float(u[s].real()), float(u[s].imag())) * zf(x[s].x, x[s].y);
      y[s] = mk<float>(v.real(), v.imag());
    }
  }
  return FQ_OK;
}

fq_status filter_internal(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi,
                          void* out, hipStream_t) {
  if (dt == FQ_C128)
    filter_one<double>(op, k, phi, coefs, static_cast<const c128*>(psi), static_cast<c128*>(out));
  else
    filter_one<float>(op, k, phi, coefs, static_cast<const c64*>(psi), static_cast<c64*>(out));
  return FQ_OK;
}

fq_status filter_mixed(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi64,
                       void* out64, hipStream_t) {
  const c128* in = static_cast<const c128*>(psi64);
  c128* out = static_cast<c128*>(out64);
  if (dt == FQ_C128)
    filter_one<double>(op, k, phi, coefs, in, out);
  else
    filter_one<float>(op, k, phi, coefs, in, out);  // single-precision arithmetic, FP64 in and out
  return FQ_OK;
}

fq_status bw_filter(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi, void* out,
                    hipStream_t s, int nvec) {
  const size_t bytes = op->dim() * (dt == FQ_C64 ? sizeof(c64) : sizeof(c128));
  for (int j = 0; j < nvec; ++j) {
    const fq_status st = filter_internal(op, k, phi, coefs, dt, static_cast<const char*>(psi) + j * bytes,
                                         static_cast<char*>(out) + j * bytes, s);
    if (st != FQ_OK) return st;
  }
  return FQ_OK;
}

fq_status get_tables(floquet_op*, double, const PhaseTables**) {
  set_error("host mock: no kicked-Ising tables");
  return FQ_EINVAL;
}

fq_status ki_set_policy(int policy) { return (policy >= 0 && policy <= 2) ? FQ_OK : FQ_EINVAL; }

template <typename Real>
fq_status ki_batch_tune(int, bool, int, const KiDesc<Real>*, const int*, unsigned, hipStream_t, KiBatchShape*,
                        double*, const KiDesc<Real>*, const KiDesc<Real>*) {
  set_error("host mock: no kicked-Ising kernels");
  return FQ_EINVAL;
}
template <typename Real>
fq_status ki_batch_filter(const KiBatchShape&, int, const KiDesc<Real>*, const int*, unsigned, hipStream_t,
                          const KiDesc<Real>*, const KiDesc<Real>*) {
  set_error("host mock: no kicked-Ising kernels");
  return FQ_EINVAL;
}
template fq_status ki_batch_tune<float>(int, bool, int, const KiDesc<float>*, const int*, unsigned, hipStream_t,
                                        KiBatchShape*, double*, const KiDesc<float>*, const KiDesc<float>*);
template fq_status ki_batch_tune<double>(int, bool, int, const KiDesc<double>*, const int*, unsigned, hipStream_t,
                                         KiBatchShape*, double*, const KiDesc<double>*, const KiDesc<double>*);
template fq_status ki_batch_filter<float>(const KiBatchShape&, int, const KiDesc<float>*, const int*, unsigned,
                                          hipStream_t, const KiDesc<float>*, const KiDesc<float>*);
template fq_status ki_batch_filter<double>(const KiBatchShape&, int, const KiDesc<double>*, const int*, unsigned,
                                           hipStream_t, const KiDesc<double>*, const KiDesc<double>*);

fq_status arnoldi_batched_solve(floquet_op* const*, int, const double*, int, int, const fq_arnoldi_opts*, const int*,
                                double*, void* const*, double*, fq_arnoldi_stats*, hipStream_t) {
  set_error("host mock: the lockstep batched solver is not part of the mock");
  return FQ_EINVAL;
}

// --- FP64 vector kernels on the host (one "row block": the whole vector) ---

hipError_t launch_dots(const c128* V, size_t ldv, int ncols, const c128* w, size_t d, c128* partial, int ldp,
                       hipStream_t) {
  const unsigned nblk = row_blocks(d);
  for (unsigned b = 0; b < nblk; ++b)
    for (int i = 0; i < ncols; ++i) partial[size_t(b) * ldp + i] = mk<double>(0, 0);
  for (int i = 0; i < ncols; ++i) {
    zd acc = 0;
    for (size_t r = 0; r < d; ++r) acc += std::conj(Z(V[size_t(i) * ldv + r])) * Z(w[r]);
    partial[i] = C(acc);
  }
  return hipSuccess;
}

hipError_t launch_reduce_cols(const c128* partial, int ldp, unsigned nblk, int ncols, c128* out, hipStream_t) {
  for (int i = 0; i < ncols; ++i) {
    zd acc = 0;
    for (unsigned b = 0; b < nblk; ++b) acc += Z(partial[size_t(b) * ldp + i]);
    out[i] = C(acc);
  }
  return hipSuccess;
}

hipError_t launch_update(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d, hipStream_t) {
  for (size_t r = 0; r < d; ++r) {
    zd acc = Z(w[r]);
    for (int i = 0; i < ncols; ++i) acc -= Z(V[size_t(i) * ldv + r]) * Z(h[i]);
    w[r] = C(acc);
  }
  return hipSuccess;
}

hipError_t launch_update_dots(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d, c128* partial,
                              int ldp, hipStream_t s) {
  launch_update(V, ldv, ncols, h, w, d, s);
  return launch_dots(V, ldv, ncols, w, d, partial, ldp, s);
}

hipError_t launch_norm2(const c128* w, size_t d, c128* partial, hipStream_t) {
  const unsigned nblk = row_blocks(d);
  double acc = 0.0;
  for (size_t r = 0; r < d; ++r) acc += std::norm(Z(w[r]));
  for (unsigned b = 0; b < nblk; ++b) partial[b] = mk<double>(b == 0 ? acc : 0.0, 0.0);
  return hipSuccess;
}

hipError_t launch_update_norm2(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d,
                               c128* partial, hipStream_t s) {
  launch_update(V, ldv, ncols, h, w, d, s);
  return launch_norm2(w, d, partial, s);
}

hipError_t launch_reduce_norm(const c128* partial, unsigned nblk, double* nrm, hipStream_t) {
  double acc = 0.0;
  for (unsigned b = 0; b < nblk; ++b) acc += partial[b].x;
  nrm[0] = std::sqrt(acc);
  nrm[1] = nrm[0] > 0.0 ? 1.0 / nrm[0] : 0.0;
  return hipSuccess;
}

hipError_t launch_scale_dev(const c128* in, const double* scale, c128* out, size_t d, hipStream_t) {
  const double a = scale[0];
  for (size_t r = 0; r < d; ++r) out[r] = mk<double>(in[r].x * a, in[r].y * a);
  return hipSuccess;
}

hipError_t launch_scale_c128(const c128* in, double are, double aim, c128* out, size_t d, hipStream_t) {
  for (size_t r = 0; r < d; ++r) out[r] = C(zd(are, aim) * Z(in[r]));
  return hipSuccess;
}

hipError_t launch_scale_c64(const c64* in, double are, double aim, c64* out, size_t d, hipStream_t) {
  for (size_t r = 0; r < d; ++r) {
    const zf v = zf(float(are), float(aim)) * zf(in[r].x, in[r].y);
    out[r] = mk<float>(v.real(), v.imag());
  }
  return hipSuccess;
}

hipError_t launch_axpy_dev(const c128* a, const c128* x, c128* y, size_t d, hipStream_t) {
  const zd av = Z(a[0]);
  for (size_t r = 0; r < d; ++r) y[r] = C(Z(y[r]) - av * Z(x[r]));
  return hipSuccess;
}

hipError_t launch_basis_gemm(const c128* V, size_t ldv, int m, const c128* Q, int p, c128* Y, size_t ldy, size_t d,
                             hipStream_t) {
  std::vector<zd> out(size_t(p) * d, zd(0, 0));  // Y may alias V
  for (int c = 0; c < p; ++c)
    for (int i = 0; i < m; ++i) {
      const zd q = Z(Q[size_t(i) * p + c]);
      for (size_t r = 0; r < d; ++r) out[size_t(c) * d + r] += Z(V[size_t(i) * ldv + r]) * q;
    }
  for (int c = 0; c < p; ++c)
    for (size_t r = 0; r < d; ++r) Y[size_t(c) * ldy + r] = C(out[size_t(c) * d + r]);
  return hipSuccess;
}

hipError_t launch_random(c128* v, size_t d, unsigned long long seed, hipStream_t) {
  uint64_t x = seed * 2862933555777941757ull + 3037000493ull;
  auto next = [&x]() {  // 64-bit xorshift (Marsaglia 2003)
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return double(x >> 11) * (1.0 / 9007199254740992.0);
  };
  for (size_t r = 0; r < d; ++r) {
    const double a = next(), b = next();
    v[r] = mk<double>(2.0 * a - 1.0, 2.0 * b - 1.0);
  }
  return hipSuccess;
}

hipError_t launch_bdots(const c128* V, size_t ldv, int ncols, const c128* W, size_t ldw, int b, size_t d,
                        c128* partial, int ldp, hipStream_t) {
  const unsigned nblk = row_blocks(d);
  for (unsigned blk = 0; blk < nblk; ++blk)
    for (int e = 0; e < ncols * b; ++e) partial[size_t(blk) * ldp + e] = mk<double>(0, 0);
  for (int i = 0; i < ncols; ++i)
    for (int c = 0; c < b; ++c) {
      zd acc = 0;
      for (size_t r = 0; r < d; ++r) acc += std::conj(Z(V[size_t(i) * ldv + r])) * Z(W[size_t(c) * ldw + r]);
      partial[size_t(i) * b + c] = C(acc);
    }
  return hipSuccess;
}

hipError_t launch_bupdate(const c128* V, size_t ldv, int ncols, const c128* H, c128* W, size_t ldw, int b, size_t d,
                          hipStream_t) {
  for (int c = 0; c < b; ++c)
    for (size_t r = 0; r < d; ++r) {
      zd acc = Z(W[size_t(c) * ldw + r]);
      for (int i = 0; i < ncols; ++i) acc -= Z(V[size_t(i) * ldv + r]) * Z(H[size_t(i) * b + c]);
      W[size_t(c) * ldw + r] = C(acc);
    }
  return hipSuccess;
}

hipError_t launch_cast_c128_to_c64(const void* in, void* out, size_t n, hipStream_t) {
  const c128* a = static_cast<const c128*>(in);
  c64* b = static_cast<c64*>(out);
  for (size_t i = 0; i < n; ++i) b[i] = mk<float>(static_cast<float>(a[i].x), static_cast<float>(a[i].y));
  return hipSuccess;
}

hipError_t launch_cast_c64_to_c128(const void* in, void* out, size_t n, hipStream_t) {
  const c64* a = static_cast<const c64*>(in);
  c128* b = static_cast<c128*>(out);
  for (size_t i = 0; i < n; ++i) b[i] = mk<double>(a[i].x, a[i].y);
  return hipSuccess;
}

}  // namespace fq

using namespace fq;

extern "C" {

const char* floquet_last_error(void) { return g_err.c_str(); }

// A mock op: U = diag(exp(i phases[s])), d = 2^L (2 <= L <= 16).
fq_status fq_mock_create(int L, const double* phases, floquet_op** out) {
  if (L < 2 || L > 16 || !phases || !out) return FQ_EINVAL;
  floquet_op* op = new floquet_op();
  op->model = FQ_CIRCUIT;  // not kicked Ising: block filters go through bw_filter
  op->L = L;
  op->periodic = 0;
  const size_t d = size_t(1) << L;
  op->gates.resize(d);
  for (size_t s = 0; s < d; ++s) op->gates[s] = std::polar(1.0, phases[s]);
  *out = op;
  return FQ_OK;
}

fq_status fq_mock_destroy(floquet_op* op) {
  if (!op) return FQ_OK;
  std::free(op->V);
  std::free(op->work);
  std::free(op->work2);
  std::free(op->dev_small);
  std::free(op->host_small);
  std::free(op->many_mem);
  std::free(op->chi_mem);
  delete op;
  return FQ_OK;
}

// Free device memory the mock reports (drives the out-of-memory checks).
void fq_mock_set_free_bytes(unsigned long long bytes) { g_free_bytes = static_cast<size_t>(bytes); }

// The filter application (1-based, counted from the last reset) whose output
// gets a NaN; -1 disables.  Also resets the application counter.
void fq_mock_set_nan_at(long long app) {
  g_nan_at = app;
  g_filter_apps = 0;
}

long long fq_mock_filter_apps(void) { return g_filter_apps; }

}  // extern "C"
