// Entanglement entropy of states (Sec. 5, Eq. (ee)).
//
// For a cut after site L_A the state is the 2^{L_A} x 2^{L-L_A} matrix M
// (row-major: site 1 is the most significant bit).  The squared singular
// values s_i^2 are the eigenvalues of the smaller Gram matrix, M M^H or
// M^H M, which is formed on the device; its eigenvalues come from a host
// Householder reduction to real symmetric tridiagonal form and implicit QL
// iterations (eigenvalues only).  S_A = -sum s_i^2 ln s_i^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "blas.h"
#include "op.h"

namespace fq {

namespace {

// Eigenvalues of a Hermitian n x n matrix (row-major, overwritten).
bool hermitian_eigenvalues(int n, std::vector<zd>& A, std::vector<double>* w) {
  auto at = [&](int i, int j) -> zd& { return A[size_t(i) * n + j]; };
  std::vector<double> diag(n, 0.0), off(n, 0.0);  // off[i] couples i-1, i
  std::vector<zd> v(n), p(n);
  for (int k = 0; k < n - 2; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(at(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const zd x0 = at(k + 1, k);
    const zd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : zd(1, 0);
    for (int i = 0; i < n; ++i) v[i] = 0;
    for (int i = k + 1; i < n; ++i) v[i] = at(i, k);
    v[k + 1] += ph * xn;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    const double tau = 2.0 / vn;
    // A <- H A H, H = I - tau v v^H (Hermitian rank-2 update on the trailing block)
    for (int i = k; i < n; ++i) {
      zd sacc = 0;
      for (int j = k + 1; j < n; ++j) sacc += at(i, j) * v[j];
      p[i] = tau * sacc;
    }
    zd K = 0;
    for (int i = k + 1; i < n; ++i) K += std::conj(v[i]) * p[i];
    K *= 0.5 * tau;
    for (int i = k; i < n; ++i) p[i] -= K * v[i];
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j) at(i, j) -= v[i] * std::conj(p[j]) + p[i] * std::conj(v[j]);
  }
  // tridiagonal with complex off-diagonals -> real by a diagonal phase similarity
  for (int i = 0; i < n; ++i) diag[i] = at(i, i).real();
  for (int i = 1; i < n; ++i) off[i] = std::abs(at(i, i - 1));
  // implicit QL (eigenvalues only)
  std::vector<double> e(n, 0.0);
  for (int i = 1; i < n; ++i) e[i - 1] = off[i];
  for (int l = 0; l < n; ++l) {
    int iter = 0, m;
    do {
      for (m = l; m < n - 1; ++m) {
        const double dd = std::fabs(diag[m]) + std::fabs(diag[m + 1]);
        if (std::fabs(e[m]) <= 1e-15 * dd) break;
      }
      if (m != l) {
        if (iter++ == 60) return false;
        double g = (diag[l + 1] - diag[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = diag[m] - diag[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
        double s = 1.0, c = 1.0, pp = 0.0;
        int i;
        for (i = m - 1; i >= l; --i) {
          double f = s * e[i], b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            diag[i + 1] -= pp;
            e[m] = 0.0;
            break;
          }
          s = f / r;
          c = g / r;
          g = diag[i + 1] - pp;
          r = (diag[i] - g) * s + 2.0 * c * b;
          pp = s * r;
          diag[i + 1] = g + pp;
          g = c * r - b;
        }
        if (r == 0.0 && i >= l) continue;
        diag[l] -= pp;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  *w = diag;
  return true;
}

}  // namespace

}  // namespace fq

using namespace fq;

extern "C" fq_status fq_host_eigvalsh(int n, double* a_host, double* w_host) {
  clear_error();
  if (n < 1 || !a_host || !w_host) {
    set_error("fq_host_eigvalsh: bad arguments");
    return FQ_EINVAL;
  }
  std::vector<zd> A(size_t(n) * n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = zd(a_host[2 * i], a_host[2 * i + 1]);
  std::vector<double> w;
  if (!hermitian_eigenvalues(n, A, &w)) {
    set_error("fq_host_eigvalsh: QL did not converge");
    return FQ_ENUMERIC;
  }
  std::sort(w.begin(), w.end());
  for (int i = 0; i < n; ++i) w_host[i] = w[i];
  return FQ_OK;
}

extern "C" fq_status entanglement_entropy(const floquet_op* op, int LA, const void* states_dev, int n_states,
                                          double* entropy_host, void* hip_stream) {
  clear_error();
  if (!op || !states_dev || !entropy_host || n_states < 0 || LA < 1 || LA >= op->L) {
    set_error("entanglement_entropy: need an op, 1 <= LA < L, states and output");
    return FQ_EINVAL;
  }
  const int L = op->L;
  const int LB = L - LA;
  const int nl = std::min(LA, LB);
  if (nl > 11) {
    set_error("entanglement_entropy: the smaller side of the cut must have <= 11 sites");
    return FQ_EINVAL;
  }
  const int n = 1 << nl;
  const size_t R = size_t(1) << LA, C = size_t(1) << LB;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  c128* G = nullptr;
  FQ_HIP_CHECK(hipMalloc(&G, sizeof(c128) * size_t(n) * n));
  std::vector<c128> hG(size_t(n) * n);
  std::vector<zd> A(size_t(n) * n);
  fq_status st = FQ_OK;
  for (int q = 0; q < n_states && st == FQ_OK; ++q) {
    const c128* X = static_cast<const c128*>(states_dev) + size_t(q) * op->dim();
    hipError_t e = LA <= LB ? launch_gram(X, C, 1, false, n, C, G, s)   // M M^H
                            : launch_gram(X, 1, C, true, n, R, G, s);   // M^H M
    if (e == hipSuccess) e = hipMemcpyAsync(hG.data(), G, hG.size() * sizeof(c128), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error(std::string("entanglement_entropy: ") + hipGetErrorString(e));
      st = FQ_EDEVICE;
      break;
    }
    for (size_t i = 0; i < A.size(); ++i) A[i] = zd(hG[i].x, hG[i].y);
    std::vector<double> w;
    if (!hermitian_eigenvalues(n, A, &w)) {
      set_error("entanglement_entropy: tridiagonal QL did not converge");
      st = FQ_ENUMERIC;
      break;
    }
    double tr = 0.0;
    for (double x : w) tr += std::max(x, 0.0);
    double S = 0.0;
    for (double x : w) {
      const double pr = x / (tr > 0 ? tr : 1.0);
      if (pr > 1e-300) S -= pr * std::log(pr);
    }
    entropy_host[q] = S;
  }
  (void)hipFree(G);
  return st;
}
