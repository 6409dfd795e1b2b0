// Block Krylov-Schur on the filter (arnoldi_eigs with opts.block = b > 1).
//
// The Krylov space of Sec. 4 is grown b vectors at a time: each step filters
// a block of b basis vectors (for the kicked Ising one launch per Horner pass
// for the whole block, through the batched pass kernels), orthogonalises the
// b results against the basis with block classical Gram-Schmidt applied twice
// (the basis is read once for all b vectors) and orthonormalises them with two
// rounds of Cholesky QR.  The decomposition
//     g(U) V_m = V_m S + V_{m..m+b} B,   B: b x m,
// is restarted like the single-vector one: the Schur form of S on the host,
// the p kept Schur vectors V_m Z_p on the device, the residual block moved
// behind them and B Z_p as the new coupling block.  A Ritz pair (theta, V Z y)
// has residual norm ||B Z y|| in the filter.  The mixed-precision scheme, the
// convergence checks inside a cycle, the Ritz vectors and the FP64 residuals
// follow the single-vector solver; the FP64 refinement starts from b random
// combinations of the complex64 Ritz vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>
#include <vector>

#include "blas.h"
#include "dense.h"
#include "ki_batched.h"
#include "krylov.h"
#include "op.h"

namespace fq {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("FQ_VERBOSE");
    return e && e[0] && e[0] != '0';
  }();
  return v;
}

#define FQ_TRY(expr)                \
  do {                              \
    fq_status st__ = (expr);        \
    if (st__ != FQ_OK) return st__; \
  } while (0)

// Cholesky G = R^H R of a b x b Hermitian matrix (column-major).  false when
// a pivot falls below rel_floor * max diag(G): the block is too ill
// conditioned for Cholesky QR.
bool cholesky_upper(const std::vector<zd>& G, int b, std::vector<zd>* R, double rel_floor) {
  R->assign(size_t(b) * b, zd(0, 0));
  auto g = [&](int i, int j) { return G[size_t(j) * b + i]; };
  auto r = [&](int i, int j) -> zd& { return (*R)[size_t(j) * b + i]; };
  double gmax = 0.0;
  for (int i = 0; i < b; ++i) gmax = std::max(gmax, g(i, i).real());
  if (!(gmax > 0.0) || !std::isfinite(gmax)) return false;
  for (int j = 0; j < b; ++j) {
    double s = g(j, j).real();
    for (int k = 0; k < j; ++k) s -= std::norm(r(k, j));
    if (!(s > rel_floor * gmax)) return false;
    const double rjj = std::sqrt(s);
    r(j, j) = rjj;
    for (int i = j + 1; i < b; ++i) {
      zd t = g(j, i);
      for (int k = 0; k < j; ++k) t -= std::conj(r(k, j)) * r(k, i);
      r(j, i) = t / rjj;
    }
  }
  return true;
}

// inverse of an upper-triangular b x b matrix (column-major)
std::vector<zd> inv_upper(const std::vector<zd>& R, int b) {
  std::vector<zd> X(size_t(b) * b, zd(0, 0));
  for (int j = 0; j < b; ++j) {
    X[size_t(j) * b + j] = 1.0 / R[size_t(j) * b + j];
    for (int i = j - 1; i >= 0; --i) {
      zd s = 0;
      for (int k = i + 1; k <= j; ++k) s += R[size_t(k) * b + i] * X[size_t(j) * b + k];
      X[size_t(j) * b + i] = -s / R[size_t(i) * b + i];
    }
  }
  return X;
}

// C = A * B for b x b column-major matrices
std::vector<zd> matmul(const std::vector<zd>& A, const std::vector<zd>& B, int b) {
  std::vector<zd> C(size_t(b) * b, zd(0, 0));
  for (int j = 0; j < b; ++j)
    for (int l = 0; l < b; ++l) {
      const zd blj = B[size_t(j) * b + l];
      for (int i = 0; i < b; ++i) C[size_t(j) * b + i] += A[size_t(l) * b + i] * blj;
    }
  return C;
}

struct Ritz {
  std::vector<zd> omega;
  std::vector<double> resid;
};

struct BlockSolver {
  floquet_op* op = nullptr;
  int nev = 0, m = 0, b = 0, k = 0, p_keep = 0, check_every = 0;
  double phi = 0.0;
  std::vector<zd> coefs;
  hipStream_t s = nullptr;
  fq_arnoldi_stats* st = nullptr;
  size_t d = 0;
  unsigned nblk = 0;
  int ldp = 0;
  std::vector<void*> mem;  // device allocations owned here
  c128* host = nullptr;    // pinned staging, (m + b) * b * 2 complex
  c128 *V = nullptr, *uy = nullptr, *ritz = nullptr, *partial = nullptr, *hdev = nullptr, *qbuf = nullptr;
  c64 *psi32 = nullptr, *x32 = nullptr;  // complex64 block (batched kicked-Ising filter)
  double* small = nullptr;
  bool batched_filter = false;
  double t_filter = 0, t_orth = 0, t_restart = 0;

  ~BlockSolver() {
    for (void* q : mem) (void)hipFree(q);
    if (host) (void)hipHostFree(host);
  }

  template <typename T>
  fq_status alloc(T** out, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
      set_error("hipMalloc of the block Krylov workspace failed");
      return FQ_ENOMEM;
    }
    mem.push_back(q);
    *out = static_cast<T*>(q);
    return FQ_OK;
  }

  fq_status setup(void* evecs_dev) {
    d = op->dim();
    nblk = row_blocks(d);
    ldp = (m + b) * b;
    size_t freeb = 0, totalb = 0;
    FQ_HIP_CHECK(hipMemGetInfo(&freeb, &totalb));
    const size_t need = d * sizeof(c128) * size_t(m + b + 1 + (evecs_dev ? 0 : nev)) + d * sizeof(c64) * 2 * b;
    if (need + (size_t(1) << 28) > freeb) {
      set_error("block Krylov workspace of " + std::to_string(need >> 20) + " MiB does not fit in free device memory");
      return FQ_ENOMEM;
    }
    FQ_TRY(alloc(&V, d * size_t(m + b)));
    FQ_TRY(alloc(&uy, d));
    if (evecs_dev)
      ritz = static_cast<c128*>(evecs_dev);
    else
      FQ_TRY(alloc(&ritz, d * size_t(nev)));
    FQ_TRY(alloc(&partial, std::max<size_t>(size_t(nblk) * ldp, 2 * size_t(nblk))));
    FQ_TRY(alloc(&hdev, size_t(m + b) * b * 2));
    FQ_TRY(alloc(&qbuf, size_t(m + b) * std::max(m, nev)));
    FQ_TRY(alloc(&small, 64));
    void* hp = nullptr;
    FQ_HIP_CHECK(hipHostMalloc(&hp, size_t(m + b) * b * 2 * sizeof(c128), hipHostMallocDefault));
    host = static_cast<c128*>(hp);
    batched_filter = coefs.empty() && (op->model != FQ_KICKED_ISING || op->L >= 4);
    if (batched_filter) {
      FQ_TRY(alloc(&psi32, d * size_t(b)));
      FQ_TRY(alloc(&x32, d * size_t(b)));
    }
    return FQ_OK;
  }

  // V[:, col + b .. col + 2b) = g(U) V[:, col .. col + b), filter arithmetic dt
  fq_status filter_block(int col, fq_dtype dt) {
    const c128* in = V + size_t(col) * d;
    c128* out = V + size_t(col + b) * d;
    if (!batched_filter) {
      for (int c = 0; c < b; ++c)
        FQ_TRY(filter_mixed(op, k, phi, coefs.empty() ? nullptr : coefs.data(), dt, in + size_t(c) * d,
                            out + size_t(c) * d, s));
      return FQ_OK;
    }
    // the block's columns are contiguous in V: one call for all b vectors
    if (dt == FQ_C64) {
      FQ_HIP_CHECK(launch_cast_c128_to_c64(in, psi32, size_t(b) * d, s));
      FQ_TRY(filter_many(op, k, phi, FQ_C64, b, psi32, x32, s));
      FQ_HIP_CHECK(launch_cast_c64_to_c128(x32, out, size_t(b) * d, s));
      return FQ_OK;
    }
    return filter_many(op, k, phi, FQ_C128, b, in, out, s);
  }

  // host copy of n complex values from the device (synchronising)
  fq_status fetch(const c128* src, size_t n, std::vector<zd>* out) {
    FQ_HIP_CHECK(hipMemcpyAsync(host, src, n * sizeof(c128), hipMemcpyDeviceToHost, s));
    FQ_HIP_CHECK(hipStreamSynchronize(s));
    out->resize(n);
    for (size_t i = 0; i < n; ++i) (*out)[i] = zd(host[i].x, host[i].y);
    return FQ_OK;
  }

  // Column-by-column classical Gram-Schmidt, twice, inside the block W (b
  // columns at V[:, col]); the fallback when the block is too ill conditioned
  // for Cholesky QR.  R (b x b, column-major): W_before = W_after R.
  // diag2: squared column norms before orthogonalisation (breakdown check).
  fq_status cgs_inside(int col, const std::vector<double>& diag2, std::vector<zd>* R) {
    c128* W = V + size_t(col) * d;
    c128* h = hdev;            // h1 of column c at h + c*b, h2 at h + (b + c)*b
    double* nrm = small + 16;  // (norm, 1/norm) of column c at nrm + 2c
    for (int c = 0; c < b; ++c) {
      c128* w = W + size_t(c) * d;
      if (c > 0) {
        c128* h1 = h + size_t(c) * b;
        c128* h2 = h + size_t(b + c) * b;
        FQ_HIP_CHECK(launch_dots(W, d, c, w, d, partial, ldp, s));
        FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, c, h1, s));
        FQ_HIP_CHECK(launch_update(W, d, c, h1, w, d, s));
        FQ_HIP_CHECK(launch_dots(W, d, c, w, d, partial, ldp, s));
        FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, c, h2, s));
        FQ_HIP_CHECK(launch_update(W, d, c, h2, w, d, s));
      }
      FQ_HIP_CHECK(launch_norm2(w, d, partial, s));
      FQ_HIP_CHECK(launch_reduce_norm(partial, nblk, nrm + 2 * c, s));
      FQ_HIP_CHECK(launch_scale_dev(w, nrm + 2 * c + 1, w, d, s));
    }
    std::vector<zd> hh;
    FQ_TRY(fetch(h, size_t(2) * b * b, &hh));
    std::vector<double> hn(2 * b);
    FQ_HIP_CHECK(hipMemcpyAsync(host, nrm, 2 * b * sizeof(double), hipMemcpyDeviceToHost, s));
    FQ_HIP_CHECK(hipStreamSynchronize(s));
    std::copy_n(reinterpret_cast<const double*>(host), 2 * b, hn.begin());
    R->assign(size_t(b) * b, zd(0, 0));
    for (int c = 0; c < b; ++c) {
      for (int i = 0; i < c; ++i) (*R)[size_t(c) * b + i] = hh[size_t(c) * b + i] + hh[size_t(b + c) * b + i];
      const double nc = hn[2 * c];
      if (!(nc > 1e-13 * std::sqrt(std::max(diag2[c], 0.0))) || !std::isfinite(nc)) {
        set_error("block Arnoldi breakdown: the new block is rank deficient (invariant subspace or dependent "
                  "start vectors)");
        return FQ_ENUMERIC;
      }
      (*R)[size_t(c) * b + c] = nc;
    }
    return FQ_OK;
  }

  // Orthonormalise the b columns at V[:, col] in place; R (b x b,
  // column-major, upper triangular) with W_before = W_after R.
  fq_status orthonormalise_block(int col, std::vector<zd>* R) {
    c128* W = V + size_t(col) * d;
    std::vector<zd> Racc(size_t(b) * b, zd(0, 0));
    for (int i = 0; i < b; ++i) Racc[size_t(i) * b + i] = 1.0;
    for (int round = 0; round < 2; ++round) {
      FQ_HIP_CHECK(launch_bdots(W, d, b, W, d, b, d, partial, ldp, s));
      FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, b * b, hdev, s));
      std::vector<zd> gt;
      FQ_TRY(fetch(hdev, size_t(b) * b, &gt));
      // gt[i*b + c] = <W_i, W_c> = G(i, c)
      std::vector<zd> G(size_t(b) * b);
      std::vector<double> diag2(b);
      for (int i = 0; i < b; ++i) {
        for (int c = 0; c < b; ++c) G[size_t(c) * b + i] = gt[size_t(i) * b + c];
        diag2[i] = gt[size_t(i) * b + i].real();
      }
      std::vector<zd> Rk;
      if (!cholesky_upper(G, b, &Rk, 1e-14)) {
        FQ_TRY(cgs_inside(col, diag2, &Rk));
        Racc = matmul(Rk, Racc, b);
        break;  // CGS2 leaves W orthonormal to working precision
      }
      const std::vector<zd> Ri = inv_upper(Rk, b);
      std::vector<c128> q(size_t(b) * b);  // k-major: q[i*b + c] = Ri(i, c)
      for (int i = 0; i < b; ++i)
        for (int c = 0; c < b; ++c)
          q[size_t(i) * b + c] = mk<double>(Ri[size_t(c) * b + i].real(), Ri[size_t(c) * b + i].imag());
      FQ_HIP_CHECK(hipMemcpyAsync(qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      FQ_HIP_CHECK(launch_basis_gemm(W, d, b, qbuf, b, W, d, d, s));
      FQ_HIP_CHECK(hipStreamSynchronize(s));  // q is pageable and goes out of scope
      Racc = matmul(Rk, Racc, b);
    }
    *R = Racc;
    return FQ_OK;
  }

  // Block step from V[:, cur - b .. cur): V[:, cur .. cur + b) and the
  // columns cur - b .. cur of H (rows 0 .. cur + b).
  fq_status block_step(int cur, fq_dtype dt, ZMat& H) {
    const int col = cur - b;
    const double t0 = now_s();
    FQ_TRY(filter_block(col, dt));
    c128* W = V + size_t(cur) * d;
    c128* h1 = hdev;
    c128* h2 = hdev + size_t(m + b) * b;
    FQ_HIP_CHECK(launch_bdots(V, d, cur, W, d, b, d, partial, ldp, s));
    FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, cur * b, h1, s));
    FQ_HIP_CHECK(launch_bupdate(V, d, cur, h1, W, d, b, d, s));
    FQ_HIP_CHECK(launch_bdots(V, d, cur, W, d, b, d, partial, ldp, s));
    FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, cur * b, h2, s));
    FQ_HIP_CHECK(launch_bupdate(V, d, cur, h2, W, d, b, d, s));
    std::vector<zd> a1, a2;
    FQ_TRY(fetch(h1, size_t(cur) * b, &a1));  // waits for the filter too
    const double t1 = now_s();
    t_filter += t1 - t0;
    FQ_TRY(fetch(h2, size_t(cur) * b, &a2));
    for (int i = 0; i < cur; ++i)
      for (int c = 0; c < b; ++c) {
        const zd v = a1[size_t(i) * b + c] + a2[size_t(i) * b + c];
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) {
          set_error("non-finite value in the block Arnoldi process (filter output overflow?)");
          return FQ_ENUMERIC;
        }
        H(i, col + c) = v;
      }
    std::vector<zd> R;
    FQ_TRY(orthonormalise_block(cur, &R));
    for (int j = 0; j < b; ++j)
      for (int i = 0; i <= j; ++i) H(cur + i, col + j) = R[size_t(j) * b + i];
    t_orth += now_s() - t1;
    return FQ_OK;
  }

  // Schur form of S = H[0:mm, 0:mm] (largest |theta| first), BZ = H[mm:mm+b,
  // 0:mm] Z, the Ritz coefficient vectors X (mm x nev) and the relative
  // estimates ||B Z y|| / (||y|| |theta|) of the nev wanted pairs.
  fq_status analyse(const ZMat& H, int mm, double tolg, ZMat* T, ZMat* Z, ZMat* BZ, ZMat* X, int* nconv,
                    double* worst) {
    const double t2 = now_s();
    *T = ZMat(mm, mm);
    for (int j = 0; j < mm; ++j)
      for (int i = 0; i < mm; ++i) (*T)(i, j) = H(i, j);
    if (!schur(*T, *Z)) {
      set_error("QR iteration on the projected matrix did not converge");
      return FQ_ENUMERIC;
    }
    schur_sort(*T, *Z, std::min(std::max(p_keep, nev), mm),
               [](const zd& a, const zd& c) { return std::abs(a) > std::abs(c); });
    *BZ = ZMat(b, mm);
    for (int c = 0; c < mm; ++c)
      for (int r = 0; r < b; ++r) {
        zd acc = 0;
        for (int i = 0; i < mm; ++i) acc += H(mm + r, i) * (*Z)(i, c);
        (*BZ)(r, c) = acc;
      }
    *nconv = 0;
    *worst = 0.0;
    *X = ZMat(mm, nev);
    for (int i = 0; i < nev; ++i) {
      const std::vector<zd> y = tri_eigvec(*T, i);
      double yn = 0.0;
      for (const zd& v : y) yn += std::norm(v);
      yn = std::sqrt(yn);
      double e2 = 0.0;
      for (int r = 0; r < b; ++r) {
        zd e = 0;
        for (int l = 0; l <= i; ++l) e += (*BZ)(r, l) * y[l];
        e2 += std::norm(e);
      }
      const double est = std::sqrt(e2) / (yn * std::max(std::abs((*T)(i, i)), 1e-300));
      *worst = std::max(*worst, est);
      if (est <= tolg) ++*nconv;
      for (int r = 0; r < mm; ++r) {
        zd acc = 0;
        for (int l = 0; l <= i; ++l) acc += (*Z)(r, l) * y[l];
        (*X)(r, i) = acc / yn;
      }
    }
    t_restart += now_s() - t2;
    return FQ_OK;
  }

  // Ritz vectors Y = V_mm X into ritz, omega = <y|U|y> and the FP64 residual
  // ||U y - omega y|| for each (Sec. 4)
  fq_status ritz_vectors(int mm, const ZMat& X, Ritz* out) {
    std::vector<c128> q(size_t(mm) * nev);
    for (int c = 0; c < nev; ++c)
      for (int i = 0; i < mm; ++i) q[size_t(i) * nev + c] = mk<double>(X(i, c).real(), X(i, c).imag());
    FQ_HIP_CHECK(hipMemcpyAsync(qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
    FQ_HIP_CHECK(launch_basis_gemm(V, d, mm, qbuf, nev, ritz, d, d, s));
    out->omega.assign(nev, zd(0, 0));
    out->resid.assign(nev, 0.0);
    for (int i = 0; i < nev; ++i) {
      c128* y = ritz + size_t(i) * d;
      FQ_HIP_CHECK(launch_norm2(y, d, partial, s));
      FQ_HIP_CHECK(launch_reduce_norm(partial, nblk, small, s));
      FQ_HIP_CHECK(launch_scale_dev(y, small + 1, y, d, s));
      FQ_TRY(apply_U_internal(op, FQ_C128, y, uy, s));
      st->n_U_apps += 1;
      c128* om = reinterpret_cast<c128*>(small + 4);
      FQ_HIP_CHECK(launch_dots(y, d, 1, uy, d, partial, ldp, s));
      FQ_HIP_CHECK(launch_reduce_cols(partial, ldp, nblk, 1, om, s));
      FQ_HIP_CHECK(launch_axpy_dev(om, y, uy, d, s));
      FQ_HIP_CHECK(launch_norm2(uy, d, partial, s));
      FQ_HIP_CHECK(launch_reduce_norm(partial, nblk, small + 6, s));
      FQ_HIP_CHECK(hipMemcpyAsync(host, small + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
      FQ_HIP_CHECK(hipStreamSynchronize(s));  // also keeps q alive until the product has run
      const double* h = reinterpret_cast<const double*>(host);
      out->omega[i] = zd(h[0], h[1]);
      out->resid[i] = h[2];
      if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2])) {
        set_error("non-finite Ritz value or residual");
        return FQ_ENUMERIC;
      }
    }
    return FQ_OK;
  }

  // Krylov-Schur run in arithmetic dt from the orthonormal start block
  // V[:, 0:b); stopping rules of the single-vector solver.
  fq_status run(fq_dtype dt, double tolg, double tol, bool check_true, int budget, bool early, int* restarts,
                bool* converged, Ritz* res) {
    ZMat H(m + b, m);
    int cur = b;
    double best = 1e300;
    int stall = 0;
    *restarts = 0;
    for (;;) {
      FQ_TRY(block_step(cur, dt, H));
      st->n_filter_apps += b;
      st->n_U_apps += static_cast<long long>(k) * b;
      if (dt == FQ_C64) st->n_U_apps_c64 += static_cast<long long>(k) * b;
      cur += b;
      const int mm = cur - b;
      const bool full = mm == m;
      const int ce = std::max(b, check_every);
      const bool probe = early && !full && mm >= nev + b && ((mm - nev) % ce < b);
      if (!full && !probe) continue;
      ZMat T, Z, BZ, X;
      int nconv = 0;
      double worst = 0.0;
      FQ_TRY(analyse(H, mm, tolg, &T, &Z, &BZ, &X, &nconv, &worst));
      if (verbose())
        std::fprintf(stderr, "[fq] block b=%d %s cycle %d: size %d, nconv %d/%d, worst rel est %.3e\n", b,
                     dt == FQ_C64 ? "c64" : "c128", *restarts, mm, nconv, nev, worst);
      const bool all = nconv >= nev;
      if (!full) {
        if (!all) continue;
        FQ_TRY(ritz_vectors(mm, X, res));
        double rmax = 0.0;
        for (double r : res->resid) rmax = std::max(rmax, r);
        if (!check_true || rmax <= tol) {
          *converged = true;
          return FQ_OK;
        }
        continue;
      }
      const bool out_of_budget = *restarts >= budget;
      if (worst < 0.5 * best) {
        best = worst;
        stall = 0;
      } else {
        ++stall;
      }
      const bool stalled = !check_true && stall >= 3 && worst < 1e-3;
      if (all || out_of_budget || stalled) {
        FQ_TRY(ritz_vectors(m, X, res));
        double rmax = 0.0;
        for (double r : res->resid) rmax = std::max(rmax, r);
        if (!check_true) {
          *converged = all;
          return FQ_OK;
        }
        if (rmax <= tol) {
          *converged = true;
          return FQ_OK;
        }
        if (out_of_budget) {
          *converged = false;
          return FQ_OK;
        }
        tolg *= 0.1;
      }
      // restart: V_p = V_m Z_p, the residual block behind it, H = [T_p; B Z_p]
      const double t3 = now_s();
      const int p = p_keep;
      std::vector<c128> q(size_t(m) * p);
      for (int c = 0; c < p; ++c)
        for (int i = 0; i < m; ++i) q[size_t(i) * p + c] = mk<double>(Z(i, c).real(), Z(i, c).imag());
      FQ_HIP_CHECK(hipMemcpyAsync(qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      FQ_HIP_CHECK(launch_basis_gemm(V, d, m, qbuf, p, V, d, d, s));
      FQ_HIP_CHECK(hipMemcpyAsync(V + size_t(p) * d, V + size_t(m) * d, size_t(b) * d * sizeof(c128),
                                  hipMemcpyDeviceToDevice, s));
      ZMat Hn(m + b, m);
      for (int jj = 0; jj < p; ++jj) {
        for (int i = 0; i <= jj; ++i) Hn(i, jj) = T(i, jj);
        for (int r = 0; r < b; ++r) Hn(p + r, jj) = BZ(r, jj);
      }
      H = Hn;
      cur = p + b;
      ++*restarts;
      FQ_HIP_CHECK(hipStreamSynchronize(s));
      t_restart += now_s() - t3;
    }
  }
};

template <typename Real>
fq_status filter_many_ki(floquet_op* op, int k, double phi, int n, const void* psi, void* out, hipStream_t s) {
  const PhaseTables* tab;
  FQ_TRY(get_tables(op, phi, &tab));
  const cpx<Real>* tlo = sizeof(Real) == 4 ? reinterpret_cast<const cpx<Real>*>(tab->tlo32)
                                           : reinterpret_cast<const cpx<Real>*>(tab->tlo64);
  const cpx<Real>* thi = sizeof(Real) == 4 ? reinterpret_cast<const cpx<Real>*>(tab->thi32)
                                           : reinterpret_cast<const cpx<Real>*>(tab->thi64);
  const size_t d = op->dim();
  // descriptors: the problems (x = out_j), then two sets whose x is the
  // kicked psi of tile group 0 / 1 (chi buffers), then the problem list.
  // The folded passes are used for complex128 with 4 vectors: at L = 20 they
  // take a 4-vector pass from 42.7 to 41.7 us, but a 2-vector pass from 24.7
  // to 26.0 us and an 8-vector pass from 77.5 to 84.3 us (the folded kernel
  // keeps one wave per SIMD less resident), and the complex64 passes (phase
  // entries prefetched) measured slower with them.
  const bool fold = sizeof(Real) == 8 && n == 4;
  const size_t need = size_t(n) * (3 * sizeof(KiDesc<Real>) + sizeof(int));
  const size_t chi_need = fold ? 2 * size_t(n) * d * sizeof(cpx<Real>) : 0;
  bool fresh = false;
  if (op->chi_cap < chi_need) {
    (void)hipFree(op->chi_mem);  // waits for work still reading it
    op->chi_mem = nullptr;
    op->chi_cap = 0;
    FQ_HIP_CHECK(hipMalloc(&op->chi_mem, chi_need));
    op->chi_cap = chi_need;
    fresh = true;
  }
  cpx<Real>* chi = fold ? static_cast<cpx<Real>*>(op->chi_mem) : nullptr;
  const void* key[5] = {psi, out, tlo, thi, chi};
  bool same = !fresh && op->many_n == n && std::equal(key, key + 5, op->many_key);
  if (op->many_cap < need) {
    (void)hipFree(op->many_mem);  // waits for work still reading it
    op->many_mem = nullptr;
    op->many_cap = 0;
    FQ_HIP_CHECK(hipMalloc(&op->many_mem, need));
    op->many_cap = need;
    same = false;
  }
  KiDesc<Real>* desc = static_cast<KiDesc<Real>*>(op->many_mem);
  int* list = reinterpret_cast<int*>(desc + 3 * size_t(n));
  if (!same) {
    std::vector<unsigned char> h(need);
    KiDesc<Real>* hd = reinterpret_cast<KiDesc<Real>*>(h.data());
    int* hl = reinterpret_cast<int*>(hd + 3 * size_t(n));
    for (int j = 0; j < n; ++j) {
      const cpx<Real>* pj = static_cast<const cpx<Real>*>(psi) + size_t(j) * d;
      cpx<Real>* c0 = fold ? chi + size_t(j) * d : nullptr;
      cpx<Real>* c1 = fold ? chi + (size_t(n) + j) * d : nullptr;
      hd[j] = KiDesc<Real>{pj, static_cast<cpx<Real>*>(out) + size_t(j) * d, tlo, thi, op->w, 0.0, {c0, c1}};
      hd[n + j] = KiDesc<Real>{pj, c0, tlo, thi, op->w, 0.0, {nullptr, nullptr}};
      hd[2 * n + j] = KiDesc<Real>{pj, c1, tlo, thi, op->w, 0.0, {nullptr, nullptr}};
      hl[j] = j;
    }
    FQ_HIP_CHECK(hipMemcpyAsync(desc, h.data(), need, hipMemcpyHostToDevice, s));
    FQ_HIP_CHECK(hipStreamSynchronize(s));  // h is pageable and local
    std::copy(key, key + 5, op->many_key);
    op->many_n = n;
  }
  const KiDesc<Real>* chi0 = fold ? desc + n : nullptr;
  const KiDesc<Real>* chi1 = fold ? desc + 2 * size_t(n) : nullptr;
  KiBatchShape sh;
  FQ_TRY(ki_batch_tune<Real>(op->L, op->sw, k, desc, list, static_cast<unsigned>(n), s, &sh, nullptr, chi0, chi1));
  return ki_batch_filter<Real>(sh, k, desc, list, static_cast<unsigned>(n), s, chi0, chi1);
}

}  // namespace

extern "C" fq_status fq_set_kernel_policy(int policy) {
  clear_error();
  return ki_set_policy(policy);
}

fq_status filter_many(floquet_op* op, int k, double phi, fq_dtype dt, int n, const void* psi, void* out,
                      hipStream_t s) {
  if (op->model == FQ_KICKED_ISING && op->L >= 4 && k >= 1 && n > 1)
    return dt == FQ_C64 ? filter_many_ki<float>(op, k, phi, n, psi, out, s)
                        : filter_many_ki<double>(op, k, phi, n, psi, out, s);
  if (op->model != FQ_KICKED_ISING && k >= 1 && n > 1) return bw_filter(op, k, phi, nullptr, dt, psi, out, s, n);
  const size_t bytes = op->dim() * (dt == FQ_C64 ? sizeof(c64) : sizeof(c128));
  for (int j = 0; j < n; ++j)
    FQ_TRY(filter_internal(op, k, phi, nullptr, dt, static_cast<const char*>(psi) + size_t(j) * bytes,
                           static_cast<char*>(out) + size_t(j) * bytes, s));
  return FQ_OK;
}

fq_status block_solve(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* o, double* evals_host,
                      void* evecs_dev, double* resid_host, fq_arnoldi_stats* stats, hipStream_t s) {
  const double t_start = now_s();
  fq_arnoldi_stats local{};
  fq_arnoldi_stats* st = stats ? stats : &local;
  *st = fq_arnoldi_stats{};
  const int b = o->block;
  if (b != 2 && b != 4 && b != 8) {
    set_error("arnoldi_eigs: block must be 0, 1, 2, 4 or 8");
    return FQ_EINVAL;
  }
  BlockSolver sv;
  sv.op = op;
  sv.nev = nev;
  sv.b = b;
  sv.m = (o->ncv / b) * b;
  if (sv.m < nev + 2 * b) {
    set_error("arnoldi_eigs: a block of b vectors needs floor(ncv / b) * b >= nev + 2b");
    return FQ_EINVAL;
  }
  if (static_cast<long long>(sv.m + b) > static_cast<long long>(op->dim())) {
    set_error("arnoldi_eigs: floor(ncv / block) * block + block must not exceed the dimension 2^L");
    return FQ_EINVAL;
  }
  if (size_t(sv.m + b) * b > 4096) {
    set_error("arnoldi_eigs: (floor(ncv / block) + 1) * block^2 must be <= 4096");
    return FQ_EINVAL;
  }
  // kept Schur vectors: about nev + (m - nev) / 2, rounded down to a multiple
  // of b so that every later block step starts on a multiple of b
  int p = (keep_count(sv.m, nev) / b) * b;
  if (p <= nev) p += b;
  if (p > sv.m - b) {
    set_error("arnoldi_eigs: ncv too small for the block size");
    return FQ_EINVAL;
  }
  sv.p_keep = p;
  sv.check_every = std::max(4, sv.m / 16);
  sv.k = o->k;
  sv.phi = phi;
  if (o->poly_coeffs)
    for (int i = 0; i <= o->k; ++i) sv.coefs.push_back(zd(o->poly_coeffs[2 * i], o->poly_coeffs[2 * i + 1]));
  sv.s = s;
  sv.st = st;
  FQ_TRY(sv.setup(evecs_dev));
  const size_t d = sv.d;

  // start block: v0 (or the seeded vector) and the seeded vectors seed + c
  for (int c = 0; c < b; ++c) {
    if (o->v0_dev && c == 0)
      FQ_HIP_CHECK(hipMemcpyAsync(sv.V, o->v0_dev, d * sizeof(c128), hipMemcpyDeviceToDevice, s));
    else
      FQ_HIP_CHECK(launch_random(sv.V + size_t(c) * d, d, o->seed + static_cast<unsigned long long>(c), s));
  }
  std::vector<zd> R;
  FQ_TRY(sv.orthonormalise_block(0, &R));

  Ritz res;
  bool conv = false;
  int restarts = 0;
  const bool probes = probes_pay(d, o->k, static_cast<size_t>(b));
  if (o->filter_dtype != FQ_C64) {
    FQ_TRY(sv.run(FQ_C128, 0.5 * o->tol, o->tol, true, o->max_restarts, probes, &restarts, &conv, &res));
  } else {
    const double tol32 = std::max(o->tol, 2e-6);
    FQ_TRY(sv.run(FQ_C64, tol32, o->tol, false, o->max_restarts, probes, &restarts, &conv, &res));
    double rmax = 0.0;
    for (double r : res.resid) rmax = std::max(rmax, r);
    if (o->refine && rmax > o->tol) {
      const double t_ref0 = now_s();
      // warm start block: column c = sum_i c_i y_i with the seed + c
      // coefficients (c < nev), seeded random vectors beyond nev
      const int nc = std::min(b, nev);
      std::vector<c128> q(size_t(nev) * nc);
      for (int c = 0; c < nc; ++c) {
        std::vector<c128> cc;
        warm_start_coefs(o->seed + static_cast<unsigned long long>(c), nev, &cc);
        for (int i = 0; i < nev; ++i) q[size_t(i) * nc + c] = cc[i];
      }
      FQ_HIP_CHECK(hipMemcpyAsync(sv.qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      FQ_HIP_CHECK(launch_basis_gemm(sv.ritz, d, nev, sv.qbuf, nc, sv.V, d, d, s));
      for (int c = nc; c < b; ++c)
        FQ_HIP_CHECK(launch_random(sv.V + size_t(c) * d, d, o->seed + static_cast<unsigned long long>(c), s));
      FQ_HIP_CHECK(hipStreamSynchronize(s));
      FQ_TRY(sv.orthonormalise_block(0, &R));
      if (o->refine_k > 0) sv.k = o->refine_k;
      int r2 = 0;
      const int budget = std::max(0, o->max_restarts - restarts);
      FQ_TRY(sv.run(FQ_C128, 0.5 * o->tol, o->tol, true, budget, true, &r2, &conv, &res));
      restarts += r2;
      st->t_refine = now_s() - t_ref0;
    }
  }
  st->n_restarts = restarts;

  // order by arc distance to the target, write outputs
  std::vector<int> order(nev);
  std::iota(order.begin(), order.end(), 0);
  const zd rot = std::polar(1.0, -phi);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return std::abs(std::arg(res.omega[a] * rot)) < std::abs(std::arg(res.omega[c] * rot));
  });
  int nconv = 0;
  double rmax = 0.0;
  for (int i = 0; i < nev; ++i) {
    const int j = order[i];
    if (evals_host) {
      evals_host[2 * i] = res.omega[j].real();
      evals_host[2 * i + 1] = res.omega[j].imag();
    }
    if (resid_host) resid_host[i] = res.resid[j];
    if (res.resid[j] <= o->tol) ++nconv;
    rmax = std::max(rmax, res.resid[j]);
  }
  if (evecs_dev) {
    bool identity = true;
    for (int i = 0; i < nev; ++i) identity = identity && order[i] == i;
    if (!identity) {  // the basis is no longer needed: permute through it
      for (int i = 0; i < nev; ++i)
        FQ_HIP_CHECK(hipMemcpyAsync(sv.V + size_t(i) * d, sv.ritz + size_t(order[i]) * d, d * sizeof(c128),
                                    hipMemcpyDeviceToDevice, s));
      FQ_HIP_CHECK(hipMemcpyAsync(sv.ritz, sv.V, size_t(nev) * d * sizeof(c128), hipMemcpyDeviceToDevice, s));
    }
  }
  FQ_HIP_CHECK(hipStreamSynchronize(s));
  st->nconv = nconv;
  st->max_residual = rmax;
  st->t_filter = sv.t_filter;
  st->t_orth = sv.t_orth;
  st->t_restart = sv.t_restart;
  st->t_total = now_s() - t_start;
  if (nconv < nev) {
    set_error("not converged: " + std::to_string(nconv) + " of " + std::to_string(nev) + " pairs meet tol");
    return FQ_NOT_CONVERGED;
  }
  return FQ_OK;
}

}  // namespace fq
