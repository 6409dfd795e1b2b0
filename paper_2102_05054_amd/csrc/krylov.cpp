// Krylov-Schur Arnoldi on the geometric-sum filter g_k(U) (Sec. 4).
//
// The paper runs ARPACK's implicitly restarted Arnoldi on g_k(U) and keeps
// the Ritz values of largest modulus (Eq. (arnoldi)); here the same Krylov
// space is restarted with Stewart's Krylov-Schur scheme, which keeps an
// orthonormal basis V (FP64, on the device) and an (m+1) x m projected
// matrix on the host:
//     g_k(U) V_m = V_m S + v_m b^T.
// Per Arnoldi step: one filter application (HIP kernels, complex64 or
// complex128), classical Gram-Schmidt twice (FP64 kernels), no host sync;
// the projection coefficients are copied back once per cycle.  At a restart
// the m x m matrix S is brought to Schur form on the host, the Ritz values of
// largest |theta| are moved to the front and the basis is rotated on the
// device (V_p = V_m Z_p).  Converged Ritz vectors |n> give omega_n = <n|U|n>
// and r_n = ||U|n> - omega_n|n>|| in FP64 (Sec. 4, Eq. (residual)).
//
// Mixed precision: with a complex64 filter the Ritz residual levels off near
// the complex64 rounding level; the solve then restarts in FP64 from a
// combination of the complex64 Ritz vectors (a warm start), which converges in
// few cycles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "blas.h"
#include "dense.h"
#include "krylov.h"
#include "op.h"

namespace fq {

// Schur form of S = H[0:mm, 0:mm] with the nsort largest |theta| first,
// b^T Z, and the Ritz coefficient vectors / relative estimates of the nev
// wanted pairs.
bool probes_pay(size_t d, int k, size_t nprob) { return double(d) * k * double(nprob) >= 16777216.0; }

int keep_count(int m, int nev) { return std::min(m - 1, std::max(nev + 1, nev + (m - nev) / 2)); }

void warm_start_coefs(unsigned long long seed, int nev, std::vector<c128>* cc) {
  cc->assign(static_cast<size_t>(nev), c128{});
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 12345;
  for (int i = 0; i < nev; ++i) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    const double ang = double(x >> 11) * (2.0 * M_PI / 9007199254740992.0);
    (*cc)[i] = mk<double>(std::cos(ang), std::sin(ang));
  }
}

fq_status analyse_decomposition(const ZMat& H, int mm, int nsort, int nev, double tolg, ZMat* T, ZMat* Z,
                              std::vector<zd>* bz, ZMat* X, int* nconv, double* worst) {
  *T = ZMat(mm, mm);
  for (int j = 0; j < mm; ++j)
    for (int i = 0; i < mm; ++i) (*T)(i, j) = H(i, j);
  if (!schur(*T, *Z)) {
    set_error("QR iteration on the projected matrix did not converge");
    return FQ_ENUMERIC;
  }
  schur_sort(*T, *Z, std::min(nsort, mm), [](const zd& a, const zd& b) { return std::abs(a) > std::abs(b); });
  bz->assign(mm, zd(0, 0));
  for (int c = 0; c < mm; ++c) {
    zd acc = 0;
    for (int i = 0; i < mm; ++i) acc += H(mm, i) * (*Z)(i, c);
    (*bz)[c] = acc;
  }
  *nconv = 0;
  *worst = 0.0;
  *X = ZMat(mm, nev);
  for (int i = 0; i < nev; ++i) {
    std::vector<zd> y = tri_eigvec(*T, i);
    double yn = 0.0;
    for (const zd& v : y) yn += std::norm(v);
    yn = std::sqrt(yn);
    zd e = 0;
    for (int l = 0; l <= i; ++l) e += (*bz)[l] * y[l];
    const double est = std::abs(e) / (yn * std::max(std::abs((*T)(i, i)), 1e-300));
    *worst = std::max(*worst, est);
    if (est <= tolg) ++*nconv;
    for (int r = 0; r < mm; ++r) {
      zd acc = 0;
      for (int l = 0; l <= i; ++l) acc += (*Z)(r, l) * y[l];
      (*X)(r, i) = acc / yn;
    }
  }
  return FQ_OK;
}


namespace {

// FQ_VERBOSE=1 in the environment prints one line per restart cycle to stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("FQ_VERBOSE");
    return e && e[0] && e[0] != '0';
  }();
  return v;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Ws {
  size_t d;
  int ncv;
  int ldp;          // leading dim of partial sums (ncv + 1)
  unsigned nblk;    // row blocks
  c128* V;          // d x (ncv + 1)
  c128* w;          // d
  c128* ritz;       // d x nev (caller's evecs or internal)
  c128* partial;    // nblk x ldp
  double* slots;    // (ncv + 1) x slot_doubles
  int slot_doubles;
  c128* qbuf;       // ncv x ncv
  c128* small;      // 8 complex scratch
  double* hslots;   // pinned host mirror of slots
};

// slot j layout (doubles): h1[ncv+1] (complex), h2[ncv+1] (complex), nrm[2]
inline c128* slot_h1(const Ws& ws, int j) { return reinterpret_cast<c128*>(ws.slots + size_t(j) * ws.slot_doubles); }
inline c128* slot_h2(const Ws& ws, int j) { return slot_h1(ws, j) + (ws.ncv + 1); }
inline double* slot_nrm(const Ws& ws, int j) { return ws.slots + size_t(j) * ws.slot_doubles + 4 * (ws.ncv + 1); }

fq_status ensure_ws(floquet_op* op, int ncv, int nev, void* evecs_dev, Ws* ws, std::vector<void*>* temp) {
  const size_t d = op->dim();
  ws->d = d;
  ws->ncv = ncv;
  ws->ldp = ncv + 1;
  ws->nblk = row_blocks(d);
  ws->slot_doubles = 4 * (ncv + 1) + 2;
  if (op->ncv_cap < ncv) {
    (void)hipFree(op->V);
    op->V = nullptr;
    op->ncv_cap = 0;
    size_t freeb = 0, totalb = 0;
    FQ_HIP_CHECK(hipMemGetInfo(&freeb, &totalb));
    const size_t need = d * sizeof(c128) * size_t(ncv + 1);
    if (need + (size_t(1) << 28) > freeb) {
      set_error("Krylov workspace of " + std::to_string(need >> 20) + " MiB does not fit in free device memory");
      return FQ_ENOMEM;
    }
    if (hipMalloc(&op->V, need) != hipSuccess) {
      set_error("hipMalloc of the Krylov basis failed");
      return FQ_ENOMEM;
    }
    op->ncv_cap = ncv;
  }
  if (!op->work) FQ_HIP_CHECK(hipMalloc(&op->work, d * sizeof(c128)));
  const size_t small_need = size_t(ws->nblk) * ws->ldp * 2 + size_t(ncv + 1) * ws->slot_doubles +
                            size_t(ncv) * ncv * 2 + 64;
  if (op->dev_small_cap < small_need) {
    (void)hipFree(op->dev_small);
    (void)hipHostFree(op->host_small);
    op->dev_small = nullptr;
    op->host_small = nullptr;
    op->dev_small_cap = 0;
    FQ_HIP_CHECK(hipMalloc(&op->dev_small, small_need * sizeof(double)));
    FQ_HIP_CHECK(hipHostMalloc(&op->host_small, small_need * sizeof(double), hipHostMallocDefault));
    op->dev_small_cap = small_need;
  }
  ws->V = static_cast<c128*>(op->V);
  ws->w = static_cast<c128*>(op->work);
  double* p = op->dev_small;
  ws->partial = reinterpret_cast<c128*>(p);
  p += size_t(ws->nblk) * ws->ldp * 2;
  ws->slots = p;
  p += size_t(ncv + 1) * ws->slot_doubles;
  ws->qbuf = reinterpret_cast<c128*>(p);
  p += size_t(ncv) * ncv * 2;
  ws->small = reinterpret_cast<c128*>(p);
  ws->hslots = op->host_small;
  if (evecs_dev) {
    ws->ritz = static_cast<c128*>(evecs_dev);
  } else {
    void* r = nullptr;
    if (hipMalloc(&r, d * sizeof(c128) * size_t(nev)) != hipSuccess) {
      set_error("hipMalloc of the Ritz vectors failed");
      return FQ_ENOMEM;
    }
    temp->push_back(r);
    ws->ritz = static_cast<c128*>(r);
  }
  return FQ_OK;
}

#define FQ_TRY(expr)               \
  do {                             \
    fq_status st__ = (expr);       \
    if (st__ != FQ_OK) return st__; \
  } while (0)

// normalise column j of V in place (returns the norm on the host)
fq_status normalize_col(const Ws& ws, int j, double* nrm_host, hipStream_t s) {
  c128* v = ws.V + size_t(j) * ws.d;
  FQ_HIP_CHECK(launch_norm2(v, ws.d, ws.partial, s));
  double* nrm = reinterpret_cast<double*>(ws.small);
  FQ_HIP_CHECK(launch_reduce_norm(ws.partial, ws.nblk, nrm, s));
  FQ_HIP_CHECK(launch_scale_dev(v, nrm + 1, v, ws.d, s));
  double h[2];
  FQ_HIP_CHECK(hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, s));
  FQ_HIP_CHECK(hipStreamSynchronize(s));
  if (nrm_host) *nrm_host = h[0];
  return FQ_OK;
}

// One Arnoldi extension step j: V[:, j+1] and the coefficients of column j.
fq_status arnoldi_step(floquet_op* op, const Ws& ws, int j, int k, double phi, const zd* coefs, fq_dtype dt,
                       hipStream_t s) {
  const c128* vj = ws.V + size_t(j) * ws.d;
  FQ_TRY(filter_mixed(op, k, phi, coefs, dt, vj, ws.w, s));
  const int nc = j + 1;
  FQ_HIP_CHECK(launch_dots(ws.V, ws.d, nc, ws.w, ws.d, ws.partial, ws.ldp, s));
  FQ_HIP_CHECK(launch_reduce_cols(ws.partial, ws.ldp, ws.nblk, nc, slot_h1(ws, j), s));
  FQ_HIP_CHECK(launch_update_dots(ws.V, ws.d, nc, slot_h1(ws, j), ws.w, ws.d, ws.partial, ws.ldp, s));
  FQ_HIP_CHECK(launch_reduce_cols(ws.partial, ws.ldp, ws.nblk, nc, slot_h2(ws, j), s));
  FQ_HIP_CHECK(launch_update_norm2(ws.V, ws.d, nc, slot_h2(ws, j), ws.w, ws.d, ws.partial, s));
  FQ_HIP_CHECK(launch_reduce_norm(ws.partial, ws.nblk, slot_nrm(ws, j), s));
  FQ_HIP_CHECK(launch_scale_dev(ws.w, slot_nrm(ws, j) + 1, ws.V + size_t(j + 1) * ws.d, ws.d, s));
  return FQ_OK;
}

struct Ritz {
  std::vector<zd> omega;
  std::vector<double> resid;
};

// Ritz vectors Y = V_m X (into ws.ritz), then omega = <y|U|y> and the FP64
// residual for each (Sec. 4).
fq_status ritz_and_residuals(floquet_op* op, const Ws& ws, int m, const ZMat& X, int nev, Ritz* out,
                             hipStream_t s, long long* uapps) {
  std::vector<c128> q(size_t(m) * nev);  // k-major
  for (int c = 0; c < nev; ++c)
    for (int i = 0; i < m; ++i) q[size_t(i) * nev + c] = mk<double>(X(i, c).real(), X(i, c).imag());
  FQ_HIP_CHECK(hipMemcpyAsync(ws.qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
  FQ_HIP_CHECK(launch_basis_gemm(ws.V, ws.d, m, ws.qbuf, nev, ws.ritz, ws.d, ws.d, s));
  out->omega.assign(nev, zd(0, 0));
  out->resid.assign(nev, 0.0);
  std::vector<double> host(size_t(nev) * 4);
  for (int i = 0; i < nev; ++i) {
    c128* y = ws.ritz + size_t(i) * ws.d;
    // renormalise (X columns are unit vectors, V orthonormal to rounding)
    FQ_HIP_CHECK(launch_norm2(y, ws.d, ws.partial, s));
    double* nrm = reinterpret_cast<double*>(ws.small);
    FQ_HIP_CHECK(launch_reduce_norm(ws.partial, ws.nblk, nrm, s));
    FQ_HIP_CHECK(launch_scale_dev(y, nrm + 1, y, ws.d, s));
    FQ_TRY(apply_U_internal(op, FQ_C128, y, ws.w, s));
    *uapps += 1;
    c128* om = ws.small + 2;
    FQ_HIP_CHECK(launch_dots(y, ws.d, 1, ws.w, ws.d, ws.partial, ws.ldp, s));
    FQ_HIP_CHECK(launch_reduce_cols(ws.partial, ws.ldp, ws.nblk, 1, om, s));
    FQ_HIP_CHECK(launch_axpy_dev(om, y, ws.w, ws.d, s));
    FQ_HIP_CHECK(launch_norm2(ws.w, ws.d, ws.partial, s));
    double* rn = reinterpret_cast<double*>(ws.small + 3);
    FQ_HIP_CHECK(launch_reduce_norm(ws.partial, ws.nblk, rn, s));
    FQ_HIP_CHECK(hipMemcpyAsync(host.data() + 4 * i, ws.small + 2, 2 * sizeof(c128), hipMemcpyDeviceToHost, s));
  }
  FQ_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < nev; ++i) {
    out->omega[i] = zd(host[4 * i], host[4 * i + 1]);
    out->resid[i] = host[4 * i + 2];
    if (!std::isfinite(out->resid[i]) || !std::isfinite(host[4 * i]) || !std::isfinite(host[4 * i + 1])) {
      set_error("non-finite Ritz value or residual");
      return FQ_ENUMERIC;
    }
  }
  return FQ_OK;
}

struct PhaseResult {
  int restarts = 0;
  bool converged = false;  // Ritz estimates met the phase tolerance
  Ritz ritz;
};

struct Solver {
  floquet_op* op;
  Ws ws;
  int nev, ncv, k, max_restarts;
  double phi;
  std::vector<zd> coefs;  // user polynomial a_0..a_k, or empty for the geometric sum
  hipStream_t s;
  fq_arnoldi_stats* st;
  double t_filter = 0, t_orth = 0, t_restart = 0;
  unsigned long long seed;

  // Krylov-Schur run in arithmetic dt from the (normalised) start vector in
  // V[:, 0].  Stops when all nev wanted Ritz estimates are below
  // tolg*|theta| and, if check_true, the FP64 residuals are below tol.
  // With `early`, the projected matrix is also analysed every few steps
  // inside a cycle, so that a run can stop before the cycle is full.
  fq_status run(fq_dtype dt, double tolg, double tol, bool check_true, int restart_budget, bool early,
                PhaseResult* res) {
    const int m = ncv;
    ZMat H(m + 1, m);
    int kk = 0;
    const int p_keep = keep_count(m, nev);
    const int check_every = std::max(4, m / 16);
    double best = 1e300;
    int stall = 0;
    for (;;) {
      double t0 = now_s();  // start of the filter/CGS2 work not yet accounted
      int copied = kk;  // columns of H already on the host
      for (int j = kk; j < m; ++j) {
        FQ_TRY(arnoldi_step(op, ws, j, k, phi, coefs.empty() ? nullptr : coefs.data(), dt, s));
        st->n_filter_apps += 1;
        st->n_U_apps += k;
        if (dt == FQ_C64) st->n_U_apps_c64 += k;
        const int mm = j + 1;
        const bool full = mm == m;
        const bool probe = early && mm >= nev + 2 && ((mm - nev - 2) % check_every == 0);
        if (!full && !probe) continue;
        const size_t bytes = size_t(mm - copied) * ws.slot_doubles * sizeof(double);
        FQ_HIP_CHECK(hipMemcpyAsync(ws.hslots + size_t(copied) * ws.slot_doubles,
                                    ws.slots + size_t(copied) * ws.slot_doubles, bytes, hipMemcpyDeviceToHost, s));
        FQ_HIP_CHECK(hipStreamSynchronize(s));
        double hn = 0.0;
        for (int jj = copied; jj < mm; ++jj) {
          const double* sl = ws.hslots + size_t(jj) * ws.slot_doubles;
          for (int i = 0; i <= jj; ++i) {
            H(i, jj) = zd(sl[2 * i] + sl[2 * (ws.ncv + 1) + 2 * i], sl[2 * i + 1] + sl[2 * (ws.ncv + 1) + 2 * i + 1]);
            hn = std::max(hn, std::abs(H(i, jj)));
          }
          const double beta = sl[4 * (ws.ncv + 1)];
          if (!std::isfinite(beta) || !std::isfinite(hn)) {
            set_error("non-finite value in the Arnoldi process (filter output overflow?)");
            return FQ_ENUMERIC;
          }
          if (beta <= 1e-14 * std::max(hn, 1e-300)) {
            // The Krylov space is invariant: g V = V H holds exactly for the
            // first jj + 1 columns (e.g. ncv = d, or a spectrum with fewer
            // distinct filter values than ncv).  Its Ritz pairs are exact.
            H(jj + 1, jj) = 0.0;
            return finish_invariant(H, jj + 1, tolg, tol, check_true, res);
          }
          H(jj + 1, jj) = beta;
        }
        copied = mm;
        const double t1 = now_s();
        const double t_seg = t1 - t0;
        t_filter += t_seg;
        // analyse the decomposition of size mm
        ZMat T, Z, X;
        std::vector<zd> bz;
        int nconv = 0;
        double worst = 0.0;
        FQ_TRY(analyse(H, mm, std::max(p_keep, nev), tolg, &T, &Z, &bz, &X, &nconv, &worst));
        if (verbose())
          std::fprintf(stderr,
                       "[fq] %s cycle %d: size %d (from %d) %.3fs, nconv %d/%d, worst rel est %.3e, |theta| %.4g..%.4g\n",
                       dt == FQ_C64 ? "c64" : "c128", res->restarts, mm, kk, t_seg, nconv, nev, worst,
                       std::abs(T(0, 0)), std::abs(T(nev - 1, nev - 1)));
        const bool all = nconv >= nev;
        if (!full) {
          if (all) {
            FQ_TRY(ritz_and_residuals(op, ws, mm, X, nev, &res->ritz, s, &st->n_U_apps));
            double rmax = 0.0;
            for (double r : res->ritz.resid) rmax = std::max(rmax, r);
            if (!check_true || rmax <= tol) {
              res->converged = true;
              return FQ_OK;
            }
          }
          t0 = now_s();  // keep extending this cycle
          continue;
        }
        const bool out_of_budget = res->restarts >= restart_budget;
        if (worst < 0.5 * best) {
          best = worst;
          stall = 0;
        } else {
          ++stall;
        }
        // complex64 phase: stop once the estimates sit at the complex64 floor
        // (no longer halving) -- not while they are still far above it
        const bool stalled = !check_true && stall >= 3 && worst < 1e-3;
        if (all || out_of_budget || stalled) {
          FQ_TRY(ritz_and_residuals(op, ws, m, X, nev, &res->ritz, s, &st->n_U_apps));
          double rmax = 0.0;
          for (double r : res->ritz.resid) rmax = std::max(rmax, r);
          if (!check_true) {
            res->converged = all;
            return FQ_OK;
          }
          if (rmax <= tol) {
            res->converged = true;
            return FQ_OK;
          }
          if (out_of_budget) {
            res->converged = false;
            return FQ_OK;
          }
          tolg *= 0.1;  // the estimates were optimistic: tighten and continue
        }
        // restart: keep p_keep Schur vectors
        const double t3 = now_s();
        const int p = p_keep;
        std::vector<c128> q(size_t(m) * p);  // k-major
        for (int c = 0; c < p; ++c)
          for (int i = 0; i < m; ++i) q[size_t(i) * p + c] = mk<double>(Z(i, c).real(), Z(i, c).imag());
        FQ_HIP_CHECK(hipMemcpyAsync(ws.qbuf, q.data(), q.size() * sizeof(c128), hipMemcpyHostToDevice, s));
        FQ_HIP_CHECK(launch_basis_gemm(ws.V, ws.d, m, ws.qbuf, p, ws.V, ws.d, ws.d, s));
        FQ_HIP_CHECK(hipMemcpyAsync(ws.V + size_t(p) * ws.d, ws.V + size_t(m) * ws.d, ws.d * sizeof(c128),
                                    hipMemcpyDeviceToDevice, s));
        ZMat Hn(m + 1, m);
        for (int jj = 0; jj < p; ++jj) {
          for (int i = 0; i <= jj; ++i) Hn(i, jj) = T(i, jj);
          Hn(p, jj) = bz[jj];
        }
        H = Hn;
        kk = p;
        ++res->restarts;
        FQ_HIP_CHECK(hipStreamSynchronize(s));
        t_restart += now_s() - t3;
      }
    }
  }

  // Ritz pairs of an invariant Krylov space of dimension mm (its residual
  // row is zero, so every Ritz estimate vanishes).
  fq_status finish_invariant(const ZMat& H, int mm, double tolg, double tol, bool check_true, PhaseResult* res) {
    if (mm < nev) {
      set_error("Arnoldi breakdown: the Krylov space became invariant at dimension " + std::to_string(mm) +
                " < nev (the start vector meets fewer than nev eigenvectors, or the spectrum is degenerate)");
      return FQ_ENUMERIC;
    }
    ZMat Hs(mm + 1, mm);
    for (int j = 0; j < mm; ++j)
      for (int i = 0; i < mm; ++i) Hs(i, j) = H(i, j);
    ZMat T, Z, X;
    std::vector<zd> bz;
    int nconv = 0;
    double worst = 0.0;
    FQ_TRY(analyse(Hs, mm, nev, tolg, &T, &Z, &bz, &X, &nconv, &worst));
    FQ_TRY(ritz_and_residuals(op, ws, mm, X, nev, &res->ritz, s, &st->n_U_apps));
    double rmax = 0.0;
    for (double r : res->ritz.resid) rmax = std::max(rmax, r);
    res->converged = check_true ? rmax <= tol : true;
    return FQ_OK;
  }

  fq_status analyse(const ZMat& H, int mm, int nsort, double tolg, ZMat* T, ZMat* Z, std::vector<zd>* bz, ZMat* X,
                    int* nconv, double* worst) {
    const double t2 = now_s();
    const fq_status st = analyse_decomposition(H, mm, nsort, nev, tolg, T, Z, bz, X, nconv, worst);
    t_restart += now_s() - t2;
    return st;
  }
};

}  // namespace

fq_status validate_arnoldi(const floquet_op* op, int nev, const fq_arnoldi_opts* o) {
  if (!op) {
    set_error("op is NULL");
    return FQ_EINVAL;
  }
  if (!o) {
    set_error("opts is NULL");
    return FQ_EINVAL;
  }
  const long long d = (long long)op->dim();
  if (nev < 1 || o->ncv < nev + 2 || o->ncv > d || o->k < 0 || !(o->tol > 0) || o->max_restarts < 0 ||
      (o->filter_dtype != FQ_C64 && o->filter_dtype != FQ_C128) || o->ncv > 3000 || o->refine_k < 0) {
    set_error("arnoldi_eigs: need 1 <= nev, nev + 2 <= ncv <= min(d, 3000), k >= 0, refine_k >= 0, tol > 0, "
              "max_restarts >= 0");
    return FQ_EINVAL;
  }
  if (o->block != 0 && o->block != 1 && o->block != 2 && o->block != 4 && o->block != 8) {
    set_error("arnoldi_eigs: block must be 0, 1, 2, 4 or 8");
    return FQ_EINVAL;
  }
  if (o->poly_coeffs) {
    if (o->refine_k != 0 && o->refine_k != o->k) {
      set_error("arnoldi_eigs: a user polynomial needs refine_k = 0 (the refinement uses the same polynomial)");
      return FQ_EINVAL;
    }
    for (int i = 0; i < 2 * (o->k + 1); ++i)
      if (!std::isfinite(o->poly_coeffs[i])) {
        set_error("arnoldi_eigs: polynomial coefficients must be finite");
        return FQ_EINVAL;
      }
  }
  return FQ_OK;
}

fq_status poly_scale_copy(floquet_op* op, zd a, fq_dtype dt, const void* psi, void* out, hipStream_t s) {
  if (dt == FQ_C64)
    FQ_HIP_CHECK(launch_scale_c64(static_cast<const c64*>(psi), a.real(), a.imag(), static_cast<c64*>(out), op->dim(), s));
  else
    FQ_HIP_CHECK(
        launch_scale_c128(static_cast<const c128*>(psi), a.real(), a.imag(), static_cast<c128*>(out), op->dim(), s));
  return FQ_OK;
}

int paper_ncv(int L, int nev) {
  const double d = std::ldexp(1.0, L);
  long long ncv = static_cast<long long>(std::floor(std::pow(2.0, L / 2.0 + 1.0)));
  ncv = std::max<long long>(ncv, 2LL * nev + 1);
  // below d: a Krylov space of dimension d is the whole space
  ncv = std::min<long long>(ncv, static_cast<long long>(d) - 1);
  return static_cast<int>(ncv);
}

int paper_k(int L, int ncv) {
  const long long k = static_cast<long long>(std::floor(0.8 * 2.0 * std::ldexp(1.0, L) / double(ncv)));
  return static_cast<int>(std::max<long long>(k, 1));
}

fq_arnoldi_opts resolve_auto(const floquet_op* op, int nev, const fq_arnoldi_opts* o) {
  fq_arnoldi_opts r = *o;
  if (!op) return r;
  if (r.ncv == 0) r.ncv = std::min(paper_ncv(op->L, nev), 3000);
  if (r.k == 0 && !r.poly_coeffs && r.ncv > 0) r.k = paper_k(op->L, r.ncv);
  return r;
}

fq_status arnoldi_solve(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* o_in, double* evals_host,
                        void* evecs_dev, double* resid_host, fq_arnoldi_stats* stats, hipStream_t s) {
  if (!o_in) {
    set_error("opts is NULL");
    return FQ_EINVAL;
  }
  const fq_arnoldi_opts oo = resolve_auto(op, nev, o_in);
  const fq_arnoldi_opts* o = &oo;
  FQ_TRY(validate_arnoldi(op, nev, o));
  if (o->block > 1) return block_solve(op, nev, phi, o, evals_host, evecs_dev, resid_host, stats, s);
  const double t_start = now_s();
  fq_arnoldi_stats local{};
  fq_arnoldi_stats* st = stats ? stats : &local;
  *st = fq_arnoldi_stats{};
  std::vector<void*> temp;
  struct Guard {
    std::vector<void*>* t;
    ~Guard() {
      for (void* p : *t) (void)hipFree(p);
    }
  } guard{&temp};

  Solver sv{};
  sv.op = op;
  sv.nev = nev;
  sv.ncv = o->ncv;
  sv.k = o->k;
  sv.max_restarts = o->max_restarts;
  sv.phi = phi;
  sv.s = s;
  sv.st = st;
  sv.seed = o->seed;
  if (o->poly_coeffs)
    for (int i = 0; i <= o->k; ++i) sv.coefs.push_back(zd(o->poly_coeffs[2 * i], o->poly_coeffs[2 * i + 1]));
  FQ_TRY(ensure_ws(op, o->ncv, nev, evecs_dev, &sv.ws, &temp));
  const size_t d = op->dim();

  // start vector
  if (o->v0_dev)
    FQ_HIP_CHECK(hipMemcpyAsync(sv.ws.V, o->v0_dev, d * sizeof(c128), hipMemcpyDeviceToDevice, s));
  else
    FQ_HIP_CHECK(launch_random(sv.ws.V, d, o->seed, s));
  double n0 = 0.0;
  FQ_TRY(normalize_col(sv.ws, 0, &n0, s));
  if (!(n0 > 0.0) || !std::isfinite(n0)) {
    set_error("start vector has zero or non-finite norm");
    return FQ_EINVAL;
  }

  PhaseResult res;
  fq_status status = FQ_OK;
  const bool mixed = o->filter_dtype == FQ_C64;
  if (!mixed) {
    FQ_TRY(sv.run(FQ_C128, 0.5 * o->tol, o->tol, true, o->max_restarts, probes_pay(op->dim(), o->k, 1), &res));
  } else {
    // complex64 phase: converge the Ritz estimates to the c64 level
    const double tol32 = std::max(o->tol, 2e-6);
    FQ_TRY(sv.run(FQ_C64, tol32, o->tol, false, o->max_restarts, probes_pay(op->dim(), o->k, 1), &res));
    double rmax = 0.0;
    for (double r : res.ritz.resid) rmax = std::max(rmax, r);
    if (o->refine && rmax > o->tol) {
      const double t_ref0 = now_s();
      // warm start: v0 = sum_i c_i y_i over the complex64 Ritz vectors
      std::vector<c128> cc;
      warm_start_coefs(o->seed, nev, &cc);
      FQ_HIP_CHECK(hipMemcpyAsync(sv.ws.qbuf, cc.data(), cc.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      FQ_HIP_CHECK(launch_basis_gemm(sv.ws.ritz, d, nev, sv.ws.qbuf, 1, sv.ws.V, d, d, s));
      FQ_TRY(normalize_col(sv.ws, 0, &n0, s));
      PhaseResult res2;
      res2.restarts = 0;
      if (o->refine_k > 0) sv.k = o->refine_k;
      const int budget = std::max(0, o->max_restarts - res.restarts);
      FQ_TRY(sv.run(FQ_C128, 0.5 * o->tol, o->tol, true, budget, true, &res2));
      res2.restarts += res.restarts;
      res = res2;
      st->t_refine = now_s() - t_ref0;
    }
  }
  st->n_restarts = res.restarts;

  // order by arc distance to the target, write outputs
  std::vector<int> order(nev);
  std::iota(order.begin(), order.end(), 0);
  const zd rot = std::polar(1.0, -phi);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return std::abs(std::arg(res.ritz.omega[a] * rot)) < std::abs(std::arg(res.ritz.omega[b] * rot));
  });
  int nconv = 0;
  double rmax = 0.0;
  for (int i = 0; i < nev; ++i) {
    const int j = order[i];
    if (evals_host) {
      evals_host[2 * i] = res.ritz.omega[j].real();
      evals_host[2 * i + 1] = res.ritz.omega[j].imag();
    }
    if (resid_host) resid_host[i] = res.ritz.resid[j];
    if (res.ritz.resid[j] <= o->tol) ++nconv;
    rmax = std::max(rmax, res.ritz.resid[j]);
  }
  if (evecs_dev) {
    // permute columns of the caller's buffer (it holds the Ritz vectors)
    bool identity = true;
    for (int i = 0; i < nev; ++i) identity = identity && order[i] == i;
    if (!identity) {
      c128* tmp = static_cast<c128*>(op->V);  // basis no longer needed
      for (int i = 0; i < nev; ++i)
        FQ_HIP_CHECK(hipMemcpyAsync(tmp + size_t(i) * d, sv.ws.ritz + size_t(order[i]) * d, d * sizeof(c128),
                                    hipMemcpyDeviceToDevice, s));
      FQ_HIP_CHECK(hipMemcpyAsync(sv.ws.ritz, tmp, size_t(nev) * d * sizeof(c128), hipMemcpyDeviceToDevice, s));
    }
  }
  FQ_HIP_CHECK(hipStreamSynchronize(s));
  st->nconv = nconv;
  st->max_residual = rmax;
  st->t_filter = sv.t_filter;
  st->t_restart = sv.t_restart;
  st->t_total = now_s() - t_start;
  if (nconv < nev) {
    set_error("not converged: " + std::to_string(nconv) + " of " + std::to_string(nev) + " pairs meet tol");
    status = FQ_NOT_CONVERGED;
  }
  return status;
}

}  // namespace fq

using namespace fq;

extern "C" {

fq_status arnoldi_eigs(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* opts, double* evals_host,
                       void* evecs_dev, double* resid_host, fq_arnoldi_stats* stats, void* hip_stream) {
  clear_error();
  if (!std::isfinite(phi)) {
    set_error("phi must be finite");
    return FQ_EINVAL;
  }
  return arnoldi_solve(op, nev, phi, opts, evals_host, evecs_dev, resid_host, stats,
                       static_cast<hipStream_t>(hip_stream));
}

fq_status arnoldi_eigs_batched(floquet_op* const* ops, int n_ops, const double* phis, int n_phi, int nev,
                               const fq_arnoldi_opts* opts, const int* k_per_op, double* evals_host,
                               void* const* evecs_dev, double* resid_host, fq_arnoldi_stats* stats,
                               void* hip_stream) {
  clear_error();
  return arnoldi_batched_solve(ops, n_ops, phis, n_phi, nev, opts, k_per_op, evals_host, evecs_dev, resid_host, stats,
                               static_cast<hipStream_t>(hip_stream));
}

fq_status fq_paper_parameters(int L, int nev, int* ncv_out, int* k_out) {
  clear_error();
  if (L < 2 || L > 30 || nev < 1 || !ncv_out || !k_out) {
    set_error("fq_paper_parameters: need 2 <= L <= 30, nev >= 1 and output pointers");
    return FQ_EINVAL;
  }
  *ncv_out = paper_ncv(L, nev);
  *k_out = paper_k(L, *ncv_out);
  return FQ_OK;
}

fq_status fq_host_schur(int n, double* a_host, double* z_host, double* w_host) {
  clear_error();
  if (n < 1 || !a_host || !z_host || !w_host) {
    set_error("fq_host_schur: bad arguments");
    return FQ_EINVAL;
  }
  ZMat A(n, n), Z;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const size_t e = size_t(j) * n + i;
      A(i, j) = zd(a_host[2 * e], a_host[2 * e + 1]);
    }
  if (!schur(A, Z)) {
    set_error("QR iteration did not converge");
    return FQ_ENUMERIC;
  }
  schur_sort(A, Z, n, [](const zd& x, const zd& y) { return std::abs(x) > std::abs(y); });
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const size_t e = size_t(j) * n + i;
      a_host[2 * e] = A(i, j).real();
      a_host[2 * e + 1] = A(i, j).imag();
      z_host[2 * e] = Z(i, j).real();
      z_host[2 * e + 1] = Z(i, j).imag();
    }
  for (int i = 0; i < n; ++i) {
    w_host[2 * i] = A(i, i).real();
    w_host[2 * i + 1] = A(i, i).imag();
  }
  return FQ_OK;
}

}  // extern "C"
