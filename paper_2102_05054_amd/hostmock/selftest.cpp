// Scenario driver of the host mock, built with the address and
// undefined-behaviour sanitizers: runs the Krylov-Schur driver through its C
// ABI on diagonal mock operators and checks the outcome of each path
// (convergence to the known pairs, restarts, the mixed-precision hand-over,
// the block solver, non-convergence, NaN detection, out-of-memory, invariant
// subspaces, the paper's parameter rule).  Exit status 0 when every scenario
// passes; a sanitizer report aborts the run.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/floquet.h"

extern "C" {
fq_status fq_mock_create(int L, const double* phases, floquet_op** out);
fq_status fq_mock_destroy(floquet_op* op);
void fq_mock_set_free_bytes(unsigned long long bytes);
void fq_mock_set_nan_at(long long app);
}

namespace {

int g_fail = 0;

void expect(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++g_fail;
}

double arc(std::complex<double> w, double phi) { return std::abs(std::arg(w * std::polar(1.0, -phi))); }

std::vector<double> random_phases(int L, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> u(-M_PI, M_PI);
  std::vector<double> p(size_t(1) << L);
  for (double& x : p) x = u(rng);
  return p;
}

fq_arnoldi_opts opts(int k, int ncv, fq_dtype dt, int block, int max_restarts = 200) {
  fq_arnoldi_opts o{};
  o.k = k;
  o.ncv = ncv;
  o.tol = 1e-10;
  o.max_restarts = max_restarts;
  o.filter_dtype = dt;
  o.refine = 1;
  o.seed = 7;
  o.block = block;
  return o;
}

struct Result {
  fq_status st;
  std::vector<std::complex<double>> ev;
  std::vector<double> res;
  fq_arnoldi_stats stats;
};

Result solve(const std::vector<double>& ph, int L, int nev, double phi, const fq_arnoldi_opts& o) {
  floquet_op* op = nullptr;
  fq_mock_create(L, ph.data(), &op);
  Result r;
  std::vector<double> ev(2 * nev), res(nev);
  r.stats = fq_arnoldi_stats{};
  r.st = arnoldi_eigs(op, nev, phi, &o, ev.data(), nullptr, res.data(), &r.stats, nullptr);
  for (int i = 0; i < nev; ++i) r.ev.emplace_back(ev[2 * i], ev[2 * i + 1]);
  r.res = res;
  fq_mock_destroy(op);
  return r;
}

// the nev eigenvalues of diag(e^{i ph}) closest to e^{i phi}, nearest first
std::vector<std::complex<double>> exact(const std::vector<double>& ph, int nev, double phi) {
  std::vector<std::complex<double>> w;
  for (double t : ph) w.push_back(std::polar(1.0, t));
  std::stable_sort(w.begin(), w.end(), [&](auto a, auto b) { return arc(a, phi) < arc(b, phi); });
  w.resize(nev);
  return w;
}

double max_diff(const std::vector<std::complex<double>>& a, const std::vector<std::complex<double>>& b) {
  double m = 0.0;
  for (size_t i = 0; i < a.size(); ++i) m = std::max(m, std::abs(a[i] - b[i]));
  return m;
}

}  // namespace

int main() {
  const int L = 8, nev = 6;
  const double phi = 1.0;
  const auto ph = random_phases(L, 11);
  const auto want = exact(ph, nev, phi);

  for (int block : {1, 2, 4})
    for (fq_dtype dt : {FQ_C128, FQ_C64}) {
      const Result r = solve(ph, L, nev, phi, opts(30, 24, dt, block));
      char msg[160];
      std::snprintf(msg, sizeof msg, "block %d %s: status %d, eigenvalue error %.2e, restarts %d", block,
                    dt == FQ_C64 ? "c64+refine" : "c128", r.st, max_diff(r.ev, want), r.stats.n_restarts);
      expect(r.st == FQ_OK && max_diff(r.ev, want) < 1e-12 &&
                 *std::max_element(r.res.begin(), r.res.end()) <= 1e-10,
             msg);
    }
  {
    // a small Krylov space: several restarts before convergence
    const Result r = solve(ph, L, nev, phi, opts(12, 14, FQ_C128, 1));
    expect(r.st == FQ_OK && r.stats.n_restarts >= 2 && max_diff(r.ev, want) < 1e-12, "restarted solve converges");
  }
  {
    // no restarts allowed: partial results with nconv = pairs meeting tol
    const Result r = solve(ph, L, nev, phi, opts(2, 10, FQ_C128, 1, 0));
    int n = 0;
    for (double x : r.res) n += x <= 1e-10;
    expect(r.st == FQ_NOT_CONVERGED && r.stats.nconv == n && n < nev, "not converged: partial nconv reported");
  }
  for (int block : {1, 4}) {
    // a NaN in the 5th filter output
    fq_mock_set_nan_at(5);
    const Result r = solve(ph, L, nev, phi, opts(30, 24, FQ_C128, block));
    fq_mock_set_nan_at(-1);
    expect(r.st == FQ_ENUMERIC, block == 1 ? "NaN in the filter -> FQ_ENUMERIC" : "NaN in a block filter -> FQ_ENUMERIC");
  }
  for (int block : {1, 4}) {
    // less free memory than the workspace needs
    fq_mock_set_free_bytes(1ull << 20);
    const Result r = solve(random_phases(12, 3), 12, 10, 0.0, opts(10, 100, FQ_C128, block));
    fq_mock_set_free_bytes(64ull << 30);
    expect(r.st == FQ_ENOMEM, block == 1 ? "oversized workspace -> FQ_ENOMEM" : "oversized block workspace -> FQ_ENOMEM");
  }
  {
    // ncv = d: the Krylov space becomes the whole space and is analysed exactly
    const auto p3 = random_phases(3, 5);
    const Result r = solve(p3, 3, 3, 0.3, opts(4, 8, FQ_C128, 1));
    expect(r.st == FQ_OK && max_diff(r.ev, exact(p3, 3, 0.3)) < 1e-12, "ncv = d: exact invariant space");
  }
  {
    // four distinct eigenvalues: the space is invariant at dimension 4 >= nev = 3
    std::vector<double> p6(64);
    for (size_t s = 0; s < p6.size(); ++s) p6[s] = 0.4 * double(s % 4);
    const Result r = solve(p6, 6, 3, 0.0, opts(6, 20, FQ_C128, 1));
    bool on = true;
    for (auto w : r.ev) {
      double best = 1e9;
      for (int j = 0; j < 4; ++j) best = std::min(best, std::abs(w - std::polar(1.0, 0.4 * j)));
      on = on && best < 1e-12;
    }
    expect(r.st == FQ_OK && on, "degenerate spectrum: invariant space of dimension 4 gives exact pairs");
    // two distinct eigenvalues, nev = 3: invariant below nev
    for (size_t s = 0; s < p6.size(); ++s) p6[s] = 0.4 * double(s % 2);
    const Result r2 = solve(p6, 6, 3, 0.0, opts(6, 20, FQ_C128, 1));
    expect(r2.st == FQ_ENUMERIC, "invariant space smaller than nev -> FQ_ENUMERIC");
  }
  {
    // paper rule: ncv = 0 and k = 0 select floor(2^(L/2+1)) and floor(0.8 * 2^(L+1) / ncv)
    const auto p10 = random_phases(10, 9);
    const Result r = solve(p10, 10, 8, 2.0, opts(0, 0, FQ_C128, 1));
    const long long k = (long long)std::floor(0.8 * 2048.0 / 64.0);
    expect(r.st == FQ_OK && max_diff(r.ev, exact(p10, 8, 2.0)) < 1e-12 &&
               (r.stats.n_U_apps - 8) == k * r.stats.n_filter_apps,
           "k = 0, ncv = 0: the paper's rule");
    int ncv = 0, kk = 0;
    fq_paper_parameters(4, 8, &ncv, &kk);
    expect(ncv == 15 && kk == 1, "paper rule keeps ncv below d");
  }
  std::printf("%s: %d failure(s)\n", g_fail ? "FAILED" : "PASSED", g_fail);
  return g_fail ? 1 : 0;
}
