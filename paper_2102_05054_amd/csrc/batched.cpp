// Lockstep batched Krylov-Schur (arnoldi_eigs_batched).
//
// Many independent eigenproblems (disorder realisations, targets phi, chain
// lengths) are solved together.  Kicked-Ising problems of one chain length,
// kick form and filter order form a bucket that advances in lockstep: every
// Arnoldi step of the bucket is one batched filter (one launch per Horner
// pass for all problems, or one launch for all k steps when a workgroup holds
// a whole state) and one batched CGS2.  The host steps in only where the
// single-problem solver does (end of a restart cycle, early convergence
// probes), and analyses the projected matrices of all problems at such a
// point on worker threads.  Each problem follows the single-problem algorithm
// of krylov.cpp (complex64 phase, FP64 warm-started refinement, the same
// restart and stopping rules and the same reduction order of every
// projection); only the interleaving of problems differs.
//
// With graph capture on (fq_set_graph_capture, the default), the k + 1 pass
// launches of a lockstep filter are captured once per (precision, range of
// active problems, filter order) into a HIP graph and replayed at every
// Arnoldi step with that range; the solve then runs on a stream of its own
// (the caller's stream is drained first and the call returns when the work
// is done, as without graphs).  Graphs hold kernel launches only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
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

#define FQ_TRY(expr)                \
  do {                              \
    fq_status st__ = (expr);        \
    if (st__ != FQ_OK) return st__; \
  } while (0)

enum class Ph { C64, C128, Done };
enum class Act { None, RitzCheck, RitzFull, Restart, PhaseEnd };

struct Prob {
  floquet_op* op = nullptr;
  double phi = 0.0;
  size_t out = 0;  // output slot (op index * n_phi + phi index)
  void* evecs = nullptr;
  // device buffers (inside the bucket's allocation, except evecs)
  c128 *V = nullptr, *w = nullptr, *ritz = nullptr, *psi64 = nullptr, *partial = nullptr;
  c64 *psi32 = nullptr, *x32 = nullptr;
  double *slots = nullptr, *small = nullptr;
  double* hslots = nullptr;  // pinned host mirror of slots
  const PhaseTables* tab_phi = nullptr;
  const PhaseTables* tab0 = nullptr;
  // solver state (as in the single-problem solver's run())
  Ph ph = Ph::C64;
  bool check_true = false, early = false;
  double tolg = 0.0;
  int budget = 0, restarts = 0, restarts_before = 0;
  int j = 0, kk = 0, copied = 0;
  ZMat H;
  double best = 1e300;
  int stall = 0;
  // decision scratch
  Act act = Act::None;
  bool all = false, oob = false, full = false, phase_converged = false;
  int mm = 0;
  ZMat T, Z, X;
  std::vector<zd> bz;
  std::vector<zd> omega;
  std::vector<double> resid;
  fq_arnoldi_stats st{};
  double t_filter0 = 0.0, t_restart0 = 0.0, t_ref0 = 0.0;
  fq_status err = FQ_OK;
  std::string msg;
};

struct Seg {
  Ph ph;
  int j;
  unsigned start, n;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Bucket {
  int L = 0, k = 0;
  int k_ref = 0;  // filter order of the FP64 refinement
  bool sw = false;
  std::vector<Prob> P;
  size_t d = 0;
  unsigned nblk = 0;
  int ncv = 0, nev = 0, sd = 0, ldp = 0, p_keep = 0, check_every = 0, qcols = 0;
  const fq_arnoldi_opts* o = nullptr;
  bool mixed = false;
  hipStream_t s = nullptr;
  // device
  void* mem = nullptr;
  KDesc* kd = nullptr;
  KiDesc<float>* f32 = nullptr;
  KiDesc<double>* f64 = nullptr;
  KiDesc<double>* app = nullptr;
  int *list = nullptr, *aux = nullptr, *ident = nullptr;
  GemmDesc* gemm = nullptr;
  RDesc* rd = nullptr;
  c128* q = nullptr;
  double* res = nullptr;
  // pinned host staging
  void* hmem = nullptr;
  int *list_h = nullptr, *aux_h = nullptr;
  GemmDesc* gemm_h = nullptr;
  RDesc* rd_h = nullptr;
  c128* q_h = nullptr;
  double* res_h = nullptr;
  KiDesc<double>* app_h = nullptr;
  bool staging_busy = false;
  // shapes
  KiBatchShape sh32, sh64, sh_app;
  bool have32 = false, have64 = false;
  // timing of the batch
  double t_filter = 0.0, t_restart = 0.0, t_begin = 0.0;
  // replayable filters (graph capture on): key (complex64?, first list slot,
  // problems, filter order)
  bool graphs = false;
  struct Graph {
    bool c64;
    unsigned pos0, n;
    int k;
    hipGraphExec_t exec;
  };
  std::vector<Graph> gcache;

  ~Bucket() {
    // replays may still be in flight on an early return
    if (!gcache.empty()) (void)hipStreamSynchronize(s);
    for (Graph& g : gcache) (void)hipGraphExecDestroy(g.exec);
    if (mem) (void)hipFree(mem);
    if (hmem) (void)hipHostFree(hmem);
  }

  fq_status sync() {
    FQ_HIP_CHECK(hipStreamSynchronize(s));
    staging_busy = false;
    return FQ_OK;
  }
  // the host is about to write pinned staging memory: wait for pending copies
  fq_status staging() {
    if (staging_busy) return sync();
    return FQ_OK;
  }
  fq_status upload(void* dst, const void* src, size_t bytes) {
    FQ_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    staging_busy = true;
    return FQ_OK;
  }
  BatchArgs args(const int* lst, unsigned n) const {
    BatchArgs a;
    a.kd = kd;
    a.list = lst;
    a.n = n;
    a.d = d;
    a.nblk = nblk;
    a.ldp = ldp;
    a.slot_doubles = sd;
    a.ncv = ncv;
    return a;
  }
};

// ---------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------
size_t prob_bytes(size_t d, int ncv, int nev, bool own_ritz, unsigned nblk, int sd, int qcols) {
  size_t b = 0;
  b += align_up(d * sizeof(c128) * size_t(ncv + 1));  // V
  b += align_up(d * sizeof(c128));                     // w
  b += align_up(d * sizeof(c128));                     // psi64
  b += 2 * align_up(d * sizeof(c64));                  // psi32, x32
  if (own_ritz) b += align_up(d * sizeof(c128) * size_t(nev));
  b += align_up(std::max<size_t>(size_t(nblk) * (ncv + 1), 2 * size_t(nblk)) * sizeof(c128));  // partial
  b += align_up(size_t(ncv + 1) * sd * sizeof(double));                                        // slots
  b += align_up(16 * sizeof(double));                                                          // small
  b += align_up(size_t(ncv) * qcols * sizeof(c128));                                           // q
  b += align_up(size_t(nev) * 4 * sizeof(double));                                             // res
  b += 512;                                                                                    // descriptors
  b += align_up(size_t(nev) * sizeof(KiDesc<double>));
  return b;
}

fq_status setup(Bucket& B) {
  const size_t np = B.P.size();
  const size_t d = B.d;
  // device block
  size_t total = 0;
  auto take = [&](size_t bytes) {
    const size_t off = total;
    total += align_up(bytes);
    return off;
  };
  const size_t o_kd = take(np * sizeof(KDesc));
  const size_t o_f32 = take(np * sizeof(KiDesc<float>));
  const size_t o_f64 = take(np * sizeof(KiDesc<double>));
  const size_t o_app = take(np * size_t(B.nev) * sizeof(KiDesc<double>));
  const size_t o_list = take(np * sizeof(int));
  const size_t o_aux = take(np * sizeof(int));
  const size_t o_ident = take(np * sizeof(int));
  const size_t o_gemm = take(np * sizeof(GemmDesc));
  const size_t o_rd = take(np * sizeof(RDesc));
  const size_t o_q = take(np * size_t(B.ncv) * B.qcols * sizeof(c128));
  const size_t o_res = take(np * size_t(B.nev) * 4 * sizeof(double));
  std::vector<size_t> o_V(np), o_w(np), o_p64(np), o_p32(np), o_x32(np), o_ritz(np), o_part(np), o_slots(np),
      o_small(np);
  const size_t part_elems = std::max<size_t>(size_t(B.nblk) * B.ldp, 2 * size_t(B.nblk));
  for (size_t i = 0; i < np; ++i) {
    o_V[i] = take(d * sizeof(c128) * size_t(B.ncv + 1));
    o_w[i] = take(d * sizeof(c128));
    o_p64[i] = take(d * sizeof(c128));
    o_p32[i] = take(d * sizeof(c64));
    o_x32[i] = take(d * sizeof(c64));
    o_ritz[i] = B.P[i].evecs ? size_t(-1) : take(d * sizeof(c128) * size_t(B.nev));
    o_part[i] = take(part_elems * sizeof(c128));
    o_slots[i] = take(size_t(B.ncv + 1) * B.sd * sizeof(double));
    o_small[i] = take(16 * sizeof(double));
  }
  size_t freeb = 0, totalb = 0;
  FQ_HIP_CHECK(hipMemGetInfo(&freeb, &totalb));
  if (total + (size_t(1) << 28) > freeb) {
    set_error("batched Krylov workspace of " + std::to_string(total >> 20) + " MiB does not fit in free device memory");
    return FQ_ENOMEM;
  }
  if (hipMalloc(&B.mem, total) != hipSuccess) {
    set_error("hipMalloc of the batched Krylov workspace failed");
    return FQ_ENOMEM;
  }
  char* base = static_cast<char*>(B.mem);
  FQ_HIP_CHECK(hipMemsetAsync(B.mem, 0, total, B.s));
  B.kd = reinterpret_cast<KDesc*>(base + o_kd);
  B.f32 = reinterpret_cast<KiDesc<float>*>(base + o_f32);
  B.f64 = reinterpret_cast<KiDesc<double>*>(base + o_f64);
  B.app = reinterpret_cast<KiDesc<double>*>(base + o_app);
  B.list = reinterpret_cast<int*>(base + o_list);
  B.aux = reinterpret_cast<int*>(base + o_aux);
  B.ident = reinterpret_cast<int*>(base + o_ident);
  B.gemm = reinterpret_cast<GemmDesc*>(base + o_gemm);
  B.rd = reinterpret_cast<RDesc*>(base + o_rd);
  B.q = reinterpret_cast<c128*>(base + o_q);
  B.res = reinterpret_cast<double*>(base + o_res);
  for (size_t i = 0; i < np; ++i) {
    Prob& p = B.P[i];
    p.V = reinterpret_cast<c128*>(base + o_V[i]);
    p.w = reinterpret_cast<c128*>(base + o_w[i]);
    p.psi64 = reinterpret_cast<c128*>(base + o_p64[i]);
    p.psi32 = reinterpret_cast<c64*>(base + o_p32[i]);
    p.x32 = reinterpret_cast<c64*>(base + o_x32[i]);
    p.ritz = p.evecs ? static_cast<c128*>(p.evecs) : reinterpret_cast<c128*>(base + o_ritz[i]);
    p.partial = reinterpret_cast<c128*>(base + o_part[i]);
    p.slots = reinterpret_cast<double*>(base + o_slots[i]);
    p.small = reinterpret_cast<double*>(base + o_small[i]);
  }
  // pinned host block
  size_t htotal = 0;
  auto htake = [&](size_t bytes) {
    const size_t off = htotal;
    htotal += align_up(bytes);
    return off;
  };
  const size_t h_list = htake(np * sizeof(int));
  const size_t h_aux = htake(np * sizeof(int));
  const size_t h_gemm = htake(np * sizeof(GemmDesc));
  const size_t h_rd = htake(np * sizeof(RDesc));
  const size_t h_q = htake(np * size_t(B.ncv) * B.qcols * sizeof(c128));
  const size_t h_res = htake(np * size_t(B.nev) * 4 * sizeof(double));
  const size_t h_app = htake(np * size_t(B.nev) * sizeof(KiDesc<double>));
  const size_t h_slots = htake(np * size_t(B.ncv + 1) * B.sd * sizeof(double));
  FQ_HIP_CHECK(hipHostMalloc(&B.hmem, htotal, hipHostMallocDefault));
  char* hb = static_cast<char*>(B.hmem);
  B.list_h = reinterpret_cast<int*>(hb + h_list);
  B.aux_h = reinterpret_cast<int*>(hb + h_aux);
  B.gemm_h = reinterpret_cast<GemmDesc*>(hb + h_gemm);
  B.rd_h = reinterpret_cast<RDesc*>(hb + h_rd);
  B.q_h = reinterpret_cast<c128*>(hb + h_q);
  B.res_h = reinterpret_cast<double*>(hb + h_res);
  B.app_h = reinterpret_cast<KiDesc<double>*>(hb + h_app);
  for (size_t i = 0; i < np; ++i)
    B.P[i].hslots = reinterpret_cast<double*>(hb + h_slots) + i * size_t(B.ncv + 1) * B.sd;
  // static descriptors
  std::vector<KDesc> kd(np);
  std::vector<KiDesc<float>> f32(np);
  std::vector<KiDesc<double>> f64(np);
  std::vector<int> ident(np);
  for (size_t i = 0; i < np; ++i) {
    const Prob& p = B.P[i];
    kd[i] = KDesc{p.V, p.w, p.partial, p.slots, p.small};
    f32[i] = KiDesc<float>{p.psi32, p.x32, p.tab_phi->tlo32, p.tab_phi->thi32, p.op->w, 0.0};
    f64[i] = KiDesc<double>{p.psi64, p.w, p.tab_phi->tlo64, p.tab_phi->thi64, p.op->w, 0.0};
    ident[i] = static_cast<int>(i);
  }
  FQ_HIP_CHECK(hipMemcpyAsync(B.kd, kd.data(), np * sizeof(KDesc), hipMemcpyHostToDevice, B.s));
  FQ_HIP_CHECK(hipMemcpyAsync(B.f32, f32.data(), np * sizeof(KiDesc<float>), hipMemcpyHostToDevice, B.s));
  FQ_HIP_CHECK(hipMemcpyAsync(B.f64, f64.data(), np * sizeof(KiDesc<double>), hipMemcpyHostToDevice, B.s));
  FQ_HIP_CHECK(hipMemcpyAsync(B.ident, ident.data(), np * sizeof(int), hipMemcpyHostToDevice, B.s));
  FQ_TRY(B.sync());  // the host vectors above go out of scope
  const std::vector<KiBatchShape> app = ki_batch_candidates(B.L, B.sw, false);
  if (app.empty()) {
    set_error("no kicked-Ising tile shape for L = " + std::to_string(B.L));
    return FQ_EINVAL;
  }
  B.sh_app = app[0];
  return FQ_OK;
}

void fresh_phase(Bucket& B, Prob& p, Ph ph, bool check_true, bool early, double tolg, int budget) {
  p.ph = ph;
  p.check_true = check_true;
  p.early = early;
  p.tolg = tolg;
  p.budget = budget;
  p.restarts = 0;
  p.j = p.kk = p.copied = 0;
  p.H = ZMat(B.ncv + 1, B.ncv);
  p.best = 1e300;
  p.stall = 0;
}

// ---------------------------------------------------------------------------
// The batched filter of the problems list[pos0 .. pos0 + n), replayed from a
// captured graph when graph capture is on
// ---------------------------------------------------------------------------
std::atomic<int> g_graph_capture{1};

template <typename Real>
fq_status run_filter(Bucket& B, const KiBatchShape& sh, int k, const KiDesc<Real>* desc, unsigned pos0, unsigned n) {
  const bool c64 = sizeof(Real) == 4;
  // the single-workgroup form is one launch for all k steps already
  if (!B.graphs || sh.single || k < 8) return ki_batch_filter<Real>(sh, k, desc, B.list + pos0, n, B.s);
  for (const Bucket::Graph& g : B.gcache)
    if (g.c64 == c64 && g.pos0 == pos0 && g.n == n && g.k == k) {
      FQ_HIP_CHECK(hipGraphLaunch(g.exec, B.s));
      return FQ_OK;
    }
  // capture: kernel launches only (the shape is tuned and its launch
  // attributes set by the eager runs of the autotuner)
  FQ_HIP_CHECK(hipStreamBeginCapture(B.s, hipStreamCaptureModeThreadLocal));
  const fq_status st = ki_batch_filter<Real>(sh, k, desc, B.list + pos0, n, B.s);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(B.s, &graph);
  if (st != FQ_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess || !graph) {
    set_error(std::string("capture of the batched filter failed: ") + hipGetErrorString(ec));
    return FQ_EDEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    set_error(std::string("instantiation of the batched filter graph failed: ") + hipGetErrorString(ei));
    return FQ_EDEVICE;
  }
  // a handful of active ranges per bucket; keep the most recent ones
  if (B.gcache.size() >= 8) {
    (void)hipGraphExecDestroy(B.gcache.front().exec);
    B.gcache.erase(B.gcache.begin());
  }
  B.gcache.push_back(Bucket::Graph{c64, pos0, n, k, exec});
  FQ_HIP_CHECK(hipGraphLaunch(exec, B.s));
  return FQ_OK;
}

// ---------------------------------------------------------------------------
// One Arnoldi step of every active problem
// ---------------------------------------------------------------------------
fq_status step(Bucket& B, const std::vector<Seg>& segs) {
  for (Ph ph : {Ph::C64, Ph::C128}) {
    unsigned pos0 = ~0u, pos1 = 0;
    for (const Seg& g : segs) {
      if (g.ph != ph) continue;
      pos0 = std::min(pos0, g.start);
      pos1 = std::max(pos1, g.start + g.n);
      if (ph == Ph::C64)
        FQ_HIP_CHECK(launch_b_cast_in<float>(B.args(B.list + g.start, g.n), B.f32, g.j, B.s));
      else
        FQ_HIP_CHECK(launch_b_cast_in<double>(B.args(B.list + g.start, g.n), B.f64, g.j, B.s));
    }
    if (pos0 >= pos1) continue;
    const unsigned n = pos1 - pos0;
    if (ph == Ph::C64) {
      FQ_TRY(run_filter<float>(B, B.sh32, B.k, B.f32, pos0, n));
      FQ_HIP_CHECK(launch_b_cast_out(B.args(B.list + pos0, n), B.f32, B.s));
    } else {
      FQ_TRY(run_filter<double>(B, B.sh64, B.mixed ? B.k_ref : B.k, B.f64, pos0, n));
    }
  }
  for (const Seg& g : segs) {
    const BatchArgs a = B.args(B.list + g.start, g.n);
    const int nc = g.j + 1;
    FQ_HIP_CHECK(launch_b_dots(a, nc, B.s));
    FQ_HIP_CHECK(launch_b_reduce_slot(a, nc, g.j, 0, B.s));
    FQ_HIP_CHECK(launch_b_update(a, nc, g.j, 0, B.s));
    FQ_HIP_CHECK(launch_b_reduce_slot(a, nc, g.j, 1, B.s));
    FQ_HIP_CHECK(launch_b_update(a, nc, g.j, 1, B.s));
    FQ_HIP_CHECK(launch_b_reduce_norm(a, g.j, B.s));
    FQ_HIP_CHECK(launch_b_scale_next(a, g.j, B.s));
  }
  return FQ_OK;
}

// ---------------------------------------------------------------------------
// Host analysis of one problem at a decision point (worker thread)
// ---------------------------------------------------------------------------
void analyse_one(Bucket& B, Prob& p) {
  const int mm = p.j;
  const int ncv = B.ncv;
  double hn = 0.0;
  for (int jj = p.copied; jj < mm; ++jj) {
    const double* sl = p.hslots + size_t(jj) * B.sd;
    for (int i = 0; i <= jj; ++i) {
      p.H(i, jj) = zd(sl[2 * i] + sl[2 * (ncv + 1) + 2 * i], sl[2 * i + 1] + sl[2 * (ncv + 1) + 2 * i + 1]);
      hn = std::max(hn, std::abs(p.H(i, jj)));
    }
    const double beta = sl[4 * (ncv + 1)];
    if (!std::isfinite(beta) || !std::isfinite(hn)) {
      p.err = FQ_ENUMERIC;
      p.msg = "non-finite value in the Arnoldi process (filter output overflow?)";
      return;
    }
    if (beta <= 1e-14 * std::max(hn, 1e-300)) {
      p.err = FQ_ENUMERIC;
      p.msg = "Arnoldi breakdown: the Krylov space became invariant before ncv vectors";
      return;
    }
    p.H(jj + 1, jj) = beta;
  }
  p.copied = mm;
  int nconv = 0;
  double worst = 0.0;
  const fq_status st = analyse_decomposition(p.H, mm, std::max(B.p_keep, B.nev), B.nev, p.tolg, &p.T, &p.Z, &p.bz,
                                             &p.X, &nconv, &worst);
  if (st != FQ_OK) {
    p.err = st;
    p.msg = floquet_last_error();
    return;
  }
  p.mm = mm;
  p.all = nconv >= B.nev;
  p.full = mm == B.ncv;
  if (!p.full) {
    p.act = p.all ? Act::RitzCheck : Act::None;
    return;
  }
  p.oob = p.restarts >= p.budget;
  if (worst < 0.5 * p.best) {
    p.best = worst;
    p.stall = 0;
  } else {
    ++p.stall;
  }
  const bool stalled = !p.check_true && p.stall >= 3 && worst < 1e-3;
  p.act = (p.all || p.oob || stalled) ? Act::RitzFull : Act::Restart;
}

template <class F>
void parallel_for(const std::vector<int>& items, F f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = std::min<unsigned>({static_cast<unsigned>(items.size()), hw, 16u});
  if (nt <= 1) {
    for (int i : items) f(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> th;
  th.reserve(nt);
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (;;) {
        const size_t i = next.fetch_add(1);
        if (i >= items.size()) break;
        f(items[i]);
      }
    });
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------------------
// Ritz vectors, omega = <y|U|y>, residuals (FP64) for the problems R
// ---------------------------------------------------------------------------
fq_status ritz(Bucket& B, const std::vector<int>& R) {
  const unsigned n = static_cast<unsigned>(R.size());
  const int nev = B.nev;
  FQ_TRY(B.staging());
  for (unsigned r = 0; r < n; ++r) {
    Prob& p = B.P[R[r]];
    c128* qh = B.q_h + size_t(r) * B.ncv * B.qcols;
    for (int c = 0; c < nev; ++c)
      for (int i = 0; i < p.mm; ++i) qh[size_t(i) * nev + c] = mk<double>(p.X(i, c).real(), p.X(i, c).imag());
    B.gemm_h[r] = GemmDesc{p.V, p.ritz, B.q + size_t(r) * B.ncv * B.qcols, B.d, p.mm, nev};
    B.rd_h[r] = RDesc{p.ritz, p.w, p.partial, B.res + size_t(r) * nev * 4};
    for (int i = 0; i < nev; ++i)
      B.app_h[size_t(i) * n + r] =
          KiDesc<double>{p.ritz + size_t(i) * B.d, p.w, p.tab0->tlo64, p.tab0->thi64, p.op->w, 0.0};
  }
  FQ_TRY(B.upload(B.q, B.q_h, size_t(n) * B.ncv * B.qcols * sizeof(c128)));
  FQ_TRY(B.upload(B.gemm, B.gemm_h, n * sizeof(GemmDesc)));
  FQ_TRY(B.upload(B.rd, B.rd_h, n * sizeof(RDesc)));
  FQ_TRY(B.upload(B.app, B.app_h, size_t(n) * nev * sizeof(KiDesc<double>)));
  FQ_HIP_CHECK(launch_b_basis_gemm(B.gemm, n, B.d, B.s, nev));
  for (int i = 0; i < nev; ++i) {
    FQ_TRY(ki_batch_apply<double>(B.sh_app, B.app + size_t(i) * n, B.ident, n, B.s));
    FQ_HIP_CHECK(launch_r_rayleigh(B.rd, n, i, B.d, B.s));
  }
  FQ_HIP_CHECK(hipMemcpyAsync(B.res_h, B.res, size_t(n) * nev * 4 * sizeof(double), hipMemcpyDeviceToHost, B.s));
  FQ_TRY(B.sync());
  for (unsigned r = 0; r < n; ++r) {
    Prob& p = B.P[R[r]];
    p.omega.assign(nev, zd(0, 0));
    p.resid.assign(nev, 0.0);
    const double* o = B.res_h + size_t(r) * nev * 4;
    for (int i = 0; i < nev; ++i) {
      p.omega[i] = zd(o[4 * i], o[4 * i + 1]);
      p.resid[i] = o[4 * i + 2];
      if (!std::isfinite(o[4 * i]) || !std::isfinite(o[4 * i + 1]) || !std::isfinite(o[4 * i + 2])) {
        p.err = FQ_ENUMERIC;
        p.msg = "non-finite Ritz value or residual";
      }
    }
    p.st.n_U_apps += nev;
  }
  return FQ_OK;
}

// ---------------------------------------------------------------------------
// Restart: V_q <- V_q Z_p, v_p <- v_m; projected matrix to Schur form
// ---------------------------------------------------------------------------
fq_status restart(Bucket& B, const std::vector<int>& S) {
  const unsigned n = static_cast<unsigned>(S.size());
  const int m = B.ncv, p_keep = B.p_keep;
  FQ_TRY(B.staging());
  for (unsigned r = 0; r < n; ++r) {
    Prob& p = B.P[S[r]];
    c128* qh = B.q_h + size_t(r) * B.ncv * B.qcols;
    for (int c = 0; c < p_keep; ++c)
      for (int i = 0; i < m; ++i) qh[size_t(i) * p_keep + c] = mk<double>(p.Z(i, c).real(), p.Z(i, c).imag());
    B.gemm_h[r] = GemmDesc{p.V, p.V, B.q + size_t(r) * B.ncv * B.qcols, B.d, m, p_keep};
    B.aux_h[r] = S[r];
  }
  FQ_TRY(B.upload(B.q, B.q_h, size_t(n) * B.ncv * B.qcols * sizeof(c128)));
  FQ_TRY(B.upload(B.gemm, B.gemm_h, n * sizeof(GemmDesc)));
  FQ_TRY(B.upload(B.aux, B.aux_h, n * sizeof(int)));
  FQ_HIP_CHECK(launch_b_basis_gemm(B.gemm, n, B.d, B.s, p_keep));
  FQ_HIP_CHECK(launch_b_copy_col(B.args(B.aux, n), m, p_keep, B.s));
  for (int qi : S) {
    Prob& p = B.P[qi];
    ZMat Hn(m + 1, m);
    for (int jj = 0; jj < p_keep; ++jj) {
      for (int i = 0; i <= jj; ++i) Hn(i, jj) = p.T(i, jj);
      Hn(p_keep, jj) = p.bz[jj];
    }
    p.H = Hn;
    p.kk = p.j = p.copied = p_keep;
    ++p.restarts;
  }
  return FQ_OK;
}

// ---------------------------------------------------------------------------
// Final output of one problem
// ---------------------------------------------------------------------------
struct Out {
  double* evals;
  double* resid;
  fq_arnoldi_stats* stats;
  double tol;
};

fq_status finish(Bucket& B, Prob& p, const Out& out) {
  const int nev = B.nev;
  std::vector<int> order(nev);
  std::iota(order.begin(), order.end(), 0);
  const zd rot = std::polar(1.0, -p.phi);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return std::abs(std::arg(p.omega[a] * rot)) < std::abs(std::arg(p.omega[b] * rot));
  });
  int nconv = 0;
  double rmax = 0.0;
  for (int i = 0; i < nev; ++i) {
    const int jx = order[i];
    out.evals[2 * nev * p.out + 2 * i] = p.omega[jx].real();
    out.evals[2 * nev * p.out + 2 * i + 1] = p.omega[jx].imag();
    if (out.resid) out.resid[nev * p.out + i] = p.resid[jx];
    if (p.resid[jx] <= out.tol) ++nconv;
    rmax = std::max(rmax, p.resid[jx]);
  }
  if (p.evecs) {
    bool identity = true;
    for (int i = 0; i < nev; ++i) identity = identity && order[i] == i;
    if (!identity) {
      // the basis is no longer needed: stage the permuted vectors there
      for (int i = 0; i < nev; ++i)
        FQ_HIP_CHECK(hipMemcpyAsync(p.V + size_t(i) * B.d, p.ritz + size_t(order[i]) * B.d, B.d * sizeof(c128),
                                    hipMemcpyDeviceToDevice, B.s));
      FQ_HIP_CHECK(
          hipMemcpyAsync(p.ritz, p.V, size_t(nev) * B.d * sizeof(c128), hipMemcpyDeviceToDevice, B.s));
    }
  }
  p.st.nconv = nconv;
  p.st.max_residual = rmax;
  p.st.n_restarts = p.restarts_before + p.restarts;
  p.st.t_filter = B.t_filter - p.t_filter0;
  p.st.t_restart = B.t_restart - p.t_restart0;
  p.st.t_total = now_s() - B.t_begin;
  if (p.t_ref0 > 0.0) p.st.t_refine = now_s() - p.t_ref0;
  if (nconv < nev) {
    p.err = FQ_NOT_CONVERGED;
    p.msg = "not converged: " + std::to_string(nconv) + " of " + std::to_string(nev) + " pairs meet tol";
  }
  p.ph = Ph::Done;
  return FQ_OK;
}

// The problems W leave the complex64 phase: FP64 warm start
// v0 = sum_i c_i y_i from their Ritz vectors, then FP64 Krylov-Schur with
// early convergence checks.
fq_status start_refine(Bucket& B, const std::vector<int>& W) {
  const unsigned n = static_cast<unsigned>(W.size());
  std::vector<c128> cc;
  warm_start_coefs(B.o->seed, B.nev, &cc);
  FQ_TRY(B.staging());
  for (unsigned r = 0; r < n; ++r) {
    Prob& p = B.P[W[r]];
    c128* qh = B.q_h + size_t(r) * B.ncv * B.qcols;
    std::copy(cc.begin(), cc.end(), qh);
    B.gemm_h[r] = GemmDesc{p.ritz, p.V, B.q + size_t(r) * B.ncv * B.qcols, B.d, B.nev, 1};
    B.aux_h[r] = W[r];
  }
  FQ_TRY(B.upload(B.q, B.q_h, size_t(n) * B.ncv * B.qcols * sizeof(c128)));
  FQ_TRY(B.upload(B.gemm, B.gemm_h, n * sizeof(GemmDesc)));
  FQ_TRY(B.upload(B.aux, B.aux_h, n * sizeof(int)));
  FQ_HIP_CHECK(launch_b_basis_gemm(B.gemm, n, B.d, B.s, 1));
  FQ_HIP_CHECK(launch_b_normalize_col(B.args(B.aux, n), 0, B.s));
  for (int qi : W) {
    Prob& p = B.P[qi];
    p.restarts_before += p.restarts;
    const int budget = std::max(0, B.o->max_restarts - p.restarts_before);
    fresh_phase(B, p, Ph::C128, true, true, 0.5 * B.o->tol, budget);
    p.t_ref0 = now_s();
  }
  if (!B.have64) {
    FQ_TRY(ki_batch_tune<double>(B.L, B.sw, B.k_ref, B.f64, B.aux, n, B.s, &B.sh64, nullptr));
    B.have64 = true;
  }
  return FQ_OK;
}

fq_status decide(Bucket& B, const Out& out) {
  std::vector<int> D;
  for (size_t qi = 0; qi < B.P.size(); ++qi) {
    Prob& p = B.P[qi];
    if (p.ph == Ph::Done) continue;
    const int mm = p.j;
    const bool full = mm == B.ncv;
    const bool probe = p.early && mm >= B.nev + 2 && ((mm - B.nev - 2) % B.check_every == 0);
    if (full || probe) D.push_back(static_cast<int>(qi));
  }
  if (D.empty()) return FQ_OK;
  for (int qi : D) {
    Prob& p = B.P[qi];
    const size_t bytes = size_t(p.j - p.copied) * B.sd * sizeof(double);
    FQ_HIP_CHECK(hipMemcpyAsync(p.hslots + size_t(p.copied) * B.sd, p.slots + size_t(p.copied) * B.sd, bytes,
                                hipMemcpyDeviceToHost, B.s));
  }
  FQ_TRY(B.sync());
  const double t0 = now_s();
  for (int qi : D) B.P[qi].act = Act::None;
  parallel_for(D, [&](int qi) { analyse_one(B, B.P[qi]); });
  std::vector<int> R;
  for (int qi : D) {
    Prob& p = B.P[qi];
    if (p.err != FQ_OK) {
      p.ph = Ph::Done;
      continue;
    }
    if (p.act == Act::RitzCheck || p.act == Act::RitzFull) R.push_back(qi);
  }
  if (!R.empty()) FQ_TRY(ritz(B, R));
  std::vector<int> S, E;
  for (int qi : D) {
    Prob& p = B.P[qi];
    if (p.ph == Ph::Done) continue;
    if (p.err != FQ_OK) {
      p.ph = Ph::Done;
      continue;
    }
    double rmax = 0.0;
    for (double r : p.resid) rmax = std::max(rmax, r);
    if (p.act == Act::RitzCheck) {
      if (!p.check_true || rmax <= B.o->tol) {
        p.phase_converged = true;
        p.act = Act::PhaseEnd;
      } else {
        p.act = Act::None;
      }
    } else if (p.act == Act::RitzFull) {
      if (!p.check_true) {
        p.phase_converged = p.all;
        p.act = Act::PhaseEnd;
      } else if (rmax <= B.o->tol) {
        p.phase_converged = true;
        p.act = Act::PhaseEnd;
      } else if (p.oob) {
        p.phase_converged = false;
        p.act = Act::PhaseEnd;
      } else {
        p.tolg *= 0.1;  // the estimates were optimistic: tighten and continue
        p.act = Act::Restart;
      }
    }
    if (p.act == Act::Restart) S.push_back(qi);
    if (p.act == Act::PhaseEnd) E.push_back(qi);
  }
  if (!S.empty()) FQ_TRY(restart(B, S));
  std::vector<int> W;
  for (int qi : E) {
    Prob& p = B.P[qi];
    double rmax = 0.0;
    for (double r : p.resid) rmax = std::max(rmax, r);
    if (p.ph == Ph::C64 && B.o->refine && rmax > B.o->tol)
      W.push_back(qi);
    else
      FQ_TRY(finish(B, p, out));
  }
  if (!W.empty()) FQ_TRY(start_refine(B, W));
  FQ_TRY(B.sync());
  B.t_restart += now_s() - t0;
  return FQ_OK;
}

fq_status run_bucket(Bucket& B, const Out& out) {
  B.t_begin = now_s();
  FQ_TRY(setup(B));
  const int np = static_cast<int>(B.P.size());
  // start vectors: the counter-based generator with the caller's seed (as the
  // single-problem solver), normalised
  for (int qi = 0; qi < np; ++qi) FQ_HIP_CHECK(launch_random(B.P[qi].V, B.d, B.o->seed, B.s));
  FQ_HIP_CHECK(launch_b_normalize_col(B.args(B.ident, np), 0, B.s));
  const bool probes = probes_pay(B.d, B.k, B.P.size());
  for (Prob& p : B.P) {
    if (B.mixed)
      fresh_phase(B, p, Ph::C64, false, probes, std::max(B.o->tol, 2e-6), B.o->max_restarts);
    else
      fresh_phase(B, p, Ph::C128, true, probes, 0.5 * B.o->tol, B.o->max_restarts);
    p.t_filter0 = 0.0;
    p.t_restart0 = 0.0;
  }
  if (B.mixed) {
    FQ_TRY(ki_batch_tune<float>(B.L, B.sw, B.k, B.f32, B.ident, np, B.s, &B.sh32, nullptr));
    B.have32 = true;
  } else {
    FQ_TRY(ki_batch_tune<double>(B.L, B.sw, B.k, B.f64, B.ident, np, B.s, &B.sh64, nullptr));
    B.have64 = true;
  }
  std::vector<std::pair<int, int>> last_keys;
  std::vector<Seg> segs;
  for (;;) {
    // active problems ordered by (precision, column)
    std::vector<std::pair<int, int>> keys;  // (ph*65536 + j, q)
    for (int qi = 0; qi < np; ++qi) {
      const Prob& p = B.P[qi];
      if (p.ph == Ph::Done) continue;
      keys.emplace_back((p.ph == Ph::C64 ? 0 : 1) * 65536 + p.j, qi);
    }
    if (keys.empty()) break;
    std::sort(keys.begin(), keys.end());
    // the list changes only at decision points (all columns advance together)
    bool same = keys.size() == last_keys.size();
    for (size_t i = 0; same && i < keys.size(); ++i) same = keys[i].second == last_keys[i].second;
    if (!same) {
      FQ_TRY(B.staging());
      for (size_t i = 0; i < keys.size(); ++i) B.list_h[i] = keys[i].second;
      FQ_TRY(B.upload(B.list, B.list_h, keys.size() * sizeof(int)));
    }
    last_keys = keys;
    segs.clear();
    for (size_t i = 0; i < keys.size(); ++i) {
      const Prob& p = B.P[keys[i].second];
      if (segs.empty() || segs.back().ph != p.ph || segs.back().j != p.j)
        segs.push_back(Seg{p.ph, p.j, static_cast<unsigned>(i), 0});
      ++segs.back().n;
    }
    const double t0 = now_s();
    FQ_TRY(step(B, segs));
    for (const auto& kq : keys) {
      Prob& p = B.P[kq.second];
      ++p.j;
      p.st.n_filter_apps += 1;
      if (p.ph == Ph::C64) {
        p.st.n_U_apps += B.k;
        p.st.n_U_apps_c64 += B.k;
      } else {
        p.st.n_U_apps += B.mixed ? B.k_ref : B.k;
      }
    }
    // decisions synchronise; time the steps up to there
    bool any = false;
    for (const auto& kq : keys) {
      const Prob& p = B.P[kq.second];
      any = any || p.j == B.ncv || (p.early && p.j >= B.nev + 2 && ((p.j - B.nev - 2) % B.check_every == 0));
    }
    if (any) {
      FQ_TRY(B.sync());
      B.t_filter += now_s() - t0;
      FQ_TRY(decide(B, out));
    } else {
      B.t_filter += now_s() - t0;
    }
  }
  return FQ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Entry: bucket the problems, run each bucket (memory permitting in chunks),
// and solve the rest (brickwork, tiny L) one by one.
// ---------------------------------------------------------------------------
fq_status arnoldi_batched_solve(floquet_op* const* ops, int n_ops, const double* phis, int n_phi, int nev,
                                const fq_arnoldi_opts* o, const int* k_per_op, double* evals_host,
                                void* const* evecs_dev, double* resid_host, fq_arnoldi_stats* stats,
                                hipStream_t s) {
  if (!ops || n_ops < 1 || !phis || n_phi < 1 || !evals_host || !o) {
    set_error("arnoldi_eigs_batched: need ops, n_ops >= 1, phis, n_phi >= 1, opts and evals_host");
    return FQ_EINVAL;
  }
  if (o->v0_dev) {
    set_error("arnoldi_eigs_batched: opts.v0_dev must be NULL (each problem uses the seeded start vector)");
    return FQ_EINVAL;
  }
  if (o->block > 1) {
    set_error("arnoldi_eigs_batched: opts.block must be 0 or 1 (block Krylov-Schur is for arnoldi_eigs)");
    return FQ_EINVAL;
  }
  if (o->poly_coeffs && k_per_op) {
    set_error("arnoldi_eigs_batched: a user polynomial fixes the filter order: k_per_op must be NULL");
    return FQ_EINVAL;
  }
  std::vector<int> ks(n_ops);
  for (int i = 0; i < n_ops; ++i) {
    fq_arnoldi_opts oi = *o;
    // k = 0 without a user polynomial: the paper's rule for this chain length
    ks[i] = k_per_op ? k_per_op[i] : ((o->k == 0 && !o->poly_coeffs && ops[i] && o->ncv > 0) ? paper_k(ops[i]->L, o->ncv) : o->k);
    oi.k = ks[i];
    FQ_TRY(validate_arnoldi(ops[i], nev, &oi));
    if (ks[i] < 1) {
      set_error("arnoldi_eigs_batched: filter orders must be >= 1");
      return FQ_EINVAL;
    }
  }
  for (int j = 0; j < n_phi; ++j)
    if (!std::isfinite(phis[j])) {
      set_error("phi must be finite");
      return FQ_EINVAL;
    }
  // graph capture needs a stream that can be captured (not the legacy null
  // stream): the solve runs on a stream of its own, after the caller's
  const bool graphs = g_graph_capture.load() != 0;
  hipStream_t own = nullptr;
  if (graphs) {
    FQ_HIP_CHECK(hipStreamSynchronize(s));
    FQ_HIP_CHECK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    s = own;
  }
  struct StreamGuard {
    hipStream_t st;
    ~StreamGuard() {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
    }
  } guard{own};
  const size_t nprob = size_t(n_ops) * n_phi;
  std::fill(evals_host, evals_host + 2 * size_t(nev) * nprob, 0.0);
  if (resid_host) std::fill(resid_host, resid_host + size_t(nev) * nprob, 0.0);
  if (stats)
    for (size_t i = 0; i < nprob; ++i) stats[i] = fq_arnoldi_stats{};
  const Out out{evals_host, resid_host, stats, o->tol};

  fq_status worst = FQ_OK;
  std::string first_err;
  auto note = [&](fq_status st, const std::string& msg) {
    if (st != FQ_OK && first_err.empty()) first_err = msg;
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (st == FQ_NOT_CONVERGED && worst == FQ_OK) worst = st;
  };

  // problems the batched kernels cover: kicked Ising, L >= 4; the others are
  // solved one by one afterwards
  std::vector<std::pair<int, int>> seq;
  // the phase-table cache of an op holds 8 entries: at most 7 targets (plus
  // phi = 0 for U) of one op are in flight at a time
  for (int j0 = 0; j0 < n_phi; j0 += 7) {
    const int j1 = std::min(n_phi, j0 + 7);
    std::map<std::tuple<int, bool, int>, std::vector<Prob>> buckets;
    for (int i = 0; i < n_ops; ++i) {
      floquet_op* op = ops[i];
      // the batched basis products run on the matrix cores only (<= 256 columns)
      // (user polynomials run one by one as well)
      if (op->model != FQ_KICKED_ISING || op->L < 4 || nev > 256 || keep_count(o->ncv, nev) > 256 ||
          o->poly_coeffs) {
        if (j0 == 0)
          for (int j = 0; j < n_phi; ++j) seq.emplace_back(i, j);
        continue;
      }
      for (int j = j0; j < j1; ++j) {
        Prob p;
        p.op = op;
        p.phi = phis[j];
        p.out = size_t(i) * n_phi + j;
        p.evecs = evecs_dev ? evecs_dev[p.out] : nullptr;
        buckets[std::make_tuple(op->L, op->sw, ks[i])].push_back(std::move(p));
      }
    }
    for (auto& kv : buckets) {
      std::vector<Prob>& all = kv.second;
      // tables of every problem of the group, fetched before any launch
      for (Prob& p : all) {
        FQ_TRY(get_tables(p.op, p.phi, &p.tab_phi));
        // the cache may have reallocated: fetch phi = 0 after phi, then re-fetch phi
        FQ_TRY(get_tables(p.op, 0.0, &p.tab0));
      }
      // pointers into op->tables can move when the vector grows: copy what the
      // device descriptors need by re-reading after every insertion is done
      for (Prob& p : all) {
        FQ_TRY(get_tables(p.op, p.phi, &p.tab_phi));
        FQ_TRY(get_tables(p.op, 0.0, &p.tab0));
      }
      const int L = std::get<0>(kv.first);
      const size_t d = size_t(1) << L;
      const int ncv = o->ncv;
      const int qcols = std::max(keep_count(ncv, nev), nev);
      const unsigned nblk = row_blocks(d);
      const int sd = 4 * (ncv + 1) + 2;
      size_t freeb = 0, totalb = 0;
      FQ_HIP_CHECK(hipMemGetInfo(&freeb, &totalb));
      const size_t per = prob_bytes(d, ncv, nev, true, nblk, sd, qcols);
      const size_t budget = freeb > (size_t(1) << 30) ? (freeb - (size_t(1) << 30)) / 10 * 8 : 0;
      size_t chunk = std::max<size_t>(1, std::min<size_t>(budget / per, 65535));
      for (size_t c0 = 0; c0 < all.size(); c0 += chunk) {
        const size_t c1 = std::min(all.size(), c0 + chunk);
        Bucket B;
        B.L = L;
        B.sw = std::get<1>(kv.first);
        B.k = std::get<2>(kv.first);
        B.k_ref = o->refine_k > 0 ? o->refine_k : B.k;
        B.d = d;
        B.nblk = nblk;
        B.ncv = ncv;
        B.nev = nev;
        B.ldp = ncv + 1;
        B.sd = sd;
        B.p_keep = keep_count(ncv, nev);
        B.check_every = std::max(4, ncv / 16);
        B.qcols = qcols;
        B.o = o;
        B.mixed = o->filter_dtype == FQ_C64;
        B.s = s;
        B.graphs = graphs;
        B.P.assign(all.begin() + c0, all.begin() + c1);
        const fq_status st = run_bucket(B, out);
        if (st != FQ_OK) {
          // a device or setup failure ends the whole call
          note(st, floquet_last_error());
          (void)hipStreamSynchronize(s);
          set_error(first_err);
          return worst;
        }
        for (Prob& p : B.P) {
          if (stats) stats[p.out] = p.st;
          note(p.err, p.msg);
        }
      }
    }
  }
  for (const auto& ij : seq) {
    const size_t pidx = size_t(ij.first) * n_phi + ij.second;
    fq_arnoldi_opts oi = *o;
    oi.k = ks[ij.first];
    const fq_status st = arnoldi_solve(ops[ij.first], nev, phis[ij.second], &oi, evals_host + 2 * nev * pidx,
                                       evecs_dev ? evecs_dev[pidx] : nullptr,
                                       resid_host ? resid_host + nev * pidx : nullptr, stats ? stats + pidx : nullptr,
                                       s);
    note(st, floquet_last_error());
  }
  if (!first_err.empty()) set_error(first_err);
  return worst;
}

fq_status set_graph_capture(int on) {
  if (on != 0 && on != 1) {
    set_error("fq_set_graph_capture: on must be 0 or 1");
    return FQ_EINVAL;
  }
  g_graph_capture.store(on);
  return FQ_OK;
}

}  // namespace fq

extern "C" fq_status fq_set_graph_capture(int on) {
  fq::clear_error();
  return fq::set_graph_capture(on);
}
