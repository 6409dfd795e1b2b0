// Batched kicked-Ising filter / U passes and their tile-shape autotuner.
#include "ki_batched.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace fq {

namespace {

// (RB, TB) pairs with compiled kernel instances (the shape list of the
// kicked-Ising launchers).
bool shape_compiled(int rb, int tb) {
  static const int S[][2] = {{0, 6}, {1, 6}, {2, 6}, {3, 6}, {4, 6}, {4, 7}, {4, 8},
                             {4, 9}, {1, 7}, {2, 7}, {2, 8}, {3, 8}, {3, 7}, {3, 9}};
  for (const auto& x : S)
    if (x[0] == rb && x[1] == tb) return true;
  return false;
}

// (RB, TB) pairs with a pipelined instance (ki_launch_pipe)
bool pipe_shape(int rb, int tb, bool c64_dt) {
  static const int S[][2] = {{2, 8}, {3, 7}, {3, 8}, {3, 9}, {4, 6}, {4, 7}, {4, 8}, {4, 9}};
  if (!c64_dt && rb > 3) return false;
  for (const auto& x : S)
    if (x[0] == rb && x[1] == tb) return true;
  return false;
}

// three: the plan runs its phase passes in the three-layout form, which
// also has 14-bit (1024-thread) tiles
bool group_ok(const KiGroup& g, size_t d, bool three) {
  const bool wide = three && g.rb == 4 && g.tb == 10;
  return g.n >= g.tb && g.rb >= 0 && g.rb + g.tb == g.n && g.rb <= 4 && g.tb <= (wide ? 10 : 9) &&
         g.tb <= g.rb + 6 && (size_t(g.ntiles) << g.n) == d && (wide || shape_compiled(g.rb, g.tb));
}

bool plan_ok(const KiPlan& p, int L, bool three = false) {
  if (p.ngroups < 2) return false;
  for (int i = 0; i < p.ngroups; ++i)
    if (!group_ok(p.grp[i], size_t(1) << L, three)) return false;
  return true;
}

bool same_plan(const KiPlan& a, const KiPlan& b) {
  if (a.ngroups != b.ngroups) return false;
  for (int i = 0; i < a.ngroups; ++i)
    if (a.grp[i].rb != b.grp[i].rb) return false;
  return true;
}

fq_status launch_err(const char* what, hipError_t e) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return FQ_EDEVICE;
}

template <typename Real>
fq_status bpass(const KiBatchShape& sh, const KiGroup& g, const KiDesc<Real>* desc, const int* list, unsigned n,
                int from_psi, int flags, bool k2, hipStream_t s, int chi = 0) {
  KiPassArgs<Real> a{};
  a.n = g.n;
  a.c = g.c;
  a.p = g.p;
  a.m = sh.m;
  a.flags = flags;
  a.psi_coef_re = 1.0;
  a.in_coef_re = 1.0;
  // few tiles in the whole launch: latency-bound, fetch the phase with the tile
  if (sh.prefetch > 0 || (sh.prefetch < 0 && size_t(g.ntiles) * n <= (sizeof(Real) == 4 ? 1024u : 512u)))
    a.flags |= KI_PREFETCH_PHASE;
  a.k1 = masks_for(g.kbits, g.n, g.rb, g.tb);
  a.k2 = k2 ? a.k1 : KickMasks{0, 0, 0, 0};
  a.chi = chi;
  a.desc = desc;
  a.list = list;
  a.from_psi = from_psi;
  a.flat = sh.flat ? 1 : 0;
  a.tile_log = 0;
  while ((1u << a.tile_log) < g.ntiles) ++a.tile_log;
  KickMasks m3;
  unsigned c3 = 0;
  const int t3 = table3_mode(g.n, g.tb, g.c, g.p, a.m);
  if (sh.three && !sh.sw && chi == 0 && g.rb == 4 && pass3_flags_ok(a.flags) && !from_psi && t3 >= 0 &&
      masks3_for(g.kbits, g.n, g.tb, &m3, &c3)) {
    a.k1 = m3;
    a.k1c = c3;
    a.t3 = t3;
    a.k2 = k2 ? m3 : KickMasks{0, 0, 0, 0};
    a.k2c = k2 ? c3 : 0u;
    const hipError_t e = ki_launch_pass3<Real>(a, g.tb, g.ntiles, s, n);
    if (e != hipSuccess) return launch_err("batched three-layout kicked-Ising pass launch failed", e);
    return FQ_OK;
  }
  // the pipelined form has no folded variant
  if (sh.pipe > 0 && chi == 0 && pipe_shape(g.rb, g.tb, sizeof(Real) == 4)) {
    const size_t items = size_t(g.ntiles) * n;
    const unsigned grid = static_cast<unsigned>(std::min<size_t>(sh.pipe, (items / 2) & ~size_t(7)));
    if (grid >= 8 && (g.ntiles & 7u) == 0u) {
      const hipError_t e = ki_launch_pipe<Real>(a, g.rb, g.tb, sh.sw, g.ntiles, n, grid, s);
      if (e != hipSuccess) return launch_err("pipelined kicked-Ising pass launch failed", e);
      return FQ_OK;
    }
  }
  const hipError_t e = ki_launch_pass<Real>(a, g.rb, g.tb, sh.sw, g.ntiles, s, n);
  if (e != hipSuccess) return launch_err("batched kicked-Ising pass launch failed", e);
  return FQ_OK;
}

template <typename Real>
fq_status bsingle(const KiBatchShape& sh, const KiDesc<Real>* desc, const int* list, unsigned n, int steps,
                  int flags, hipStream_t s) {
  KiSingleArgs<Real> a{};
  a.in_coef_re = 1.0;
  a.L = sh.L;
  a.m = sh.m;
  a.steps = steps;
  a.flags = flags;
  a.kick = masks_for((1u << sh.L) - 1u, std::max(sh.L, 6), sh.srb, sh.stb);
  a.desc = desc;
  a.list = list;
  a.from_psi = 1;
  const bool regs = (1 << sh.srb) * int(sizeof(cpx<Real>)) <= 128;
  const hipError_t e = ki_launch_single<Real>(a, sh.srb, sh.stb, sh.sw, regs, n, s, true);
  if (e != hipSuccess) return launch_err("batched single-tile kicked-Ising launch failed", e);
  return FQ_OK;
}

}  // namespace

std::vector<KiBatchShape> ki_batch_candidates(int L, bool sw, bool c64_dt) {
  std::vector<KiBatchShape> v;
  KiBatchShape base;
  base.L = L;
  base.m = (L + 1) / 2;
  base.sw = sw;
  if (L <= 13) {
    int rb, tb;
    single_shape(L, &rb, &tb);
    for (int delta : {0, 1, -1}) {
      int t = tb + delta, r = L - t;
      if (L < 6) {
        if (delta != 0) continue;
        t = 6;
        r = 0;
      }
      if (r < 0 || r > 4 || t < 6 || t > 9 || t > r + 6 || !shape_compiled(r, t)) continue;
      KiBatchShape c = base;
      c.single = true;
      c.srb = r;
      c.stb = t;
      v.push_back(c);
    }
  }
  const KiPlan pl = make_plan(L, c64_dt, false);
  std::vector<KiPlan> plans;
  if (plan_ok(pl, L)) plans.push_back(pl);
  for (int rbv : {4, 3, 2}) {
    KiPlan q = pl;
    for (int i = 0; i < q.ngroups; ++i) {
      KiGroup& g = q.grp[i];
      const int tb = g.n - rbv;
      if (tb >= 6 && tb <= 9 && tb <= rbv + 6 && shape_compiled(rbv, tb)) {
        g.rb = rbv;
        g.tb = tb;
      }
    }
    if (!plan_ok(q, L)) continue;
    bool dup = false;
    for (const KiPlan& o : plans) dup = dup || same_plan(o, q);
    if (!dup) plans.push_back(q);
  }
  for (const KiPlan& q : plans) {
    KiBatchShape c = base;
    c.plan = q;
    v.push_back(c);
  }
  // the three-layout Horner passes for plans of 16-amplitude tiles only,
  // with the 14-bit complex64 tiles where they apply
  if (!sw) {
    std::vector<KiPlan> plans3 = plans;
    const KiPlan wide = make_plan(L, c64_dt, c64_dt);
    bool dup = false;
    for (const KiPlan& o : plans3) dup = dup || (same_plan(o, wide) && o.grp[0].n == wide.grp[0].n);
    if (!dup && plan_ok(wide, L, true)) plans3.push_back(wide);
    // high-bit tiles of 128-byte chunks (one more contiguous bit): fewer,
    // longer runs per row of the state in the high-bit pass
    KiPlan wide_chunk = make_plan_chunk(L, c64_dt ? 4 : 3);
    for (int i = 0; i < wide_chunk.ngroups; ++i) {
      wide_chunk.grp[i].rb = 4;
      wide_chunk.grp[i].tb = wide_chunk.grp[i].n - 4;
    }
    if (wide_chunk.ngroups == 2 && plan_ok(wide_chunk, L, true)) plans3.push_back(wide_chunk);
    for (const KiPlan& q : plans3) {
      bool all4 = q.ngroups == 2;
      for (int i = 0; i < q.ngroups; ++i) all4 = all4 && q.grp[i].rb == 4;
      if (!all4) continue;
      KiBatchShape c = base;
      c.plan = q;
      c.three = true;
      v.push_back(c);
    }
  }
  return v;
}

template <typename Real>
fq_status ki_batch_filter(const KiBatchShape& sh, int k, const KiDesc<Real>* desc, const int* list, unsigned n,
                          hipStream_t s, const KiDesc<Real>* chi0, const KiDesc<Real>* chi1) {
  if (n == 0) return FQ_OK;
  if (k < 1) {
    set_error("internal: batched filter needs k >= 1");
    return FQ_EINVAL;
  }
  if (sh.single) return bsingle<Real>(sh, desc, list, n, k, KI_ADD_PSI, s);
  if (sh.chunk > 0 && n > sh.chunk) {
    KiBatchShape one = sh;
    one.chunk = 0;
    for (unsigned c0 = 0; c0 < n; c0 += sh.chunk) {
      const fq_status st = ki_batch_filter<Real>(one, k, desc, list + c0, std::min(sh.chunk, n - c0), s, chi0, chi1);
      if (st != FQ_OK) return st;
    }
    return FQ_OK;
  }
  const KiPlan& pl = sh.plan;
  if (!plan_ok(pl, sh.L, sh.three)) {
    set_error("internal: inconsistent batched kicked-Ising tile plan");
    return FQ_EINVAL;
  }
  fq_status st;
  if (pl.ngroups == 2) {
    const bool fold = chi0 && chi1 && k >= 2 && !sh.three;
    if (fold) {
      // chi_g = K_g psi for both groups
      st = bpass<Real>(sh, pl.grp[0], chi0, list, n, 1, 0, false, s);
      if (st != FQ_OK) return st;
      st = bpass<Real>(sh, pl.grp[1], chi1, list, n, 1, 0, false, s);
      if (st != FQ_OK) return st;
    }
    // prologue: kick of the second group on psi; then alternate the groups
    st = bpass<Real>(sh, pl.grp[1], desc, list, n, 1, 0, false, s);
    if (st != FQ_OK) return st;
    for (int step = 1; step <= k; ++step) {
      const int g = (step - 1) & 1;
      st = bpass<Real>(sh, pl.grp[g], desc, list, n, 0, KI_PHASE | KI_ADD_PSI, step < k, s,
                       fold && step < k ? g + 1 : 0);
      if (st != FQ_OK) return st;
    }
    return FQ_OK;
  }
  for (int step = 1; step <= k; ++step) {
    st = bpass<Real>(sh, pl.grp[2], desc, list, n, step == 1 ? 1 : 0, 0, false, s);
    if (st != FQ_OK) return st;
    st = bpass<Real>(sh, pl.grp[1], desc, list, n, 0, 0, false, s);
    if (st != FQ_OK) return st;
    st = bpass<Real>(sh, pl.grp[0], desc, list, n, 0, KI_PHASE | KI_ADD_PSI, false, s);
    if (st != FQ_OK) return st;
  }
  return FQ_OK;
}

template <typename Real>
fq_status ki_batch_apply(const KiBatchShape& sh, const KiDesc<Real>* desc, const int* list, unsigned n,
                         hipStream_t s) {
  if (n == 0) return FQ_OK;
  if (sh.single) return bsingle<Real>(sh, desc, list, n, 1, 0, s);
  const KiPlan& pl = sh.plan;
  if (!plan_ok(pl, sh.L, sh.three)) {
    set_error("internal: inconsistent batched kicked-Ising tile plan");
    return FQ_EINVAL;
  }
  for (int gi = pl.ngroups - 1; gi >= 0; --gi) {
    const fq_status st =
        bpass<Real>(sh, pl.grp[gi], desc, list, n, gi == pl.ngroups - 1 ? 1 : 0, gi == 0 ? KI_PHASE : 0, false, s);
    if (st != FQ_OK) return st;
  }
  return FQ_OK;
}

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, bool, bool, int, int>, KiBatchShape> g_tuned;
int g_policy = FQ_POLICY_AUTO;  // guarded by g_tune_mu

// FQ_VERBOSE=1 prints the tuner's choice to stderr.
// FQ_VERBOSE=1: the tuner's choice per case; 2: every candidate's timing
int tune_verbose() {
  static const int v = [] {
    const char* e = std::getenv("FQ_VERBOSE");
    return (e && e[0] >= '1' && e[0] <= '9') ? e[0] - '0' : 0;
  }();
  return v;
}

int size_class(unsigned n) {
  int c = 0;
  while ((1u << c) < n) ++c;
  return c;
}
}  // namespace

template <typename Real>
fq_status ki_batch_shape_untimed(int L, bool sw, int k, unsigned n, KiBatchShape* out) {
  const bool c64_dt = sizeof(Real) == 4;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(L, sw, c64_dt, k, size_class(n)));
    if (it != g_tuned.end()) {
      *out = it->second;
      return FQ_OK;
    }
  }
  // the first candidate of ki_batch_candidates, built without containers
  KiBatchShape c;
  c.L = L;
  c.m = (L + 1) / 2;
  c.sw = sw;
  if (L <= 13) {
    int rb, tb;
    single_shape(L, &rb, &tb);
    if (L < 6) {
      rb = 0;
      tb = 6;
    }
    if (rb >= 0 && rb <= 4 && tb >= 6 && tb <= 9 && tb <= rb + 6 && shape_compiled(rb, tb)) {
      c.single = true;
      c.srb = rb;
      c.stb = tb;
      *out = c;
      return FQ_OK;
    }
  }
  c.plan = make_plan(L, c64_dt, c64_dt && !sw);
  for (int i = 0; i < c.plan.ngroups; ++i) c.three = c.three || c.plan.grp[i].tb > 9;
  if (!plan_ok(c.plan, L, c.three)) {
    set_error("no kicked-Ising tile shape for L = " + std::to_string(L));
    return FQ_EINVAL;
  }
  *out = c;
  return FQ_OK;
}

template fq_status ki_batch_shape_untimed<float>(int, bool, int, unsigned, KiBatchShape*);
template fq_status ki_batch_shape_untimed<double>(int, bool, int, unsigned, KiBatchShape*);

fq_status ki_set_policy(int policy) {
  if (policy != FQ_POLICY_AUTO && policy != FQ_POLICY_TILE && policy != FQ_POLICY_PIPE) {
    set_error("fq_set_kernel_policy: policy must be FQ_POLICY_AUTO, FQ_POLICY_TILE or FQ_POLICY_PIPE");
    return FQ_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (policy != g_policy) g_tuned.clear();
  g_policy = policy;
  return FQ_OK;
}

template <typename Real>
fq_status ki_batch_tune(int L, bool sw, int k, const KiDesc<Real>* desc, const int* list, unsigned n,
                        hipStream_t s, KiBatchShape* out, double* best_us, const KiDesc<Real>* chi0,
                        const KiDesc<Real>* chi1) {
  const bool c64_dt = sizeof(Real) == 4;
  const auto key = std::make_tuple(L, sw, c64_dt, k, size_class(n));
  int policy;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    policy = g_policy;
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      *out = it->second;
      if (best_us) *best_us = -1.0;
      return FQ_OK;
    }
  }
  const std::vector<KiBatchShape> cands = ki_batch_candidates(L, sw, c64_dt);
  if (cands.empty()) {
    set_error("no kicked-Ising tile shape for L = " + std::to_string(L));
    return FQ_EINVAL;
  }
  const int kt = std::min(k, 32);
  hipEvent_t e0, e1;
  FQ_HIP_CHECK(hipEventCreate(&e0));
  FQ_HIP_CHECK(hipEventCreate(&e1));
  // time per Horner step of one candidate (negative: could not be launched)
  auto time_one = [&](const KiBatchShape& c) -> double {
    if (ki_batch_filter<Real>(c, kt, desc, list, n, s, chi0, chi1) != FQ_OK) {
      (void)hipGetLastError();
      return -1.0;
    }
    (void)hipEventRecord(e0, s);
    bool ok = true;
    for (int r = 0; r < 2 && ok; ++r) ok = ki_batch_filter<Real>(c, kt, desc, list, n, s, chi0, chi1) == FQ_OK;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || !ok) {
      (void)hipGetLastError();
      return -1.0;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return 1000.0 * ms / (2.0 * kt);
  };
  KiBatchShape best = cands[0];
  double best_t = -1.0;
  std::vector<std::pair<double, KiBatchShape>> timed;  // every launchable candidate
  auto consider = [&](const KiBatchShape& c) {
    const double us = time_one(c);
    if (tune_verbose() >= 2)
      std::fprintf(stderr, "[fq]   candidate rb/tb %d/%d chunk %u flat %d prefetch %d pipe %u three %d: %.2f us/step\n",
                   c.single ? c.srb : c.plan.grp[0].rb, c.single ? c.stb : c.plan.grp[0].tb, c.chunk, c.flat ? 1 : 0,
                   c.prefetch, c.pipe, c.three ? 1 : 0, us);
    if (us >= 0.0) timed.emplace_back(us, c);
    if (us >= 0.0 && (best_t < 0.0 || us < best_t)) {
      best_t = us;
      best = c;
    }
  };
  // stage 1: tile shapes
  for (const KiBatchShape& c : cands) consider(c);
  // stage 2: sub-batch size (down to one problem at a time: states too
  // large to gain from sharing a launch), stage 3: XCD mapping (multi-pass
  // shapes)
  if (best_t >= 0.0 && !best.single) {
    const KiBatchShape base = best;
    for (unsigned ch : {256u, 128u, 64u, 32u, 16u, 2u, 1u}) {
      if (ch >= n || (ch < 16 && n > 8)) continue;
      KiBatchShape c = base;
      c.chunk = ch;
      consider(c);
    }
    KiBatchShape c = best;
    c.flat = true;
    consider(c);
    for (int pf : {0, 1}) {
      KiBatchShape q = best;
      q.prefetch = pf;
      consider(q);
    }
    // stage 4: persistent pipelined passes, 1, 2 or 4 workgroups per CU
    // (the only choice under FQ_POLICY_PIPE, skipped under FQ_POLICY_TILE)
    int dev = 0, cus = 0;
    if (policy != FQ_POLICY_TILE && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      const KiBatchShape base2 = best;
      if (policy == FQ_POLICY_PIPE) best_t = -1.0;
      for (unsigned per_cu : {1u, 2u, 4u}) {
        KiBatchShape p = base2;
        p.pipe = (static_cast<unsigned>(cus) * per_cu) & ~7u;
        if (p.pipe >= 8) consider(p);
      }
    }
  }
  // single timings of candidates within a few per cent of each other are at
  // the mercy of clock and power drift: the three fastest are timed twice
  // more, interleaved, and the best of each one's three timings decides
  if (policy == FQ_POLICY_PIPE)  // the pipelined candidates only
    timed.erase(std::remove_if(timed.begin(), timed.end(),
                               [](const std::pair<double, KiBatchShape>& x) { return x.second.pipe == 0; }),
                timed.end());
  if (timed.size() > 1) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<double, KiBatchShape>& x, const std::pair<double, KiBatchShape>& y) {
                       return x.first < y.first;
                     });
    const size_t top = std::min<size_t>(3, timed.size());
    for (int r = 0; r < 2; ++r)
      for (size_t i = 0; i < top; ++i) {
        const double us = time_one(timed[i].second);
        if (us >= 0.0) timed[i].first = std::min(timed[i].first, us);
      }
    size_t bi = 0;
    for (size_t i = 1; i < top; ++i)
      if (timed[i].first < timed[bi].first) bi = i;
    best_t = timed[bi].first;
    best = timed[bi].second;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_t < 0.0) {
    set_error("no kicked-Ising tile shape could be launched for L = " + std::to_string(L));
    return FQ_EDEVICE;
  }
  if (tune_verbose())
    std::fprintf(stderr,
                 "[fq] tuned L=%d %s n=%u k=%d: %s rb/tb %d/%d chunk %u flat %d prefetch %d pipe %u three %d: %.2f us/step\n",
                 L, c64_dt ? "c64" : "c128", n, k, best.single ? "single" : "multi-pass",
                 best.single ? best.srb : best.plan.grp[0].rb, best.single ? best.stb : best.plan.grp[0].tb,
                 best.chunk, best.flat ? 1 : 0, best.prefetch, best.pipe, best.three ? 1 : 0, best_t);
  *out = best;
  if (best_us) *best_us = best_t;
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (g_policy == policy) g_tuned[key] = best;
  return FQ_OK;
}

template fq_status ki_batch_filter<float>(const KiBatchShape&, int, const KiDesc<float>*, const int*, unsigned,
                                          hipStream_t, const KiDesc<float>*, const KiDesc<float>*);
template fq_status ki_batch_filter<double>(const KiBatchShape&, int, const KiDesc<double>*, const int*, unsigned,
                                           hipStream_t, const KiDesc<double>*, const KiDesc<double>*);
template fq_status ki_batch_apply<float>(const KiBatchShape&, const KiDesc<float>*, const int*, unsigned,
                                         hipStream_t);
template fq_status ki_batch_apply<double>(const KiBatchShape&, const KiDesc<double>*, const int*, unsigned,
                                          hipStream_t);
template fq_status ki_batch_tune<float>(int, bool, int, const KiDesc<float>*, const int*, unsigned, hipStream_t,
                                        KiBatchShape*, double*, const KiDesc<float>*, const KiDesc<float>*);
template fq_status ki_batch_tune<double>(int, bool, int, const KiDesc<double>*, const int*, unsigned, hipStream_t,
                                         KiBatchShape*, double*, const KiDesc<double>*, const KiDesc<double>*);

}  // namespace fq
