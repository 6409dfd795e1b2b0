// C ABI of the Floquet library: operator construction, U and filter
// application (kicked Ising here; brickwork in bw_kernels.hip), error plumbing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "op.h"

namespace fq {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

namespace {

// ---------------------------------------------------------------------------
// Kicked-Ising diagonal tables (FP64, rounded once to complex64).
// ---------------------------------------------------------------------------

// bond list in bit coordinates: (bit u, bit v, J)
struct Bond {
  int u, v;
  double J;
};

std::vector<Bond> ki_bonds(const floquet_op* op) {
  std::vector<Bond> b;
  const int L = op->L;
  for (int i = 1; i <= L - 1; ++i) b.push_back({L - i, L - i - 1, op->J[i - 1]});
  if (op->periodic && L >= 2) b.push_back({0, L - 1, op->J[L - 1]});
  return b;
}

inline int zbit(uint64_t s, int bit) { return 1 - 2 * int((s >> bit) & 1u); }

fq_status build_tables(floquet_op* op, double phi, PhaseTables* t) {
  const int L = op->L, m = op->m;
  const size_t nlo = size_t(1) << m;
  const size_t nhi = size_t(4) << (L - m);
  std::vector<zd> lo(nlo), hi(nhi);
  const auto bonds = ki_bonds(op);
  // per-U scale of the factored kicks, and the target rotation
  const zd pre = std::pow(op->site_scale, L) * std::polar(1.0, -phi);
  for (size_t s = 0; s < nlo; ++s) {
    double E = 0.0;
    for (const Bond& b : bonds)
      if (b.u < m && b.v < m) E += b.J * zbit(s, b.u) * zbit(s, b.v);
    for (int i = 1; i <= L; ++i) {
      const int bit = L - i;
      if (bit < m) E += op->h[i - 1] * zbit(s, bit);
    }
    lo[s] = pre * std::polar(1.0, -E);
  }
  for (size_t idx = 0; idx < nhi; ++idx) {
    const uint64_t shi = idx >> 2;
    const int b0 = int((idx >> 1) & 1u), bm1 = int(idx & 1u);
    // full-width index carrying the high bits and the two low boundary bits
    uint64_t s = shi << m;
    double E = 0.0;
    auto bitval = [&](int bit) -> int {
      if (bit >= m) return zbit(s, bit);
      if (bit == 0) return 1 - 2 * b0;
      if (bit == m - 1) return 1 - 2 * bm1;
      return 0;  // not reached for a valid split
    };
    for (const Bond& b : bonds) {
      const bool ulo = b.u < m, vlo = b.v < m;
      if (ulo && vlo) continue;
      E += b.J * bitval(b.u) * bitval(b.v);
    }
    for (int i = 1; i <= L; ++i) {
      const int bit = L - i;
      if (bit >= m) E += op->h[i - 1] * zbit(s, bit);
    }
    hi[idx] = std::polar(1.0, -E);
  }
  std::vector<c64> lo32(nlo), hi32(nhi);
  std::vector<c128> lo64(nlo), hi64(nhi);
  for (size_t i = 0; i < nlo; ++i) {
    lo64[i] = mk<double>(lo[i].real(), lo[i].imag());
    lo32[i] = mk<float>(float(lo[i].real()), float(lo[i].imag()));
  }
  for (size_t i = 0; i < nhi; ++i) {
    hi64[i] = mk<double>(hi[i].real(), hi[i].imag());
    hi32[i] = mk<float>(float(hi[i].real()), float(hi[i].imag()));
  }
  t->phi = phi;
  FQ_HIP_CHECK(hipMalloc(&t->tlo32, nlo * sizeof(c64)));
  FQ_HIP_CHECK(hipMalloc(&t->thi32, nhi * sizeof(c64)));
  FQ_HIP_CHECK(hipMalloc(&t->tlo64, nlo * sizeof(c128)));
  FQ_HIP_CHECK(hipMalloc(&t->thi64, nhi * sizeof(c128)));
  FQ_HIP_CHECK(hipMemcpy(t->tlo32, lo32.data(), nlo * sizeof(c64), hipMemcpyHostToDevice));
  FQ_HIP_CHECK(hipMemcpy(t->thi32, hi32.data(), nhi * sizeof(c64), hipMemcpyHostToDevice));
  FQ_HIP_CHECK(hipMemcpy(t->tlo64, lo64.data(), nlo * sizeof(c128), hipMemcpyHostToDevice));
  FQ_HIP_CHECK(hipMemcpy(t->thi64, hi64.data(), nhi * sizeof(c128), hipMemcpyHostToDevice));
  return FQ_OK;
}

void free_tables(PhaseTables& t) {
  (void)hipFree(t.tlo32);
  (void)hipFree(t.thi32);
  (void)hipFree(t.tlo64);
  (void)hipFree(t.thi64);
  t = PhaseTables{};
}

}  // namespace

// ---------------------------------------------------------------------------
// Tile shapes and plans
// ---------------------------------------------------------------------------

// (RB, TB) for a tile of n <= 13 bits: at most 16 amplitudes per thread
// (RB <= 4), up to 512 threads, every bit reachable (TB <= RB + 6).
void tile_shape(int n, int* rb, int* tb) {
  if (n <= 6) {
    *tb = 6;
    *rb = 0;
    return;
  }
  *rb = std::min(4, n - 6);
  *tb = n - *rb;
}

// Multi-pass tiles: few tiles per CU (small states) favour more waves per
// tile (8 amplitudes per thread, up to 512 threads).
void pass_shape(int n, unsigned ntiles, int* rb, int* tb) {
  tile_shape(n, rb, tb);
  if (ntiles <= 512 && n >= 10 && n <= 12) {
    *rb = 3;
    *tb = n - 3;
  }
}

// Register bits go to layout A (q >= TB) or B (q < RB); every other tile
// bit is a lane bit of layout B (lane q - RB), where the low lane indices
// are exchanged with DPP row permutes.
KickMasks masks_for(unsigned kbits, int n, int rb, int tb) {
  KickMasks k{0, 0, 0, 0};
  for (int q = 0; q < n; ++q) {
    if (!((kbits >> q) & 1u)) continue;
    if (q < rb)
      k.regB |= 1u << q;
    else if (q >= tb)
      k.regA |= 1u << (q - tb);
    else if (tb <= 6 && rb == 0)
      k.laneA |= 1u << q;  // one layout only (no register bits)
    else
      k.laneB |= 1u << (q - rb);
  }
  return k;
}

int pass3_shift_host(int tb) { return tb == 10 ? 6 : (tb == 9 ? 5 : 4); }

int table3_mode(int n, int tb, int c, int p, int m) {
  if (tb < 6 || tb > 10 || n != 4 + tb || m < 2) return -1;
  const int S = pass3_shift_host(tb);
  bool lo = true, hi = true;
  for (int j = S; j < S + 4; ++j) {
    const int gb = j < c ? j : p + (j - c);  // global bit of tile bit j
    if (gb >= m) lo = false;
    if (gb < m) hi = false;
    if (gb == 0 || gb == m - 1) lo = false;
  }
  return lo ? 0 : (hi ? 1 : -1);
}

// Each kicked bit goes to the first layout that holds it in a register (A:
// bits tb..n-1, B: bits 0..3, C: bits S..S+3); bits 4 .. S-1 (bit 4 of a
// 13-bit tile, bits 4 and 5 of a 14-bit tile) to B's lanes 0 .. S-5.
bool masks3_for(unsigned kbits, int n, int tb, KickMasks* ab, unsigned* c) {
  if (tb < 6 || tb > 10 || n != 4 + tb) return false;
  const int S = pass3_shift_host(tb);
  KickMasks k{0, 0, 0, 0};
  unsigned cm = 0, done = 0;
  auto take = [&](int q) { return ((kbits >> q) & 1u) && !((done >> q) & 1u); };
  for (int q = tb; q < n; ++q)
    if (take(q)) {
      k.regA |= 1u << (q - tb);
      done |= 1u << q;
    }
  for (int q = 0; q < 4; ++q)
    if (take(q)) {
      k.regB |= 1u << q;
      done |= 1u << q;
    }
  for (int q = 4; q < S; ++q)
    if (take(q)) {
      k.laneB |= 1u << (q - 4);
      done |= 1u << q;
    }
  for (int q = S; q < S + 4 && q < n; ++q)
    if (take(q)) {
      cm |= 1u << (q - S);
      done |= 1u << q;
    }
  if (done != (kbits & ((1u << n) - 1u)) || (kbits >> n) != 0u) return false;
  *ab = k;
  *c = cm;
  return true;
}

// Single-workgroup kernel: as many waves as the reachability rule allows.
void single_shape(int L, int* rb, int* tb) {
  if (L <= 6) {
    *tb = 6;
    *rb = 0;
    return;
  }
  int t = std::min(8, (L + 6) / 2);
  if (L >= 13) t = L - 4;  // 16 amplitudes per thread above 2^12
  *tb = t;
  *rb = L - t;
}

KiPlan make_plan_chunk(int L, int c) {
  KiPlan pl;
  const int tot = L + c;
  const int nlo = (tot + 1) / 2, nhi = tot - nlo;
  if (c < 1 || nhi <= c || nlo > 13) return pl;  // ngroups = 0: no such plan
  pl.ngroups = 2;
  KiGroup& lo = pl.grp[0];
  lo.n = nlo;
  lo.c = nlo;
  lo.p = nlo;
  lo.kbits = (1u << nlo) - 1u;
  lo.ntiles = 1u << (L - nlo);
  KiGroup& hi = pl.grp[1];
  hi.n = nhi;
  hi.c = c;
  hi.p = nlo;
  hi.kbits = ((1u << nhi) - 1u) & ~((1u << c) - 1u);
  hi.ntiles = 1u << (L - nhi);
  for (int i = 0; i < 2; ++i) pass_shape(pl.grp[i].n, pl.grp[i].ntiles, &pl.grp[i].rb, &pl.grp[i].tb);
  return pl;
}

KiPlan make_plan(int L, bool c64_dt, bool wide) {
  KiPlan pl;
  // chunk of contiguous amplitudes in the high-bit tiles: 64 bytes, or 32
  // bytes when that keeps both tiles at <= 13 bits (<= 512 threads).  With
  // wide (complex64 in the direct kick form), a low-bit tile of 14 bits
  // (the three-layout pass with 1024 threads and 136 KiB of LDS) keeps the
  // 64-byte chunk where 13 bits would need a 32-byte one (L = 24); the
  // high-bit tile stays at <= 13 bits, since its kick-only passes run in the
  // other pass kernel
  const int nmax = 13;
  int c = c64_dt ? 3 : 2;
  if (c64_dt && wide && L + 3 == 2 * nmax + 1) {
    const int nlo = nmax + 1, nhi = L + 3 - nlo;
    pl.ngroups = 2;
    KiGroup& lo = pl.grp[0];
    lo.n = nlo;
    lo.c = nlo;
    lo.p = nlo;
    lo.kbits = (1u << nlo) - 1u;
    lo.ntiles = 1u << (L - nlo);
    lo.rb = 4;
    lo.tb = nlo - 4;
    KiGroup& hi = pl.grp[1];
    hi.n = nhi;
    hi.c = 3;
    hi.p = nlo;
    hi.kbits = ((1u << nhi) - 1u) & ~7u;
    hi.ntiles = 1u << (L - nhi);
    pass_shape(hi.n, hi.ntiles, &hi.rb, &hi.tb);
    return pl;
  }
  if (c64_dt && L + 3 > 2 * nmax && L + 2 <= 2 * nmax) c = 2;
  if (L + c <= 2 * nmax) {
    const int tot = L + c;
    const int nlo = (tot + 1) / 2;
    const int nhi = tot - nlo;
    pl.ngroups = 2;
    KiGroup& lo = pl.grp[0];
    lo.n = nlo;
    lo.c = nlo;
    lo.p = nlo;
    lo.kbits = (1u << nlo) - 1u;
    lo.ntiles = 1u << (L - nlo);
    KiGroup& hi = pl.grp[1];
    hi.n = nhi;
    hi.c = c;
    hi.p = nlo;
    hi.kbits = ((1u << nhi) - 1u) & ~((1u << c) - 1u);
    hi.ntiles = 1u << (L - nhi);
  } else {
    // three groups: [0, n1), chunk + [n1, n1 + s2), chunk + [n1 + s2, L)
    const int n1 = nmax;
    const int rest = L - n1;
    const int s2 = (rest + 1) / 2, s3 = rest - s2;
    pl.ngroups = 3;
    KiGroup& g0 = pl.grp[0];
    g0.n = n1;
    g0.c = n1;
    g0.p = n1;
    g0.kbits = (1u << n1) - 1u;
    g0.ntiles = 1u << (L - n1);
    KiGroup& g1 = pl.grp[1];
    g1.n = c + s2;
    g1.c = c;
    g1.p = n1;
    g1.kbits = ((1u << g1.n) - 1u) & ~((1u << c) - 1u);
    g1.ntiles = 1u << (L - g1.n);
    KiGroup& g2 = pl.grp[2];
    g2.n = c + s3;
    g2.c = c;
    g2.p = n1 + s2;
    g2.kbits = ((1u << g2.n) - 1u) & ~((1u << c) - 1u);
    g2.ntiles = 1u << (L - g2.n);
  }
  for (int i = 0; i < pl.ngroups; ++i) pass_shape(pl.grp[i].n, pl.grp[i].ntiles, &pl.grp[i].rb, &pl.grp[i].tb);
  return pl;
}

bool single_ok(int L, bool) { return L <= 13; }

namespace {

// ---------------------------------------------------------------------------
// Kicked-Ising launches
// ---------------------------------------------------------------------------
template <typename Real>
struct TabSel;
template <>
struct TabSel<float> {
  static const c64* lo(const PhaseTables* t) { return t->tlo32; }
  static const c64* hi(const PhaseTables* t) { return t->thi32; }
};
template <>
struct TabSel<double> {
  static const c128* lo(const PhaseTables* t) { return t->tlo64; }
  static const c128* hi(const PhaseTables* t) { return t->thi64; }
};

template <typename Real>
fq_status ki_single(floquet_op* op, const PhaseTables* tab, const void* psi, const void* xin, void* out, int steps,
                    int flags, const double2* coefs, zd in_coef, unsigned nblocks, size_t stride, hipStream_t s) {
  int rb, tb;
  single_shape(op->L, &rb, &tb);
  KiSingleArgs<Real> a{};
  a.xin = static_cast<const cpx<Real>*>(xin);
  a.xout = static_cast<cpx<Real>*>(out);
  a.psi = static_cast<const cpx<Real>*>(psi);
  a.tlo = TabSel<Real>::lo(tab);
  a.thi = TabSel<Real>::hi(tab);
  a.coefs = coefs;
  a.w = op->w;
  a.in_coef_re = in_coef.real();
  a.in_coef_im = in_coef.imag();
  a.batch_stride = stride;
  a.L = op->L;
  a.m = op->m;
  a.steps = steps;
  a.flags = flags;
  if (in_coef != zd(1.0, 0.0)) a.flags |= KI_SCALE_IN;
  a.kick = masks_for((1u << op->L) - 1u, std::max(op->L, 6), rb, tb);
  const int R = 1 << rb;
  const bool regs = R * int(sizeof(cpx<Real>)) <= 128;
  hipError_t e = ki_launch_single<Real>(a, rb, tb, op->sw, regs, nblocks, s);
  if (e != hipSuccess) {
    set_error(std::string("single-tile kicked-Ising launch failed: ") + hipGetErrorString(e));
    return FQ_EDEVICE;
  }
  return FQ_OK;
}

template <typename Real>
fq_status ki_pass(floquet_op* op, const KiGroup& gp, const PhaseTables* tab, const void* xin, void* xout,
                  const void* psi, int flags, bool k2, zd psi_coef, zd in_coef, hipStream_t s) {
  // a tile must cover every thread of the workgroup and stay inside the state
  // (1024-thread tiles: complex64 three-layout passes only, checked below)
  if (gp.n < gp.tb || gp.rb + gp.tb != gp.n || gp.rb > 4 || gp.tb > 10 || gp.tb > gp.rb + 6 || gp.n > op->L ||
      (size_t(gp.ntiles) << gp.n) != op->dim()) {
    set_error("internal: inconsistent kicked-Ising tile plan");
    return FQ_EINVAL;
  }
  KiPassArgs<Real> a{};
  a.xin = static_cast<const cpx<Real>*>(xin);
  a.xout = static_cast<cpx<Real>*>(xout);
  a.psi = static_cast<const cpx<Real>*>(psi);
  a.tlo = TabSel<Real>::lo(tab);
  a.thi = TabSel<Real>::hi(tab);
  a.w = op->w;
  a.psi_coef_re = psi_coef.real();
  a.psi_coef_im = psi_coef.imag();
  a.in_coef_re = in_coef.real();
  a.in_coef_im = in_coef.imag();
  a.n = gp.n;
  a.c = gp.c;
  a.p = gp.p;
  a.m = op->m;
  a.flags = flags;
  if (in_coef != zd(1.0, 0.0)) a.flags |= KI_SCALE_IN;
  if ((flags & KI_ADD_PSI) && psi_coef != zd(1.0, 0.0)) a.flags |= KI_PSI_COEF;
  // few tiles per CU (latency-bound): fetch the phase entries with the tile;
  // complex128 only for the smallest states (register budget)
  if (gp.ntiles <= (sizeof(Real) == 4 ? 1024u : 512u)) a.flags |= KI_PREFETCH_PHASE;
  // passes with the phase over 16-amplitude tiles: the three-layout form
  KickMasks m3;
  unsigned c3 = 0;
  const int t3 = table3_mode(gp.n, gp.tb, gp.c, gp.p, op->m);
  if (!op->sw && gp.rb == 4 && pass3_flags_ok(a.flags) && t3 >= 0 && masks3_for(gp.kbits, gp.n, gp.tb, &m3, &c3)) {
    a.k1 = m3;
    a.k1c = c3;
    a.t3 = t3;
    a.k2 = k2 ? m3 : KickMasks{0, 0, 0, 0};
    a.k2c = k2 ? c3 : 0u;
    hipError_t e = ki_launch_pass3<Real>(a, gp.tb, gp.ntiles, s);
    if (e != hipSuccess) {
      set_error(std::string("kicked-Ising three-layout pass launch failed: ") + hipGetErrorString(e));
      return FQ_EDEVICE;
    }
    return FQ_OK;
  }
  if (gp.tb > 9) {
    set_error("internal: a 1024-thread kicked-Ising tile needs the three-layout pass");
    return FQ_EINVAL;
  }
  a.k1 = masks_for(gp.kbits, gp.n, gp.rb, gp.tb);
  a.k2 = k2 ? a.k1 : KickMasks{0, 0, 0, 0};
  hipError_t e = ki_launch_pass<Real>(a, gp.rb, gp.tb, op->sw, gp.ntiles, s);
  if (e != hipSuccess) {
    set_error(std::string("kicked-Ising pass launch failed: ") + hipGetErrorString(e));
    return FQ_EDEVICE;
  }
  return FQ_OK;
}

template <typename Real>
fq_status ki_apply_U(floquet_op* op, const void* psi, void* out, hipStream_t s) {
  const PhaseTables* tab;
  fq_status st = get_tables(op, 0.0, &tab);
  if (st != FQ_OK) return st;
  const bool c64_dt = sizeof(Real) == 4;
  const int smax = c64_dt ? op->single_max_L64 : op->single_max_L128;
  if (op->L <= smax && single_ok(op->L, c64_dt))
    return ki_single<Real>(op, tab, psi, psi, out, 1, 0, nullptr, zd(1, 0), 1, 0, s);
  const KiPlan& pl = c64_dt ? op->plan64 : op->plan128;
  const void* in = psi;
  for (int gi = pl.ngroups - 1; gi >= 0; --gi) {
    const bool last = gi == 0;
    st = ki_pass<Real>(op, pl.grp[gi], tab, in, out, nullptr, last ? KI_PHASE : 0, false, zd(1, 0), zd(1, 0), s);
    if (st != FQ_OK) return st;
    in = out;
  }
  return FQ_OK;
}

// Horner: w = a_k psi; k times w <- a_{step} psi + D K w.  For the geometric
// sum all a are 1 and the rotation lives in the tables.
template <typename Real>
fq_status ki_filter(floquet_op* op, int k, double phi, const zd* coefs, const void* psi, void* out,
                    hipStream_t s) {
  const PhaseTables* tab;
  fq_status st = get_tables(op, coefs ? 0.0 : phi, &tab);
  if (st != FQ_OK) return st;
  const size_t d = op->dim();
  const zd a_k = coefs ? coefs[k] : zd(1.0, 0.0);
  const bool c64_dt = sizeof(Real) == 4;
  const int smax = c64_dt ? op->single_max_L64 : op->single_max_L128;
  if (op->L <= smax && single_ok(op->L, c64_dt)) {
    const double2* cdev = nullptr;
    if (coefs) {
      if (op->coefs_cap < size_t(k)) {
        (void)hipFree(op->coefs_dev);
        op->coefs_dev = nullptr;
        op->coefs_cap = 0;
        FQ_HIP_CHECK(hipMalloc(&op->coefs_dev, sizeof(double2) * std::max(k, 16)));
        op->coefs_cap = std::max(k, 16);
      }
      std::vector<double2> hc(k);
      for (int i = 0; i < k; ++i) {
        hc[i].x = coefs[k - 1 - i].real();
        hc[i].y = coefs[k - 1 - i].imag();
      }
      FQ_HIP_CHECK(hipMemcpyAsync(op->coefs_dev, hc.data(), sizeof(double2) * k, hipMemcpyHostToDevice, s));
      FQ_HIP_CHECK(hipStreamSynchronize(s));
      cdev = op->coefs_dev;
    }
    return ki_single<Real>(op, tab, psi, psi, out, k, KI_ADD_PSI, cdev, a_k, 1, 0, s);
  }
  (void)d;
  const KiPlan& pl = c64_dt ? op->plan64 : op->plan128;
  if (pl.ngroups == 2) {
    // prologue: kick of group 1 (hi) on a_k psi; then steps alternate lo, hi, ...
    st = ki_pass<Real>(op, pl.grp[1], tab, psi, out, nullptr, 0, false, zd(1, 0), a_k, s);
    if (st != FQ_OK) return st;
    for (int step = 1; step <= k; ++step) {
      const KiGroup& gp = pl.grp[(step - 1) & 1];
      const zd c = coefs ? coefs[k - step] : zd(1.0, 0.0);
      st = ki_pass<Real>(op, gp, tab, out, out, psi, KI_PHASE | KI_ADD_PSI, step < k, c, zd(1, 0), s);
      if (st != FQ_OK) return st;
    }
    return FQ_OK;
  }
  // three groups: kick g2, kick g1, then kick g0 + phase + psi
  for (int step = 1; step <= k; ++step) {
    const void* in = step == 1 ? psi : out;
    const zd inc = step == 1 ? a_k : zd(1, 0);
    st = ki_pass<Real>(op, pl.grp[2], tab, in, out, nullptr, 0, false, zd(1, 0), inc, s);
    if (st != FQ_OK) return st;
    st = ki_pass<Real>(op, pl.grp[1], tab, out, out, nullptr, 0, false, zd(1, 0), zd(1, 0), s);
    if (st != FQ_OK) return st;
    const zd c = coefs ? coefs[k - step] : zd(1.0, 0.0);
    st = ki_pass<Real>(op, pl.grp[0], tab, out, out, psi, KI_PHASE | KI_ADD_PSI, false, c, zd(1, 0), s);
    if (st != FQ_OK) return st;
  }
  return FQ_OK;
}

fq_status check_ptrs(const floquet_op* op, const void* a, const void* b) {
  if (!op) {
    set_error("op is NULL");
    return FQ_EINVAL;
  }
  if (!a || !b) {
    set_error("device pointer is NULL");
    return FQ_EINVAL;
  }
  return FQ_OK;
}

}  // namespace

fq_status get_tables(floquet_op* op, double phi, const PhaseTables** out) {
  for (const PhaseTables& t : op->tables)
    if (t.phi == phi) {
      *out = &t;
      return FQ_OK;
    }
  if (op->tables.size() >= 8) {
    // tables may still be read by queued work: drain before freeing
    FQ_HIP_CHECK(hipDeviceSynchronize());
    free_tables(op->tables.front());
    op->tables.erase(op->tables.begin());
  }
  PhaseTables t;
  fq_status st = build_tables(op, phi, &t);
  if (st != FQ_OK) {
    free_tables(t);
    return st;
  }
  op->tables.push_back(t);
  *out = &op->tables.back();
  return FQ_OK;
}

fq_status apply_U_internal(floquet_op* op, fq_dtype dt, const void* psi, void* out, hipStream_t s) {
  if (op->model != FQ_KICKED_ISING) return bw_apply_U(op, dt, psi, out, s);
  return dt == FQ_C64 ? ki_apply_U<float>(op, psi, out, s) : ki_apply_U<double>(op, psi, out, s);
}

fq_status filter_internal(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi,
                          void* out, hipStream_t s) {
  const size_t bytes = op->dim() * (dt == FQ_C64 ? sizeof(c64) : sizeof(c128));
  if (k == 0) {
    if (coefs) return poly_scale_copy(op, coefs[0], dt, psi, out, s);
    FQ_HIP_CHECK(hipMemcpyAsync(out, psi, bytes, hipMemcpyDeviceToDevice, s));
    return FQ_OK;
  }
  if (op->model != FQ_KICKED_ISING) return bw_filter(op, k, phi, coefs, dt, psi, out, s);
  return dt == FQ_C64 ? ki_filter<float>(op, k, phi, coefs, psi, out, s)
                      : ki_filter<double>(op, k, phi, coefs, psi, out, s);
}

fq_status ensure_scratch32(floquet_op* op) {
  if (!op->psi32) FQ_HIP_CHECK(hipMalloc(&op->psi32, op->dim() * sizeof(c64)));
  if (!op->out32) FQ_HIP_CHECK(hipMalloc(&op->out32, op->dim() * sizeof(c64)));
  return FQ_OK;
}

fq_status filter_mixed(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi64,
                       void* out64, hipStream_t s) {
  if (dt == FQ_C128) return filter_internal(op, k, phi, coefs, FQ_C128, psi64, out64, s);
  fq_status st = ensure_scratch32(op);
  if (st != FQ_OK) return st;
  FQ_HIP_CHECK(launch_cast_c128_to_c64(psi64, op->psi32, op->dim(), s));
  st = filter_internal(op, k, phi, coefs, FQ_C64, op->psi32, op->out32, s);
  if (st != FQ_OK) return st;
  FQ_HIP_CHECK(launch_cast_c64_to_c128(op->out32, out64, op->dim(), s));
  return FQ_OK;
}

}  // namespace fq

using namespace fq;

extern "C" {

const char* floquet_last_error(void) { return g_last_error.c_str(); }

fq_status create_floquet_op(const fq_model_desc* desc, floquet_op** out) {
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return FQ_EINVAL;
  }
  *out = nullptr;
  if (!desc) {
    set_error("desc is NULL");
    return FQ_EINVAL;
  }
  if (desc->L < 2 || desc->L > 30) {
    set_error("L must satisfy 2 <= L <= 30");
    return FQ_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    set_error("no HIP device available");
    return FQ_EDEVICE;
  }
  std::unique_ptr<floquet_op> op(new floquet_op());
  op->model = desc->model;
  op->L = desc->L;
  op->periodic = desc->periodic ? 1 : 0;
  FQ_HIP_CHECK(hipGetDevice(&op->device));
  if (desc->model == FQ_KICKED_ISING) {
    if (!desc->J || !desc->h || desc->gates) {
      set_error("kicked Ising needs J and h (and gates == NULL)");
      return FQ_EINVAL;
    }
    if (!std::isfinite(desc->g)) {
      set_error("g must be finite");
      return FQ_EINVAL;
    }
    op->J.assign(desc->J, desc->J + desc->L);
    op->h.assign(desc->h, desc->h + desc->L);
    for (int i = 0; i < desc->L; ++i)
      if (!std::isfinite(op->J[i]) || !std::isfinite(op->h[i])) {
        set_error("J and h must be finite");
        return FQ_EINVAL;
      }
    op->g = desc->g;
    const double c = std::cos(desc->g), sn = std::sin(desc->g);
    if (std::fabs(sn) <= 2.0 * std::fabs(c)) {
      op->sw = false;
      op->w = -sn / c;
      op->site_scale = zd(c, 0.0);
    } else {
      op->sw = true;
      op->w = c / sn;
      op->site_scale = zd(0.0, -sn);
    }
    op->m = (op->L + 1) / 2;
    op->plan64 = make_plan(op->L, true, !op->sw);
    op->plan128 = make_plan(op->L, false, false);
    const PhaseTables* t;
    fq_status st = get_tables(op.get(), 0.0, &t);
    if (st != FQ_OK) return st;
  } else if (desc->model == FQ_BRICKWORK) {
    if (!desc->gates || desc->J || desc->h) {
      set_error("brickwork needs gates (and J == h == NULL)");
      return FQ_EINVAL;
    }
    if (desc->n_gates != desc->L + 1) {
      set_error("brickwork needs n_gates == L + 1");
      return FQ_EINVAL;
    }
    // count complex entries: two-site gates 16, one-site 4
    const int L = desc->L;
    const int n_single = 2;
    const int n_pair = L - 1;
    const size_t n_c = size_t(n_pair) * 16 + size_t(n_single) * 4;
    op->gates.resize(n_c);
    for (size_t i = 0; i < n_c; ++i) {
      op->gates[i] = zd(desc->gates[2 * i], desc->gates[2 * i + 1]);
      if (!std::isfinite(desc->gates[2 * i]) || !std::isfinite(desc->gates[2 * i + 1])) {
        set_error("gates must be finite");
        return FQ_EINVAL;
      }
    }
    fq_status st = bw_create(op.get());
    if (st != FQ_OK) return st;
  } else if (desc->model == FQ_CIRCUIT) {
    if (!desc->gates || desc->J || desc->h || !desc->gate_sites || !desc->gate_widths || desc->n_gates < 1) {
      set_error("circuit needs gates, gate_sites, gate_widths, n_gates >= 1 (and J == h == NULL)");
      return FQ_EINVAL;
    }
    const int L = desc->L;
    size_t n_c = 0;
    for (int q = 0; q < desc->n_gates; ++q) {
      const int i = desc->gate_sites[q], w = desc->gate_widths[q];
      if ((w != 1 && w != 2) || i < 1 || i + w - 1 > L) {
        set_error("circuit gate " + std::to_string(q) + ": need width 1 or 2 and sites inside 1..L");
        return FQ_EINVAL;
      }
      op->gate_sites.push_back(i);
      op->gate_widths.push_back(w);
      n_c += w == 1 ? 4 : 16;
    }
    if (n_c > (size_t(1) << 15) * 16) {
      set_error("circuit: too many gates");
      return FQ_EINVAL;
    }
    op->gates.resize(n_c);
    for (size_t i = 0; i < n_c; ++i) {
      op->gates[i] = zd(desc->gates[2 * i], desc->gates[2 * i + 1]);
      if (!std::isfinite(desc->gates[2 * i]) || !std::isfinite(desc->gates[2 * i + 1])) {
        set_error("gates must be finite");
        return FQ_EINVAL;
      }
    }
    fq_status st = bw_create(op.get());
    if (st != FQ_OK) return st;
  } else {
    set_error("unknown model");
    return FQ_EINVAL;
  }
  *out = op.release();
  return FQ_OK;
}

fq_status destroy_floquet_op(floquet_op* op) {
  clear_error();
  if (!op) return FQ_OK;
  (void)hipDeviceSynchronize();
  for (PhaseTables& t : op->tables) free_tables(t);
  bw_destroy(op);
  (void)hipFree(op->psi32);
  (void)hipFree(op->out32);
  (void)hipFree(op->coefs_dev);
  (void)hipFree(op->many_mem);
  (void)hipFree(op->chi_mem);
  (void)hipFree(op->V);
  (void)hipFree(op->work);
  (void)hipFree(op->work2);
  (void)hipFree(op->dev_small);
  (void)hipHostFree(op->host_small);
  delete op;
  return FQ_OK;
}

long long floquet_op_dim(const floquet_op* op) { return op ? (long long)op->dim() : 0; }

fq_status apply_U(floquet_op* op, fq_dtype dtype, const void* psi_dev, void* out_dev, void* hip_stream) {
  clear_error();
  fq_status st = check_ptrs(op, psi_dev, out_dev);
  if (st != FQ_OK) return st;
  if (dtype != FQ_C64 && dtype != FQ_C128) {
    set_error("bad dtype");
    return FQ_EINVAL;
  }
  return apply_U_internal(op, dtype, psi_dev, out_dev, static_cast<hipStream_t>(hip_stream));
}

fq_status apply_filter(floquet_op* op, int k, double phi, fq_dtype dtype, const void* psi_dev, void* out_dev,
                       void* hip_stream) {
  clear_error();
  fq_status st = check_ptrs(op, psi_dev, out_dev);
  if (st != FQ_OK) return st;
  if (k < 0 || !std::isfinite(phi) || (dtype != FQ_C64 && dtype != FQ_C128)) {
    set_error("apply_filter: need k >= 0, finite phi and a valid dtype");
    return FQ_EINVAL;
  }
  if (psi_dev == out_dev) {
    set_error("apply_filter: out must not alias psi");
    return FQ_EINVAL;
  }
  return filter_internal(op, k, phi, nullptr, dtype, psi_dev, out_dev, static_cast<hipStream_t>(hip_stream));
}

fq_status apply_filter_many(floquet_op* op, int k, double phi, fq_dtype dtype, int n_vec, const void* psi_dev,
                            void* out_dev, void* hip_stream) {
  clear_error();
  fq_status st = check_ptrs(op, psi_dev, out_dev);
  if (st != FQ_OK) return st;
  if (k < 0 || !std::isfinite(phi) || (dtype != FQ_C64 && dtype != FQ_C128) || n_vec < 1 || n_vec > 65535) {
    set_error("apply_filter_many: need k >= 0, finite phi, a valid dtype and 1 <= n_vec <= 65535");
    return FQ_EINVAL;
  }
  const size_t bytes = op->dim() * size_t(n_vec) * (dtype == FQ_C64 ? sizeof(c64) : sizeof(c128));
  const char* a = static_cast<const char*>(psi_dev);
  const char* b = static_cast<const char*>(out_dev);
  if (a < b + bytes && b < a + bytes) {
    set_error("apply_filter_many: out must not overlap psi");
    return FQ_EINVAL;
  }
  return filter_many(op, k, phi, dtype, n_vec, psi_dev, out_dev, static_cast<hipStream_t>(hip_stream));
}

fq_status apply_polynomial(floquet_op* op, int k, const double* coeffs_host, fq_dtype dtype, const void* psi_dev,
                           void* out_dev, void* hip_stream) {
  clear_error();
  fq_status st = check_ptrs(op, psi_dev, out_dev);
  if (st != FQ_OK) return st;
  if (k < 0 || !coeffs_host || (dtype != FQ_C64 && dtype != FQ_C128)) {
    set_error("apply_polynomial: need k >= 0, coefficients and a valid dtype");
    return FQ_EINVAL;
  }
  if (psi_dev == out_dev) {
    set_error("apply_polynomial: out must not alias psi");
    return FQ_EINVAL;
  }
  std::vector<zd> c(k + 1);
  for (int i = 0; i <= k; ++i) {
    c[i] = zd(coeffs_host[2 * i], coeffs_host[2 * i + 1]);
    if (!std::isfinite(c[i].real()) || !std::isfinite(c[i].imag())) {
      set_error("apply_polynomial: coefficients must be finite");
      return FQ_EINVAL;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  return filter_internal(op, k, 0.0, c.data(), dtype, psi_dev, out_dev, s);
}

}  // extern "C"
