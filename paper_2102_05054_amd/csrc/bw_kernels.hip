// Brickwork random-circuit passes (Sec. 2, Eq. (U), Eq. (unitary)).
//
// U = U_a U_b with U_b acting first.  Cutting the chain at an even site c_s,
// the gates split into a right block on sites c_s..L (U_b's gates from
// (c_s, c_s+1) on, then U_a's gates right of c_s) and a left block on sites
// 1..c_s; the right block's U_a gates commute with the left block's U_b
// gates, so U = U_L U_R with U_R first -- the light-cone split behind the
// paper's two-GEMM product (Eq. (matvec)), used here as two tile passes.
//   right pass: tile = global bits [0, L - c_s], contiguous;
//   left pass:  tile = a chunk of low bits + global bits [L - c_s, L),
//               then e^{-i phi} and +psi for the Horner step.
// One Horner step = right pass (read w, write w) + left pass (read w, read
// psi, write w).  Inside a tile the gates are applied in windows of WB
// consecutive tile bits: each thread takes the 2^WB amplitudes of one window
// group from LDS into registers, applies the window's gates in order, and
// writes them back.  A host scheduler fills each window with up to eight
// gates of either layer whose bits lie inside it and whose earlier gates on
// the same sites are done, so any order of local gates (more layers, other
// gate sets) maps onto the same windows.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <deque>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "bw_kernels.h"
#include "op.h"

namespace fq {

namespace {

__device__ __forceinline__ int bw_phys(int j) { return j + (j >> 4); }

// 4x4 gate on window bits (L0, L0+1)
template <typename Real, int WB, int L0>
__device__ __forceinline__ void gate2(cpx<Real> (&v)[1 << WB], const cpx<Real> (&m)[16]) {
  constexpr int lo = 1 << L0, hi = 1 << (L0 + 1);
#pragma unroll
  for (int base = 0; base < (1 << WB); ++base) {
    if (base & (lo | hi)) continue;
    const int idx[4] = {base, base | lo, base | hi, base | hi | lo};  // local index 2*b_hi + b_lo
    cpx<Real> x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = v[idx[c]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cpx<Real> acc = cmul(m[4 * r], x[0]);
#pragma unroll
      for (int c = 1; c < 4; ++c) acc = cfma(m[4 * r + c], x[c], acc);
      v[idx[r]] = acc;
    }
  }
}

template <typename Real, int WB, int L0>
__device__ __forceinline__ void gate1(cpx<Real> (&v)[1 << WB], const cpx<Real> (&m)[16]) {
  constexpr int bit = 1 << L0;
#pragma unroll
  for (int base = 0; base < (1 << WB); ++base) {
    if (base & bit) continue;
    const cpx<Real> x = v[base], y = v[base | bit];
    v[base] = cfma(m[1], y, cmul(m[0], x));
    v[base | bit] = cfma(m[3], y, cmul(m[2], x));
  }
}

// kind 2: two-site gate on window bits (l, l+1); kind 1: one-site gate on l
template <typename Real, int WB>
__device__ __forceinline__ void apply_gate(cpx<Real> (&v)[1 << WB], int kind, int l, const cpx<Real> (&m)[16]) {
  if (kind == 2) {
    if (l == 0) gate2<Real, WB, 0>(v, m);
    if constexpr (WB >= 3)
      if (l == 1) gate2<Real, WB, 1>(v, m);
    if constexpr (WB >= 4)
      if (l == 2) gate2<Real, WB, 2>(v, m);
    if constexpr (WB >= 5)
      if (l == 3) gate2<Real, WB, 3>(v, m);
  } else {
    if (l == 0) gate1<Real, WB, 0>(v, m);
    if (l == 1) gate1<Real, WB, 1>(v, m);
    if constexpr (WB >= 3)
      if (l == 2) gate1<Real, WB, 2>(v, m);
    if constexpr (WB >= 4)
      if (l == 3) gate1<Real, WB, 3>(v, m);
    if constexpr (WB >= 5)
      if (l == 4) gate1<Real, WB, 4>(v, m);
  }
}

// Window and gate fields are made wave-uniform (scalar registers), so that
// the gate dispatch branches on scalars and the matrices are scalar loads.
struct WinU {
  int b, first, count;
};
__device__ __forceinline__ WinU load_win(const BwWin* p) {
  const int2 raw = *reinterpret_cast<const int2*>(p);
  const int x = __builtin_amdgcn_readfirstlane(raw.x);
  const int y = __builtin_amdgcn_readfirstlane(raw.y);
  WinU w;
  w.b = static_cast<int16_t>(x & 0xffff);
  w.first = static_cast<int16_t>((x >> 16) & 0xffff);
  w.count = static_cast<int16_t>(y & 0xffff);
  return w;
}
struct GateU {
  int kind, l, mat;
};
__device__ __forceinline__ GateU load_gate(const BwGate* p) {
  const int x = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int*>(p));
  GateU g;
  g.kind = x & 0xff;
  g.l = (x >> 8) & 0xff;
  g.mat = (x >> 16) & 0xffff;
  return g;
}

// Apply the window's gates, in order, to the group of 2^WB amplitudes held in
// v, with one matrix live at a time, read (scalar loads, served by the scalar
// cache) just before its gate.  A complex128 matrix takes 64 scalar
// registers: holding two or more across the window spills scalar registers
// into vector lanes, where every matrix use costs a lane read; one at a time,
// a window can take any number of gates, and fewer windows mean fewer LDS
// round trips.
template <typename Real, int WB>
__device__ __forceinline__ void window_gates(cpx<Real> (&v)[1 << WB], const WinU& w, const BwGate* __restrict__ gates,
                                             const cpx<Real>* __restrict__ mats) {
#pragma unroll 1
  for (int q = 0; q < w.count; ++q) {
    const GateU g = load_gate(gates + w.first + q);
    cpx<Real> m[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) m[i] = mats[16 * g.mat + i];
    apply_gate<Real, WB>(v, g.kind, g.l, m);
    asm volatile("" ::: "memory");  // keeps the next matrix's loads after this gate
  }
}

template <typename Real, int WB, int TB>
__global__ void __launch_bounds__(1 << TB)
    bw_pass_kernel(BwPassArgs a, const cpx<Real>* __restrict__ mats, const BwWin* __restrict__ wins,
                   const BwGate* __restrict__ gates) {
  using C = cpx<Real>;
  constexpr int T = 1 << TB;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x;
  const int N = 1 << a.n;
  const uint32_t item = xcd_tile(blockIdx.x, gridDim.x);
  const TileMap tm = make_tile_map(item & ((1u << a.tile_bits) - 1u), a.n, a.c, a.p);
  const size_t voff = size_t(item >> a.tile_bits) * a.vstride;
  const C* __restrict__ xin = static_cast<const C*>(a.xin) + voff;
  C* __restrict__ xout = static_cast<C*>(a.xout) + voff;
  const int ngroups = N >> WB;
  // insert WB zero bits at position b: the first amplitude of window group g
  auto group_base = [](uint32_t g, int b) {
    return static_cast<int>((g & ((1u << b) - 1u)) | ((g >> b) << (b + WB)));
  };
  // The first window is applied on the way in and the last on the way out
  // (one LDS write, resp. read, instead of a full round trip each) when
  // every thread owns a window group.  For a window at low tile bits the
  // lanes then touch strided 16-byte pieces, but consecutive accesses of a
  // thread fill the same lines: fusing at any position measured 1-3 %
  // faster than only for windows at tile bit 4 and up (L = 16..20).
  const bool own = ngroups >= T;
  int first = 0, last = a.nwin;
  if (own && a.nwin > 0) first = 1;
  if (own && a.nwin > first) last = a.nwin - 1;
  if (first == 1) {
    const WinU w = load_win(wins);
    for (int g = tid; g < ngroups; g += T) {
      const int base = group_base(uint32_t(g), w.b);
      C v[1 << WB];
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) v[m] = xin[tm.g(base + (m << w.b))];
      window_gates<Real, WB>(v, w, gates, mats);
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) lds[bw_phys(base + (m << w.b))] = v[m];
    }
  } else {
    for (int j = tid; j < N; j += T) lds[bw_phys(j)] = xin[tm.g(j)];
  }
  __syncthreads();
  for (int wi = first; wi < last; ++wi) {
    const WinU w = load_win(wins + wi);
    for (int g = tid; g < ngroups; g += T) {
      const int base = group_base(uint32_t(g), w.b);
      C v[1 << WB];
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) v[m] = lds[bw_phys(base + (m << w.b))];
      window_gates<Real, WB>(v, w, gates, mats);
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) lds[bw_phys(base + (m << w.b))] = v[m];
    }
    __syncthreads();
  }
  const C rot = mk<Real>(static_cast<Real>(a.rot_re), static_cast<Real>(a.rot_im));
  const C pc = mk<Real>(static_cast<Real>(a.psi_coef_re), static_cast<Real>(a.psi_coef_im));
  const C* __restrict__ psi = static_cast<const C*>(a.psi) + voff;
  auto finish = [&](C x, uint32_t g) {
    if (a.flags & BW_ROT) x = cmul(x, rot);
    if (a.flags & BW_ADD_PSI) x = (a.flags & BW_PSI_COEF) ? cfma(psi[g], pc, x) : cadd(x, psi[g]);
    xout[g] = x;
  };
  if (last < a.nwin) {
    const WinU w = load_win(wins + last);
    for (int g = tid; g < ngroups; g += T) {
      const int base = group_base(uint32_t(g), w.b);
      C v[1 << WB];
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) v[m] = lds[bw_phys(base + (m << w.b))];
      window_gates<Real, WB>(v, w, gates, mats);
#pragma unroll
      for (int m = 0; m < (1 << WB); ++m) finish(v[m], tm.g(base + (m << w.b)));
    }
  } else {
    for (int j = tid; j < N; j += T) finish(lds[bw_phys(j)], tm.g(j));
  }
}

// Tile pass with one window group per thread kept in registers, moved
// between windows through LDS one plane at a time (real parts, then
// imaginary parts): the LDS holds sizeof(Real) bytes per amplitude instead
// of twice that, so that more workgroups fit a CU (complex128 2^11 / 2^12
// tiles: 17 / 35 KB; complex64 2^13 / 2^14 tiles: 34 / 68 KB).  Between two
// windows a thread writes the real parts of its sixteen amplitudes at the
// current window's positions, reads the real parts at the next window's
// positions into the freed registers, and does the same for the imaginary
// parts (three barriers instead of one; a thread only rewrites positions it
// owns in the next layout, which nobody else reads).  The first window is
// applied on the way in from global memory, the last on the way out.
template <typename Real, int WB, int TB>
__global__ void __launch_bounds__(1 << TB)
    bw_pass_split_kernel(BwPassArgs a, const cpx<Real>* __restrict__ mats, const BwWin* __restrict__ wins,
                         const BwGate* __restrict__ gates) {
  using C = cpx<Real>;
  constexpr int R = 1 << WB;
  extern __shared__ char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  const uint32_t g = threadIdx.x;  // the thread's window group
  const uint32_t item = xcd_tile(blockIdx.x, gridDim.x);
  const TileMap tm = make_tile_map(item & ((1u << a.tile_bits) - 1u), a.n, a.c, a.p);
  const size_t voff = size_t(item >> a.tile_bits) * a.vstride;
  const C* __restrict__ xin = static_cast<const C*>(a.xin) + voff;
  C* __restrict__ xout = static_cast<C*>(a.xout) + voff;
  auto group_base = [](uint32_t gg, int b) {
    return static_cast<int>((gg & ((1u << b) - 1u)) | ((gg >> b) << (b + WB)));
  };
  int b = 0;
  if (a.nwin > 0) b = load_win(wins).b;
  int base = group_base(g, b);
  C v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = xin[tm.g(base + (m << b))];
  for (int wi = 0; wi < a.nwin; ++wi) {
    const WinU w = load_win(wins + wi);
    if (wi > 0) {
      const int nbase = group_base(g, w.b);
#pragma unroll
      for (int m = 0; m < R; ++m) lds[bw_phys(base + (m << b))] = v[m].x;
      __syncthreads();
#pragma unroll
      for (int m = 0; m < R; ++m) v[m].x = lds[bw_phys(nbase + (m << w.b))];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < R; ++m) lds[bw_phys(base + (m << b))] = v[m].y;
      __syncthreads();
#pragma unroll
      for (int m = 0; m < R; ++m) v[m].y = lds[bw_phys(nbase + (m << w.b))];
      base = nbase;
      b = w.b;
    }
    window_gates<Real, WB>(v, w, gates, mats);
  }
  const C rot = mk<Real>(static_cast<Real>(a.rot_re), static_cast<Real>(a.rot_im));
  const C pc = mk<Real>(static_cast<Real>(a.psi_coef_re), static_cast<Real>(a.psi_coef_im));
  const C* __restrict__ psi = static_cast<const C*>(a.psi) + voff;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const uint32_t gi = tm.g(base + (m << b));
    C x = v[m];
    if (a.flags & BW_ROT) x = cmul(x, rot);
    if (a.flags & BW_ADD_PSI) x = (a.flags & BW_PSI_COEF) ? cfma(psi[gi], pc, x) : cadd(x, psi[gi]);
    xout[gi] = x;
  }
}

size_t bw_lds_bytes(int n, size_t elem) { return size_t((1 << n) + (1 << (n - 4 > 0 ? n - 4 : 0)) + 1) * elem; }

template <typename Real, int WB, int TB>
hipError_t launch_bw_split(const BwPassArgs& a, unsigned nitems, hipStream_t s) {
  const size_t shmem = bw_lds_bytes(a.n, sizeof(Real));
  auto kern = bw_pass_split_kernel<Real, WB, TB>;
  static size_t attr_bytes = 65536;  // dynamic LDS admitted so far
  if (shmem > attr_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
    attr_bytes = shmem;
  }
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(1 << TB), shmem, s, a, static_cast<const cpx<Real>*>(a.mats), a.wins,
                     a.gates);
  return hipGetLastError();
}

template <typename Real, int WB, int TB>
hipError_t launch_bw_t(const BwPassArgs& a, unsigned nitems, hipStream_t s) {
  const size_t shmem = bw_lds_bytes(a.n, sizeof(cpx<Real>));
  auto kern = bw_pass_kernel<Real, WB, TB>;
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(1 << TB), shmem, s, a, static_cast<const cpx<Real>*>(a.mats), a.wins,
                     a.gates);
  return hipGetLastError();
}

}  // namespace

// Tile kernels take one thread per window group (2^(n - wb) of them, at
// least one wave): with more threads than groups the extra lanes idle through
// every window.  Launches too small to give every SIMD a wave that way take
// larger workgroups (up to 256 threads, 512 for 2^13-amplitude and larger
// tiles, and for complex64 2^12), whose extra threads still share the tile's
// loads and stores.
hipError_t bw_launch_pass(const BwPassArgs& a, bool c64_dt, int wb, unsigned nitems, hipStream_t s) {
  // complex64 2^13- and 2^14-amplitude tiles: one window group per thread
  // (512 and 1024 threads), planes through 34 and 68 KiB of LDS.  Against
  // a persistent kernel that kept the whole tile in LDS (136 KiB for 2^14:
  // one workgroup per CU) and prefetched the next tile into registers, the
  // L = 24 Horner step went from 359 to 272 us.
  if (c64_dt && wb == 4 && a.n == 13) return launch_bw_split<float, 4, 9>(a, nitems, s);
  if (c64_dt && wb == 4 && a.n == 14) return launch_bw_split<float, 4, 10>(a, nitems, s);
  const int tb_max = (a.n >= 13 || (c64_dt && a.n >= 12)) ? 9 : 8;
  int tb = std::max(6, std::min(tb_max, a.n - wb));
  while (tb < tb_max && (static_cast<uint64_t>(nitems) << (tb - 6)) < 1024u) ++tb;
  if (c64_dt) {
    if (wb == 4) {
      if (tb == 9) return launch_bw_t<float, 4, 9>(a, nitems, s);
      if (tb == 8) return launch_bw_t<float, 4, 8>(a, nitems, s);
      if (tb == 7) return launch_bw_t<float, 4, 7>(a, nitems, s);
      return launch_bw_t<float, 4, 6>(a, nitems, s);
    }
    if (wb == 3) return launch_bw_t<float, 3, 6>(a, nitems, s);
    if (wb == 2) return launch_bw_t<float, 2, 6>(a, nitems, s);
  } else {
    // one window group per thread in 2^11- and 2^12-amplitude tiles: the
    // plane-split form (L = 20, 4 vectors: 27.3 -> 24.2 us per U and
    // vector; for 2^13-amplitude tiles its extra barriers cost more than the
    // smaller LDS gains, since registers already limit those to one
    // workgroup per CU: 651 -> 664 us per step at L = 24)
    if (wb == 4 && tb == a.n - 4 && tb <= 8) {
      if (tb == 8) return launch_bw_split<double, 4, 8>(a, nitems, s);
      if (tb == 7) return launch_bw_split<double, 4, 7>(a, nitems, s);
    }
    if (wb == 4) {
      if (tb == 9) return launch_bw_t<double, 4, 9>(a, nitems, s);
      if (tb == 8) return launch_bw_t<double, 4, 8>(a, nitems, s);
      if (tb == 7) return launch_bw_t<double, 4, 7>(a, nitems, s);
      return launch_bw_t<double, 4, 6>(a, nitems, s);
    }
    if (wb == 3) return launch_bw_t<double, 3, 6>(a, nitems, s);
    if (wb == 2) return launch_bw_t<double, 2, 6>(a, nitems, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Host: gate programs
// ---------------------------------------------------------------------------

namespace {

struct GateRef {
  int site;   // first site (1-based)
  int width;  // 1 or 2
  int mat;    // matrix index
};

// Sites of every gate in the flat order: layer b then layer a (see floquet.h).
void layout(int L, std::vector<std::vector<int>>* lb, std::vector<std::vector<int>>* la) {
  lb->clear();
  la->clear();
  if (L % 2 == 0) {
    lb->push_back({1});
    for (int i = 2; i <= L - 2; i += 2) lb->push_back({i, i + 1});
    lb->push_back({L});
    for (int i = 1; i <= L - 1; i += 2) la->push_back({i, i + 1});
  } else {
    lb->push_back({1});
    for (int i = 2; i <= L - 1; i += 2) lb->push_back({i, i + 1});
    for (int i = 1; i <= L - 2; i += 2) la->push_back({i, i + 1});
    la->push_back({L});
  }
}

// A gate of one pass: tile low bit q, width 1 or 2, matrix index.  Gates are
// listed in program order (the layer acting first, then the second).
struct PGate {
  int q, width, mat;
};

// Windows of wb consecutive tile bits covering all gates of a pass.  A window
// takes, in program order, every remaining gate inside it whose earlier
// gates on shared bits are already applied (in earlier windows or earlier in
// this one); gates on disjoint bits commute, so this reproduces the program.
// Greedy placement: the window starts at the first remaining gate's low bit
// or up to wb - 2 bits below it, whichever placement applies the most gates.
void schedule_windows_greedy(const std::vector<PGate>& g, int n, int wb, size_t kMaxGates,
                             std::vector<BwWin>* wins, std::vector<BwGate>* out) {
  const size_t G = g.size();
  std::vector<char> done(G, 0);
  auto overlaps = [&](size_t i, size_t j) { return g[i].q < g[j].q + g[j].width && g[j].q < g[i].q + g[i].width; };
  auto pick = [&](int b, std::vector<size_t>* sel) {
    std::vector<char> d = done;
    sel->clear();
    for (size_t j = 0; j < G && sel->size() < kMaxGates; ++j) {
      if (d[j] || g[j].q < b || g[j].q + g[j].width > b + wb) continue;
      bool ready = true;
      for (size_t i = 0; i < j && ready; ++i)
        if (!d[i] && overlaps(i, j)) ready = false;
      if (ready) {
        d[j] = 1;
        sel->push_back(j);
      }
    }
  };
  size_t left = G;
  while (left > 0) {
    size_t f = 0;
    while (done[f]) ++f;
    std::vector<size_t> best, cur;
    int bb = 0;
    for (int dq = 0; dq == 0 || dq < wb - 1; ++dq) {
      const int b = std::max(0, std::min(g[f].q - dq, n - wb));
      pick(b, &cur);
      if (cur.size() > best.size()) {
        best = cur;
        bb = b;
      }
    }
    wins->push_back(BwWin{static_cast<int16_t>(bb), static_cast<int16_t>(out->size()),
                          static_cast<int16_t>(best.size()), 0});
    for (size_t j : best) {
      out->push_back(BwGate{static_cast<int8_t>(g[j].width), static_cast<int8_t>(g[j].q - bb),
                            static_cast<int16_t>(g[j].mat)});
      done[j] = 1;
      --left;
    }
  }
}

// The gates one window at bit b applies to the applied set `done` (bit j =
// gate j), by the rule above; returns the new set and appends the gates, in
// program order, to sel (if given).
uint64_t window_step(const std::vector<PGate>& g, uint64_t done, int b, int wb, size_t kMaxGates,
                     std::vector<size_t>* sel) {
  size_t taken = 0;
  for (size_t j = 0; j < g.size() && taken < kMaxGates; ++j) {
    if (((done >> j) & 1u) || g[j].q < b || g[j].q + g[j].width > b + wb) continue;
    bool ready = true;
    for (size_t i = 0; i < j && ready; ++i)
      if (!((done >> i) & 1u) && g[i].q < g[j].q + g[j].width && g[j].q < g[i].q + g[i].width) ready = false;
    if (!ready) continue;
    done |= uint64_t(1) << j;
    ++taken;
    if (sel) sel->push_back(j);
  }
  return done;
}

// Fewest windows: a breadth-first search over the applied-gate sets, one
// window placement (b = 0 .. n - wb) per step.  The greedy placement misses
// windows that straddle two earlier ones (a brickwork pass of 13 bits takes 6
// windows greedily, 4 this way).  Among the shortest schedules the first and
// the last window sit as high as possible, up to line_bits: the tile kernels
// apply them on the way in from and out to global memory, where a window at
// bit b leaves runs of 2^b consecutive amplitudes across the lanes (whole
// 128-byte lines from b = line_bits on).  A brickwork pass reaches a few
// hundred sets; programs of more than 64 gates, or whose search passes 2^16
// sets, keep the greedy schedule.
void schedule_windows(const std::vector<PGate>& g, int n, int wb, size_t kMaxGates, int line_bits,
                      std::vector<BwWin>* wins, std::vector<BwGate>* out) {
  const size_t G = g.size();
  if (G == 0) return;
  if (G > 64 || n < wb) {
    schedule_windows_greedy(g, n, wb, kMaxGates, wins, out);
    return;
  }
  const uint64_t full = G == 64 ? ~uint64_t(0) : (uint64_t(1) << G) - 1u;
  struct Node {
    int level, score;  // windows so far; score of the first window
    uint64_t from;     // best predecessor set
    int b;             // bit of the window from it
  };
  std::unordered_map<uint64_t, Node> node;
  std::vector<uint64_t> order{0};  // breadth-first order
  node.emplace(0, Node{0, 0, 0, -1});
  int depth = -1, best = -1, best_b = -1;
  uint64_t best_from = 0;
  bool overflow = false;
  for (size_t qi = 0; qi < order.size() && !overflow; ++qi) {
    const uint64_t s = order[qi];
    const Node ns = node.at(s);
    if (depth >= 0 && ns.level >= depth) break;  // no shorter schedule remains
    for (int b = 0; b + wb <= n; ++b) {
      const uint64_t t = window_step(g, s, b, wb, kMaxGates, nullptr);
      if (t == s) continue;
      const int score = ns.level == 0 ? std::min(b, line_bits) : ns.score;
      if (t == full) {
        depth = ns.level + 1;
        if (score + std::min(b, line_bits) > best) {
          best = score + std::min(b, line_bits);
          best_from = s;
          best_b = b;
        }
        continue;
      }
      auto it = node.find(t);
      if (it == node.end()) {
        if (node.size() >= (size_t(1) << 16)) {
          overflow = true;
          break;
        }
        node.emplace(t, Node{ns.level + 1, score, s, b});
        order.push_back(t);
      } else if (it->second.level == ns.level + 1 && score > it->second.score) {
        it->second.score = score;
        it->second.from = s;
        it->second.b = b;
      }
    }
  }
  if (overflow || best < 0) {
    schedule_windows_greedy(g, n, wb, kMaxGates, wins, out);
    return;
  }
  std::vector<int> bits{best_b};
  for (uint64_t s = best_from; s != 0; s = node.at(s).from) bits.push_back(node.at(s).b);
  std::reverse(bits.begin(), bits.end());
  uint64_t done = 0;
  for (int b : bits) {
    std::vector<size_t> sel;
    done = window_step(g, done, b, wb, kMaxGates, &sel);
    wins->push_back(BwWin{static_cast<int16_t>(b), static_cast<int16_t>(out->size()),
                          static_cast<int16_t>(sel.size()), 0});
    for (size_t j : sel)
      out->push_back(BwGate{static_cast<int8_t>(g[j].width), static_cast<int8_t>(g[j].q - b),
                            static_cast<int16_t>(g[j].mat)});
  }
  if (done != full) {  // cannot happen: every step of the search applied its gates
    wins->clear();
    out->clear();
    schedule_windows_greedy(g, n, wb, kMaxGates, wins, out);
  }
}

}  // namespace

struct BwProgram {
  // per pass: windows on the device, tile geometry
  struct Pass {
    int n, c, p, wb;
    unsigned ntiles;
    BwWin* wins = nullptr;
    BwGate* gates = nullptr;
    int nwin = 0;
  };
  int L = 0;  // amplitudes per vector: 2^L
  int npass = 0;
  Pass pass[2];  // [0] applied first (right block), [1] second (left block)
  void* mats = nullptr;  // 16-entry matrices, complex64 or complex128 (rounded once)
  bool c64 = true;

  ~BwProgram() {
    for (Pass& p : pass) {
      (void)hipFree(p.wins);
      (void)hipFree(p.gates);
    }
    (void)hipFree(mats);
  }
};

namespace {

// The gates in acting order: the brickwork layout (U_b, then U_a) or a
// general circuit's list.
std::vector<GateRef> gate_refs(const floquet_op* op) {
  std::vector<GateRef> refs;
  if (op->model == FQ_CIRCUIT) {
    for (size_t q = 0; q < op->gate_sites.size(); ++q)
      refs.push_back({op->gate_sites[q], op->gate_widths[q], static_cast<int>(q)});
    return refs;
  }
  std::vector<std::vector<int>> lb, la;
  layout(op->L, &lb, &la);
  int mi = 0;
  for (const auto* lst : {&lb, &la})
    for (const auto& sites : *lst) refs.push_back({sites[0], static_cast<int>(sites.size()), mi++});
  return refs;
}

// Right block of the cut at site cs: in acting order, every gate on sites >= cs
// whose earlier gates on shared sites are all in the block.  The rest (the
// left block) then commutes past it, so U = U_left U_right with U_right first.
// Returns the membership and the largest site a left-block gate touches.
std::vector<char> right_block(const std::vector<GateRef>& refs, int cs, int* left_max_site) {
  const size_t G = refs.size();
  std::vector<char> right(G, 0);
  *left_max_site = 0;
  for (size_t j = 0; j < G; ++j) {
    const int j0 = refs[j].site, j1 = refs[j].site + refs[j].width - 1;
    bool r = j0 >= cs;
    for (size_t i = 0; i < j && r; ++i) {
      const int i0 = refs[i].site, i1 = refs[i].site + refs[i].width - 1;
      if (!right[i] && i0 <= j1 && j0 <= i1) r = false;
    }
    right[j] = r ? 1 : 0;
    if (!r) *left_max_site = std::max(*left_max_site, j1);
  }
  return right;
}

fq_status build_program(floquet_op* op, bool c64_dt, std::shared_ptr<BwProgram>* out) {
  const int L = op->L;
  auto prog = std::make_shared<BwProgram>();
  prog->c64 = c64_dt;
  prog->L = L;
  const std::vector<GateRef> refs = gate_refs(op);
  // matrices: each padded to 16 complex (one-site gates use the first 4)
  std::vector<c128> mats;
  size_t pos = 0;
  for (const GateRef& r : refs) {
    const int nn = r.width == 1 ? 4 : 16;
    if (pos + nn > op->gates.size()) {
      set_error("internal: gate matrices shorter than the gate list");
      return FQ_EINVAL;
    }
    for (int e = 0; e < 16; ++e) {
      const zd z = e < nn ? op->gates[pos + e] : zd(0, 0);
      mats.push_back(mk<double>(z.real(), z.imag()));
    }
    pos += nn;
  }
  if (mats.size() / 16 > 32767) {
    set_error("circuit: too many gates for the window descriptors");
    return FQ_EINVAL;
  }
  if (c64_dt) {
    std::vector<c64> m32(mats.size());
    for (size_t i = 0; i < mats.size(); ++i) m32[i] = mk<float>(float(mats[i].x), float(mats[i].y));
    FQ_HIP_CHECK(hipMalloc(&prog->mats, m32.size() * sizeof(c64)));
    FQ_HIP_CHECK(hipMemcpy(prog->mats, m32.data(), m32.size() * sizeof(c64), hipMemcpyHostToDevice));
  } else {
    FQ_HIP_CHECK(hipMalloc(&prog->mats, mats.size() * sizeof(c128)));
    FQ_HIP_CHECK(hipMemcpy(prog->mats, mats.data(), mats.size() * sizeof(c128), hipMemcpyHostToDevice));
  }

  const int nmax = c64_dt ? 13 : 12;
  // window width: 4 bits (16 amplitudes per thread); 5-bit windows with all
  // fitting gates cover a 13-bit block in 3 instead of 7 windows but raise
  // register use so much that the pass gets slower (392 against 377 us at
  // L = 24)
  auto window_bits = [&](int n) { return std::min(4, n); };
  auto upload = [&](BwProgram::Pass& ps, const std::vector<PGate>& g) -> fq_status {
    std::vector<BwWin> wins;
    std::vector<BwGate> gl;
    if (!g.empty())
      schedule_windows(g, ps.n, ps.wb, kBwWindowGates, c64_dt ? 4 : 3, &wins, &gl);
    ps.nwin = static_cast<int>(wins.size());
    FQ_HIP_CHECK(hipMalloc(&ps.wins, std::max<size_t>(1, wins.size()) * sizeof(BwWin)));
    FQ_HIP_CHECK(hipMalloc(&ps.gates, std::max<size_t>(1, gl.size()) * sizeof(BwGate)));
    if (!wins.empty()) {
      FQ_HIP_CHECK(hipMemcpy(ps.wins, wins.data(), wins.size() * sizeof(BwWin), hipMemcpyHostToDevice));
      FQ_HIP_CHECK(hipMemcpy(ps.gates, gl.data(), gl.size() * sizeof(BwGate), hipMemcpyHostToDevice));
    }
    return FQ_OK;
  };
  if (L <= nmax) {
    prog->npass = 1;
    BwProgram::Pass& ps = prog->pass[0];
    ps.n = L;
    ps.c = L;
    ps.p = L;
    ps.wb = window_bits(L);
    ps.ntiles = 1;
    std::vector<PGate> g;
    for (const GateRef& r : refs) g.push_back({L - (r.site + r.width - 1), r.width, r.mat});
    return (upload(ps, g) == FQ_OK) ? (*out = prog, FQ_OK) : FQ_EDEVICE;
  }
  // choose the cut site c_s and chunk c so that both tiles fit in LDS (<= 14
  // bits complex64, <= 13 bits complex128), balancing the two tiles; for the
  // brickwork this gives an even c_s (the light cone of U_a U_b)
  const int nfit = c64_dt ? 14 : 13;
  int best_cs = -1, best_c = 0, best_left = 0;
  for (int c = c64_dt ? 3 : 2; c >= 1 && best_cs < 0; --c) {
    int best_span = 1 << 30, best_sum = 1 << 30;
    for (int cs = 2; cs <= L - 1; ++cs) {
      int left_max = 0;
      (void)right_block(refs, cs, &left_max);
      const int nR = L - cs + 1, nL = std::max(left_max, 1) + c;
      if (left_max >= L) continue;
      const int span = std::max(nR, nL), sum = nR + nL;
      if (nR <= nfit && nL <= nfit && (span < best_span || (span == best_span && sum < best_sum))) {
        best_span = span;
        best_sum = sum;
        best_cs = cs;
        best_left = std::max(left_max, 1);
      }
    }
    if (best_cs >= 0) best_c = c;
  }
  if (best_cs < 0) {
    set_error("no two-block split of the circuit for L = " + std::to_string(L) +
              " (light cone too wide for tiles of " + std::to_string(nfit) + " bits)");
    return FQ_EINVAL;
  }
  const int cs = best_cs, c = best_c;
  int left_max = 0;
  const std::vector<char> right = right_block(refs, cs, &left_max);
  prog->npass = 2;
  // right block: sites cs..L -> global bits [0, L-cs]
  BwProgram::Pass& pr = prog->pass[0];
  pr.n = L - cs + 1;
  pr.c = pr.n;
  pr.p = pr.n;
  pr.wb = window_bits(pr.n);
  pr.ntiles = 1u << (L - pr.n);
  // left block: sites 1..best_left -> global bits [L-best_left, L); tile bit = c + (gbit - (L-best_left))
  BwProgram::Pass& pl = prog->pass[1];
  pl.n = best_left + c;
  pl.c = c;
  pl.p = L - best_left;
  pl.wb = window_bits(pl.n);
  pl.ntiles = 1u << (L - pl.n);
  for (int which = 0; which < 2; ++which) {
    BwProgram::Pass& ps = prog->pass[which];
    std::vector<PGate> g;
    for (size_t q = 0; q < refs.size(); ++q) {
      if ((right[q] != 0) != (which == 0)) continue;
      const GateRef& r = refs[q];
      const int gbit_lo = L - (r.site + r.width - 1);  // global bit of the gate's last (low) site
      const int tbit = which == 0 ? gbit_lo : c + (gbit_lo - pl.p);
      if (tbit < (which == 0 ? 0 : c) || tbit + r.width > ps.n) {
        set_error("internal: circuit gate outside its block");
        return FQ_EINVAL;
      }
      g.push_back({tbit, r.width, r.mat});
    }
    fq_status st = upload(ps, g);
    if (st != FQ_OK) return st;
  }
  *out = prog;
  return FQ_OK;
}

// One pass over nvec vectors (at stride 2^L), in launches of at most 2^22
// (vector, tile) items (a dispatch holds fewer than 2^32 work-items).
fq_status run_pass(const BwProgram& prog, int which, const void* in, void* out, const void* psi, int flags,
                   zd rot, zd psi_coef, int nvec, hipStream_t s) {
  const BwProgram::Pass& ps = prog.pass[which];
  const size_t d = size_t(1) << prog.L;
  const size_t bytes = d * (prog.c64 ? sizeof(c64) : sizeof(c128));
  int tile_bits = 0;
  while ((1u << tile_bits) < ps.ntiles) ++tile_bits;
  const int per_launch = std::max(1, std::min(nvec, static_cast<int>((1u << 22) >> tile_bits)));
  BwPassArgs a{};
  a.mats = prog.mats;
  a.wins = ps.wins;
  a.gates = ps.gates;
  a.nwin = ps.nwin;
  a.n = ps.n;
  a.c = ps.c;
  a.p = ps.p;
  a.flags = flags;
  a.rot_re = rot.real();
  a.rot_im = rot.imag();
  a.psi_coef_re = psi_coef.real();
  a.psi_coef_im = psi_coef.imag();
  a.tile_bits = tile_bits;
  a.vstride = d;
  for (int v0 = 0; v0 < nvec; v0 += per_launch) {
    const int nv = std::min(per_launch, nvec - v0);
    const size_t off = size_t(v0) * bytes;
    a.xin = static_cast<const char*>(in) + off;
    a.xout = static_cast<char*>(out) + off;
    a.psi = psi ? static_cast<const char*>(psi) + off : nullptr;
    hipError_t e = bw_launch_pass(a, prog.c64, ps.wb, ps.ntiles * static_cast<unsigned>(nv), s);
    if (e != hipSuccess) {
      set_error(std::string("brickwork pass launch failed: ") + hipGetErrorString(e));
      return FQ_EDEVICE;
    }
  }
  return FQ_OK;
}

}  // namespace

fq_status bw_create(floquet_op* op) {
  // a circuit whose light cone fits complex64 tiles but not the smaller
  // complex128 ones keeps the complex64 program; the complex128 calls then
  // fail with FQ_EINVAL
  const fq_status s32 = build_program(op, true, &op->bw32);
  const std::string e32 = floquet_last_error();
  const fq_status s64 = build_program(op, false, &op->bw64);
  const std::string e64 = floquet_last_error();
  if (s32 != FQ_OK && s32 != FQ_EINVAL) {
    set_error(e32);
    return s32;
  }
  if (s64 != FQ_OK && s64 != FQ_EINVAL) {
    set_error(e64);
    return s64;
  }
  if (s32 != FQ_OK && s64 != FQ_OK) {
    set_error(e32);
    return FQ_EINVAL;
  }
  if (s32 != FQ_OK) op->bw_missing = "complex64: " + e32;
  if (s64 != FQ_OK) op->bw_missing = "complex128: " + e64;
  clear_error();
  return FQ_OK;
}

void bw_destroy(floquet_op* op) {
  op->bw32.reset();
  op->bw64.reset();
}

// the program of dtype, or nullptr (with the error set) if it could not be built
const BwProgram* program_for(const floquet_op* op, fq_dtype dt) {
  const BwProgram* p = dt == FQ_C64 ? op->bw32.get() : op->bw64.get();
  if (!p) set_error("this circuit has no " + op->bw_missing);
  return p;
}

fq_status bw_apply_U(floquet_op* op, fq_dtype dt, const void* psi, void* out, hipStream_t s) {
  const BwProgram* pp = program_for(op, dt);
  if (!pp) return FQ_EINVAL;
  const BwProgram& prog = *pp;
  const void* in = psi;
  for (int i = 0; i < prog.npass; ++i) {
    fq_status st = run_pass(prog, i, in, out, nullptr, 0, zd(1, 0), zd(1, 0), 1, s);
    if (st != FQ_OK) return st;
    in = out;
  }
  return FQ_OK;
}

// Horner: w = a_k psi; k times w <- a psi + rot * U w (rot = e^{-i phi} for
// the geometric sum, 1 for a general polynomial), for nvec vectors at stride
// 2^L, every pass one launch for all of them.
fq_status bw_filter(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi, void* out,
                    hipStream_t s, int nvec) {
  const BwProgram* pp = program_for(op, dt);
  if (!pp) return FQ_EINVAL;
  const BwProgram& prog = *pp;
  const zd rot = coefs ? zd(1, 0) : std::polar(1.0, -phi);
  const zd a_k = coefs ? coefs[k] : zd(1, 0);
  if (a_k != zd(1, 0)) {
    const size_t bytes = op->dim() * (dt == FQ_C64 ? sizeof(c64) : sizeof(c128));
    for (int v = 0; v < nvec; ++v) {
      fq_status st = poly_scale_copy(op, a_k, dt, static_cast<const char*>(psi) + size_t(v) * bytes,
                                     static_cast<char*>(out) + size_t(v) * bytes, s);
      if (st != FQ_OK) return st;
    }
  }
  for (int step = 1; step <= k; ++step) {
    const void* in = (step == 1 && a_k == zd(1, 0)) ? psi : out;
    const zd c = coefs ? coefs[k - step] : zd(1, 0);
    const int last_flags = BW_ROT | BW_ADD_PSI | (c != zd(1, 0) ? BW_PSI_COEF : 0);
    for (int i = 0; i < prog.npass; ++i) {
      const bool last = i == prog.npass - 1;
      fq_status st = run_pass(prog, i, i == 0 ? in : out, out, psi, last ? last_flags : 0, rot, c, nvec, s);
      if (st != FQ_OK) return st;
    }
  }
  return FQ_OK;
}

}  // namespace fq

extern "C" fq_status fq_host_bw_schedule(int n, int wb, int ngates, const int* q, const int* w, int line_bits,
                                         int* nwin_out, int* win_b, int* win_first, int* win_count,
                                         int* order) {
  using namespace fq;
  clear_error();
  const bool arrays = ngates == 0 || (q && w && win_b && win_first && win_count && order);
  if (n < 1 || n > 30 || wb < 1 || wb > 5 || wb > n || ngates < 0 || ngates > 32767 || line_bits < 0 ||
      !nwin_out || !arrays) {
    set_error("fq_host_bw_schedule: bad arguments");
    return FQ_EINVAL;
  }
  std::vector<PGate> g;
  for (int i = 0; i < ngates; ++i) {
    if ((w[i] != 1 && w[i] != 2) || q[i] < 0 || q[i] + w[i] > n || w[i] > wb) {
      set_error("fq_host_bw_schedule: gate " + std::to_string(i) + " outside the tile or wider than a window");
      return FQ_EINVAL;
    }
    g.push_back(PGate{q[i], w[i], i});
  }
  std::vector<BwWin> wins;
  std::vector<BwGate> gl;
  schedule_windows(g, n, wb, kBwWindowGates, line_bits, &wins, &gl);
  *nwin_out = static_cast<int>(wins.size());
  for (size_t j = 0; j < wins.size(); ++j) {
    win_b[j] = wins[j].b;
    win_first[j] = wins[j].first;
    win_count[j] = wins[j].count;
  }
  for (size_t k = 0; k < gl.size(); ++k) order[k] = gl[k].mat;
  return FQ_OK;
}
