// Kicked-Ising Floquet passes on gfx950:  U = D K,  K = prod_i exp(-i g X_i).
//
// The kick is applied in factored form.  exp(-i g X) = c (1 - i t X) with
// t = tan g when |tan g| <= 2 ("direct" form: (a, b) -> (a + i w b, b + i w a),
// w = -t, scale c per site), otherwise exp(-i g X) = (-i s)(X + i u) with
// u = cot g ("swapped" form: (a, b) -> (b + i w a, a + i w b), w = u, scale
// -i s per site).  Each output is two FMAs per real component; the product of
// the per-site scales is folded into the diagonal phase table, which is
// applied exactly once per U.
//
// The diagonal D = exp(-i E(s)) comes from two tables rounded once from FP64:
//   phase(s) = Tlo[s mod 2^m] * Thi[(s >> m) << 2 | b_0 << 1 | b_{m-1}],
// Thi also carrying the bonds that cross bit m-1|m and the periodic bond
// between bits 0 and L-1.
//
// Horner step of the geometric sum (Sec. 3, Eq. (geo)):  w <- psi + D K w
// (the target rotation e^{-i phi} is folded into the tables).  K = K_A K_B for
// the bits A, B held by two tile shapes; the factors commute and D is
// diagonal, so a pass over tiles of group S can finish one step and start the
// next:  K_S -> D -> +psi -> K_S.  Passes alternate between the groups; a
// prologue applies the other group's kick to psi and the last pass omits the
// trailing kick.  One pass = one Horner step = read w, read psi, write w.
//
// Kernel templates and launchers; ki_kernels_f32.hip / ki_kernels_f64.hip
// instantiate them per precision (two translation units build in parallel).
#pragma once

#include "tile_engine.h"
#include "ki_kernels.h"

namespace fq {

// One-qubit kicks on the register bits selected by mask.  In the direct form
// every register bit is processed, with weight 0 (an exact identity) where
// the mask is clear: straight-line code whose butterflies the compiler can
// interleave, instead of one branch per bit, whose joins made it copy the
// whole register array (measured: about as many moves as FMAs).
template <typename Real, int RB, bool SW>
__device__ __forceinline__ void kick_regs(cpx<Real> (&v)[1 << RB], unsigned mask, Real w) {
  if constexpr (!SW) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const Real wi = ((mask >> i) & 1u) ? w : Real(0);
#pragma unroll
      for (int m = 0; m < (1 << RB); ++m) {
        if (m & (1 << i)) continue;
        const int m2 = m | (1 << i);
        const cpx<Real> a = v[m], b = v[m2];
        v[m] = xpiwy(a, wi, b);
        v[m2] = xpiwy(b, wi, a);
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    if (mask & (1u << i)) {
#pragma unroll
      for (int m = 0; m < (1 << RB); ++m) {
        if (m & (1 << i)) continue;
        const int m2 = m | (1 << i);
        const cpx<Real> a = v[m], b = v[m2];
        if constexpr (SW) {
          v[m] = xpiwy(b, w, a);
          v[m2] = xpiwy(a, w, b);
        } else {
          v[m] = xpiwy(a, w, b);
          v[m2] = xpiwy(b, w, a);
        }
      }
    }
  }
}

// Value of lane (lane ^ 2^LB) without going through LDS: DPP row permutes
// for lane bits 0..3 (quad_perm xor 1, xor 2; half-row mirror then xor 3
// for xor 4; row rotate by 8 for xor 8) and the gfx950 permlane swaps for
// lane bits 4 and 5 (each output register holds the even / odd half of every
// lane pair; the lane picks its partner's).
__device__ __forceinline__ unsigned lane_xor_u32(unsigned u, int lb) {
  const int x = static_cast<int>(u);
  switch (lb) {
    // bound_ctrl set: every source lane of these patterns is valid, and the
    // "old" operand is then never read, so no register is zeroed for it
    case 0:
      return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, true));
    case 1:
      return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, true));
    case 2: {
      const int y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, true);
      return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, y, 0x1B, 0xF, 0xF, true));
    }
    case 3:
      return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, true));
    case 4: {
      const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
      return (threadIdx.x & 16u) ? r[0] : r[1];
    }
    default: {
      const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
      return (threadIdx.x & 32u) ? r[0] : r[1];
    }
  }
}

__device__ __forceinline__ float lane_xor(float v, int lb) { return __uint_as_float(lane_xor_u32(__float_as_uint(v), lb)); }
__device__ __forceinline__ double lane_xor(double v, int lb) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = lane_xor_u32(static_cast<unsigned>(b), lb);
  const unsigned hi = lane_xor_u32(static_cast<unsigned>(b >> 32), lb);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// mask: lane bits (0..5) to butterfly across the wavefront; in the direct
// form lane bits 0..NL-1 are processed with weight 0 where the mask is
// clear (see kick_regs), NL being the number of lane bits the layout can
// hold kicked bits in.
template <typename Real, int RB, bool SW, int NL = 6>
__device__ __forceinline__ void kick_lanes(cpx<Real> (&v)[1 << RB], unsigned mask, Real w) {
  if constexpr (!SW) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const Real wl = ((mask >> l) & 1u) ? w : Real(0);
#pragma unroll
      for (int m = 0; m < (1 << RB); ++m) {
        cpx<Real> p;
        p.x = lane_xor(v[m].x, l);
        p.y = lane_xor(v[m].y, l);
        v[m] = xpiwy(v[m], wl, p);
      }
    }
    return;
  }
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    if (mask & (1u << l)) {
#pragma unroll
      for (int m = 0; m < (1 << RB); ++m) {
        cpx<Real> p;
        p.x = lane_xor(v[m].x, l);
        p.y = lane_xor(v[m].y, l);
        if constexpr (SW)
          v[m] = xpiwy(p, w, v[m]);
        else
          v[m] = xpiwy(v[m], w, p);
      }
    }
  }
}

// lane bits that can carry kicked tile bits in layout A / layout B (see
// masks_for): layout A only for tiles without register bits, layout B the
// tile bits RB .. TB-1
template <int RB, int TB>
constexpr int lanes_a() {
  return RB == 0 ? (TB < 6 ? TB : 6) : 0;
}
template <int RB, int TB>
constexpr int lanes_b() {
  return RB == 0 ? 0 : (TB - RB < 6 ? TB - RB : 6);
}

template <typename Real>
__device__ __forceinline__ cpx<Real> ki_phase(const cpx<Real>* __restrict__ tlo,
                                              const cpx<Real>* __restrict__ thi, uint32_t g, int m) {
  const uint32_t lo = g & ((1u << m) - 1u);
  const uint32_t hi = ((g >> m) << 2) | ((g & 1u) << 1) | ((g >> (m - 1)) & 1u);
  return cmul(gload(tlo, lo), gload(thi, hi));
}

// ---------------------------------------------------------------------------
// One pass over all tiles of one group (see ki_kernels.h for the fields).
// ---------------------------------------------------------------------------
// BATCH: 0 one problem, 1 batched, 2 batched with the folded form
// (KiPassArgs::chi; a kernel of its own, as its extra registers would lower
// the occupancy of the plain form)
template <typename Real, int RB, int TB, bool SW, bool PF, int BATCH>
__global__ void __launch_bounds__(1 << TB) ki_pass_kernel(KiPassArgs<Real> a) {
  using C = cpx<Real>;
  constexpr int R = 1 << RB;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x;
  uint32_t tile;
  const C* __restrict__ xin;
  C* __restrict__ xout;
  const C* __restrict__ psi;
  const C* __restrict__ tlo;
  const C* __restrict__ thi;
  Real w;
  if constexpr (BATCH != 0) {
    uint32_t q;
    if (a.flat) {
      const uint32_t idx = xcd_tile(blockIdx.x, gridDim.x);
      q = idx >> a.tile_log;
      tile = idx & ((1u << a.tile_log) - 1u);
    } else {
      q = blockIdx.y;
      tile = xcd_tile(blockIdx.x, gridDim.x);
    }
    const KiDesc<Real>& D = a.desc[a.list[q]];
    xin = a.from_psi ? D.psi : D.x;
    xout = D.x;
    psi = (BATCH == 2 && a.chi > 0) ? D.chi[a.chi - 1] : D.psi;
    tlo = D.tlo;
    thi = D.thi;
    w = static_cast<Real>(D.w);
  } else {
    tile = xcd_tile(blockIdx.x, gridDim.x);
    xin = a.xin;
    xout = a.xout;
    psi = a.psi;
    tlo = a.tlo;
    thi = a.thi;
    w = static_cast<Real>(a.w);
  }
  const TileMap tm = make_tile_map(tile, a.n, a.c, a.p);
  const bool do_ph = (a.flags & KI_PHASE) != 0;
  const bool do_ps = (a.flags & KI_ADD_PSI) != 0;
  // folded form (KiPassArgs::chi): the phase is applied in layout B
  bool fold = false, fold_b = false;
  if constexpr (BATCH == 2) {
    fold = a.chi > 0;
    fold_b = fold && ((a.k1.regB | a.k1.laneB | a.k2.regB | a.k2.laneB) != 0u);
  }

  // The tile and psi are read in layout A (consecutive lanes <-> consecutive
  // addresses) at the start; the phase and +psi are applied in layout A too,
  // so every global access of the pass is coalesced.
  C v[R], ps[R], tl[PF ? R : 1], th[PF ? R : 1];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = gload(xin, tm.g(tid + (m << TB)));
  if (do_ps) {
#pragma unroll
    for (int m = 0; m < R; ++m) ps[m] = gload(psi, tm.g(tid + (m << TB)));
  }
  // with few tiles per CU (small states) the pass is latency-bound: fetch the
  // phase-table entries together with the tile instead of mid-pass
  constexpr bool pre_ph = PF;
  if constexpr (PF) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const uint32_t g = tm.g(fold_b ? (tid << RB) + m : tid + (m << TB));
      tl[m] = gload(tlo, g & ((1u << a.m) - 1u));
      th[m] = gload(thi, ((g >> a.m) << 2) | ((g & 1u) << 1) | ((g >> (a.m - 1)) & 1u));
    }
  }
  if (a.flags & KI_SCALE_IN) {
    const C s = mk<Real>(static_cast<Real>(a.in_coef_re), static_cast<Real>(a.in_coef_im));
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cmul(v[m], s);
  }

  if (fold) {
    // K D K x + chi: the A part of the first kick, then in layout B its B
    // part, the phase and the B part of the second kick, back in A the A
    // part of the second kick and chi (read in layout A)
    kick_regs<Real, RB, SW>(v, a.k1.regA, w);
    kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k1.laneA, w);
    if (fold_b) a_to_b<Real, RB, TB>(v, lds, tid);
    kick_regs<Real, RB, SW>(v, a.k1.regB, w);
    kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k1.laneB, w);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int t = fold_b ? (tid << RB) + m : tid + (m << TB);
      if constexpr (pre_ph)
        v[m] = cmul(v[m], cmul(tl[m], th[m]));
      else
        v[m] = cmul(v[m], ki_phase(tlo, thi, tm.g(t), a.m));
    }
    kick_regs<Real, RB, SW>(v, a.k2.regB, w);
    kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k2.laneB, w);
    if (fold_b) b_to_a<Real, RB, TB>(v, lds, tid);
    kick_regs<Real, RB, SW>(v, a.k2.regA, w);
    kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k2.laneA, w);
    const C pc = mk<Real>(static_cast<Real>(a.psi_coef_re), static_cast<Real>(a.psi_coef_im));
    const bool coef = (a.flags & KI_PSI_COEF) != 0;
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = coef ? cfma(ps[m], pc, v[m]) : cadd(v[m], ps[m]);
#pragma unroll
    for (int m = 0; m < R; ++m) gstore(xout, tm.g(tid + (m << TB)), v[m]);
    return;
  }

  // first kick of this group: layout A, then layout B, back to A.  A thread
  // rewrites only LDS slots it read itself (B slots in b_to_a, A slots in
  // the next a_to_b), so the barrier inside each layout change suffices.
  kick_regs<Real, RB, SW>(v, a.k1.regA, w);
  kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k1.laneA, w);
  if (a.k1.regB | a.k1.laneB) {
    a_to_b<Real, RB, TB>(v, lds, tid);
    kick_regs<Real, RB, SW>(v, a.k1.regB, w);
    kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k1.laneB, w);
    b_to_a<Real, RB, TB>(v, lds, tid);
  }

  if (do_ph || do_ps) {
    const C pc = mk<Real>(static_cast<Real>(a.psi_coef_re), static_cast<Real>(a.psi_coef_im));
    const bool coef = (a.flags & KI_PSI_COEF) != 0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      C x = v[m];
      if constexpr (pre_ph) {
        if (do_ph) x = cmul(x, cmul(tl[m], th[m]));
      } else {
        if (do_ph) x = cmul(x, ki_phase(tlo, thi, tm.g(tid + (m << TB)), a.m));
      }
      if (do_ps) x = coef ? cfma(ps[m], pc, x) : cadd(x, ps[m]);
      v[m] = x;
    }
  }

  // second kick (starts the next Horner step): layout A, then B, back to A
  if (a.k2.regA | a.k2.laneA | a.k2.regB | a.k2.laneB) {
    kick_regs<Real, RB, SW>(v, a.k2.regA, w);
    kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k2.laneA, w);
    if (a.k2.regB | a.k2.laneB) {
      a_to_b<Real, RB, TB>(v, lds, tid);
      kick_regs<Real, RB, SW>(v, a.k2.regB, w);
      kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k2.laneB, w);
      b_to_a<Real, RB, TB>(v, lds, tid);
    }
  }

#pragma unroll
  for (int m = 0; m < R; ++m) gstore(xout, tm.g(tid + (m << TB)), v[m]);
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined form of a batched pass.  The grid (a
// multiple of 8 workgroups) walks the nitems = nprob * 2^tile_log (problem,
// tile) items, problem-major; workgroup g runs on XCD g mod 8 and takes
// every (grid/8)-th item of that XCD's contiguous eighth of the items, so
// neighbouring tiles share one L2.  Per item the loads of psi and of the
// phase-table entries of the current tile are issued first and the next
// tile's state after them: the in-order memory counter then lets the next
// tile's loads stay in flight through the kicks, the phase and the store of
// the current one.  Arithmetic and layout changes are those of
// ki_pass_kernel.
// ---------------------------------------------------------------------------
template <typename Real>
struct KiPipeItem {
  const cpx<Real>* xin;
  cpx<Real>* xout;
  const cpx<Real>* psi;
  const cpx<Real>* tlo;
  const cpx<Real>* thi;
  Real w;
  TileMap tm;
};

// desc / list arrive as restrict kernel parameters: read-only for the
// kernel, so the compiler loads them through the scalar cache (lgkmcnt), not
// with vector loads that would have to wait behind the prefetch (vmcnt).
template <typename Real>
__device__ __forceinline__ KiPipeItem<Real> ki_pipe_item(const KiPassArgs<Real>& a, const KiDesc<Real>* __restrict__ desc,
                                                         const int* __restrict__ list, uint32_t item) {
  const uint32_t q = item >> a.tile_log;
  const uint32_t tile = item & ((1u << a.tile_log) - 1u);
  const KiDesc<Real>& D = desc[list[q]];
  KiPipeItem<Real> r;
  r.xin = a.from_psi ? D.psi : D.x;
  r.xout = D.x;
  r.psi = D.psi;
  r.tlo = D.tlo;
  r.thi = D.thi;
  r.w = static_cast<Real>(D.w);
  r.tm = make_tile_map(tile, a.n, a.c, a.p);
  return r;
}

// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt and
// lgkmcnt left at their maxima)
template <int N>
constexpr int vmcnt_imm() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  return 0x0F70 | (N & 15) | ((N >> 4) << 14);
}

template <typename Real, int RB, int TB, bool SW>
__global__ void __launch_bounds__(1 << TB)
    ki_pipe_kernel(KiPassArgs<Real> a, uint32_t nitems, const KiDesc<Real>* __restrict__ desc,
                   const int* __restrict__ list) {
  using C = cpx<Real>;
  constexpr int R = 1 << RB;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x;
  const uint32_t per_xcd = nitems >> 3;
  const uint32_t stride = gridDim.x >> 3;
  const uint32_t first = (blockIdx.x & 7u) * per_xcd;
  uint32_t local = blockIdx.x >> 3;
  if (local >= per_xcd) return;
  const bool do_ph = (a.flags & KI_PHASE) != 0;
  const bool do_ps = (a.flags & KI_ADD_PSI) != 0;
  const uint32_t mlo = (1u << a.m) - 1u;

  KiPipeItem<Real> cur = ki_pipe_item(a, desc, list, first + local);
  C v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = gload(cur.xin, cur.tm.g(tid + (m << TB)));
  for (;;) {
    // this tile's state (the previous iteration's prefetch) has arrived once
    // at most the R stores issued after it are outstanding
    __builtin_amdgcn_s_waitcnt(vmcnt_imm<R>());
    // this tile's psi and phase entries, then the next tile's state.  The
    // loads are issued whatever the flags and also for the last item (which
    // re-reads its own tile): with one load sequence on every path the
    // compiler's wait counts stay exact and never drain the prefetch.
    C ps[R], tl[R], th[R];
#pragma unroll
    for (int m = 0; m < R; ++m) ps[m] = gload(cur.psi, cur.tm.g(tid + (m << TB)));
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const uint32_t g = cur.tm.g(tid + (m << TB));
      tl[m] = gload(cur.tlo, g & mlo);
      th[m] = gload(cur.thi, ((g >> a.m) << 2) | ((g & 1u) << 1) | ((g >> (a.m - 1)) & 1u));
    }
    const uint32_t here = first + local;
    local += stride;
    const bool more = local < per_xcd;
    const KiPipeItem<Real> nxt = ki_pipe_item(a, desc, list, more ? first + local : here);
    C vn[R];
#pragma unroll
    for (int m = 0; m < R; ++m) vn[m] = gload(nxt.xin, nxt.tm.g(tid + (m << TB)));
    // keep the prefetch ahead of the work below (no sinking towards its use)
    asm volatile("" ::: "memory");

    const Real w = cur.w;
    kick_regs<Real, RB, SW>(v, a.k1.regA, w);
    kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k1.laneA, w);
    if (a.k1.regB | a.k1.laneB) {  // as in ki_pass_kernel: no barrier between layout changes
      a_to_b<Real, RB, TB>(v, lds, tid);
      kick_regs<Real, RB, SW>(v, a.k1.regB, w);
      kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k1.laneB, w);
      b_to_a<Real, RB, TB>(v, lds, tid);
    }
    if (do_ph || do_ps) {
#pragma unroll
      for (int m = 0; m < R; ++m) {
        C x = v[m];
        if (do_ph) x = cmul(x, cmul(tl[m], th[m]));
        if (do_ps) x = cadd(x, ps[m]);
        v[m] = x;
      }
    }
    if (a.k2.regA | a.k2.laneA | a.k2.regB | a.k2.laneB) {
      kick_regs<Real, RB, SW>(v, a.k2.regA, w);
      kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.k2.laneA, w);
      if (a.k2.regB | a.k2.laneB) {
        a_to_b<Real, RB, TB>(v, lds, tid);
        kick_regs<Real, RB, SW>(v, a.k2.regB, w);
        kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.k2.laneB, w);
        b_to_a<Real, RB, TB>(v, lds, tid);
      }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) gstore(cur.xout, cur.tm.g(tid + (m << TB)), v[m]);
    if (!more) break;
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = vn[m];
    cur = nxt;
    // the next tile's layout changes write only LDS slots this thread read
    // last (its layout-A slots): no barrier needed here either
  }
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup (n = L, or n = 6 with idle lanes for L < 6):
// all k Horner steps in one launch.  psi stays in registers (layout B) when
// it fits (PSI_REGS, which also keeps the phases), otherwise both are re-read
// each step (L1/L2-resident).
// coefs (device, k entries, may be NULL): coefficient of psi in step s, used
// for general polynomials; NULL means 1.
// ---------------------------------------------------------------------------
template <typename Real, int RB, int TB, bool SW, bool PSI_REGS, bool BATCH>
__global__ void __launch_bounds__(1 << TB) ki_single_kernel(KiSingleArgs<Real> a) {
  using C = cpx<Real>;
  constexpr int R = 1 << RB;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x;
  const uint32_t dim = 1u << a.L;
  const C* __restrict__ psi;
  const C* __restrict__ xin;
  C* __restrict__ xout;
  const C* __restrict__ tlo;
  const C* __restrict__ thi;
  Real w;
  if constexpr (BATCH) {
    // one workgroup per problem of the list
    const KiDesc<Real>& D = a.desc[a.list[blockIdx.x]];
    psi = D.psi;
    xin = a.from_psi ? D.psi : D.x;
    xout = D.x;
    tlo = D.tlo;
    thi = D.thi;
    w = static_cast<Real>(D.w);
  } else {
    // problems at a fixed stride (one workgroup each)
    const size_t off = static_cast<size_t>(blockIdx.x) * a.batch_stride;
    psi = a.psi + off;
    xin = a.xin + off;
    xout = a.xout + off;
    tlo = a.tlo;
    thi = a.thi;
    w = static_cast<Real>(a.w);
  }

  // layout B: tid*R + m
  C v[R];
  C ps[PSI_REGS ? R : 1];
  C ph[PSI_REGS ? R : 1];
  const bool active = static_cast<uint32_t>(tid << RB) < dim;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const uint32_t g = (tid << RB) + m;
    v[m] = active ? xin[g] : mk<Real>(0, 0);
    if constexpr (PSI_REGS) {
      ps[m] = active ? psi[g] : mk<Real>(0, 0);
      ph[m] = active ? ki_phase(tlo, thi, g, a.m) : mk<Real>(0, 0);
    }
  }
  if (a.flags & KI_SCALE_IN) {
    const C s = mk<Real>(static_cast<Real>(a.in_coef_re), static_cast<Real>(a.in_coef_im));
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cmul(v[m], s);
  }

  for (int step = 0; step < a.steps; ++step) {
    kick_regs<Real, RB, SW>(v, a.kick.regB, w);
    kick_lanes<Real, RB, SW, lanes_b<RB, TB>()>(v, a.kick.laneB, w);
    if constexpr (RB > 0) {
      b_to_a<Real, RB, TB>(v, lds, tid);
      kick_regs<Real, RB, SW>(v, a.kick.regA, w);
      kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.kick.laneA, w);
      __syncthreads();
      a_to_b<Real, RB, TB>(v, lds, tid);
      __syncthreads();
    } else {
      kick_lanes<Real, RB, SW, lanes_a<RB, TB>()>(v, a.kick.laneA, w);
    }
    C coef = mk<Real>(1, 0);
    const bool use_coef = a.coefs != nullptr;
    if (use_coef) {
      const double2 cc = a.coefs[step];
      coef = mk<Real>(static_cast<Real>(cc.x), static_cast<Real>(cc.y));
    }
#pragma unroll
    for (int m = 0; m < R; ++m) {
      C x;
      if constexpr (PSI_REGS)
        x = cmul(v[m], ph[m]);
      else
        x = active ? cmul(v[m], ki_phase(tlo, thi, (tid << RB) + m, a.m)) : v[m];
      if (a.flags & KI_ADD_PSI) {
        C p;
        if constexpr (PSI_REGS)
          p = ps[m];
        else
          p = active ? psi[(tid << RB) + m] : mk<Real>(0, 0);
        x = use_coef ? cfma(p, coef, x) : cadd(x, p);
      }
      v[m] = x;
    }
  }
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) xout[(tid << RB) + m] = v[m];
  }
}

// ---------------------------------------------------------------------------
// Horner pass in three register layouts (direct kick form).  A workgroup of
// T = 2^TB threads holds a tile of n = 4 + TB bits, 16 amplitudes per
// thread, in one of
//   A: j = t + T m                                   registers: bits TB .. n-1
//   B: j = 16 t + m                                  registers: bits 0..3,
//                                                    lanes 0..S-5: bits 4..S-1
//   C: j = (t mod 2^S) + 2^S m + 2^(S+4) (t >> S)    registers: bits S .. S+3
// with S = 4 for TB <= 8, 5 for TB = 9 (bit 4 takes a DPP xor 1 in B) and 6
// for TB = 10 (bits 4 and 5: DPP xor 1 and xor 2 in B; complex64 only, the
// tile fills 136 KiB of LDS).  Every other kicked bit is a register bit of
// one layout: two FMAs per amplitude and bit, where the two-layout pass moves
// five of thirteen bits across lanes.  Per pass: kick A, A->B, kick B, B->C,
// kick C, phase and +psi in C (psi read in C order: 2^S consecutive tile
// indices per group of lanes), kick C, C->B, kick B, B->A, kick A, store --
// four layout changes, as in the two-layout pass.  The phase-table entries
// are requested first and multiplied together while the tile is in flight.
// Flags: KI_PHASE always; KI_ADD_PSI optional (with KI_PSI_COEF: + c psi);
// no second kick and no psi for the last pass of a U application.
// ---------------------------------------------------------------------------
template <int TB>
constexpr int pass3_shift() {
  return TB == 10 ? 6 : (TB == 9 ? 5 : 4);
}

// Tile index of register 0 of thread t in layout L (0 = A, 1 = B, 2 = C);
// register m sits pass3_step<TB, L>() tile indices further on.
template <int TB, int L>
__device__ __forceinline__ uint32_t pass3_index0(uint32_t t) {
  constexpr int S = pass3_shift<TB>();
  if constexpr (L == 0)
    return t;
  else if constexpr (L == 1)
    return t << 4;
  else
    return (t & ((1u << S) - 1u)) + ((t >> S) << (S + 4));
}
template <int TB, int L>
constexpr uint32_t pass3_step() {
  return L == 0 ? (1u << TB) : (L == 1 ? 1u : (1u << pass3_shift<TB>()));
}
// LDS slot distance between consecutive registers (padding of lds_phys<4>:
// steps of at least 16 tile indices gain one pad slot per 16)
template <int TB, int L>
constexpr uint32_t pass3_lds_step() {
  return pass3_step<TB, L>() >= 16 ? pass3_step<TB, L>() + pass3_step<TB, L>() / 16 : pass3_step<TB, L>();
}

// Layout FROM -> TO through LDS.  A thread writes only the slots it read in
// the previous change (its FROM slots), so one barrier per change suffices.
template <typename Real, int TB, int FROM, int TO>
__device__ __forceinline__ void relayout3(cpx<Real> (&v)[16], cpx<Real>* lds, uint32_t tid) {
  cpx<Real>* w = lds + lds_phys<4>(pass3_index0<TB, FROM>(tid));
  const cpx<Real>* r = lds + lds_phys<4>(pass3_index0<TB, TO>(tid));
#pragma unroll
  for (int m = 0; m < 16; ++m) w[m * pass3_lds_step<TB, FROM>()] = v[m];
  lds_barrier();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = r[m * pass3_lds_step<TB, TO>()];
}

// Amplitude access with a uniform base and a 32-bit element offset (the
// launcher admits states of at most 2^32 bytes): one offset register per
// access instead of a 64-bit address.
template <typename Real>
__device__ __forceinline__ cpx<Real> gload32(const cpx<Real>* p, uint32_t i) {
  using V = typename gvec2<Real>::type;
  typedef const __attribute__((address_space(1))) char* GB;
  typedef const __attribute__((address_space(1))) V* GP;
  const V x = *(GP)((GB)p + i * uint32_t(sizeof(V)));  // C-style: address-space cast
  return mk<Real>(x.x, x.y);
}
template <typename Real>
__device__ __forceinline__ void gstore32(cpx<Real>* p, uint32_t i, cpx<Real> c) {
  using V = typename gvec2<Real>::type;
  typedef __attribute__((address_space(1))) char* GB;
  typedef __attribute__((address_space(1))) V* GP;
  V x;
  x.x = c.x;
  x.y = c.y;
  *(GP)((GB)p + i * uint32_t(sizeof(V))) = x;
}

template <typename Real, int TB, int BATCH>
__global__ void __launch_bounds__(1 << TB) ki_pass3_kernel(KiPassArgs<Real> a) {
  using C = cpx<Real>;
  constexpr int R = 16;
  constexpr int S = pass3_shift<TB>();
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const uint32_t tid = threadIdx.x;
  uint32_t tile;
  const C* __restrict__ xin;
  C* __restrict__ xout;
  const C* __restrict__ psi;
  const C* __restrict__ tlo;
  const C* __restrict__ thi;
  Real w;
  if constexpr (BATCH != 0) {
    uint32_t q;
    if (a.flat) {
      const uint32_t idx = xcd_tile(blockIdx.x, gridDim.x);
      q = idx >> a.tile_log;
      tile = idx & ((1u << a.tile_log) - 1u);
    } else {
      q = blockIdx.y;
      tile = xcd_tile(blockIdx.x, gridDim.x);
    }
    const KiDesc<Real>& D = a.desc[a.list[q]];
    xin = a.from_psi ? D.psi : D.x;
    xout = D.x;
    psi = D.psi;
    tlo = D.tlo;
    thi = D.thi;
    w = static_cast<Real>(D.w);
  } else {
    tile = xcd_tile(blockIdx.x, gridDim.x);
    xin = a.xin;
    xout = a.xout;
    psi = a.psi;
    tlo = a.tlo;
    thi = a.thi;
    w = static_cast<Real>(a.w);
  }
  const TileMap tm = make_tile_map(tile, a.n, a.c, a.p);
  const uint32_t mlo = (1u << a.m) - 1u;
  // global index of register m of layouts A and C: g(index0) + m * stride
  // (the register step is a power of two; below the chunk it stays in the
  // chunk, above it moves the high part only)
  const uint32_t cw = 1u << a.c;
  const uint32_t stA = pass3_step<TB, 0>() < cw ? pass3_step<TB, 0>() : (pass3_step<TB, 0>() >> a.c) << a.p;
  const uint32_t stC = pass3_step<TB, 2>() < cw ? pass3_step<TB, 2>() : (pass3_step<TB, 2>() >> a.c) << a.p;
  const uint32_t gA = tm.g(pass3_index0<TB, 0>(tid));
  const uint32_t gC = tm.g(pass3_index0<TB, 2>(tid));

  // the tile in layout A, then the phase-table entries of the layout-C
  // amplitudes (multiplied together once the first kick is done).  Layout C's
  // register bits lie all below the table split (t3 = 0: the low-table index
  // steps with the register, the high-table entry is the thread's) or all
  // above it (t3 = 1: the other way round); no register bit is a boundary
  // bit of the split, and register 0's index has them clear, so the varying
  // index is base + m * step.
  C tv[R], v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = gload32(xin, gA + uint32_t(m) * stA);
  const uint32_t ilo = gC & mlo;
  const uint32_t ihi = ((gC >> a.m) << 2) | ((gC & 1u) << 1) | ((gC >> (a.m - 1)) & 1u);
  const C* __restrict__ tvar = a.t3 ? thi : tlo;
  const uint32_t ivar = a.t3 ? ihi : ilo;
  const uint32_t svar = a.t3 ? (stC >> a.m) << 2 : stC;
#pragma unroll
  for (int m = 0; m < R; ++m) tv[m] = gload32(tvar, ivar + uint32_t(m) * svar);
  const C tc = a.t3 ? gload32(tlo, ilo) : gload32(thi, ihi);

  // first kick (finishes the Horner step begun by the previous pass)
  kick_regs<Real, 4, false>(v, a.k1.regA, w);
  C ph[R];
#pragma unroll
  for (int m = 0; m < R; ++m) ph[m] = cmul(tv[m], tc);
  relayout3<Real, TB, 0, 1>(v, lds, tid);
  // without psi, the input stands in for it with coefficient 0 (finite
  // values, so the product vanishes)
  const bool add_psi = (a.flags & KI_ADD_PSI) != 0;
  const bool coef = !add_psi || (a.flags & KI_PSI_COEF) != 0;
  const C pc = add_psi ? mk<Real>(static_cast<Real>(a.psi_coef_re), static_cast<Real>(a.psi_coef_im))
                       : mk<Real>(Real(0), Real(0));
  const C* __restrict__ pin = add_psi ? psi : xin;
  C ps[R];
#pragma unroll
  for (int m = 0; m < R; ++m) ps[m] = gload32(pin, gC + uint32_t(m) * stC);
  kick_regs<Real, 4, false>(v, a.k1.regB, w);
  if constexpr (S > 4) kick_lanes<Real, 4, false, S - 4>(v, a.k1.laneB, w);
  relayout3<Real, TB, 1, 2>(v, lds, tid);
  kick_regs<Real, 4, false>(v, a.k1c, w);
  if (coef) {
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cfma(ps[m], pc, cmul(v[m], ph[m]));
  } else {
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cadd(cmul(v[m], ph[m]), ps[m]);
  }

  // second kick (starts the next step), or straight back to layout A
  if (a.k2.regA | a.k2.regB | a.k2.laneB | a.k2c) {
    kick_regs<Real, 4, false>(v, a.k2c, w);
    relayout3<Real, TB, 2, 1>(v, lds, tid);
    kick_regs<Real, 4, false>(v, a.k2.regB, w);
    if constexpr (S > 4) kick_lanes<Real, 4, false, S - 4>(v, a.k2.laneB, w);
    relayout3<Real, TB, 1, 0>(v, lds, tid);
    kick_regs<Real, 4, false>(v, a.k2.regA, w);
  } else {
    relayout3<Real, TB, 2, 0>(v, lds, tid);
  }
  // the store offsets are recomputed from an opaque copy of the tile base:
  // otherwise the compiler keeps the sixteen load offsets live (as 64-bit
  // addresses) across the whole pass
  uint32_t gS = gA;
  asm volatile("" : "+v"(gS));
#pragma unroll
  for (int m = 0; m < R; ++m) gstore32(xout, gS + uint32_t(m) * stA, v[m]);
}

// ---------------------------------------------------------------------------
// Host launchers: runtime (RB, TB, SW) -> template instance.
// ---------------------------------------------------------------------------
namespace {

template <typename Real, int RB, int TB, bool SW, bool PF, int BATCH>
hipError_t launch_pass_t(const KiPassArgs<Real>& a, unsigned ntiles, unsigned nprob, hipStream_t s) {
  const size_t shmem = static_cast<size_t>(lds_slots<RB, TB>()) * sizeof(cpx<Real>);
  auto kern = ki_pass_kernel<Real, RB, TB, SW, PF, BATCH>;
  static bool attr_set = false;
  if (!attr_set && shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const dim3 grid = BATCH == 0 ? dim3(ntiles) : (a.flat ? dim3(ntiles * nprob) : dim3(ntiles, nprob));
  hipLaunchKernelGGL(kern, grid, dim3(1 << TB), shmem, s, a);
  return hipGetLastError();
}

template <typename Real, int TB, int BATCH>
hipError_t launch_pass3_t(const KiPassArgs<Real>& a, unsigned ntiles, unsigned nprob, hipStream_t s) {
  const size_t shmem = static_cast<size_t>(lds_slots<4, TB>()) * sizeof(cpx<Real>);
  auto kern = ki_pass3_kernel<Real, TB, BATCH>;
  static bool attr_set = false;
  if (!attr_set && shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const dim3 grid = BATCH == 0 ? dim3(ntiles) : (a.flat ? dim3(ntiles * nprob) : dim3(ntiles, nprob));
  hipLaunchKernelGGL(kern, grid, dim3(1 << TB), shmem, s, a);
  return hipGetLastError();
}

template <typename Real, int RB, int TB, bool SW>
hipError_t launch_pipe_t(const KiPassArgs<Real>& a, uint32_t nitems, unsigned grid, hipStream_t s) {
  const size_t shmem = static_cast<size_t>(lds_slots<RB, TB>()) * sizeof(cpx<Real>);
  auto kern = ki_pipe_kernel<Real, RB, TB, SW>;
  static bool attr_set = false;
  if (!attr_set && shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(1 << TB), shmem, s, a, nitems, a.desc, a.list);
  return hipGetLastError();
}

template <typename Real, int RB, int TB, bool SW, bool PSI_REGS, bool BATCH>
hipError_t launch_single_tt(const KiSingleArgs<Real>& a, unsigned nblocks, hipStream_t s) {
  const size_t shmem = static_cast<size_t>(lds_slots<RB, TB>()) * sizeof(cpx<Real>);
  auto kern = ki_single_kernel<Real, RB, TB, SW, PSI_REGS, BATCH>;
  static bool attr_set = false;
  if (!attr_set && shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(1 << TB), shmem, s, a);
  return hipGetLastError();
}

template <typename Real, int RB, int TB, bool SW>
hipError_t launch_single_t(const KiSingleArgs<Real>& a, unsigned nblocks, bool psi_regs, bool batched,
                           hipStream_t s) {
  if (batched)
    return psi_regs ? launch_single_tt<Real, RB, TB, SW, true, true>(a, nblocks, s)
                    : launch_single_tt<Real, RB, TB, SW, false, true>(a, nblocks, s);
  return psi_regs ? launch_single_tt<Real, RB, TB, SW, true, false>(a, nblocks, s)
                  : launch_single_tt<Real, RB, TB, SW, false, false>(a, nblocks, s);
}

}  // namespace

#define FQ_SHAPES(X) X(0, 6) X(1, 6) X(2, 6) X(3, 6) X(4, 6) X(4, 7) X(4, 8) X(4, 9) X(1, 7) X(2, 7) X(2, 8) X(3, 8) X(3, 7) X(3, 9)

template <typename Real>
hipError_t ki_launch_pass(const KiPassArgs<Real>& a, int rb, int tb, bool sw, unsigned ntiles, hipStream_t s,
                          unsigned nprob) {
  const bool pf = (a.flags & KI_PREFETCH_PHASE) != 0;
  if (nprob > 0 && (!a.desc || !a.list || nprob > 65535u)) return hipErrorInvalidValue;
  // the folded form exists for complex128 batched passes only
  if (a.chi > 0 && (nprob == 0 || sizeof(Real) != 8)) return hipErrorInvalidValue;
  if (nprob > 0 && a.flat && (ntiles != (1u << a.tile_log) || size_t(ntiles) * nprob > 0x7fffffffu))
    return hipErrorInvalidValue;
#define FQ_CASE4(RB_, TB_, PF_)                                                                    \
  if (nprob > 0) {                                                                                 \
    if constexpr (sizeof(Real) == 8) {                                                             \
      if (a.chi > 0)                                                                               \
        return sw ? launch_pass_t<Real, RB_, TB_, true, PF_, 2>(a, ntiles, nprob, s)               \
                  : launch_pass_t<Real, RB_, TB_, false, PF_, 2>(a, ntiles, nprob, s);             \
    }                                                                                              \
    return sw ? launch_pass_t<Real, RB_, TB_, true, PF_, 1>(a, ntiles, nprob, s)                   \
              : launch_pass_t<Real, RB_, TB_, false, PF_, 1>(a, ntiles, nprob, s);                 \
  }                                                                                                \
  return sw ? launch_pass_t<Real, RB_, TB_, true, PF_, 0>(a, ntiles, 1, s)                         \
            : launch_pass_t<Real, RB_, TB_, false, PF_, 0>(a, ntiles, 1, s);
#define FQ_CASE(RB_, TB_)                                                                          \
  if (rb == RB_ && tb == TB_) {                                                                    \
    if (pf) {                                                                                      \
      FQ_CASE4(RB_, TB_, true)                                                                     \
    }                                                                                              \
    FQ_CASE4(RB_, TB_, false)                                                                      \
  }
  FQ_SHAPES(FQ_CASE)
#undef FQ_CASE
#undef FQ_CASE4
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t ki_launch_pass3(const KiPassArgs<Real>& a, int tb, unsigned ntiles, hipStream_t s, unsigned nprob) {
  {
    // 32-bit byte offsets: at most 2^32 / sizeof(amplitude) amplitudes
    // (register steps stay linear in the tile map: the chunk is the whole
    // tile or at most 16 amplitudes)
    if (a.n != 4 + tb || a.chi != 0 || (size_t(ntiles) << a.n) > ((size_t(1) << 32) / sizeof(cpx<Real>)) ||
        (a.c != a.n && a.c > 4))
      return hipErrorInvalidValue;
    if (nprob > 0 && (!a.desc || !a.list || nprob > 65535u)) return hipErrorInvalidValue;
    if (nprob > 0 && a.flat && (ntiles != (1u << a.tile_log) || size_t(ntiles) * nprob > 0x7fffffffu))
      return hipErrorInvalidValue;
#define FQ_CASE(TB_)                                                            \
  if (tb == TB_)                                                                \
    return nprob > 0 ? launch_pass3_t<Real, TB_, 1>(a, ntiles, nprob, s)        \
                     : launch_pass3_t<Real, TB_, 0>(a, ntiles, 1, s);
    FQ_CASE(6)
    FQ_CASE(7)
    FQ_CASE(8)
    FQ_CASE(9)
    if constexpr (sizeof(Real) == 4) {
      FQ_CASE(10)
    }
#undef FQ_CASE
    return hipErrorInvalidValue;
  }
}

// complex128 with 16 amplitudes per thread would spill (prefetched state,
// psi and two phase factors live at once): no pipelined instance
template <typename Real, int RB, int TB>
hipError_t launch_pipe_sw(const KiPassArgs<Real>& a, bool sw, uint32_t nitems, unsigned grid, hipStream_t s) {
  if constexpr (sizeof(Real) == 8 && RB > 3) {
    return hipErrorInvalidValue;
  } else {
    return sw ? launch_pipe_t<Real, RB, TB, true>(a, nitems, grid, s)
              : launch_pipe_t<Real, RB, TB, false>(a, nitems, grid, s);
  }
}

// multi-pass tile shapes with a pipelined instance
#define FQ_PIPE_SHAPES(X) X(2, 8) X(3, 7) X(3, 8) X(3, 9) X(4, 6) X(4, 7) X(4, 8) X(4, 9)

template <typename Real>
hipError_t ki_launch_pipe(const KiPassArgs<Real>& a, int rb, int tb, bool sw, unsigned ntiles, unsigned nprob,
                          unsigned grid, hipStream_t s) {
  if (!a.desc || !a.list || nprob == 0 || nprob > 65535u || ntiles != (1u << a.tile_log) || (ntiles & 7u) != 0u)
    return hipErrorInvalidValue;
  const size_t nitems = size_t(ntiles) * nprob;
  if (nitems > 0x7fffffffu || grid == 0 || (grid & 7u) != 0u || grid > nitems) return hipErrorInvalidValue;
#define FQ_CASE(RB_, TB_) \
  if (rb == RB_ && tb == TB_) return launch_pipe_sw<Real, RB_, TB_>(a, sw, static_cast<uint32_t>(nitems), grid, s);
  FQ_PIPE_SHAPES(FQ_CASE)
#undef FQ_CASE
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t ki_launch_single(const KiSingleArgs<Real>& a, int rb, int tb, bool sw, bool psi_regs,
                            unsigned nblocks, hipStream_t s, bool batched) {
  if (batched && (!a.desc || !a.list)) return hipErrorInvalidValue;
#define FQ_CASE(RB_, TB_)                                                                   \
  if (rb == RB_ && tb == TB_)                                                               \
    return sw ? launch_single_t<Real, RB_, TB_, true>(a, nblocks, psi_regs, batched, s)     \
              : launch_single_t<Real, RB_, TB_, false>(a, nblocks, psi_regs, batched, s);
  FQ_SHAPES(FQ_CASE)
#undef FQ_CASE
  return hipErrorInvalidValue;
}

}  // namespace fq
