// Launch interface of the kicked-Ising kernels (library-internal).
#pragma once

#include "common.h"

namespace fq {

enum : int {
  KI_PHASE = 1,      // multiply by the diagonal phase table after the first kick
  KI_ADD_PSI = 2,    // add psi (times psi_coef if KI_PSI_COEF)
  KI_PSI_COEF = 4,
  KI_SCALE_IN = 8,   // multiply the loaded tile by in_coef
  KI_PREFETCH_PHASE = 16,  // load the phase-table entries with the tile
};

// Which one-qubit butterflies to apply, split by where the bit lives
// (see tile_engine.h): register bits of layout A / B, lane bits of A / B.
struct KickMasks {
  unsigned regA, laneA, regB, laneB;
};

// Per-problem pointers of a batched launch (one problem per blockIdx.y of a
// pass, per workgroup of the single-tile kernel): psi, the state x, the phase
// tables and the butterfly weight of that problem's operator.
template <typename Real>
struct KiDesc {
  const cpx<Real>* psi;
  cpx<Real>* x;
  const cpx<Real>* tlo;
  const cpx<Real>* thi;
  double w;
  double pad;
  // chi[g] = K_g psi, the kick of tile group g applied to psi (or null): a
  // pass that ends with the kick of its own group then adds chi[g] instead
  // of kicking psi (KiPassArgs::chi)
  const cpx<Real>* chi[2];
};

template <typename Real>
struct KiPassArgs {
  const cpx<Real>* xin;
  cpx<Real>* xout;
  const cpx<Real>* psi;
  const cpx<Real>* tlo;
  const cpx<Real>* thi;
  double w;                 // butterfly weight (tan or cot form)
  double psi_coef_re, psi_coef_im;
  double in_coef_re, in_coef_im;
  int n, c, p, m;           // tile bits, chunk bits, position of the high run, table split
  int flags;
  KickMasks k1, k2;         // before / after the phase
  // batched launches: problem desc[list[blockIdx.y]]; the pass reads psi
  // (from_psi) or x and writes x.  With flat, the grid is one-dimensional
  // over (problem, tile) pairs, problem-major, dealt to the XCDs in
  // contiguous runs, so that all tiles of a problem share one L2
  // (tile_log = log2 of the tiles per problem).
  const KiDesc<Real>* desc;
  const int* list;
  int from_psi;
  int flat, tile_log;
  // batched passes with k2 == k1 (kick, phase, +psi, the same kick again):
  // chi = g + 1 computes K D K x + chi[g] with chi[g] = K psi from the
  // problem's descriptor.  The kicks commute, so the layout-B parts of both
  // kicks and the phase run between one A->B and one B->A change (two
  // layout changes per pass instead of four).  0: plain psi.
  int chi;
  // three-layout passes (ki_launch_pass3): kicked register bits of layout C
  // for the first / second kick (k1 / k2 carry layouts A and B and B's lane 0),
  // and the phase table that varies over layout C's registers (0: the low
  // table, one high-table entry per thread; 1: the high table, one low entry)
  unsigned k1c, k2c;
  int t3;
};

template <typename Real>
struct KiSingleArgs {
  const cpx<Real>* xin;
  cpx<Real>* xout;
  const cpx<Real>* psi;
  const cpx<Real>* tlo;
  const cpx<Real>* thi;
  const double2* coefs;     // per-step coefficient of psi, or NULL (= 1)
  double w;
  double in_coef_re, in_coef_im;
  size_t batch_stride;      // amplitudes between problems (blockIdx.x)
  int L, m, steps, flags;
  KickMasks kick;
  // batched launches: workgroup b runs problem desc[list[b]], reading psi
  // (from_psi) or x and writing x
  const KiDesc<Real>* desc;
  const int* list;
  int from_psi;
};

// nprob > 0 selects the batched kernels (a.desc / a.list, nprob problems).
template <typename Real>
hipError_t ki_launch_pass(const KiPassArgs<Real>& a, int rb, int tb, bool sw, unsigned ntiles, hipStream_t s,
                          unsigned nprob = 0);
// Persistent pipelined form of a batched pass: `grid` workgroups (a multiple
// of 8, at most nprob * ntiles) walk the (problem, tile) items, each loading
// its next tile while it works on the current one.  a.tile_log = log2 ntiles;
// a.flat is ignored.  Shapes: (RB, TB) in {(2,8), (3,7), (3,8), (3,9)}, and
// (4,6..9) in complex64.
template <typename Real>
hipError_t ki_launch_pipe(const KiPassArgs<Real>& a, int rb, int tb, bool sw, unsigned ntiles, unsigned nprob,
                          unsigned grid, hipStream_t s);
// Horner pass (KI_PHASE | KI_ADD_PSI, no coefficients) over a tile of
// n = 4 + tb bits in three register layouts, so that every kicked bit but at
// most one (a DPP lane bit) is a register bit in one of them; complex64 only
// (complex128 would need twice the registers).  nprob as in ki_launch_pass.
template <typename Real>
hipError_t ki_launch_pass3(const KiPassArgs<Real>& a, int tb, unsigned ntiles, hipStream_t s, unsigned nprob = 0);

template <typename Real>
hipError_t ki_launch_single(const KiSingleArgs<Real>& a, int rb, int tb, bool sw, bool psi_regs,
                            unsigned nblocks, hipStream_t s, bool batched = false);

hipError_t launch_cast_c128_to_c64(const void* in, void* out, size_t n, hipStream_t s);
hipError_t launch_cast_c64_to_c128(const void* in, void* out, size_t n, hipStream_t s);

}  // namespace fq
