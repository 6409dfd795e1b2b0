// Launch interface of the brickwork kernels (library-internal).
#pragma once

#include "tile_engine.h"

namespace fq {

enum : int {
  BW_ROT = 1,       // multiply by rot (e^{-i phi}) after the gates
  BW_ADD_PSI = 2,   // add psi (times psi_coef if BW_PSI_COEF)
  BW_PSI_COEF = 4,
};

// One gate of a window: kind 2 = two-site gate on window bits (l, l+1),
// local index 2*b_{l+1} + b_l; kind 1 = one-site gate on window bit l.  mat
// indexes the 16-entry matrices.
struct BwGate {
  int8_t kind, l;
  int16_t mat;
};
static_assert(sizeof(BwGate) == 4, "BwGate is read as one 32-bit word");

// Gates per window at most (the kernels apply them one matrix at a time).
constexpr size_t kBwWindowGates = 8;

// One window: the gates gates[first .. first + count) act inside tile bits
// [b, b + WB) and are applied in this order, with the window's 2^WB
// amplitudes held in registers (one LDS round trip per window).
struct BwWin {
  int16_t b, first, count, pad;
};
static_assert(sizeof(BwWin) == 8, "BwWin is read as one 64-bit word");

// A launch covers nvec vectors of vstride amplitudes each (vector v at
// offset v * vstride of xin, xout and psi); its work items are (vector, tile)
// pairs, item = v * 2^tile_bits + tile.
struct BwPassArgs {
  const void* xin;
  void* xout;
  const void* psi;
  const void* mats;  // 16-entry matrices in the pass precision
  const BwWin* wins;
  const BwGate* gates;
  int nwin;
  int n, c, p;
  int flags;
  int tile_bits;  // log2(tiles per vector)
  unsigned long long vstride;
  double rot_re, rot_im;
  double psi_coef_re, psi_coef_im;
};

// nitems = tiles per vector x vectors
hipError_t bw_launch_pass(const BwPassArgs& a, bool c64_dt, int wb, unsigned nitems, hipStream_t s);

}  // namespace fq
