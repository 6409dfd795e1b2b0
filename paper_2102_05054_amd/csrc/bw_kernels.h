// Launch interface of the brickwork kernels (library-internal).
#pragma once

#include "tile_engine.h"

namespace fq {

enum : int {
  BW_ROT = 1,       // multiply by rot (e^{-i phi}) after the gates
  BW_ADD_PSI = 2,   // add psi (times psi_coef if BW_PSI_COEF)
  BW_PSI_COEF = 4,
};

// One window: up to three gates of one layer inside tile bits [b, b + wb).
// kind 2 = two-site gate on local bits (l, l+1), local index 2*b_{l+1} + b_l;
// kind 1 = one-site gate on local bit l.  mat indexes 16-entry matrices.
struct BwWindow {
  int8_t b, ngates;
  int8_t kind[3];
  int8_t l[3];
  int16_t mat[3];
  int16_t pad;
};
static_assert(sizeof(BwWindow) == 16, "BwWindow is read as one 16-byte word");

struct BwPassArgs {
  const void* xin;
  void* xout;
  const void* psi;
  const void* mats;  // 16-entry matrices in the pass precision
  const BwWindow* wins;
  int nwin;
  int n, c, p;
  int flags;
  double rot_re, rot_im;
  double psi_coef_re, psi_coef_im;
};

hipError_t bw_launch_pass(const BwPassArgs& a, bool c64_dt, int wb, unsigned ntiles, hipStream_t s);

}  // namespace fq
