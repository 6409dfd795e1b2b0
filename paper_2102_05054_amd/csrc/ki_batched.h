// Batched kicked-Ising filter and U passes: many independent problems of one
// chain length L (own couplings, own target phase, own vectors) advanced
// together, one launch per Horner pass for the whole batch.
#pragma once

#include <vector>

#include "op.h"

namespace fq {

// How a batch applies U: one workgroup per problem running all k steps in
// one launch (small L), or the multi-pass tile plan with one launch per pass
// covering every problem (blockIdx.y = problem).
struct KiBatchShape {
  int L = 0, m = 0;
  bool sw = false;
  bool single = false;
  int srb = 0, stb = 0;  // single-workgroup tile
  KiPlan plan;           // multi-pass plan
  // multi-pass only: run the k steps on sub-batches of at most `chunk`
  // problems (0 = all at once), so that a sub-batch's states stay in the
  // Infinity Cache across passes; `flat` keeps each problem on one XCD
  unsigned chunk = 0;
  bool flat = false;
  // multi-pass only: persistent pipelined passes with this many workgroups
  // (0 = one workgroup per tile); a group with fewer than two tiles per
  // workgroup, or without a pipelined instance, keeps one workgroup per tile
  unsigned pipe = 0;
  // phase-table entries fetched with the tile (1), mid-pass (0), or by the
  // tile-count rule (-1): fetching early costs registers and occupancy
  int prefetch = -1;
  // multi-pass only: Horner passes of 16-amplitude tiles in the three-layout
  // form (ki_launch_pass3; no folded or pipelined variant)
  bool three = false;
};

// Candidate shapes for (L, kick form, precision), the default first.
std::vector<KiBatchShape> ki_batch_candidates(int L, bool sw, bool c64_dt);

// x_q = g_k(U_q) psi_q for the problems desc[list[0..n)] (geometric sum; the
// rotation e^{-i phi_q} and the kick scales live in each problem's tables).
// With chi0 / chi1 (descriptors whose x is the problem's desc.chi[0] /
// desc.chi[1] buffer, same indexing as desc) two-group plans first write
// chi_g = K_g psi and then run every Horner pass but the last in the folded
// form (KiPassArgs::chi).
template <typename Real>
fq_status ki_batch_filter(const KiBatchShape& sh, int k, const KiDesc<Real>* desc, const int* list, unsigned n,
                          hipStream_t s, const KiDesc<Real>* chi0 = nullptr, const KiDesc<Real>* chi1 = nullptr);

// x_q = U_q psi_q.
template <typename Real>
fq_status ki_batch_apply(const KiBatchShape& sh, const KiDesc<Real>* desc, const int* list, unsigned n,
                         hipStream_t s);

// fq_set_kernel_policy: which pass forms the autotuner may pick.
fq_status ki_set_policy(int policy);

// Autotuner: times the candidate shapes on the given problems (their x
// buffers are overwritten) for min(k, 32) Horner steps, then the sub-batch
// sizes, the XCD mapping, the phase-table prefetch and the pipelined
// persistent form (1, 2, 4 workgroups per CU) for the fastest shape, and returns the fastest
// combination; results are cached per (L, kick form, precision, k, batch size
// class).  best_us (optional) receives the time per Horner step of the batch.
template <typename Real>
fq_status ki_batch_tune(int L, bool sw, int k, const KiDesc<Real>* desc, const int* list, unsigned n,
                        hipStream_t s, KiBatchShape* out, double* best_us, const KiDesc<Real>* chi0 = nullptr,
                        const KiDesc<Real>* chi1 = nullptr);

// The shape ki_batch_tune would return, without timing anything (no events,
// no trial launches): the cached tuner choice for this (L, kick form,
// precision, k, batch size class) if there is one, otherwise the default
// candidate (single workgroup for L <= 13, else the standard multi-pass plan).
template <typename Real>
fq_status ki_batch_shape_untimed(int L, bool sw, int k, unsigned n, KiBatchShape* out);

}  // namespace fq
