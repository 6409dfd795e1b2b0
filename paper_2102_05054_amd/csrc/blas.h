// FP64 vector kernels of the Krylov side (library-internal launch interface).
//
// Basis layout: V is d x ncols complex128, column-major with leading
// dimension ldv (column i at V + i*ldv), one Krylov vector per column.
#pragma once

#include "common.h"
#include "ki_kernels.h"

namespace fq {

// rows handled by one workgroup of the row-blocked kernels
constexpr int kRowsPerThread = 4;
constexpr int kBlockThreads = 256;
inline unsigned row_blocks(size_t d) {
  const size_t per = size_t(kRowsPerThread) * kBlockThreads;
  return static_cast<unsigned>((d + per - 1) / per);
}

// partial[b*ldp + i] = sum_{rows r of block b} conj(V[r, i]) * w[r],  i < ncols
hipError_t launch_dots(const c128* V, size_t ldv, int ncols, const c128* w, size_t d, c128* partial, int ldp,
                       hipStream_t s);
// out[i] = sum_b partial[b*ldp + i]; if acc != NULL also acc[i] += out[i]
hipError_t launch_reduce_cols(const c128* partial, int ldp, unsigned nblk, int ncols, c128* out, hipStream_t s);
// w -= V h  (h: ncols complex128 on the device)
hipError_t launch_update(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d, hipStream_t s);
// fused: w -= V h, then partial dots of the updated w against V (one read of V per row block
// for the update, one for the dots, issued back to back so the second read hits cache)
hipError_t launch_update_dots(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d,
                              c128* partial, int ldp, hipStream_t s);
// partial[b] = sum_{rows r of block b} |w[r]|^2 (stored in .x)
hipError_t launch_norm2(const c128* w, size_t d, c128* partial, hipStream_t s);
// w -= V h, then partial[b] = sum |w|^2 over the block's rows
hipError_t launch_update_norm2(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d,
                               c128* partial, hipStream_t s);
// nrm[0] = sqrt(sum_b partial[b].x), nrm[1] = 1/nrm[0] (0 if nrm[0] == 0)
hipError_t launch_reduce_norm(const c128* partial, unsigned nblk, double* nrm, hipStream_t s);
// out = in * scale[0] (scale read from device memory)
hipError_t launch_scale_dev(const c128* in, const double* scale, c128* out, size_t d, hipStream_t s);
// out = a * in
hipError_t launch_scale_c128(const c128* in, double are, double aim, c128* out, size_t d, hipStream_t s);
hipError_t launch_scale_c64(const c64* in, double are, double aim, c64* out, size_t d, hipStream_t s);
// y = y - a * x   (a on the device, complex)
hipError_t launch_axpy_dev(const c128* a, const c128* x, c128* y, size_t d, hipStream_t s);
// Y[:, c] = sum_{i<m} V[:, i] Q[i, c] for c < p.  Y may equal V (in place, p <= m).
// Q: m x p complex128, k-major (Q[i*p + c]) on the device.  FP64 matrix cores
// for p <= 256 and d a multiple of 16.
hipError_t launch_basis_gemm(const c128* V, size_t ldv, int m, const c128* Q, int p, c128* Y, size_t ldy,
                             size_t d, hipStream_t s);
// G (n x n, row-major) = sum_t A(i,t) conj(A(j,t)), A(i,t) = X[i*si + t*st],
// conjugated when conj_in
hipError_t launch_gram(const c128* X, size_t si, size_t st, bool conj_in, int n, size_t T, c128* G, hipStream_t s);
// v[i] = counter-based uniform complex in [-1, 1)^2 from (seed, i)
hipError_t launch_random(c128* v, size_t d, unsigned long long seed, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched forms (many independent problems of one size d in one launch).
// ---------------------------------------------------------------------------

// One problem of a batched Krylov solve (device-resident descriptor).
struct KDesc {
  c128* V;         // d x (ncv + 1), column-major, leading dimension d
  c128* w;         // d
  c128* partial;   // nblk x ldp
  double* slots;   // (ncv + 1) x slot_doubles: h1[ncv+1], h2[ncv+1] (complex), beta, 1/beta
  double* small;   // 16 doubles of scratch (norm, 1/norm)
};

// Problems kd[list[0..n)] of size d; blockIdx.y walks the list.
struct BatchArgs {
  const KDesc* kd;
  const int* list;
  unsigned n;
  size_t d;
  unsigned nblk;   // row_blocks(d)
  int ldp;         // ncv + 1
  int slot_doubles;
  int ncv;
};

// Y = V Q (m x p, k-major) for one problem; ld = d for V and Y.  Y may be V.
struct GemmDesc {
  const c128* V;
  c128* Y;
  const c128* Q;
  size_t ld;
  int m, p;
};

// Ritz pairs of one problem: Y holds the vectors (column i at Y + i*d), u is
// scratch for U y, partial >= 2 * row_blocks(d) complex, out[4i..4i+3] =
// (Re omega, Im omega, residual, 1/||y||).
struct RDesc {
  c128* Y;
  c128* u;
  c128* partial;
  double* out;
};

// CGS2 of Arnoldi column j with ncols = j + 1 basis vectors (see arnoldi_step)
hipError_t launch_b_dots(const BatchArgs& a, int ncols, hipStream_t s);
hipError_t launch_b_reduce_slot(const BatchArgs& a, int ncols, int j, int which, hipStream_t s);
hipError_t launch_b_update(const BatchArgs& a, int ncols, int j, int which, hipStream_t s);
hipError_t launch_b_reduce_norm(const BatchArgs& a, int j, hipStream_t s);
hipError_t launch_b_scale_next(const BatchArgs& a, int j, hipStream_t s);
// V[:, col] /= ||V[:, col]||
hipError_t launch_b_normalize_col(const BatchArgs& a, int col, hipStream_t s);
// V[:, to] = V[:, from]
hipError_t launch_b_copy_col(const BatchArgs& a, int from, int to, hipStream_t s);
// fd[q].psi = V[:, j] in the filter precision; w = fd[q].x (complex64 state)
template <typename Real>
hipError_t launch_b_cast_in(const BatchArgs& a, const KiDesc<Real>* fd, int j, hipStream_t s);
hipError_t launch_b_cast_out(const BatchArgs& a, const KiDesc<float>* fd, hipStream_t s);
// n basis products on the FP64 matrix cores (p <= pmax <= 256 in every
// descriptor, d a multiple of 16; 64 rows per workgroup when d is a multiple of 64)
hipError_t launch_b_basis_gemm(const GemmDesc* g, unsigned n, size_t d, hipStream_t s, int pmax);
// Ritz pair i of n problems, after u = U y: omega, residual; y normalised
hipError_t launch_r_rayleigh(const RDesc* rd, unsigned n, int i, size_t d, hipStream_t s);

// Block forms for b in {1, 2, 4, 8} vectors W[:, c] at W + c*ldw:
// partial[blk*ldp + i*b + c] = row-block sums of conj(V[r, i]) W[r, c]
// (reduce with launch_reduce_cols over ncols*b entries);
hipError_t launch_bdots(const c128* V, size_t ldv, int ncols, const c128* W, size_t ldw, int b, size_t d,
                        c128* partial, int ldp, hipStream_t s);
// W[:, c] -= sum_i V[:, i] H[i*b + c]  (H: ncols x b on the device, ncols*b <= 4096)
hipError_t launch_bupdate(const c128* V, size_t ldv, int ncols, const c128* H, c128* W, size_t ldw, int b, size_t d,
                          hipStream_t s);

}  // namespace fq
