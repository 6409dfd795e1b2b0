// FP64 kernels of the Krylov side: Gram-Schmidt projections, norms, scaling,
// the restart / Ritz-vector basis product and the start vector.
//
// The projections h = V^H w and w -= V h with a single new vector are
// matrix-vector products (0.5 flop per byte of V), bound by HBM bandwidth;
// they stream V column by column with every lane reading consecutive rows.
// Reductions use a fixed tree (wavefront shuffles, then the four waves), so
// results are bitwise reproducible for a given launch shape.
#include "blas.h"

namespace fq {

namespace {

constexpr int RPT = kRowsPerThread;
constexpr int NT = kBlockThreads;
constexpr int NCH = 8;  // columns per reduction round

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  return v;
}

// Reduce NCH complex per-thread values over the block; thread c < nvalid
// receives value c in (ox, oy).
__device__ __forceinline__ void block_sum_nch(double (&ax)[NCH], double (&ay)[NCH], double (*red)[2 * NCH],
                                              int tid) {
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    ax[c] = wave_sum(ax[c]);
    ay[c] = wave_sum(ay[c]);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      red[wv][2 * c] = ax[c];
      red[wv][2 * c + 1] = ay[c];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void dots_body(const c128* __restrict__ V, size_t ldv, int ncols,
                                          const c128* __restrict__ w, size_t d, c128* __restrict__ partial, int ldp,
                                          unsigned blk) {
  __shared__ double red[NT / 64][2 * NCH];
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blk) * NT * RPT + tid;
  c128 wr[RPT];
  bool ok[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    ok[t] = r < d;
    wr[t] = ok[t] ? w[r] : mk<double>(0, 0);
  }
  for (int i0 = 0; i0 < ncols; i0 += NCH) {
    double ax[NCH], ay[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      ax[c] = 0.0;
      ay[c] = 0.0;
      if (i0 + c < ncols) {
        const c128* col = V + size_t(i0 + c) * ldv;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          if (ok[t]) {
            const c128 v = col[r0 + size_t(t) * NT];
            ax[c] += v.x * wr[t].x + v.y * wr[t].y;
            ay[c] += v.x * wr[t].y - v.y * wr[t].x;
          }
        }
      }
    }
    block_sum_nch(ax, ay, red, tid);
    if (tid < NCH && i0 + tid < ncols) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) {
        sx += red[q][2 * tid];
        sy += red[q][2 * tid + 1];
      }
      partial[size_t(blk) * ldp + i0 + tid] = mk<double>(sx, sy);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(NT) dots_kernel(const c128* __restrict__ V, size_t ldv, int ncols,
                                                  const c128* __restrict__ w, size_t d, c128* __restrict__ partial,
                                                  int ldp) {
  dots_body(V, ldv, ncols, w, d, partial, ldp, blockIdx.x);
}

// out[i] = sum over row blocks of partial[b*ldp + i] (column i of one problem)
__device__ __forceinline__ void reduce_cols_body(const c128* __restrict__ partial, int ldp, unsigned nblk,
                                                 c128* __restrict__ out, int i) {
  __shared__ double red[NT / 64][2];
  const int tid = threadIdx.x;
  double sx = 0.0, sy = 0.0;
  for (unsigned b = tid; b < nblk; b += NT) {
    const c128 v = partial[size_t(b) * ldp + i];
    sx += v.x;
    sy += v.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = sx;
    red[tid >> 6][1] = sy;
  }
  __syncthreads();
  if (tid == 0) {
    double tx = 0.0, ty = 0.0;
    for (int q = 0; q < NT / 64; ++q) {
      tx += red[q][0];
      ty += red[q][1];
    }
    out[i] = mk<double>(tx, ty);
  }
}

__global__ void __launch_bounds__(NT) reduce_cols_kernel(const c128* __restrict__ partial, int ldp, unsigned nblk,
                                                         c128* __restrict__ out) {
  reduce_cols_body(partial, ldp, nblk, out, blockIdx.x);
}

template <bool DOTS, bool NORM>
__device__ __forceinline__ void update_body(const c128* __restrict__ V, size_t ldv, int ncols,
                                            const c128* __restrict__ h, c128* __restrict__ w, size_t d,
                                            c128* __restrict__ partial, int ldp, unsigned blk) {
  extern __shared__ c128 hs[];
  __shared__ double red[NT / 64][2 * NCH];
  const int tid = threadIdx.x;
  for (int i = tid; i < ncols; i += NT) hs[i] = h[i];
  __syncthreads();
  const size_t r0 = static_cast<size_t>(blk) * NT * RPT + tid;
  c128 acc[RPT];
  bool ok[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    ok[t] = r < d;
    acc[t] = ok[t] ? w[r] : mk<double>(0, 0);
  }
  int i = 0;
  for (; i + 4 <= ncols; i += 4) {
    c128 v[4][RPT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < RPT; ++t) v[u][t] = ok[t] ? V[size_t(i + u) * ldv + r0 + size_t(t) * NT] : mk<double>(0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const c128 hh = hs[i + u];
#pragma unroll
      for (int t = 0; t < RPT; ++t) acc[t] = csub(acc[t], cmul(v[u][t], hh));
    }
  }
  for (; i < ncols; ++i) {
    const c128 hh = hs[i];
#pragma unroll
    for (int t = 0; t < RPT; ++t)
      if (ok[t]) acc[t] = csub(acc[t], cmul(V[size_t(i) * ldv + r0 + size_t(t) * NT], hh));
  }
#pragma unroll
  for (int t = 0; t < RPT; ++t)
    if (ok[t]) w[r0 + size_t(t) * NT] = acc[t];

  if constexpr (NORM) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < RPT; ++t) s += acc[t].x * acc[t].x + acc[t].y * acc[t].y;
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6][0] = s;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int q = 0; q < NT / 64; ++q) tot += red[q][0];
      partial[blk] = mk<double>(tot, 0.0);
    }
  }
  if constexpr (DOTS) {
    for (int i0 = 0; i0 < ncols; i0 += NCH) {
      double ax[NCH], ay[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        ax[c] = 0.0;
        ay[c] = 0.0;
        if (i0 + c < ncols) {
          const c128* col = V + size_t(i0 + c) * ldv;
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
            if (ok[t]) {
              const c128 v = col[r0 + size_t(t) * NT];
              ax[c] += v.x * acc[t].x + v.y * acc[t].y;
              ay[c] += v.x * acc[t].y - v.y * acc[t].x;
            }
          }
        }
      }
      block_sum_nch(ax, ay, red, tid);
      if (tid < NCH && i0 + tid < ncols) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) {
          sx += red[q][2 * tid];
          sy += red[q][2 * tid + 1];
        }
        partial[size_t(blk) * ldp + i0 + tid] = mk<double>(sx, sy);
      }
      __syncthreads();
    }
  }
}

template <bool DOTS, bool NORM>
__global__ void __launch_bounds__(NT) update_kernel(const c128* __restrict__ V, size_t ldv, int ncols,
                                                    const c128* __restrict__ h, c128* __restrict__ w, size_t d,
                                                    c128* __restrict__ partial, int ldp) {
  update_body<DOTS, NORM>(V, ldv, ncols, h, w, d, partial, ldp, blockIdx.x);
}

__device__ __forceinline__ void norm2_body(const c128* __restrict__ w, size_t d, c128* __restrict__ partial,
                                           unsigned blk) {
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blk) * NT * RPT + tid;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    if (r < d) {
      const c128 v = w[r];
      s += v.x * v.x + v.y * v.y;
    }
  }
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < NT / 64; ++q) tot += red[q];
    partial[blk] = mk<double>(tot, 0.0);
  }
}

__global__ void __launch_bounds__(NT) norm2_kernel(const c128* __restrict__ w, size_t d, c128* __restrict__ partial) {
  norm2_body(w, d, partial, blockIdx.x);
}

__device__ __forceinline__ void reduce_norm_body(const c128* __restrict__ partial, unsigned nblk,
                                                 double* __restrict__ nrm) {
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (unsigned b = tid; b < nblk; b += NT) s += partial[b].x;
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < NT / 64; ++q) tot += red[q];
    const double n = sqrt(tot);
    nrm[0] = n;
    nrm[1] = n > 0.0 ? 1.0 / n : 0.0;
  }
}

__global__ void __launch_bounds__(NT) reduce_norm_kernel(const c128* __restrict__ partial, unsigned nblk,
                                                         double* __restrict__ nrm) {
  reduce_norm_body(partial, nblk, nrm);
}

__global__ void scale_dev_kernel(const c128* __restrict__ in, const double* __restrict__ scale, c128* __restrict__ out,
                                 size_t d) {
  const double a = scale[0];
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x) {
    const c128 v = in[i];
    out[i] = mk<double>(v.x * a, v.y * a);
  }
}

template <typename Real>
__global__ void scale_kernel(const cpx<Real>* __restrict__ in, double are, double aim, cpx<Real>* __restrict__ out,
                             size_t d) {
  const cpx<Real> a = mk<Real>(static_cast<Real>(are), static_cast<Real>(aim));
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x)
    out[i] = cmul(in[i], a);
}

__global__ void axpy_dev_kernel(const c128* __restrict__ a, const c128* __restrict__ x, c128* __restrict__ y,
                                size_t d) {
  const c128 aa = a[0];
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x)
    y[i] = csub(y[i], cmul(aa, x[i]));
}

// Y[r, c] = sum_i V[r, i] Q[i, c] for a block of BR rows staged in LDS
// (transposed, lds[i*BR + r]); all of a block's rows are read before any is
// written, so Y may alias V.  Q is k-major: Q[i*p + c].  Fallback for p > 256.
__global__ void __launch_bounds__(NT) basis_gemm_kernel(const c128* __restrict__ V, size_t ldv, int m,
                                                        const c128* __restrict__ Q, int p, c128* Y, size_t ldy,
                                                        size_t d, int BR) {
  extern __shared__ c128 st[];
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blockIdx.x) * BR;
  for (int idx = tid; idx < BR * m; idx += NT) {
    const int i = idx / BR, r = idx % BR;
    const size_t row = r0 + r;
    st[idx] = row < d ? V[size_t(i) * ldv + row] : mk<double>(0, 0);
  }
  __syncthreads();
  for (int o = tid; o < BR * p; o += NT) {
    const int r = o % BR, c = o / BR;
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < m; ++i) {
      const c128 a = st[i * BR + r];
      const c128 b = Q[size_t(i) * p + c];
      sx += a.x * b.x - a.y * b.y;
      sy += a.x * b.y + a.y * b.x;
    }
    const size_t row = r0 + r;
    if (row < d) Y[size_t(c) * ldy + row] = mk<double>(sx, sy);
  }
}

// The same product on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  One
// wavefront owns 16 rows and all p <= 256 columns, streaming V's 16-row
// slices over k in steps of 4 and keeping the 16x16 output tiles of the real
// and imaginary parts in accumulators; rows are written only after the last
// k, so Y may alias V.  Complex product with four real MFMAs per tile:
//   Re += Vr Qr + (-Vi) Qi,   Im += Vr Qi + Vi Qr.
// Operand layout: A lane l = A[l%16][l/16], B lane l = B[l/16][l%16],
// D lane l register r = D[4r + l/16][l%16].
typedef double fq_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void basis_gemm_mfma_body(const c128* __restrict__ V, size_t ldv, int m,
                                                     const c128* __restrict__ Q, int p, c128* Y, size_t ldy,
                                                     unsigned blk) {
  constexpr int MAXT = 16;
  const int l = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blk) * 16;
  const int ntile = (p + 15) >> 4;
  fq_d4 accr[MAXT], acci[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    accr[t] = fq_d4{0.0, 0.0, 0.0, 0.0};
    acci[t] = fq_d4{0.0, 0.0, 0.0, 0.0};
  }
  const int lr = l & 15, lk = l >> 4;
  for (int k0 = 0; k0 < m; k0 += 4) {
    const int k = k0 + lk;
    const c128 a = k < m ? V[size_t(k) * ldv + r0 + lr] : mk<double>(0, 0);
    const double nai = -a.y;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < ntile) {
        const int col = (t << 4) + lr;
        const c128 b = (k < m && col < p) ? Q[size_t(k) * p + col] : mk<double>(0, 0);
        accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, accr[t], 0, 0, 0);
        accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, b.y, accr[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acci[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < ntile) {
      const int col = (t << 4) + lr;
      if (col < p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * r + lk;
          Y[size_t(col) * ldy + r0 + i] = mk<double>(accr[t][r], acci[t][r]);
        }
      }
    }
  }
}

__global__ void __launch_bounds__(64) basis_gemm_mfma_kernel(const c128* __restrict__ V, size_t ldv, int m,
                                                             const c128* __restrict__ Q, int p, c128* Y, size_t ldy) {
  basis_gemm_mfma_body(V, ldv, m, Q, p, Y, ldy, blockIdx.x);
}

// Same product with 64 rows per workgroup (4 waves of 16 rows): chunks of
// kGemmKc rows of Q are staged through LDS, so that a workgroup reads Q once
// from L2 for 64 rows of V instead of once per 16, and four waves share each
// chunk.  Y may equal V: a workgroup writes only its own rows, after all of
// its reads.
// MAXT: 16-column tiles of Y a wave accumulates (>= ceil(p / 16)); fewer
// tiles, fewer accumulator registers, more waves per SIMD.
constexpr int kGemmKc = 8;
template <int MAXT>
__device__ __forceinline__ void basis_gemm_mfma64_body(const c128* __restrict__ V, size_t ldv, int m,
                                                       const c128* __restrict__ Q, int p, c128* Y, size_t ldy,
                                                       unsigned block) {
  extern __shared__ char gemm_smem[];
  c128* qs = reinterpret_cast<c128*>(gemm_smem);  // kGemmKc x p
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const size_t r0 = static_cast<size_t>(block) * 64 + 16 * (tid >> 6);
  const int ntile = (p + 15) >> 4;
  fq_d4 accr[MAXT], acci[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    accr[t] = fq_d4{0.0, 0.0, 0.0, 0.0};
    acci[t] = fq_d4{0.0, 0.0, 0.0, 0.0};
  }
  const int lr = l & 15, lk = l >> 4;
  for (int c0 = 0; c0 < m; c0 += kGemmKc) {
    const int kc = min(kGemmKc, m - c0);
    __syncthreads();  // the previous chunk has been read
    for (int e = tid; e < kGemmKc * p; e += 256) {
      const int kk = e / p;
      qs[e] = kk < kc ? Q[size_t(c0 + kk) * p + (e - kk * p)] : mk<double>(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < kGemmKc; k0 += 4) {
      const int kk = k0 + lk;
      const c128 a = kk < kc ? V[size_t(c0 + kk) * ldv + r0 + lr] : mk<double>(0, 0);
      const double nai = -a.y;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t < ntile) {
          const int col = (t << 4) + lr;
          const c128 b = col < p ? qs[kk * p + col] : mk<double>(0, 0);
          accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, accr[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, b.y, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acci[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci[t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < ntile) {
      const int col = (t << 4) + lr;
      if (col < p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * r + lk;
          Y[size_t(col) * ldy + r0 + i] = mk<double>(accr[t][r], acci[t][r]);
        }
      }
    }
  }
}

template <int MAXT>
__global__ void __launch_bounds__(256) basis_gemm_mfma64_kernel(const c128* __restrict__ V, size_t ldv, int m,
                                                                const c128* __restrict__ Q, int p, c128* Y,
                                                                size_t ldy) {
  basis_gemm_mfma64_body<MAXT>(V, ldv, m, Q, p, Y, ldy, blockIdx.x);
}

// Gram matrix G[i][j] = sum_t A(i,t) conj(A(j,t)), A(i,t) = X[i*si + t*st]
// (conjugated if cj): 16x16 output tiles, 64-long t chunks staged in LDS.
__global__ void __launch_bounds__(256) gram_kernel(const c128* __restrict__ X, size_t si, size_t st, int cj, int n,
                                                   size_t T, c128* __restrict__ G) {
  __shared__ c128 As[16][65], Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  double sx = 0.0, sy = 0.0;
  for (size_t t0 = 0; t0 < T; t0 += 64) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      const size_t t = t0 + c;
      c128 a = mk<double>(0, 0), b = mk<double>(0, 0);
      if (t < T) {
        if (i0 + r < n) a = X[size_t(i0 + r) * si + t * st];
        if (j0 + r < n) b = X[size_t(j0 + r) * si + t * st];
        if (cj) {
          a.y = -a.y;
          b.y = -b.y;
        }
      }
      As[r][c] = a;
      Bs[r][c] = b;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 64; ++c) {
      const c128 a = As[ty][c], b = Bs[tx][c];
      sx += a.x * b.x + a.y * b.y;  // a * conj(b)
      sy += a.y * b.x - a.x * b.y;
    }
    __syncthreads();
  }
  if (i0 + ty < n && j0 + tx < n) G[size_t(i0 + ty) * n + (j0 + tx)] = mk<double>(sx, sy);
}

// ---------------------------------------------------------------------------
// Batched forms: blockIdx.y selects problem kd[list[blockIdx.y]] (or the
// descriptor blockIdx.y); each block then runs the single-problem body, so a
// batched solve does exactly the arithmetic of the single-problem one.
// ---------------------------------------------------------------------------
__device__ __forceinline__ const KDesc& bprob(const KDesc* kd, const int* list) { return kd[list[blockIdx.y]]; }
__device__ __forceinline__ c128* slot_c(const KDesc& P, int j, int sd, int off) {
  return reinterpret_cast<c128*>(P.slots + size_t(j) * sd) + off;
}

__global__ void __launch_bounds__(NT) b_dots_kernel(const KDesc* kd, const int* list, int ncols, size_t d, int ldp) {
  const KDesc& P = bprob(kd, list);
  dots_body(P.V, d, ncols, P.w, d, P.partial, ldp, blockIdx.x);
}

// h (which = 0: first projection, 1: second) of column j from the partial sums
__global__ void __launch_bounds__(NT) b_reduce_slot_kernel(const KDesc* kd, const int* list, int ldp, unsigned nblk,
                                                           int j, int sd, int off) {
  const KDesc& P = bprob(kd, list);
  reduce_cols_body(P.partial, ldp, nblk, slot_c(P, j, sd, off), blockIdx.x);
}

template <bool DOTS, bool NORM>
__global__ void __launch_bounds__(NT) b_update_kernel(const KDesc* kd, const int* list, int ncols, size_t d, int ldp,
                                                      int j, int sd, int off) {
  const KDesc& P = bprob(kd, list);
  update_body<DOTS, NORM>(P.V, d, ncols, slot_c(P, j, sd, off), P.w, d, P.partial, ldp, blockIdx.x);
}

__global__ void __launch_bounds__(NT) b_reduce_norm_kernel(const KDesc* kd, const int* list, unsigned nblk, int j,
                                                           int sd, int off_d) {
  const KDesc& P = bprob(kd, list);
  reduce_norm_body(P.partial, nblk, P.slots + size_t(j) * sd + off_d);
}

// V[:, j+1] = w / beta_j
__global__ void b_scale_next_kernel(const KDesc* kd, const int* list, size_t d, int j, int sd, int off_d) {
  const KDesc& P = bprob(kd, list);
  const double a = P.slots[size_t(j) * sd + off_d + 1];
  c128* out = P.V + size_t(j + 1) * d;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x) {
    const c128 v = P.w[i];
    out[i] = mk<double>(v.x * a, v.y * a);
  }
}

__global__ void __launch_bounds__(NT) b_norm2_col_kernel(const KDesc* kd, const int* list, size_t d, int col) {
  const KDesc& P = bprob(kd, list);
  norm2_body(P.V + size_t(col) * d, d, P.partial, blockIdx.x);
}

__global__ void __launch_bounds__(NT) b_reduce_norm_small_kernel(const KDesc* kd, const int* list, unsigned nblk) {
  const KDesc& P = bprob(kd, list);
  reduce_norm_body(P.partial, nblk, P.small);
}

__global__ void b_scale_col_kernel(const KDesc* kd, const int* list, size_t d, int col) {
  const KDesc& P = bprob(kd, list);
  const double a = P.small[1];
  c128* v = P.V + size_t(col) * d;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x) {
    const c128 x = v[i];
    v[i] = mk<double>(x.x * a, x.y * a);
  }
}

__global__ void b_copy_col_kernel(const KDesc* kd, const int* list, size_t d, int from, int to) {
  const KDesc& P = bprob(kd, list);
  const c128* a = P.V + size_t(from) * d;
  c128* b = P.V + size_t(to) * d;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x) b[i] = a[i];
}

// filter input: psi (complex64 or complex128 buffer of the problem) = V[:, j]
template <typename Real>
__global__ void b_cast_in_kernel(const KDesc* kd, const KiDesc<Real>* fd, const int* list, size_t d, int j) {
  const int q = list[blockIdx.y];
  const c128* v = kd[q].V + size_t(j) * d;
  cpx<Real>* out = const_cast<cpx<Real>*>(fd[q].psi);
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x)
    out[i] = mk<Real>(static_cast<Real>(v[i].x), static_cast<Real>(v[i].y));
}

// filter output (complex64 state x) -> w
__global__ void b_cast_out_kernel(const KDesc* kd, const KiDesc<float>* fd, const int* list, size_t d) {
  const int q = list[blockIdx.y];
  const c64* x = fd[q].x;
  c128* w = kd[q].w;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x)
    w[i] = mk<double>(x[i].x, x[i].y);
}

__global__ void __launch_bounds__(64) b_basis_gemm_kernel(const GemmDesc* g) {
  const GemmDesc& G = g[blockIdx.y];
  basis_gemm_mfma_body(G.V, G.ld, G.m, G.Q, G.p, G.Y, G.ld, blockIdx.x);
}

// the 64-row form of the single-problem rotation, one problem per blockIdx.y
template <int MAXT>
__global__ void __launch_bounds__(256) b_basis_gemm64_kernel(const GemmDesc* g) {
  const GemmDesc& G = g[blockIdx.y];
  basis_gemm_mfma64_body<MAXT>(G.V, G.ld, G.m, G.Q, G.p, G.Y, G.ld, blockIdx.x);
}

// Ritz pairs: y = Y[:, i] (not yet normalised), u = U y.
// partial[2b] = sum |y|^2, partial[2b + 1] = sum conj(y) u over block b.
__global__ void __launch_bounds__(NT) r_dots2_kernel(const RDesc* rd, int i, size_t d) {
  __shared__ double red[NT / 64][2 * NCH];
  const RDesc& R = rd[blockIdx.y];
  const c128* y = R.Y + size_t(i) * d;
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blockIdx.x) * NT * RPT + tid;
  double ax[NCH], ay[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) ax[c] = ay[c] = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    if (r < d) {
      const c128 a = y[r], b = R.u[r];
      ax[0] += a.x * a.x + a.y * a.y;
      ax[1] += a.x * b.x + a.y * b.y;
      ay[1] += a.x * b.y - a.y * b.x;
    }
  }
  block_sum_nch(ax, ay, red, tid);
  if (tid < 2) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) {
      sx += red[q][2 * tid];
      sy += red[q][2 * tid + 1];
    }
    R.partial[2 * size_t(blockIdx.x) + tid] = mk<double>(sx, sy);
  }
}

// out[4i..4i+1] = omega = <y|u> / <y|y>, out[4i+3] = 1 / ||y||
__global__ void __launch_bounds__(NT) r_reduce2_kernel(const RDesc* rd, int i, unsigned nblk) {
  __shared__ double red[NT / 64][3];
  const RDesc& R = rd[blockIdx.y];
  const int tid = threadIdx.x;
  double yy = 0.0, ux = 0.0, uy = 0.0;
  for (unsigned b = tid; b < nblk; b += NT) {
    yy += R.partial[2 * size_t(b)].x;
    const c128 v = R.partial[2 * size_t(b) + 1];
    ux += v.x;
    uy += v.y;
  }
  yy = wave_sum(yy);
  ux = wave_sum(ux);
  uy = wave_sum(uy);
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = yy;
    red[tid >> 6][1] = ux;
    red[tid >> 6][2] = uy;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, bx = 0.0, by = 0.0;
    for (int q = 0; q < NT / 64; ++q) {
      a += red[q][0];
      bx += red[q][1];
      by += red[q][2];
    }
    double* o = R.out + 4 * size_t(i);
    o[0] = a > 0.0 ? bx / a : 0.0;
    o[1] = a > 0.0 ? by / a : 0.0;
    o[3] = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
  }
}

// u -= omega y; y /= ||y||; partial[b] = sum |u|^2
__global__ void __launch_bounds__(NT) r_axpy_norm_kernel(const RDesc* rd, int i, size_t d) {
  __shared__ double red[NT / 64];
  const RDesc& R = rd[blockIdx.y];
  c128* y = R.Y + size_t(i) * d;
  const double* o = R.out + 4 * size_t(i);
  const c128 om = mk<double>(o[0], o[1]);
  const double inv = o[3];
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blockIdx.x) * NT * RPT + tid;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    if (r < d) {
      const c128 a = y[r];
      const c128 u = csub(R.u[r], cmul(om, a));
      s += u.x * u.x + u.y * u.y;
      y[r] = mk<double>(a.x * inv, a.y * inv);
    }
  }
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < NT / 64; ++q) tot += red[q];
    R.partial[blockIdx.x] = mk<double>(tot, 0.0);
  }
}

// out[4i+2] = ||U y - omega y|| / ||y||
__global__ void __launch_bounds__(NT) r_reduce_rn_kernel(const RDesc* rd, int i, unsigned nblk) {
  __shared__ double red[NT / 64];
  const RDesc& R = rd[blockIdx.y];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (unsigned b = tid; b < nblk; b += NT) s += R.partial[b].x;
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < NT / 64; ++q) tot += red[q];
    double* o = R.out + 4 * size_t(i);
    o[2] = sqrt(tot) * o[3];
  }
}

// ---------------------------------------------------------------------------
// Block forms (block Krylov-Schur): b vectors W[:, c] = W + c*ldw at once, so
// that V is read once for the whole block.
// ---------------------------------------------------------------------------
// partial[blk*ldp + i*B + c] = sum over the block's rows of conj(V[r, i]) W[r, c]
template <int B>
__global__ void __launch_bounds__(NT) bdots_kernel(const c128* __restrict__ V, size_t ldv, int ncols,
                                                   const c128* __restrict__ W, size_t ldw, size_t d,
                                                   c128* __restrict__ partial, int ldp) {
  constexpr int NCB = NCH / B > 0 ? NCH / B : 1;  // V columns per reduction round
  __shared__ double red[NT / 64][2 * NCH];
  const int tid = threadIdx.x;
  const size_t r0 = static_cast<size_t>(blockIdx.x) * NT * RPT + tid;
  c128 wr[RPT][B];
  bool ok[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    ok[t] = r < d;
#pragma unroll
    for (int c = 0; c < B; ++c) wr[t][c] = ok[t] ? W[size_t(c) * ldw + r] : mk<double>(0, 0);
  }
  for (int i0 = 0; i0 < ncols; i0 += NCB) {
    double ax[NCH], ay[NCH];
#pragma unroll
    for (int q = 0; q < NCH; ++q) ax[q] = ay[q] = 0.0;
#pragma unroll
    for (int u = 0; u < NCB; ++u) {
      if (i0 + u < ncols) {
        const c128* col = V + size_t(i0 + u) * ldv;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          if (ok[t]) {
            const c128 v = col[r0 + size_t(t) * NT];
#pragma unroll
            for (int c = 0; c < B; ++c) {
              ax[u * B + c] += v.x * wr[t][c].x + v.y * wr[t][c].y;
              ay[u * B + c] += v.x * wr[t][c].y - v.y * wr[t][c].x;
            }
          }
        }
      }
    }
    block_sum_nch(ax, ay, red, tid);
    if (tid < NCB * B && i0 + tid / B < ncols) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) {
        sx += red[q][2 * tid];
        sy += red[q][2 * tid + 1];
      }
      partial[size_t(blockIdx.x) * ldp + size_t(i0) * B + tid] = mk<double>(sx, sy);
    }
    __syncthreads();
  }
}

// W[:, c] -= sum_{i < ncols} V[:, i] H[i*B + c]   (H on the device)
template <int B>
__global__ void __launch_bounds__(NT) bupdate_kernel(const c128* __restrict__ V, size_t ldv, int ncols,
                                                     const c128* __restrict__ H, c128* __restrict__ W, size_t ldw,
                                                     size_t d) {
  extern __shared__ c128 hs[];
  const int tid = threadIdx.x;
  for (int i = tid; i < ncols * B; i += NT) hs[i] = H[i];
  __syncthreads();
  const size_t r0 = static_cast<size_t>(blockIdx.x) * NT * RPT + tid;
  c128 acc[RPT][B];
  bool ok[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const size_t r = r0 + size_t(t) * NT;
    ok[t] = r < d;
#pragma unroll
    for (int c = 0; c < B; ++c) acc[t][c] = ok[t] ? W[size_t(c) * ldw + r] : mk<double>(0, 0);
  }
  for (int i = 0; i < ncols; ++i) {
    c128 v[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) v[t] = ok[t] ? V[size_t(i) * ldv + r0 + size_t(t) * NT] : mk<double>(0, 0);
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const c128 hh = hs[i * B + c];
#pragma unroll
      for (int t = 0; t < RPT; ++t) acc[t][c] = csub(acc[t][c], cmul(v[t], hh));
    }
  }
#pragma unroll
  for (int t = 0; t < RPT; ++t)
    if (ok[t]) {
#pragma unroll
      for (int c = 0; c < B; ++c) W[size_t(c) * ldw + r0 + size_t(t) * NT] = acc[t][c];
    }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void random_kernel(c128* __restrict__ v, size_t d, unsigned long long seed) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < d; i += size_t(gridDim.x) * blockDim.x) {
    const uint64_t a = splitmix64(seed * 0x100000001B3ull + 2 * i);
    const uint64_t b = splitmix64(seed * 0x100000001B3ull + 2 * i + 1);
    const double ua = double(a >> 11) * (1.0 / 9007199254740992.0);
    const double ub = double(b >> 11) * (1.0 / 9007199254740992.0);
    v[i] = mk<double>(2.0 * ua - 1.0, 2.0 * ub - 1.0);
  }
}

unsigned grid_for(size_t d) {
  const size_t b = (d + 255) / 256;
  return static_cast<unsigned>(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_dots(const c128* V, size_t ldv, int ncols, const c128* w, size_t d, c128* partial, int ldp,
                       hipStream_t s) {
  hipLaunchKernelGGL(dots_kernel, dim3(row_blocks(d)), dim3(NT), 0, s, V, ldv, ncols, w, d, partial, ldp);
  return hipGetLastError();
}

hipError_t launch_reduce_cols(const c128* partial, int ldp, unsigned nblk, int ncols, c128* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(ncols), dim3(NT), 0, s, partial, ldp, nblk, out);
  return hipGetLastError();
}

hipError_t launch_update(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d, hipStream_t s) {
  hipLaunchKernelGGL((update_kernel<false, false>), dim3(row_blocks(d)), dim3(NT), sizeof(c128) * ncols, s, V, ldv,
                     ncols, h, w, d, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_update_dots(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d,
                              c128* partial, int ldp, hipStream_t s) {
  hipLaunchKernelGGL((update_kernel<true, false>), dim3(row_blocks(d)), dim3(NT), sizeof(c128) * ncols, s, V, ldv,
                     ncols, h, w, d, partial, ldp);
  return hipGetLastError();
}

hipError_t launch_update_norm2(const c128* V, size_t ldv, int ncols, const c128* h, c128* w, size_t d,
                               c128* partial, hipStream_t s) {
  hipLaunchKernelGGL((update_kernel<false, true>), dim3(row_blocks(d)), dim3(NT), sizeof(c128) * ncols, s, V, ldv,
                     ncols, h, w, d, partial, 0);
  return hipGetLastError();
}

hipError_t launch_norm2(const c128* w, size_t d, c128* partial, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel, dim3(row_blocks(d)), dim3(NT), 0, s, w, d, partial);
  return hipGetLastError();
}

hipError_t launch_reduce_norm(const c128* partial, unsigned nblk, double* nrm, hipStream_t s) {
  hipLaunchKernelGGL(reduce_norm_kernel, dim3(1), dim3(NT), 0, s, partial, nblk, nrm);
  return hipGetLastError();
}

hipError_t launch_scale_dev(const c128* in, const double* scale, c128* out, size_t d, hipStream_t s) {
  hipLaunchKernelGGL(scale_dev_kernel, dim3(grid_for(d)), dim3(256), 0, s, in, scale, out, d);
  return hipGetLastError();
}

hipError_t launch_scale_c128(const c128* in, double are, double aim, c128* out, size_t d, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(d)), dim3(256), 0, s, in, are, aim, out, d);
  return hipGetLastError();
}

hipError_t launch_scale_c64(const c64* in, double are, double aim, c64* out, size_t d, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(d)), dim3(256), 0, s, in, are, aim, out, d);
  return hipGetLastError();
}

hipError_t launch_axpy_dev(const c128* a, const c128* x, c128* y, size_t d, hipStream_t s) {
  hipLaunchKernelGGL(axpy_dev_kernel, dim3(grid_for(d)), dim3(256), 0, s, a, x, y, d);
  return hipGetLastError();
}

hipError_t launch_basis_gemm(const c128* V, size_t ldv, int m, const c128* Q, int p, c128* Y, size_t ldy, size_t d,
                             hipStream_t s) {
  if (p <= 256 && d % 64 == 0 && d >= 64) {
    const size_t shmem = size_t(kGemmKc) * p * sizeof(c128);  // <= 32 KB
    const dim3 grid(static_cast<unsigned>(d / 64));
    const int ntile = (p + 15) / 16;
    if (ntile <= 4)
      hipLaunchKernelGGL(basis_gemm_mfma64_kernel<4>, grid, dim3(256), shmem, s, V, ldv, m, Q, p, Y, ldy);
    else if (ntile <= 8)
      hipLaunchKernelGGL(basis_gemm_mfma64_kernel<8>, grid, dim3(256), shmem, s, V, ldv, m, Q, p, Y, ldy);
    else if (ntile <= 12)
      hipLaunchKernelGGL(basis_gemm_mfma64_kernel<12>, grid, dim3(256), shmem, s, V, ldv, m, Q, p, Y, ldy);
    else
      hipLaunchKernelGGL(basis_gemm_mfma64_kernel<16>, grid, dim3(256), shmem, s, V, ldv, m, Q, p, Y, ldy);
    return hipGetLastError();
  }
  if (p <= 256 && d % 16 == 0 && d >= 16) {
    hipLaunchKernelGGL(basis_gemm_mfma_kernel, dim3(static_cast<unsigned>(d / 16)), dim3(64), 0, s, V, ldv, m, Q, p,
                       Y, ldy);
    return hipGetLastError();
  }
  int BR = 64;
  while (BR > 1 && size_t(BR) * m * sizeof(c128) > 65536) BR >>= 1;
  const size_t shmem = size_t(BR) * m * sizeof(c128);
  if (shmem > 65536) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>((d + BR - 1) / BR);
  hipLaunchKernelGGL(basis_gemm_kernel, dim3(grid), dim3(NT), shmem, s, V, ldv, m, Q, p, Y, ldy, d, BR);
  return hipGetLastError();
}

hipError_t launch_gram(const c128* X, size_t si, size_t st, bool conj_in, int n, size_t T, c128* G, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>((n + 15) / 16);
  hipLaunchKernelGGL(gram_kernel, dim3(nb, nb), dim3(256), 0, s, X, si, st, conj_in ? 1 : 0, n, T, G);
  return hipGetLastError();
}

hipError_t launch_random(c128* v, size_t d, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(random_kernel, dim3(grid_for(d)), dim3(256), 0, s, v, d, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launchers
// ---------------------------------------------------------------------------
namespace {
unsigned grid_rows(size_t d) {
  const size_t b = (d + 255) / 256;
  return static_cast<unsigned>(b < 1024 ? (b ? b : 1) : 1024);
}
bool batch_ok(const BatchArgs& a) { return a.kd && a.list && a.n > 0 && a.n <= 65535u; }
}  // namespace

hipError_t launch_b_dots(const BatchArgs& a, int ncols, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_dots_kernel, dim3(a.nblk, a.n), dim3(NT), 0, s, a.kd, a.list, ncols, a.d, a.ldp);
  return hipGetLastError();
}

hipError_t launch_b_reduce_slot(const BatchArgs& a, int ncols, int j, int which, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_reduce_slot_kernel, dim3(ncols, a.n), dim3(NT), 0, s, a.kd, a.list, a.ldp, a.nblk, j,
                     a.slot_doubles, which * (a.ncv + 1));
  return hipGetLastError();
}

hipError_t launch_b_update(const BatchArgs& a, int ncols, int j, int which, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  const size_t sh = sizeof(c128) * ncols;
  if (which == 0)
    hipLaunchKernelGGL((b_update_kernel<true, false>), dim3(a.nblk, a.n), dim3(NT), sh, s, a.kd, a.list, ncols, a.d,
                       a.ldp, j, a.slot_doubles, 0);
  else
    hipLaunchKernelGGL((b_update_kernel<false, true>), dim3(a.nblk, a.n), dim3(NT), sh, s, a.kd, a.list, ncols, a.d,
                       a.ldp, j, a.slot_doubles, a.ncv + 1);
  return hipGetLastError();
}

hipError_t launch_b_reduce_norm(const BatchArgs& a, int j, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_reduce_norm_kernel, dim3(1, a.n), dim3(NT), 0, s, a.kd, a.list, a.nblk, j, a.slot_doubles,
                     4 * (a.ncv + 1));
  return hipGetLastError();
}

hipError_t launch_b_scale_next(const BatchArgs& a, int j, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_scale_next_kernel, dim3(grid_rows(a.d), a.n), dim3(256), 0, s, a.kd, a.list, a.d, j,
                     a.slot_doubles, 4 * (a.ncv + 1));
  return hipGetLastError();
}

hipError_t launch_b_normalize_col(const BatchArgs& a, int col, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_norm2_col_kernel, dim3(a.nblk, a.n), dim3(NT), 0, s, a.kd, a.list, a.d, col);
  hipLaunchKernelGGL(b_reduce_norm_small_kernel, dim3(1, a.n), dim3(NT), 0, s, a.kd, a.list, a.nblk);
  hipLaunchKernelGGL(b_scale_col_kernel, dim3(grid_rows(a.d), a.n), dim3(256), 0, s, a.kd, a.list, a.d, col);
  return hipGetLastError();
}

hipError_t launch_b_copy_col(const BatchArgs& a, int from, int to, hipStream_t s) {
  if (!batch_ok(a)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_copy_col_kernel, dim3(grid_rows(a.d), a.n), dim3(256), 0, s, a.kd, a.list, a.d, from, to);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_b_cast_in(const BatchArgs& a, const KiDesc<Real>* fd, int j, hipStream_t s) {
  if (!batch_ok(a) || !fd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_cast_in_kernel<Real>, dim3(grid_rows(a.d), a.n), dim3(256), 0, s, a.kd, fd, a.list, a.d, j);
  return hipGetLastError();
}
template hipError_t launch_b_cast_in<float>(const BatchArgs&, const KiDesc<float>*, int, hipStream_t);
template hipError_t launch_b_cast_in<double>(const BatchArgs&, const KiDesc<double>*, int, hipStream_t);

hipError_t launch_b_cast_out(const BatchArgs& a, const KiDesc<float>* fd, hipStream_t s) {
  if (!batch_ok(a) || !fd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_cast_out_kernel, dim3(grid_rows(a.d), a.n), dim3(256), 0, s, a.kd, fd, a.list, a.d);
  return hipGetLastError();
}

hipError_t launch_b_basis_gemm(const GemmDesc* g, unsigned n, size_t d, hipStream_t s, int pmax) {
  if (!g || n == 0 || n > 65535u || d % 16 != 0 || d < 16 || pmax < 1 || pmax > 256) return hipErrorInvalidValue;
  if (d % 64 == 0) {
    // 64 rows per workgroup, Q staged in LDS (as launch_basis_gemm)
    const size_t shmem = size_t(kGemmKc) * pmax * sizeof(c128);
    const dim3 grid(static_cast<unsigned>(d / 64), n);
    const int ntile = (pmax + 15) / 16;
    if (ntile <= 4)
      hipLaunchKernelGGL(b_basis_gemm64_kernel<4>, grid, dim3(256), shmem, s, g);
    else if (ntile <= 8)
      hipLaunchKernelGGL(b_basis_gemm64_kernel<8>, grid, dim3(256), shmem, s, g);
    else if (ntile <= 12)
      hipLaunchKernelGGL(b_basis_gemm64_kernel<12>, grid, dim3(256), shmem, s, g);
    else
      hipLaunchKernelGGL(b_basis_gemm64_kernel<16>, grid, dim3(256), shmem, s, g);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(b_basis_gemm_kernel, dim3(static_cast<unsigned>(d / 16), n), dim3(64), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_r_rayleigh(const RDesc* rd, unsigned n, int i, size_t d, hipStream_t s) {
  if (!rd || n == 0 || n > 65535u) return hipErrorInvalidValue;
  const unsigned nblk = row_blocks(d);
  hipLaunchKernelGGL(r_dots2_kernel, dim3(nblk, n), dim3(NT), 0, s, rd, i, d);
  hipLaunchKernelGGL(r_reduce2_kernel, dim3(1, n), dim3(NT), 0, s, rd, i, nblk);
  hipLaunchKernelGGL(r_axpy_norm_kernel, dim3(nblk, n), dim3(NT), 0, s, rd, i, d);
  hipLaunchKernelGGL(r_reduce_rn_kernel, dim3(1, n), dim3(NT), 0, s, rd, i, nblk);
  return hipGetLastError();
}

hipError_t launch_bdots(const c128* V, size_t ldv, int ncols, const c128* W, size_t ldw, int b, size_t d,
                        c128* partial, int ldp, hipStream_t s) {
  const dim3 grid(row_blocks(d));
  switch (b) {
    case 1: hipLaunchKernelGGL(bdots_kernel<1>, grid, dim3(NT), 0, s, V, ldv, ncols, W, ldw, d, partial, ldp); break;
    case 2: hipLaunchKernelGGL(bdots_kernel<2>, grid, dim3(NT), 0, s, V, ldv, ncols, W, ldw, d, partial, ldp); break;
    case 4: hipLaunchKernelGGL(bdots_kernel<4>, grid, dim3(NT), 0, s, V, ldv, ncols, W, ldw, d, partial, ldp); break;
    case 8: hipLaunchKernelGGL(bdots_kernel<8>, grid, dim3(NT), 0, s, V, ldv, ncols, W, ldw, d, partial, ldp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bupdate(const c128* V, size_t ldv, int ncols, const c128* H, c128* W, size_t ldw, int b, size_t d,
                          hipStream_t s) {
  const dim3 grid(row_blocks(d));
  const size_t sh = sizeof(c128) * size_t(ncols) * b;
  if (sh > 65536) return hipErrorInvalidValue;
  switch (b) {
    case 1: hipLaunchKernelGGL(bupdate_kernel<1>, grid, dim3(NT), sh, s, V, ldv, ncols, H, W, ldw, d); break;
    case 2: hipLaunchKernelGGL(bupdate_kernel<2>, grid, dim3(NT), sh, s, V, ldv, ncols, H, W, ldw, d); break;
    case 4: hipLaunchKernelGGL(bupdate_kernel<4>, grid, dim3(NT), sh, s, V, ldv, ncols, H, W, ldw, d); break;
    case 8: hipLaunchKernelGGL(bupdate_kernel<8>, grid, dim3(NT), sh, s, V, ldv, ncols, H, W, ldw, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fq
