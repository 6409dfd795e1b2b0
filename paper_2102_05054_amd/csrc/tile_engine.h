// Register/LDS tile engine for matrix-free passes over a 2^L state on gfx950.
//
// A workgroup of T = 2^TB threads owns a tile of N = 2^n amplitudes,
// n = TB + RB, each thread holding R = 2^RB of them in registers.  Two
// register layouts are used:
//
//   layout A: thread t, register m  <->  tile index j = t + m*T
//             (registers = the top RB tile bits; consecutive lanes hold
//              consecutive tile indices, so global loads/stores coalesce)
//   layout B: thread t, register m  <->  tile index j = t*R + m
//             (registers = the bottom RB tile bits)
//
// A one-qubit operation on tile bit q is done
//   - in registers      if q <  RB   (layout B) or q >= TB (layout A),
//   - by a lane shuffle if RB <= q < 6  (layout A, lane bit q) or
//                         6 <= q < TB (layout B, lane bit q - RB),
// which covers every bit when RB <= 6 and TB <= RB + 6.  Switching layouts is
// one LDS round trip with one padding slot every R entries, so that both the
// A-order writes and the B-order reads (stride R+1) are free of bank
// conflicts.
//
// Tile <-> global index: tile bits [0, c) are global bits [0, c) (a contiguous
// chunk), tile bits [c, n) are global bits [p, p + n - c); the tile id fills
// the remaining global bits, low ones first.
#pragma once

#include "common.h"

namespace fq {

template <int RB>
__device__ __forceinline__ int lds_phys(int j) {
  return RB > 0 ? j + (j >> RB) : j;
}

template <int RB, int TB>
__host__ __device__ constexpr int lds_slots() {
  return RB > 0 ? (1 << (RB + TB)) + (1 << TB) : (1 << TB);
}

struct TileMap {
  uint32_t base;  // global index of tile element 0
  int c, p;

  __device__ __forceinline__ uint32_t g(uint32_t j) const {
    return base | (j & ((1u << c) - 1u)) | ((j >> c) << p);
  }
};

__device__ __forceinline__ TileMap make_tile_map(uint32_t tile, int n, int c, int p) {
  TileMap t;
  const uint32_t low = tile & ((1u << (p - c)) - 1u);
  const uint32_t high = tile >> (p - c);
  t.base = (low << c) | (high << (p + n - c));
  t.c = c;
  t.p = p;
  return t;
}

// Workgroup -> tile order.  Workgroups are dealt round-robin to the eight
// XCDs; giving each XCD a contiguous run of tiles keeps tiles that share
// 128-byte lines (neighbouring chunks) in the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t ntiles) {
  if ((ntiles & 7u) != 0u) return bid;
  return (bid & 7u) * (ntiles >> 3) + (bid >> 3);
}

// Global-memory accesses of amplitudes through address-space-1 pointers.
// Pointers read from a descriptor are generic, and the compiler would emit
// flat accesses, which also count in the LDS/scalar counter (lgkmcnt): every
// LDS wait would then drain the state loads in flight as well.
template <typename Real>
struct gvec2;
template <>
struct gvec2<float> {
  typedef float __attribute__((ext_vector_type(2))) type;
};
template <>
struct gvec2<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};

template <typename Real>
__device__ __forceinline__ cpx<Real> gload(const cpx<Real>* p, uint32_t i) {
  using V = typename gvec2<Real>::type;
  typedef const __attribute__((address_space(1))) V* GP;
  const V v = ((GP)p)[i];  // C-style: reinterpret and address-space cast
  return mk<Real>(v.x, v.y);
}

template <typename Real>
__device__ __forceinline__ void gstore(cpx<Real>* p, uint32_t i, cpx<Real> c) {
  using V = typename gvec2<Real>::type;
  V v;
  v.x = c.x;
  v.y = c.y;
  typedef __attribute__((address_space(1))) V* GP;
  ((GP)p)[i] = v;
}

// Workgroup barrier that orders LDS accesses only: global loads still in
// flight (a prefetch, psi) are not waited for, unlike __syncthreads(), whose
// release fence drains every outstanding memory access.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Layout A <-> B through LDS.  The caller synchronises before reuse.
template <typename Real, int RB, int TB>
__device__ __forceinline__ void a_to_b(cpx<Real> (&v)[1 << RB], cpx<Real>* lds, int tid) {
  if constexpr (RB > 0) {
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) lds[lds_phys<RB>(tid + (m << TB))] = v[m];
    lds_barrier();
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) v[m] = lds[lds_phys<RB>((tid << RB) + m)];
  }
}

template <typename Real, int RB, int TB>
__device__ __forceinline__ void b_to_a(cpx<Real> (&v)[1 << RB], cpx<Real>* lds, int tid) {
  if constexpr (RB > 0) {
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) lds[lds_phys<RB>((tid << RB) + m)] = v[m];
    lds_barrier();
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) v[m] = lds[lds_phys<RB>(tid + (m << TB))];
  }
}

template <typename Real>
__device__ __forceinline__ cpx<Real> shfl_xor_c(cpx<Real> a, int mask) {
  cpx<Real> r;
  r.x = __shfl_xor(a.x, mask);
  r.y = __shfl_xor(a.y, mask);
  return r;
}

}  // namespace fq
