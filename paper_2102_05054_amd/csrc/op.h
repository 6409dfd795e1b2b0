// The floquet_op object and the library-internal operator interface used by
// the Krylov driver.
#pragma once

#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "ki_kernels.h"

namespace fq {

using zd = std::complex<double>;

// Device phase tables of the kicked-Ising diagonal for one target rotation.
struct PhaseTables {
  double phi = 0.0;
  c64* tlo32 = nullptr;
  c64* thi32 = nullptr;
  c128* tlo64 = nullptr;
  c128* thi64 = nullptr;
};

// One tile shape of a multi-pass plan.
struct KiGroup {
  int n, c, p, rb, tb;
  unsigned ntiles;
  unsigned kbits;  // tile bits the kick acts on
};

struct KiPlan {
  bool single = false;
  int rb = 0, tb = 6;  // single-tile shape
  int ngroups = 0;
  KiGroup grp[3];
};

// Brickwork: per-pass gate program (see bw_kernels.h).
struct BwProgram;

// Kicked-Ising tile plans (floquet_api.cpp).
void tile_shape(int n, int* rb, int* tb);
void pass_shape(int n, unsigned ntiles, int* rb, int* tb);
KickMasks masks_for(unsigned kbits, int n, int rb, int tb);
// Kicked bits per layout of the three-layout pass (ki_launch_pass3, tiles of
// n = 4 + tb bits): regA / regB / laneB (B's lane 0) in *ab, layout C's
// register bits in *c.  false when the tile shape has no three-layout form.
bool masks3_for(unsigned kbits, int n, int tb, KickMasks* ab, unsigned* c);
// Phase-table access of the three-layout pass for a tile map (n tile bits,
// chunk c, high run at p) and table split m: 0 when layout C's register bits
// are all below the split and off its two boundary bits (bits 0 and m - 1),
// so that each thread needs one high-table entry; 1 when they are all at or
// above the split (one low-table entry); -1 otherwise (no three-layout form).
int table3_mode(int n, int tb, int c, int p, int m);
void single_shape(int L, int* rb, int* tb);
// Tile plan of a chain of L sites; wide admits the 14-bit complex64 tiles of
// the three-layout pass (direct kick form only).
KiPlan make_plan(int L, bool c64_dt, bool wide);
// Two-group plan with c contiguous bits (the chunk) in the high-bit tiles;
// ngroups = 0 if the tiles would exceed 13 bits.
KiPlan make_plan_chunk(int L, int c);
// Flags the three-layout pass takes: the phase, optionally + psi (with a
// coefficient); not the input scale of the first pass.
inline bool pass3_flags_ok(int flags) {
  return (flags & ~(KI_PREFETCH_PHASE | KI_ADD_PSI | KI_PSI_COEF)) == KI_PHASE;
}
int pass3_shift_host(int tb);
bool single_ok(int L, bool c64_dt);

}  // namespace fq

struct floquet_op {
  fq_model model;
  int L;
  int periodic;
  std::vector<double> J, h;
  double g = 0.0;
  std::vector<fq::zd> gates;  // brickwork / circuit matrices, flat as given
  std::vector<int> gate_sites, gate_widths;  // circuit: first site and width of each gate
  int device = 0;

  // kicked Ising kick form
  bool sw = false;
  double w = 0.0;
  fq::zd site_scale{1.0, 0.0};
  int m = 1;  // phase table split

  std::vector<fq::PhaseTables> tables;  // cache, keyed by phi
  fq::KiPlan plan64, plan128;           // multi-pass plans per dtype
  int single_max_L64 = 10, single_max_L128 = 10;

  // brickwork / circuit device programs (one per dtype), owned; a circuit
  // whose light cone is too wide for one precision's tiles lacks that program
  std::shared_ptr<fq::BwProgram> bw32, bw64;
  std::string bw_missing;  // why a program is missing

  // scratch for the mixed-precision filter and the polynomial coefficients
  void* psi32 = nullptr;
  void* out32 = nullptr;
  double2* coefs_dev = nullptr;
  size_t coefs_cap = 0;

  // apply_filter_many: device descriptors + problem list of the last call
  // (re-uploaded only when the vectors, count, precision or tables change)
  void* many_mem = nullptr;
  size_t many_cap = 0;
  const void* many_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int many_n = 0;
  // ... and the kicked psi of each tile group (2 x n states) for its folded passes
  void* chi_mem = nullptr;
  size_t chi_cap = 0;

  // Krylov workspace (complex128): V (d x ncv_cap+1) and helpers
  void* V = nullptr;
  int ncv_cap = 0;
  void* work = nullptr;      // d complex128
  void* work2 = nullptr;     // d complex128
  double* dev_small = nullptr;  // reduction scratch
  size_t dev_small_cap = 0;
  double* host_small = nullptr; // pinned host mirror
  size_t host_small_cap = 0;

  size_t dim() const { return size_t(1) << L; }
};

namespace fq {

// Library-internal entry points shared by the ABI and the Krylov driver.
fq_status get_tables(floquet_op* op, double phi, const PhaseTables** out);
fq_status apply_U_internal(floquet_op* op, fq_dtype dt, const void* psi, void* out, hipStream_t s);
// out = sum_m coef_m ... : geometric sum if coefs == nullptr (rotation phi),
// otherwise the polynomial with k+1 host coefficients (phi ignored).
fq_status filter_internal(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt,
                          const void* psi, void* out, hipStream_t s);
// FP64 state in, FP64 state out, filter arithmetic in dt (casts around it for c64);
// coefs as for filter_internal.
fq_status filter_mixed(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi64,
                       void* out64, hipStream_t s);
fq_status ensure_scratch32(floquet_op* op);
// out_j = g_k(U) psi_j for n vectors (vector j at offset j*d of psi / out), in dt;
// one launch per Horner pass for all n vectors
fq_status filter_many(floquet_op* op, int k, double phi, fq_dtype dt, int n, const void* psi, void* out,
                      hipStream_t s);
// out = a * psi
fq_status poly_scale_copy(floquet_op* op, zd a, fq_dtype dt, const void* psi, void* out, hipStream_t s);

// brickwork
fq_status bw_create(floquet_op* op);
void bw_destroy(floquet_op* op);
fq_status bw_apply_U(floquet_op* op, fq_dtype dt, const void* psi, void* out, hipStream_t s);
// nvec vectors at stride 2^L, one launch per pass for all of them
fq_status bw_filter(floquet_op* op, int k, double phi, const zd* coefs, fq_dtype dt, const void* psi,
                    void* out, hipStream_t s, int nvec = 1);

}  // namespace fq
