// Pieces of the Krylov-Schur driver shared by the single-problem solver
// (krylov.cpp) and the lockstep batched solver (batched.cpp).
#pragma once

#include <vector>

#include "common.h"
#include "dense.h"

struct floquet_op;

namespace fq {

// Schur form of S = H[0:mm, 0:mm] with the nsort largest |theta| first, the
// coupling b^T Z of the residual row, the Ritz coefficient vectors X (mm x nev)
// and the relative Ritz estimates of the nev wanted pairs (nconv of them
// below tolg, the largest in worst).  Host only; thread-safe.
fq_status analyse_decomposition(const ZMat& H, int mm, int nsort, int nev, double tolg, ZMat* T, ZMat* Z,
                                std::vector<zd>* bz, ZMat* X, int* nconv, double* worst);

// The paper's parameter rule (Sec. 5, caption of Table "bench"): n_cv =
// floor(2^(L/2+1)), at least 2 nev + 1 and below d; k = floor(0.8 2^(L+1) / n_cv),
// at least 1.
int paper_ncv(int L, int nev);
int paper_k(int L, int ncv);

// Options with ncv = 0 / k = 0 (no user polynomial) replaced by the rule
// (ncv also capped at 3000).
fq_arnoldi_opts resolve_auto(const floquet_op* op, int nev, const fq_arnoldi_opts* o);

// Argument checks shared by arnoldi_eigs and arnoldi_eigs_batched.
fq_status validate_arnoldi(const floquet_op* op, int nev, const fq_arnoldi_opts* o);

// Whether convergence checks inside a cycle (every max(4, m/16) steps) are
// worth their host synchronisation and small Schur analysis: when one filter
// application of the batch costs at least 2^24 amplitude updates.  A warm
// started FP64 refinement always checks.
bool probes_pay(size_t d, int k, size_t nprob);

// Schur vectors kept at a restart: p = nev + (m - nev) / 2, within [nev + 1, m - 1].
int keep_count(int m, int nev);

// Unit-modulus coefficients of the FP64 warm start v0 = sum_i c_i y_i.
void warm_start_coefs(unsigned long long seed, int nev, std::vector<c128>* cc);

// Single-problem solve (arnoldi_eigs).
fq_status arnoldi_solve(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* o, double* evals_host,
                        void* evecs_dev, double* resid_host, fq_arnoldi_stats* stats, hipStream_t s);

// Block Krylov-Schur solve (arnoldi_eigs with opts->block in {2, 4, 8});
// the options were validated by the caller.
fq_status block_solve(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* o, double* evals_host,
                      void* evecs_dev, double* resid_host, fq_arnoldi_stats* stats, hipStream_t s);

// Lockstep batched solve (arnoldi_eigs_batched); k_per_op may be NULL.
fq_status arnoldi_batched_solve(floquet_op* const* ops, int n_ops, const double* phis, int n_phi, int nev,
                                const fq_arnoldi_opts* o, const int* k_per_op, double* evals_host,
                                void* const* evecs_dev, double* resid_host, fq_arnoldi_stats* stats,
                                hipStream_t s);
// Graph replay of the lockstep filters (fq_set_graph_capture): 0 or 1.
fq_status set_graph_capture(int on);

}  // namespace fq
