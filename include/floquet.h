/*
 * floquet.h -- C ABI of the MI355X (gfx950) polynomial-filter Floquet
 * eigensolver.
 *
 * The library finds the eigenpairs of a many-qubit Floquet unitary U (one
 * driving period, dimension d = 2^L) whose eigenvalues lie closest to a target
 * e^{i phi} on the unit circle, by running Arnoldi on the geometric-sum filter
 *     g_k(U) = sum_{n=0..k} (e^{-i phi} U)^n            (Sec. 3, Eq. (geo))
 * and recovering omega_n = <n|U|n> with residual ||U|n> - omega_n|n>||
 * (Sec. 4, Eq. (residual)).  U is never stored: it is applied matrix-free.
 *
 * Conventions shared by every entry point
 *  - A state is d = 2^L amplitudes in natural index order, interleaved
 *    complex: complex64 = {float re, im}, complex128 = {double re, im}.
 *  - Site i (1-based) of the chain is bit L-i of the index (site 1 = most
 *    significant bit; the C-order reshaping of Eq. (matvec) and Eq. (ee)).
 *  - Pointers named *_dev are device (HBM) pointers owned by the caller, e.g.
 *    torch tensors' data_ptr(); *_host pointers are host memory owned by the
 *    caller.  The library never frees caller memory.
 *  - hip_stream is a hipStream_t (NULL = the null stream).  apply_U and
 *    apply_filter are asynchronous on that stream; arnoldi_eigs* are
 *    host-driven and return after all their device work has finished.
 *  - No entry point throws.  Every call returns an fq_status; on failure
 *    floquet_last_error() gives a message for the calling thread.
 *  - An op is not thread-safe: one host thread (and one stream) at a time.
 */
#ifndef FLOQUET_H
#define FLOQUET_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct floquet_op floquet_op; /* opaque; owned by the library */

typedef enum {
  FQ_OK = 0,
  FQ_NOT_CONVERGED = 1, /* partial results are valid, see stats.nconv */
  FQ_EINVAL = -1,       /* bad argument (size, pointer, option) */
  FQ_ENOMEM = -2,       /* device or host allocation failed */
  FQ_EDEVICE = -3,      /* a HIP call failed (no device, launch error, ...) */
  FQ_ENUMERIC = -4      /* NaN/Inf, or a Krylov breakdown without an invariant subspace */
} fq_status;

typedef enum { FQ_C64 = 0, FQ_C128 = 1 } fq_dtype;

typedef enum { FQ_KICKED_ISING = 0, FQ_BRICKWORK = 1, FQ_CIRCUIT = 2 } fq_model;

/*
 * Model description (host memory, copied by create_floquet_op).
 *
 * FQ_KICKED_ISING: U = D K with K = prod_i exp(-i g X_i) acting first and
 *   D = diag exp(-i E(s)), E(s) = sum_i J_i z_i z_{i+1} + h_i z_i, z_i = 1-2b_i.
 *   J[L], h[L]: J[i-1] couples sites i, i+1; with periodic != 0 the bond
 *   (L, 1) uses J[L-1], otherwise J[L-1] is ignored.  gates must be NULL.
 *
 * FQ_BRICKWORK: the two-layer brickwork circuit of Sec. 2, Eq. (U) and
 *   Eq. (unitary): U = U_a U_b, U_b acting first.  gates is a flat complex128
 *   array (interleaved re, im) of n_gates = L + 1 matrices: first U_b's gates,
 *   then U_a's, each layer from site 1 to site L.  For even L,
 *     U_b = u_1, u_{2,3}, u_{4,5}, ..., u_{L-2,L-1}, u_L   and
 *     U_a = u_{1,2}, u_{3,4}, ..., u_{L-1,L};
 *   for odd L, U_b = u_1, u_{2,3}, ..., u_{L-1,L} and
 *     U_a = u_{1,2}, ..., u_{L-2,L-1}, u_L.
 *   Two-site gates are row-major 4x4 with local index 2 b_i + b_{i+1};
 *   one-site gates are row-major 2x2.  J, h must be NULL.
 *
 * FQ_CIRCUIT: any local Floquet circuit (the method needs only a local U,
 *   Sec. 2): n_gates gates in the order they act, gate q on the sites
 *   gate_sites[q] (1-based) .. gate_sites[q] + gate_widths[q] - 1, width 1
 *   or 2 (nearest neighbours, open chain); gates holds their matrices back to
 *   back (4 or 16 complex128 entries, same conventions as above).  The U pass
 *   splits the chain into two blocks along the gates' light cone; a circuit
 *   whose light cone is too wide for two blocks of <= 14 (complex64) / 13
 *   (complex128) sites plus a chunk gives FQ_EINVAL (for L > 13).  J, h must
 *   be NULL.  gate_sites and gate_widths are ignored by the other models.
 *
 * L must satisfy 2 <= L <= 30.
 */
typedef struct {
  fq_model model;
  int L;
  int periodic;
  const double* J;
  const double* h;
  double g;
  const double* gates;
  int n_gates;
  const int* gate_sites;   /* FQ_CIRCUIT: n_gates first sites (1-based) */
  const int* gate_widths;  /* FQ_CIRCUIT: n_gates widths (1 or 2) */
} fq_model_desc;

/* Build an operator: copies the model, builds device phase/gate tables.
 * Returns FQ_EINVAL for a bad description, FQ_EDEVICE without a usable GPU. */
fq_status create_floquet_op(const fq_model_desc* desc, floquet_op** out);

/* Frees the op, its tables and its Krylov workspace.  NULL is accepted. */
fq_status destroy_floquet_op(floquet_op* op);

/* d = 2^L of the op (0 for NULL). */
long long floquet_op_dim(const floquet_op* op);

/*
 * out = U psi (Sec. 2; the product the filter is built from).
 * psi_dev, out_dev: d amplitudes of dtype.  In-place (out == psi) is allowed.
 * Asynchronous on hip_stream.
 */
fq_status apply_U(floquet_op* op, fq_dtype dtype, const void* psi_dev, void* out_dev,
                  void* hip_stream);

/*
 * out = g_k(U) psi = sum_{n=0..k} (e^{-i phi} U)^n psi   (Sec. 3, Eq. (geo)),
 * evaluated by the Horner recurrence w <- psi + e^{-i phi} U w, k times from
 * w = psi.  k >= 0; k = 0 copies psi.  out must not alias psi.
 * Asynchronous on hip_stream.
 */
fq_status apply_filter(floquet_op* op, int k, double phi, fq_dtype dtype,
                       const void* psi_dev, void* out_dev, void* hip_stream);

/*
 * out_j = g_k(U) psi_j for n_vec vectors at once (Sec. 3, Eq. (geo); the
 * filter of a block of Krylov vectors, Sec. 4).  psi_dev / out_dev hold n_vec
 * states of dtype back to back (vector j at offset j*d); out must not overlap
 * psi.  Every op advances all vectors in one launch per Horner pass:
 * kicked-Ising ops (L >= 4, k >= 1) with a tile shape picked by a timing
 * autotuner on the first call for each (k, precision, vector-count class),
 * which also writes out; brickwork and circuit ops with their two tile passes
 * over (vector, tile) work items.  Calls on one op must not run
 * concurrently on different streams (the op's launch descriptors are shared).
 * Asynchronous on hip_stream.  FQ_EINVAL for k < 0, non-finite phi, n_vec
 * outside 1..65535 or overlapping buffers.
 */
fq_status apply_filter_many(floquet_op* op, int k, double phi, fq_dtype dtype, int n_vec,
                            const void* psi_dev, void* out_dev, void* hip_stream);

/*
 * apply_filter_many without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same out_j = g_k(U) psi_j for n_vec
 * vectors, for kicked-Ising ops with L >= 4 only.  The launch descriptors and
 * the phase tables for phi live in a fixed 4 MiB file-scope device array of
 * the library (one per GPU, resolved on the first call on each device),
 * refilled by two small kernels on hip_stream at every call; the passes are
 * the plain batched ones with the tile shape the autotuner cached for this
 * (L, precision, k, vector-count class), or the default shape (no timing, no
 * trial launches).  Results agree with apply_filter_many to rounding.
 * The op's device must be current.  Calls that overlap on one GPU (several
 * streams or threads) race on the array.  Asynchronous on hip_stream.
 * FQ_EINVAL for other models, L < 4, k < 0, non-finite phi, n_vec outside
 * 1..64, overlapping buffers or another current device.
 */
fq_status apply_filter_many_noalloc(floquet_op* op, int k, double phi, fq_dtype dtype, int n_vec,
                                    const void* psi_dev, void* out_dev, void* hip_stream);

/*
 * out = sum_{m=0..k} a_m U^m psi, a general polynomial filter (Sec. 3,
 * Eq. (poly)), evaluated by Horner's rule w <- a_{m} psi + U w from w = a_k psi.
 * coeffs_host: k+1 complex128 coefficients a_0..a_k (interleaved re, im).
 * out must not alias psi.  Asynchronous on hip_stream.
 */
fq_status apply_polynomial(floquet_op* op, int k, const double* coeffs_host, fq_dtype dtype,
                           const void* psi_dev, void* out_dev, void* hip_stream);

/* Options of arnoldi_eigs. */
typedef struct {
  int k;                   /* filter order (>= 0).  0 without poly_coeffs: the paper's rule
                              k = floor(0.8 * 2^(L+1) / ncv) for the ncv used (Sec. 5, Table
                              "bench" caption; fq_paper_parameters) */
  int ncv;                 /* Krylov dimension, nev + 2 <= ncv <= min(d, 3000).  0: the paper's
                              rule n_cv = floor(2^(L/2+1)), at least 2 nev + 1, below d, capped
                              at 3000 (arnoldi_eigs only; arnoldi_eigs_batched needs ncv > 0) */
  double tol;              /* residual tolerance on ||U v - omega v|| */
  int max_restarts;        /* Krylov-Schur restarts before FQ_NOT_CONVERGED */
  fq_dtype filter_dtype;   /* FQ_C64: filter in complex64, rest FP64 */
  int refine;              /* with FQ_C64: finish in FP64 until tol is met */
  unsigned long long seed; /* start vector seed when v0_dev is NULL */
  const void* v0_dev;      /* optional complex128 start vector (d), or NULL */
  int refine_k;            /* filter order of the FP64 refinement (0: k) */
  const double* poly_coeffs; /* optional host array of k+1 complex128 a_0..a_k (interleaved re,
                                im): the Arnoldi filter becomes sum_m a_m U^m (Sec. 3, Eq. (poly),
                                e.g. a damped kernel) instead of the geometric sum; the pairs of
                                largest |p(omega)| are returned, ordered by arc distance to phi.
                                NULL: geometric sum.  Needs refine_k = 0 or k. */
  int block;               /* 0 or 1: single-vector Krylov-Schur.  2, 4 or 8: block Krylov-Schur,
                              the space grown by this many filtered vectors per step (one batched
                              filter launch per Horner pass for the block; Sec. 4's method with a
                              block start space).  Needs floor(ncv / block) * block >= nev + 2 *
                              block; arnoldi_eigs only (arnoldi_eigs_batched: FQ_EINVAL). */
} fq_arnoldi_opts;

/* Counters and per-phase wall times (seconds) of one solve. */
typedef struct {
  int nconv;                 /* eigenpairs meeting tol */
  int n_restarts;            /* Krylov-Schur restarts, both phases */
  long long n_filter_apps;   /* g_k(U) applications */
  long long n_U_apps;        /* U applications, filter and residual checks */
  long long n_U_apps_c64;    /* of which in complex64 */
  double t_filter, t_orth, t_restart, t_refine, t_total;
  double max_residual;       /* max over the returned pairs */
} fq_arnoldi_stats;

/*
 * The nev eigenpairs of U closest to e^{i phi} (Sec. 3-4): Krylov-Schur
 * Arnoldi on g_k(U) selecting the largest |lambda| (Sec. 4, Eq. (arnoldi)),
 * then omega_n = <n|U|n> and r_n = ||U|n> - omega_n|n>|| in FP64.
 *
 * evals_host:  2*nev doubles, omega_n interleaved (re, im), sorted by
 *              |arg(omega e^{-i phi})| ascending (Rayleigh quotients, not
 *              renormalised onto the circle).
 * evecs_dev:   d x nev complex128, column-major (vector n at offset n*d),
 *              unit 2-norm, arbitrary phase.  May be NULL.
 * resid_host:  nev doubles r_n.  May be NULL.
 * stats:       may be NULL.
 * The op keeps a d x ncv complex128 workspace between calls (freed by
 * destroy_floquet_op).  Returns FQ_NOT_CONVERGED (results valid for the
 * first stats.nconv pairs) when max_restarts is reached, FQ_ENOMEM when the
 * workspace does not fit, FQ_EINVAL for nev < 1, ncv < nev + 2, ncv > min(d, 3000),
 * k < 0 or tol <= 0, FQ_ENUMERIC for NaN/Inf in the filter output or a Krylov
 * space that becomes invariant with fewer than nev vectors.  A space that
 * becomes invariant with at least nev vectors (ncv = d, or fewer distinct
 * filter values than ncv) is analysed as it stands: its Ritz pairs are exact.
 */
fq_status arnoldi_eigs(floquet_op* op, int nev, double phi, const fq_arnoldi_opts* opts,
                       double* evals_host, void* evecs_dev, double* resid_host,
                       fq_arnoldi_stats* stats, void* hip_stream);

/*
 * Many independent problems in one call (the disorder averages of Sec. 5):
 * every op in ops[0..n_ops) and every target in phis[0..n_phi) (problem
 * p = i*n_phi + j).  Ops may have different L and couplings.
 * k_per_op:   n_ops filter orders (host), or NULL for opts->k everywhere; the
 *             rule of fq_paper_parameters gives one per chain length.
 * evals_host: n_ops*n_phi*2*nev doubles; evecs_dev: n_ops*n_phi pointers (each
 * d_i x nev complex128, or NULL); resid_host: n_ops*n_phi*nev doubles or NULL;
 * stats: n_ops*n_phi entries or NULL.  opts->v0_dev must be NULL (every
 * problem starts from the seeded vector).
 * Kicked-Ising problems (L >= 4, nev and the kept Schur vectors <= 256) of one
 * chain length, kick form and filter order advance in lockstep: one launch
 * per Horner pass and per CGS2 kernel for all of them, the projected
 * matrices analysed on host threads.  Each problem runs the algorithm of
 * arnoldi_eigs; its stats times are those of its batch.  Other problems are
 * solved one after another.  The workspace (about d*(ncv+nev+5)*16 bytes per
 * problem) is allocated per batch and freed before return; batches are split
 * to fit free device memory.  Returns the worst status over problems
 * (FQ_EINVAL also for k_per_op[i] < 1 or a non-NULL opts->v0_dev).
 */
fq_status arnoldi_eigs_batched(floquet_op* const* ops, int n_ops, const double* phis, int n_phi,
                               int nev, const fq_arnoldi_opts* opts, const int* k_per_op,
                               double* evals_host, void* const* evecs_dev, double* resid_host,
                               fq_arnoldi_stats* stats, void* hip_stream);

/*
 * Entanglement entropy S_A = -sum_i s_i^2 ln s_i^2 of n_states complex128
 * states for the cut between sites LA and LA+1 (Sec. 5, Eq. (ee)); s_i are the
 * singular values of the state reshaped as a 2^LA x 2^(L-LA) matrix (site 1 =
 * most significant bit), normalised so that sum s_i^2 = 1.
 * states_dev: n_states x d complex128, state q at offset q*d (e.g. the evecs of
 * arnoldi_eigs).  entropy_host: n_states doubles.  Requires 1 <= LA < L and
 * min(LA, L-LA) <= 11.  Synchronous on hip_stream.
 */
fq_status entanglement_entropy(const floquet_op* op, int LA, const void* states_dev, int n_states,
                               double* entropy_host, void* hip_stream);

/*
 * The paper's parameter rule for large L (Sec. 5 and the caption of Table
 * "bench"): n_cv = floor(2^(L/2 + 1)), raised to at least 2*nev + 1 (Sec. 4:
 * n_cv > 2 n_ev) and lowered to at most 2^L - 1 (a Krylov space of dimension
 * 2^L is the whole space), and k = floor(0.8 * 2^(L+1) / n_cv), the Krylov dimension
 * sitting at 80% of the eigenvalue count on the outer "apple" line of
 * g_k (Sec. 3, last paragraph).  Host-only; returns FQ_EINVAL for L outside
 * [2, 30] or nev < 1.
 */
fq_status fq_paper_parameters(int L, int nev, int* ncv_out, int* k_out);

/*
 * Kernel choice of the batched kicked-Ising passes (arnoldi_eigs_batched,
 * apply_filter_many, block solves), process-wide:
 *   FQ_POLICY_AUTO (0): the autotuner times one-workgroup-per-tile and
 *     persistent pipelined passes and keeps the faster (default);
 *   FQ_POLICY_TILE (1): one workgroup per tile only;
 *   FQ_POLICY_PIPE (2): persistent pipelined passes wherever a tile shape has
 *     them (a workgroup loads its next tile while it works on the current one).
 * All three compute the same arithmetic.  Changing the policy drops the
 * tuner's cached choices.  FQ_EINVAL for other values.  Not thread-safe with
 * concurrent solves.
 */
enum { FQ_POLICY_AUTO = 0, FQ_POLICY_TILE = 1, FQ_POLICY_PIPE = 2 };
fq_status fq_set_kernel_policy(int policy);

/*
 * HIP-graph replay of the lockstep filters of arnoldi_eigs_batched (the
 * batched filter steps of Sec. 5's disorder averages), process-wide:
 *   1 (default): the k + 1 pass launches of a bucket's filter step are
 *     captured once per precision, filter order and range of active problems
 *     into a HIP graph and replayed at every Arnoldi step with that range;
 *     the call then runs on a non-blocking stream of its own, after draining
 *     the caller's stream (it returns when its work is done either way);
 *   0: the passes are launched one by one on the caller's stream.
 * Both compute the same arithmetic in the same order.  FQ_EINVAL for other
 * values.  Not thread-safe with concurrent solves.
 */
fq_status fq_set_graph_capture(int on);

/* Message of the last failing call on this thread ("" if none). */
const char* floquet_last_error(void);

/*
 * Host-only helper exposed for testing the small dense step of the restart:
 * complex Schur form A = Z T Z^H of an n x n complex128 matrix (column-major,
 * interleaved), reordered so that the eigenvalues of largest modulus come
 * first.  a_host is overwritten by T; z_host receives Z (n x n); w_host
 * receives the n eigenvalues (diagonal of T).  Returns FQ_ENUMERIC if the QR
 * iteration does not converge.
 */
fq_status fq_host_schur(int n, double* a_host, double* z_host, double* w_host);

/*
 * Host-only helper exposed for testing the eigenvalue step of
 * entanglement_entropy: ascending eigenvalues of an n x n Hermitian
 * complex128 matrix (row-major, interleaved; overwritten).
 */
fq_status fq_host_eigvalsh(int n, double* a_host, double* w_host);

/*
 * Host-only helper exposed for testing the window schedule of the brickwork
 * and circuit passes (Sec. 2, Eq. (U)): the gates of one pass, in acting
 * order, on a tile of n bits (gate i on tile bits q[i] .. q[i] + w[i] - 1,
 * w[i] = 1 or 2), grouped into windows of wb consecutive tile bits.  A window
 * applies, in acting order, every remaining gate inside it whose earlier
 * gates on shared bits are done (at most eight); the schedule has the fewest
 * windows (breadth-first search; a greedy placement beyond 64 gates), and
 * among those its first and last windows start as high as line_bits.
 * Outputs: *nwin_out windows, window j at bit win_b[j] applying the gates
 * order[win_first[j] .. win_first[j] + win_count[j]); every array holds at
 * least ngates entries.  FQ_EINVAL for bad sizes, a missing array or a gate
 * outside the tile.
 */
fq_status fq_host_bw_schedule(int n, int wb, int ngates, const int* q, const int* w, int line_bits,
                              int* nwin_out, int* win_b, int* win_first, int* win_count, int* order);

#ifdef __cplusplus
}
#endif

#endif /* FLOQUET_H */
