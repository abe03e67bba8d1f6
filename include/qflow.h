/*
 * qflow.h -- C ABI of libqflow, the GPU hot path of singles-and-doubles
 * Quantum Flow (QFlow) with N=1 Trotter downfolding, for AMD Instinct MI355X
 * (gfx950).
 *
 * Conventions shared by every call
 *   - Orbitals are spatial, 0-based, occupied first: O = {0..n_occ-1},
 *     V = {n_occ..n_orb-1} (the index sets of the paper's "Numerical
 *     Implementation" section).  o = n_occ, v = n_orb - n_occ.
 *   - Arrays are row-major FP64 unless stated.  t1 is [o][v] (t_i^a with
 *     a relative to n_occ), t2 is [o][o][v][v] with t2[i][j][a][b] =
 *     t2[j][i][b][a]; they define sigma = T - T^dagger, T = sum t1 E_ai +
 *     1/2 sum t2 E_ai E_bj (the anti-Hermitian operator of Eq. (1)).
 *   - "device" pointers are HIP device memory owned by the caller (for
 *     example a torch tensor's data_ptr()); "host" pointers are ordinary
 *     host memory.  The library never frees caller memory and keeps no
 *     caller pointer after a call returns.
 *   - Calls enqueue work on the context's stream and return; only
 *     qflow_load_integrals and qflow_flow_step synchronise that stream.
 *   - Every call returns a qflow_status.  Argument errors are detected
 *     before any work is enqueued; the message is available from
 *     qflow_last_error.  Device errors surface as QFLOW_E_DEVICE at the next
 *     synchronising call.  Per-space failures never fail a batch: they are
 *     reported in the status arrays.  No call exits, aborts or throws.
 *   - A context is not thread safe; use one context per stream.
 */
#ifndef QFLOW_H
#define QFLOW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qflow_ctx qflow_ctx;

/* One active space (Eq. (3) partition): n_o occupied then n_v virtual
 * absolute orbital indices in orb[], each group ascending.  Supported sizes:
 * (n_o, n_v) = (2,2), (3,3) and (4,4) (36, 400 and 4900 determinants), mixed
 * freely in one list; other sizes give QFLOW_E_UNSUPPORTED, and so does a
 * list whose largest space needs more LDS than the device offers. */
typedef struct {
  int32_t n_o, n_v;
  int32_t orb[8];
} qflow_space;

typedef enum {
  QFLOW_OK = 0,
  QFLOW_E_INVALID_ARG = -1,
  QFLOW_E_SYMMETRY = -2,      /* integrals not real 8-fold symmetric / not finite */
  QFLOW_E_OOM = -3,
  QFLOW_E_DEVICE = -4,
  QFLOW_E_NOT_CONVERGED = -5, /* per-space status: eigensolver hit max_iter */
  QFLOW_E_REF_WEIGHT = -6,    /* per-space status: |c_Phi| < 0.1 */
  QFLOW_E_STATE = -7,         /* call order violated (e.g. no integrals loaded) */
  QFLOW_E_UNSUPPORTED = -8
} qflow_status;

/* Arithmetic of the residual contractions (ladder intermediates). */
typedef enum { QFLOW_FP64 = 0, QFLOW_FP32 = 1, QFLOW_BF16X3 = 2 } qflow_precision;

/* flow_step flags: low 4 bits = qflow_precision (the arithmetic of the ladder
 * and ring contractions: FP64; FP32 operands with FP64 sums; BF16x3 = hi+lo
 * bf16 operands with FP32 partial and FP64 sums). */
enum {
  QFLOW_UNOWNED_FROZEN = 1 << 4, /* amplitudes no space owns keep their value */
  QFLOW_GRAPH = 1 << 5,          /* run the step's device work as a captured HIP graph,
                                    re-captured when K, flags, the array pointers or
                                    the context's buffers change */
  QFLOW_DIIS = 1 << 6,           /* Pulay DIIS on the pool vector [t1 | t2] after the
                                    update: the last 8 (updated pool, change) pairs;
                                    from the third consecutive DIIS step on, the pool
                                    becomes the combination of updated pools whose
                                    changes have the least norm (coefficients summing
                                    to one; Gaussian elimination with partial pivoting,
                                    a pivot below 1e-14 max|B| drops the oldest pair).
                                    A step without the flag, a new space list or new
                                    integrals end the history. */
  QFLOW_SOLVER_VQE = 1 << 7      /* solve the spaces with the UCCSD-VQE solver of
                                    qflow_solve_vqe_batch, each started from the pool's
                                    amplitudes of its orbitals, instead of the CI
                                    eigensolver and its cluster analysis; every space
                                    then writes its optimised parameters (stopping rule:
                                    qflow_set_vqe).  (2,2) and (3,3) spaces only. */
};

/* Create a context on HIP device `device`; hip_stream is a hipStream_t to
 * enqueue on, or NULL for a stream the context creates.  The context also
 * creates a second stream of its own (default priority): outside the
 * stage-timed eager flow step, H_N's ladder and ring contractions and then
 * the J, Lo and Z pieces run there beside Yg's chain, the per-space
 * Hamiltonians' tables beside the residual, and their sigma1 x two-body and
 * occupied-pair ladder parts beside their element terms; all are joined
 * back into the main stream by events
 * before anything reads them, so every call still completes in the main
 * stream's order (and a captured step captures both).  *out is NULL on
 * failure. */
int qflow_create(qflow_ctx** out, int device, void* hip_stream);

/* Release every resource of ctx; NULL is accepted.  Idempotent per pointer. */
int qflow_destroy(qflow_ctx* ctx);

/* Text of the last error on ctx (never NULL; "" if none). */
const char* qflow_last_error(const qflow_ctx* ctx);

/* Load the Hamiltonian H of Eq. (1): h[n][n] (device) and chemist-order
 * two-electron integrals eri[n][n][n][n] = (pq|rs) (device).  Checks that h
 * is symmetric and eri 8-fold symmetric to sym_tol (absolute) and finite
 * (QFLOW_E_SYMMETRY otherwise), then builds the Fock matrix of Phi
 * f_pq = h_pq + sum_k [2(pq|kk) - (pk|kq)], E_ref = sum_k (h_kk + f_kk),
 * eps_p = f_pp, and the device layouts of the integrals.  n_orb <= 128,
 * 1 <= n_occ < n_orb, n_occ <= 64 (QFLOW_E_INVALID_ARG otherwise).
 * Synchronises the stream. */
int qflow_load_integrals(qflow_ctx* ctx, int32_t n_orb, int32_t n_occ, const double* h,
                         const double* eri, double sym_tol);

/* Reference quantities of the loaded Hamiltonian: *e_ref (host), eps[n_orb]
 * (host, may be NULL), fock[n_orb*n_orb] (host, may be NULL). */
int qflow_reference(qflow_ctx* ctx, double* e_ref, double* eps, double* fock);

/* MP2 first-order amplitudes t2 = (ia|jb)/(e_i+e_j-e_a-e_b) and
 * t1 = f_ia/(e_i-e_a) into t1, t2 (device). */
int qflow_mp2_guess(qflow_ctx* ctx, double* t1, double* t2);

/* Global residual of the transformed Hamiltonian
 *   Hbar(sigma) = H + [H_N, sigma]_2 + 1/2 [[F_N, sigma]_2, sigma]_2
 * (the N=1 similarity transform of Eqs. (6)-(7) with every amplitude
 * external, commutators kept to two-body rank):
 *   r1[i][a] = <Phi_i^a|Hbar|Phi>, r2[i][j][a][b] = <Phi_{i alpha j beta}^{a alpha b beta}|Hbar|Phi>,
 *   *e0 = <Phi|Hbar|Phi>.
 * t1, t2, r1, r2, e0 are device pointers; precision selects the arithmetic
 * of the ladder contractions. */
int qflow_residual(qflow_ctx* ctx, const double* t1, const double* t2, double* r1, double* r2,
                   double* e0, int precision);

/* Number of doubles the CAS-form Hamiltonian of one space occupies:
 * 1 + na^2 + na^4 with na = n_o + n_v. */
int64_t qflow_heff_size(const qflow_space* space);

/* Downfolded Hamiltonian of every space (Eq. (6) at N=1, G = exp(sigma_ext),
 * sigma_ext = sigma minus the amplitudes whose indices all lie in the space,
 * Eq. (3)), restricted to the space's orbitals and written relative to the
 * empty active space: at heff + heff_off[k] (device buffer; heff_off host,
 * K+1 entries, each block qflow_heff_size long) the layout is
 *   [Ec, h[na][na], g[na][na][na][na]] with g in chemist order (pq|rs),
 * local orbital order = spaces[k].orb.  spaces is a host array. */
int qflow_build_heff(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const double* t1,
                     const double* t2, double* heff, const int64_t* heff_off, int precision);

/* Number of doubles of the local amplitudes of one space:
 * n_o*n_v + (n_o*n_v)^2. */
int64_t qflow_amp_size(const qflow_space* space);

/* Number of doubles of one space's CI vector: C(na, n_o)^2 (determinants
 * with n_o alpha and n_o beta electrons in the space's na orbitals). */
int64_t qflow_ci_size(const qflow_space* space);

/* Lowest eigenpair of every space's CAS matrix (determinants with n_o alpha
 * and n_o beta electrons in the space's orbitals: the span of P + Q_int of
 * Eq. (6)), by Davidson iteration in FP64.  Outputs (device): energy[K] (the
 * E(i) of Eq. (5), eigenvalue reading), c0[K] (reference coefficient of the
 * normalised eigenvector, made >= 0), amp + amp_off[k] (amp_off host, K+1
 * entries): the intermediate-normalised cluster amplitudes t1[n_o][n_v] then
 * t2[n_o][n_o][n_v][n_v] (local indices; t2[i][j][a][b] pairs i,a alpha with
 * j,b beta), iters[K], status[K] (QFLOW_OK, QFLOW_E_NOT_CONVERGED,
 * QFLOW_E_REF_WEIGHT).  Converged when the residual norm of the normalised
 * Ritz vector is < tol.
 * ci_warm (device, may be NULL) with ci_off (host, K+1 entries, blocks of
 * qflow_ci_size): in, a start vector per space (all zeros: start from the
 * reference determinant); out, the normalised eigenvector with c0 >= 0,
 * determinants ordered alpha string major, strings lexicographic. */
int qflow_solve_active_batch(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                             const double* heff, const int64_t* heff_off, double* energy,
                             double* c0, double* amp, const int64_t* amp_off, double* ci_warm,
                             const int64_t* ci_off, int32_t* iters, int32_t* status, double tol,
                             int32_t max_iter);

/* The paper's own active-space solver ("Numerical Implementation"): per
 * space, the UCCSD parameters theta of sigma_int = T - T^dagger (the space's
 * spin-adapted singles t1[I][A] and doubles t2[I][J][A][B] = t2[J][I][B][A],
 * T = sum t1 E_AI + 1/2 sum t2 E_AI E_BJ with spin-summed excitation
 * operators, local indices) minimising the energy of Eq. (5) for the trial
 * state e^{sigma_int} |Phi> of Eq. (8) at N = 1:
 *   E(theta) = <Phi| e^{-sigma_int} H_eff e^{sigma_int} |Phi>,
 * evaluated exactly in the space's determinant basis (the CAS matrix of
 * qflow_solve_active_batch) in FP64: e^{sigma_int} applied by its Taylor
 * series to 1e-17 relative, the exact gradient by 8-point Gauss-Legendre
 * quadrature of the exponential's Frechet derivative, minimised by BFGS
 * with an Armijo line search from the diagonal inverse Hessian
 * 1 / (4 max(d, 0.05)) (d: excitation energy of the parameter's determinant)
 * until the largest gradient entry is below gtol.
 * heff, heff_off as for qflow_solve_active_batch.  theta0 (device): the start
 * parameters in the amp layout (t1[n_o][n_v] then t2[n_o][n_o][n_v][n_v] per
 * space at amp_off[k], host offsets, K+1 entries; t2 must be pair
 * symmetric: the (I,A) <= (J,B) entry of each pair is read).  Outputs
 * (device): amp (the optimised parameters, same layout, both entries of every
 * pair; may be theta0 itself), energy[K] (E(theta)), iters[K] (BFGS
 * iterations), status[K] (QFLOW_OK, or QFLOW_E_NOT_CONVERGED after max_iter
 * iterations; max_iter = 0 only evaluates E(theta0)).  (2,2) and (3,3) spaces
 * only (a (4,4) space's workgroup would need 1.6 MB of LDS):
 * QFLOW_E_UNSUPPORTED otherwise.  Synchronises the stream. */
int qflow_solve_vqe_batch(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                          const double* heff, const int64_t* heff_off, const double* theta0,
                          double* amp, const int64_t* amp_off, double* energy, int32_t* iters,
                          int32_t* status, double gtol, int32_t max_iter);

/* Truncation of the downfolded Hamiltonian of Eq. (6) at N = 1 used by
 * qflow_residual, qflow_build_heff, qflow_flow_step and qflow_autotune:
 *   QFLOW_TRUNC_F (default)  H + [H_N, s]_2 + 1/2 [[F_N, s]_2, s]_2,
 *   QFLOW_TRUNC_H            the same + 1/2 [[V_N, s]_2, s]_2 (V_N the
 *                            two-body part of H_N), the next term of the
 *                            expansion (closing paragraph of "Results"),
 * s = sigma_ext of the space (sigma for the residual); every commutator is
 * truncated to its 0-, 1- and 2-body parts, the inner one before the outer
 * one is taken.  QFLOW_TRUNC_H evaluates its term directly, with no global
 * intermediates: [V_N, sigma]_2 over all n^4 elements once per call, then per
 * space its own W = [V_N, s]_2 (n^4 doubles, up to 4 GiB of spaces at a time)
 * and [W, s]_2 on the space's orbitals, a cost of order n^4 (o^2 + v^2 + o v)
 * + K n^4 + K na^4 n^2 operations: a path for problems of tens of orbitals.
 * It takes at most 64 orbitals: QFLOW_E_UNSUPPORTED here (integrals
 * loaded) or at the first call that would use it (integrals loaded later).
 * Windowed sweeps take QFLOW_TRUNC_F only.  Unknown values are
 * QFLOW_E_INVALID_ARG. */
enum { QFLOW_TRUNC_F = 0, QFLOW_TRUNC_H = 1 };
int qflow_set_truncation(qflow_ctx* ctx, int truncation);

/* Stopping rule of the VQE solves inside qflow_flow_step (QFLOW_SOLVER_VQE):
 * largest gradient entry below gtol, at most max_iter BFGS iterations (the
 * space then has status QFLOW_E_NOT_CONVERGED and writes none of its
 * amplitudes).  Defaults: 1e-10, 500.  gtol <= 0 or max_iter < 0 is
 * QFLOW_E_INVALID_ARG. */
int qflow_set_vqe(qflow_ctx* ctx, double gtol, int32_t max_iter);

/* Bytes of device memory qflow_solve_active_batch_static may use: 128 MiB,
 * held by every device the library runs on from its first context until the
 * process ends. */
#define QFLOW_STATIC_SCRATCH_BYTES (128u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as qflow_solve_active_batch, with the same arguments, results and
 * errors, that allocates nothing.  Its space records, class lists, offsets,
 * work counter and Davidson work areas live in one file-scope device array of
 * QFLOW_STATIC_SCRATCH_BYTES; the library resolves that array's address on
 * each device once, at qflow_create.  It follows the context's Davidson
 * schedule (qflow_set_tuning), so its results equal those of
 * qflow_solve_active_batch bit for bit.  A batch needs 256-byte-aligned
 * sections of 256 bytes (the persistent launch's work counter), 40 K
 * (records), 4 K (class lists) and 4 x 8 (K + 1) (offsets) bytes, plus
 * 8 x 24 H bytes of work per space whose CI vectors have H = ns (ns + 1) / 2
 * spin-flip symmetric entries (ns strings per spin; 8 x 27 H for the (4,4)
 * class): about 40 KB per (3,3) space, so at most about 3,300 (3,3), 33,000
 * (2,2) or 249 (4,4) spaces per call; a larger batch returns
 * QFLOW_E_UNSUPPORTED before any work is enqueued.  The work areas need no
 * initial contents; the counter is reset by a kernel on the stream.  Every
 * call on one device shares that device's array and overwrites it: calls
 * that overlap on one device (several contexts or streams, or threads) race
 * and must be serialised by the caller.  The call copies the records from
 * host memory and synchronises the stream. */
int qflow_solve_active_batch_static(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                                    const double* heff, const int64_t* heff_off, double* energy,
                                    double* c0, double* amp, const int64_t* amp_off,
                                    double* ci_warm, const int64_t* ci_off, int32_t* iters,
                                    int32_t* status, double tol, int32_t max_iter);

/* One QFlow macro-iteration ("Numerical Implementation": the process groups
 * downfold and solve their spaces, write the optimised amplitudes back into
 * the global pool, each excitation being written by the first space in
 * energy order that reaches it, and meet at a barrier at the end of each
 * sweep).  Here the sweep is a Jacobi sweep: every space reads the pool as it
 * was on entry, then the pool is updated once, as at that barrier:
 *   1. build every space's downfolded Hamiltonian from (t1, t2),
 *   2. solve every space,
 *   3. write each amplitude from the space that owns it (owner1[o][v],
 *      owner2[o][o][v][v] device int32 arrays, -1 = unowned, owner2
 *      pair-symmetric); spaces whose status is not QFLOW_OK leave their
 *      amplitudes unchanged,
 *   4. unowned amplitudes take t <- t - R/Delta (Delta = eps_a - eps_i,
 *      eps_a + eps_b - eps_i - eps_j) unless QFLOW_UNOWNED_FROZEN.
 * The context keeps each space's eigenvector and starts the next flow step's
 * solve of that space from it while the space list stays the same; a new
 * list starts every solve from the reference determinant.
 * t1, t2 (device) are updated in place.  energy[K] (device) receives E(i);
 * *e_mean (host) = mean_i E(i), *max_dt (host) = max |t_new - t_old|.
 * Synchronises the stream. */
int qflow_flow_step(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const int32_t* owner1,
                    const int32_t* owner2, double* t1, double* t2, double* energy, double* e_mean,
                    double* max_dt, int32_t flags);

/* One windowed Gauss-Seidel sweep (the process groups of the paper's
 * parallel implementation take spaces in Delta-eps order and update the pool
 * as they finish): the spaces, in the given order, are taken in consecutive
 * windows of `window` spaces; for each window the downfolded Hamiltonians
 * are built from the pool as it stands, the window's spaces are solved, and
 * the amplitudes they own are written into t1, t2 before the next window.
 * Amplitudes no space owns take t <- t - R/Delta with R from the pool at the
 * start of the sweep (unless QFLOW_UNOWNED_FROZEN), so window >= K gives the
 * same result as qflow_flow_step.  Arguments as for qflow_flow_step; flags:
 * precision and QFLOW_UNOWNED_FROZEN (QFLOW_GRAPH and QFLOW_DIIS are
 * rejected with QFLOW_E_UNSUPPORTED); window < 1 is QFLOW_E_INVALID_ARG.
 * Each window recomputes every global intermediate, so a sweep costs about
 * ceil(K / window) times the global part of a flow step.  *max_dt = max
 * |t_end - t_start|.  Synchronises the stream. */
int qflow_flow_sweep_windowed(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                              const int32_t* owner1, const int32_t* owner2, double* t1,
                              double* t2, double* energy, int32_t window, double* e_mean,
                              double* max_dt, int32_t flags);

/* Per-space results of the eigensolves of the last qflow_flow_step (or
 * windowed sweep) on ctx: iters[K] (Davidson iterations) and status[K]
 * (QFLOW_OK, QFLOW_E_NOT_CONVERGED, QFLOW_E_REF_WEIGHT), host arrays, either
 * may be NULL.  K must be the length of that step's space list.
 * Synchronises the stream. */
int qflow_last_solve(qflow_ctx* ctx, int32_t K, int32_t* iters, int32_t* status);

/* Stopping rule of the eigensolves inside qflow_flow_step and
 * qflow_flow_sweep_windowed: a space's Davidson iteration stops when the
 * residual norm of its normalised Ritz vector falls below tol, or after
 * max_iter iterations with per-space status QFLOW_E_NOT_CONVERGED (that space
 * then writes none of its amplitudes in that step).  Defaults: 1e-10, 200.
 * tol <= 0 or max_iter < 1 is QFLOW_E_INVALID_ARG. */
int qflow_set_solver(qflow_ctx* ctx, double tol, int32_t max_iter);

/* Launch choices of a context (each changes only the schedule, never the
 * arithmetic beyond the summation order of split products):
 *   davidson      QFLOW_DAV_PER_CLASS: one launch per size class, a workgroup
 *                 per space; QFLOW_DAV_PERSISTENT: one persistent launch over
 *                 every size class, as many workgroups as fit taking spaces from
 *                 a shared counter, the costliest class first;
 *   split_target  matrix-core products split K until about split_target
 *                 workgroups per compute unit are available (1..16);
 *   f64_tile      FP64 products: 0 = the tile that pads the columns less,
 *                 1 = 128 x 96, 2 = 128 x 128;
 *   z_mode        as qflow_set_z_mode;
 *   block_44      threads per (4,4) space in per-class launches: 512 or 1024.
 * Defaults: QFLOW_DAV_PER_CLASS, 4, 0, QFLOW_Z_AUTO, 512. */
enum { QFLOW_DAV_PER_CLASS = 0, QFLOW_DAV_PERSISTENT = 1 };
typedef struct {
  int32_t davidson, split_target, f64_tile, z_mode, block_44;
} qflow_tuning;

/* Set (QFLOW_E_INVALID_ARG for a value out of range) or read the context's
 * launch choices.  A flow step captured as a graph is captured again after a
 * change. */
int qflow_set_tuning(qflow_ctx* ctx, const qflow_tuning* tuning);
int qflow_get_tuning(const qflow_ctx* ctx, qflow_tuning* tuning);

/* Autotuner: choose the launch choices for this problem (loaded integrals,
 * the space list, the flags' precision and QFLOW_GRAPH) by timing flow steps.
 * Starting from the current choices it varies one choice at a time
 * (davidson, split_target in {2, 4, 8}, f64_tile in {0, 1, 2} on the FP64
 * path, z_mode in {QFLOW_Z_SPACE, QFLOW_Z_DENSE}, block_44 in {512, 1024}
 * when the list holds (4,4) spaces) and keeps a change when it
 * lowers the device time of three flow steps (HIP events, after one untimed
 * step), each candidate starting from the same pool (copies of t1, t2, device;
 * the caller's arrays are not changed) with cold eigensolver starts.
 * QFLOW_DIIS is ignored while timing.  The result is applied to ctx and
 * written to *out (may be NULL).  cache_path (may be NULL): a JSON object
 * file, one entry per line, keyed by the orbital counts, the size-class
 * counts, the precision and graph flag and the device's architecture name;
 * an existing entry is applied without timing, a new one is added.  report
 * (host, may be NULL): the timed candidates as text, NUL-terminated within
 * report_len bytes.  Afterwards the next flow step starts its eigensolves
 * from the reference determinant and a new DIIS history.  Synchronises the
 * stream. */
int qflow_autotune(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const int32_t* owner1,
                   const int32_t* owner2, const double* t1, const double* t2, int32_t flags,
                   const char* cache_path, qflow_tuning* out, char* report, int32_t report_len);

/* Per-stage device times of the last qflow_flow_step in milliseconds (HIP
 * events on the context's stream), in the order: [F,sigma] intermediate,
 * ladder contraction of H_N, ladder contraction of [F,sigma], ring operand
 * packing, ring contractions (four matrix-core GEMMs), one-body ring terms,
 * sigma1 applied to the two-body parts (the residual's pieces), residual,
 * build_heff (with the dense Z when that form is taken), solve, update,
 * then the whole step.  A step run with QFLOW_GRAPH reports -1 for the
 * stages and only the whole.  n is the capacity of ms (host).  Returns the
 * count written (at most 12). */
int qflow_last_timings(const qflow_ctx* ctx, float* ms, int n);

/* How the downfolded Hamiltonians get the terms where sigma's one-body part
 * meets a two-body operator, Z = sigma1 X over the first index with
 * X = H_N + Yg/2 (the [X_2, sigma_1] part of the commutators of Eq. (6)):
 *   QFLOW_Z_AUTO   per call, the form that moves fewer bytes (default);
 *   QFLOW_Z_SPACE  per space, from the rows of H_N and Yg the space touches;
 *   QFLOW_Z_DENSE  one dense Z per build (n^4 doubles of device memory,
 *                  allocated by this call or the next one given spaces); this
 *                  form also takes the occupied-pair ladders of the same
 *                  commutators, sum_{t,u occ} X_pqtu t2[t,u,r,s], as one
 *                  table over all pairs p <= q (n(n+1)/2 (o^2 + v^2) doubles).
 * The forms agree to rounding.  Another mode is QFLOW_E_INVALID_ARG; a flow
 * step captured as a graph is captured again after a change. */
typedef enum { QFLOW_Z_AUTO = 0, QFLOW_Z_SPACE = 1, QFLOW_Z_DENSE = 2 } qflow_z_mode;
int qflow_set_z_mode(qflow_ctx* ctx, int mode);

/* Algorithm 1 (coverage-driven active-space sampling), host only.
 * Draws (Otilde, Vtilde) of sizes (no, nv) from {0..No-1} and
 * {No..No+Nv-1} without replacement by partial Fisher-Yates shuffles driven
 * by the uniforms u[0..n_u) (one per swap), discards candidates that cover
 * no remaining (o1<o2, v1<v2) tuple, stops when every tuple is covered or
 * after `cap` accepted spaces (cap <= 0: no cap), and sorts the result by
 * Delta eps = sum eps_v - sum eps_o ascending (stable; ties by orbital
 * lists).  eps: host, No+Nv entries.  out: host, capacity `max_out`.
 * *K_out = spaces written, *used = uniforms consumed.  QFLOW_E_INVALID_ARG
 * if the uniforms or the output capacity run out. */
int qflow_sample_spaces(int32_t No, int32_t Nv, int32_t no, int32_t nv, const double* eps,
                        const double* u, int64_t n_u, int32_t cap, qflow_space* out,
                        double* delta_eps, int32_t max_out, int32_t* K_out, int64_t* used);

/* Ownership (host; "Numerical Implementation", the assignment of each
 * excitation to the first active space, in the Delta-eps order of
 * Algorithm 1, that can reach it, so that every amplitude is written once per
 * sweep): owner1[i][a], owner2[i][j][a][b] = index of the first space in list
 * order that reaches the amplitude, or -1.  owner2 is keyed on the spatial
 * pair, owner2[i][j][a][b] = owner2[j][i][b][a].  owner1 holds No*Nv and
 * owner2 No*No*Nv*Nv int32 (host, caller-owned).  A space with n_o or n_v
 * below 1, more than 8 orbitals, or an orbital outside its block gives
 * QFLOW_E_INVALID_ARG (the arrays are then partly written). */
int qflow_build_owners(int32_t No, int32_t Nv, int32_t K, const qflow_space* spaces,
                       int32_t* owner1, int32_t* owner2);

#ifdef __cplusplus
}
#endif

#endif /* QFLOW_H */
