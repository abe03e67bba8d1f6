// Launch wrappers of the libqflow kernels (all enqueue on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qflow_cas.h"

namespace qf {

struct SpaceDev {            // device copy of one active space
  int na, nocc;
  int orb[8];
};

// integral preparation
void launch_sym_check(const double* h, const double* eri, int n, double* partial, int nblocks,
                      hipStream_t st);
void launch_fock(const double* h, const double* eri, int n, int o, double* f, hipStream_t st);
void launch_repack(const double* eri, int n, int o, double* V, double* W, hipStream_t st);
void launch_mp2(const double* f, const double* V, int n, int o, double* t1, double* t2,
                hipStream_t st);

// intermediates of one amplitude set
// U = [G, sigma_2]_2 (dense n^4) for a Hermitian one-body G, and its
// virtual-virtual rows in ladder layout into wv (FP64), wv32 (FP32) or the
// BF16 hi/lo planes wvb_hi / wvb_lo (rows padded to bf16_pad(v*v), padding
// zeroed by the caller) when one is given (k_prep.hip).  With U NULL only
// the compact parts P and Q are formed (read through Sigma2Lazy).  Scratch:
// A12 2*n*v + n*o, t2T 3*o*o*v*v (packed from t2 here when pack_t2),
// P 4*n*o*o*v and Q 2*n*o*v*v doubles.
void launch_sigma2(const double* g, const double* t2, int n, int o, double* A12, double* t2T,
                   bool pack_t2, double* P, double* Q, double* part, size_t part_cap, double* U,
                   double* wv, float* wv32, __bf16* wvb_hi, __bf16* wvb_lo, hipStream_t st);
// y1 = one-body part of [F_N, sigma], scal[2] = its scalar part
void launch_yg1(const double* f, const double* t1, const double* t2, int n, int o, double* y1,
                double* scal, hipStream_t st);
void launch_fill(double* x, size_t count, double value, hipStream_t st);
void launch_copy(const double* src, double* dst, size_t count, hipStream_t st);
// ring intermediates (layouts in qflow_eval.h, DenseOp)
void launch_pack_ring_A(const double* X, int n, int o, double* Aa, double* A22, hipStream_t st);
void launch_pack_ring_T(const double* t2, int o, int v, double* Ta, double* T22, hipStream_t st);
// the same operands rounded to FP32 (mixed-precision contractions)
void launch_pack_ring_A(const double* X, int n, int o, float* Aa, float* A22, hipStream_t st);
void launch_pack_ring_T(const double* t2, int o, int v, float* Ta, float* T22, hipStream_t st);
// ... and as BF16 hi/lo planes, rows padded to bf16_pad(2ov) and bf16_pad(ov)
// (padding zeroed by the caller once)
void launch_pack_ring_A_bf16(const double* X, int n, int o, __bf16* Ah, __bf16* Al, __bf16* A22h,
                             __bf16* A22l, hipStream_t st);
void launch_pack_ring_T_bf16(const double* t2, int o, int v, __bf16* Th, __bf16* Tl, __bf16* T22h,
                             __bf16* T22l, hipStream_t st);
// The sigma1 x two-body pieces of H_N + Yg/2 that the residual needs
// (k_residual.hip, k_zv / k_zo): zv [v][v][o][o], zo [o][o][v][v].
// Dense Z = sigma1 (Xh + Xy/2) over the first index, n^4 doubles (k_prep.hip,
// k_sigma1_x).
void launch_sigma1_x(const double* Xh, const double* Xy, const double* t1, int n, int o,
                     double* Z, hipStream_t st);
void launch_z_vvoo(const double* Xh, const double* Xy, const double* t1, int n, int o, double* zv,
                   double* zo, hipStream_t st);
// operands of the occupied-occupied ladder Lo (k_prep.hip)
void launch_pack_t2_vvoo(const double* t2, int o, int v, double* T, hipStream_t st);
void launch_pack_x_oooo(const double* X, int n, int o, double* Xo, hipStream_t st);
// one-body ring operands (layouts in k_prep.hip, k_pack_j_A / k_pack_j_B)
void launch_pack_j_A(const double* X, int n, int o, double* A1, double* A2, hipStream_t st);
void launch_pack_j_B(const double* t2, int o, int v, double* B1, double* B2, hipStream_t st);
// C[M][N] = scale * sum_k A[m][k] B[n][k] on the FP64 matrix cores.  When
// the tile grid alone cannot fill the chip the K range is split; each split
// writes its own M*N slice of `part` (capacity part_cap doubles, may be NULL
// for no split) and the slices are summed in a fixed order, so the result is
// deterministic.
constexpr int kMaxSplits = 128;
// Launch choices of the matrix-core products (set by the context before it
// enqueues them): K is split until about split_target workgroups per compute
// unit are available; f64_tile picks the FP64 tile (0: the one that pads N
// less, 1: 128 x 96, 2: 128 x 128).
struct GemmTuning {
  int split_target = 4;
  int f64_tile = 0;
};
void set_gemm_tuning(const GemmTuning& t);
// nb (1..4) products C[b] = scale A[b] B[b]^T of one shape in one launch
// (host arrays of device pointers); -1 for another nb.
int launch_gemm_nt_f64_batch(const double* const* A, const double* const* B, double* const* C,
                             int nb, int M, int N, int K, double scale, double* part,
                             size_t part_cap, hipStream_t st);
void launch_gemm_nt_f64(const double* A, const double* B, double* C, int M, int N, int K,
                        double scale, double* part, size_t part_cap, hipStream_t st);
// The same with FP32 operands on the FP32 matrix cores: products summed in
// FP32 over 64 consecutive k, those partial sums accumulated in FP64.
void launch_gemm_nt_f32(const float* A, const float* B, double* C, int M, int N, int K,
                        double scale, double* part, size_t part_cap, hipStream_t st);
void launch_cvt_f32(const double* src, float* dst, size_t count, hipStream_t st);
// The same with BF16x3 operands (x = hi + lo, both bf16, rows of Kp = a
// multiple of 32 k, zero padded) on the BF16 matrix cores: lo*hi + hi*lo +
// hi*hi in FP32 per 32 k, FP64 sums every 64 k.
inline int bf16_pad(int K) { return (K + 31) / 32 * 32; }
void launch_gemm_nt_bf16x3(const __bf16* Ah, const __bf16* Al, const __bf16* Bh, const __bf16* Bl,
                           double* C, int M, int N, int Kp, double scale, double* part,
                           size_t part_cap, hipStream_t st);
void launch_split_bf16(const double* src, int rows, int K, int Kp, __bf16* hi, __bf16* lo,
                       hipStream_t st);

// residual of Hbar(sigma)
struct RingOps {            // global intermediates of H_N and of Yg
  const double *ga_h, *g22_h, *j1_h, *j2_h, *ga_y, *g22_y, *j1_y, *j2_y;
  const double *zv, *zo;     // [v][v][o][o], [o][o][v][v]: sigma1 x two-body pieces (residual)
  const double *u_h;         // [x1, sigma_2]_2 of H_N (= two-body of Yg), dense
  const double *s2p, *s2q;   // compact parts of [y1, sigma_2]_2 (Sigma2Lazy)
  const double *c1_h, *c1_y; // [n][n] one-body parts of [H_N, sigma] and [Yg, sigma]
  const double *lo_h, *lo_y; // [v*v][o*o] occupied-occupied ladders
  const double *pf;          // compact parts P1..P4 of [F, sigma_2] (launch_sigma2)
  const double *qf;          // compact parts Q1, Q2 of [F, sigma_2] (launch_sigma2)
};
// One-body parts of [H_N, sigma] and [Yg, sigma] for every (p,q) into
// c1h, c1y ([n][n] each; the buffers RingOps.c1_h / c1_y point to), then the
// residual r1, r2 and the zero-body parts (scal[0], scal[1], e0).  part:
// scratch of 2*ceil(v/8)*n*n doubles.
void launch_residual(const double* f, const double* V, const double* y1, const double* y2,
                     const double* L, const double* LY, const RingOps& rings, const double* t1,
                     const double* t2, int n, int o, double* scal, double* c1h, double* c1y,
                     double* part, double* r1, double* r2, double* e0, hipStream_t st);

// per-space downfolded Hamiltonians in CAS form
// The per-element kernels run one launch per size class (cls_idx / cls_off
// as for launch_davidson; task_slots[c] = task count of class c,
// task_slots[3 + c] = the slots of its two-body elements, which come first); K = the
// number of spaces in the lists (cls_off[3]).  zc: the dense
// Z = sigma1 (H_N + Yg/2) (launch_sigma1_x), read by the element kernels; when
// NULL, k_heff_z adds that part per space from the rows of H_N and Yg.
// mpd: the dense occupied-pair ladder table (launch_pack_x_pairs), or NULL
// for the per-space form.  fs1: scratch of 2 n^2 doubles.  zs (or NULL):
// sum over the classes of count_c * na_c^4 doubles; with it the per-space
// sigma1 x two-body and occupied-pair ladder kernels write into zs, which
// the CAS rewrite adds, and with st2 (or NULL) they run there (forked from
// st by fork_ev, joined back by join_ev before the CAS rewrite).  phase:
// 0 launches only fs1 and the per-space tables (which read prepare's
// outputs, not the residual's), 1 everything after them, -1 both.
// Returns the first error of the event calls.
hipError_t launch_heff(const double* f, const double* V, const double* y1, const double* y2,
                       const double* L, const double* LY, const RingOps& rings, const double* t1,
                       const double* t2, int n,
                       int o, const double* scal, const SpaceDev* spaces, const int64_t* heff_off,
                       const int32_t* task_table, int task_stride, const int* task_slots,
                       const int32_t* cls_idx, const int* cls_off, int K, int na_max,
                       double* tab, double* fs1, const double* zc, const double* mpd, double* heff,
                       hipStream_t st, double* zs, hipStream_t st2, hipEvent_t fork_ev,
                       hipEvent_t join_ev, int phase = -1, const double* xtra = nullptr);
// The next DUCC truncation, 1/2 [[V_N, s]_2, s]_2 (k_vdouble.hip).  A W buffer
// holds a dense operator over all orbitals: two-body [n^4], one-body [n^2],
// zero-body; vd_space_doubles(n) doubles.
size_t vd_space_doubles(int n);
// wg = [V_N, sigma]_2
void launch_vd_global(const double* V, const double* t1, const double* t2, int n, int o,
                      double* wg, hipStream_t st);
// spaces k0 .. k0+kb-1 of the list: their W (into wsp, kb buffers), then
// 1/2 [W, s]_2 on the space's orbitals into xtra at heff_off[k], in the
// layout of the H_eff block before its CAS form ([x0, x1, x2], local indices)
void launch_vd_spaces(const double* V, const double* t1, const double* t2,
                      const SpaceDev* spaces, int k0, int kb, int n, int o, const double* wg,
                      double* wsp, const int64_t* heff_off, double* xtra, hipStream_t st);
// r2 += 1/2 [wg, sigma]_2 (a,b,i,j), r1 += 1/2 [wg, sigma]_1 (a,i), *e0 +=
// its zero-body part (e0 may be NULL)
void launch_vd_resid(const double* wg, const double* t1, const double* t2, int n, int o,
                     double* r1, double* r2, double* e0, hipStream_t st);
// Operand of the dense occupied-pair ladder (k_heff.hip): xp[tri(p,q)][(t,u)]
// = (H_N + Yg/2)(p,q,t,u), p <= q, t, u occupied; n(n+1)/2 x o^2 doubles.  The
// ladder mpd = xp T^T with T[(a,b)][(t,u)] = t2[t,u,a,b] (launch_pack_t2_vvoo).
void launch_pack_x_pairs(const double* Xh, const double* Xy, int n, int o, double* xp,
                         hipStream_t st);
// doubles of per-space scratch tables for spaces of up to na_max orbitals
int heff_table_stride(int na_max);
// doubles of dynamic LDS the build of a space of na orbitals takes
int heff_lds_doubles(int na);
// output-element order of the per-space kernels (host; see strings.cpp)
int build_tasks(int na, int ne, int32_t* out, int cap);
constexpr int kTaskStride = 4608;   // >= padded task count of a (4,4) space

// per-space Davidson eigensolver and cluster analysis
struct DavidsonArgs {
  const SpaceDev* spaces;
  const Strings* strings;     // one table per size class, indexed by nocc-2
  const double* heff;
  const int64_t* heff_off;
  double* work;               // per space: dav_layout(...).work doubles
  const int64_t* work_off;
  double* energy;
  double* c0;
  double* amp;
  const int64_t* amp_off;
  double* ci;                 // per space: ns^2 eigenvector, start and result (NULL: none)
  const int64_t* ci_off;
  int32_t* iters;
  int32_t* status;
  double tol;
  int max_iter;
  int maxsub;
  int K;
  int* counter = nullptr;     // work counter of the persistent launch (one int)
  int big_block = 512;        // threads per (4,4) space in per-class launches: 512 or 1024
};
// Memory of one space's solve (doubles): LDS holds the integrals, the
// same-spin string Hamiltonian, the full vector sigma reads, the subspace
// problem and the replacement lists; the basis and its sigma vectors (spin-
// flip symmetric, kept as their halves of ns (ns + 1) / 2 entries) sit in the
// space's global work area, and so do the diagonal, Ritz sigma and residual
// halves when they would not fit in LDS as well (the (4,4) class).
struct DavLayout {
  int lds;        // doubles of dynamic LDS
  int64_t work;   // doubles of global work
  bool big;       // diagonal / Ritz sigma / residual vectors in global memory
};
constexpr int kDavBigDets = 1024;
// threads per space: 256, and 512 for the (4,4) class, whose LDS admits one
// block per compute unit (two wavefronts per SIMD hide the LDS gathers)
__host__ __device__ constexpr int dav_block(int na) { return na >= 8 ? 512 : 256; }
// (blk: threads of the workgroup solving the space; 0 = dav_block(na))
__host__ __device__ constexpr DavLayout dav_layout(int na, int ne, int maxsub, int blk = 0) {
  int ns = 1;
  for (int i = 0; i < ne; ++i) ns = ns * (na - i) / (i + 1);
  const int D = ns * ns, DU = ns * (ns + 1) / 2, nrep = ne * (1 + na - ne),
            n4 = na * na * na * na;
  const bool big = D > kDavBigDets;
  const int lds = n4 + ns * (ns | 1) + D + 3 * maxsub * maxsub + maxsub + 4 +
                  (blk > 0 ? blk : dav_block(na)) / 64 * maxsub + (ns * nrep + 1) / 2 +
                  (big ? 0 : 3 * DU);
  return DavLayout{lds, (int64_t)(2 * maxsub + (big ? 3 : 0)) * DU, big};
}
// cls_idx lists the spaces of class c (nocc = c + 2) at [cls_off[c],
// cls_off[c+1]) (cls_off on the host, 4 entries).  persistent = false: one
// launch per size class, a workgroup per space.  persistent = true: one
// launch over every class; as many workgroups as fit on the device (threads
// and LDS sized for the largest class present) take spaces from the counter
// a.counter (reset by the launch, on the stream), the largest class first,
// until the list is exhausted.
void launch_davidson(const DavidsonArgs& a, const int32_t* cls_idx, const int* cls_off,
                     hipStream_t st, bool persistent = false);

// UCCSD-VQE solve of every (2,2) and (3,3) space of the class lists: the
// parameters of sigma_int minimising <Phi|e^-sigma H_eff e^sigma|Phi>, started
// from theta0 (per space in the amp layout: t1[n_o][n_v] then
// t2[n_o][n_o][n_v][n_v]); writes energy, the parameters (amp layout), iters
// and status (0, or -5 when max_iter BFGS iterations did not bring the largest
// gradient entry below gtol); c0 = 1.
struct VqeArgs {
  const SpaceDev* spaces;
  const Strings* strings;
  const double* heff;
  const int64_t* heff_off;
  const double* theta0;
  const int64_t* amp_off;
  double* energy;
  double* c0;
  double* amp;
  int32_t* iters;
  int32_t* status;
  double gtol;
  int max_iter;
  int K;
};
int vqe_lds_bytes(int nocc);   // dynamic LDS of one space's workgroup (-1: unsupported)
void launch_vqe(const VqeArgs& a, const int32_t* cls_idx, const int* cls_off, hipStream_t st);
// the pool's amplitudes of every space into the amp layout (local indices)
void launch_gather_local(const SpaceDev* spaces, const int64_t* amp_off, const double* t1,
                         const double* t2, int n, int o, int K, double* out, hipStream_t st);

// pool update
void launch_update(const double* t1, const double* t2, const double* r1, const double* r2,
                   const double* f, const int32_t* owner1, const int32_t* owner2, int n, int o,
                   bool unowned_step, double* t1n, double* t2n, hipStream_t st);
// spaces k0 .. k0+K-1 write the amplitudes they own
void launch_scatter_owned(const SpaceDev* spaces, const double* amp, const int64_t* amp_off,
                          const int32_t* status, const int32_t* owner1, const int32_t* owner2,
                          int n, int o, int k0, int K, double* t1n, double* t2n, hipStream_t st);
// t[i] = owner[i] < 0 ? tn[i] : t[i] over t1 and t2 (the unowned step of a
// windowed sweep, taken from the pool at its start)
void launch_merge_unowned(const double* t1n, const double* t2n, const int32_t* owner1,
                          const int32_t* owner2, int o, int v, double* t1, double* t2,
                          hipStream_t st);
// DIIS over the amplitude vector [t1 | t2]: up to kDiisMax (t_new, error)
// pairs in T and E (kDiisMax * N doubles each), the Gram matrix of the
// errors, the pair count and the extrapolation coefficients in one device
// struct (zeroed to start a history).  From the kDiisStart-th pair on,
// t1n / t2n are replaced by the extrapolated vector.  part: kDiisMax *
// kDiisParts doubles of scratch.
constexpr int kDiisMax = 8;
constexpr int kDiisStart = 3;
constexpr double kDiisPivotTol = 1e-14;
constexpr int kDiisParts = 1024;
struct DiisState {
  int count, pad;
  double B[kDiisMax * kDiisMax];
  double c[kDiisMax];
};
void launch_diis(const double* t1, const double* t2, int o, int v, double* T, double* E,
                 DiisState* state, double* part, double* t1n, double* t2n, hipStream_t st);
// mean energy and max |t_new - t_old| into out2[0..1]; part holds
// kFinishParts doubles of scratch
constexpr int kFinishParts = 512;
void launch_finish(const double* energy, int K, const double* t1, const double* t2,
                   const double* t1n, const double* t2n, int o, int v, double* part,
                   double* out2, hipStream_t st);

}  // namespace qf
