// libqflow host runtime: context, device workspaces and the C ABI of
// include/qflow.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/qflow.h"
#include "kernels.h"
#include "qflow_cas.h"

namespace qf {
bool build_strings(int na, int ne, Strings* S);
}

using qf::SpaceDev;

namespace {

constexpr int kMaxSub = 12;        // Davidson subspace before restart
constexpr int kStages = 11;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GraphKey {
  int32_t K = -1, flags = 0;
  const void *t1 = nullptr, *t2 = nullptr, *o1 = nullptr, *o2 = nullptr, *energy = nullptr;
  uint64_t epoch = 0;
  bool operator==(const GraphKey& b) const {
    return K == b.K && flags == b.flags && t1 == b.t1 && t2 == b.t2 && o1 == b.o1 &&
           o2 == b.o2 && energy == b.energy && epoch == b.epoch;
  }
};

}  // namespace

// Work memory of qflow_solve_active_batch_static: one file-scope array, of
// which every device the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: host code uses only the address resolved below.
static __device__ __align__(256) unsigned char scratch[QFLOW_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current),
// resolved once per device and kept.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

struct qflow_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // H_N's contractions (they need only t2), then J, Lo and Z (once Yg's
  // two-body part is written) run here beside Yg's chain, joined back into
  // `stream` by events; their split-K slices go to gpart2
  hipStream_t stream2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipEvent_t y_ev = nullptr;   // Yg's two-body part written (J, Lo, Z may start)
  // the same for the per-space Hamiltonians: their sigma1 x two-body and
  // occupied-pair ladder parts run on stream2 into zsum
  hipEvent_t fork2_ev = nullptr, join2_ev = nullptr;
  hipEvent_t tabf_ev = nullptr, tab_ev = nullptr;   // the tables on stream2
  std::string err;
  // problem
  int n = 0, o = 0, v = 0;
  bool loaded = false;
  double e_ref = 0.0;
  std::vector<double> fock;
  // device state
  DevBuf f, V, W, y1, y2, wy, L, LY, scal, r1, r2, t1n, t2n;
  // ring intermediates: packed operands (H constant, Yg per step) and outputs
  DevBuf ra_h, r22_h, ra_y, r22_y, rta, rt22, ga_h, g22_h, ga_y, g22_y, jh, jy;
  // one-body ring terms: packed operands (A of H constant, A of Yg and B per
  // step) and the split-K slices
  DevBuf ja_h, ja_y, jb;
  DevBuf gpart;   // split-K slices of the matrix-core contractions
  DevBuf gpart2;  // the same for the contractions on stream2
  // Z = sigma1 X (first index) of H_N and Yg, n^4 each
  DevBuf zv, zo;   // sigma1 x two-body pieces of the residual
  DevBuf zc;       // dense sigma1 (H_N + Yg/2), n^4, when some call takes that form
  DevBuf xp, mp;   // dense occupied-pair ladder: its operand and the table (same form)
  DevBuf zsum;     // per space na^4: those parts of H_eff made on stream2
  int z_mode = QFLOW_Z_AUTO;
  DevBuf dtpart;   // per-block maxima of |t_new - t_old|
  // [G, sigma_2]_2 scratch (packed one-body, transposed t2, GEMM outputs)
  // and U_Y = [y1, sigma_2]_2
  DevBuf a12, t2T, sp, sq, sp_f, sq_f;   // sp_f, sq_f keep the [F, sigma_2] parts
  DevBuf fs1;                            // one-body external sums of the marked tables
  DevBuf c1h, c1y;   // one-body parts of [H_N, sigma] and [Yg, sigma], [n][n]
  // FP32 operands of the mixed-precision ladder and ring products
  DevBuf w32, wy32, t2_32, ra32_h, r22_32_h, ra32_y, r22_32_y, rta32, rt22_32;
  bool h32_ready = false;   // w32, ra32_h, r22_32_h hold the loaded H_N
  // BF16x3 operands (hi and lo halves in one buffer each, rows padded to 32 k)
  DevBuf wb, wyb, t2b, rab_h, r22b_h, rab_y, r22b_y, rtab, rt22b;
  bool hb_ready = false;
  // occupied-occupied ladders: packed t2 [v*v][o*o], X_oooo of H (constant)
  // and Yg [o*o][o*o], outputs Lo of H and Yg [v*v][o*o]
  DevBuf lo_t, lo_xh, lo_xy, lo_h, lo_y;
  DevBuf ci, ci_off;   // eigenvectors kept between flow steps (warm starts)
  // DIIS history (QFLOW_DIIS): pairs (t_new, error), scratch, device state
  DevBuf diis_t, diis_e, diis_part, diis_state;
  bool diis_active = false;   // the device state holds a running history
  DevBuf heff, heff_off, amp, amp_off, work, work_off, energy, c0, iters, status, spaces,
      strings, out2, partial, tasks, mtab;
  // spaces grouped by size class (nocc 2, 3, 4): indices at [cls_off[c], cls_off[c+1])
  DevBuf cls_idx;
  int cls_off[4] = {0, 0, 0, 0};
  // windowed sweeps: per window of win_size consecutive spaces, the class
  // lists at win_idx + win_base[w] with offsets win_off[4w .. 4w+3]
  DevBuf win_idx, t1s, t2s;
  std::vector<int> win_base, win_off;
  int win_size = 0;
  // task slots per class, then the slots of its two-body elements (first)
  int task_slots[6] = {0, 0, 0, 0, 0, 0};
  int lds_limit = 64 * 1024;   // dynamic LDS bytes a block may use
  // host mirror of the last uploaded space list
  std::vector<qflow_space> last_spaces;
  std::vector<int64_t> h_heff_off, h_amp_off, h_work_off, h_ci_off;
  int na_max = 0;
  int slots_max = 0;
  hipEvent_t ev[kStages + 1] = {};
  // captured flow step (QFLOW_GRAPH) and what it was captured for
  hipGraphExec_t graph_exec = nullptr;
  GraphKey graph_key{};
  uint64_t epoch = 0;   // bumped whenever a device buffer is (re)allocated
  float stage_ms[kStages] = {};
  float total_ms = 0.f;
  bool timed = false;
  void* scratch = nullptr;   // this device's copy of `scratch` (device address)
  // stopping rule of the flow steps' eigensolves (qflow_set_solver)
  double dav_tol = 1e-10;
  int dav_max_iter = 200;
  // launch choices (qflow_set_tuning / qflow_autotune); z_mode lives above
  int dav_persistent = 0, split_target = 4, f64_tile = 0, block_44 = 512;
  DevBuf dav_counter;          // work counter of the persistent Davidson launch
  DevBuf tune_t1, tune_t2, tune_e;   // the autotuner's copies of the pool, energies
  // the UCCSD-VQE solver (QFLOW_SOLVER_VQE): stopping rule, start parameters
  double vqe_gtol = 1e-10;
  int vqe_max_iter = 500;
  DevBuf vqe_theta;
  // truncation of the downfolded Hamiltonian (qflow_set_truncation); for
  // QFLOW_TRUNC_H: Wg, a batch of per-space W buffers, the per-space extra
  // terms (laid out like heff)
  int trunc = QFLOW_TRUNC_F;
  DevBuf vd_wg, vd_wsp, vd_xtra;
  int vd_batch = 0;
};

namespace {

int fail(qflow_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define QF_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, QFLOW_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

int ensure(qflow_ctx* ctx, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return QFLOW_OK;
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(ctx, QFLOW_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  ++ctx->epoch;
  return QFLOW_OK;
}

template <class T>
T* P(DevBuf& b) {
  return static_cast<T*>(b.p);
}

#define QF_TRY(expr)            \
  do {                          \
    int r_ = (expr);            \
    if (r_ != QFLOW_OK) return r_; \
  } while (0)

int na_of(const qflow_space& s) { return s.n_o + s.n_v; }

int check_spaces(qflow_ctx* ctx, int32_t K, const qflow_space* spaces) {
  if (K < 0) return fail(ctx, QFLOW_E_INVALID_ARG, "K < 0");
  if (K > 0 && !spaces) return fail(ctx, QFLOW_E_INVALID_ARG, "spaces is NULL");
  for (int k = 0; k < K; ++k) {
    const qflow_space& s = spaces[k];
    if (s.n_o < 2 || s.n_o > 4 || s.n_v != s.n_o)
      return fail(ctx, QFLOW_E_UNSUPPORTED,
                  "space " + std::to_string(k) + ": only (2,2), (3,3) and (4,4) spaces");
    for (int a = 0; a < na_of(s); ++a) {
      const int p = s.orb[a];
      const bool occ = a < s.n_o;
      if (p < 0 || p >= ctx->n || (occ && p >= ctx->o) || (!occ && p < ctx->o))
        return fail(ctx, QFLOW_E_INVALID_ARG, "space " + std::to_string(k) + ": bad orbital");
      if (a > 0 && a != s.n_o && s.orb[a - 1] >= p)
        return fail(ctx, QFLOW_E_INVALID_ARG,
                    "space " + std::to_string(k) + ": orbitals not ascending");
    }
  }
  return QFLOW_OK;
}

bool same_spaces(const qflow_ctx* ctx, int32_t K, const qflow_space* spaces) {
  return (int)ctx->last_spaces.size() == K &&
         (K == 0 || std::memcmp(ctx->last_spaces.data(), spaces, sizeof(qflow_space) * K) == 0);
}

// Upload the space list (and its derived offsets) when it changed.
// The sigma1 x two-body part of the space Hamiltonians, for the spaces of
// the class lists cls_off: dense (form Z = sigma1 (H_N + Yg/2) once: read
// both operators, write Z, 3 n^4 doubles) when that moves fewer doubles than
// the per-space gathers (both operators, na^3 rows of n per space), unless
// the mode says otherwise.
bool z_dense_for(const qflow_ctx* ctx, const int* cls_off) {
  if (ctx->z_mode != QFLOW_Z_AUTO) return ctx->z_mode == QFLOW_Z_DENSE;
  double rows = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double na = 2 * (c + 2);
    rows += (double)(cls_off[c + 1] - cls_off[c]) * na * na * na;
  }
  const double n = ctx->n;
  return 2.0 * rows * n > 3.0 * n * n * n * n;
}

// The dense form also takes the occupied-pair ladders as one table over all
// pairs p <= q (k_heff_pp otherwise gathers the rows per space).
int ensure_zc(qflow_ctx* ctx) {
  if (!ctx->loaded || !z_dense_for(ctx, ctx->cls_off)) return QFLOW_OK;
  const size_t n = ctx->n, o = ctx->o, v = ctx->v, npair = n * (n + 1) / 2;
  QF_TRY(ensure(ctx, ctx->xp, sizeof(double) * npair * o * o));
  QF_TRY(ensure(ctx, ctx->mp, sizeof(double) * npair * v * v));
  return ensure(ctx, ctx->zc, sizeof(double) * n * n * n * n);
}

int upload_space_list(qflow_ctx* ctx, int32_t K, const qflow_space* spaces);

// doubles of the stream2 part buffer for the class lists cls_off
size_t zsum_doubles(const int* cls_off) {
  size_t d = 0;
  for (int c = 0; c < 3; ++c) {
    const size_t na = 2 * (c + 2);
    d += (size_t)(cls_off[c + 1] - cls_off[c]) * na * na * na * na;
  }
  return d;
}

int upload_spaces(qflow_ctx* ctx, int32_t K, const qflow_space* spaces) {
  QF_TRY(upload_space_list(ctx, K, spaces));
  return ensure_zc(ctx);   // outside any graph capture
}

// The next truncation's direct evaluation costs O(K n^4) per step.
constexpr int kTruncHMaxOrb = 64;

// Buffers of the next truncation for the uploaded list (outside any capture):
// Wg, W of up to vd_batch spaces at once (at most 4 GiB), the extra terms.
int ensure_vdouble(qflow_ctx* ctx, int32_t K, int64_t xtra_doubles) {
  if (ctx->trunc != QFLOW_TRUNC_H) return QFLOW_OK;
  if (ctx->n > kTruncHMaxOrb)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "QFLOW_TRUNC_H takes at most 64 orbitals");
  const size_t wn = qf::vd_space_doubles(ctx->n);
  const size_t cap = (size_t)4 << 30;
  ctx->vd_batch = (int)std::max<size_t>(1, std::min<size_t>(std::max(K, 1), cap / (wn * 8)));
  QF_TRY(ensure(ctx, ctx->vd_wg, sizeof(double) * wn));
  if (K > 0) {
    QF_TRY(ensure(ctx, ctx->vd_wsp, sizeof(double) * wn * ctx->vd_batch));
    QF_TRY(ensure(ctx, ctx->vd_xtra, sizeof(double) * std::max<int64_t>(xtra_doubles, 1)));
  }
  return QFLOW_OK;
}

int upload_space_list(qflow_ctx* ctx, int32_t K, const qflow_space* spaces) {
  if (same_spaces(ctx, K, spaces) && ctx->spaces.p) return QFLOW_OK;
  std::vector<SpaceDev> dev(std::max(K, 1));
  ctx->h_heff_off.assign(K + 1, 0);
  ctx->h_amp_off.assign(K + 1, 0);
  ctx->h_ci_off.assign(K + 1, 0);
  ctx->h_work_off.assign(K + 1, 0);
  int lds = 0, na_max = 0, slots_max = 0;
  std::vector<int32_t> cls[3];
  for (int k = 0; k < K; ++k) {
    const qflow_space& s = spaces[k];
    dev[k].na = na_of(s);
    dev[k].nocc = s.n_o;
    for (int a = 0; a < 8; ++a) dev[k].orb[a] = a < dev[k].na ? s.orb[a] : 0;
    const int na = dev[k].na;
    const int64_t nt1 = (int64_t)s.n_o * s.n_v;
    ctx->h_heff_off[k + 1] = ctx->h_heff_off[k] + qflow_heff_size(&s);
    ctx->h_amp_off[k + 1] = ctx->h_amp_off[k] + nt1 + nt1 * nt1;
    const qf::DavLayout lay = qf::dav_layout(na, s.n_o, kMaxSub);
    ctx->h_work_off[k + 1] = ctx->h_work_off[k] + lay.work;
    ctx->h_ci_off[k + 1] = ctx->h_ci_off[k] + qflow_ci_size(&s);
    lds = std::max(lds, lay.lds);
    lds = std::max(lds, qf::heff_lds_doubles(na));
    na_max = std::max(na_max, na);
    slots_max = std::max(slots_max, ctx->task_slots[s.n_o - 2]);
    cls[s.n_o - 2].push_back(k);
  }
  if ((size_t)lds * sizeof(double) > (size_t)ctx->lds_limit)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "active space too large for the device's LDS");
  ctx->na_max = na_max;
  ctx->slots_max = slots_max;
  std::vector<int32_t> idx;
  for (int c = 0; c < 3; ++c) {
    ctx->cls_off[c] = (int)idx.size();
    idx.insert(idx.end(), cls[c].begin(), cls[c].end());
  }
  ctx->cls_off[3] = (int)idx.size();
  idx.resize(std::max(K, 1), 0);
  QF_TRY(ensure(ctx, ctx->cls_idx, sizeof(int32_t) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->spaces, sizeof(SpaceDev) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->heff_off, sizeof(int64_t) * (K + 1)));
  QF_TRY(ensure(ctx, ctx->amp_off, sizeof(int64_t) * (K + 1)));
  QF_TRY(ensure(ctx, ctx->work_off, sizeof(int64_t) * (K + 1)));
  QF_TRY(ensure(ctx, ctx->work, sizeof(double) * std::max<int64_t>(ctx->h_work_off[K], 1)));
  QF_TRY(ensure(ctx, ctx->heff, sizeof(double) * std::max<int64_t>(ctx->h_heff_off[K], 1)));
  QF_TRY(ensure(ctx, ctx->zsum, sizeof(double) * std::max<size_t>(zsum_doubles(ctx->cls_off), 1)));
  QF_TRY(ensure(ctx, ctx->amp, sizeof(double) * std::max<int64_t>(ctx->h_amp_off[K], 1)));
  QF_TRY(ensure(ctx, ctx->ci_off, sizeof(int64_t) * (K + 1)));
  QF_TRY(ensure(ctx, ctx->ci, sizeof(double) * std::max<int64_t>(ctx->h_ci_off[K], 1)));
  // a new space list starts every solve cold
  qf::launch_fill(P<double>(ctx->ci), (size_t)std::max<int64_t>(ctx->h_ci_off[K], 1), 0.0,
                  ctx->stream);
  QF_TRY(ensure(ctx, ctx->energy, sizeof(double) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->c0, sizeof(double) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->iters, sizeof(int32_t) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->status, sizeof(int32_t) * std::max(K, 1)));
  QF_TRY(ensure(ctx, ctx->mtab,
                sizeof(double) * (size_t)std::max(K, 1) * qf::heff_table_stride(std::max(na_max, 4))));
  QF_HIP(hipMemcpyAsync(ctx->spaces.p, dev.data(), sizeof(SpaceDev) * std::max(K, 1),
                        hipMemcpyHostToDevice, ctx->stream));
  QF_HIP(hipMemcpyAsync(ctx->heff_off.p, ctx->h_heff_off.data(), sizeof(int64_t) * (K + 1),
                        hipMemcpyHostToDevice, ctx->stream));
  QF_HIP(hipMemcpyAsync(ctx->amp_off.p, ctx->h_amp_off.data(), sizeof(int64_t) * (K + 1),
                        hipMemcpyHostToDevice, ctx->stream));
  QF_HIP(hipMemcpyAsync(ctx->work_off.p, ctx->h_work_off.data(), sizeof(int64_t) * (K + 1),
                        hipMemcpyHostToDevice, ctx->stream));
  QF_HIP(hipMemcpyAsync(ctx->ci_off.p, ctx->h_ci_off.data(), sizeof(int64_t) * (K + 1),
                        hipMemcpyHostToDevice, ctx->stream));
  QF_HIP(hipMemcpyAsync(ctx->cls_idx.p, idx.data(), sizeof(int32_t) * std::max(K, 1),
                        hipMemcpyHostToDevice, ctx->stream));
  // the host vectors must outlive the asynchronous copies
  QF_HIP(hipStreamSynchronize(ctx->stream));
  ctx->last_spaces.assign(spaces, spaces + K);
  ++ctx->epoch;   // launch shapes of the per-space kernels follow the list
  ctx->diis_active = false;   // a new list starts a new DIIS history
  ctx->win_size = 0;
  return QFLOW_OK;
}

int require_loaded(qflow_ctx* ctx) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (!ctx->loaded) return fail(ctx, QFLOW_E_STATE, "no integrals loaded");
  return QFLOW_OK;
}

qf::RingOps rings_of(qflow_ctx* ctx) {
  const size_t nv = (size_t)ctx->n * ctx->v;
  return qf::RingOps{P<double>(ctx->ga_h), P<double>(ctx->g22_h), P<double>(ctx->jh),
                     P<double>(ctx->jh) + nv,  P<double>(ctx->ga_y), P<double>(ctx->g22_y),
                     P<double>(ctx->jy),       P<double>(ctx->jy) + nv,
                     P<double>(ctx->zv),       P<double>(ctx->zo),
                     P<double>(ctx->y2),       P<double>(ctx->sp),       P<double>(ctx->sq),
                     P<double>(ctx->c1h),      P<double>(ctx->c1y),
                     P<double>(ctx->lo_h),     P<double>(ctx->lo_y),
                     P<double>(ctx->sp_f),     P<double>(ctx->sq_f)};
}

// BF16x3 operands: a [rows][K] FP64 matrix becomes hi and lo bf16 halves of
// [rows][Kp] each, stored one after the other in one buffer.
struct Split {
  __bf16* hi;
  __bf16* lo;
};
Split split_of(DevBuf& b, size_t rows, int K) {
  __bf16* base = P<__bf16>(b);
  return Split{base, base + rows * (size_t)qf::bf16_pad(K)};
}
int ensure_split(qflow_ctx* ctx, DevBuf& b, size_t rows, int K) {
  return ensure(ctx, b, sizeof(__bf16) * 2 * rows * (size_t)qf::bf16_pad(K));
}
void split(const double* src, size_t rows, int K, Split d, hipStream_t st) {
  qf::launch_split_bf16(src, (int)rows, K, qf::bf16_pad(K), d.hi, d.lo, st);
}

int ensure_bf16(qflow_ctx* ctx) {
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  const size_t n2 = (size_t)n * n, n2p = (size_t)n * (n + 1) / 2, ov = (size_t)o * v;
  QF_TRY(ensure_split(ctx, ctx->wb, n2p, v * v));
  QF_TRY(ensure_split(ctx, ctx->wyb, n2p, v * v));
  QF_TRY(ensure_split(ctx, ctx->t2b, (size_t)o * o, v * v));
  QF_TRY(ensure_split(ctx, ctx->rab_h, n2, (int)(2 * ov)));
  QF_TRY(ensure_split(ctx, ctx->r22b_h, n2, (int)ov));
  QF_TRY(ensure_split(ctx, ctx->rab_y, n2, (int)(2 * ov)));
  QF_TRY(ensure_split(ctx, ctx->r22b_y, n2, (int)ov));
  QF_TRY(ensure_split(ctx, ctx->rtab, ov, (int)(2 * ov)));
  QF_TRY(ensure_split(ctx, ctx->rt22b, ov, (int)ov));
  if (!ctx->hb_ready) {
    hipStream_t st = ctx->stream;
    // the per-step ring operands are packed straight into their planes and
    // never write the K padding: zero it (whole buffers) once here
    for (DevBuf* b : {&ctx->rab_y, &ctx->r22b_y, &ctx->rtab, &ctx->rt22b, &ctx->wyb})
      qf::launch_fill(P<double>(*b), b->bytes / sizeof(double), 0.0, st);
    split(P<double>(ctx->W), n2p, v * v, split_of(ctx->wb, n2p, v * v), st);
    split(P<double>(ctx->ra_h), n2, (int)(2 * ov), split_of(ctx->rab_h, n2, (int)(2 * ov)), st);
    split(P<double>(ctx->r22_h), n2, (int)ov, split_of(ctx->r22b_h, n2, (int)ov), st);
    QF_HIP(hipGetLastError());
    ctx->hb_ready = true;
  }
  return QFLOW_OK;
}

// Yg = [F,sigma], the ladder intermediates L = W t2^T, LY = WY t2^T and the
// ring intermediates (Ga, G22 by matrix cores; J1, J2) of H_N and Yg
// FP32 copies of the ladder and ring GEMM operands for the mixed-precision
// contractions; those of H_N are converted once per integral load.
int ensure_mixed(qflow_ctx* ctx) {
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  const size_t n2 = (size_t)n * n, n2p = (size_t)n * (n + 1) / 2, ov = (size_t)o * v;
  QF_TRY(ensure(ctx, ctx->w32, sizeof(float) * n2p * v * v));
  QF_TRY(ensure(ctx, ctx->wy32, sizeof(float) * n2p * v * v));
  QF_TRY(ensure(ctx, ctx->t2_32, sizeof(float) * ov * ov));
  QF_TRY(ensure(ctx, ctx->ra32_h, sizeof(float) * n2 * 2 * ov));
  QF_TRY(ensure(ctx, ctx->r22_32_h, sizeof(float) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->ra32_y, sizeof(float) * n2 * 2 * ov));
  QF_TRY(ensure(ctx, ctx->r22_32_y, sizeof(float) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->rta32, sizeof(float) * ov * 2 * ov));
  QF_TRY(ensure(ctx, ctx->rt22_32, sizeof(float) * ov * ov));
  if (!ctx->h32_ready) {
    qf::launch_cvt_f32(P<double>(ctx->W), P<float>(ctx->w32), n2p * v * v, ctx->stream);
    qf::launch_pack_ring_A(P<double>(ctx->V), n, o, P<float>(ctx->ra32_h), P<float>(ctx->r22_32_h),
                           ctx->stream);
    QF_HIP(hipGetLastError());
    ctx->h32_ready = true;
  }
  return QFLOW_OK;
}

// Yg = [F,sigma], the ladder intermediates L = W t2^T, LY = WY t2^T and the
// ring intermediates (Ga, G22 by matrix cores; J1, J2) of H_N and Yg.  With
// QFLOW_FP32 the ladder and ring products (the o^2 v^4 and o^3 v^3
// contractions) take FP32 operands on the FP32 matrix cores, FP64 sums.
int prepare(qflow_ctx* ctx, const double* t1, const double* t2, int precision) {
  if (precision != QFLOW_FP64 && precision != QFLOW_FP32 && precision != QFLOW_BF16X3)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "unknown precision");
  const bool mixed = precision == QFLOW_FP32;
  const bool bf3 = precision == QFLOW_BF16X3;
  qf::GemmTuning gt;
  gt.split_target = ctx->split_target;
  gt.f64_tile = ctx->f64_tile;
  qf::set_gemm_tuning(gt);
  if (mixed) QF_TRY(ensure_mixed(ctx));
  if (bf3) QF_TRY(ensure_bf16(ctx));
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  const size_t n2 = (size_t)n * n, ov = (size_t)o * v;
  double* part = P<double>(ctx->gpart);
  const size_t pcap = ctx->gpart.bytes / sizeof(double);
  hipStream_t st = ctx->stream;
  const int npair = n * (n + 1) / 2;   // ladder rows p <= q
  const size_t n2p = (size_t)npair;
  const int kp = qf::bf16_pad(v * v);
  // t2 as the ladder operand, and the ring operands of t2 (read by the
  // contractions of H_N and of Yg)
  Split tb{};
  if (bf3) {
    tb = split_of(ctx->t2b, (size_t)o * o, v * v);
    split(t2, (size_t)o * o, v * v, tb, st);
    const Split ta = split_of(ctx->rtab, ov, (int)(2 * ov)), t22 = split_of(ctx->rt22b, ov, (int)ov);
    qf::launch_pack_ring_T_bf16(t2, o, v, ta.hi, ta.lo, t22.hi, t22.lo, st);
  } else if (mixed) {
    qf::launch_cvt_f32(t2, P<float>(ctx->t2_32), ov * ov, st);
    qf::launch_pack_ring_T(t2, o, v, P<float>(ctx->rta32), P<float>(ctx->rt22_32), st);
  } else {
    qf::launch_pack_ring_T(t2, o, v, P<double>(ctx->rta), P<double>(ctx->rt22), st);
  }
  // H_N's particle-particle ladder and ring contractions need nothing else:
  // outside the stage-timed mode they run on stream2 beside the Yg chain
  // (their own split-K slices) and are joined back at the end of this
  // function; in it they keep their place in the stage order.
  auto ladder_h = [&](hipStream_t s, double* pp, size_t pc) {
    if (bf3) {
      const Split wb = split_of(ctx->wb, n2p, v * v);
      qf::launch_gemm_nt_bf16x3(wb.hi, wb.lo, tb.hi, tb.lo, P<double>(ctx->L), npair, o * o, kp,
                                1.0, pp, pc, s);
    } else if (mixed) {
      qf::launch_gemm_nt_f32(P<float>(ctx->w32), P<float>(ctx->t2_32), P<double>(ctx->L), npair,
                             o * o, v * v, 1.0, pp, pc, s);
    } else {
      qf::launch_gemm_nt_f64(P<double>(ctx->W), t2, P<double>(ctx->L), npair, o * o, v * v, 1.0,
                             pp, pc, s);
    }
  };
  auto rings_h = [&](hipStream_t s, double* pp, size_t pc) {
    if (bf3) {
      const int ka = qf::bf16_pad((int)(2 * ov)), k22 = qf::bf16_pad((int)ov);
      const Split ta = split_of(ctx->rtab, ov, (int)(2 * ov)), t22 = split_of(ctx->rt22b, ov, (int)ov);
      const Split ah = split_of(ctx->rab_h, n2, (int)(2 * ov)), a22h = split_of(ctx->r22b_h, n2, (int)ov);
      qf::launch_gemm_nt_bf16x3(ah.hi, ah.lo, ta.hi, ta.lo, P<double>(ctx->ga_h), (int)n2, (int)ov,
                                ka, 1.0, pp, pc, s);
      qf::launch_gemm_nt_bf16x3(a22h.hi, a22h.lo, t22.hi, t22.lo, P<double>(ctx->g22_h), (int)n2,
                                (int)ov, k22, 1.0, pp, pc, s);
    } else if (mixed) {
      qf::launch_gemm_nt_f32(P<float>(ctx->ra32_h), P<float>(ctx->rta32), P<double>(ctx->ga_h),
                             (int)n2, (int)ov, (int)(2 * ov), 1.0, pp, pc, s);
      qf::launch_gemm_nt_f32(P<float>(ctx->r22_32_h), P<float>(ctx->rt22_32), P<double>(ctx->g22_h),
                             (int)n2, (int)ov, (int)ov, 1.0, pp, pc, s);
    } else {
      qf::launch_gemm_nt_f64(P<double>(ctx->ra_h), P<double>(ctx->rta), P<double>(ctx->ga_h),
                             (int)n2, (int)ov, (int)(2 * ov), 1.0, pp, pc, s);
      qf::launch_gemm_nt_f64(P<double>(ctx->r22_h), P<double>(ctx->rt22), P<double>(ctx->g22_h),
                             (int)n2, (int)ov, (int)ov, 1.0, pp, pc, s);
    }
  };
  // J, Lo and the residual's vvoo Z pieces read Yg's two-body part (and t2,
  // t1) but nothing that Yg's ladder and rings write
  auto tail_y = [&](hipStream_t s, double* pp, size_t pc) -> int {
    // one-body ring terms J1, J2 of H_N and Yg
    const size_t kj = (size_t)o * o * v;
    double* b1 = P<double>(ctx->jb);
    double* b2 = b1 + (size_t)v * kj;
    qf::launch_pack_j_B(t2, o, v, b1, b2, s);
    qf::launch_pack_j_A(P<double>(ctx->y2), n, o, P<double>(ctx->ja_y),
                        P<double>(ctx->ja_y) + (size_t)n * kj, s);
    {   // J1, J2 of H_N and of Yg: four products of one shape in one launch
      const double* ja[4] = {P<double>(ctx->ja_h), P<double>(ctx->ja_h) + (size_t)n * kj,
                             P<double>(ctx->ja_y), P<double>(ctx->ja_y) + (size_t)n * kj};
      const double* jbs[4] = {b1, b2, b1, b2};
      double* jc[4] = {P<double>(ctx->jh), P<double>(ctx->jh) + (size_t)n * v, P<double>(ctx->jy),
                       P<double>(ctx->jy) + (size_t)n * v};
      (void)qf::launch_gemm_nt_f64_batch(ja, jbs, jc, 4, n, v, (int)kj, -1.0, pp, pc, s);
    }
    // occupied-occupied ladders Lo of H_N and Yg
    qf::launch_pack_t2_vvoo(t2, o, v, P<double>(ctx->lo_t), s);
    qf::launch_pack_x_oooo(P<double>(ctx->y2), n, o, P<double>(ctx->lo_xy), s);
    {
      const double* la[2] = {P<double>(ctx->lo_t), P<double>(ctx->lo_t)};
      const double* lb[2] = {P<double>(ctx->lo_xh), P<double>(ctx->lo_xy)};
      double* lc[2] = {P<double>(ctx->lo_h), P<double>(ctx->lo_y)};
      (void)qf::launch_gemm_nt_f64_batch(la, lb, lc, 2, v * v, o * o, o * o, 1.0, pp, pc, s);
    }
    if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[6], s));
    // sigma1 x two-body pieces of H_N + Yg/2 for the residual (the per-space
    // Hamiltonians evaluate theirs in k_heff_z)
    qf::launch_z_vvoo(P<double>(ctx->V), P<double>(ctx->y2), t1, n, o, P<double>(ctx->zv),
                      P<double>(ctx->zo), s);
    return QFLOW_OK;
  };
  const bool fork = !ctx->timed;
  if (fork) {
    hipStream_t sh = ctx->stream2;
    double* ph = P<double>(ctx->gpart2);
    const size_t pch = ctx->gpart2.bytes / sizeof(double);
    QF_HIP(hipEventRecord(ctx->fork_ev, st));
    QF_HIP(hipStreamWaitEvent(sh, ctx->fork_ev, 0));
    ladder_h(sh, ph, pch);
    rings_h(sh, ph, pch);
  }
  // Yg = [F_N, sigma]: one-body and scalar, two-body (+ its ladder slab), and
  // the compact parts of [y1, sigma_2]_2 (the one-body part of Yg against
  // sigma's two-body), which stay in sp / sq for the lookups
  qf::launch_yg1(P<double>(ctx->f), t1, t2, n, o, P<double>(ctx->y1), P<double>(ctx->scal), st);
  const int npo = o * n - o * (o - 1) / 2;   // non-zero ladder rows of Yg (see below)
  Split wyb_rows{};
  if (bf3) {   // Yg's ladder rows go straight into BF16 planes (npo rows each)
    const Split wyb = split_of(ctx->wyb, (size_t)n * (n + 1) / 2, v * v);
    wyb_rows = Split{wyb.hi, wyb.hi + (size_t)npo * kp};
  }
  qf::launch_sigma2(P<double>(ctx->f), t2, n, o, P<double>(ctx->a12), P<double>(ctx->t2T), true,
                    P<double>(ctx->sp_f), P<double>(ctx->sq_f), part, pcap, P<double>(ctx->y2),
                    (mixed || bf3) ? nullptr : P<double>(ctx->wy),
                    mixed ? P<float>(ctx->wy32) : nullptr, wyb_rows.hi, wyb_rows.lo, st);
  if (fork) {   // Yg's two-body part is complete: J, Lo, Z follow H_N's products on stream2
    hipStream_t sh = ctx->stream2;
    QF_HIP(hipEventRecord(ctx->y_ev, st));
    QF_HIP(hipStreamWaitEvent(sh, ctx->y_ev, 0));
    QF_TRY(tail_y(sh, P<double>(ctx->gpart2), ctx->gpart2.bytes / sizeof(double)));
    QF_HIP(hipEventRecord(ctx->join_ev, sh));
  }
  qf::launch_sigma2(P<double>(ctx->y1), t2, n, o, P<double>(ctx->a12), P<double>(ctx->t2T),
                    false, P<double>(ctx->sp), P<double>(ctx->sq), part, pcap, nullptr, nullptr,
                    nullptr, nullptr, nullptr, st);
  // rows of Yg's ladder operand with p virtual (then q virtual too) vanish:
  // the Yg ladder runs over the first npo = o*n - o(o-1)/2 rows only
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[1], st));
  if (!fork) ladder_h(st, part, pcap);
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[2], st));
  if (bf3) {
    qf::launch_gemm_nt_bf16x3(wyb_rows.hi, wyb_rows.lo, tb.hi, tb.lo, P<double>(ctx->LY), npo,
                              o * o, kp, 1.0, part, pcap, st);
  } else if (mixed) {
    qf::launch_gemm_nt_f32(P<float>(ctx->wy32), P<float>(ctx->t2_32), P<double>(ctx->LY), npo,
                           o * o, v * v, 1.0, part, pcap, st);
  } else {
    qf::launch_gemm_nt_f64(P<double>(ctx->wy), t2, P<double>(ctx->LY), npo, o * o, v * v, 1.0,
                           part, pcap, st);
  }
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[3], st));
  if (bf3) {
    const Split ay = split_of(ctx->rab_y, n2, (int)(2 * ov));
    const Split a22y = split_of(ctx->r22b_y, n2, (int)ov);
    qf::launch_pack_ring_A_bf16(P<double>(ctx->y2), n, o, ay.hi, ay.lo, a22y.hi, a22y.lo, st);
  } else if (mixed) {
    qf::launch_pack_ring_A(P<double>(ctx->y2), n, o, P<float>(ctx->ra32_y),
                           P<float>(ctx->r22_32_y), st);
  } else {
    qf::launch_pack_ring_A(P<double>(ctx->y2), n, o, P<double>(ctx->ra_y), P<double>(ctx->r22_y),
                           st);
  }
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[4], st));
  if (!fork) rings_h(st, part, pcap);
  if (bf3) {
    const int ka = qf::bf16_pad((int)(2 * ov)), k22 = qf::bf16_pad((int)ov);
    const Split ta = split_of(ctx->rtab, ov, (int)(2 * ov)), t22 = split_of(ctx->rt22b, ov, (int)ov);
    const Split ay = split_of(ctx->rab_y, n2, (int)(2 * ov)), a22y = split_of(ctx->r22b_y, n2, (int)ov);
    qf::launch_gemm_nt_bf16x3(ay.hi, ay.lo, ta.hi, ta.lo, P<double>(ctx->ga_y), (int)n2, (int)ov,
                              ka, 1.0, part, pcap, st);
    qf::launch_gemm_nt_bf16x3(a22y.hi, a22y.lo, t22.hi, t22.lo, P<double>(ctx->g22_y), (int)n2,
                              (int)ov, k22, 1.0, part, pcap, st);
  } else if (mixed) {
    const float* ta = P<float>(ctx->rta32);
    const float* t22 = P<float>(ctx->rt22_32);
    qf::launch_gemm_nt_f32(P<float>(ctx->ra32_y), ta, P<double>(ctx->ga_y), (int)n2, (int)ov,
                           (int)(2 * ov), 1.0, part, pcap, st);
    qf::launch_gemm_nt_f32(P<float>(ctx->r22_32_y), t22, P<double>(ctx->g22_y), (int)n2, (int)ov,
                           (int)ov, 1.0, part, pcap, st);
  } else {
    qf::launch_gemm_nt_f64(P<double>(ctx->ra_y), P<double>(ctx->rta), P<double>(ctx->ga_y),
                           (int)n2, (int)ov, (int)(2 * ov), 1.0, part, pcap, st);
    qf::launch_gemm_nt_f64(P<double>(ctx->r22_y), P<double>(ctx->rt22), P<double>(ctx->g22_y),
                           (int)n2, (int)ov, (int)ov, 1.0, part, pcap, st);
  }
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[5], st));
  if (!fork) QF_TRY(tail_y(st, part, pcap));
  if (fork) QF_HIP(hipStreamWaitEvent(st, ctx->join_ev, 0));   // stream2's part
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

}  // namespace

extern "C" {

int qflow_create(qflow_ctx** out, int device, void* hip_stream) {
  if (!out) return QFLOW_E_INVALID_ARG;
  *out = nullptr;
  qflow_ctx* ctx = new (std::nothrow) qflow_ctx();
  if (!ctx) return QFLOW_E_OOM;
  ctx->device = device;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete ctx;
    return QFLOW_E_DEVICE;
  }
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return QFLOW_E_DEVICE;
    }
    ctx->own_stream = true;
  }
  for (auto& ev : ctx->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      qflow_destroy(ctx);
      return QFLOW_E_DEVICE;
    }
  if (hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->y_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->fork2_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->join2_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->tabf_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->tab_ev, hipEventDisableTiming) != hipSuccess) {
    qflow_destroy(ctx);
    return QFLOW_E_DEVICE;
  }
  if (scratch_address(device, &ctx->scratch) != hipSuccess) {
    qflow_destroy(ctx);
    return QFLOW_E_DEVICE;
  }
  int lds_limit = 0;
  if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess &&
      lds_limit > 0)
    ctx->lds_limit = lds_limit;
  std::vector<qf::Strings> tabs(3);
  for (int s = 0; s < 3; ++s) qf::build_strings(2 * (s + 2), s + 2, &tabs[s]);
  std::vector<int32_t> task_tab(3 * qf::kTaskStride, -1);
  for (int s = 0; s < 3; ++s) {
    const int32_t* tt = &task_tab[s * qf::kTaskStride];
    ctx->task_slots[s] = qf::build_tasks(2 * (s + 2), s + 2, &task_tab[s * qf::kTaskStride],
                                         qf::kTaskStride);
    int two = 0;   // the two-body groups come first (kind 2 in bits 24..)
    while (two < ctx->task_slots[s] && (tt[two] < 0 || (tt[two] >> 24) == 2)) ++two;
    ctx->task_slots[3 + s] = two;
  }
  if (ensure(ctx, ctx->strings, sizeof(qf::Strings) * 3) != QFLOW_OK ||
      hipMemcpy(ctx->strings.p, tabs.data(), sizeof(qf::Strings) * 3, hipMemcpyHostToDevice) !=
          hipSuccess ||
      ensure(ctx, ctx->tasks, sizeof(int32_t) * task_tab.size()) != QFLOW_OK ||
      hipMemcpy(ctx->tasks.p, task_tab.data(), sizeof(int32_t) * task_tab.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      ensure(ctx, ctx->scal, sizeof(double) * 8) != QFLOW_OK ||
      ensure(ctx, ctx->out2, sizeof(double) * 2) != QFLOW_OK ||
      ensure(ctx, ctx->dav_counter, sizeof(int) * 2) != QFLOW_OK) {
    qflow_destroy(ctx);
    return QFLOW_E_DEVICE;
  }
  *out = ctx;
  return QFLOW_OK;
}

int qflow_destroy(qflow_ctx* ctx) {
  if (!ctx) return QFLOW_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->stream2) (void)hipStreamSynchronize(ctx->stream2);
  DevBuf* bufs[] = {&ctx->ra_h,   &ctx->r22_h,    &ctx->ra_y,   &ctx->r22_y,    &ctx->rta,
                    &ctx->rt22,   &ctx->ga_h,     &ctx->g22_h,  &ctx->ga_y,     &ctx->g22_y,
                    &ctx->jh,     &ctx->jy,       &ctx->ja_h,   &ctx->ja_y,     &ctx->jb,
                    &ctx->gpart,  &ctx->gpart2, &ctx->zv,       &ctx->zo,      &ctx->zc,     &ctx->xp,     &ctx->mp,     &ctx->zsum,     &ctx->dtpart,
                    &ctx->a12,    &ctx->t2T,      &ctx->sp,     &ctx->sq,       &ctx->sp_f,     &ctx->sq_f,     &ctx->fs1,
                    &ctx->c1h,
                    &ctx->c1y,    &ctx->lo_t,     &ctx->lo_xh,  &ctx->lo_xy,    &ctx->lo_h,
                    &ctx->lo_y,   &ctx->w32,      &ctx->wy32,   &ctx->t2_32,    &ctx->ra32_h,
                    &ctx->r22_32_h, &ctx->ra32_y, &ctx->r22_32_y, &ctx->rta32,  &ctx->rt22_32,
                    &ctx->wb,     &ctx->wyb,      &ctx->t2b,    &ctx->rab_h,    &ctx->r22b_h,
                    &ctx->rab_y,  &ctx->r22b_y,   &ctx->rtab,   &ctx->rt22b,
                    &ctx->f,      &ctx->V,        &ctx->W,      &ctx->y1,       &ctx->y2,
                    &ctx->wy,     &ctx->L,        &ctx->LY,     &ctx->scal,     &ctx->r1,
                    &ctx->r2,     &ctx->t1n,      &ctx->t2n,    &ctx->heff,     &ctx->heff_off,
                    &ctx->amp,    &ctx->amp_off,  &ctx->work,   &ctx->work_off, &ctx->energy,
                    &ctx->ci,     &ctx->ci_off,
                    &ctx->c0,     &ctx->iters,    &ctx->status, &ctx->spaces,   &ctx->strings,
                    &ctx->out2,   &ctx->partial, &ctx->tasks, &ctx->mtab,   &ctx->cls_idx,
                    &ctx->diis_t, &ctx->diis_e, &ctx->diis_part, &ctx->diis_state,
                    &ctx->win_idx, &ctx->t1s,    &ctx->t2s,
                    &ctx->dav_counter, &ctx->tune_t1, &ctx->tune_t2, &ctx->tune_e,
                    &ctx->vqe_theta, &ctx->vd_wg, &ctx->vd_wsp, &ctx->vd_xtra};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  if (ctx->stream2) (void)hipStreamDestroy(ctx->stream2);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  if (ctx->y_ev) (void)hipEventDestroy(ctx->y_ev);
  if (ctx->fork2_ev) (void)hipEventDestroy(ctx->fork2_ev);
  if (ctx->join2_ev) (void)hipEventDestroy(ctx->join2_ev);
  if (ctx->tabf_ev) (void)hipEventDestroy(ctx->tabf_ev);
  if (ctx->tab_ev) (void)hipEventDestroy(ctx->tab_ev);
  delete ctx;
  return QFLOW_OK;
}

const char* qflow_last_error(const qflow_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int qflow_load_integrals(qflow_ctx* ctx, int32_t n_orb, int32_t n_occ, const double* h,
                         const double* eri, double sym_tol) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (!h || !eri) return fail(ctx, QFLOW_E_INVALID_ARG, "h or eri is NULL");
  if (n_orb < 2 || n_orb > 128 || n_occ < 1 || n_occ >= n_orb || n_occ > 64)
    return fail(ctx, QFLOW_E_INVALID_ARG, "need 1 <= n_occ < n_orb <= 128 and n_occ <= 64");
  if (!(sym_tol >= 0.0)) return fail(ctx, QFLOW_E_INVALID_ARG, "sym_tol must be >= 0");
  QF_HIP(hipSetDevice(ctx->device));
  ctx->loaded = false;
  const int n = n_orb, o = n_occ, v = n - o;
  const size_t n2 = (size_t)n * n, n4 = n2 * n2, n2p = (size_t)n * (n + 1) / 2;
  ctx->n = n;
  ctx->o = o;
  ctx->v = v;
  const int nblk = 1024;
  QF_TRY(ensure(ctx, ctx->partial, sizeof(double) * nblk));
  qf::launch_sym_check(h, eri, n, P<double>(ctx->partial), nblk, ctx->stream);
  std::vector<double> part(nblk);
  QF_HIP(hipMemcpyAsync(part.data(), ctx->partial.p, sizeof(double) * nblk,
                        hipMemcpyDeviceToHost, ctx->stream));
  QF_HIP(hipStreamSynchronize(ctx->stream));
  double asym = 0.0;
  for (double x : part) asym = std::max(asym, std::isnan(x) ? INFINITY : x);
  if (!(asym <= sym_tol))
    return fail(ctx, QFLOW_E_SYMMETRY,
                "integrals not finite or not symmetric: max deviation " + std::to_string(asym));
  QF_TRY(ensure(ctx, ctx->f, sizeof(double) * n2));
  QF_TRY(ensure(ctx, ctx->V, sizeof(double) * n4));
  QF_TRY(ensure(ctx, ctx->W, sizeof(double) * n2p * v * v));
  QF_TRY(ensure(ctx, ctx->y1, sizeof(double) * n2));
  QF_TRY(ensure(ctx, ctx->y2, sizeof(double) * n4));
  QF_TRY(ensure(ctx, ctx->wy, sizeof(double) * n2p * v * v));
  QF_TRY(ensure(ctx, ctx->L, sizeof(double) * n2p * o * o));
  QF_TRY(ensure(ctx, ctx->LY, sizeof(double) * n2p * o * o));
  QF_TRY(ensure(ctx, ctx->r1, sizeof(double) * o * v));
  QF_TRY(ensure(ctx, ctx->r2, sizeof(double) * (size_t)o * o * v * v));
  QF_TRY(ensure(ctx, ctx->t1n, sizeof(double) * o * v));
  QF_TRY(ensure(ctx, ctx->t2n, sizeof(double) * (size_t)o * o * v * v));
  const size_t ov = (size_t)o * v;
  QF_TRY(ensure(ctx, ctx->ra_h, sizeof(double) * n2 * 2 * ov));
  QF_TRY(ensure(ctx, ctx->r22_h, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->ra_y, sizeof(double) * n2 * 2 * ov));
  QF_TRY(ensure(ctx, ctx->r22_y, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->rta, sizeof(double) * ov * 2 * ov));
  QF_TRY(ensure(ctx, ctx->rt22, sizeof(double) * ov * ov));
  QF_TRY(ensure(ctx, ctx->ga_h, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->g22_h, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->ga_y, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->g22_y, sizeof(double) * n2 * ov));
  QF_TRY(ensure(ctx, ctx->jh, sizeof(double) * 2 * n * v));
  QF_TRY(ensure(ctx, ctx->jy, sizeof(double) * 2 * n * v));
  const size_t kj = (size_t)o * o * v;
  QF_TRY(ensure(ctx, ctx->ja_h, sizeof(double) * 2 * n * kj));
  QF_TRY(ensure(ctx, ctx->ja_y, sizeof(double) * 2 * n * kj));
  QF_TRY(ensure(ctx, ctx->jb, sizeof(double) * 2 * v * kj));
  // split-K slices: up to 8 of the ladder output (n^2 o^2) or 128 of J (n v)
  // (also the one-body ring partials, 2*ceil(v/8)*n^2)
  QF_TRY(ensure(ctx, ctx->gpart,
                sizeof(double) * std::max({8 * n2 * o * o, (size_t)qf::kMaxSplits * n * v,
                                           2 * (size_t)((v + 7) / 8) * n2})));
  // stream2's products take the same split counts as on the main stream
  QF_TRY(ensure(ctx, ctx->gpart2, ctx->gpart.bytes));
  QF_TRY(ensure(ctx, ctx->zv, sizeof(double) * o * o * v * v));
  QF_TRY(ensure(ctx, ctx->zo, sizeof(double) * o * o * v * v));
  // Yg's two-body part, its ladder rows and LY vanish on fixed
  // orbital-class patterns for every sigma; the kernels never write those
  // entries, so they are zeroed here once
  qf::launch_fill(P<double>(ctx->y2), n4, 0.0, ctx->stream);
  qf::launch_fill(P<double>(ctx->wy), n2p * v * v, 0.0, ctx->stream);
  qf::launch_fill(P<double>(ctx->LY), n2p * o * o, 0.0, ctx->stream);
  QF_TRY(ensure(ctx, ctx->dtpart, sizeof(double) * qf::kFinishParts));
  QF_TRY(ensure(ctx, ctx->a12, sizeof(double) * (2 * n * v + n * o)));
  QF_TRY(ensure(ctx, ctx->t2T, sizeof(double) * 3 * o * o * v * v));
  QF_TRY(ensure(ctx, ctx->sp, sizeof(double) * 4 * n * o * o * v));
  QF_TRY(ensure(ctx, ctx->sq, sizeof(double) * 2 * n * o * v * v));
  QF_TRY(ensure(ctx, ctx->sp_f, sizeof(double) * 4 * n * o * o * v));
  QF_TRY(ensure(ctx, ctx->sq_f, sizeof(double) * 2 * n * o * v * v));
  QF_TRY(ensure(ctx, ctx->fs1, sizeof(double) * 2 * n * n));
  QF_TRY(ensure(ctx, ctx->c1h, sizeof(double) * n2));
  QF_TRY(ensure(ctx, ctx->c1y, sizeof(double) * n2));
  QF_TRY(ensure(ctx, ctx->lo_t, sizeof(double) * o * o * v * v));
  QF_TRY(ensure(ctx, ctx->lo_xh, sizeof(double) * o * o * o * o));
  QF_TRY(ensure(ctx, ctx->lo_xy, sizeof(double) * o * o * o * o));
  QF_TRY(ensure(ctx, ctx->lo_h, sizeof(double) * o * o * v * v));
  QF_TRY(ensure(ctx, ctx->lo_y, sizeof(double) * o * o * v * v));
  qf::launch_fock(h, eri, n, o, P<double>(ctx->f), ctx->stream);
  qf::launch_repack(eri, n, o, P<double>(ctx->V), P<double>(ctx->W), ctx->stream);
  qf::launch_pack_ring_A(P<double>(ctx->V), n, o, P<double>(ctx->ra_h), P<double>(ctx->r22_h),
                         ctx->stream);
  qf::launch_pack_j_A(P<double>(ctx->V), n, o, P<double>(ctx->ja_h),
                      P<double>(ctx->ja_h) + (size_t)n * o * o * v, ctx->stream);
  qf::launch_pack_x_oooo(P<double>(ctx->V), n, o, P<double>(ctx->lo_xh), ctx->stream);
  QF_HIP(hipGetLastError());
  ctx->fock.assign(n2, 0.0);
  std::vector<double> hh(n2);
  QF_HIP(hipMemcpyAsync(ctx->fock.data(), ctx->f.p, sizeof(double) * n2, hipMemcpyDeviceToHost,
                        ctx->stream));
  QF_HIP(hipMemcpyAsync(hh.data(), h, sizeof(double) * n2, hipMemcpyDeviceToHost, ctx->stream));
  QF_HIP(hipStreamSynchronize(ctx->stream));
  double e = 0.0;
  for (int k = 0; k < o; ++k) e += hh[(size_t)k * n + k] + ctx->fock[(size_t)k * n + k];
  ctx->e_ref = e;
  double sc[8] = {0, 0, 0, e, 0, 0, 0, 0};
  QF_HIP(hipMemcpy(ctx->scal.p, sc, sizeof(sc), hipMemcpyHostToDevice));
  ctx->loaded = true;
  ctx->h32_ready = false;
  ctx->diis_active = false;
  ++ctx->epoch;   // sizes may have changed without a reallocation
  ctx->hb_ready = false;
  ctx->last_spaces.clear();
  return QFLOW_OK;
}

int qflow_reference(qflow_ctx* ctx, double* e_ref, double* eps, double* fock) {
  QF_TRY(require_loaded(ctx));
  if (e_ref) *e_ref = ctx->e_ref;
  const int n = ctx->n;
  if (eps)
    for (int p = 0; p < n; ++p) eps[p] = ctx->fock[(size_t)p * n + p];
  if (fock) std::memcpy(fock, ctx->fock.data(), sizeof(double) * n * n);
  return QFLOW_OK;
}

int qflow_mp2_guess(qflow_ctx* ctx, double* t1, double* t2) {
  QF_TRY(require_loaded(ctx));
  if (!t1 || !t2) return fail(ctx, QFLOW_E_INVALID_ARG, "t1 or t2 is NULL");
  qf::launch_mp2(P<double>(ctx->f), P<double>(ctx->V), ctx->n, ctx->o, t1, t2, ctx->stream);
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

int qflow_residual(qflow_ctx* ctx, const double* t1, const double* t2, double* r1, double* r2,
                   double* e0, int precision) {
  QF_TRY(require_loaded(ctx));
  if (!t1 || !t2 || !r1 || !r2 || !e0)
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL array argument");
  QF_TRY(ensure_vdouble(ctx, 0, 1));
  QF_TRY(prepare(ctx, t1, t2, precision));
  qf::launch_residual(P<double>(ctx->f), P<double>(ctx->V), P<double>(ctx->y1),
                      P<double>(ctx->y2), P<double>(ctx->L), P<double>(ctx->LY), rings_of(ctx),
                      t1, t2, ctx->n, ctx->o, P<double>(ctx->scal), P<double>(ctx->c1h),
                      P<double>(ctx->c1y), P<double>(ctx->gpart), r1, r2, e0, ctx->stream);
  if (ctx->trunc == QFLOW_TRUNC_H) {
    qf::launch_vd_global(P<double>(ctx->V), t1, t2, ctx->n, ctx->o, P<double>(ctx->vd_wg),
                         ctx->stream);
    qf::launch_vd_resid(P<double>(ctx->vd_wg), t1, t2, ctx->n, ctx->o, r1, r2, e0, ctx->stream);
  }
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

int64_t qflow_heff_size(const qflow_space* s) {
  if (!s) return 0;
  const int64_t na = s->n_o + s->n_v;
  return 1 + na * na + na * na * na * na;
}

int64_t qflow_amp_size(const qflow_space* s) {
  if (!s) return 0;
  const int64_t nt1 = (int64_t)s->n_o * s->n_v;
  return nt1 + nt1 * nt1;
}

int64_t qflow_ci_size(const qflow_space* s) {
  if (!s || s->n_o < 1 || s->n_v < 0) return 0;
  const int na = s->n_o + s->n_v;
  int64_t ns = 1;
  for (int i = 0; i < s->n_o; ++i) ns = ns * (na - i) / (i + 1);
  return ns * ns;
}

namespace {

int check_offsets(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const int64_t* off,
                  int64_t (*size)(const qflow_space*), const char* what) {
  if (!off) return fail(ctx, QFLOW_E_INVALID_ARG, std::string(what) + " is NULL");
  for (int k = 0; k < K; ++k)
    if (off[k] < 0 || off[k + 1] - off[k] < size(&spaces[k]))
      return fail(ctx, QFLOW_E_INVALID_ARG,
                  std::string(what) + ": block " + std::to_string(k) + " too small");
  return QFLOW_OK;
}

// The downfolded Hamiltonians of the spaces in the class lists idx / cls_off
// (count = cls_off[3]; the whole list when idx is NULL), after the residual
// and zero-body parts of the pool (t1, t2).
// Wg = [V_N, sigma]_2, then 1/2 [[V_N, s]_2, s]_2 on every space's orbitals
// into vd_xtra (the list's order, offsets heff_off_dev)
int run_vdouble(qflow_ctx* ctx, int32_t K, const double* t1, const double* t2,
                const int64_t* heff_off_dev) {
  const int n = ctx->n, o = ctx->o;
  qf::launch_vd_global(P<double>(ctx->V), t1, t2, n, o, P<double>(ctx->vd_wg), ctx->stream);
  for (int k0 = 0; k0 < K; k0 += ctx->vd_batch)
    qf::launch_vd_spaces(P<double>(ctx->V), t1, t2, P<SpaceDev>(ctx->spaces), k0,
                         std::min(ctx->vd_batch, K - k0), n, o, P<double>(ctx->vd_wg),
                         P<double>(ctx->vd_wsp), heff_off_dev, P<double>(ctx->vd_xtra),
                         ctx->stream);
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

int run_heff(qflow_ctx* ctx, int32_t K, const double* t1, const double* t2, double* heff,
             const int64_t* heff_off_dev, const int32_t* idx = nullptr,
             const int* cls_off = nullptr) {
  if (!idx) {
    idx = P<int32_t>(ctx->cls_idx);
    cls_off = ctx->cls_off;
  } else {
    K = cls_off[3];
  }
  // the zsum parts need a block per space of the lists; they run on stream2
  // except in the stage-timed eager step, which keeps one stream (as in
  // prepare) and the same arithmetic.  With stream2 the per-space tables
  // (phase 0) run there too, beside the residual, whose outputs they do
  // not read.
  const bool use_zs = ctx->zsum.bytes >= sizeof(double) * zsum_doubles(cls_off);
  const bool split = K > 0 && use_zs && !ctx->timed;
  const bool vd = ctx->trunc == QFLOW_TRUNC_H;
  auto heff_phase = [&](hipStream_t s, bool dense, int phase) {
    return qf::launch_heff(P<double>(ctx->f), P<double>(ctx->V), P<double>(ctx->y1),
                           P<double>(ctx->y2), P<double>(ctx->L), P<double>(ctx->LY),
                           rings_of(ctx), t1, t2, ctx->n, ctx->o, P<double>(ctx->scal),
                           P<SpaceDev>(ctx->spaces), heff_off_dev, P<int32_t>(ctx->tasks),
                           qf::kTaskStride, ctx->task_slots, idx, cls_off, K, ctx->na_max,
                           P<double>(ctx->mtab), P<double>(ctx->fs1),
                           dense ? P<double>(ctx->zc) : nullptr,
                           dense ? P<double>(ctx->mp) : nullptr, heff, s,
                           use_zs ? P<double>(ctx->zsum) : nullptr,
                           ctx->timed ? nullptr : ctx->stream2, ctx->fork2_ev, ctx->join2_ev,
                           phase, vd && K > 0 ? P<double>(ctx->vd_xtra) : nullptr);
  };
  // the next truncation (whole lists only): Wg, then every space's extra
  // terms, on the main stream ahead of the residual that reads Wg
  if (vd) QF_TRY(run_vdouble(ctx, K, t1, t2, heff_off_dev));
  if (split) {
    QF_HIP(hipEventRecord(ctx->tabf_ev, ctx->stream));
    QF_HIP(hipStreamWaitEvent(ctx->stream2, ctx->tabf_ev, 0));
    QF_HIP(heff_phase(ctx->stream2, false, 0));
    QF_HIP(hipEventRecord(ctx->tab_ev, ctx->stream2));
  }
  // zero-body parts of [H_N, sigma] and [Yg, sigma] (scal[0], scal[1])
  qf::launch_residual(P<double>(ctx->f), P<double>(ctx->V), P<double>(ctx->y1),
                      P<double>(ctx->y2), P<double>(ctx->L), P<double>(ctx->LY), rings_of(ctx),
                      t1, t2, ctx->n, ctx->o, P<double>(ctx->scal), P<double>(ctx->c1h),
                      P<double>(ctx->c1y), P<double>(ctx->gpart), P<double>(ctx->r1),
                      P<double>(ctx->r2), nullptr, ctx->stream);
  if (vd)
    qf::launch_vd_resid(P<double>(ctx->vd_wg), t1, t2, ctx->n, ctx->o, P<double>(ctx->r1),
                        P<double>(ctx->r2), nullptr, ctx->stream);
  if (ctx->timed) QF_HIP(hipEventRecord(ctx->ev[8], ctx->stream));
  const size_t n = ctx->n;
  const size_t npair = n * (n + 1) / 2, oo = (size_t)ctx->o * ctx->o,
               vv = (size_t)ctx->v * ctx->v;
  const bool dense = K > 0 && z_dense_for(ctx, cls_off) &&
                     ctx->zc.bytes >= sizeof(double) * n * n * n * n &&
                     ctx->xp.bytes >= sizeof(double) * npair * oo &&
                     ctx->mp.bytes >= sizeof(double) * npair * vv;
  if (dense) {
    qf::launch_sigma1_x(P<double>(ctx->V), P<double>(ctx->y2), t1, ctx->n, ctx->o,
                        P<double>(ctx->zc), ctx->stream);
    qf::launch_pack_x_pairs(P<double>(ctx->V), P<double>(ctx->y2), ctx->n, ctx->o,
                            P<double>(ctx->xp), ctx->stream);
    qf::launch_gemm_nt_f64(P<double>(ctx->xp), P<double>(ctx->lo_t), P<double>(ctx->mp),
                           (int)npair, (int)vv, (int)oo, 1.0, P<double>(ctx->gpart),
                           ctx->gpart.bytes / sizeof(double), ctx->stream);
  }
  if (K > 0) {
    if (split) QF_HIP(hipStreamWaitEvent(ctx->stream, ctx->tab_ev, 0));
    QF_HIP(heff_phase(ctx->stream, dense, split ? 1 : -1));
  }
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

int run_solve(qflow_ctx* ctx, int32_t K, const double* heff, const int64_t* heff_off_dev,
              double* energy, double* c0, double* amp, const int64_t* amp_off_dev, double* ci,
              const int64_t* ci_off_dev, int32_t* iters, int32_t* status, double tol,
              int32_t max_iter, const int32_t* idx = nullptr, const int* cls_off = nullptr) {
  if (!idx) {
    idx = P<int32_t>(ctx->cls_idx);
    cls_off = ctx->cls_off;
  } else {
    K = cls_off[3];
  }
  if (K == 0) return QFLOW_OK;
  qf::DavidsonArgs a;
  a.spaces = P<SpaceDev>(ctx->spaces);
  a.strings = P<qf::Strings>(ctx->strings);
  a.heff = heff;
  a.heff_off = heff_off_dev;
  a.work = P<double>(ctx->work);
  a.work_off = P<int64_t>(ctx->work_off);
  a.energy = energy;
  a.c0 = c0;
  a.amp = amp;
  a.amp_off = amp_off_dev;
  a.ci = ci;
  a.ci_off = ci_off_dev;
  a.iters = iters;
  a.status = status;
  a.tol = tol;
  a.max_iter = max_iter;
  a.maxsub = kMaxSub;
  a.K = K;
  a.counter = P<int>(ctx->dav_counter);
  a.big_block = ctx->block_44;
  qf::launch_davidson(a, idx, cls_off, ctx->stream, ctx->dav_persistent != 0);
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

// QFLOW_E_UNSUPPORTED unless every size class present in cls_off has a VQE
// kernel whose workgroup fits the device's LDS.
int check_vqe(qflow_ctx* ctx, const int* cls_off) {
  for (int c = 0; c < 3; ++c) {
    if (cls_off[c + 1] == cls_off[c]) continue;
    const int bytes = qf::vqe_lds_bytes(c + 2);
    if (bytes < 0 || bytes > ctx->lds_limit)
      return fail(ctx, QFLOW_E_UNSUPPORTED,
                  "the VQE solver takes (2,2) and (3,3) spaces only");
  }
  return QFLOW_OK;
}

// UCCSD-VQE solve of every space of the uploaded list from the parameters
// theta0 (amp layout); results as run_solve's, with c0 = 1.
int run_vqe(qflow_ctx* ctx, const double* heff, const int64_t* heff_off_dev,
            const double* theta0, const int64_t* amp_off_dev, double* energy, double* amp,
            int32_t* iters, int32_t* status, double gtol, int max_iter) {
  const int K = ctx->cls_off[3];
  if (K == 0) return QFLOW_OK;
  QF_TRY(check_vqe(ctx, ctx->cls_off));
  qf::VqeArgs a;
  a.spaces = P<SpaceDev>(ctx->spaces);
  a.strings = P<qf::Strings>(ctx->strings);
  a.heff = heff;
  a.heff_off = heff_off_dev;
  a.theta0 = theta0;
  a.amp_off = amp_off_dev;
  a.energy = energy;
  a.c0 = P<double>(ctx->c0);
  a.amp = amp;
  a.iters = iters;
  a.status = status;
  a.gtol = gtol;
  a.max_iter = max_iter;
  a.K = K;
  qf::launch_vqe(a, P<int32_t>(ctx->cls_idx), ctx->cls_off, ctx->stream);
  QF_HIP(hipGetLastError());
  return QFLOW_OK;
}

// The device work of one flow step on ctx->stream: no allocation and no host
// synchronisation, so that it can be captured into a graph.
// With `timed` the stage boundaries are marked by events (not under capture).
int enqueue_step(qflow_ctx* ctx, int32_t K, const int32_t* owner1, const int32_t* owner2,
                 double* t1, double* t2, double* energy, int precision, bool step, bool diis,
                 bool timed, bool vqe = false) {
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  hipStream_t st = ctx->stream;
  ctx->timed = timed;
  if (timed) QF_HIP(hipEventRecord(ctx->ev[0], st));
  int r = prepare(ctx, t1, t2, precision);
  if (r == QFLOW_OK) {
    if (timed) QF_HIP(hipEventRecord(ctx->ev[7], st));
    r = run_heff(ctx, K, t1, t2, P<double>(ctx->heff), P<int64_t>(ctx->heff_off));
  }
  if (r == QFLOW_OK) {
    if (timed) QF_HIP(hipEventRecord(ctx->ev[9], st));
    if (vqe) {
      // every space starts from the pool's amplitudes of its orbitals
      qf::launch_gather_local(P<SpaceDev>(ctx->spaces), P<int64_t>(ctx->amp_off), t1, t2, n, o, K,
                              P<double>(ctx->vqe_theta), st);
      r = run_vqe(ctx, P<double>(ctx->heff), P<int64_t>(ctx->heff_off),
                  P<double>(ctx->vqe_theta), P<int64_t>(ctx->amp_off), P<double>(ctx->energy),
                  P<double>(ctx->amp), P<int32_t>(ctx->iters), P<int32_t>(ctx->status),
                  ctx->vqe_gtol, ctx->vqe_max_iter);
    } else {
      r = run_solve(ctx, K, P<double>(ctx->heff), P<int64_t>(ctx->heff_off),
                    P<double>(ctx->energy), P<double>(ctx->c0), P<double>(ctx->amp),
                    P<int64_t>(ctx->amp_off), P<double>(ctx->ci), P<int64_t>(ctx->ci_off),
                    P<int32_t>(ctx->iters), P<int32_t>(ctx->status), ctx->dav_tol,
                    ctx->dav_max_iter);
    }
  }
  ctx->timed = false;
  if (r != QFLOW_OK) return r;
  if (timed) QF_HIP(hipEventRecord(ctx->ev[10], st));
  qf::launch_update(t1, t2, P<double>(ctx->r1), P<double>(ctx->r2), P<double>(ctx->f), owner1,
                    owner2, n, o, step, P<double>(ctx->t1n), P<double>(ctx->t2n), st);
  if (K > 0)
    qf::launch_scatter_owned(P<SpaceDev>(ctx->spaces), P<double>(ctx->amp),
                             P<int64_t>(ctx->amp_off), P<int32_t>(ctx->status), owner1, owner2,
                             n, o, 0, K, P<double>(ctx->t1n), P<double>(ctx->t2n), st);
  if (diis)
    qf::launch_diis(t1, t2, o, v, P<double>(ctx->diis_t), P<double>(ctx->diis_e),
                    P<qf::DiisState>(ctx->diis_state), P<double>(ctx->diis_part),
                    P<double>(ctx->t1n), P<double>(ctx->t2n), st);
  qf::launch_finish(P<double>(ctx->energy), K, t1, t2, P<double>(ctx->t1n), P<double>(ctx->t2n),
                    o, v, P<double>(ctx->dtpart), P<double>(ctx->out2), st);
  // the new pool and energies into the caller's arrays (copy kernels, no
  // memory-copy nodes in a captured graph)
  qf::launch_copy(P<double>(ctx->t1n), t1, (size_t)o * v, st);
  qf::launch_copy(P<double>(ctx->t2n), t2, (size_t)o * o * v * v, st);
  if (K > 0) qf::launch_copy(P<double>(ctx->energy), energy, (size_t)K, st);
  QF_HIP(hipGetLastError());
  if (timed) QF_HIP(hipEventRecord(ctx->ev[11], st));
  return QFLOW_OK;
}

// Class lists of each window of W consecutive spaces of the uploaded list.
int build_windows(qflow_ctx* ctx, int32_t K, int32_t W) {
  if (ctx->win_size == W) return QFLOW_OK;
  const int nwin = std::max(1, (K + W - 1) / W);
  std::vector<int32_t> idx;
  ctx->win_base.assign(nwin, 0);
  ctx->win_off.assign(4 * nwin, 0);
  for (int w = 0; w < nwin; ++w) {
    const int k0 = w * W, k1 = std::min(K, k0 + W);
    ctx->win_base[w] = (int)idx.size();
    for (int c = 0; c < 3; ++c) {
      ctx->win_off[4 * w + c] = (int)idx.size() - ctx->win_base[w];
      for (int k = k0; k < k1; ++k)
        if (ctx->last_spaces[k].n_o - 2 == c) idx.push_back(k);
    }
    ctx->win_off[4 * w + 3] = (int)idx.size() - ctx->win_base[w];
  }
  idx.resize(std::max<size_t>(idx.size(), 1), 0);
  QF_TRY(ensure(ctx, ctx->win_idx, sizeof(int32_t) * idx.size()));
  QF_HIP(hipMemcpy(ctx->win_idx.p, idx.data(), sizeof(int32_t) * idx.size(),
                   hipMemcpyHostToDevice));
  ctx->win_size = W;
  return QFLOW_OK;
}

}  // namespace

int qflow_build_heff(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const double* t1,
                     const double* t2, double* heff, const int64_t* heff_off, int precision) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!t1 || !t2 || !heff) return fail(ctx, QFLOW_E_INVALID_ARG, "NULL array argument");
  QF_TRY(check_offsets(ctx, K, spaces, heff_off, qflow_heff_size, "heff_off"));
  QF_TRY(upload_spaces(ctx, K, spaces));
  QF_TRY(ensure_vdouble(ctx, K, heff_off[K]));
  DevBuf off;
  QF_TRY(ensure(ctx, off, sizeof(int64_t) * (K + 1)));
  hipError_t e = hipMemcpy(off.p, heff_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice);
  int r = (e == hipSuccess) ? prepare(ctx, t1, t2, precision)
                            : fail(ctx, QFLOW_E_DEVICE, "heff_off upload failed");
  if (r == QFLOW_OK) r = run_heff(ctx, K, t1, t2, heff, P<int64_t>(off));
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(off.p);
  return r;
}

int qflow_solve_active_batch(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                             const double* heff, const int64_t* heff_off, double* energy,
                             double* c0, double* amp, const int64_t* amp_off, double* ci_warm,
                             const int64_t* ci_off, int32_t* iters, int32_t* status, double tol,
                             int32_t max_iter) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!heff || !energy || !c0 || !amp || !iters || !status)
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL array argument");
  if (!(tol > 0.0) || max_iter < 1) return fail(ctx, QFLOW_E_INVALID_ARG, "bad tol or max_iter");
  QF_TRY(check_offsets(ctx, K, spaces, heff_off, qflow_heff_size, "heff_off"));
  QF_TRY(check_offsets(ctx, K, spaces, amp_off, qflow_amp_size, "amp_off"));
  if (ci_warm) QF_TRY(check_offsets(ctx, K, spaces, ci_off, qflow_ci_size, "ci_off"));
  QF_TRY(upload_spaces(ctx, K, spaces));
  DevBuf off;
  QF_TRY(ensure(ctx, off, sizeof(int64_t) * 3 * (K + 1)));
  int64_t* d_hoff = P<int64_t>(off);
  int64_t* d_aoff = d_hoff + (K + 1);
  int64_t* d_coff = d_aoff + (K + 1);
  int r = QFLOW_OK;
  if (hipMemcpy(d_hoff, heff_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(d_aoff, amp_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) != hipSuccess ||
      (ci_warm &&
       hipMemcpy(d_coff, ci_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) != hipSuccess))
    r = fail(ctx, QFLOW_E_DEVICE, "offset upload failed");
  if (r == QFLOW_OK)
    r = run_solve(ctx, K, heff, d_hoff, energy, c0, amp, d_aoff, ci_warm, ci_warm ? d_coff : nullptr,
                  iters, status, tol, max_iter);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(off.p);
  return r;
}

int qflow_solve_vqe_batch(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                          const double* heff, const int64_t* heff_off, const double* theta0,
                          double* amp, const int64_t* amp_off, double* energy, int32_t* iters,
                          int32_t* status, double gtol, int32_t max_iter) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!heff || !theta0 || !amp || !energy || !iters || !status)
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL array argument");
  if (!(gtol > 0.0) || max_iter < 0) return fail(ctx, QFLOW_E_INVALID_ARG, "bad gtol or max_iter");
  QF_TRY(check_offsets(ctx, K, spaces, heff_off, qflow_heff_size, "heff_off"));
  QF_TRY(check_offsets(ctx, K, spaces, amp_off, qflow_amp_size, "amp_off"));
  QF_TRY(upload_spaces(ctx, K, spaces));
  QF_TRY(check_vqe(ctx, ctx->cls_off));
  DevBuf off;
  QF_TRY(ensure(ctx, off, sizeof(int64_t) * 2 * (K + 1)));
  int64_t* d_hoff = P<int64_t>(off);
  int64_t* d_aoff = d_hoff + (K + 1);
  int r = QFLOW_OK;
  if (hipMemcpy(d_hoff, heff_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(d_aoff, amp_off, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) != hipSuccess)
    r = fail(ctx, QFLOW_E_DEVICE, "offset upload failed");
  if (r == QFLOW_OK)
    r = run_vqe(ctx, heff, d_hoff, theta0, d_aoff, energy, amp, iters, status, gtol, max_iter);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(off.p);
  return r;
}

int qflow_solve_active_batch_static(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                                    const double* heff, const int64_t* heff_off, double* energy,
                                    double* c0, double* amp, const int64_t* amp_off,
                                    double* ci_warm, const int64_t* ci_off, int32_t* iters,
                                    int32_t* status, double tol, int32_t max_iter) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!heff || !energy || !c0 || !amp || !iters || !status)
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL array argument");
  if (!(tol > 0.0) || max_iter < 1) return fail(ctx, QFLOW_E_INVALID_ARG, "bad tol or max_iter");
  QF_TRY(check_offsets(ctx, K, spaces, heff_off, qflow_heff_size, "heff_off"));
  QF_TRY(check_offsets(ctx, K, spaces, amp_off, qflow_amp_size, "amp_off"));
  if (ci_warm) QF_TRY(check_offsets(ctx, K, spaces, ci_off, qflow_ci_size, "ci_off"));
  if (!ctx->scratch) return fail(ctx, QFLOW_E_STATE, "no scratch address on this device");
  if (K == 0) return QFLOW_OK;
  QF_HIP(hipSetDevice(ctx->device));
  // host records of the list: space descriptors, class lists, work offsets
  std::vector<SpaceDev> dev(K);
  std::vector<int64_t> work_off(K + 1, 0);
  std::vector<int32_t> cls[3];
  int lds = 0;
  for (int k = 0; k < K; ++k) {
    const qflow_space& s = spaces[k];
    dev[k].na = na_of(s);
    dev[k].nocc = s.n_o;
    for (int a = 0; a < 8; ++a) dev[k].orb[a] = a < dev[k].na ? s.orb[a] : 0;
    const qf::DavLayout lay = qf::dav_layout(dev[k].na, s.n_o, kMaxSub);
    work_off[k + 1] = work_off[k] + lay.work;
    lds = std::max(lds, lay.lds);
    cls[s.n_o - 2].push_back(k);
  }
  if ((size_t)lds * sizeof(double) > (size_t)ctx->lds_limit)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "active space too large for the device's LDS");
  int cls_off[4];
  std::vector<int32_t> idx;
  for (int c = 0; c < 3; ++c) {
    cls_off[c] = (int)idx.size();
    idx.insert(idx.end(), cls[c].begin(), cls[c].end());
  }
  cls_off[3] = (int)idx.size();
  // scratch layout, each section 256-byte aligned: work counter of the
  // persistent launch | descriptors | class lists | heff, amp, ci and work
  // offsets | Davidson work areas
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_ctr = 256, b_sp = up(sizeof(SpaceDev) * K), b_idx = up(sizeof(int32_t) * K),
               b_off = up(sizeof(int64_t) * (K + 1));
  const size_t head = b_ctr + b_sp + b_idx + 4 * b_off;
  const size_t need = head + sizeof(double) * (size_t)work_off[K];
  if (need > (size_t)QFLOW_STATIC_SCRATCH_BYTES)
    return fail(ctx, QFLOW_E_UNSUPPORTED,
                "batch needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                    std::to_string((size_t)QFLOW_STATIC_SCRATCH_BYTES));
  std::vector<unsigned char> host(head, 0);
  std::memcpy(host.data() + b_ctr, dev.data(), sizeof(SpaceDev) * K);
  std::memcpy(host.data() + b_ctr + b_sp, idx.data(), sizeof(int32_t) * K);
  unsigned char* offs = host.data() + b_ctr + b_sp + b_idx;
  std::memcpy(offs, heff_off, sizeof(int64_t) * (K + 1));
  std::memcpy(offs + b_off, amp_off, sizeof(int64_t) * (K + 1));
  if (ci_warm) std::memcpy(offs + 2 * b_off, ci_off, sizeof(int64_t) * (K + 1));
  std::memcpy(offs + 3 * b_off, work_off.data(), sizeof(int64_t) * (K + 1));
  unsigned char* base = static_cast<unsigned char*>(ctx->scratch);
  unsigned char* d_offs = base + b_ctr + b_sp + b_idx;
  QF_HIP(hipMemcpyAsync(base, host.data(), head, hipMemcpyHostToDevice, ctx->stream));
  qf::DavidsonArgs a;
  a.spaces = reinterpret_cast<const SpaceDev*>(base + b_ctr);
  a.strings = P<qf::Strings>(ctx->strings);
  a.heff = heff;
  a.heff_off = reinterpret_cast<const int64_t*>(d_offs);
  a.work = reinterpret_cast<double*>(base + head);
  a.work_off = reinterpret_cast<const int64_t*>(d_offs + 3 * b_off);
  a.energy = energy;
  a.c0 = c0;
  a.amp = amp;
  a.amp_off = reinterpret_cast<const int64_t*>(d_offs + b_off);
  a.ci = ci_warm;
  a.ci_off = ci_warm ? reinterpret_cast<const int64_t*>(d_offs + 2 * b_off) : nullptr;
  a.iters = iters;
  a.status = status;
  a.tol = tol;
  a.max_iter = max_iter;
  a.maxsub = kMaxSub;
  a.K = K;
  a.counter = reinterpret_cast<int*>(base);
  a.big_block = ctx->block_44;
  qf::launch_davidson(a, reinterpret_cast<const int32_t*>(base + b_ctr + b_sp), cls_off,
                      ctx->stream, ctx->dav_persistent != 0);
  const hipError_t el = hipGetLastError();
  // the host records must outlive the copy
  QF_HIP(hipStreamSynchronize(ctx->stream));
  if (el != hipSuccess)
    return fail(ctx, QFLOW_E_DEVICE, std::string("davidson launch: ") + hipGetErrorString(el));
  return QFLOW_OK;
}

int qflow_flow_step(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const int32_t* owner1,
                    const int32_t* owner2, double* t1, double* t2, double* energy,
                    double* e_mean, double* max_dt, int32_t flags) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!owner1 || !owner2 || !t1 || !t2 || !e_mean || !max_dt || (K > 0 && !energy))
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL argument");
  const int precision = flags & 15;
  if (precision != QFLOW_FP64 && precision != QFLOW_FP32 && precision != QFLOW_BF16X3)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "unknown precision");
  QF_TRY(upload_spaces(ctx, K, spaces));
  // allocations and one-time conversions happen here, outside any capture
  if (precision == QFLOW_FP32) QF_TRY(ensure_mixed(ctx));
  if (precision == QFLOW_BF16X3) QF_TRY(ensure_bf16(ctx));
  const bool step = !(flags & QFLOW_UNOWNED_FROZEN);
  const bool diis = (flags & QFLOW_DIIS) != 0;
  const bool vqe = (flags & QFLOW_SOLVER_VQE) != 0;
  hipStream_t st = ctx->stream;
  QF_TRY(ensure_vdouble(ctx, K, ctx->h_heff_off[K]));
  if (vqe) {
    QF_TRY(check_vqe(ctx, ctx->cls_off));
    QF_TRY(ensure(ctx, ctx->vqe_theta, sizeof(double) * std::max<int64_t>(ctx->h_amp_off[K], 1)));
  }
  if (diis) {
    const size_t N = (size_t)ctx->o * ctx->v + (size_t)ctx->o * ctx->o * ctx->v * ctx->v;
    QF_TRY(ensure(ctx, ctx->diis_t, sizeof(double) * qf::kDiisMax * N));
    QF_TRY(ensure(ctx, ctx->diis_e, sizeof(double) * qf::kDiisMax * N));
    QF_TRY(ensure(ctx, ctx->diis_part, sizeof(double) * qf::kDiisMax * qf::kDiisParts));
    QF_TRY(ensure(ctx, ctx->diis_state, sizeof(qf::DiisState)));
    if (!ctx->diis_active) {   // start a history: zero the device state
      qf::launch_fill(P<double>(ctx->diis_state), sizeof(qf::DiisState) / sizeof(double), 0.0,
                      st);
      ctx->diis_active = true;
    }
  } else {
    ctx->diis_active = false;
  }
  if (flags & QFLOW_GRAPH) {
    const GraphKey key{K, flags, t1, t2, owner1, owner2, energy, ctx->epoch};
    if (!ctx->graph_exec || !(key == ctx->graph_key)) {
      if (ctx->graph_exec) {
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
      }
      QF_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const int r =
          enqueue_step(ctx, K, owner1, owner2, t1, t2, energy, precision, step, diis, false, vqe);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &graph);
      if (r != QFLOW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      if (e != hipSuccess)
        return fail(ctx, QFLOW_E_DEVICE, std::string("stream capture: ") + hipGetErrorString(e));
      const hipError_t ei = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        ctx->graph_exec = nullptr;
        return fail(ctx, QFLOW_E_DEVICE, std::string("graph instantiation: ") +
                                             hipGetErrorString(ei));
      }
      ctx->graph_key = key;
    }
    QF_HIP(hipEventRecord(ctx->ev[0], st));
    QF_HIP(hipGraphLaunch(ctx->graph_exec, st));
    QF_HIP(hipEventRecord(ctx->ev[kStages], st));
  } else {
    QF_TRY(enqueue_step(ctx, K, owner1, owner2, t1, t2, energy, precision, step, diis, true, vqe));
  }
  double out[2];
  QF_HIP(hipMemcpyAsync(out, ctx->out2.p, sizeof(out), hipMemcpyDeviceToHost, st));
  QF_HIP(hipStreamSynchronize(st));
  *e_mean = out[0];
  *max_dt = out[1];
  // stage times: Yg | ladder GEMM (H) | ladder GEMM (Yg) | ring packing | ring GEMMs | J |
  // Z | residual | heff | solve | update; a graph replay is timed as a whole
  for (int s = 0; s < kStages; ++s) {
    float ms = -1.f;
    if (!(flags & QFLOW_GRAPH) &&
        hipEventElapsedTime(&ms, ctx->ev[s], ctx->ev[s + 1]) != hipSuccess)
      ms = -1.f;
    ctx->stage_ms[s] = ms;
  }
  float total = -1.f;
  if (hipEventElapsedTime(&total, ctx->ev[0], ctx->ev[kStages]) != hipSuccess) total = -1.f;
  ctx->total_ms = total;
  return QFLOW_OK;
}

int qflow_flow_sweep_windowed(qflow_ctx* ctx, int32_t K, const qflow_space* spaces,
                              const int32_t* owner1, const int32_t* owner2, double* t1,
                              double* t2, double* energy, int32_t window, double* e_mean,
                              double* max_dt, int32_t flags) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!owner1 || !owner2 || !t1 || !t2 || !e_mean || !max_dt || (K > 0 && !energy))
    return fail(ctx, QFLOW_E_INVALID_ARG, "NULL argument");
  if (window < 1) return fail(ctx, QFLOW_E_INVALID_ARG, "window < 1");
  if (flags & (QFLOW_GRAPH | QFLOW_DIIS | QFLOW_SOLVER_VQE))
    return fail(ctx, QFLOW_E_UNSUPPORTED,
                "windowed sweeps take none of QFLOW_GRAPH, QFLOW_DIIS, QFLOW_SOLVER_VQE");
  if (ctx->trunc != QFLOW_TRUNC_F)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "windowed sweeps take the DUCC(2F) truncation only");
  const int precision = flags & 15;
  if (precision != QFLOW_FP64 && precision != QFLOW_FP32 && precision != QFLOW_BF16X3)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "unknown precision");
  QF_TRY(upload_spaces(ctx, K, spaces));
  if (precision == QFLOW_FP32) QF_TRY(ensure_mixed(ctx));
  if (precision == QFLOW_BF16X3) QF_TRY(ensure_bf16(ctx));
  QF_TRY(build_windows(ctx, K, window));
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  const size_t nt1 = (size_t)o * v, nt2 = nt1 * nt1;
  QF_TRY(ensure(ctx, ctx->t1s, sizeof(double) * nt1));
  QF_TRY(ensure(ctx, ctx->t2s, sizeof(double) * nt2));
  const bool step = !(flags & QFLOW_UNOWNED_FROZEN);
  hipStream_t st = ctx->stream;
  ctx->timed = false;
  qf::launch_copy(t1, P<double>(ctx->t1s), nt1, st);
  qf::launch_copy(t2, P<double>(ctx->t2s), nt2, st);
  const int nwin = (int)ctx->win_base.size();
  for (int w = 0; w < nwin; ++w) {
    const int32_t* idx = P<int32_t>(ctx->win_idx) + ctx->win_base[w];
    const int* off = &ctx->win_off[4 * w];
    const int k0 = w * window, count = off[3];
    // global intermediates and residual of the pool as it stands
    QF_TRY(prepare(ctx, t1, t2, precision));
    QF_TRY(run_heff(ctx, 0, t1, t2, P<double>(ctx->heff), P<int64_t>(ctx->heff_off), idx, off));
    // the unowned step takes the residual of the pool at the start of the
    // sweep (the first window's); its result is merged after the last window
    if (w == 0)
      qf::launch_update(t1, t2, P<double>(ctx->r1), P<double>(ctx->r2), P<double>(ctx->f),
                        owner1, owner2, n, o, step, P<double>(ctx->t1n), P<double>(ctx->t2n),
                        st);
    QF_TRY(run_solve(ctx, 0, P<double>(ctx->heff), P<int64_t>(ctx->heff_off),
                     P<double>(ctx->energy), P<double>(ctx->c0), P<double>(ctx->amp),
                     P<int64_t>(ctx->amp_off), P<double>(ctx->ci), P<int64_t>(ctx->ci_off),
                     P<int32_t>(ctx->iters), P<int32_t>(ctx->status), ctx->dav_tol,
                     ctx->dav_max_iter, idx, off));
    if (count > 0)
      qf::launch_scatter_owned(P<SpaceDev>(ctx->spaces), P<double>(ctx->amp),
                               P<int64_t>(ctx->amp_off), P<int32_t>(ctx->status), owner1, owner2,
                               n, o, k0, std::min(window, K - k0), t1, t2, st);
  }
  qf::launch_merge_unowned(P<double>(ctx->t1n), P<double>(ctx->t2n), owner1, owner2, o, v, t1, t2,
                           st);
  qf::launch_finish(P<double>(ctx->energy), K, P<double>(ctx->t1s), P<double>(ctx->t2s), t1, t2,
                    o, v, P<double>(ctx->dtpart), P<double>(ctx->out2), st);
  if (K > 0) qf::launch_copy(P<double>(ctx->energy), energy, (size_t)K, st);
  QF_HIP(hipGetLastError());
  double out[2];
  QF_HIP(hipMemcpyAsync(out, ctx->out2.p, sizeof(out), hipMemcpyDeviceToHost, st));
  QF_HIP(hipStreamSynchronize(st));
  *e_mean = out[0];
  *max_dt = out[1];
  return QFLOW_OK;
}

int qflow_set_z_mode(qflow_ctx* ctx, int mode) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (mode != QFLOW_Z_AUTO && mode != QFLOW_Z_SPACE && mode != QFLOW_Z_DENSE)
    return fail(ctx, QFLOW_E_INVALID_ARG, "unknown Z mode");
  QF_HIP(hipSetDevice(ctx->device));
  ctx->z_mode = mode;
  ++ctx->epoch;   // a captured step follows the mode
  return ensure_zc(ctx);
}

int qflow_last_solve(qflow_ctx* ctx, int32_t K, int32_t* iters, int32_t* status) {
  if (!ctx || K < 0) return QFLOW_E_INVALID_ARG;
  if (K != (int32_t)ctx->last_spaces.size())
    return fail(ctx, QFLOW_E_INVALID_ARG, "K differs from the last flow step's list");
  if (K == 0) return QFLOW_OK;
  QF_HIP(hipSetDevice(ctx->device));
  QF_HIP(hipStreamSynchronize(ctx->stream));
  if (iters)
    QF_HIP(hipMemcpy(iters, ctx->iters.p, sizeof(int32_t) * K, hipMemcpyDeviceToHost));
  if (status)
    QF_HIP(hipMemcpy(status, ctx->status.p, sizeof(int32_t) * K, hipMemcpyDeviceToHost));
  return QFLOW_OK;
}

int qflow_set_solver(qflow_ctx* ctx, double tol, int32_t max_iter) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (!(tol > 0.0) || max_iter < 1) return fail(ctx, QFLOW_E_INVALID_ARG, "bad tol or max_iter");
  ctx->dav_tol = tol;
  ctx->dav_max_iter = max_iter;
  ++ctx->epoch;   // a captured step holds the old values in its kernel arguments
  return QFLOW_OK;
}

int qflow_set_truncation(qflow_ctx* ctx, int truncation) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (truncation != QFLOW_TRUNC_F && truncation != QFLOW_TRUNC_H)
    return fail(ctx, QFLOW_E_INVALID_ARG, "unknown truncation");
  if (truncation == QFLOW_TRUNC_H && ctx->loaded && ctx->n > kTruncHMaxOrb)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "QFLOW_TRUNC_H takes at most 64 orbitals");
  ctx->trunc = truncation;
  ++ctx->epoch;   // a captured step follows the truncation
  return QFLOW_OK;
}

int qflow_set_vqe(qflow_ctx* ctx, double gtol, int32_t max_iter) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (!(gtol > 0.0) || max_iter < 0) return fail(ctx, QFLOW_E_INVALID_ARG, "bad gtol or max_iter");
  ctx->vqe_gtol = gtol;
  ctx->vqe_max_iter = max_iter;
  ++ctx->epoch;   // a captured step holds the old values in its kernel arguments
  return QFLOW_OK;
}

int qflow_set_tuning(qflow_ctx* ctx, const qflow_tuning* t) {
  if (!ctx) return QFLOW_E_INVALID_ARG;
  if (!t) return fail(ctx, QFLOW_E_INVALID_ARG, "NULL tuning");
  if ((t->davidson != QFLOW_DAV_PER_CLASS && t->davidson != QFLOW_DAV_PERSISTENT) ||
      t->split_target < 1 || t->split_target > 16 || t->f64_tile < 0 || t->f64_tile > 2 ||
      (t->z_mode != QFLOW_Z_AUTO && t->z_mode != QFLOW_Z_SPACE && t->z_mode != QFLOW_Z_DENSE) ||
      (t->block_44 != 512 && t->block_44 != 1024))
    return fail(ctx, QFLOW_E_INVALID_ARG, "tuning value out of range");
  ctx->dav_persistent = t->davidson;
  ctx->block_44 = t->block_44;
  ctx->split_target = t->split_target;
  ctx->f64_tile = t->f64_tile;
  return qflow_set_z_mode(ctx, t->z_mode);   // bumps the epoch (graph re-capture)
}

int qflow_get_tuning(const qflow_ctx* ctx, qflow_tuning* t) {
  if (!ctx || !t) return QFLOW_E_INVALID_ARG;
  t->davidson = ctx->dav_persistent;
  t->split_target = ctx->split_target;
  t->f64_tile = ctx->f64_tile;
  t->z_mode = ctx->z_mode;
  t->block_44 = ctx->block_44;
  return QFLOW_OK;
}

}  // extern "C"

namespace {

std::string tune_key(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, int flags) {
  int cls[3] = {0, 0, 0};
  for (int k = 0; k < K; ++k) ++cls[spaces[k].n_o - 2];
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << "n=" << ctx->n << " o=" << ctx->o << " classes=" << cls[0] << "/" << cls[1] << "/"
    << cls[2] << " precision=" << (flags & 15) << " graph=" << ((flags & QFLOW_GRAPH) ? 1 : 0)
    << " arch=" << arch;
  return k.str();
}

bool read_int_field(const std::string& line, const char* name, int* v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  return std::sscanf(line.c_str() + p + pat.size(), " %d", v) == 1;
}

// Entries of the cache file: one `"key": {...}` per line.
std::vector<std::pair<std::string, std::string>> read_cache(const char* path) {
  std::vector<std::pair<std::string, std::string>> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    const size_t b = a == std::string::npos ? a : line.find("\": {", a + 1);
    const size_t c = line.rfind('}');
    if (a == std::string::npos || b == std::string::npos || c == std::string::npos || c < b)
      continue;
    out.emplace_back(line.substr(a + 1, b - a - 1), line.substr(b + 3, c - b - 2));
  }
  return out;
}

bool write_cache(const char* path, const std::vector<std::pair<std::string, std::string>>& e) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return false;
  f << "{\n";
  for (size_t i = 0; i < e.size(); ++i)
    f << "\"" << e[i].first << "\": " << e[i].second << (i + 1 < e.size() ? ",\n" : "\n");
  f << "}\n";
  return (bool)f;
}

}  // namespace

extern "C" {

int qflow_autotune(qflow_ctx* ctx, int32_t K, const qflow_space* spaces, const int32_t* owner1,
                   const int32_t* owner2, const double* t1, const double* t2, int32_t flags,
                   const char* cache_path, qflow_tuning* out, char* report, int32_t report_len) {
  QF_TRY(require_loaded(ctx));
  QF_TRY(check_spaces(ctx, K, spaces));
  if (!owner1 || !owner2 || !t1 || !t2) return fail(ctx, QFLOW_E_INVALID_ARG, "NULL argument");
  const int precision = flags & 15;
  if (precision != QFLOW_FP64 && precision != QFLOW_FP32 && precision != QFLOW_BF16X3)
    return fail(ctx, QFLOW_E_UNSUPPORTED, "unknown precision");
  flags &= ~QFLOW_DIIS;
  QF_HIP(hipSetDevice(ctx->device));
  const std::string key = tune_key(ctx, K, spaces, flags);
  std::ostringstream rep;
  auto finish = [&](const qflow_tuning& t) {
    if (out) *out = t;
    if (report && report_len > 0) {
      const std::string r = rep.str();
      const size_t n = std::min((size_t)report_len - 1, r.size());
      std::memcpy(report, r.data(), n);
      report[n] = '\0';
    }
  };
  std::vector<std::pair<std::string, std::string>> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    for (auto& e : cache)
      if (e.first == key) {
        qflow_tuning t{};
        if (read_int_field(e.second, "davidson", &t.davidson) &&
            read_int_field(e.second, "split_target", &t.split_target) &&
            read_int_field(e.second, "f64_tile", &t.f64_tile) &&
            read_int_field(e.second, "z_mode", &t.z_mode) &&
            read_int_field(e.second, "block_44", &t.block_44) &&
            qflow_set_tuning(ctx, &t) == QFLOW_OK) {
          rep << "cached: " << key << " -> " << e.second << "\n";
          finish(t);
          return QFLOW_OK;
        }
      }
  }
  const size_t n1 = (size_t)ctx->o * ctx->v, n2 = n1 * n1;
  QF_TRY(ensure(ctx, ctx->tune_t1, sizeof(double) * n1));
  QF_TRY(ensure(ctx, ctx->tune_t2, sizeof(double) * n2));
  QF_TRY(ensure(ctx, ctx->tune_e, sizeof(double) * std::max(K, 1)));
  // one candidate: the same start pool, cold eigensolver starts, one untimed
  // and three timed flow steps
  auto measure = [&](const qflow_tuning& t, float* ms) -> int {
    QF_TRY(qflow_set_tuning(ctx, &t));
    QF_TRY(upload_spaces(ctx, K, spaces));
    qf::launch_copy(t1, P<double>(ctx->tune_t1), n1, ctx->stream);
    qf::launch_copy(t2, P<double>(ctx->tune_t2), n2, ctx->stream);
    qf::launch_fill(P<double>(ctx->ci), ctx->ci.bytes / sizeof(double), 0.0, ctx->stream);
    double em = 0.0, dt = 0.0;
    float total = 0.f;
    for (int s = 0; s < 4; ++s) {
      QF_TRY(qflow_flow_step(ctx, K, spaces, owner1, owner2, P<double>(ctx->tune_t1),
                             P<double>(ctx->tune_t2), P<double>(ctx->tune_e), &em, &dt, flags));
      if (s > 0) total += ctx->total_ms;
    }
    *ms = total / 3.f;
    rep << "davidson=" << t.davidson << " split_target=" << t.split_target
        << " f64_tile=" << t.f64_tile << " z_mode=" << t.z_mode << " block_44=" << t.block_44
        << ": " << *ms << " ms\n";
    return QFLOW_OK;
  };
  qflow_tuning best{};
  QF_TRY(qflow_get_tuning(ctx, &best));
  float best_ms = 0.f;
  QF_TRY(measure(best, &best_ms));
  bool has44 = false;
  for (int k = 0; k < K; ++k) has44 = has44 || spaces[k].n_o == 4;
  std::vector<std::vector<int>> values = {{QFLOW_DAV_PER_CLASS, QFLOW_DAV_PERSISTENT},
                                          {2, 4, 8},
                                          precision == QFLOW_FP64 ? std::vector<int>{0, 1, 2}
                                                                  : std::vector<int>{best.f64_tile},
                                          {QFLOW_Z_SPACE, QFLOW_Z_DENSE},
                                          has44 ? std::vector<int>{512, 1024}
                                                : std::vector<int>{best.block_44}};
  for (int d = 0; d < 5; ++d)
    for (int val : values[d]) {
      qflow_tuning c = best;
      int* field[5] = {&c.davidson, &c.split_target, &c.f64_tile, &c.z_mode, &c.block_44};
      if (*field[d] == val) continue;
      *field[d] = val;
      float ms = 0.f;
      QF_TRY(measure(c, &ms));
      if (ms < best_ms) {
        best = c;
        best_ms = ms;
      }
    }
  QF_TRY(qflow_set_tuning(ctx, &best));
  // the caller's next step: cold eigensolver starts, no DIIS history
  qf::launch_fill(P<double>(ctx->ci), ctx->ci.bytes / sizeof(double), 0.0, ctx->stream);
  ctx->diis_active = false;
  QF_HIP(hipStreamSynchronize(ctx->stream));
  rep << "chosen: davidson=" << best.davidson << " split_target=" << best.split_target
      << " f64_tile=" << best.f64_tile << " z_mode=" << best.z_mode
      << " block_44=" << best.block_44 << " (" << best_ms << " ms)\n";
  if (cache_path) {
    std::ostringstream v;
    v << "{\"davidson\": " << best.davidson << ", \"split_target\": " << best.split_target
      << ", \"f64_tile\": " << best.f64_tile << ", \"z_mode\": " << best.z_mode
      << ", \"block_44\": " << best.block_44 << ", \"ms\": " << best_ms << "}";
    bool found = false;
    for (auto& e : cache)
      if (e.first == key) {
        e.second = v.str();
        found = true;
      }
    if (!found) cache.emplace_back(key, v.str());
    if (!write_cache(cache_path, cache))
      return fail(ctx, QFLOW_E_INVALID_ARG, std::string("cannot write ") + cache_path);
  }
  finish(best);
  return QFLOW_OK;
}

int qflow_last_timings(const qflow_ctx* ctx, float* ms, int n) {
  if (!ctx || !ms) return 0;
  const int c = std::min(n, kStages + 1);
  for (int s = 0; s < c; ++s) ms[s] = s < kStages ? ctx->stage_ms[s] : ctx->total_ms;
  return c;
}

}  // extern "C"
