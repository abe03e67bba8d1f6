// Integral preparation, the [F,sigma] intermediate and the pool update.
#include <hip/hip_runtime.h>

#include <math.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// integral preparation
// ---------------------------------------------------------------------------

__global__ void k_sym_check(const double* __restrict__ h, const double* __restrict__ eri, int n,
                            double* partial) {
  const size_t n2 = (size_t)n * n, n4 = n2 * n2;
  double m = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n4;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(idx % n), r = (int)(idx / n % n), q = (int)(idx / n2 % n),
              p = (int)(idx / (n2 * n));
    const double x = eri[idx];
    if (!isfinite(x)) m = INFINITY;
    m = fmax(m, fabs(x - eri[(((size_t)q * n + p) * n + r) * n + s]));
    m = fmax(m, fabs(x - eri[(((size_t)p * n + q) * n + s) * n + r]));
    m = fmax(m, fabs(x - eri[(((size_t)r * n + s) * n + p) * n + q]));
    if (idx < n2) {
      const double y = h[idx];
      if (!isfinite(y)) m = INFINITY;
      m = fmax(m, fabs(y - h[(idx % n) * n + idx / n]));
    }
  }
  __shared__ double red[kBlock / 64];
  m = wave_max(m);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = red[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) x = fmax(x, red[w]);
    partial[blockIdx.x] = x;
  }
}

__global__ void k_fock(const double* __restrict__ h, const double* __restrict__ eri, int n, int o,
                       double* f) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int p = idx / n, q = idx % n;
  double x = h[idx];
  for (int k = 0; k < o; ++k)
    x += 2.0 * eri[(((size_t)p * n + q) * n + k) * n + k] - eri[(((size_t)p * n + k) * n + k) * n + q];
  f[idx] = x;
}

// V[p][q][r][s] = (pr|qs); W[(pq)][(cd)] = V[p][q][o+c][o+d]
__global__ void k_repack(const double* __restrict__ eri, int n, int o, double* V, double* W) {
  const size_t n2 = (size_t)n * n, n4 = n2 * n2;
  const int v = n - o;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n4;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(idx % n), r = (int)(idx / n % n), q = (int)(idx / n2 % n),
              p = (int)(idx / (n2 * n));
    const double x = eri[(((size_t)p * n + r) * n + q) * n + s];
    V[idx] = x;
    if (r >= o && s >= o && p <= q)
      W[tri_row(p, q, n) * v * v + (size_t)(r - o) * v + (s - o)] = x;
  }
}

__global__ void k_mp2(const double* __restrict__ f, const double* __restrict__ V, int n, int o,
                      double* t1, double* t2) {
  const int v = n - o;
  const size_t nt2 = (size_t)o * o * v * v;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nt2 + (size_t)o * v;
       idx += (size_t)gridDim.x * blockDim.x) {
    if (idx < nt2) {
      const int b = (int)(idx % v), a = (int)(idx / v % v), j = (int)(idx / v / v % o),
                i = (int)(idx / v / v / o);
      const double den = f[i * n + i] + f[j * n + j] - f[(o + a) * n + o + a] - f[(o + b) * n + o + b];
      t2[idx] = V[(((size_t)i * n + j) * n + o + a) * n + o + b] / den;
    } else {
      const size_t k = idx - nt2;
      const int i = (int)(k / v), a = (int)(k % v);
      t1[k] = f[i * n + o + a] / (f[i * n + i] - f[(o + a) * n + o + a]);
    }
  }
}

// ---------------------------------------------------------------------------
// Yg = [F_N, sigma] (dense two-body, one-body, zero-body) and its
// virtual-virtual block in ladder layout
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// U = [G, sigma_2]_2 for a Hermitian one-body G (G = f gives the two-body part
// of Yg = [F_N, sigma]; G = y1 the one-body-times-two-body part of
// [Yg, sigma]).  With sigma(a,b,i,j) = t2[i,j,a,b] = -sigma(i,j,a,b):
//   U_pqrs = [r~s, q!~r] sum_{t~q} G_pt sigma_tqrs + [r~s, p!~r] sum_{t~p} G_qt sigma_ptrs
//          - [p~q, s!~p] sum_{t~s} G_tr sigma_pqts - [p~q, r!~p] sum_{t~r} G_ts sigma_pqrt
// (~ = same occupied/virtual class).  The sums over virtual t are four
// matrix-core GEMMs over K = v with A1[p][t] = G[p][o+t], A2[p][t] = G[o+t][p]:
//   P1 = A1 t2T^T, P2 = A1 t2^T, P3 = A2 t2T^T, P4 = A2 t2^T   ([n][o*o*v] each)
// where t2 is read as [(i,j,a)][b] and t2T[i][j][b][a] = t2[i][j][a][b].  The
// sums over occupied t with r, s virtual are two GEMMs over K = o with
// Ao[p][t] = G[p][t] (t occupied), scaled by -1:
//   Q1 = -Ao Tq^T, Tq[(q,a,b)][t] = t2[t][q][a][b];  Q2 = -Ao Tp^T, Tp[(p,a,b)][t] = t2[p][t][a][b]
// ([n][o*v*v] each); those with p, q virtual are done while assembling.
// ---------------------------------------------------------------------------

__global__ void k_pack_onebody(const double* __restrict__ g, int n, int o, double* A1,
                               double* A2) {
  const int v = n - o;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * v) return;
  const int p = e / v, t = e % v;
  A1[e] = g[p * n + o + t];
  A2[e] = g[(o + t) * n + p];
}

__global__ void k_pack_onebody_occ(const double* __restrict__ g, int n, int o, double* Ao) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * o) return;
  Ao[e] = g[(e / o) * n + e % o];
}

// Tq[(q,a,b)][t] = t2[t][q][a][b], Tp[(p,a,b)][t] = t2[p][t][a][b]
__global__ void k_pack_t2_occ(const double* __restrict__ t2, int o, int v, double* Tq,
                              double* Tp) {
  const size_t vv = (size_t)v * v, tot = (size_t)o * o * vv;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e % o);
    const size_t row = e / o;
    const int i = (int)(row / vv);
    const size_t ab = row % vv;
    Tq[e] = t2[((size_t)t * o + i) * vv + ab];
    Tp[e] = t2[((size_t)i * o + t) * vv + ab];
  }
}

__global__ void k_pack_t2T(const double* __restrict__ t2, int o, int v, double* t2T) {
  const size_t tot = (size_t)o * o * v * v;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t ij = e / ((size_t)v * v);
    const int b = (int)(e / v % v), a = (int)(e % v);
    t2T[e] = t2[(ij * v + a) * v + b];
  }
}

// One workgroup per (p,q): the row U[p][q][:][:] (contiguous), and, for
// p <= q, its virtual-virtual part in ladder layout (row tri_row(p,q)) when
// wv is given.  Only the entries that can be non-zero for the (p,q) class are
// visited; the others were zeroed once when the arrays were allocated:
//   p, q occupied: all (r,s) but occupied-occupied (Q1 + Q2, P3, P4 terms)
//   one of p, q occupied: (r,s) both occupied (P1 or P2) or both virtual (Q2 or Q1)
//   p, q virtual: r or s occupied (P1 + P2 and the sums over occupied t of
//   g[t][r] t2[t][s][p][q] and g[t][s] t2[r][t][p][q], with g's occupied rows
//   and those t2 elements staged in LDS)
// Writers of the ladder rows: FP64, FP32, or BF16 hi/lo planes with rows
// padded to kp (padding zeroed once by the caller).
struct LadderRows {
  double* f64;
  float* f32;
  __bf16 *hi, *lo;
  size_t stride;   // elements per row
  __device__ bool on() const { return f64 || f32 || hi; }
  __device__ void put(size_t row, size_t k, double x) const {
    const size_t i = row * stride + k;
    if (f64) f64[i] = x;
    else if (f32) f32[i] = (float)x;
    else store_bf16_split(x, hi, lo, i);
  }
};

constexpr int kAssembleParts = 8;

template <class WT>
__global__ __launch_bounds__(256) void k_sigma2_assemble(const double* __restrict__ g,
                                                         const double* __restrict__ t2,
                                                         const double* __restrict__ P,
                                                         const double* __restrict__ Q, int n,
                                                         int o, double* U, WT wv) {
  extern __shared__ double sg[];   // p, q virtual: tpq[o*o] | g occupied rows [o][n]
  const int v = n - o;
  // workgroups [0, n^2): pair (p, q), part 0; after them, parts 1 ..
  // kAssembleParts-1 of the occupied pairs, whose rows are the longest
  int p, q, part = 0;
  if (blockIdx.x < (unsigned)(n * n)) {
    p = blockIdx.x / n;
    q = blockIdx.x % n;
  } else {
    const int j = blockIdx.x - n * n, pair = j / (kAssembleParts - 1);
    p = pair / o;
    q = pair % o;
    part = 1 + j % (kAssembleParts - 1);
  }
  const bool op = p < o, oq = q < o;
  const size_t ov2 = (size_t)o * o * v, nv = (size_t)n * ov2;
  const double* P1 = P;
  const double* P2 = P + nv;
  const double* P3 = P + 2 * nv;
  const double* P4 = P + 3 * nv;
  const size_t ovv = (size_t)o * v * v, vv = (size_t)v * v;
  const double* Q1 = Q;
  const double* Q2 = Q + (size_t)n * ovv;
  const size_t row = ((size_t)p * n + q) * n * n;
  const bool lad = wv.on() && p <= q;
  const size_t wrow = tri_row(p, q, n);
  if (op && oq) {
    const size_t pq = ((size_t)p * o + q) * v;
    for (int e = threadIdx.x + part * blockDim.x; e < n * n; e += kAssembleParts * blockDim.x) {
      const int r = e / n, s_ = e % n;
      if (r < o && s_ < o) continue;
      double x = 0.0;
      if (r >= o && s_ >= o) {
        const size_t rs = (size_t)(r - o) * v + (s_ - o);
        x += Q1[(size_t)p * ovv + (size_t)q * vv + rs];
        x += Q2[(size_t)q * ovv + (size_t)p * vv + rs];
      }
      if (s_ >= o) x += P3[(size_t)r * ov2 + pq + (s_ - o)];
      if (r >= o) x += P4[(size_t)s_ * ov2 + pq + (r - o)];
      U[row + e] = x;
      if (lad && r >= o && s_ >= o) wv.put(wrow, (size_t)(r - o) * v + (s_ - o), x);
    }
  } else if (op != oq) {
    const int o2 = o * o;
    for (int e = threadIdx.x; e < o2 + v * v; e += blockDim.x) {
      double x = 0.0;
      if (e < o2) {   // r, s occupied
        const int r = e / o, s_ = e % o;
        const size_t rs = ((size_t)r * o + s_) * v;
        x += op ? P1[(size_t)p * ov2 + rs + (q - o)] : P2[(size_t)q * ov2 + rs + (p - o)];
        U[row + (size_t)r * n + s_] = x;
      } else {        // r, s virtual
        const int f = e - o2, r = o + f / v, s_ = o + f % v;
        x += op ? Q2[(size_t)q * ovv + (size_t)p * vv + f] : Q1[(size_t)p * ovv + (size_t)q * vv + f];
        U[row + (size_t)r * n + s_] = x;
        if (lad) wv.put(wrow, f, x);
      }
    }
  } else {
    double* tpq = sg;
    double* go = sg + o * o;
    for (int e = threadIdx.x; e < o * o; e += blockDim.x)
      tpq[e] = t2[((size_t)e * v + (p - o)) * v + (q - o)];
    for (int e = threadIdx.x; e < o * n; e += blockDim.x) go[e] = g[e];
    __syncthreads();
    const int on = o * n;
    for (int e = threadIdx.x; e < on + v * o; e += blockDim.x) {
      int r, s_;
      if (e < on) {
        r = e / n;
        s_ = e % n;
      } else {
        r = o + (e - on) / o;
        s_ = (e - on) % o;
      }
      double x = 0.0;
      if (r < o && s_ < o) {
        const size_t rs = ((size_t)r * o + s_) * v;
        x += P1[(size_t)p * ov2 + rs + (q - o)];
        x += P2[(size_t)q * ov2 + rs + (p - o)];
      }
      if (s_ < o)
        for (int t = 0; t < o; ++t) x -= go[t * n + r] * tpq[t * o + s_];
      if (r < o)
        for (int t = 0; t < o; ++t) x -= go[t * n + s_] * tpq[r * o + t];
      U[row + (size_t)r * n + s_] = x;
    }
  }
}

// one wavefront per element of y1; the last wavefront computes the scalar
__global__ __launch_bounds__(256) void k_yg1(const double* __restrict__ f,
                                             const double* __restrict__ t1,
                                             const double* __restrict__ t2, int n, int o,
                                             double* y1, double* scal) {
  const int v = n - o;
  const int lane = threadIdx.x % 64;
  const int idx = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (idx > n * n) return;
  Yg Y{f, Sigma{t1, t2, n, o, v}, n, o, lane, 64};
  const double x = wave_sum(idx < n * n ? Y.one(idx / n, idx % n) : Y.zero());
  if (lane == 0) {
    if (idx < n * n)
      y1[idx] = x;
    else
      scal[2] = x;
  }
}

__global__ void k_fill(double* x, size_t count, double value) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    x[i] = value;
}

// ---------------------------------------------------------------------------
// pool update
// ---------------------------------------------------------------------------

__global__ void k_update(const double* __restrict__ t1, const double* __restrict__ t2,
                         const double* __restrict__ r1, const double* __restrict__ r2,
                         const double* __restrict__ f, const int32_t* __restrict__ owner1,
                         const int32_t* __restrict__ owner2, int n, int o, int step,
                         double* t1n, double* t2n) {
  const int v = n - o;
  const size_t nt2 = (size_t)o * o * v * v, tot = nt2 + (size_t)o * v;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    if (idx < nt2) {
      double x = t2[idx];
      if (step && owner2[idx] < 0) {
        const int b = (int)(idx % v), a = (int)(idx / v % v), j = (int)(idx / v / v % o),
                  i = (int)(idx / v / v / o);
        const double den = f[(o + a) * n + o + a] + f[(o + b) * n + o + b] - f[i * n + i] - f[j * n + j];
        x -= r2[idx] / den;
      }
      t2n[idx] = x;
    } else {
      const size_t e = idx - nt2;
      double x = t1[e];
      if (step && owner1[e] < 0) {
        const int i = (int)(e / v), a = (int)(e % v);
        x -= r1[e] / (f[(o + a) * n + o + a] - f[i * n + i]);
      }
      t1n[e] = x;
    }
  }
}

__global__ void k_scatter_owned(const SpaceDev* __restrict__ spaces, const double* __restrict__ amp,
                                const int64_t* __restrict__ amp_off,
                                const int32_t* __restrict__ status,
                                const int32_t* __restrict__ owner1,
                                const int32_t* __restrict__ owner2, int n, int o, int k0,
                                double* t1n, double* t2n) {
  const int k = k0 + blockIdx.x;
  if (status[k] != 0) return;
  const SpaceDev& sp = spaces[k];   // (a reference: no private copy to index)
  const int ne = sp.nocc, nv = sp.na - sp.nocc, v = n - o;
  const double* x = amp + amp_off[k];
  const int nt1 = ne * nv;
  for (int e = threadIdx.x; e < nt1 + nt1 * nt1; e += blockDim.x) {
    if (e < nt1) {
      const int i = sp.orb[e / nv], a = sp.orb[ne + e % nv] - o;
      if (owner1[i * v + a] == k) t1n[i * v + a] = x[e];
    } else {
      const int q = e - nt1;
      const int b = q % nv, a = q / nv % nv, j = q / (nv * nv) % ne, i = q / (nv * nv * ne);
      const int I = sp.orb[i], J = sp.orb[j], Av = sp.orb[ne + a] - o, Bv = sp.orb[ne + b] - o;
      const size_t g = (((size_t)I * o + J) * v + Av) * v + Bv;
      if (owner2[g] == k) t2n[g] = x[e];
    }
  }
}

// out[0] = mean energy (fixed summation order), out[1] = max |t_new - t_old|
// max |t_new - t_old| in two passes: per-block maxima, then one block
// combines them and forms the mean energy.
constexpr int kFinishBlocks = kFinishParts;

__global__ __launch_bounds__(256) void k_dt_max(const double* __restrict__ t1,
                                                const double* __restrict__ t2,
                                                const double* __restrict__ t1n,
                                                const double* __restrict__ t2n, int o, int v,
                                                double* part) {
  __shared__ double red[4];
  const size_t nt2 = (size_t)o * o * v * v, nt1 = (size_t)o * v;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double m = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt2; i += stride)
    m = fmax(m, fabs(t2n[i] - t2[i]));
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt1; i += stride)
    m = fmax(m, fabs(t1n[i] - t1[i]));
  m = wave_max(m);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ energy, int K,
                                                const double* __restrict__ part, int nparts,
                                                double* out) {
  __shared__ double rm[4], re[4];
  double m = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, part[i]);
  for (int k = threadIdx.x; k < K; k += blockDim.x) e += energy[k];
  m = wave_max(m);
  e = wave_sum(e);
  if (threadIdx.x % 64 == 0) {
    rm[threadIdx.x / 64] = m;
    re[threadIdx.x / 64] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (K > 0) ? (re[0] + re[1] + re[2] + re[3]) / K : 0.0;
    out[1] = fmax(fmax(rm[0], rm[1]), fmax(rm[2], rm[3]));
  }
}

// ---------------------------------------------------------------------------
// DIIS over the amplitude vector x = [t1 | t2] (N = o v + o^2 v^2 doubles)
// ---------------------------------------------------------------------------

// Store the plainly updated vector xn and its error e = xn - x in the slot of
// the new pair (count % kDiisMax), and the partial sums of e . E_j over this
// block for every held pair j (part[j * gridDim.x + block]).
__global__ __launch_bounds__(256) void k_diis_store(const double* __restrict__ t1n,
                                                    const double* __restrict__ t2n,
                                                    const double* __restrict__ t1,
                                                    const double* __restrict__ t2, int o, int v,
                                                    double* T, double* E,
                                                    const DiisState* __restrict__ state,
                                                    double* part) {
  __shared__ double red[4][kDiisMax];
  const size_t nt1 = (size_t)o * v, N = nt1 + (size_t)o * o * v * v;
  const int count = state->count;
  const int slot = count % kDiisMax;
  const int held = min(count + 1, kDiisMax);   // pairs held once this one is stored
  double acc[kDiisMax];
#pragma unroll
  for (int j = 0; j < kDiisMax; ++j) acc[j] = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double xn = i < nt1 ? t1n[i] : t2n[i - nt1];
    const double x = i < nt1 ? t1[i] : t2[i - nt1];
    const double e = xn - x;
    T[(size_t)slot * N + i] = xn;
    E[(size_t)slot * N + i] = e;
#pragma unroll
    for (int j = 0; j < kDiisMax; ++j)
      if (j < held) acc[j] += e * (j == slot ? e : E[(size_t)j * N + i]);
  }
#pragma unroll
  for (int j = 0; j < kDiisMax; ++j) {
    const double w = wave_sum(acc[j]);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64][j] = w;
  }
  __syncthreads();
  if (threadIdx.x < kDiisMax)
    part[threadIdx.x * gridDim.x + blockIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// One thread: sums the partials into the new row and column of B, counts the
// pair, and sets the extrapolation coefficients c (by slot): from the
// start-th pair on, the solution of [B 1; 1^T 0][c; lam] = [0; 1] over the
// held pairs (Gaussian elimination with partial pivoting; a pivot below
// kDiisPivotTol * max|B| drops the oldest pair and the system is solved
// again), else the newest vector alone.
__global__ void k_diis_solve(const double* __restrict__ part, int nparts, DiisState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int count = st->count;
  const int slot = count % kDiisMax;
  const int held = min(count + 1, kDiisMax);
  for (int j = 0; j < held; ++j) {
    double b = 0.0;
    for (int q = 0; q < nparts; ++q) b += part[j * nparts + q];
    st->B[slot * kDiisMax + j] = b;
    st->B[j * kDiisMax + slot] = b;
  }
  st->count = count + 1;
  for (int j = 0; j < kDiisMax; ++j) st->c[j] = 0.0;
  // held pairs in chronological order, oldest first
  int order[kDiisMax];
  for (int i = 0; i < held; ++i) order[i] = (count + 1 - held + i) % kDiisMax;
  if (count + 1 < kDiisStart) {
    st->c[slot] = 1.0;
    return;
  }
  for (int first = 0; first < held; ++first) {
    const int m = held - first;
    if (m == 1) break;
    double A[kDiisMax + 1][kDiisMax + 2];
    double scale = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        A[i][j] = st->B[order[first + i] * kDiisMax + order[first + j]];
        scale = fmax(scale, fabs(A[i][j]));
      }
    for (int i = 0; i < m; ++i) {
      A[i][m] = 1.0;
      A[m][i] = 1.0;
      A[i][m + 1] = 0.0;
    }
    A[m][m] = 0.0;
    A[m][m + 1] = 1.0;
    bool singular = false;
    for (int col = 0; col <= m && !singular; ++col) {
      int piv = col;
      for (int r = col + 1; r <= m; ++r)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      if (fabs(A[piv][col]) < kDiisPivotTol * scale) {
        singular = true;
        break;
      }
      if (piv != col)
        for (int c = 0; c <= m + 1; ++c) {
          const double tmp = A[col][c];
          A[col][c] = A[piv][c];
          A[piv][c] = tmp;
        }
      for (int r = col + 1; r <= m; ++r) {
        const double f = A[r][col] / A[col][col];
        for (int c = col; c <= m + 1; ++c) A[r][c] -= f * A[col][c];
      }
    }
    if (singular) continue;
    double x[kDiisMax + 1];
    for (int r = m; r >= 0; --r) {
      double y = A[r][m + 1];
      for (int c = r + 1; c <= m; ++c) y -= A[r][c] * x[c];
      x[r] = y / A[r][r];
    }
    for (int i = 0; i < m; ++i) st->c[order[first + i]] = x[i];
    return;
  }
  st->c[slot] = 1.0;
}

// x_out = sum_j c_j T_j over the held pairs, oldest first, into t1n / t2n.
__global__ __launch_bounds__(256) void k_diis_extrap(const double* __restrict__ T,
                                                     const DiisState* __restrict__ st, int o,
                                                     int v, double* t1n, double* t2n) {
  const size_t nt1 = (size_t)o * v, N = nt1 + (size_t)o * o * v * v;
  const int count = st->count;   // already includes the new pair
  const int held = min(count, kDiisMax);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    double x = 0.0;
    for (int q = 0; q < held; ++q) {
      const int j = (count - held + q) % kDiisMax;
      const double c = st->c[j];
      if (c != 0.0) x += c * T[(size_t)j * N + i];
    }
    if (i < nt1)
      t1n[i] = x;
    else
      t2n[i - nt1] = x;
  }
}

// ---------------------------------------------------------------------------
// ring intermediates: operand packing and the o^2 v one-body contraction
// ---------------------------------------------------------------------------

// K index of the ring contractions: k = u * v + (t - o), u occupied, t virtual.
// Aa[(a,b)][k]      = 2 X[a,u,b,t] - X[a,u,t,b],  Aa[(a,b)][ov + k] = -X[a,u,b,t]
// A22[(a,b)][k]     = X[a,u,t,b]
template <class T>
__global__ void k_pack_ring_A(const double* __restrict__ X, int n, int o, T* Aa, T* A22) {
  const int v = n - o;
  const size_t ov = (size_t)o * v, rows = (size_t)n * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < rows * ov;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / ov, k = idx % ov;
    const int a = (int)(row / n), b = (int)(row % n), u = (int)(k / v), t = o + (int)(k % v);
    const double x1 = X[(((size_t)a * n + u) * n + b) * n + t];
    const double x2 = X[(((size_t)a * n + u) * n + t) * n + b];
    Aa[row * 2 * ov + k] = (T)(2.0 * x1 - x2);
    Aa[row * 2 * ov + ov + k] = (T)(-x1);
    A22[row * ov + k] = (T)x2;
  }
}

// Ta[(g,d)][k] = t2[u,d,t,g], Ta[(g,d)][ov + k] = t2[d,u,t,g], T22[(g,d)][k] = t2[d,u,t,g]
// with row (g,d) = (g - o) * o + d.
template <class T>
__global__ void k_pack_ring_T(const double* __restrict__ t2, int o, int v, T* Ta, T* T22) {
  const size_t ov = (size_t)o * v;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ov * ov;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / ov, k = idx % ov;
    const int g = (int)(row / o), d = (int)(row % o), u = (int)(k / v), t = (int)(k % v);
    const double s1 = t2[(((size_t)u * o + d) * v + t) * v + g];
    const double s2 = t2[(((size_t)d * o + u) * v + t) * v + g];
    Ta[row * 2 * ov + k] = (T)s1;
    Ta[row * 2 * ov + ov + k] = (T)s2;
    T22[row * ov + k] = (T)s2;
  }
}

// The same operands as BF16 hi/lo planes (rows padded to a multiple of 32 k;
// the padding is zeroed once when the planes are allocated and never written).
// Workgroup (a, u, 32 consecutive b): the transposed operand X[a][u][t][b] is
// read row by row (b fastest) into LDS, then every output row segment (a, b;
// u, all virtual t) is written with t fastest, both reads of X coalesced.
constexpr int kRingTileB = 32;

__global__ __launch_bounds__(256) void k_pack_ring_A_bf16(const double* __restrict__ X, int n,
                                                          int o, __bf16* Ah, __bf16* Al, int kpa,
                                                          __bf16* A22h, __bf16* A22l, int kp22) {
  extern __shared__ double xt[];   // [v][kRingTileB + 1]: X[a][u][o+t][b0+bb]
  constexpr int LD = kRingTileB + 1;
  const int v = n - o, nbt = (n + kRingTileB - 1) / kRingTileB;
  const int a = blockIdx.x / (o * nbt), u = blockIdx.x / nbt % o,
            b0 = blockIdx.x % nbt * kRingTileB;
  const size_t ov = (size_t)o * v;
  const double* slab = X + ((size_t)a * n + u) * n * n;   // X[a][u][*][*]
  for (int e = threadIdx.x; e < v * kRingTileB; e += blockDim.x) {
    const int t = e / kRingTileB, bb = e % kRingTileB;
    xt[t * LD + bb] = b0 + bb < n ? slab[(size_t)(o + t) * n + b0 + bb] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < v * kRingTileB; e += blockDim.x) {
    const int bb = e / v, t = e % v, b = b0 + bb;
    if (b >= n) break;   // e grows with bb
    const double x1 = slab[(size_t)b * n + o + t];
    const double x2 = xt[t * LD + bb];
    const size_t row = (size_t)a * n + b, k = (size_t)u * v + t;
    store_bf16_split(2.0 * x1 - x2, Ah, Al, row * kpa + k);
    store_bf16_split(-x1, Ah, Al, row * kpa + ov + k);
    store_bf16_split(x2, A22h, A22l, row * kp22 + k);
  }
}

__global__ void k_pack_ring_T_bf16(const double* __restrict__ t2, int o, int v, __bf16* Th,
                                   __bf16* Tl, int kpa, __bf16* T22h, __bf16* T22l, int kp22) {
  const size_t ov = (size_t)o * v;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ov * ov;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / ov, k = idx % ov;
    const int g = (int)(row / o), d = (int)(row % o), u = (int)(k / v), t = (int)(k % v);
    const double s1 = t2[(((size_t)u * o + d) * v + t) * v + g];
    const double s2 = t2[(((size_t)d * o + u) * v + t) * v + g];
    store_bf16_split(s1, Th, Tl, row * kpa + k);
    store_bf16_split(s2, Th, Tl, row * kpa + ov + k);
    store_bf16_split(s2, T22h, T22l, row * kp22 + k);
  }
}

// Z(p,q,r,s) = sum_t sigma1(p,t) X(t,q,r,s) with X = Xh + Xy/2 (the two-body
// parts of H_N and Yg): the one-body part of sigma (t1) applied to the first
// index.  With X Hermitian and pair symmetric and sigma1 anti-Hermitian, the
// four terms of [X, sigma1]_2 are -(Z_pqrs + Z_qpsr + Z_rspq + Z_srqp).  The
// dense form, for calls whose spaces would gather more of X than n^4.
// sigma1(a,i) = t1[i][a], sigma1(i,a) = -t1[i][a].  One thread per column
// c = (q,r,s); t1 is staged in LDS (o*v doubles) and read by broadcast.
constexpr int kZChunk = 16;

// W adjacent columns per thread (W = 2: 16-byte loads and stores; the host
// picks W = 2 when n^3 is even).
template <int W>
__global__ __launch_bounds__(256) void k_sigma1_x(const double* __restrict__ Xh,
                                                  const double* __restrict__ Xy,
                                                  const double* __restrict__ t1, int n, int o,
                                                  double* Z) {
  typedef double vw __attribute__((ext_vector_type(W)));
  extern __shared__ double ts[];   // t1, o*v
  const int v = n - o;
  for (int e = threadIdx.x; e < o * v; e += blockDim.x) ts[e] = t1[e];
  __syncthreads();
  const size_t n3 = (size_t)n * n * n;
  const size_t c = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * W;
  if (c >= n3) return;
  auto ld = [&](int t) {
    return *reinterpret_cast<const vw*>(Xh + (size_t)t * n3 + c) +
           0.5 * *reinterpret_cast<const vw*>(Xy + (size_t)t * n3 + c);
  };
  // (plain stores: Z's lines that stay in the last-level cache serve the
  // lookups of the per-space kernels that follow)
  auto st = [&](int p, vw x) { *reinterpret_cast<vw*>(Z + (size_t)p * n3 + c) = x; };
  // p occupied: Z[p][c] = -sum_{t virtual} t1[p][t-o] X[t][c]; the column of
  // X is read eight rows at a time to keep several loads in flight.
  for (int p0 = 0; p0 < o; p0 += kZChunk) {
    vw acc[kZChunk];
#pragma unroll
    for (int i = 0; i < kZChunk; ++i) acc[i] = vw(0.0);
    int t = o;
    for (; t + 8 <= n; t += 8) {
      vw x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = ld(t + j);
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = 0; i < kZChunk; ++i)
          if (p0 + i < o) acc[i] -= ts[(p0 + i) * v + (t + j - o)] * x[j];
    }
    for (; t < n; ++t) {
      const vw x = ld(t);
#pragma unroll
      for (int i = 0; i < kZChunk; ++i)
        if (p0 + i < o) acc[i] -= ts[(p0 + i) * v + (t - o)] * x;
    }
#pragma unroll
    for (int i = 0; i < kZChunk; ++i)
      if (p0 + i < o) st(p0 + i, acc[i]);
  }
  // p virtual: Z[p][c] = sum_{t occupied} t1[t][p-o] X[t][c]
  for (int t0 = 0; t0 < o; t0 += kZChunk) {
    vw xo[kZChunk];
#pragma unroll
    for (int i = 0; i < kZChunk; ++i) xo[i] = (t0 + i < o) ? ld(t0 + i) : vw(0.0);
    for (int p = o; p < n; ++p) {
      vw acc = vw(0.0);
#pragma unroll
      for (int i = 0; i < kZChunk; ++i)
        if (t0 + i < o) acc += ts[(t0 + i) * v + (p - o)] * xo[i];
      if (t0 > 0) acc += *reinterpret_cast<const vw*>(Z + (size_t)p * n3 + c);
      st(p, acc);
    }
  }
}

// Operands of the occupied-occupied ladder Lo[(a,b)][(i,j)] =
// sum_{t,u occupied} t2[t,u,a,b] X(t,u,i,j):  T[(a,b)][(t,u)] = t2[t,u,a,b]
// (v*v rows) and Xo[(i,j)][(t,u)] = X[t,u,i,j] (o*o rows).
__global__ void k_pack_t2_vvoo(const double* __restrict__ t2, int o, int v, double* T) {
  const size_t oo = (size_t)o * o, tot = oo * v * v;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t ab = e / oo, tu = e % oo;
    T[e] = t2[tu * v * v + ab];
  }
}

__global__ void k_pack_x_oooo(const double* __restrict__ X, int n, int o, double* Xo) {
  const int oo = o * o;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= oo * oo) return;
  const int ij = e / oo, tu = e % oo;
  const int i = ij / o, j = ij % o, t = tu / o, u = tu % o;
  Xo[e] = X[(((size_t)t * n + u) * n + i) * n + j];
}

// Operands of the one-body ring terms as K-contiguous matrices over
// k = (t*o + u)*v + (w - o), t and u occupied, w virtual:
//   J1[p][q] = - sum_k X[w,p,t,u] (2 t2[t,u,w,q] - t2[t,u,q,w])
//   J2[p][q] = - sum_k (2 X[t,u,w,p] - X[t,u,p,w]) t2[t,u,w,q]
// A1[p][k] = X[w,p,t,u], A2[p][k] = 2 X[t,u,w,p] - X[t,u,p,w] (n rows each),
// B1[q][k] = 2 t2[t,u,w,q] - t2[t,u,q,w], B2[q][k] = t2[t,u,w,q] (v rows each).
__global__ __launch_bounds__(256) void k_pack_j_A(const double* __restrict__ X, int n, int o,
                                                  double* A1, double* A2) {
  const int v = n - o;
  const size_t K = (size_t)o * o * v;
  const size_t total = (size_t)n * K;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / K);
    const int k = (int)(e % K);
    const int w = o + k % v, u = k / v % o, t = k / (v * o);
    A1[e] = X[(((size_t)w * n + p) * n + t) * n + u];
    A2[e] = 2.0 * X[(((size_t)t * n + u) * n + w) * n + p] - X[(((size_t)t * n + u) * n + p) * n + w];
  }
}

__global__ __launch_bounds__(256) void k_pack_j_B(const double* __restrict__ t2, int o, int v,
                                                  double* B1, double* B2) {
  const size_t K = (size_t)o * o * v;
  const size_t total = (size_t)v * K;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(e / K);
    const int k = (int)(e % K);
    const int w = k % v, tu = k / v;   // w relative to o
    const double x = t2[((size_t)tu * v + w) * v + q];
    B1[e] = 2.0 * x - t2[((size_t)tu * v + q) * v + w];
    B2[e] = x;
  }
}

}  // namespace

void launch_sym_check(const double* h, const double* eri, int n, double* partial, int nblocks,
                      hipStream_t st) {
  k_sym_check<<<nblocks, kBlock, 0, st>>>(h, eri, n, partial);
}

void launch_fock(const double* h, const double* eri, int n, int o, double* f, hipStream_t st) {
  k_fock<<<grid_for((size_t)n * n), kBlock, 0, st>>>(h, eri, n, o, f);
}

void launch_repack(const double* eri, int n, int o, double* V, double* W, hipStream_t st) {
  const size_t n4 = (size_t)n * n * n * n;
  k_repack<<<grid_for(n4, kBlock, 65536), kBlock, 0, st>>>(eri, n, o, V, W);
}

void launch_mp2(const double* f, const double* V, int n, int o, double* t1, double* t2,
                hipStream_t st) {
  const size_t v = n - o;
  k_mp2<<<grid_for(o * o * v * v + o * v, kBlock, 65536), kBlock, 0, st>>>(f, V, n, o, t1, t2);
}

void launch_sigma2(const double* g, const double* t2, int n, int o, double* A12, double* t2T,
                   bool pack_t2, double* P, double* Q, double* part, size_t part_cap, double* U,
                   double* wv, float* wv32, __bf16* wvb_hi, __bf16* wvb_lo, hipStream_t st) {
  const int v = n - o;
  const size_t nv = (size_t)n * v, ov2 = (size_t)o * o * v, ovv = (size_t)o * v * v;
  const size_t o2v2 = (size_t)o * ovv;
  // scratch layout: A12 = [A1 | A2 | Ao], t2T = [t2T | Tq | Tp]
  double* Ao = A12 + 2 * nv;
  double* Tq = t2T + o2v2;
  double* Tp = Tq + o2v2;
  k_pack_onebody<<<grid_for(nv), kBlock, 0, st>>>(g, n, o, A12, A12 + nv);
  k_pack_onebody_occ<<<grid_for((size_t)n * o), kBlock, 0, st>>>(g, n, o, Ao);
  if (pack_t2) {
    k_pack_t2T<<<grid_for(o2v2, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, t2T);
    k_pack_t2_occ<<<grid_for(o2v2, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, Tq, Tp);
  }
  const double* pa[4] = {A12, A12, A12 + nv, A12 + nv};
  const double* pb[4] = {t2T, t2, t2T, t2};
  double* pc[4] = {P, P + n * ov2, P + 2 * n * ov2, P + 3 * n * ov2};
  (void)launch_gemm_nt_f64_batch(pa, pb, pc, 4, n, (int)ov2, v, 1.0, part, part_cap, st);
  const double* qa[2] = {Ao, Ao};
  const double* qb[2] = {Tq, Tp};
  double* qc[2] = {Q, Q + (size_t)n * ovv};
  (void)launch_gemm_nt_f64_batch(qa, qb, qc, 2, n, (int)ovv, o, -1.0, part, part_cap, st);
  const size_t lds = (size_t)(o * o + o * n) * sizeof(double);
  if (U) {
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sigma2_assemble<LadderRows>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const LadderRows rows{wv, wv32, wvb_hi, wvb_lo, wvb_hi ? (size_t)bf16_pad(v * v) : (size_t)v * v};
    k_sigma2_assemble<<<n * n + o * o * (kAssembleParts - 1), kBlock, lds, st>>>(g, t2, P, Q, n,
                                                                                  o, U, rows);
  }
}

void launch_yg1(const double* f, const double* t1, const double* t2, int n, int o, double* y1,
                double* scal, hipStream_t st) {
  k_yg1<<<grid_for(((size_t)n * n + 1) * 64), kBlock, 0, st>>>(f, t1, t2, n, o, y1, scal);
}

void launch_pack_ring_A(const double* X, int n, int o, double* Aa, double* A22, hipStream_t st) {
  const size_t work = (size_t)n * n * o * (n - o);
  k_pack_ring_A<<<grid_for(work, kBlock, 65536), kBlock, 0, st>>>(X, n, o, Aa, A22);
}

void launch_pack_ring_A(const double* X, int n, int o, float* Aa, float* A22, hipStream_t st) {
  const size_t work = (size_t)n * n * o * (n - o);
  k_pack_ring_A<<<grid_for(work, kBlock, 65536), kBlock, 0, st>>>(X, n, o, Aa, A22);
}

void launch_pack_ring_T(const double* t2, int o, int v, double* Ta, double* T22, hipStream_t st) {
  const size_t ov = (size_t)o * v;
  k_pack_ring_T<<<grid_for(ov * ov, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, Ta, T22);
}

void launch_pack_ring_A_bf16(const double* X, int n, int o, __bf16* Ah, __bf16* Al, __bf16* A22h,
                             __bf16* A22l, hipStream_t st) {
  const size_t ov = (size_t)o * (n - o);
  const int nbt = (n + kRingTileB - 1) / kRingTileB;
  const size_t lds = (size_t)(n - o) * (kRingTileB + 1) * sizeof(double);
  k_pack_ring_A_bf16<<<(unsigned)(n * o * nbt), kBlock, lds, st>>>(
      X, n, o, Ah, Al, bf16_pad((int)(2 * ov)), A22h, A22l, bf16_pad((int)ov));
}

void launch_pack_ring_T_bf16(const double* t2, int o, int v, __bf16* Th, __bf16* Tl, __bf16* T22h,
                             __bf16* T22l, hipStream_t st) {
  const size_t ov = (size_t)o * v;
  k_pack_ring_T_bf16<<<grid_for(ov * ov, kBlock, 65536), kBlock, 0, st>>>(
      t2, o, v, Th, Tl, bf16_pad((int)(2 * ov)), T22h, T22l, bf16_pad((int)ov));
}

void launch_pack_ring_T(const double* t2, int o, int v, float* Ta, float* T22, hipStream_t st) {
  const size_t ov = (size_t)o * v;
  k_pack_ring_T<<<grid_for(ov * ov, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, Ta, T22);
}

void launch_sigma1_x(const double* Xh, const double* Xy, const double* t1, int n, int o,
                     double* Z, hipStream_t st) {
  const size_t n3 = (size_t)n * n * n;
  const size_t lds = (size_t)o * (n - o) * sizeof(double);
  if (n3 % 2 == 0)
    k_sigma1_x<2><<<(unsigned)((n3 / 2 + kBlock - 1) / kBlock), kBlock, lds, st>>>(Xh, Xy, t1,
                                                                                   n, o, Z);
  else
    k_sigma1_x<1><<<(unsigned)((n3 + kBlock - 1) / kBlock), kBlock, lds, st>>>(Xh, Xy, t1, n, o,
                                                                               Z);
}

void launch_pack_t2_vvoo(const double* t2, int o, int v, double* T, hipStream_t st) {
  k_pack_t2_vvoo<<<grid_for((size_t)o * o * v * v, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, T);
}

void launch_pack_x_oooo(const double* X, int n, int o, double* Xo, hipStream_t st) {
  k_pack_x_oooo<<<grid_for((size_t)o * o * o * o), kBlock, 0, st>>>(X, n, o, Xo);
}

void launch_pack_j_A(const double* X, int n, int o, double* A1, double* A2, hipStream_t st) {
  const size_t total = (size_t)n * o * o * (n - o);
  k_pack_j_A<<<grid_for(total, kBlock, 65536), kBlock, 0, st>>>(X, n, o, A1, A2);
}

void launch_pack_j_B(const double* t2, int o, int v, double* B1, double* B2, hipStream_t st) {
  const size_t total = (size_t)v * o * o * v;
  k_pack_j_B<<<grid_for(total, kBlock, 65536), kBlock, 0, st>>>(t2, o, v, B1, B2);
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void launch_copy(const double* src, double* dst, size_t count, hipStream_t st) {
  k_copy<<<grid_for(count, kBlock, 65536), kBlock, 0, st>>>(src, dst, count);
}

void launch_fill(double* x, size_t count, double value, hipStream_t st) {
  k_fill<<<grid_for(count, kBlock, 65536), kBlock, 0, st>>>(x, count, value);
}

void launch_update(const double* t1, const double* t2, const double* r1, const double* r2,
                   const double* f, const int32_t* owner1, const int32_t* owner2, int n, int o,
                   bool unowned_step, double* t1n, double* t2n, hipStream_t st) {
  const size_t v = n - o;
  k_update<<<grid_for(o * o * v * v + o * v, kBlock, 65536), kBlock, 0, st>>>(
      t1, t2, r1, r2, f, owner1, owner2, n, o, unowned_step ? 1 : 0, t1n, t2n);
}

void launch_scatter_owned(const SpaceDev* spaces, const double* amp, const int64_t* amp_off,
                          const int32_t* status, const int32_t* owner1, const int32_t* owner2,
                          int n, int o, int k0, int K, double* t1n, double* t2n, hipStream_t st) {
  k_scatter_owned<<<K, kBlock, 0, st>>>(spaces, amp, amp_off, status, owner1, owner2, n, o, k0,
                                         t1n, t2n);
}

// The inverse of the write-back without ownership: space k's slice of the
// pool in the local amplitude layout (t1[I][A], then t2[I][J][A][B]).
__global__ void k_gather_local(const SpaceDev* __restrict__ spaces,
                               const int64_t* __restrict__ amp_off, const double* __restrict__ t1,
                               const double* __restrict__ t2, int n, int o, double* out) {
  const int k = blockIdx.x;
  const SpaceDev& sp = spaces[k];
  const int ne = sp.nocc, nv = sp.na - sp.nocc, v = n - o;
  double* x = out + amp_off[k];
  const int nt1 = ne * nv;
  for (int e = threadIdx.x; e < nt1 + nt1 * nt1; e += blockDim.x) {
    if (e < nt1) {
      x[e] = t1[sp.orb[e / nv] * v + sp.orb[ne + e % nv] - o];
    } else {
      const int q = e - nt1;
      const int b = q % nv, a = q / nv % nv, j = q / (nv * nv) % ne, i = q / (nv * nv * ne);
      const int I = sp.orb[i], J = sp.orb[j], Av = sp.orb[ne + a] - o, Bv = sp.orb[ne + b] - o;
      x[e] = t2[(((size_t)I * o + J) * v + Av) * v + Bv];
    }
  }
}

void launch_gather_local(const SpaceDev* spaces, const int64_t* amp_off, const double* t1,
                         const double* t2, int n, int o, int K, double* out, hipStream_t st) {
  if (K <= 0) return;
  k_gather_local<<<K, kBlock, 0, st>>>(spaces, amp_off, t1, t2, n, o, out);
}

__global__ void k_merge_unowned(const double* __restrict__ t1n, const double* __restrict__ t2n,
                                const int32_t* __restrict__ owner1,
                                const int32_t* __restrict__ owner2, size_t nt1, size_t nt2,
                                double* t1, double* t2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt1 + nt2;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < nt2) {
      if (owner2[i] < 0) t2[i] = t2n[i];
    } else if (owner1[i - nt2] < 0) {
      t1[i - nt2] = t1n[i - nt2];
    }
  }
}

void launch_merge_unowned(const double* t1n, const double* t2n, const int32_t* owner1,
                          const int32_t* owner2, int o, int v, double* t1, double* t2,
                          hipStream_t st) {
  const size_t nt1 = (size_t)o * v, nt2 = nt1 * nt1;
  k_merge_unowned<<<grid_for(nt1 + nt2, kBlock, 65536), kBlock, 0, st>>>(t1n, t2n, owner1,
                                                                          owner2, nt1, nt2, t1, t2);
}

void launch_diis(const double* t1, const double* t2, int o, int v, double* T, double* E,
                 DiisState* state, double* part, double* t1n, double* t2n, hipStream_t st) {
  k_diis_store<<<kDiisParts, kBlock, 0, st>>>(t1n, t2n, t1, t2, o, v, T, E, state, part);
  k_diis_solve<<<1, 64, 0, st>>>(part, kDiisParts, state);
  const size_t N = (size_t)o * v + (size_t)o * o * v * v;
  k_diis_extrap<<<grid_for(N, kBlock, 65536), kBlock, 0, st>>>(T, state, o, v, t1n, t2n);
}

void launch_finish(const double* energy, int K, const double* t1, const double* t2,
                   const double* t1n, const double* t2n, int o, int v, double* part,
                   double* out2, hipStream_t st) {
  k_dt_max<<<kFinishBlocks, kBlock, 0, st>>>(t1, t2, t1n, t2n, o, v, part);
  k_finish<<<1, kBlock, 0, st>>>(energy, K, part, kFinishBlocks, out2);
}

}  // namespace qf
