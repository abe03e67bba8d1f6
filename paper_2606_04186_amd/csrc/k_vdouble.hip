// The next DUCC truncation: 1/2 [[V_N, s]_2, s]_2 (V_N the two-body part of
// H_N, s = sigma_ext of a space), the paper's first lever on the correlation
// the DUCC(2F) expansion leaves out (closing paragraph of "Results").
//
// By bilinearity, with tau = sigma_int of the space,
//   W   = [V_N, s]_2 = [V_N, sigma]_2 - [V_N, tau]_2        (a dense operator
//         over all orbitals: the global Wg less a per-space part),
//   [W, s]_2 restricted to the space = [W, sigma]_2 - [W, tau]_2 on active
//         outputs.
// Every element is evaluated by the spin-free commutator of qflow_eval.h
// with direct loops (no global intermediates): Wg costs O(n^4 (o^2 + v^2 +
// o v)), each space's W a pass over n^4 elements and its active outputs
// O(na^4 n^2).  This is a path for small problems (the operator W of every
// space is materialised, n^4 doubles each, a batch of spaces at a time).
#include <hip/hip_runtime.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// V_N as the A operand: its two-body part V[p][q][r][s] = (pr|qs), no
// one-body part
struct TwoBodyOp {
  static constexpr bool kHasL = false;
  static constexpr bool kSparse3 = false;
  static constexpr bool kFull = false;
  const double* x2;
  int n;
  QF_HD double one(int, int) const { return 0.0; }
  QF_HD double two(int p, int q, int r, int s) const {
    return x2[(((size_t)p * n + q) * n + r) * n + s];
  }
  QF_HD bool act(int) const { return true; }
};

// A dense operator over all orbitals: two-body x2[n^4], then one-body x1[n^2],
// then the zero-body part (the layout of every W buffer)
struct DenseW {
  static constexpr bool kHasL = false;
  static constexpr bool kSparse3 = false;
  static constexpr bool kFull = false;
  const double* w;
  int n;
  QF_HD double one(int p, int q) const {
    return w[(size_t)n * n * n * n + (size_t)p * n + q];
  }
  QF_HD double two(int p, int q, int r, int s) const {
    return w[(((size_t)p * n + q) * n + r) * n + s];
  }
  QF_HD bool act(int) const { return true; }
};

QF_HD size_t w_size(int n) { return (size_t)n * n * n * n + (size_t)n * n + 1; }

// element e of a W buffer of [A, B]: two-body, one-body, zero-body
template <class AOp, class BOp>
__device__ double comm_element(const Comm<AOp, BOp>& c, size_t e, int n) {
  const size_t n2 = (size_t)n * n, n4 = n2 * n2;
  if (e < n4) {
    const int s = (int)(e % n), r = (int)(e / n % n), q = (int)(e / n2 % n), p = (int)(e / (n2 * n));
    return c.c2(p, q, r, s);
  }
  if (e < n4 + n2) {
    const size_t pq = e - n4;
    return c.c1((int)(pq / n), (int)(pq % n));
  }
  return c.c0();
}

__device__ void build_active(const SpaceDev& sp, Active& A) {
  if (threadIdx.x == 0) {
    A.na = sp.na;
    A.nocc = sp.nocc;
    for (int a = 0; a < kMaxAct; ++a) A.orb[a] = a < sp.na ? sp.orb[a] : 0;
  }
  for (int p = threadIdx.x; p < kMaxOrb; p += blockDim.x) A.pos[p] = -1;
  __syncthreads();
  if (threadIdx.x < sp.na) A.pos[sp.orb[threadIdx.x]] = (int8_t)threadIdx.x;
  __syncthreads();
}

// Wg = [V_N, sigma]_2
__global__ __launch_bounds__(256) void k_vd_global(const double* __restrict__ V,
                                                   const double* __restrict__ t1,
                                                   const double* __restrict__ t2, int n, int o,
                                                   double* wg) {
  const TwoBodyOp a{V, n};
  const Sigma s{t1, t2, n, o, n - o};
  const Comm<TwoBodyOp, Sigma> c{a, s, n, o};
  const size_t tot = w_size(n);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x)
    wg[e] = comm_element(c, e, n);
}

// W of spaces k0 .. k0 + gridDim.y - 1: Wg - [V_N, tau]_2
__global__ __launch_bounds__(256) void k_vd_space(const double* __restrict__ V,
                                                  const double* __restrict__ t1,
                                                  const double* __restrict__ t2,
                                                  const SpaceDev* __restrict__ spaces, int k0,
                                                  int n, int o, const double* __restrict__ wg,
                                                  double* wsp) {
  __shared__ Active A;
  build_active(spaces[k0 + blockIdx.y], A);
  const TwoBodyOp a{V, n};
  const Tau tau{Sigma{t1, t2, n, o, n - o}, &A};
  const Comm<TwoBodyOp, Tau> c{a, tau, n, o};
  const size_t tot = w_size(n);
  double* w = wsp + blockIdx.y * tot;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x)
    w[e] = wg[e] - comm_element(c, e, n);
}

// 1/2 ([W, sigma]_2 - [W, tau]_2) on the space's own orbitals, in the layout
// of its H_eff block before the CAS form: [x0, x1[na][na], x2[na][na][na][na]]
__global__ __launch_bounds__(256) void k_vd_add(const double* __restrict__ t1,
                                                const double* __restrict__ t2,
                                                const SpaceDev* __restrict__ spaces, int k0,
                                                int n, int o, const double* __restrict__ wsp,
                                                const int64_t* __restrict__ heff_off,
                                                double* xtra) {
  __shared__ Active A;
  const int k = k0 + blockIdx.x;
  build_active(spaces[k], A);
  const int na = A.na, n2 = na * na, n4 = n2 * n2;
  const DenseW w{wsp + blockIdx.x * w_size(n), n};
  const Sigma s{t1, t2, n, o, n - o};
  const Tau tau{s, &A};
  const Comm<DenseW, Sigma> cs{w, s, n, o};
  const Comm<DenseW, Tau> ct{w, tau, n, o};
  double* out = xtra + heff_off[k];
  for (int e = threadIdx.x; e < 1 + n2 + n4; e += blockDim.x) {
    double x;
    if (e == 0) {
      x = cs.c0() - ct.c0();
    } else if (e < 1 + n2) {
      const int p = A.orb[(e - 1) / na], q = A.orb[(e - 1) % na];
      x = cs.c1(p, q) - ct.c1(p, q);
    } else {
      const int f = e - 1 - n2;
      const int p = A.orb[f / (n2 * na)], q = A.orb[f / n2 % na], r = A.orb[f / na % na],
                s_ = A.orb[f % na];
      x = cs.c2(p, q, r, s_) - ct.c2(p, q, r, s_);
    }
    out[e] = 0.5 * x;
  }
}

// the residual's share: 1/2 [Wg, sigma]_2 projected on the doubles (a,b,i,j)
// and singles (a,i), and its zero-body part
__global__ __launch_bounds__(256) void k_vd_resid(const double* __restrict__ wg,
                                                  const double* __restrict__ t1,
                                                  const double* __restrict__ t2, int n, int o,
                                                  double* r1, double* r2, double* e0) {
  const int v = n - o;
  const DenseW w{wg, n};
  const Sigma s{t1, t2, n, o, v};
  const Comm<DenseW, Sigma> c{w, s, n, o};
  const size_t nd = (size_t)o * o * v * v, ns = (size_t)o * v;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nd + ns + 1;
       e += (size_t)gridDim.x * blockDim.x) {
    if (e < nd) {   // r2[i][j][a][b]
      const int b = (int)(e % v), a = (int)(e / v % v), j = (int)(e / ((size_t)v * v) % o),
                i = (int)(e / ((size_t)v * v * o));
      r2[e] += 0.5 * c.c2(o + a, o + b, i, j);
    } else if (e < nd + ns) {   // r1[i][a]
      const size_t ia = e - nd;
      const int i = (int)(ia / v), a = (int)(ia % v);
      r1[ia] += 0.5 * c.c1(o + a, i);
    } else if (e0) {
      *e0 += 0.5 * c.c0();
    }
  }
}

}  // namespace

size_t vd_space_doubles(int n) { return w_size(n); }

void launch_vd_global(const double* V, const double* t1, const double* t2, int n, int o,
                      double* wg, hipStream_t st) {
  k_vd_global<<<grid_for(w_size(n), kBlock, 65536), kBlock, 0, st>>>(V, t1, t2, n, o, wg);
}

void launch_vd_spaces(const double* V, const double* t1, const double* t2,
                      const SpaceDev* spaces, int k0, int kb, int n, int o, const double* wg,
                      double* wsp, const int64_t* heff_off, double* xtra, hipStream_t st) {
  if (kb <= 0) return;
  const unsigned bx = (unsigned)std::min<size_t>((w_size(n) + kBlock - 1) / kBlock, 1024);
  k_vd_space<<<dim3(bx, kb), kBlock, 0, st>>>(V, t1, t2, spaces, k0, n, o, wg, wsp);
  k_vd_add<<<kb, kBlock, 0, st>>>(t1, t2, spaces, k0, n, o, wsp, heff_off, xtra);
}

void launch_vd_resid(const double* wg, const double* t1, const double* t2, int n, int o,
                     double* r1, double* r2, double* e0, hipStream_t st) {
  const size_t v = n - o;
  k_vd_resid<<<grid_for((size_t)o * o * v * v + o * v + 1, kBlock, 65536), kBlock, 0, st>>>(
      wg, t1, t2, n, o, r1, r2, e0);
}

}  // namespace qf
