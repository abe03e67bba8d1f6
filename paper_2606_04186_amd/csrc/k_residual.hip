// Global residual of the transformed Hamiltonian.
#include <hip/hip_runtime.h>

#include <math.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// residual of Hbar(sigma)
// ---------------------------------------------------------------------------

// Workgroup (a, bc virtual b starting at b0): the elements (a, b; i, j) are
// evaluated with (i, j) fastest, so that the lookups (X, L, Lo, Ga, G22, ...
// all [..][i][j]) run along memory, into LDS, then written to r2[i][j][a][b]
// with b fastest.  bc is a power of two with bc o^2 <= 8192 (at most 16).
__global__ __launch_bounds__(256) void k_residual2(GlobalOps g, int bc, double* r2) {
  extern __shared__ double rt[];   // [bc][o*o]
  const int n = g.n, o = g.o, v = n - o, oo = o * o;
  const int nbc = (v + bc - 1) / bc;
  const int a = blockIdx.x / nbc, b0 = blockIdx.x % nbc * bc;
  const float inv_o = 1.0f / (float)o;
  const Sigma s{g.t1, g.t2, n, o, v};
  const DenseOp H{g.f, g.V, g.L, n, o, g.ga_h, g.g22_h, g.j1_h, g.j2_h, g.u_h, g.lo_h};
  const DenseOp Y{g.y1, g.y2, g.LY, n, o, g.ga_y, g.g22_y, g.j1_y, g.j2_y, nullptr, g.lo_y,
                   Sigma2Lazy{g.y1, g.t2, g.s2p, g.s2q, n, o}};
  const auto cH = make_comm(H, s, n, o);
  const auto cY = make_comm(Y, s, n, o);
  for (int bb = 0; bb < bc && b0 + bb < v; ++bb)
    for (int ij = threadIdx.x; ij < oo; ij += blockDim.x) {
      const int b = b0 + bb;
      // i = ij / o in single precision ((ij + 1/2)/o is at least 1/(2o) from
      // an integer; ij < 2^12)
      const int i = (int)(((float)ij + 0.5f) * inv_o), j = ij - i * o;
      const int pa = o + a, pb = o + b;
      // the sigma1 x two-body part of both commutators, -(Z_abij + Z_baji +
      // Z_ijab + Z_jiba) of H_N + Yg/2, from the pieces of k_zv and k_zo
      const double w = g.zv[(((size_t)a * v + b) * o + i) * o + j] +
                       g.zv[(((size_t)b * v + a) * o + j) * o + i] +
                       g.zo[(((size_t)i * o + j) * v + a) * v + b] +
                       g.zo[(((size_t)j * o + i) * v + b) * v + a];
      rt[bb * oo + ij] = H.two(pa, pb, i, j) + cH.c2(pa, pb, i, j) + 0.5 * cY.c2(pa, pb, i, j) - w;
    }
  __syncthreads();
  const int lbc = __ffs(bc) - 1;   // bc = 2^lbc
  for (int e = threadIdx.x; e < oo * bc; e += blockDim.x) {
    const int ij = e >> lbc, bb = e & (bc - 1);
    if (b0 + bb < v) r2[((size_t)ij * v + a) * v + b0 + bb] = rt[bb * oo + ij];
  }
}

// Z = sigma1 X over the first index, X = H_N + Yg/2 (two-body parts; both
// Hermitian and pair symmetric), on the two orbital classes the residual
// needs (a, b virtual; i, j occupied; sigma1(a,k) = t1[k][a],
// sigma1(i,c) = -t1[i][c]):
//   zv[a][b][i][j] = Z_abij =  sum_{k occ} t1[k][a] X[k][b][i][j]
//   zo[i][j][a][b] = Z_ijab = -sum_{c vir} t1[i][c] X[c][j][a][b]
// One thread per element of zv (j fastest; the o v o o block of X is small
// and stays in cache).
__global__ void k_zv(const double* __restrict__ Xh, const double* __restrict__ Xy,
                     const double* __restrict__ t1, int n, int o, double* zv) {
  const int v = n - o;
  const size_t tot = (size_t)v * v * o * o;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % o), i = (int)(e / o % o), b = (int)(e / o / o % v),
              a = (int)(e / o / o / v);
    double z = 0.0;
    for (int k = 0; k < o; ++k) {
      const size_t x = (((size_t)k * n + o + b) * n + i) * n + j;
      z += t1[k * v + a] * (Xh[x] + 0.5 * Xy[x]);
    }
    zv[e] = z;
  }
}

// zo: workgroup (j, a), one thread per b; the rows X[c][j][a][*] are read
// coalesced and t1 is staged in LDS (o*v doubles).
__global__ __launch_bounds__(128) void k_zo(const double* __restrict__ Xh,
                                            const double* __restrict__ Xy,
                                            const double* __restrict__ t1, int n, int o,
                                            double* zo) {
  extern __shared__ double ts[];
  const int v = n - o;
  for (int e = threadIdx.x; e < o * v; e += blockDim.x) ts[e] = t1[e];
  __syncthreads();
  const int j = blockIdx.x / v, a = blockIdx.x % v;
  constexpr int kChunk = 16;   // occupied i per pass over the rows
  for (int b = threadIdx.x; b < v; b += blockDim.x)
    for (int i0 = 0; i0 < o; i0 += kChunk) {
      double acc[kChunk];
#pragma unroll
      for (int i = 0; i < kChunk; ++i) acc[i] = 0.0;
#pragma unroll 4
      for (int c = 0; c < v; ++c) {
        const size_t x = (((size_t)(o + c) * n + j) * n + o + a) * n + o + b;
        const double xv = Xh[x] + 0.5 * Xy[x];
#pragma unroll
        for (int i = 0; i < kChunk; ++i)
          if (i0 + i < o) acc[i] -= ts[(i0 + i) * v + c] * xv;
      }
#pragma unroll
      for (int i = 0; i < kChunk; ++i)
        if (i0 + i < o) zo[(((size_t)(i0 + i) * o + j) * v + a) * v + b] = acc[i];
    }
}

// one-body parts of [H_N, sigma] and [Yg, sigma] for all (p,q): one wavefront
// per element, lanes split the contraction loops
__global__ __launch_bounds__(256) void k_comm1(GlobalOps g, double* c1h, double* c1y) {
  const int n = g.n, o = g.o, v = n - o;
  const int lane = threadIdx.x % 64;
  const int idx = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (idx >= 2 * n * n) return;
  const int which = idx / (n * n), e = idx % (n * n);
  const Sigma s{g.t1, g.t2, n, o, v};
  double x;
  if (which == 0) {
    const DenseOp H{g.f, g.V, g.L, n, o, g.ga_h, g.g22_h, g.j1_h, g.j2_h, g.u_h, g.lo_h};
    auto c = make_comm_split(H, s, n, o, lane, 64);
    c.ring1 = false;
    x = c.c1(e / n, e % n);
  } else {
    const DenseOp Y{g.y1, g.y2, g.LY, n, o, g.ga_y, g.g22_y, g.j1_y, g.j2_y, nullptr, g.lo_y,
                   Sigma2Lazy{g.y1, g.t2, g.s2p, g.s2q, n, o}};
    auto c = make_comm_split(Y, s, n, o, lane, 64);
    c.ring1 = false;
    x = c.c1(e / n, e % n);
  }
  x = wave_sum(x);
  if (lane == 0) (which == 0 ? c1h : c1y)[e] = x;
}

// The sigma1 x X_2 part of the one-body commutator for all (p,q):
//   R[p][q] = sum_{t occ, u vir} t1[t][u] (2 X_uptq - X_upqt + 2 X_tpuq - X_tpqu)
// (X pair symmetric, X_pqrs = X_qpsr).
// Block (p, chunk of u, operator), one thread per q; chunk partials go to
// part[op][chunk][n][n] and are added in a fixed order by k_comm1_sum.
constexpr int kRingChunk = 8;

__global__ __launch_bounds__(128) void k_comm1_ring(const double* __restrict__ X0,
                                                    const double* __restrict__ X1,
                                                    const double* __restrict__ t1, int n, int o,
                                                    double* part) {
  const int v = n - o;
  const int nch = (v + kRingChunk - 1) / kRingChunk;
  const int p = blockIdx.x, ch = blockIdx.y, op = blockIdx.z;
  const int q = threadIdx.x;
  const double* X = op == 0 ? X0 : X1;
  const size_t n2 = (size_t)n * n, n3 = n2 * n;
  double acc = 0.0;
  if (q < n) {
    const int u0 = o + ch * kRingChunk, u1 = min(n, u0 + kRingChunk);
    for (int u = u0; u < u1; ++u)
      for (int t = 0; t < o; ++t) {
        const double w = t1[t * v + (u - o)];
        // X_upqt = X_putq and X_tpqu = X_ptuq (pair symmetry): all four reads
        // run along q
        const double x = 2.0 * X[u * n3 + p * n2 + (size_t)t * n + q] - X[p * n3 + u * n2 + (size_t)t * n + q] +
                         2.0 * X[t * n3 + p * n2 + (size_t)u * n + q] - X[p * n3 + t * n2 + (size_t)u * n + q];
        acc += w * x;
      }
    part[(((size_t)op * nch + ch) * n + p) * n + q] = acc;
  }
}

__global__ void k_comm1_sum(const double* __restrict__ part, int n, int nch, double* c1h,
                            double* c1y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n2 = n * n;
  if (e >= 2 * n2) return;
  const int op = e / n2, pq = e % n2;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[((size_t)op * nch + c) * n2 + pq];
  (op == 0 ? c1h : c1y)[pq] += s;
}

__global__ void k_residual1(GlobalOps g, double* r1) {
  const int n = g.n, o = g.o, v = n - o;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= o * v) return;
  const int i = idx / v, a = o + idx % v;
  r1[idx] = g.f[a * n + i] + g.c1_h[a * n + i] + 0.5 * g.c1_y[a * n + i];
}

// scal[0] = [H_N,sigma]_0, scal[1] = [Yg,sigma]_0 (scal[3] = E_ref, set at
// load); one wavefront, lanes split the contraction loops
__global__ __launch_bounds__(64) void k_residual0(GlobalOps g, double* scal, double* e0) {
  const int n = g.n, o = g.o, v = n - o;
  const int lane = threadIdx.x;
  const Sigma s{g.t1, g.t2, n, o, v};
  const DenseOp H{g.f, g.V, g.L, n, o, g.ga_h, g.g22_h, g.j1_h, g.j2_h, g.u_h, g.lo_h};
  const DenseOp Y{g.y1, g.y2, g.LY, n, o, g.ga_y, g.g22_y, g.j1_y, g.j2_y, nullptr, g.lo_y,
                   Sigma2Lazy{g.y1, g.t2, g.s2p, g.s2q, n, o}};
  const double zh = wave_sum(make_comm_split(H, s, n, o, lane, 64).c0());
  const double zy = wave_sum(make_comm_split(Y, s, n, o, lane, 64).c0());
  if (lane == 0) {
    scal[0] = zh;
    scal[1] = zy;
    if (e0) *e0 = scal[3] + zh + 0.5 * zy;
  }
}

}  // namespace

void launch_z_vvoo(const double* Xh, const double* Xy, const double* t1, int n, int o, double* zv,
                   double* zo, hipStream_t st) {
  const size_t v = n - o;
  k_zv<<<grid_for(v * v * o * o, kBlock, 65536), kBlock, 0, st>>>(Xh, Xy, t1, n, o, zv);
  k_zo<<<(unsigned)(o * v), 128, (size_t)o * v * sizeof(double), st>>>(Xh, Xy, t1, n, o, zo);
}

void launch_residual(const double* f, const double* V, const double* y1, const double* y2,
                     const double* L, const double* LY, const RingOps& rings, const double* t1,
                     const double* t2, int n, int o, double* scal, double* c1h, double* c1y,
                     double* part, double* r1, double* r2, double* e0, hipStream_t st) {
  GlobalOps g{f, V, y1, y2, L, LY, t1, t2, n, o, rings.ga_h, rings.g22_h, rings.j1_h,
              rings.j2_h, rings.ga_y, rings.g22_y, rings.j1_y, rings.j2_y,
              rings.zv,   rings.zo,  rings.u_h, rings.s2p, rings.s2q, rings.c1_h, rings.c1_y,
              rings.lo_h, rings.lo_y, rings.pf};
  const size_t v = n - o;
  k_comm1<<<grid_for((size_t)2 * n * n * 64), kBlock, 0, st>>>(g, c1h, c1y);
  const int nch = (int)((v + kRingChunk - 1) / kRingChunk);
  k_comm1_ring<<<dim3(n, nch, 2), 128, 0, st>>>(V, y2, t1, n, o, part);
  k_comm1_sum<<<grid_for((size_t)2 * n * n), kBlock, 0, st>>>(part, n, nch, c1h, c1y);
  int bc = 16;
  while (bc > 1 && bc * o * o > 8192) bc /= 2;
  const unsigned nbc = (unsigned)((v + bc - 1) / bc);
  k_residual2<<<(unsigned)v * nbc, kBlock, (size_t)bc * o * o * sizeof(double), st>>>(g, bc, r2);
  k_residual1<<<grid_for(o * v), kBlock, 0, st>>>(g, r1);
  k_residual0<<<1, 64, 0, st>>>(g, scal, e0);
}

}  // namespace qf
