// Batched Davidson eigensolver with cluster analysis.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// batched Davidson: one block per space
// ---------------------------------------------------------------------------

// Sum over the block of BLK threads, the same value returned to every
// thread.  red: LDS scratch of one double per wavefront.
template <int BLK>
__device__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < BLK / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Orders the LDS accesses of one wavefront (the lanes exchange values through
// LDS between the steps of a rotation).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lowest eigenpair of the symmetric m x m matrix A (LDS, row-major,
// destroyed; m <= 64) by cyclic Jacobi rotations, run by wavefront 0 alone:
// lane k applies each rotation to row/column k, and the lanes exchange values
// through LDS within the one wavefront, so no rotation waits at a workgroup
// barrier.  V (LDS, m x m) receives the eigenvectors; every thread gets theta
// and y[0..m) (LDS) the eigenvector.  flag: one double of LDS.
__device__ void jacobi_lowest(double* A, double* V, int m, double* theta, double* y,
                              double* flag) {
  const int k = threadIdx.x;
  if (k < 64) {
    for (int e = k; e < m * m; e += 64) V[e] = (e / m == e % m) ? 1.0 : 0.0;
    wave_lds_sync();
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0, dia = 0.0;
      for (int e = k; e < m * m; e += 64) {
        const int i = e / m, j = e % m;
        if (i == j) dia += A[e] * A[e];
        else if (j > i) off += A[e] * A[e];
      }
      off = wave_sum(off);
      dia = wave_sum(dia);
      if (off <= 1e-32 * (dia + 1e-300)) break;   // the same on every lane
      for (int p = 0; p < m; ++p)
        for (int q = p + 1; q < m; ++q) {
          const double apq = A[p * m + q];
          if (apq == 0.0) continue;
          const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
          wave_lds_sync();
          if (k < m) {
            const double akp = A[k * m + p], akq = A[k * m + q];
            A[k * m + p] = c * akp - s * akq;
            A[k * m + q] = s * akp + c * akq;
          }
          wave_lds_sync();
          if (k < m) {
            const double apk = A[p * m + k], aqk = A[q * m + k];
            A[p * m + k] = c * apk - s * aqk;
            A[q * m + k] = s * apk + c * aqk;
            const double vkp = V[k * m + p], vkq = V[k * m + q];
            V[k * m + p] = c * vkp - s * vkq;
            V[k * m + q] = s * vkp + c * vkq;
          }
          wave_lds_sync();
        }
    }
    int best = 0;
    for (int i = 1; i < m; ++i)
      if (A[i * m + i] < A[best * m + best]) best = i;
    if (k < m) y[k] = V[k * m + best];
    if (k == 0) flag[0] = A[best * m + best];
  }
  __syncthreads();
  *theta = flag[0];
}

constexpr int binom(int n, int k) { return k == 0 ? 1 : binom(n - 1, k - 1) * n / k; }

// Replacement lists of one size class packed for LDS: src | pq << 8 | (sgn > 0) << 16.
__device__ inline int rep_src(int r) { return r & 255; }
__device__ inline int rep_pq(int r) { return (r >> 8) & 255; }
__device__ inline double rep_sgn(int r) { return (r >> 16) ? 1.0 : -1.0; }

// Position u = Ia (Ia + 1) / 2 + Ib of the pair Ia >= Ib in the half of a
// determinant vector that a spin-flip symmetric vector is stored by.
__device__ inline void half_pair(int u, int& ia, int& ib) {
  int a = (int)((sqrtf(8.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
  while ((a + 1) * (a + 2) / 2 <= u) ++a;
  while (a * (a + 1) / 2 > u) --a;
  ia = a;
  ib = u - a * (a + 1) / 2;
}

// One space of NA orbitals and NE electrons per spin, one block of
// kDavBlock = BLK threads (memory layout: dav_layout(NA, NE, maxsub, BLK)).
//
// The downfolded Hamiltonian is spin-free, so exchanging the alpha and beta
// strings commutes with it; the start vector (the reference determinant, or
// the previous eigenvector made symmetric) and the diagonal preconditioner
// are symmetric under that exchange, and so is every vector of the
// iteration: c(Ia, Ib) = c(Ib, Ia) (the singlet-like sector of reading
// R15).  Each vector is therefore kept as its half Ia >= Ib, the entries off
// the diagonal scaled by sqrt(2), so that dot products, norms and
// Gram-Schmidt on the halves equal those of the full vectors, and sigma is
// evaluated only on that half: half the products and half the vector
// traffic of the full form, the same eigenpair.  The sigma input is
// expanded to the full vector in LDS; the final Ritz vector is expanded for
// the eigenvector output and the cluster analysis.  Gram dot products are
// reduced for all basis vectors at once; the correction is orthogonalised by
// classical Gram-Schmidt (a second pass when the first loses most of the
// norm).
template <int NA, int NE, int BLK>
__device__ void davidson_space(const DavidsonArgs& a, int k, const SpaceDev& sp, double* sm) {
  constexpr int kDavBlock = BLK;
  constexpr int NS = binom(NA, NE), NR = NE * (1 + NA - NE), D = NS * NS;
  constexpr int DU = NS * (NS + 1) / 2;
  constexpr int N2 = NA * NA, N4 = N2 * N2;
  constexpr int NW = kDavBlock / 64;
  constexpr double kSqrt2 = 1.4142135623730951, kInvSqrt2 = 0.7071067811865476;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const Strings& S = a.strings[sp.nocc - 2];
  const int MS = a.maxsub;
  const double* hin = a.heff + a.heff_off[k];
  const double Ec = hin[0];
  const double* h = hin + 1;
  constexpr bool BIG = dav_layout(NA, NE, 1).big;
  double* g = sm;                       // N4
  // Hs rows padded to an odd stride: lanes reading Hs[ib][J] for different
  // ib then fall on different LDS banks
  constexpr int HS = NS | 1;
  double* Hs = g + N4;                  // NS x HS
  double* xv = Hs + NS * HS;            // D  full Ritz vector / sigma input
  double* Gm = xv + D;                  // MS^2
  double* Aw = Gm + MS * MS;            // MS^2
  double* Vw = Aw + MS * MS;            // MS^2
  double* yv = Vw + MS * MS;            // MS
  double* misc = yv + MS;               // 4
  double* red = misc + 4;               // NW * MS
  int* rep = reinterpret_cast<int*>(red + NW * MS);   // NS*NR
  double* bb = a.work + a.work_off[k];  // MS x DU (halves)
  double* ss = bb + (size_t)MS * DU;    // MS x DU
  // diagonal, Ritz sigma and residual (halves): LDS after the replacement
  // lists, or the global work area after the sigma vectors
  double* dg = BIG ? ss + (size_t)MS * DU : reinterpret_cast<double*>(rep) + (NS * NR + 1) / 2;
  double* hx = dg + DU;
  double* rv = hx + DU;
  for (int e = tid; e < N4; e += kDavBlock) g[e] = hin[1 + N2 + e];
  for (int e = tid; e < NS * NR; e += kDavBlock) {
    const int I = e / NR, f = e % NR;
    rep[e] = S.src[I][f] | (S.pq[I][f] << 8) | ((S.sgn[I][f] > 0) << 16);
  }
  __syncthreads();
  // same-spin string Hamiltonian Hs[I][J] = <I| sum k_pq E_pq + 1/2 sum g E_pq E_rs |J>,
  // k_pq = h_pq - 1/2 sum_r g(pr|rq): thread I scatters the one- and two-step
  // replacements of string I into row I (one thread per row, in a fixed order)
  double* kk = rv;   // N2 <= DU doubles; rv is free until the iterations start
  for (int e = tid; e < NS * HS; e += kDavBlock) Hs[e] = 0.0;
  for (int e = tid; e < N2; e += kDavBlock) {
    const int p = e / NA, q = e % NA;
    double x = h[p * NA + q];
    for (int t = 0; t < NA; ++t) x -= 0.5 * g[((p * NA + t) * NA + t) * NA + q];
    kk[e] = x;
  }
  __syncthreads();
  if (tid < NS) {
    const int I = tid;
    double* row = Hs + I * HS;
    for (int f = 0; f < NR; ++f) {
      const int r = rep[I * NR + f];
      row[rep_src(r)] += rep_sgn(r) * kk[rep_pq(r)];
      const int Kst = rep_src(r);
      const double* gr = g + rep_pq(r) * N2;
      for (int f2 = 0; f2 < NR; ++f2) {
        const int r2 = rep[Kst * NR + f2];
        row[rep_src(r2)] += 0.5 * rep_sgn(r) * rep_sgn(r2) * gr[rep_pq(r2)];
      }
    }
  }
  __syncthreads();
  for (int u = tid; u < DU; u += kDavBlock) {
    int ia, ib;
    half_pair(u, ia, ib);
    dg[u] = cas_diag(S, Hs, HS, g, Ec, ia, ib);
  }
  // starting vector: the stored eigenvector of this space's previous solve
  // when there is one (non-zero), made symmetric, else the reference
  // determinant
  double* civ = a.ci ? a.ci + a.ci_off[k] : nullptr;
  double cn = 0.0;
  if (civ)
    for (int u = tid; u < DU; u += kDavBlock) {
      int ia, ib;
      half_pair(u, ia, ib);
      const double c = 0.5 * (civ[ia * NS + ib] + civ[ib * NS + ia]);
      cn += (ia == ib ? 1.0 : 2.0) * c * c;
    }
  cn = block_sum<kDavBlock>(cn, red);
  const bool warm = cn > 0.25;
  const double cinv = warm ? 1.0 / sqrt(cn) : 0.0;
  for (int u = tid; u < DU; u += kDavBlock) {
    double x = u == 0 ? 1.0 : 0.0;
    if (warm) {
      int ia, ib;
      half_pair(u, ia, ib);
      x = 0.5 * (civ[ia * NS + ib] + civ[ib * NS + ia]) * cinv * (ia == ib ? 1.0 : kSqrt2);
    }
    bb[u] = x;
  }
  __syncthreads();
  // the full vector of a half one into xv (LDS)
  auto expand = [&](const double* half) {
    for (int u = tid; u < DU; u += kDavBlock) {
      int ia, ib;
      half_pair(u, ia, ib);
      const double c = ia == ib ? half[u] : half[u] * kInvSqrt2;
      xv[ia * NS + ib] = c;
      xv[ib * NS + ia] = c;
    }
  };
  // sigma of the full c (LDS) on the half Ia >= Ib, scaled, into out (global)
  auto sigma = [&](const double* c, double* out) {
#pragma unroll 1
    for (int u = tid; u < DU; u += kDavBlock) {
      int ia, ib;
      half_pair(u, ia, ib);
      int jb[NR], rs[NR];
      double sb[NR];
#pragma unroll
      for (int f = 0; f < NR; ++f) {
        const int r = rep[ib * NR + f];
        jb[f] = rep_src(r);
        rs[f] = rep_pq(r);
        sb[f] = rep_sgn(r);
      }
      double x = Ec * c[ia * NS + ib];
#pragma unroll
      for (int J = 0; J < NS; ++J)
        x += Hs[ia * HS + J] * c[J * NS + ib] + Hs[ib * HS + J] * c[ia * NS + J];
#pragma unroll
      for (int e = 0; e < NR; ++e) {
        const int r = rep[ia * NR + e];
        const double* gr = g + rep_pq(r) * N2;
        const double* cr = c + rep_src(r) * NS;
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < NR; ++f) acc += sb[f] * gr[rs[f]] * cr[jb[f]];
        x += rep_sgn(r) * acc;
      }
      out[u] = ia == ib ? x : x * kSqrt2;
    }
  };
  // the dot products of vec with basis vectors 0..m-1, reduced together
  auto dots = [&](const double* vec, int m, double* outv) {
    for (int i = 0; i < m; ++i) {
      double d = 0.0;
      for (int u = tid; u < DU; u += kDavBlock) d += bb[(size_t)i * DU + u] * vec[u];
      d = wave_sum(d);
      if (lane == 0) red[wv * MS + i] = d;
    }
    __syncthreads();
    for (int i = tid; i < m; i += kDavBlock) {
      double d = 0.0;
      for (int w = 0; w < NW; ++w) d += red[w * MS + i];
      outv[i] = d;
    }
    __syncthreads();
  };
  int m = 1, it = 0;
  bool conv = false;
  double theta = 0.0;
  for (it = 0; it < a.max_iter; ++it) {
    // sigma of the newest basis vector
    expand(bb + (size_t)(m - 1) * DU);
    __syncthreads();
    double* sn = ss + (size_t)(m - 1) * DU;
    sigma(xv, sn);
    __syncthreads();
    dots(sn, m, yv);   // yv as scratch: the new column of the projected matrix
    for (int i = tid; i < m; i += kDavBlock) {
      Gm[i * MS + (m - 1)] = yv[i];
      Gm[(m - 1) * MS + i] = yv[i];
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += kDavBlock) Aw[e] = Gm[(e / m) * MS + e % m];
    __syncthreads();
    jacobi_lowest(Aw, Vw, m, &theta, yv, misc + 1);
    // Ritz vector (full, into xv), its sigma (half, hx) and the residual (half, rv)
    double rn = 0.0;
    for (int u = tid; u < DU; u += kDavBlock) {
      double x = 0.0, y = 0.0;
      for (int i = 0; i < m; ++i) {
        x += yv[i] * bb[(size_t)i * DU + u];
        y += yv[i] * ss[(size_t)i * DU + u];
      }
      int ia, ib;
      half_pair(u, ia, ib);
      const double c = ia == ib ? x : x * kInvSqrt2;
      xv[ia * NS + ib] = c;
      xv[ib * NS + ia] = c;
      hx[u] = y;
      rv[u] = y - theta * x;
      rn += rv[u] * rv[u];
    }
    rn = sqrt(block_sum<kDavBlock>(rn, red));
    if (rn < a.tol) {
      conv = true;
      ++it;
      break;
    }
    if (m == MS) {   // restart from the Ritz vector
      for (int u = tid; u < DU; u += kDavBlock) {
        int ia, ib;
        half_pair(u, ia, ib);
        const double c = xv[ia * NS + ib];
        bb[u] = ia == ib ? c : c * kSqrt2;
        ss[u] = hx[u];
      }
      if (tid == 0) Gm[0] = theta;
      m = 1;
      __syncthreads();
    }
    // diagonal-preconditioned correction, orthogonalised by classical
    // Gram-Schmidt; a second pass only when the first left less than
    // 1/sqrt(2) of its norm (the Daniel-Gragg-Kaufman-Stewart criterion)
    double n0 = 0.0;
    for (int u = tid; u < DU; u += kDavBlock) {
      double den = dg[u] - theta;
      if (fabs(den) < 1e-8) den = (den < 0.0 ? -1e-8 : 1e-8);
      rv[u] = -rv[u] / den;
      n0 += rv[u] * rv[u];
    }
    n0 = sqrt(block_sum<kDavBlock>(n0, red));
    double nr = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      dots(rv, m, Aw);   // Aw as scratch
      nr = 0.0;
      for (int u = tid; u < DU; u += kDavBlock) {
        double x = rv[u];
        for (int i = 0; i < m; ++i) x -= Aw[i] * bb[(size_t)i * DU + u];
        rv[u] = x;
        nr += x * x;
      }
      nr = sqrt(block_sum<kDavBlock>(nr, red));   // (also orders the rv writes)
      if (nr > 0.70710678118654752 * n0) break;   // the same on every thread
      n0 = nr;
    }
    if (nr < 1e-14) {
      conv = rn < 1e3 * a.tol;
      ++it;
      break;
    }
    double* bnew = bb + (size_t)m * DU;
    for (int u = tid; u < DU; u += kDavBlock) bnew[u] = rv[u] / nr;
    ++m;
    __syncthreads();
  }
  __syncthreads();
  // sign convention: reference coefficient >= 0
  const double sgn = (xv[0] < 0.0) ? -1.0 : 1.0;
  const double c0 = sgn * xv[0];
  if (civ)
    for (int e = tid; e < D; e += kDavBlock) civ[e] = sgn * xv[e];
  if (tid == 0) {
    a.energy[k] = theta;
    a.c0[k] = c0;
    a.iters[k] = it;
    int st = conv ? 0 : -5;
    if (c0 < 0.1) st = -6;
    a.status[k] = st;
  }
  // intermediate-normalised cluster amplitudes
  constexpr int nv = NA - NE, ne = NE;
  double* amp = a.amp + a.amp_off[k];
  const double inv = (c0 > 0.0) ? sgn / c0 : 0.0;
  for (int e = tid; e < ne * nv; e += kDavBlock) {
    const int i = e / nv, b = e % nv;
    amp[e] = S.exc_sgn[i][b] * xv[S.exc_str[i][b] * NS] * inv;
  }
  constexpr int nt1 = ne * nv;
  for (int e = tid; e < nt1 * nt1; e += kDavBlock) {
    const int b = e % nv, av = e / nv % nv, j = e / (nv * nv) % ne, i = e / (nv * nv * ne);
    const double ta = S.exc_sgn[i][av] * xv[S.exc_str[i][av] * NS] * inv;
    const double tb = S.exc_sgn[j][b] * xv[S.exc_str[j][b] * NS] * inv;
    const double c2 = S.exc_sgn[i][av] * S.exc_sgn[j][b] *
                      xv[S.exc_str[i][av] * NS + S.exc_str[j][b]] * inv;
    amp[nt1 + e] = c2 - ta * tb;
  }
}

template <int NA, int NE, int BLK>
__global__ __launch_bounds__(BLK) void k_davidson(DavidsonArgs a,
                                                  const int32_t* __restrict__ idx) {
  extern __shared__ double sm[];
  const int k = idx[blockIdx.x];
  const SpaceDev sp = a.spaces[k];
  davidson_space<NA, NE, BLK>(a, k, sp, sm);
}

// Persistent form: workgroups of dav_block(NAMAX) threads loop taking the
// next position from a.counter; positions run over the (4,4) class, then
// (3,3), then (2,2) (the costliest spaces first, so that the small ones fill
// the tail).  off = the class offsets of idx; every workgroup leaves once
// the counter passes the end of the list.
template <int NAMAX>
__global__ __launch_bounds__(dav_block(NAMAX)) void k_davidson_persistent(
    DavidsonArgs a, const int32_t* __restrict__ idx, int4 off) {
  constexpr int BLK = dav_block(NAMAX);
  extern __shared__ double sm[];
  __shared__ int item;
  const int n4 = off.w - off.z, n3 = off.z - off.y, total = off.w - off.x;
  for (;;) {
    // the previous space is done with LDS (and with `item`) on every thread
    __syncthreads();
    if (threadIdx.x == 0) item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int w = item;
    if (w >= total) break;
    const int pos = w < n4 ? off.z + w : (w < n4 + n3 ? off.y + (w - n4) : off.x + (w - n4 - n3));
    const int k = idx[pos];
    const SpaceDev sp = a.spaces[k];
    if constexpr (NAMAX >= 8) {
      if (sp.nocc == 4) {
        davidson_space<8, 4, BLK>(a, k, sp, sm);
        continue;
      }
    }
    if constexpr (NAMAX >= 6) {
      if (sp.nocc == 3) {
        davidson_space<6, 3, BLK>(a, k, sp, sm);
        continue;
      }
    }
    davidson_space<4, 2, BLK>(a, k, sp, sm);
  }
}

__global__ void k_set_counter(int* c) { *c = 0; }

template <int NA, int NE, int BLK = dav_block(NA)>
void launch_class(const DavidsonArgs& a, const int32_t* idx, int count, hipStream_t st) {
  if (count <= 0) return;
  const size_t bytes = (size_t)dav_layout(NA, NE, a.maxsub, BLK).lds * sizeof(double);
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_davidson<NA, NE, BLK>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  k_davidson<NA, NE, BLK><<<count, BLK, bytes, st>>>(a, idx);
}

template <int NAMAX>
void launch_persistent(const DavidsonArgs& a, const int32_t* idx, const int* cls_off,
                       hipStream_t st) {
  constexpr int BLK = dav_block(NAMAX);
  const int total = cls_off[3] - cls_off[0];
  size_t lds = 0;
  for (int c = 0; c < 3; ++c)
    if (cls_off[c + 1] > cls_off[c] && 2 * (c + 2) <= NAMAX)
      lds = std::max(lds, (size_t)dav_layout(2 * (c + 2), c + 2, a.maxsub, BLK).lds);
  const size_t bytes = lds * sizeof(double);
  const void* fn = reinterpret_cast<const void*>(&k_davidson_persistent<NAMAX>);
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLK, bytes) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int grid = std::max(1, std::min(total, per_cu * cus));
  k_set_counter<<<1, 1, 0, st>>>(a.counter);
  k_davidson_persistent<NAMAX><<<grid, BLK, bytes, st>>>(
      a, idx, make_int4(cls_off[0], cls_off[1], cls_off[2], cls_off[3]));
}

}  // namespace

void launch_davidson(const DavidsonArgs& a, const int32_t* cls_idx, const int* cls_off,
                     hipStream_t st, bool persistent) {
  if (persistent && a.counter && cls_off[3] > cls_off[0]) {
    if (cls_off[3] > cls_off[2])
      launch_persistent<8>(a, cls_idx, cls_off, st);
    else if (cls_off[2] > cls_off[1])
      launch_persistent<6>(a, cls_idx, cls_off, st);
    else
      launch_persistent<4>(a, cls_idx, cls_off, st);
    return;
  }
  launch_class<4, 2>(a, cls_idx + cls_off[0], cls_off[1] - cls_off[0], st);
  launch_class<6, 3>(a, cls_idx + cls_off[1], cls_off[2] - cls_off[1], st);
  if (a.big_block == 1024)
    launch_class<8, 4, 1024>(a, cls_idx + cls_off[2], cls_off[3] - cls_off[2], st);
  else
    launch_class<8, 4>(a, cls_idx + cls_off[2], cls_off[3] - cls_off[2], st);
}

}  // namespace qf
