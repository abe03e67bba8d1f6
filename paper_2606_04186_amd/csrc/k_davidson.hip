// Batched Davidson eigensolver with cluster analysis.
#include <hip/hip_runtime.h>

#include <math.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// batched Davidson: one wavefront per space
// ---------------------------------------------------------------------------

// Lowest eigenpair of the symmetric m x m matrix A (row-major, destroyed) by
// cyclic Jacobi rotations; V (m x m) receives eigenvectors.
__device__ void jacobi_lowest(double* A, double* V, int m, double* theta, double* y) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) V[i * m + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < m; ++i) {
      dia += A[i * m + i] * A[i * m + i];
      for (int j = i + 1; j < m; ++j) off += A[i * m + j] * A[i * m + j];
    }
    if (off <= 1e-32 * (dia + 1e-300)) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (apq == 0.0) continue;
        const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = c * akp - s * akq;
          A[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = c * apk - s * aqk;
          A[q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[k * m + p], vkq = V[k * m + q];
          V[k * m + p] = c * vkp - s * vkq;
          V[k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  int best = 0;
  for (int i = 1; i < m; ++i)
    if (A[i * m + i] < A[best * m + best]) best = i;
  *theta = A[best * m + best];
  for (int i = 0; i < m; ++i) y[i] = V[i * m + best];
}

__global__ __launch_bounds__(64) void k_davidson(DavidsonArgs a) {
  extern __shared__ double sm[];
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const SpaceDev sp = a.spaces[k];
  const Strings& S = a.strings[sp.nocc - 2];
  const int na = S.na, ns = S.nstr, D = ns * ns, MS = a.maxsub;
  const double* hin = a.heff + a.heff_off[k];
  const double Ec = hin[0];
  const double* h = hin + 1;
  double* g = sm;                       // na^4
  double* Hs = g + na * na * na * na;   // ns^2
  double* dg = Hs + ns * ns;            // D
  double* xv = dg + D;                  // D  Ritz vector / sigma staging
  double* hx = xv + D;                  // D
  double* rv = hx + D;                  // D
  double* G = rv + D;                   // MS^2
  double* Aw = G + MS * MS;             // MS^2
  double* Vw = Aw + MS * MS;            // MS^2
  double* yv = Vw + MS * MS;            // MS
  double* misc = yv + MS;               // 4
  double* bb = a.work + a.work_off[k];  // MS x D
  double* ss = bb + (size_t)MS * D;     // MS x D
  for (int e = lane; e < na * na * na * na; e += 64) g[e] = hin[1 + na * na + e];
  __syncthreads();
  for (int e = lane; e < ns * ns; e += 64) Hs[e] = same_spin_element(S, h, g, e / ns, e % ns);
  __syncthreads();
  for (int e = lane; e < D; e += 64) {
    dg[e] = cas_diag(S, Hs, g, Ec, e / ns, e % ns);
    bb[e] = (e == 0) ? 1.0 : 0.0;
  }
  __syncthreads();
  int m = 1, it = 0;
  bool conv = false;
  double theta = 0.0;
  for (it = 0; it < a.max_iter; ++it) {
    // sigma of the newest basis vector
    const double* bn = bb + (size_t)(m - 1) * D;
    for (int e = lane; e < D; e += 64) xv[e] = bn[e];
    __syncthreads();
    double* sn = ss + (size_t)(m - 1) * D;
    for (int e = lane; e < D; e += 64) sn[e] = cas_sigma(S, Hs, g, Ec, xv, e / ns, e % ns);
    __syncthreads();
    for (int i = 0; i < m; ++i) {
      double d = 0.0;
      for (int e = lane; e < D; e += 64) d += bb[(size_t)i * D + e] * sn[e];
      d = wave_sum(d);
      if (lane == 0) {
        G[i * MS + (m - 1)] = d;
        G[(m - 1) * MS + i] = d;
      }
    }
    __syncthreads();
    if (lane == 0) {
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Aw[i * m + j] = G[i * MS + j];
      jacobi_lowest(Aw, Vw, m, &misc[0], yv);
    }
    __syncthreads();
    theta = misc[0];
    double rn = 0.0;
    for (int e = lane; e < D; e += 64) {
      double x = 0.0, y = 0.0;
      for (int i = 0; i < m; ++i) {
        x += yv[i] * bb[(size_t)i * D + e];
        y += yv[i] * ss[(size_t)i * D + e];
      }
      xv[e] = x;
      hx[e] = y;
      rv[e] = y - theta * x;
      rn += rv[e] * rv[e];
    }
    rn = sqrt(wave_sum(rn));
    __syncthreads();
    if (rn < a.tol) {
      conv = true;
      ++it;
      break;
    }
    if (m == MS) {   // restart from the Ritz vector
      for (int e = lane; e < D; e += 64) {
        bb[e] = xv[e];
        ss[e] = hx[e];
      }
      if (lane == 0) G[0] = theta;
      m = 1;
      __syncthreads();
    }
    // diagonal-preconditioned correction, orthogonalised twice
    for (int e = lane; e < D; e += 64) {
      double den = dg[e] - theta;
      if (fabs(den) < 1e-8) den = (den < 0.0 ? -1e-8 : 1e-8);
      rv[e] = -rv[e] / den;
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < m; ++i) {
        double d = 0.0;
        for (int e = lane; e < D; e += 64) d += bb[(size_t)i * D + e] * rv[e];
        d = wave_sum(d);
        for (int e = lane; e < D; e += 64) rv[e] -= d * bb[(size_t)i * D + e];
        __syncthreads();
      }
    double nr = 0.0;
    for (int e = lane; e < D; e += 64) nr += rv[e] * rv[e];
    nr = sqrt(wave_sum(nr));
    if (nr < 1e-14) {
      conv = rn < 1e3 * a.tol;
      ++it;
      break;
    }
    double* bnew = bb + (size_t)m * D;
    for (int e = lane; e < D; e += 64) bnew[e] = rv[e] / nr;
    ++m;
    __syncthreads();
  }
  __syncthreads();
  // sign convention: reference coefficient >= 0
  const double sgn = (xv[0] < 0.0) ? -1.0 : 1.0;
  const double c0 = sgn * xv[0];
  if (lane == 0) {
    a.energy[k] = theta;
    a.c0[k] = c0;
    a.iters[k] = it;
    int st = conv ? 0 : -5;
    if (c0 < 0.1) st = -6;
    a.status[k] = st;
  }
  // intermediate-normalised cluster amplitudes
  const int nv = na - S.ne, ne = S.ne;
  double* amp = a.amp + a.amp_off[k];
  const double inv = (c0 > 0.0) ? sgn / c0 : 0.0;
  for (int e = lane; e < ne * nv; e += 64) {
    const int i = e / nv, b = e % nv;
    amp[e] = S.exc_sgn[i][b] * xv[S.exc_str[i][b] * ns] * inv;
  }
  const int nt1 = ne * nv;
  for (int e = lane; e < nt1 * nt1; e += 64) {
    const int b = e % nv, av = e / nv % nv, j = e / (nv * nv) % ne, i = e / (nv * nv * ne);
    const double ta = S.exc_sgn[i][av] * xv[S.exc_str[i][av] * ns] * inv;
    const double tb = S.exc_sgn[j][b] * xv[S.exc_str[j][b] * ns] * inv;
    const double c2 = S.exc_sgn[i][av] * S.exc_sgn[j][b] *
                      xv[S.exc_str[i][av] * ns + S.exc_str[j][b]] * inv;
    amp[nt1 + e] = c2 - ta * tb;
  }
}

}  // namespace

void launch_davidson(const DavidsonArgs& a, int lds_doubles, hipStream_t st) {
  k_davidson<<<a.K, 64, (size_t)lds_doubles * sizeof(double), st>>>(a);
}

}  // namespace qf
