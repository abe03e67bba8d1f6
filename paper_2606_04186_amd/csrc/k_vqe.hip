// Batched UCCSD-VQE active-space solver (the paper's solver): for every
// space, the spin-adapted singles and doubles theta of sigma_int = T - T^dag
// (T = sum theta1 E_AI + 1/2 sum theta2 E_AI E_BJ, the pool's convention)
// minimising E(theta) = <Phi| e^{-sigma_int} H_eff e^{sigma_int} |Phi>
// (Eqs. (5) and (8) at N = 1), evaluated exactly in the space's determinant
// basis.  One workgroup per space:
//   * E_PQ (spin summed) acts on a CI vector through a per-string table
//     (string, pq) -> source string and sign, built from the replacement
//     lists;
//   * A v = sigma_int v from 9 + 9 single excitations of v (T v =
//     sum_IA E_AI (theta1 v + 1/2 sum_JB theta2 E_BJ v), T^dag v likewise with
//     de-excitations);
//   * e^{xA} v by its Taylor series, summed until a term falls below 1e-17 of
//     the sum;
//   * H v (the CAS matrix of the downfolded Hamiltonian) by the same
//     string-driven product as the Davidson solver, on full vectors;
//   * the gradient dE/dtheta_k = 2 int_0^1 lam(s)^T G_k phi(s) ds with
//     phi(s) = e^{(1-s)A} Phi and lam(s) = e^{-sA} H psi, by 8-point
//     Gauss-Legendre quadrature (the integrand is entire in s; the error is
//     of order |A|^16 / 16!);
//   * BFGS with an Armijo backtracking line search, the inverse Hessian
//     started from the diagonal 1 / (4 max(d_k, 0.05)) with d_k the
//     excitation energy of the parameter's determinant, until the largest
//     gradient entry is below gtol.
#include <hip/hip_runtime.h>

#include <math.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"

namespace qf {

namespace {

constexpr int kVqeBlock = 512;
constexpr int kVqeNodes = 8;
// Gauss-Legendre nodes and weights on [0, 1]
__constant__ double kGLx[kVqeNodes] = {
    0.019855071751231856, 0.10166676129318664, 0.2372337950418355, 0.4082826787521751,
    0.5917173212478249,   0.7627662049581645,  0.8983332387068134, 0.9801449282487681};
__constant__ double kGLw[kVqeNodes] = {
    0.05061426814518813, 0.11119051722668724, 0.15685332293894363, 0.18134189168918100,
    0.18134189168918100, 0.15685332293894363, 0.11119051722668724, 0.05061426814518813};

constexpr int binom_v(int n, int k) { return k == 0 ? 1 : binom_v(n - 1, k - 1) * n / k; }

template <int NA, int NE>
struct VqeShape {
  static constexpr int NS = binom_v(NA, NE), D = NS * NS, NR = NE * (1 + NA - NE);
  static constexpr int NV = NA - NE, NT1 = NE * NV, NP = NT1 + NT1 * (NT1 + 1) / 2;
  static constexpr int N2 = NA * NA, N4 = N2 * N2, HS = NS | 1;
  // LDS doubles: g, Hs, string tables (ints), vectors, BFGS state, scratch
  static constexpr int NVEC = 4 + 2 * NT1 + 4;   // psi, w, phi, lam, 2 NT1 sets, 4 scratch
  // ... BFGS (NP^2 + 8 NP), dot products (NT1 + NT1^2), 1/2 theta2 table
  // (NT1^2), reduction slots (2 per wavefront)
  static constexpr int LDS = N4 + NS * HS + (NS * N2 + NS * NR + 1) / 2 + NVEC * D +
                             NP * NP + 8 * NP + NT1 + 2 * NT1 * NT1 + 2 * (kVqeBlock / 64);
};

__device__ double vqe_block_sum(double x, double* red) {
  x = wave_sum(x);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kVqeBlock / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ double vqe_block_max(double x, double* red) {
  x = wave_max(x);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kVqeBlock / 64; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

template <int NA, int NE>
struct VqeSpace {
  using S_ = VqeShape<NA, NE>;
  static constexpr int NS = S_::NS, D = S_::D, NR = S_::NR, NV = S_::NV, NT1 = S_::NT1,
                       NP = S_::NP, N2 = S_::N2, N4 = S_::N4, HS = S_::HS;
  const Strings& S;
  double Ec;
  double *g, *Hs, *red;
  int *emap, *rep;
  double *psi, *w, *phi, *lam, *setA, *setB, *s0, *s1, *s2, *s3;
  double *Hinv, *th, *gr, *p, *sv, *yv, *th2, *g2, *dk, *t2h;

  // (E_PQ v)(Ia, Ib) for spin-summed E_PQ, P,Q local orbitals; out = or += (acc)
  __device__ void apply_E(int P, int Q, const double* v, double* out, bool acc) const {
    const int pq = P * NA + Q;
    for (int e = threadIdx.x; e < D; e += kVqeBlock) {
      const int ia = e / NS, ib = e % NS;
      double x = 0.0;
      const int sa = emap[ia * N2 + pq], sb = emap[ib * N2 + pq];
      if (sa != 0) x += (sa > 0 ? 1.0 : -1.0) * v[(abs(sa) - 1) * NS + ib];
      if (sb != 0) x += (sb > 0 ? 1.0 : -1.0) * v[ia * NS + (abs(sb) - 1)];
      out[e] = acc ? out[e] + x : x;
    }
  }

  // (E_PQ v) at (ia, ib) for the table entry pq = P * NA + Q
  __device__ double e_at(int pq, const double* v, int ia, int ib) const {
    double x = 0.0;
    const int sa = emap[ia * N2 + pq], sb = emap[ib * N2 + pq];
    if (sa != 0) x += (sa > 0 ? 1.0 : -1.0) * v[(abs(sa) - 1) * NS + ib];
    if (sb != 0) x += (sb > 0 ? 1.0 : -1.0) * v[ia * NS + (abs(sb) - 1)];
    return x;
  }

  // 1/2 theta2 as a full NT1 x NT1 table; after every change of th
  __device__ void prep_theta() {
    for (int q = threadIdx.x; q < NT1 * NT1; q += kVqeBlock) t2h[q] = 0.5 * t2(q / NT1, q % NT1);
    __syncthreads();
  }

  // out = x A v with A = T - T^dag of the parameters th:
  //   T v     = sum_IA E_AI S_IA,  S_IA = theta1 v + 1/2 sum_JB theta2 E_BJ v,
  //   T^dag v = sum_IA E_IA R_IA,  R_IA = theta1 v + 1/2 sum_JB theta2 E_JB v
  // (E_AI and E_BJ commute, as do E_IA and E_JB).  Each thread forms, for
  // its entry f, every E_BJ v and E_JB v at f and accumulates S_IA[f] and
  // R_IA[f] in registers (written to setA, setB); after one barrier each
  // output gathers its sources from those: two barriers in all, and few LDS
  // reads per product.  With y given, also y += out and, per wavefront,
  // (max |out|, max |y|) into slot[2 w], slot[2 w + 1] (visible after the
  // closing barrier).  out distinct from v, setA, setB.
  __device__ void apply_A(double x, const double* v, double* out, double* y = nullptr,
                          double* slot = nullptr) {
    for (int f = threadIdx.x; f < D; f += kVqeBlock) {
      const int fa = f / NS, fb = f % NS;
      const double vf = v[f];
      double sx[NT1], rx[NT1];
#pragma unroll
      for (int ia = 0; ia < NT1; ++ia) sx[ia] = rx[ia] = th[ia] * vf;
#pragma unroll 1
      for (int jb = 0; jb < NT1; ++jb) {
        const int J = jb / NV, B = NE + jb % NV;
        const double u = e_at(B * NA + J, v, fa, fb);
        const double l = e_at(J * NA + B, v, fa, fb);
#pragma unroll
        for (int ia = 0; ia < NT1; ++ia) {
          const double c = t2h[ia * NT1 + jb];
          sx[ia] += c * u;
          rx[ia] += c * l;
        }
      }
#pragma unroll
      for (int ia = 0; ia < NT1; ++ia) {
        setA[ia * D + f] = sx[ia];
        setB[ia * D + f] = rx[ia];
      }
    }
    __syncthreads();
    double tm = 0.0, ym = 0.0;
    for (int e = threadIdx.x; e < D; e += kVqeBlock) {
      const int ja = e / NS, jb2 = e % NS;
      double acc = 0.0;
#pragma unroll 1
      for (int ia = 0; ia < NT1; ++ia) {
        const int I = ia / NV, A = NE + ia % NV;
        acc += e_at(A * NA + I, setA + ia * D, ja, jb2) - e_at(I * NA + A, setB + ia * D, ja, jb2);
      }
      out[e] = x * acc;
      if (y) {
        y[e] += x * acc;
        tm = fmax(tm, fabs(x * acc));
        ym = fmax(ym, fabs(y[e]));
      }
    }
    if (y) {
      tm = wave_max(tm);
      ym = wave_max(ym);
      if (threadIdx.x % 64 == 0) {
        slot[2 * (threadIdx.x / 64)] = tm;
        slot[2 * (threadIdx.x / 64) + 1] = ym;
      }
    }
    __syncthreads();
  }

  // theta2 of the pair of singles (p1, p2), symmetric
  __device__ double t2(int p1, int p2) const {
    const int a = min(p1, p2), b = max(p1, p2);
    return th[NT1 + a * NT1 - a * (a - 1) / 2 + (b - a)];
  }

  // y = e^{xA} v (Taylor series, terms up to the first one below 1e-17 of
  // the sum).  Term n = (x/n) A term(n-1) is formed by one product whose
  // output loop also adds it to y and takes the stopping test's maxima, so
  // each term costs the product's two barriers; terms alternate between s0
  // and s1.
  __device__ void expm_apply(double x, const double* v, double* y) {
    constexpr int NW = kVqeBlock / 64;
    for (int e = threadIdx.x; e < D; e += kVqeBlock) {
      y[e] = v[e];
      s0[e] = v[e];
    }
    __syncthreads();
    double* a = s0;
    double* b = s1;
    for (int n = 1; n <= 60; ++n) {
      apply_A(x / n, a, b, y, red);
      double tm = 0.0, ym = 0.0;
      for (int w_ = 0; w_ < NW; ++w_) {
        tm = fmax(tm, red[2 * w_]);
        ym = fmax(ym, red[2 * w_ + 1]);
      }
      if (tm <= 1e-17 * ym) break;
      double* t = a;   // (the next product writes red only after its first barrier)
      a = b;
      b = t;
    }
  }

  // out = H v on full vectors (the CAS matrix of the space)
  __device__ void apply_H(const double* v, double* out) const {
    for (int e = threadIdx.x; e < D; e += kVqeBlock) {
      const int ia = e / NS, ib = e % NS;
      double x = Ec * v[e];
      for (int J = 0; J < NS; ++J)
        x += Hs[ia * HS + J] * v[J * NS + ib] + Hs[ib * HS + J] * v[ia * NS + J];
      for (int f = 0; f < NR; ++f) {
        const int r = rep[ia * NR + f];
        const double* gr = g + ((r >> 8) & 255) * N2;
        const double* cr = v + (r & 255) * NS;
        double acc = 0.0;
        for (int f2 = 0; f2 < NR; ++f2) {
          const int r2 = rep[ib * NR + f2];
          acc += ((r2 >> 16) ? 1.0 : -1.0) * gr[(r2 >> 8) & 255] * cr[r2 & 255];
        }
        x += ((r >> 16) ? 1.0 : -1.0) * acc;
      }
      out[e] = x;
    }
    __syncthreads();
  }

  // E(theta) into the return value; psi = e^{A} Phi, w = H psi
  __device__ double energy() {
    prep_theta();
    for (int e = threadIdx.x; e < D; e += kVqeBlock) s2[e] = e == 0 ? 1.0 : 0.0;
    __syncthreads();
    expm_apply(1.0, s2, psi);
    apply_H(psi, w);
    double d = 0.0;
    for (int e = threadIdx.x; e < D; e += kVqeBlock) d += psi[e] * w[e];
    return vqe_block_sum(d, red);
  }

  // out[p] = a . S_p (p < NT1), out[NT1 + p1 NT1 + p2] = P_p1 . Q_p2: one
  // thread per dot product, one barrier
  __device__ void phase_dots(const double* a, const double* S, const double* P, const double* Q,
                             double* out) const {
    for (int q = threadIdx.x; q < NT1 + NT1 * NT1; q += kVqeBlock) {
      const double *x, *y;
      if (q < NT1) {
        x = a;
        y = S + q * D;
      } else {
        x = P + ((q - NT1) / NT1) * D;
        y = Q + ((q - NT1) % NT1) * D;
      }
      double d = 0.0;
      for (int e = 0; e < D; ++e) d += x[e] * y[e];
      out[q] = d;
    }
    __syncthreads();
  }

  // gr += c (singles: out[p]; pairs (a <= b): f out[NT1 + a NT1 + b], f = 1/2
  // for a = b), then a barrier
  __device__ void phase_add(double c, const double* out) {
    for (int k = threadIdx.x; k < NP; k += kVqeBlock) {
      if (k < NT1) {
        gr[k] += c * out[k];
      } else {
        int a = 0, r = k - NT1;
        while (r >= NT1 - a) {
          r -= NT1 - a;
          ++a;
        }
        const int b = a + r;
        gr[k] += c * (a == b ? 0.5 : 1.0) * out[NT1 + a * NT1 + b];
      }
    }
    __syncthreads();
  }

  // gradient into gr (energy() must have set psi, w and the theta table for th):
  // dE/dtheta_k = 2 int_0^1 lam(s)^T G_k phi(s) ds, phi(s) = e^{(1-s)A} Phi,
  // lam(s) = e^{-sA} w, by Gauss-Legendre quadrature; phi and lam move from
  // node to node by the exponential of the node spacing.  Singles
  // G = E_AI - E_IA: lam.E_AI phi - phi.E_AI lam; pairs G = E_AI E_BJ -
  // E_JB E_IA: (E_IA lam).(E_BJ phi) - (E_BJ lam).(E_IA phi).
  __device__ void gradient() {
    for (int k = threadIdx.x; k < NP; k += kVqeBlock) gr[k] = 0.0;
    double* dots = dk + NP;   // NT1 + NT1^2 doubles after the diagonal
    for (int e = threadIdx.x; e < D; e += kVqeBlock) s2[e] = e == 0 ? 1.0 : 0.0;
    __syncthreads();
    double* fp = phi;   // phi and lam at the current node
    double* lp = lam;
    double* tmp = s2;   // the free vector (Phi is no longer needed once phi(s_0) is formed)
    expm_apply(1.0 - kGLx[0], s2, fp);
    expm_apply(-kGLx[0], w, lp);
    for (int q = 0; q < kVqeNodes; ++q) {
      if (q > 0) {
        const double ds = kGLx[q] - kGLx[q - 1];
        expm_apply(-ds, fp, tmp);   // phi(s_q) = e^{-(s_q - s_{q-1}) A} phi(s_{q-1})
        double* t = fp;
        fp = tmp;
        tmp = t;
        expm_apply(-ds, lp, tmp);
        t = lp;
        lp = tmp;
        tmp = t;
      }
      const double wt = 2.0 * kGLw[q];
      // phase 1: X_p = E_AI phi (setA), Y_p = E_IA lam (setB)
      for (int r = threadIdx.x; r < NT1 * D; r += kVqeBlock) {
        const int p1 = r / D, e = r % D;
        const int I = p1 / NV, A = NE + p1 % NV;
        setA[r] = e_at(A * NA + I, fp, e / NS, e % NS);
        setB[r] = e_at(I * NA + A, lp, e / NS, e % NS);
      }
      __syncthreads();
      phase_dots(lp, setA, setB, setA, dots);   // lam.X_p, Y_p1.X_p2
      phase_add(wt, dots);
      // phase 2: X'_p = E_IA phi (setA), Y'_p = E_AI lam (setB)
      for (int r = threadIdx.x; r < NT1 * D; r += kVqeBlock) {
        const int p1 = r / D, e = r % D;
        const int I = p1 / NV, A = NE + p1 % NV;
        setA[r] = e_at(I * NA + A, fp, e / NS, e % NS);
        setB[r] = e_at(A * NA + I, lp, e / NS, e % NS);
      }
      __syncthreads();
      phase_dots(fp, setB, setA, setB, dots);   // phi.Y'_p, X'_p1.Y'_p2
      phase_add(-wt, dots);
    }
  }
};

template <int NA, int NE>
__device__ void vqe_space(const VqeArgs& a, int k, const SpaceDev& sp, double* sm) {
  using V = VqeSpace<NA, NE>;
  constexpr int NS = V::NS, D = V::D, NR = V::NR, NV = V::NV, NT1 = V::NT1, NP = V::NP,
                N2 = V::N2, N4 = V::N4, HS = V::HS;
  const int tid = threadIdx.x;
  const Strings& S = a.strings[sp.nocc - 2];
  const double* hin = a.heff + a.heff_off[k];
  V q{S};
  q.Ec = hin[0];
  const double* h = hin + 1;
  double* cur = sm;
  q.g = cur;
  cur += N4;
  q.Hs = cur;
  cur += NS * HS;
  q.emap = reinterpret_cast<int*>(cur);
  q.rep = q.emap + NS * N2;
  cur += (NS * N2 + NS * NR + 1) / 2;
  q.psi = cur;
  q.w = q.psi + D;
  q.phi = q.w + D;
  q.lam = q.phi + D;
  q.setA = q.lam + D;
  q.setB = q.setA + NT1 * D;
  q.s0 = q.setB + NT1 * D;
  q.s1 = q.s0 + D;
  q.s2 = q.s1 + D;
  q.s3 = q.s2 + D;
  cur = q.s3 + D;
  q.Hinv = cur;
  cur += NP * NP;
  q.th = cur;
  q.gr = q.th + NP;
  q.p = q.gr + NP;
  q.sv = q.p + NP;
  q.yv = q.sv + NP;
  q.th2 = q.yv + NP;
  q.g2 = q.th2 + NP;
  q.dk = q.g2 + NP;   // NP diagonal, then NT1 + NT1*NT1 dots
  cur = q.dk + NP + NT1 + NT1 * NT1;
  q.t2h = cur;        // NT1*NT1
  cur += NT1 * NT1;
  q.red = cur;        // 2 per wavefront
  // integrals, string tables
  for (int e = tid; e < N4; e += kVqeBlock) q.g[e] = hin[1 + N2 + e];
  for (int e = tid; e < NS * N2; e += kVqeBlock) q.emap[e] = 0;
  for (int e = tid; e < NS * NR; e += kVqeBlock) {
    const int I = e / NR, f = e % NR;
    q.rep[e] = S.src[I][f] | (S.pq[I][f] << 8) | ((S.sgn[I][f] > 0) << 16);
  }
  __syncthreads();
  for (int e = tid; e < NS * NR; e += kVqeBlock) {
    const int I = e / NR, f = e % NR;
    q.emap[I * N2 + S.pq[I][f]] = (S.src[I][f] + 1) * (S.sgn[I][f] > 0 ? 1 : -1);
  }
  // same-spin string Hamiltonian, as in the Davidson solver
  double* kk = q.s0;
  for (int e = tid; e < NS * HS; e += kVqeBlock) q.Hs[e] = 0.0;
  for (int e = tid; e < N2; e += kVqeBlock) {
    const int pp = e / NA, qq = e % NA;
    double x = h[pp * NA + qq];
    for (int t = 0; t < NA; ++t) x -= 0.5 * q.g[((pp * NA + t) * NA + t) * NA + qq];
    kk[e] = x;
  }
  __syncthreads();
  if (tid < NS) {
    const int I = tid;
    double* row = q.Hs + I * HS;
    for (int f = 0; f < NR; ++f) {
      const int r = q.rep[I * NR + f];
      const double sg = (r >> 16) ? 1.0 : -1.0;
      row[r & 255] += sg * kk[(r >> 8) & 255];
      const int Kst = r & 255;
      const double* grow = q.g + ((r >> 8) & 255) * N2;
      for (int f2 = 0; f2 < NR; ++f2) {
        const int r2 = q.rep[Kst * NR + f2];
        row[r2 & 255] += 0.5 * sg * ((r2 >> 16) ? 1.0 : -1.0) * grow[(r2 >> 8) & 255];
      }
    }
  }
  __syncthreads();
  // start: the pool's amplitudes of the space (amp layout: t1[NE][NV], then
  // t2[NE][NE][NV][NV]); diagonal of the initial inverse Hessian from the
  // excitation energies of the parameters' determinants
  const double* t0 = a.theta0 + a.amp_off[k];
  for (int kp = tid; kp < NP; kp += kVqeBlock) {
    double x, d;
    if (kp < NT1) {
      x = t0[kp];
      const int I = kp / NV, A = NE + kp % NV;
      // the alpha string of I -> A from the reference string (string 0)
      int str = -1;
      for (int s_ = 0; s_ < NS && str < 0; ++s_) {
        const int m = q.emap[s_ * N2 + A * NA + I];
        if (m != 0 && abs(m) - 1 == 0) str = s_;
      }
      d = str >= 0 ? cas_diag(S, q.Hs, HS, q.g, q.Ec, str, 0) - cas_diag(S, q.Hs, HS, q.g, q.Ec, 0, 0)
                   : 1.0;
    } else {
      int r = kp - NT1, p1 = 0;
      while (r >= NT1 - p1) {
        r -= NT1 - p1;
        ++p1;
      }
      const int p2 = p1 + r;
      const int I = p1 / NV, A = NE + p1 % NV, J = p2 / NV, B = NE + p2 % NV;
      x = t0[NT1 + ((I * NE + J) * NV + (A - NE)) * NV + (B - NE)];
      int sa = -1, sb = -1;
      for (int s_ = 0; s_ < NS; ++s_) {
        const int m1 = q.emap[s_ * N2 + A * NA + I], m2 = q.emap[s_ * N2 + B * NA + J];
        if (m1 != 0 && abs(m1) - 1 == 0) sa = s_;
        if (m2 != 0 && abs(m2) - 1 == 0) sb = s_;
      }
      d = (sa >= 0 && sb >= 0)
              ? cas_diag(S, q.Hs, HS, q.g, q.Ec, sa, sb) - cas_diag(S, q.Hs, HS, q.g, q.Ec, 0, 0)
              : 1.0;
    }
    q.th[kp] = x;
    q.dk[kp] = 1.0 / (4.0 * fmax(d, 0.05));
  }
  __syncthreads();
  auto reset_hinv = [&]() {
    for (int e = tid; e < NP * NP; e += kVqeBlock)
      q.Hinv[e] = (e / NP == e % NP) ? q.dk[e / NP] : 0.0;
    __syncthreads();
  };
  reset_hinv();
  double E = q.energy();
  q.gradient();
  int it = 0;
  bool conv = false;
  for (it = 0; it < a.max_iter; ++it) {
    double gm = 0.0;
    for (int kp = tid; kp < NP; kp += kVqeBlock) gm = fmax(gm, fabs(q.gr[kp]));
    gm = vqe_block_max(gm, q.red);
    if (gm < a.gtol) {
      conv = true;
      break;
    }
    // direction p = -Hinv g; restart from the diagonal if not a descent
    double gp = 0.0;
    for (int r = tid; r < NP; r += kVqeBlock) {
      double x = 0.0;
      for (int c = 0; c < NP; ++c) x -= q.Hinv[r * NP + c] * q.gr[c];
      q.p[r] = x;
      gp += x * q.gr[r];
    }
    gp = vqe_block_sum(gp, q.red);
    if (!(gp < 0.0)) {
      reset_hinv();
      gp = 0.0;
      for (int r = tid; r < NP; r += kVqeBlock) {
        q.p[r] = -q.dk[r] * q.gr[r];
        gp += q.p[r] * q.gr[r];
      }
      gp = vqe_block_sum(gp, q.red);
    }
    // Armijo backtracking; at the energy's resolution the full step is taken
    double alpha = 1.0, En = E;
    bool accepted = false;
    for (int tries = 0; tries < 40; ++tries) {
      for (int kp = tid; kp < NP; kp += kVqeBlock) {
        q.th2[kp] = q.th[kp];
        q.th[kp] = q.th2[kp] + alpha * q.p[kp];
      }
      __syncthreads();
      En = q.energy();
      const bool resolved = fabs(gp) * alpha > 1e-13 * fmax(1.0, fabs(E));
      if (!resolved || En <= E + 1e-4 * alpha * gp) {
        accepted = true;
        break;
      }
      for (int kp = tid; kp < NP; kp += kVqeBlock) q.th[kp] = q.th2[kp];
      __syncthreads();
      alpha *= 0.5;
    }
    if (!accepted) {   // keep theta, restart from the diagonal inverse Hessian
      E = q.energy();
      reset_hinv();
      continue;
    }
    // new gradient; BFGS update of the inverse Hessian
    for (int kp = tid; kp < NP; kp += kVqeBlock) q.g2[kp] = q.gr[kp];
    __syncthreads();
    q.gradient();
    double sy = 0.0;
    for (int kp = tid; kp < NP; kp += kVqeBlock) {
      q.sv[kp] = alpha * q.p[kp];
      q.yv[kp] = q.gr[kp] - q.g2[kp];
      sy += q.sv[kp] * q.yv[kp];
    }
    sy = vqe_block_sum(sy, q.red);
    E = En;
    if (sy > 1e-30) {
      const double rho = 1.0 / sy;
      // Hy = Hinv y (into th2), yHy
      double yhy = 0.0;
      for (int r = tid; r < NP; r += kVqeBlock) {
        double x = 0.0;
        for (int c = 0; c < NP; ++c) x += q.Hinv[r * NP + c] * q.yv[c];
        q.th2[r] = x;
        yhy += x * q.yv[r];
      }
      yhy = vqe_block_sum(yhy, q.red);
      // H <- H - rho (Hy s^T + s (Hy)^T) + (rho^2 yHy + rho) s s^T
      for (int e = tid; e < NP * NP; e += kVqeBlock) {
        const int r = e / NP, c = e % NP;
        q.Hinv[e] += -rho * (q.th2[r] * q.sv[c] + q.sv[r] * q.th2[c]) +
                     (rho * rho * yhy + rho) * q.sv[r] * q.sv[c];
      }
      __syncthreads();
    }
  }
  // outputs: energy, the parameters as local amplitudes, status
  if (tid == 0) {
    a.energy[k] = E;
    a.iters[k] = it;
    a.status[k] = conv ? 0 : -5;
    a.c0[k] = 1.0;
  }
  double* amp = a.amp + a.amp_off[k];
  for (int e = tid; e < NT1; e += kVqeBlock) amp[e] = q.th[e];
  for (int e = tid; e < NT1 * NT1; e += kVqeBlock) {
    const int p1 = e / NT1, p2 = e % NT1;
    const int I = p1 / NV, A = p1 % NV, J = p2 / NV, B = p2 % NV;
    amp[NT1 + ((I * NE + J) * NV + A) * NV + B] = q.t2(p1, p2);
  }
}

template <int NA, int NE>
__global__ __launch_bounds__(kVqeBlock) void k_vqe(VqeArgs a, const int32_t* __restrict__ idx) {
  extern __shared__ double sm[];
  const int k = idx[blockIdx.x];
  vqe_space<NA, NE>(a, k, a.spaces[k], sm);
}

template <int NA, int NE>
void launch_vqe_class(const VqeArgs& a, const int32_t* idx, int count, hipStream_t st) {
  if (count <= 0) return;
  const size_t bytes = (size_t)VqeShape<NA, NE>::LDS * sizeof(double);
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vqe<NA, NE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  k_vqe<NA, NE><<<count, kVqeBlock, bytes, st>>>(a, idx);
}

}  // namespace

int vqe_lds_bytes(int nocc) {
  if (nocc == 2) return (int)(VqeShape<4, 2>::LDS * sizeof(double));
  if (nocc == 3) return (int)(VqeShape<6, 3>::LDS * sizeof(double));
  return -1;
}

void launch_vqe(const VqeArgs& a, const int32_t* cls_idx, const int* cls_off, hipStream_t st) {
  launch_vqe_class<4, 2>(a, cls_idx + cls_off[0], cls_off[1] - cls_off[0], st);
  launch_vqe_class<6, 3>(a, cls_idx + cls_off[1], cls_off[2] - cls_off[1], st);
}

}  // namespace qf
