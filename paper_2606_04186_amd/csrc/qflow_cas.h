// Active-space CI pieces: determinant strings, the CAS-form Hamiltonian of
// one space and its sigma vector.
//
// A space of na orbitals (the first ne of them occupied in Phi) carries ne
// alpha and ne beta electrons.  Alpha (and beta) strings are the
// combinations of ne orbitals out of na in lexicographic order; string 0 is
// the reference.  A determinant is |Ia Ib> = (alpha creators of Ia, ascending)
// (beta creators of Ib, ascending)|vac>, stored as C[Ia * nstr + Ib].  With
// alpha creators first, E^alpha_pq takes signs from the alpha string only and
// E^beta_pq from the beta string only.
//
// The downfolded operator arrives normal ordered with respect to Phi as
// (x0, x1[p,q], x2[p,q,r,s]) (x2 the opposite-spin block, (pr|qs)-like).
// Relative to the empty active space it reads
//   H = Ec + sum h_pq E_pq + 1/2 sum g(pq|rs) (E_pq E_rs - d_qr E_ps),
//   h_pq = x1_pq - sum_k (2 x2_pkqk - x2_pkkq),
//   Ec   = x0 - 2 sum_k x1_kk + sum_kl (2 x2_klkl - x2_kllk),
//   g(pq|rs) = x2_prqs,
// with k,l over the active occupied orbitals.  g keeps only the four-fold
// symmetry (pq|rs) = (rs|pq) = (qp|sr) of a Hermitian spin-free operator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef QF_HD
#define QF_HD __host__ __device__ inline
#endif

namespace qf {

constexpr int kMaxStr = 70;    // C(8,4)
constexpr int kMaxRep = 20;    // ne + ne*(na-ne) <= 4 + 16

// Single-replacement lists: for target string I, entries e < nrep give the
// source string src, the orbital pair (p,q) as p*na+q and the sign of
// <I| a+_p a_q |src>.
struct Strings {
  int na, ne, nstr, nrep;
  int16_t src[kMaxStr][kMaxRep];
  int16_t pq[kMaxStr][kMaxRep];
  int8_t sgn[kMaxStr][kMaxRep];
  uint8_t occ[kMaxStr][8];            // occupied orbitals of each string
  // single excitations of the reference: string and sign of a+_a a_i |ref>
  int16_t exc_str[4][4];              // [i][a - ne]
  int8_t exc_sgn[4][4];
};

// CAS-form Hamiltonian of one space: Ec, h[na][na], g[na^4] (chemist order).
QF_HD void cas_form(int na, int ne, const double* x1, const double* x2, double x0,
                    double* Ec, double* h, double* g) {
  double e = x0;
  for (int k = 0; k < ne; ++k) e -= 2.0 * x1[k * na + k];
  for (int k = 0; k < ne; ++k)
    for (int l = 0; l < ne; ++l)
      e += 2.0 * x2[((k * na + l) * na + k) * na + l] - x2[((k * na + l) * na + l) * na + k];
  *Ec = e;
  for (int p = 0; p < na; ++p)
    for (int q = 0; q < na; ++q) {
      double s = x1[p * na + q];
      for (int k = 0; k < ne; ++k)
        s -= 2.0 * x2[((p * na + k) * na + q) * na + k] - x2[((p * na + k) * na + k) * na + q];
      h[p * na + q] = s;
    }
  for (int p = 0; p < na; ++p)
    for (int q = 0; q < na; ++q)
      for (int r = 0; r < na; ++r)
        for (int s = 0; s < na; ++s)
          g[((p * na + q) * na + r) * na + s] = x2[((p * na + r) * na + q) * na + s];
}

// Same-spin string Hamiltonian Hs[I][J] = <I| sum k_pq E_pq
//   + 1/2 sum g(pq|rs) E_pq E_rs |J> over one spin, k_pq = h_pq - 1/2 sum_r g(pr|rq).
QF_HD double same_spin_element(const Strings& S, const double* h, const double* g, int I, int J) {
  const int na = S.na;
  double x = 0.0;
  for (int e = 0; e < S.nrep; ++e) {
    if (S.src[I][e] != J) continue;
    int p = S.pq[I][e] / na, q = S.pq[I][e] % na;
    double k = h[p * na + q];
    for (int r = 0; r < na; ++r) k -= 0.5 * g[((p * na + r) * na + r) * na + q];
    x += S.sgn[I][e] * k;
  }
  for (int e = 0; e < S.nrep; ++e) {
    int K = S.src[I][e];
    int p = S.pq[I][e] / na, q = S.pq[I][e] % na;
    for (int f = 0; f < S.nrep; ++f) {
      if (S.src[K][f] != J) continue;
      int r = S.pq[K][f] / na, s = S.pq[K][f] % na;
      x += 0.5 * S.sgn[I][e] * S.sgn[K][f] * g[((p * na + q) * na + r) * na + s];
    }
  }
  return x;
}

// Diagonal of the CAS matrix at determinant (Ia, Ib).
QF_HD double cas_diag(const Strings& S, const double* Hs, const double* g, double Ec, int Ia, int Ib) {
  const int na = S.na, n = S.nstr;
  double d = Ec + Hs[Ia * n + Ia] + Hs[Ib * n + Ib];
  for (int a = 0; a < S.ne; ++a)
    for (int b = 0; b < S.ne; ++b) {
      int p = S.occ[Ia][a], r = S.occ[Ib][b];
      d += g[((p * na + p) * na + r) * na + r];
    }
  return d;
}

// One element of sigma = H c at determinant (Ia, Ib).
QF_HD double cas_sigma(const Strings& S, const double* Hs, const double* g, double Ec,
                       const double* c, int Ia, int Ib) {
  const int na = S.na, n = S.nstr;
  double x = Ec * c[Ia * n + Ib];
  for (int J = 0; J < n; ++J) x += Hs[Ia * n + J] * c[J * n + Ib] + Hs[Ib * n + J] * c[Ia * n + J];
  for (int e = 0; e < S.nrep; ++e) {
    int Ja = S.src[Ia][e];
    int pq = S.pq[Ia][e];
    double sa = S.sgn[Ia][e];
    double acc = 0.0;
    for (int f = 0; f < S.nrep; ++f) {
      int Jb = S.src[Ib][f];
      acc += S.sgn[Ib][f] * g[pq * na * na + S.pq[Ib][f]] * c[Ja * n + Jb];
    }
    x += sa * acc;
  }
  return x;
}

}  // namespace qf
