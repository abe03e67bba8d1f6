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

// Diagonal of the CAS matrix at determinant (Ia, Ib); Hs is the same-spin
// string Hamiltonian with rows hs_stride apart.
QF_HD double cas_diag(const Strings& S, const double* Hs, int hs_stride, const double* g, double Ec,
                      int Ia, int Ib) {
  const int na = S.na;
  double d = Ec + Hs[Ia * hs_stride + Ia] + Hs[Ib * hs_stride + Ib];
  for (int a = 0; a < S.ne; ++a)
    for (int b = 0; b < S.ne; ++b) {
      int p = S.occ[Ia][a], r = S.occ[Ib][b];
      d += g[((p * na + p) * na + r) * na + r];
    }
  return d;
}


}  // namespace qf
