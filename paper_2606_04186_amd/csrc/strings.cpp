// Host construction of the determinant-string tables used by the active-space
// CI kernels (layout documented in qflow_cas.h).
#include <cstring>
#include <vector>

#include "qflow_cas.h"

namespace qf {

static int popc(unsigned x) { return __builtin_popcount(x); }

// sign of a+_p a_q acting on string J (bitmask); requires q in J and
// (p not in J or p == q)
static int repl_sign(unsigned J, int p, int q) {
  int s = (popc(J & ((1u << q) - 1u)) & 1) ? -1 : 1;
  unsigned Jp = J & ~(1u << q);
  s *= (popc(Jp & ((1u << p) - 1u)) & 1) ? -1 : 1;
  return s;
}

bool build_strings(int na, int ne, Strings* S) {
  if (na > 8 || ne > 4 || ne < 1 || ne >= na) return false;
  std::memset(S, 0, sizeof(Strings));
  std::vector<unsigned> strs;
  for (unsigned m = 0; m < (1u << na); ++m)
    if (popc(m) == ne) strs.push_back(m);
  if ((int)strs.size() > kMaxStr) return false;
  S->na = na;
  S->ne = ne;
  S->nstr = (int)strs.size();
  S->nrep = ne * (1 + na - ne);
  auto index = [&](unsigned m) {
    for (size_t k = 0; k < strs.size(); ++k)
      if (strs[k] == m) return (int)k;
    return -1;
  };
  for (int I = 0; I < S->nstr; ++I) {
    unsigned mI = strs[I];
    int e = 0, o = 0;
    for (int p = 0; p < na; ++p)
      if (mI >> p & 1u) S->occ[I][o++] = (uint8_t)p;
    for (int p = 0; p < na; ++p) {
      if (!(mI >> p & 1u)) continue;
      for (int q = 0; q < na; ++q) {
        if (q != p && (mI >> q & 1u)) continue;
        unsigned J = (q == p) ? mI : ((mI & ~(1u << p)) | (1u << q));
        S->src[I][e] = (int16_t)index(J);
        S->pq[I][e] = (int16_t)(p * na + q);
        S->sgn[I][e] = (int8_t)repl_sign(J, p, q);
        ++e;
      }
    }
  }
  unsigned ref = (1u << ne) - 1u;
  for (int i = 0; i < ne; ++i)
    for (int a = ne; a < na; ++a) {
      if (a - ne >= 4) continue;
      unsigned J = (ref & ~(1u << i)) | (1u << a);
      S->exc_str[i][a - ne] = (int16_t)index(J);
      S->exc_sgn[i][a - ne] = (int8_t)repl_sign(ref, a, i);
    }
  return true;
}

// Output-element order for the per-space Hamiltonian kernels: two-body
// elements grouped by their occupied/virtual pattern, then one-body elements,
// then the scalar; every group is padded with idle entries (-1) to a multiple
// of the 64-lane wavefront so that a wavefront evaluates one pattern (one set
// of terms).  Entry = kind << 24 | a << 18 | b << 12 | c << 6 | d with kind
// 2, 1, 0 for two-, one- and zero-body.
// The downfolded operator is Hermitian and spin-free, so its two-body block
// obeys x2_pqrs = x2_qpsr = x2_rspq = x2_srqp and its one-body block is
// symmetric.  Only the lexicographically smallest member of each such orbit
// is a task; the kernels write every distinct member.
static bool canonical2(int a, int b, int c, int d) {
  const int key = ((a * 64 + b) * 64 + c) * 64 + d;
  return key <= ((b * 64 + a) * 64 + d) * 64 + c && key <= ((c * 64 + d) * 64 + a) * 64 + b &&
         key <= ((d * 64 + c) * 64 + b) * 64 + a;
}

int build_tasks(int na, int ne, int32_t* out, int cap) {
  int m = 0;
  auto pad = [&]() {
    while (m % 64) {
      if (m >= cap) return false;
      out[m++] = -1;
    }
    return true;
  };
  for (int pat = 0; pat < 16; ++pat) {
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < na; ++b)
        for (int c = 0; c < na; ++c)
          for (int d = 0; d < na; ++d) {
            const int bits = ((a < ne) << 3) | ((b < ne) << 2) | ((c < ne) << 1) | (d < ne);
            if (bits != pat || !canonical2(a, b, c, d)) continue;
            if (m >= cap) return -1;
            out[m++] = (2 << 24) | (a << 18) | (b << 12) | (c << 6) | d;
          }
    if (!pad()) return -1;
  }
  for (int pat = 0; pat < 4; ++pat) {
    for (int a = 0; a < na; ++a)
      for (int b = a; b < na; ++b) {
        if ((((a < ne) << 1) | (b < ne)) != pat) continue;
        if (m >= cap) return -1;
        out[m++] = (1 << 24) | (a << 18) | (b << 12);
      }
    if (!pad()) return -1;
  }
  if (m >= cap) return -1;
  out[m++] = 0;
  if (!pad()) return -1;
  return m;
}

}  // namespace qf
