// Spin-free element evaluator of the downfolded Hamiltonian (Eq. (6), N=1).
//
// A singlet operator is held in spatial orbitals as
//   X = x0 + sum_pq X1[p,q] E_pq + 1/2 sum_pqrs X2[p,q,r,s] sum_{st} {p+_s q+_t s_t r_s}
// with X2[p,q,r,s] the opposite-spin block (p,r on spin s; q,s on spin t) and
// X2[p,q,r,s] = X2[q,p,s,r].  For the bare Hamiltonian X2[p,q,r,s] = (pr|qs).
//
// comm(A,B) below evaluates one element of the normal-ordered commutator
// [A,B] kept to its 0-, 1- and 2-body parts, written directly in this
// spin-free form (the spin sums of the spin-orbital expressions carried out by
// hand).  B is always a cluster operator sigma = T - T^dagger (or a piece of
// it), which has only the excitation blocks S1[v,o] = t1, S1[o,v] = -t1,
// S2[vv,oo] = t2 and S2[oo,vv] = -t2; every loop runs only over index ranges
// where B can be non-zero.
//
// The transformed Hamiltonian of one active space A is
//   Hbar = H + [H_N, s] + 1/2 [[F_N, s], s],  s = sigma_ext = sigma - tau,
// tau = the amplitudes whose indices all lie in A (Eq. (3)).  By bilinearity
//   [H,s] = [H,sigma] - [H,tau]
//   [[F,s],s] = [Yg,sigma] - [Yg,tau] - [Ft,sigma] + [Ft,tau]
// with Yg = [F,sigma] (global, tabulated) and Ft = [F,tau] (evaluated on the
// fly; non-zero only with at least three active indices).  [., sigma] terms use
// the global ladder intermediates L^A[(pq),(ij)] = sum_cd A[p,q,c,d] t2[i,j,c,d]
// for their virtual-virtual contractions.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define QF_HD __host__ __device__ inline
// kept out of line: called from many loop bodies, inlining it everywhere
// multiplies code size without saving work
#define QF_HD_OUTLINE __host__ __device__ __attribute__((noinline))

namespace qf {

constexpr int kMaxOrb = 128;   // orbital limit of the per-space position map
constexpr int kMaxAct = 8;     // active orbitals per space

struct Dims {
  int n, o, v;
};

// ---------------------------------------------------------------------------
// cluster operator pieces
// ---------------------------------------------------------------------------

// Active-space membership: pos[p] = local position of orbital p or -1.
struct Active {
  int na, nocc;              // active orbitals, of which the first nocc occupied
  int orb[kMaxAct];          // absolute orbital indices, occupied first
  int8_t pos[kMaxOrb];
  int next_o, next_v;        // external (inactive) occupied / virtual counts
  uint8_t ext[kMaxOrb];      // external occupied, then external virtual orbitals
  QF_HD bool act(int p) const { return pos[p] >= 0; }
  QF_HD int nact(bool occ) const { return occ ? nocc : na - nocc; }
  QF_HD int actv(bool occ, int k) const { return occ ? orb[k] : orb[nocc + k]; }
  QF_HD int next(bool occ) const { return occ ? next_o : next_v; }
  QF_HD int extv(bool occ, int k) const { return occ ? ext[k] : ext[next_o + k]; }
};

// Fill the external lists of A (host or a single device thread).
QF_HD void active_fill_ext(Active& A, int n, int o) {
  int m = 0;
  for (int p = 0; p < o; ++p)
    if (A.pos[p] < 0) A.ext[m++] = (uint8_t)p;
  A.next_o = m;
  for (int p = o; p < n; ++p)
    if (A.pos[p] < 0) A.ext[m++] = (uint8_t)p;
  A.next_v = m - A.next_o;
}

// Row of the ordered pair (p,q), p <= q, among the n(n+1)/2 such pairs.
QF_HD size_t tri_row(int p, int q, int n) { return (size_t)p * (2 * n - p + 1) / 2 + (q - p); }

// sigma = T - T^dagger from t1[o][v], t2[o][o][v][v].
struct Sigma {
  static constexpr bool kFull = true;
  const double* t1;
  const double* t2;
  int n, o, v;
  QF_HD double one(int p, int q) const {
    if (p >= o && q < o) return t1[q * v + (p - o)];
    if (p < o && q >= o) return -t1[p * v + (q - o)];
    return 0.0;
  }
  QF_HD double two(int p, int q, int r, int s) const {
    if (p >= o && q >= o && r < o && s < o)
      return t2[(((size_t)r * o + s) * v + (p - o)) * v + (q - o)];
    if (p < o && q < o && r >= o && s >= o)
      return -t2[(((size_t)p * o + q) * v + (r - o)) * v + (s - o)];
    return 0.0;
  }
  // loop ranges for indices contracted with this operator
  QF_HD int nocc() const { return o; }
  QF_HD int occ(int k) const { return k; }
  QF_HD int nvir() const { return v; }
  QF_HD int vir(int k) const { return o + k; }
};

// tau = the part of sigma whose indices all lie in the active space.
struct Tau {
  static constexpr bool kFull = false;
  Sigma s;
  const Active* A;
  QF_HD double one(int p, int q) const {
    return (A->act(p) && A->act(q)) ? s.one(p, q) : 0.0;
  }
  QF_HD double two(int p, int q, int r, int s_) const {
    return (A->act(p) && A->act(q) && A->act(r) && A->act(s_)) ? s.two(p, q, r, s_) : 0.0;
  }
  QF_HD int nocc() const { return A->nocc; }
  QF_HD int occ(int k) const { return A->orb[k]; }
  QF_HD int nvir() const { return A->na - A->nocc; }
  QF_HD int vir(int k) const { return A->orb[A->nocc + k]; }
};

// ---------------------------------------------------------------------------
// the "A" operators
// ---------------------------------------------------------------------------

// U = [G, sigma_2]_2 of a Hermitian one-body G evaluated from the compact
// contractions of the K = v and K = o GEMMs (P1..P4, Q1, Q2; layouts as in
// launch_sigma2) instead of a dense n^4 array: a few lookups per element.
// Zero unless r,s or p,q share a class.  (g and t2 are kept for callers that
// name them; every case reads P and Q.)
struct Sigma2Lazy {
  const double* g;    // G [n][n]
  const double* t2;
  const double* P;    // [4][n][o*o*v]
  const double* Q;    // [2][n][o*v*v]
  int n, o;
  QF_HD double operator()(int p, int q, int r, int s) const {
    const int v = n - o;
    const bool op = p < o, oq = q < o, or_ = r < o, os = s < o;
    const size_t ov2 = (size_t)o * o * v, nv = (size_t)n * ov2;
    const size_t vv = (size_t)v * v, ovv = (size_t)o * vv;
    double x = 0.0;
    if (or_ == os) {
      if (or_) {
        const size_t rs = ((size_t)r * o + s) * v;
        if (!oq) x += P[(size_t)p * ov2 + rs + (q - o)];
        if (!op) x += P[nv + (size_t)q * ov2 + rs + (p - o)];
      } else {
        const size_t rs = (size_t)(r - o) * v + (s - o);
        if (oq) x += Q[(size_t)p * ovv + (size_t)q * vv + rs];
        if (op) x += Q[(size_t)n * ovv + (size_t)q * ovv + (size_t)p * vv + rs];
      }
    }
    if (op == oq) {
      if (op) {
        const size_t pq = ((size_t)p * o + q) * v;
        if (!os) x += P[2 * nv + (size_t)r * ov2 + pq + (s - o)];
        if (!or_) x += P[3 * nv + (size_t)s * ov2 + pq + (r - o)];
      } else {
        // p, q virtual: -sum_{t occ} G_tr t2[t,s,p,q] (s occupied) and
        // -sum_{t occ} G_ts t2[r,t,p,q] (r occupied) are Q1[r][(s,p,q)] and
        // Q2[s][(r,p,q)] (G symmetric)
        const size_t ab = (size_t)(p - o) * v + (q - o);
        if (os) x += Q[(size_t)r * ovv + (size_t)s * vv + ab];
        if (or_) x += Q[(size_t)n * ovv + (size_t)s * ovv + (size_t)r * vv + ab];
      }
    }
    return x;
  }
};

// Dense operator A (H_N, or Yg) with its global contractions against sigma:
//   L[(pq)][(ij)]       = sum_{c,d virtual} A[p,q,c,d] t2[i,j,c,d]       (ladder)
//   Ga[(ab)][(g d)]     = sum_{u occ, t virt} (2 A[a,u,b,t] - A[a,u,t,b]) t2[u,d,t,g]
//                                           - A[a,u,b,t] t2[d,u,t,g]      (rings)
//   G22[(ab)][(g d)]    = sum_{u occ, t virt} A[a,u,t,b] t2[d,u,t,g]
//   J1[p][q]            = - sum_{t,u occ, w virt} A[w,p,t,u] (2 t2[t,u,w,q] - t2[t,u,q,w])
//   J2[q][p]            = - sum_{t,u occ, w virt} t2[t,u,w,p] (2 A[t,u,w,q] - A[t,u,q,w])
// (g, q, p in J virtual; column index of Ga/G22 = (g - o) * o + d).
struct DenseOp {
  static constexpr bool kHasL = true;
  static constexpr bool kSparse3 = false;
  const double* x1;   // [n][n]
  const double* x2;   // [n][n][n][n]
  const double* L;    // [n(n+1)/2][o*o], rows p <= q
  int n, o;
  const double* Ga = nullptr;    // [n*n][v*o]
  const double* G22 = nullptr;   // [n*n][v*o]
  const double* J1 = nullptr;    // [n][v]
  const double* J2 = nullptr;    // [n][v]
  const double* U = nullptr;     // [n][n][n][n], [x1, sigma_2]_2; when NULL, Ul is used
  const double* Lo = nullptr;    // [v*v][o*o], sum_{tu occ} t2[t,u,a,b] x2(t,u,i,j)
  Sigma2Lazy Ul{};
  // [n][n][n][n], sum_t sigma1(p,t) x2(t,q,r,s); NULL when the caller adds
  // this part itself
  const double* Z = nullptr;
  QF_HD double one(int p, int q) const { return x1[p * n + q]; }
  QF_HD double two(int p, int q, int r, int s) const {
    return x2[(((size_t)p * n + q) * n + r) * n + s];
  }
  // L holds the rows p <= q only (packed, tri_row); L[(q,p)][(j,i)] = L[(p,q)][(i,j)]
  // by the pair symmetry of A and t2
  QF_HD double lad(int p, int q, int i, int j) const {
    return p <= q ? L[tri_row(p, q, n) * o * o + i * o + j]
                  : L[tri_row(q, p, n) * o * o + j * o + i];
  }
  QF_HD double ga(int a, int b, int g, int d) const {
    return Ga[((size_t)a * n + b) * (size_t)(n - o) * o + (size_t)(g - o) * o + d];
  }
  QF_HD double g22(int a, int b, int g, int d) const {
    return G22[((size_t)a * n + b) * (size_t)(n - o) * o + (size_t)(g - o) * o + d];
  }
  QF_HD double j1(int p, int q) const { return J1[p * (n - o) + (q - o)]; }
  QF_HD double j2(int q, int p) const { return J2[q * (n - o) + (p - o)]; }
  QF_HD double z(int p, int q, int r, int s) const {
    return Z[(((size_t)p * n + q) * n + r) * n + s];
  }
  QF_HD double u(int p, int q, int r, int s) const {
    return U ? U[(((size_t)p * n + q) * n + r) * n + s] : Ul(p, q, r, s);
  }
  QF_HD double lo(int a, int b, int i, int j) const {
    const int v = n - o;
    return Lo[((size_t)(a - o) * v + (b - o)) * o * o + i * o + j];
  }
  QF_HD bool act(int) const { return true; }
};

// An operator restricted to the active space in local indices (positions in
// A.orb, occupied first): x1[a][b], x2[a][b][c][d].  [X, tau] restricted to
// the space involves only X restricted to the space, so Comm<LocalOp,
// LocalOp> with n = na, o = nocc evaluates it entirely from these arrays;
// as the B operand (tau) its loop ranges are the active orbitals.
struct LocalOp {
  static constexpr bool kHasL = false;
  static constexpr bool kSparse3 = false;
  static constexpr bool kFull = false;
  const double* x1;
  const double* x2;
  int na, no;
  QF_HD double one(int p, int q) const { return x1[p * na + q]; }
  QF_HD double two(int p, int q, int r, int s) const {
    return x2[((p * na + q) * na + r) * na + s];
  }
  QF_HD bool act(int) const { return true; }
  QF_HD int nocc() const { return no; }
  QF_HD int occ(int k) const { return k; }
  QF_HD int nvir() const { return na - no; }
  QF_HD int vir(int k) const { return no + k; }
};

// Ft = [F_N, tau]: non-zero only where at least three indices (two-body) or
// one index (one-body) are active.
struct FtauOp {
  static constexpr bool kHasL = false;
  static constexpr bool kSparse3 = true;
  const double* f;
  Tau tau;
  int n, o;
  QF_HD bool act(int p) const { return tau.A->act(p); }
  QF_HD double one(int p, int q) const {
    const Active* A = tau.A;
    if (!A->act(p) && !A->act(q)) return 0.0;
    return one_full(p, q);
  }
  QF_HD_OUTLINE double one_full(int p, int q) const {
    const Active* A = tau.A;
    double r = 0.0;
    for (int k = 0; k < A->na; ++k) {
      int t = A->orb[k];
      r += f[p * n + t] * tau.one(t, q) - tau.one(p, t) * f[t * n + q];
    }
    // sum_tu (n_t - n_u) f_tu (2 tau_uptq - tau_upqt)
    for (int a = 0; a < A->nocc; ++a)
      for (int b = A->nocc; b < A->na; ++b) {
        int t = A->orb[a], u = A->orb[b];
        r += f[t * n + u] * (2.0 * tau.two(u, p, t, q) - tau.two(u, p, q, t));
        r -= f[u * n + t] * (2.0 * tau.two(t, p, u, q) - tau.two(t, p, q, u));
      }
    return r;
  }
  QF_HD double two(int p, int q, int r, int s) const {
    const Active* A = tau.A;
    int na = (int)A->act(p) + (int)A->act(q) + (int)A->act(r) + (int)A->act(s);
    if (na < 3) return 0.0;
    return two_full(p, q, r, s);
  }
  QF_HD_OUTLINE double two_full(int p, int q, int r, int s) const {
    const Active* A = tau.A;
    double x = 0.0;
    for (int k = 0; k < A->na; ++k) {
      int t = A->orb[k];
      x += f[p * n + t] * tau.two(t, q, r, s) + f[q * n + t] * tau.two(p, t, r, s)
         - f[t * n + r] * tau.two(p, q, t, s) - f[t * n + s] * tau.two(p, q, r, t);
    }
    return x;
  }
  QF_HD double zero() const {
    const Active* A = tau.A;
    double z = 0.0;
    for (int a = 0; a < A->nocc; ++a)
      for (int b = A->nocc; b < A->na; ++b) {
        int t = A->orb[a], u = A->orb[b];
        z += f[t * n + u] * tau.one(u, t) - f[u * n + t] * tau.one(t, u);
      }
    return 2.0 * z;
  }
};

// ---------------------------------------------------------------------------
// the commutator elements
// ---------------------------------------------------------------------------

template <class AOp, class BOp>
struct Comm {
  const AOp& a;
  const BOp& b;
  int n, o;
  // Work split: every contraction loop runs over indices ln, ln+nl, ...; the
  // caller sums the partial results of the nl lanes (nl = 1: one evaluator
  // does everything).  Terms without a loop are taken by lane 0.
  int ln = 0, nl = 1;
  // false: leave out the sigma1 x A_2 part of the one-body element (the
  // caller evaluates it for all (p,q) at once)
  bool ring1 = true;
  // false (dense A): leave out the occupied-pair ladders of the two-body
  // element that have no precomputed form, sum_{t,u occ} A_pqtu t2[t,u,r,s]
  // (r,s virtual, p,q not both occupied) and its mirror (p,q virtual, r,s
  // not both occupied); the caller adds them (per-space tables)
  bool pp_loops = true;

  QF_HD bool occ(int p) const { return p < o; }
  QF_HD bool lead() const { return ln == 0; }
  static constexpr bool kUseL = AOp::kHasL && BOp::kFull;
  static constexpr bool kRestrict = AOp::kSparse3 && BOp::kFull;

  // loops over the block of index p (occupied or virtual), contracted with B
  template <class F>
  QF_HD void over_block(bool occupied, F fn) const {
    if (occupied)
      for (int k = ln; k < b.nocc(); k += nl) fn(b.occ(k));
    else
      for (int k = ln; k < b.nvir(); k += nl) fn(b.vir(k));
  }
  // pairs (t in block bt, u in block bu), t fastest
  template <class F>
  QF_HD void over_pair(bool bt, bool bu, F fn) const {
    const int nt = bt ? b.nocc() : b.nvir(), nu = bu ? b.nocc() : b.nvir();
    for (int k = ln; k < nt * nu; k += nl) {
      const int it = k % nt, iu = k / nt;
      fn(bt ? b.occ(it) : b.vir(it), bu ? b.occ(iu) : b.vir(iu));
    }
  }

  // sum_{t,u virtual} A[p,q,t,u] B[t,u,r,s]  (r,s occupied)
  QF_HD double ladder_vv(int p, int q, int r, int s) const {
    if constexpr (kUseL) {
      return lead() ? a.lad(p, q, r, s) : 0.0;
    } else {
      double x = 0.0;
      over_pair(false, false, [&](int t, int u) {
        if constexpr (kRestrict) {
          if ((int)a.act(p) + (int)a.act(q) + (int)a.act(t) + (int)a.act(u) < 3) return;
        }
        x += a.two(p, q, t, u) * b.two(t, u, r, s);
      });
      return x;
    }
  }

  // sum_{t,u virtual} B[p,q,t,u] A[t,u,r,s]  (p,q occupied)
  QF_HD double ladder_vv_rev(int p, int q, int r, int s) const {
    if constexpr (kUseL) {
      // B[p,q,c,d] = -t2[p,q,c,d]; A[c,d,r,s] = A[r,s,c,d] (Hermitian)
      return lead() ? -a.lad(r, s, p, q) : 0.0;
    } else {
      double x = 0.0;
      over_pair(false, false, [&](int t, int u) {
        if constexpr (kRestrict) {
          if ((int)a.act(r) + (int)a.act(s) + (int)a.act(t) + (int)a.act(u) < 3) return;
        }
        x += b.two(p, q, t, u) * a.two(t, u, r, s);
      });
      return x;
    }
  }

  // ----- two-body element [A,B][p,q,r,s] -----
  QF_HD double c2(int p, int q, int r, int s) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q), or_ = occ(r), os = occ(s);
    // one-body A x two-body B:
    //   sum_t [A_pt B_tqrs + A_qt B_ptrs - A_tr B_pqts - A_ts B_pqrt]
    if constexpr (kUseL) {
      if (lead()) res += a.u(p, q, r, s);   // precomputed [A_1, B_2]_2
    } else {
      if (or_ == os && oq != or_)
        over_block(oq, [&](int t) { res += a.one(p, t) * b.two(t, q, r, s); });
      if (or_ == os && op != or_)
        over_block(op, [&](int t) { res += a.one(q, t) * b.two(p, t, r, s); });
      if (op == oq && os != op)
        over_block(os, [&](int t) { res -= a.one(t, r) * b.two(p, q, t, s); });
      if (op == oq && or_ != op)
        over_block(or_, [&](int t) { res -= a.one(t, s) * b.two(p, q, r, t); });
    }
    // one-body B x two-body A:
    //   - sum_t [B_pt A_tqrs + B_qt A_ptrs - B_tr A_pqts - B_ts A_pqrt]
    // = -(Z_pqrs + Z_qpsr + Z_rspq + Z_srqp) with Z = B A over the first index
    // (A Hermitian and pair symmetric, B anti-Hermitian).  A dense operator
    // either carries Z or leaves this part to the caller (per-space tables,
    // the residual's vvoo pieces).
    if constexpr (kUseL) {
      if (lead() && a.Z) res -= a.z(p, q, r, s) + a.z(q, p, s, r) + a.z(r, s, p, q) + a.z(s, r, q, p);
    } else {
      over_block(!op, [&](int t) { res -= b.one(p, t) * a.two(t, q, r, s); });
      over_block(!oq, [&](int t) { res -= b.one(q, t) * a.two(p, t, r, s); });
      over_block(!or_, [&](int t) { res += b.one(t, r) * a.two(p, q, t, s); });
      over_block(!os, [&](int t) { res += b.one(t, s) * a.two(p, q, r, t); });
    }
    // ladders: sum_tu (1 - n_t - n_u)(A_pqtu B_turs - B_pqtu A_turs)
    if (or_ && os) res += ladder_vv(p, q, r, s);
    // (the occupied-occupied / virtual-virtual cases are the precomputed Lo,
    // using A_pqtu = A_tupq)
    if (!or_ && !os) {
      bool done = false;
      if constexpr (kUseL) {
        if (op && oq) {
          if (lead()) res += a.lo(r, s, p, q);
          done = true;
        }
      }
      if (!done && (!kUseL || pp_loops))
        over_pair(true, true, [&](int t, int u) { res -= a.two(p, q, t, u) * b.two(t, u, r, s); });
    }
    if (!op && !oq) {
      bool done = false;
      if constexpr (kUseL) {
        if (or_ && os) {
          if (lead()) res += a.lo(p, q, r, s);
          done = true;
        }
      }
      if (!done && (!kUseL || pp_loops))
        over_pair(true, true, [&](int t, int u) { res += b.two(p, q, t, u) * a.two(t, u, r, s); });
    }
    if (op && oq) res -= ladder_vv_rev(p, q, r, s);
    // particle-hole terms: Xa(p,q,r,s) - Xb - Xc + Xa(q,p,s,r)
    res += xa(p, q, r, s) - xb(p, q, r, s) - xc(p, q, r, s) + xa(q, p, s, r);
    return res;
  }

  // sum over t virtual, u occupied, both contracted with B (t fastest)
  template <class F>
  QF_HD void over_vo(F fn) const {
    over_pair(false, true, fn);
  }

  // Xa = sum_{t v, u o} [ -A_putr B_tqus + 2 A_purt B_tqus - A_purt B_tqsu
  //                       + B_putr A_tqus - 2 B_purt A_tqus + B_purt A_tqsu ]
  QF_HD double xa(int p, int q, int r, int s) const {
    double x = 0.0;
    if constexpr (kUseL) {
      if (!lead()) return 0.0;
      if (!occ(q) && occ(s)) x += a.ga(p, r, q, s);
      if (occ(p) && !occ(r)) x += a.ga(s, q, r, p);
      return x;
    }
    if (!occ(q) && occ(s))
      over_vo([&](int t, int u) {
        x += (2.0 * a.two(p, u, r, t) - a.two(p, u, t, r)) * b.two(t, q, u, s)
           - a.two(p, u, r, t) * b.two(t, q, s, u);
      });
    if (occ(p) && !occ(r))
      over_vo([&](int t, int u) {
        x += (b.two(p, u, t, r) - 2.0 * b.two(p, u, r, t)) * a.two(t, q, u, s)
           + b.two(p, u, r, t) * a.two(t, q, s, u);
      });
    return x;
  }
  // Xb = sum_{t v, u o} [A_qutr B_tpsu - B_qutr A_tpsu]
  QF_HD double xb(int p, int q, int r, int s) const {
    double x = 0.0;
    if constexpr (kUseL) {
      if (!lead()) return 0.0;
      if (!occ(p) && occ(s)) x += a.g22(q, r, p, s);
      if (occ(q) && !occ(r)) x += a.g22(s, p, r, q);
      return x;
    }
    if (!occ(p) && occ(s))
      over_vo([&](int t, int u) { x += a.two(q, u, t, r) * b.two(t, p, s, u); });
    if (occ(q) && !occ(r))
      over_vo([&](int t, int u) { x -= b.two(q, u, t, r) * a.two(t, p, s, u); });
    return x;
  }
  // Xc = sum_{t v, u o} [A_puts B_tqru - B_puts A_tqru]
  QF_HD double xc(int p, int q, int r, int s) const {
    double x = 0.0;
    if constexpr (kUseL) {
      if (!lead()) return 0.0;
      if (!occ(q) && occ(r)) x += a.g22(p, s, q, r);
      if (occ(p) && !occ(s)) x += a.g22(r, q, s, p);
      return x;
    }
    if (!occ(q) && occ(r))
      over_vo([&](int t, int u) { x += a.two(p, u, t, s) * b.two(t, q, r, u); });
    if (occ(p) && !occ(s))
      over_vo([&](int t, int u) { x -= b.two(p, u, t, s) * a.two(t, q, r, u); });
    return x;
  }

  // ----- one-body element [A,B][p,q] -----
  QF_HD double c1(int p, int q) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q);
    // sum_t (A_pt B_tq - B_pt A_tq)
    over_block(!oq, [&](int t) { res += a.one(p, t) * b.one(t, q); });
    over_block(!op, [&](int t) { res -= b.one(p, t) * a.one(t, q); });
    // sum_tu (n_t - n_u) [A_tu (2 B_uptq - B_upqt) - B_tu (2 A_uptq - A_upqt)]
    if (!op && oq)   // t occupied, u virtual
      over_pair(true, false, [&](int t, int u) {
        res += a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
      });
    if (op && !oq)   // t virtual, u occupied (sign -1)
      over_pair(false, true, [&](int t, int u) {
        res -= a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
      });
    if (ring1)
      over_pair(true, false, [&](int t, int u) {
        res -= b.one(t, u) * (2.0 * a.two(u, p, t, q) - a.two(u, p, q, t));
        res += b.one(u, t) * (2.0 * a.two(t, p, u, q) - a.two(t, p, q, u));
      });
    // sum_tuw (n_t n_u nb_w + nb_t nb_u n_w)
    //      [A_wptu (2 B_tuwq - B_tuqw) - B_wptu (2 A_tuwq - A_tuqw)]
    // (t,u occupied, w virtual): B_tuwq needs q virtual, B_wptu needs p virtual
    if constexpr (kUseL) {
      if (lead()) {
        if (!oq) res += a.j1(p, q);
        if (!op) res += a.j2(q, p);
      }
    } else if (!oq || !op)
      over_pair(true, true, [&](int t, int u) {
        if constexpr (kRestrict) {
          int c = (int)a.act(t) + (int)a.act(u) + (int)a.act(p) + (int)a.act(q);
          if (c < 1) return;
        }
        for (int m = 0; m < b.nvir(); ++m) {
          int w = b.vir(m);
          if (!oq) res += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
          if (!op) res -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
        }
      });
    // (t,u virtual, w occupied): B_tuwq needs q occupied, B_wptu needs p occupied
    if (oq) res += c1_vvo(p, q);
    if (op) res += c1_vvo_rev(p, q);
    return res;
  }

  // sum_{w o; t,u v} A_wptu (2 B_tuwq - B_tuqw), q occupied
  QF_HD double c1_vvo(int p, int q) const {
    double x = 0.0;
    if constexpr (kUseL) {
      for (int w = ln; w < o; w += nl) x += 2.0 * a.lad(w, p, w, q) - a.lad(w, p, q, w);
    } else {
      over_pair(false, false, [&](int t, int u) {
        for (int m = 0; m < b.nocc(); ++m) {
          const int w = b.occ(m);
          if constexpr (kRestrict) {
            if ((int)a.act(w) + (int)a.act(p) + (int)a.act(t) + (int)a.act(u) < 3) continue;
          }
          x += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
        }
      });
    }
    return x;
  }

  // - sum_{w o; t,u v} B_wptu (2 A_tuwq - A_tuqw), p occupied
  QF_HD double c1_vvo_rev(int p, int q) const {
    double x = 0.0;
    if constexpr (kUseL) {
      // B_wptu = -t2[w,p,t,u]; A_tuwq = A_wqtu (Hermitian)
      for (int w = ln; w < o; w += nl) x += 2.0 * a.lad(w, q, w, p) - a.lad(q, w, w, p);
    } else {
      over_pair(false, false, [&](int t, int u) {
        for (int m = 0; m < b.nocc(); ++m) {
          const int w = b.occ(m);
          if constexpr (kRestrict) {
            if ((int)a.act(w) + (int)a.act(q) + (int)a.act(t) + (int)a.act(u) < 3) continue;
          }
          x -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
        }
      });
    }
    return x;
  }

  // ----- zero-body part -----
  QF_HD double c0() const {
    double z = 0.0;
    // 2 sum_tu (n_t - n_u) A_tu B_ut
    over_pair(true, false, [&](int t, int u) {
      z += 2.0 * (a.one(t, u) * b.one(u, t) - a.one(u, t) * b.one(t, u));
    });
    // sum_{tu o, wx v} [A_tuwx (2 B_wxtu - B_wxut) - B_tuwx (2 A_wxtu - A_wxut)]
    if constexpr (kUseL) {
      over_pair(true, true, [&](int t, int u) {
        z += 4.0 * a.lad(t, u, t, u) - a.lad(t, u, u, t) - a.lad(u, t, t, u);
      });
    } else {
      over_pair(true, true, [&](int t, int u) {
        for (int m = 0; m < b.nvir(); ++m)
          for (int r = 0; r < b.nvir(); ++r) {
            const int w = b.vir(m), x = b.vir(r);
            if constexpr (kRestrict) {
              if ((int)a.act(t) + (int)a.act(u) + (int)a.act(w) + (int)a.act(x) < 3) continue;
            }
            z += a.two(t, u, w, x) * (2.0 * b.two(w, x, t, u) - b.two(w, x, u, t))
               - b.two(t, u, w, x) * (2.0 * a.two(w, x, t, u) - a.two(w, x, u, t));
          }
      });
    }
    return z;
  }
};

template <class AOp, class BOp>
QF_HD Comm<AOp, BOp> make_comm_split(const AOp& a, const BOp& b, int n, int o, int ln, int nl) {
  return Comm<AOp, BOp>{a, b, n, o, ln, nl};
}

// ---------------------------------------------------------------------------
// [E, sigma] restricted to the active space, E = the part of [F,tau] with
// exactly one index outside the space.  For outputs inside the space,
//   [Ft,sigma] - [Ft,tau] = [E,sigma]
// because the all-active part of Ft meets only amplitudes inside the space
// (where sigma = tau), and E cannot contract with tau.  Every term of
// [E,sigma] therefore has exactly one external contracted index (E's
// external leg); the loops below enumerate only those index combinations.
// ---------------------------------------------------------------------------
// Loop policy over the external index: either the external orbitals
// themselves (kMarked = false), or, with the sum over the external orbital x
// moved inside per-space tables, the active orbital t that E's Fock leg
// attaches to (kMarked = true; the index is passed as the marker -1-t).
// The marker of the marked evaluation: the active orbital t that E's Fock leg
// attaches to, carried as its own type so that each accessor call resolves
// the marked slot at compile time.
struct Mk {
  int t;
};

template <class EOp, class BOp, bool kMarked = false, class ActT = Active>
struct CommE {
  const EOp& a;        // E accessor (one index external, or marked)
  const BOp& b;        // sigma accessor (one index external, or marked)
  const ActT& A;
  int n, o;
  // Lane split of the one- and zero-body elements: the terms are taken in
  // turn by lanes ln, ln + nl, ...; the caller sums the nl partial results.
  int ln = 0, nl = 1;

  // In marked mode every index is local (the position in A.orb, occupied
  // first) and markers are negative; the class tests below never see markers.
  QF_HD bool occ(int p) const {
    if constexpr (kMarked) return p < A.nocc;
    else return p < o;
  }
  QF_HD int act_at(bool occupied, int m) const {
    if constexpr (kMarked) return occupied ? m : A.nocc + m;
    else return A.actv(occupied, m);
  }

  template <class F>
  QF_HD void over_ext(bool occupied, F fn) const {
    if constexpr (kMarked) {
#pragma unroll 1
      for (int t = 0; t < A.na; ++t) fn(Mk{t});
    } else {
#pragma unroll 1
      for (int k = 0; k < A.next(occupied); ++k) fn(A.extv(occupied, k));
    }
  }
  // (t in block bt, u in block bu) with exactly one of t, u external
  template <class F>
  QF_HD void pair1(bool bt, bool bu, F fn) const {
    over_ext(bt, [&](auto x) {
#pragma unroll 1
      for (int m = 0; m < A.nact(bu); ++m) fn(x, act_at(bu, m));
    });
#pragma unroll 1
    for (int k = 0; k < A.nact(bt); ++k) {
      const int t = act_at(bt, k);
      over_ext(bu, [&](auto x) { fn(t, x); });
    }
  }
  // (t, u, w) with exactly one external
  template <class F>
  QF_HD void triple1(bool bt, bool bu, bool bw, F fn) const {
    over_ext(bt, [&](auto x) {
#pragma unroll 1
      for (int j = 0; j < A.nact(bu); ++j)
#pragma unroll 1
        for (int k = 0; k < A.nact(bw); ++k) fn(x, act_at(bu, j), act_at(bw, k));
    });
#pragma unroll 1
    for (int i = 0; i < A.nact(bt); ++i)
      over_ext(bu, [&](auto x) {
#pragma unroll 1
        for (int k = 0; k < A.nact(bw); ++k) fn(act_at(bt, i), x, act_at(bw, k));
      });
#pragma unroll 1
    for (int i = 0; i < A.nact(bt); ++i)
#pragma unroll 1
      for (int j = 0; j < A.nact(bu); ++j)
        over_ext(bw, [&](auto x) { fn(act_at(bt, i), act_at(bu, j), x); });
  }

  QF_HD double c2(int p, int q, int r, int s) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q), or_ = occ(r), os = occ(s);
    if (or_ == os && oq != or_) over_ext(oq, [&](auto t) { res += a.one(p, t) * b.two(t, q, r, s); });
    if (or_ == os && op != or_) over_ext(op, [&](auto t) { res += a.one(q, t) * b.two(p, t, r, s); });
    if (op == oq && os != op) over_ext(os, [&](auto t) { res -= a.one(t, r) * b.two(p, q, t, s); });
    if (op == oq && or_ != op) over_ext(or_, [&](auto t) { res -= a.one(t, s) * b.two(p, q, r, t); });
    over_ext(!op, [&](auto t) { res -= b.one(p, t) * a.two(t, q, r, s); });
    over_ext(!oq, [&](auto t) { res -= b.one(q, t) * a.two(p, t, r, s); });
    over_ext(!or_, [&](auto t) { res += b.one(t, r) * a.two(p, q, t, s); });
    over_ext(!os, [&](auto t) { res += b.one(t, s) * a.two(p, q, r, t); });
    if (or_ && os) pair1(false, false, [&](auto t, auto u) { res += a.two(p, q, t, u) * b.two(t, u, r, s); });
    if (!or_ && !os) pair1(true, true, [&](auto t, auto u) { res -= a.two(p, q, t, u) * b.two(t, u, r, s); });
    if (!op && !oq) pair1(true, true, [&](auto t, auto u) { res += b.two(p, q, t, u) * a.two(t, u, r, s); });
    if (op && oq) pair1(false, false, [&](auto t, auto u) { res -= b.two(p, q, t, u) * a.two(t, u, r, s); });
    res += xa(p, q, r, s) - xb(p, q, r, s) - xc(p, q, r, s) + xa(q, p, s, r);
    return res;
  }
  QF_HD double xa(int p, int q, int r, int s) const {
    double x = 0.0;
    if (!occ(q) && occ(s))
      pair1(false, true, [&](auto t, auto u) {
        x += (2.0 * a.two(p, u, r, t) - a.two(p, u, t, r)) * b.two(t, q, u, s)
           - a.two(p, u, r, t) * b.two(t, q, s, u);
      });
    if (occ(p) && !occ(r))
      pair1(false, true, [&](auto t, auto u) {
        x += (b.two(p, u, t, r) - 2.0 * b.two(p, u, r, t)) * a.two(t, q, u, s)
           + b.two(p, u, r, t) * a.two(t, q, s, u);
      });
    return x;
  }
  QF_HD double xb(int p, int q, int r, int s) const {
    double x = 0.0;
    if (!occ(p) && occ(s)) pair1(false, true, [&](auto t, auto u) { x += a.two(q, u, t, r) * b.two(t, p, s, u); });
    if (occ(q) && !occ(r)) pair1(false, true, [&](auto t, auto u) { x -= b.two(q, u, t, r) * a.two(t, p, s, u); });
    return x;
  }
  QF_HD double xc(int p, int q, int r, int s) const {
    double x = 0.0;
    if (!occ(q) && occ(r)) pair1(false, true, [&](auto t, auto u) { x += a.two(p, u, t, s) * b.two(t, q, r, u); });
    if (occ(p) && !occ(s)) pair1(false, true, [&](auto t, auto u) { x -= b.two(p, u, t, s) * a.two(t, q, r, u); });
    return x;
  }

  // ----- lane-split enumerations (the one- and zero-body elements) -----
  QF_HD int ext_count(bool occupied) const {
    if constexpr (kMarked) return A.na;
    else return A.next(occupied);
  }
  template <class F>
  QF_HD void ext_call(bool occupied, int k, F fn) const {
    if constexpr (kMarked) fn(Mk{k});
    else fn(A.extv(occupied, k));
  }
  // The index tuples over the blocks b[0..N) with exactly one external
  // index, as one flat range: segment s holds the tuples whose external is
  // in position s.  Lane ln takes the flat indices ln, ln + nl, ...; g gets
  // the segment and the tuple (the external's number in position s, active
  // positions elsewhere).
  template <int N, class G>
  QF_HD void s_flat(const bool (&b)[N], G g) const {
    int base = 0;
#pragma unroll
    for (int s = 0; s < N; ++s) {
      int dim[N], size = 1;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        dim[i] = i == s ? ext_count(b[i]) : A.nact(b[i]);
        size *= dim[i];
      }
      const int j0 = (((ln - base) % nl) + nl) % nl;
#pragma unroll 1
      for (int j = j0; j < size; j += nl) {
        int id[N], r = j;
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
          id[i] = r % dim[i];
          r /= dim[i];
        }
        g(s, id);
      }
      base += size;
    }
  }
  // fn(t, u): exactly one of t (block bt), u (block bu) external
  template <class F>
  QF_HD void s_pair1(bool bt, bool bu, F fn) const {
    const bool b[2] = {bt, bu};
    s_flat<2>(b, [&](int s, const int* id) {
      if (s == 0) ext_call(bt, id[0], [&](auto x) { fn(x, act_at(bu, id[1])); });
      else ext_call(bu, id[1], [&](auto x) { fn(act_at(bt, id[0]), x); });
    });
  }
  // fn(t, u, w): exactly one external
  template <class F>
  QF_HD void s_triple1(bool bt, bool bu, bool bw, F fn) const {
    const bool b[3] = {bt, bu, bw};
    s_flat<3>(b, [&](int s, const int* id) {
      if (s == 0) {
        ext_call(bt, id[0], [&](auto x) { fn(x, act_at(bu, id[1]), act_at(bw, id[2])); });
      } else if (s == 1) {
        ext_call(bu, id[1], [&](auto x) { fn(act_at(bt, id[0]), x, act_at(bw, id[2])); });
      } else {
        ext_call(bw, id[2], [&](auto x) { fn(act_at(bt, id[0]), act_at(bu, id[1]), x); });
      }
    });
  }
  template <class F>
  QF_HD void s_ext(bool occupied, F fn) const {
#pragma unroll 1
    for (int k = ln; k < ext_count(occupied); k += nl) ext_call(occupied, k, fn);
  }

  QF_HD double c1(int p, int q) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q);
    s_ext(!oq, [&](auto t) { res += a.one(p, t) * b.one(t, q); });
    s_ext(!op, [&](auto t) { res -= b.one(p, t) * a.one(t, q); });
    if (!op && oq)
      s_pair1(true, false, [&](auto t, auto u) {
        res += a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
      });
    if (op && !oq)
      s_pair1(false, true, [&](auto t, auto u) {
        res -= a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
      });
    s_pair1(true, false, [&](auto t, auto u) {
      res -= b.one(t, u) * (2.0 * a.two(u, p, t, q) - a.two(u, p, q, t));
      res += b.one(u, t) * (2.0 * a.two(t, p, u, q) - a.two(t, p, q, u));
    });
    // (t,u occupied, w virtual) and (t,u virtual, w occupied), one external
    if (!oq || !op)
      s_triple1(true, true, false, [&](auto t, auto u, auto w) {
        if (!oq) res += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
        if (!op) res -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
      });
    if (oq || op)
      s_triple1(false, false, true, [&](auto t, auto u, auto w) {
        if (oq) res += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
        if (op) res -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
      });
    return res;
  }

  QF_HD double c0() const {
    double z = 0.0;
    s_pair1(true, false, [&](auto t, auto u) {
      z += 2.0 * (a.one(t, u) * b.one(u, t) - a.one(u, t) * b.one(t, u));
    });
    // (t,u occupied; w,x virtual) with exactly one external among the four
    auto term = [&](auto t, auto u, auto w, auto x) {
      z += a.two(t, u, w, x) * (2.0 * b.two(w, x, t, u) - b.two(w, x, u, t))
         - b.two(t, u, w, x) * (2.0 * a.two(w, x, t, u) - a.two(w, x, u, t));
    };
    const bool blk[4] = {true, true, false, false};
    s_flat<4>(blk, [&](int s, const int* id) {
      // position s holds the external's number, not an active position
      auto at = [&](int i) { return act_at(i < 2, id[i]); };
      if (s == 0) ext_call(true, id[0], [&](auto e) { term(e, at(1), at(2), at(3)); });
      else if (s == 1) ext_call(true, id[1], [&](auto e) { term(at(0), e, at(2), at(3)); });
      else if (s == 2) ext_call(false, id[2], [&](auto e) { term(at(0), at(1), e, at(3)); });
      else ext_call(false, id[3], [&](auto e) { term(at(0), at(1), at(2), e); });
    });
    return z;
  }
};

// Per-space tables for the marked evaluation of [E,sigma] (na local
// orbitals, local index = position in the space):
//   tau1[a][b], tau2[a][b][c][d]  sigma restricted to the space,
//   D1[j][t][a]   = sum_{x outside} f[x][t] sigma1 with x in slot j, a in the other,
//   D2[j][t][abc] = sum_{x outside} f[x][t] sigma2 with x in slot j, (a,b,c) in the
//                   other slots in order.
// With E's external leg x in slot k, E = sgn_k sum_t f[x][t] tau(t in slot k)
// (sgn = +1 for creator slots 0,1 and -1 for annihilator slots 2,3 of the
// two-body part; +1 / -1 for slots 0 / 1 of the one-body part), so every
// product E * sigma summed over x becomes sum_t sgn_k tau(..t..) D_j(t; ..).
struct MarkTables {
  const double* tau1;
  const double* tau2;
  const double* D1;
  const double* D2;
  int na;
};

QF_HD int mark_sizes(int na, int* tau1, int* tau2, int* d1, int* d2) {
  *tau1 = na * na;
  *tau2 = na * na * na * na;
  *d1 = 2 * na * na;
  *d2 = 2 * na * na * na * na;   // D_0 and D_1; D_2, D_3 follow by anti-Hermiticity
  return *tau1 + *tau2 + *d1 + *d2;
}

// Shape of a space of NA orbitals (NA/2 occupied) for the marked evaluation,
// known at compile time so that its loops and strides fold to constants.
template <int NA>
struct MarkedShape {
  static constexpr int na = NA, nocc = NA / 2;
  QF_HD static constexpr int nact(bool occ) { return occ ? nocc : na - nocc; }
};

template <int NA>
struct MarkedE {
  MarkTables T;
  static constexpr int na = NA;
  QF_HD double one(Mk p, int q) const { return T.tau1[p.t * na + q]; }
  QF_HD double one(int p, Mk q) const { return -T.tau1[p * na + q.t]; }
  QF_HD double t2(int a, int b, int c, int d) const {
    return T.tau2[((a * na + b) * na + c) * na + d];
  }
  QF_HD double two(Mk p, int q, int r, int s) const { return t2(p.t, q, r, s); }
  QF_HD double two(int p, Mk q, int r, int s) const { return t2(p, q.t, r, s); }
  QF_HD double two(int p, int q, Mk r, int s) const { return -t2(p, q, r.t, s); }
  QF_HD double two(int p, int q, int r, Mk s) const { return -t2(p, q, r, s.t); }
};

template <int NA>
struct MarkedSigma {
  MarkTables T;
  static constexpr int na = NA, n3 = NA * NA * NA;
  QF_HD double one(Mk p, int q) const { return T.D1[(0 * na + p.t) * na + q]; }
  QF_HD double one(int p, Mk q) const { return T.D1[(1 * na + q.t) * na + p]; }
  QF_HD double d(int j, int t, int a, int b, int c) const {
    return T.D2[(j * na + t) * n3 + (a * na + b) * na + c];
  }
  // D_2(t;a,b,c) = -D_0(t;c,a,b) and D_3(t;a,b,c) = -D_1(t;c,a,b)
  QF_HD double two(Mk p, int q, int r, int s) const { return d(0, p.t, q, r, s); }
  QF_HD double two(int p, Mk q, int r, int s) const { return d(1, q.t, p, r, s); }
  QF_HD double two(int p, int q, Mk r, int s) const { return -d(0, r.t, s, p, q); }
  QF_HD double two(int p, int q, int r, Mk s) const { return -d(1, s.t, r, p, q); }
};

template <class AOp, class BOp>
QF_HD Comm<AOp, BOp> make_comm(const AOp& a, const BOp& b, int n, int o) {
  return Comm<AOp, BOp>{a, b, n, o};
}

// Yg = [F_N, sigma]: only the one-body-A terms survive.
struct Yg {
  const double* f;
  Sigma s;
  int n, o;
  // lane split of the contraction loops (as in Comm); the caller sums lanes
  int ln = 0, nl = 1;
  QF_HD bool occ(int p) const { return p < o; }
  template <class F>
  QF_HD void over_block(bool occupied, F fn) const {
    if (occupied)
      for (int t = ln; t < o; t += nl) fn(t);
    else
      for (int t = o + ln; t < n; t += nl) fn(t);
  }
  // (t occupied, u virtual) pairs, split over lanes
  template <class F>
  QF_HD void over_ov(F fn) const {
    const int v = n - o;
    for (int k = ln; k < o * v; k += nl) fn(k / v, o + k % v);
  }
  QF_HD double two(int p, int q, int r, int s_) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q), or_ = occ(r), os = occ(s_);
    if (or_ == os && oq != or_)
      over_block(oq, [&](int t) { res += f[p * n + t] * s.two(t, q, r, s_); });
    if (or_ == os && op != or_)
      over_block(op, [&](int t) { res += f[q * n + t] * s.two(p, t, r, s_); });
    if (op == oq && os != op)
      over_block(os, [&](int t) { res -= f[t * n + r] * s.two(p, q, t, s_); });
    if (op == oq && or_ != op)
      over_block(or_, [&](int t) { res -= f[t * n + s_] * s.two(p, q, r, t); });
    return res;
  }
  QF_HD double one(int p, int q) const {
    double res = 0.0;
    over_block(!occ(q), [&](int t) { res += f[p * n + t] * s.one(t, q); });
    over_block(!occ(p), [&](int t) { res -= s.one(p, t) * f[t * n + q]; });
    if (!occ(p) && occ(q))
      over_ov([&](int t, int u) {
        res += f[t * n + u] * (2.0 * s.two(u, p, t, q) - s.two(u, p, q, t));
      });
    if (occ(p) && !occ(q))
      over_ov([&](int u, int t) {
        res -= f[t * n + u] * (2.0 * s.two(u, p, t, q) - s.two(u, p, q, t));
      });
    return res;
  }
  QF_HD double zero() const {
    double z = 0.0;
    over_ov([&](int t, int u) {
      z += 2.0 * (f[t * n + u] * s.one(u, t) - f[u * n + t] * s.one(t, u));
    });
    return z;
  }
};

}  // namespace qf
