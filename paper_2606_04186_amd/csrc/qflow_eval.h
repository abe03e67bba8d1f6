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
  QF_HD bool act(int p) const { return pos[p] >= 0; }
};

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

// Dense operator with a ladder intermediate L[(pq)][(ij)] (H_N, or Yg).
struct DenseOp {
  static constexpr bool kHasL = true;
  static constexpr bool kSparse3 = false;
  const double* x1;   // [n][n]
  const double* x2;   // [n][n][n][n]
  const double* L;    // [n*n][o*o]
  int n, o;
  QF_HD double one(int p, int q) const { return x1[p * n + q]; }
  QF_HD double two(int p, int q, int r, int s) const {
    return x2[(((size_t)p * n + q) * n + r) * n + s];
  }
  QF_HD double lad(int p, int q, int i, int j) const {
    return L[((size_t)p * n + q) * o * o + i * o + j];
  }
  QF_HD bool act(int) const { return true; }
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

  QF_HD bool occ(int p) const { return p < o; }
  static constexpr bool kUseL = AOp::kHasL && BOp::kFull;
  static constexpr bool kRestrict = AOp::kSparse3 && BOp::kFull;

  // loops over the block of index p (occupied or virtual), contracted with B
  template <class F>
  QF_HD void over_block(bool occupied, F fn) const {
    if (occupied)
      for (int k = 0; k < b.nocc(); ++k) fn(b.occ(k));
    else
      for (int k = 0; k < b.nvir(); ++k) fn(b.vir(k));
  }

  // sum_{t,u virtual} A[p,q,t,u] B[t,u,r,s]  (r,s occupied)
  QF_HD double ladder_vv(int p, int q, int r, int s) const {
    if constexpr (kUseL) {
      return a.lad(p, q, r, s);
    } else {
      double x = 0.0;
      if constexpr (kRestrict) {
        // A needs >= 3 active indices among (p,q,t,u)
        int npq = (int)a.act(p) + (int)a.act(q);
        if (npq == 0) return 0.0;
        for (int k = 0; k < b.nvir(); ++k) {
          int t = b.vir(k);
          bool at = a.act(t);
          if (npq + (int)at < 2) continue;
          if (npq + (int)at >= 3) {
            for (int m = 0; m < b.nvir(); ++m) {
              int u = b.vir(m);
              x += a.two(p, q, t, u) * b.two(t, u, r, s);
            }
          } else {
            for (int m = 0; m < b.nvir(); ++m) {
              int u = b.vir(m);
              if (a.act(u)) x += a.two(p, q, t, u) * b.two(t, u, r, s);
            }
          }
        }
      } else {
        for (int k = 0; k < b.nvir(); ++k)
          for (int m = 0; m < b.nvir(); ++m) {
            int t = b.vir(k), u = b.vir(m);
            x += a.two(p, q, t, u) * b.two(t, u, r, s);
          }
      }
      return x;
    }
  }

  // sum_{t,u virtual} B[p,q,t,u] A[t,u,r,s]  (p,q occupied)
  QF_HD double ladder_vv_rev(int p, int q, int r, int s) const {
    if constexpr (kUseL) {
      // B[p,q,c,d] = -t2[p,q,c,d]; A[c,d,r,s] = A[r,s,c,d] (Hermitian)
      return -a.lad(r, s, p, q);
    } else {
      double x = 0.0;
      if constexpr (kRestrict) {
        int nrs = (int)a.act(r) + (int)a.act(s);
        if (nrs == 0) return 0.0;
        for (int k = 0; k < b.nvir(); ++k) {
          int t = b.vir(k);
          bool at = a.act(t);
          if (nrs + (int)at < 2) continue;
          for (int m = 0; m < b.nvir(); ++m) {
            int u = b.vir(m);
            if (nrs + (int)at >= 3 || a.act(u)) x += b.two(p, q, t, u) * a.two(t, u, r, s);
          }
        }
      } else {
        for (int k = 0; k < b.nvir(); ++k)
          for (int m = 0; m < b.nvir(); ++m) {
            int t = b.vir(k), u = b.vir(m);
            x += b.two(p, q, t, u) * a.two(t, u, r, s);
          }
      }
      return x;
    }
  }

  // ----- two-body element [A,B][p,q,r,s] -----
  QF_HD double c2(int p, int q, int r, int s) const {
    double res = 0.0;
    const bool op = occ(p), oq = occ(q), or_ = occ(r), os = occ(s);
    // one-body A x two-body B:
    //   sum_t [A_pt B_tqrs + A_qt B_ptrs - A_tr B_pqts - A_ts B_pqrt]
    if (or_ == os && oq != or_)
      over_block(oq, [&](int t) { res += a.one(p, t) * b.two(t, q, r, s); });
    if (or_ == os && op != or_)
      over_block(op, [&](int t) { res += a.one(q, t) * b.two(p, t, r, s); });
    if (op == oq && os != op)
      over_block(os, [&](int t) { res -= a.one(t, r) * b.two(p, q, t, s); });
    if (op == oq && or_ != op)
      over_block(or_, [&](int t) { res -= a.one(t, s) * b.two(p, q, r, t); });
    // one-body B x two-body A:
    //   - sum_t [B_pt A_tqrs + B_qt A_ptrs - B_tr A_pqts - B_ts A_pqrt]
    over_block(!op, [&](int t) { res -= b.one(p, t) * a.two(t, q, r, s); });
    over_block(!oq, [&](int t) { res -= b.one(q, t) * a.two(p, t, r, s); });
    over_block(!or_, [&](int t) { res += b.one(t, r) * a.two(p, q, t, s); });
    over_block(!os, [&](int t) { res += b.one(t, s) * a.two(p, q, r, t); });
    // ladders: sum_tu (1 - n_t - n_u)(A_pqtu B_turs - B_pqtu A_turs)
    if (or_ && os) res += ladder_vv(p, q, r, s);
    if (!or_ && !os) {
      double x = 0.0;
      for (int k = 0; k < b.nocc(); ++k)
        for (int m = 0; m < b.nocc(); ++m) {
          int t = b.occ(k), u = b.occ(m);
          x += a.two(p, q, t, u) * b.two(t, u, r, s);
        }
      res -= x;
    }
    if (!op && !oq) {
      double x = 0.0;
      for (int k = 0; k < b.nocc(); ++k)
        for (int m = 0; m < b.nocc(); ++m) {
          int t = b.occ(k), u = b.occ(m);
          x += b.two(p, q, t, u) * a.two(t, u, r, s);
        }
      res += x;
    }
    if (op && oq) res -= ladder_vv_rev(p, q, r, s);
    // particle-hole terms: Xa(p,q,r,s) - Xb - Xc + Xa(q,p,s,r)
    res += xa(p, q, r, s) - xb(p, q, r, s) - xc(p, q, r, s) + xa(q, p, s, r);
    return res;
  }

  // sum over t virtual, u occupied, both contracted with B
  template <class F>
  QF_HD void over_vo(F fn) const {
    for (int k = 0; k < b.nvir(); ++k) {
      int t = b.vir(k);
      for (int m = 0; m < b.nocc(); ++m) fn(t, b.occ(m));
    }
  }

  // Xa = sum_{t v, u o} [ -A_putr B_tqus + 2 A_purt B_tqus - A_purt B_tqsu
  //                       + B_putr A_tqus - 2 B_purt A_tqus + B_purt A_tqsu ]
  QF_HD double xa(int p, int q, int r, int s) const {
    double x = 0.0;
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
    if (!occ(p) && occ(s))
      over_vo([&](int t, int u) { x += a.two(q, u, t, r) * b.two(t, p, s, u); });
    if (occ(q) && !occ(r))
      over_vo([&](int t, int u) { x -= b.two(q, u, t, r) * a.two(t, p, s, u); });
    return x;
  }
  // Xc = sum_{t v, u o} [A_puts B_tqru - B_puts A_tqru]
  QF_HD double xc(int p, int q, int r, int s) const {
    double x = 0.0;
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
      for (int k = 0; k < b.nocc(); ++k)
        for (int m = 0; m < b.nvir(); ++m) {
          int t = b.occ(k), u = b.vir(m);
          res += a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
        }
    if (op && !oq)   // t virtual, u occupied (sign -1)
      for (int k = 0; k < b.nvir(); ++k)
        for (int m = 0; m < b.nocc(); ++m) {
          int t = b.vir(k), u = b.occ(m);
          res -= a.one(t, u) * (2.0 * b.two(u, p, t, q) - b.two(u, p, q, t));
        }
    for (int k = 0; k < b.nocc(); ++k)
      for (int m = 0; m < b.nvir(); ++m) {
        int t = b.occ(k), u = b.vir(m);
        res -= b.one(t, u) * (2.0 * a.two(u, p, t, q) - a.two(u, p, q, t));
        res += b.one(u, t) * (2.0 * a.two(t, p, u, q) - a.two(t, p, q, u));
      }
    // sum_tuw (n_t n_u nb_w + nb_t nb_u n_w)
    //      [A_wptu (2 B_tuwq - B_tuqw) - B_wptu (2 A_tuwq - A_tuqw)]
    // (t,u occupied, w virtual): B_tuwq needs q virtual, B_wptu needs p virtual
    if (!oq || !op) {
      double x = 0.0;
      for (int k = 0; k < b.nocc(); ++k)
        for (int l = 0; l < b.nocc(); ++l) {
          int t = b.occ(k), u = b.occ(l);
          if constexpr (kRestrict) {
            int c = (int)a.act(t) + (int)a.act(u) + (int)a.act(p) + (int)a.act(q);
            if (c < 1) continue;
          }
          for (int m = 0; m < b.nvir(); ++m) {
            int w = b.vir(m);
            if (!oq) x += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
            if (!op) x -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
          }
        }
      res += x;
    }
    // (t,u virtual, w occupied): B_tuwq needs q occupied, B_wptu needs p occupied
    if (oq) res += c1_vvo(p, q);
    if (op) res += c1_vvo_rev(p, q);
    return res;
  }

  // sum_{w o; t,u v} A_wptu (2 B_tuwq - B_tuqw), q occupied
  QF_HD double c1_vvo(int p, int q) const {
    if constexpr (kUseL) {
      double x = 0.0;
      for (int w = 0; w < o; ++w) x += 2.0 * a.lad(w, p, w, q) - a.lad(w, p, q, w);
      return x;
    } else {
      double x = 0.0;
      for (int m = 0; m < b.nocc(); ++m) {
        int w = b.occ(m);
        for (int k = 0; k < b.nvir(); ++k) {
          int t = b.vir(k);
          if constexpr (kRestrict) {
            // A[w,p,t,u] needs at least three active indices
            int c3 = (int)a.act(w) + (int)a.act(p) + (int)a.act(t);
            if (c3 < 2) continue;
            if (c3 == 2) {
              for (int l = 0; l < b.nvir(); ++l) {
                int u = b.vir(l);
                if (a.act(u))
                  x += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
              }
              continue;
            }
          }
          for (int l = 0; l < b.nvir(); ++l) {
            int u = b.vir(l);
            x += a.two(w, p, t, u) * (2.0 * b.two(t, u, w, q) - b.two(t, u, q, w));
          }
        }
      }
      return x;
    }
  }

  // - sum_{w o; t,u v} B_wptu (2 A_tuwq - A_tuqw), p occupied
  QF_HD double c1_vvo_rev(int p, int q) const {
    if constexpr (kUseL) {
      // B_wptu = -t2[w,p,t,u]; A_tuwq = A_wqtu (Hermitian)
      double x = 0.0;
      for (int w = 0; w < o; ++w) x += 2.0 * a.lad(w, q, w, p) - a.lad(q, w, w, p);
      return x;
    } else {
      double x = 0.0;
      for (int m = 0; m < b.nocc(); ++m) {
        int w = b.occ(m);
        for (int k = 0; k < b.nvir(); ++k) {
          int t = b.vir(k);
          if constexpr (kRestrict) {
            // A[t,u,w,q] needs at least three active indices
            int c3 = (int)a.act(w) + (int)a.act(q) + (int)a.act(t);
            if (c3 < 2) continue;
            if (c3 == 2) {
              for (int l = 0; l < b.nvir(); ++l) {
                int u = b.vir(l);
                if (a.act(u))
                  x -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
              }
              continue;
            }
          }
          for (int l = 0; l < b.nvir(); ++l) {
            int u = b.vir(l);
            x -= b.two(w, p, t, u) * (2.0 * a.two(t, u, w, q) - a.two(t, u, q, w));
          }
        }
      }
      return x;
    }
  }

  // ----- zero-body part -----
  QF_HD double c0() const {
    double z = 0.0;
    // 2 sum_tu (n_t - n_u) A_tu B_ut
    for (int k = 0; k < b.nocc(); ++k)
      for (int m = 0; m < b.nvir(); ++m) {
        int t = b.occ(k), u = b.vir(m);
        z += 2.0 * (a.one(t, u) * b.one(u, t) - a.one(u, t) * b.one(t, u));
      }
    // sum_{tu o, wx v} [A_tuwx (2 B_wxtu - B_wxut) - B_tuwx (2 A_wxtu - A_wxut)]
    if constexpr (kUseL) {
      for (int t = 0; t < o; ++t)
        for (int u = 0; u < o; ++u)
          z += 4.0 * a.lad(t, u, t, u) - a.lad(t, u, u, t) - a.lad(u, t, t, u);
    } else {
      for (int k = 0; k < b.nocc(); ++k)
        for (int l = 0; l < b.nocc(); ++l)
          for (int m = 0; m < b.nvir(); ++m) {
            int t = b.occ(k), u = b.occ(l), w = b.vir(m);
            if constexpr (kRestrict) {
              int c = (int)a.act(t) + (int)a.act(u) + (int)a.act(w);
              if (c < 2) continue;
              if (c == 2) {
                for (int r = 0; r < b.nvir(); ++r) {
                  int x = b.vir(r);
                  if (!a.act(x)) continue;
                  z += a.two(t, u, w, x) * (2.0 * b.two(w, x, t, u) - b.two(w, x, u, t))
                     - b.two(t, u, w, x) * (2.0 * a.two(w, x, t, u) - a.two(w, x, u, t));
                }
                continue;
              }
            }
            for (int r = 0; r < b.nvir(); ++r) {
              int x = b.vir(r);
              z += a.two(t, u, w, x) * (2.0 * b.two(w, x, t, u) - b.two(w, x, u, t))
                 - b.two(t, u, w, x) * (2.0 * a.two(w, x, t, u) - a.two(w, x, u, t));
            }
          }
    }
    return z;
  }
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
  QF_HD bool occ(int p) const { return p < o; }
  template <class F>
  QF_HD void over_block(bool occupied, F fn) const {
    if (occupied)
      for (int t = 0; t < o; ++t) fn(t);
    else
      for (int t = o; t < n; ++t) fn(t);
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
      for (int t = 0; t < o; ++t)
        for (int u = o; u < n; ++u)
          res += f[t * n + u] * (2.0 * s.two(u, p, t, q) - s.two(u, p, q, t));
    if (occ(p) && !occ(q))
      for (int t = o; t < n; ++t)
        for (int u = 0; u < o; ++u)
          res -= f[t * n + u] * (2.0 * s.two(u, p, t, q) - s.two(u, p, q, t));
    return res;
  }
  QF_HD double zero() const {
    double z = 0.0;
    for (int t = 0; t < o; ++t)
      for (int u = o; u < n; ++u)
        z += 2.0 * (f[t * n + u] * s.one(u, t) - f[u * n + t] * s.one(t, u));
    return z;
  }
};

}  // namespace qf
