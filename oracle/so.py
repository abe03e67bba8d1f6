"""Spin-orbital normal-ordered operators and the truncated commutator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An operator is X = x0 + sum_pq x1[p,q] {p+ q} + 1/4 sum_pqrs x2[p,q,r,s] {p+ q+ s r}
with x2 antisymmetric in (p,q) and in (r,s); braces denote normal order with
respect to the closed-shell reference Phi (occupied spin orbitals are holes).

Operators are evaluated lazily on index blocks: every index set passed to
``one``/``two`` lies entirely in the occupied block ('o') or entirely in the
virtual block ('v'), so an operator can report structurally zero blocks and the
commutator skips them.  Skipping a block whose elements are all zero changes no
result.

``comm0/comm1/comm2`` give the 0-, 1- and 2-body parts of the exact commutator
[A,B] of two operators of rank <= 2; the 3-body part is dropped.  This is the
normal-ordered two-body truncation used in the in-medium similarity
renormalisation group (Hergert et al., Phys. Rep. 621, 165 (2016), the
single-reference commutator expressions), re-derived here from Wick's theorem:

  [A,B]_0 = sum_tu (n_t-n_u) A_tu B_ut
            + 1/4 sum_tuwx n_t n_u nb_w nb_x (A_tuwx B_wxtu - B_tuwx A_wxtu)
  [A,B]_pq = sum_t (A_pt B_tq - B_pt A_tq)
            + sum_tu (n_t-n_u) (A_tu B_uptq - B_tu A_uptq)
            + 1/2 sum_tuw (n_t n_u nb_w + nb_t nb_u n_w)(A_wptu B_tuwq - B_wptu A_tuwq)
  [A,B]_pqrs = (1-P_pq) sum_t (A_pt B_tqrs - B_pt A_tqrs)
            - (1-P_rs) sum_t (A_tr B_pqts - B_tr A_pqts)
            + 1/2 sum_tu (1-n_t-n_u)(A_pqtu B_turs - B_pqtu A_turs)
            + (1-P_pq)(1-P_rs) X_pqrs,
    X_pqrs = - sum_tu nb_t n_u (A_putr B_tqus - B_putr A_tqus)

with n = 1 on holes, nb = 1 - n, and P_pq exchanging p and q.  These are pinned
against exact Fock-space commutators in the test suite.
"""
from __future__ import annotations

import numpy as np


class Blocks:
    """Spin-orbital index blocks of a problem with n spatial, o occupied."""

    def __init__(self, n: int, o: int):
        self.n, self.o = n, o
        self.N = 2 * n
        self.O = np.arange(0, 2 * o)            # occupied spin orbitals
        self.V = np.arange(2 * o, 2 * n)        # virtual spin orbitals

    def full(self, lab):
        return self.O if lab == "o" else self.V

    def split(self, idx):
        """Split an index array into ('o', occ part) and ('v', vir part)."""
        idx = np.asarray(idx, dtype=np.int64)
        out = []
        occ = idx[idx < 2 * self.o]
        vir = idx[idx >= 2 * self.o]
        if len(occ):
            out.append(("o", occ))
        if len(vir):
            out.append(("v", vir))
        return out


def _es(spec, *ops):
    """np.einsum with a BLAS-backed contraction order."""
    return np.einsum(spec, *ops, optimize=True)


def spin_delta(I, J):
    return (np.asarray(I)[:, None] % 2 == np.asarray(J)[None, :] % 2).astype(float)


class Op:
    """Base lazy operator.  Index arguments are (label, array) pairs."""

    def zero(self) -> float:
        return 0.0

    def one(self, I, J) -> np.ndarray:
        return np.zeros((len(I[1]), len(J[1])))

    def two(self, I, J, K, L) -> np.ndarray:
        return np.zeros((len(I[1]), len(J[1]), len(K[1]), len(L[1])))

    def nz1(self, a, b) -> bool:
        return True

    def nz2(self, a, b, c, d) -> bool:
        return True


class Hamiltonian(Op):
    """H_N: Fock matrix f and antisymmetrised <pq||rs> from chemist (pq|rs)."""

    def __init__(self, f: np.ndarray, eri: np.ndarray, e0: float = 0.0):
        self.f, self.eri, self.e0 = f, eri, e0

    def zero(self):
        return self.e0

    def one(self, I, J):
        i, j = I[1], J[1]
        return self.f[np.ix_(i // 2, j // 2)] * spin_delta(i, j)

    def two(self, I, J, K, L):
        p, q, r, s = I[1], J[1], K[1], L[1]
        P, Q, R, S = p // 2, q // 2, r // 2, s // 2
        # <pq|rs> = (PR|QS) d(sp,sr) d(sq,ss)
        direct = self.eri[np.ix_(P, R, Q, S)].transpose(0, 2, 1, 3)
        direct = direct * spin_delta(p, r)[:, None, :, None] * spin_delta(q, s)[None, :, None, :]
        exch = self.eri[np.ix_(P, S, Q, R)].transpose(0, 2, 3, 1)
        exch = exch * spin_delta(p, s)[:, None, None, :] * spin_delta(q, r)[None, :, :, None]
        return direct - exch


class Fock(Op):
    """One-body operator F_N = sum f_pq {p+ q}."""

    def __init__(self, f: np.ndarray):
        self.f = f

    def one(self, I, J):
        i, j = I[1], J[1]
        return self.f[np.ix_(i // 2, j // 2)] * spin_delta(i, j)

    def nz2(self, a, b, c, d):
        return False


class Cluster(Op):
    """sigma = T - T^dagger built from spin-adapted spatial amplitudes.

    T1 = sum t1[i,a] E_ai and T2 = 1/2 sum t2[i,j,a,b] E_ai E_bj, i.e. in spin
    orbitals t_{i s, a s} = t1[i,a], and
      t_{i s j s', a s b s'} = t2[i,j,a,b] d(..) - t2[j,i,a,b] d(..)
    which gives t2 for opposite spins and t2[i,j,a,b] - t2[i,j,b,a] for equal
    spins.  ``mask`` (a set of spatial orbitals) removes every amplitude whose
    indices all lie in the mask: that turns sigma into sigma_ext of Eq. (3).
    """

    def __init__(self, blocks: Blocks, t1, t2, mask=None):
        self.b = blocks
        self.t1, self.t2 = t1, t2
        self.o = blocks.o
        self.mask = None
        if mask is not None:
            m = np.zeros(blocks.n, dtype=bool)
            m[list(mask)] = True
            self.mask = m

    def nz1(self, a, b):
        return a != b

    def nz2(self, a, b, c, d):
        return (a == b == "v" and c == d == "o") or (a == b == "o" and c == d == "v")

    def _full(self):
        """Dense spin-orbital t1[2o,2v] and antisymmetric t2[2o,2o,2v,2v]
        (built once; slices are cut from them)."""
        if getattr(self, "_so", None) is None:
            o, v = self.o, self.t1.shape[1]
            i = np.arange(2 * o)
            a = np.arange(2 * o, 2 * (o + v))
            I, A = i // 2, a // 2 - o
            t1 = self.t1[np.ix_(I, A)] * spin_delta(i, a)
            d = self.t2[np.ix_(I, I, A, A)]
            d = d * spin_delta(i, a)[:, None, :, None] * spin_delta(i, a)[None, :, None, :]
            e = self.t2[np.ix_(I, I, A, A)].transpose(1, 0, 2, 3)
            e = e * spin_delta(i, a)[None, :, :, None] * spin_delta(i, a)[:, None, None, :]
            self._so = (t1, d - e)
        return self._so

    def _t1(self, i, a):
        """spin-orbital t_{i,a}: i occupied, a virtual (arrays)."""
        o2 = 2 * self.o
        x = self._full()[0][np.ix_(i, a - o2)]
        if self.mask is not None:
            mi, ma = np.nonzero(self.mask[i // 2])[0], np.nonzero(self.mask[a // 2])[0]
            x[np.ix_(mi, ma)] = 0.0
        return x

    def _t2_masked(self):
        """The dense antisymmetric spin-orbital t2 with the mask applied
        (every amplitude whose four spatial indices lie in the space set to
        zero), built once and kept read-only so that no caller can alter it."""
        if getattr(self, "_t2m", None) is None:
            x = self._full()[1].copy()
            if self.mask is not None:
                o2 = 2 * self.o
                occ = np.nonzero(self.mask[np.arange(o2) // 2])[0]
                vir = np.nonzero(self.mask[(np.arange(x.shape[2]) + o2) // 2])[0]
                x[np.ix_(occ, occ, vir, vir)] = 0.0
            x.flags.writeable = False
            self._t2m = x
        return self._t2m

    def _t2(self, i, j, a, b):
        """spin-orbital t_{ij}^{ab} (antisymmetric), shape [i,j,a,b]:
        t2[i,j,a,b] for opposite spins, t2[i,j,a,b] - t2[i,j,b,a] for equal;
        amplitudes with every index in the mask are zero.  A request for the
        whole occupied and virtual ranges returns the stored (read-only)
        array itself."""
        o2 = 2 * self.o
        x = self._t2_masked()
        if (len(i) == len(j) == o2 and len(a) == len(b) == x.shape[2]
                and np.array_equal(i, np.arange(o2)) and np.array_equal(j, np.arange(o2))
                and np.array_equal(a, np.arange(o2, o2 + x.shape[2]))
                and np.array_equal(b, np.arange(o2, o2 + x.shape[2]))):
            return x
        return x[np.ix_(i, j, a - o2, b - o2)]

    def one(self, I, J):
        if I[0] == "v" and J[0] == "o":
            return self._t1(J[1], I[1]).T
        if I[0] == "o" and J[0] == "v":
            return -self._t1(I[1], J[1])
        return np.zeros((len(I[1]), len(J[1])))

    def two(self, I, J, K, L):
        if I[0] == J[0] == "v" and K[0] == L[0] == "o":
            # sigma_{ab ij} = t_{ij}^{ab}
            return self._t2(K[1], L[1], I[1], J[1]).transpose(2, 3, 0, 1)
        if I[0] == J[0] == "o" and K[0] == L[0] == "v":
            # sigma_{ij ab} = -t_{ij}^{ab}
            return -self._t2(I[1], J[1], K[1], L[1])
        return np.zeros((len(I[1]), len(J[1]), len(K[1]), len(L[1])))


def _occ(lab):
    return 1.0 if lab == "o" else 0.0


def comm0(A: Op, B: Op, bl: Blocks) -> float:
    O, V = ("o", bl.O), ("v", bl.V)
    z = 0.0
    # sum_tu (n_t - n_u) A_tu B_ut : only (t,u) in (o,v) or (v,o) survive
    for (T, U, w) in ((O, V, 1.0), (V, O, -1.0)):
        if A.nz1(T[0], U[0]) and B.nz1(U[0], T[0]):
            z += w * _es("tu,ut->", A.one(T, U), B.one(U, T))
    # 1/4 sum n_t n_u nb_w nb_x (A_tuwx B_wxtu - B_tuwx A_wxtu)
    if A.nz2("o", "o", "v", "v") and B.nz2("v", "v", "o", "o"):
        z += 0.25 * _es("tuwx,wxtu->", A.two(O, O, V, V), B.two(V, V, O, O))
    if B.nz2("o", "o", "v", "v") and A.nz2("v", "v", "o", "o"):
        z -= 0.25 * _es("tuwx,wxtu->", B.two(O, O, V, V), A.two(V, V, O, O))
    return float(z)


def _comm1_ordered(A: Op, B: Op, P, Q, bl: Blocks) -> np.ndarray:
    """The A-first half of [A,B]_1 on blocks P,Q (the full result is this
    minus the same with A and B exchanged)."""
    O, V = ("o", bl.O), ("v", bl.V)
    out = np.zeros((len(P[1]), len(Q[1])))
    for T in (O, V):
        if A.nz1(P[0], T[0]) and B.nz1(T[0], Q[0]):
            out += A.one(P, T) @ B.one(T, Q)
    for (T, U, w) in ((O, V, 1.0), (V, O, -1.0)):
        if A.nz1(T[0], U[0]) and B.nz2(U[0], P[0], T[0], Q[0]):
            out += w * _es("tu,uptq->pq", A.one(T, U), B.two(U, P, T, Q))
    # (t,u occupied, w virtual) and (t,u virtual, w occupied)
    for (T, W) in ((O, V), (V, O)):
        if A.nz2(W[0], P[0], T[0], T[0]) and B.nz2(T[0], T[0], W[0], Q[0]):
            out += 0.5 * _es("wptu,tuwq->pq", A.two(W, P, T, T), B.two(T, T, W, Q))
    return out


def comm1(A: Op, B: Op, P, Q, bl: Blocks) -> np.ndarray:
    return _comm1_ordered(A, B, P, Q, bl) - _comm1_ordered(B, A, P, Q, bl)


def _z(P, Q, R, S):
    return np.zeros((len(P[1]), len(Q[1]), len(R[1]), len(S[1])))


def _g1(A, B, P, Q, R, S, bl):
    """sum_t (A_pt B_tqrs - B_pt A_tqrs)."""
    out = _z(P, Q, R, S)
    for T in (("o", bl.O), ("v", bl.V)):
        if A.nz1(P[0], T[0]) and B.nz2(T[0], Q[0], R[0], S[0]):
            out += _es("pt,tqrs->pqrs", A.one(P, T), B.two(T, Q, R, S))
        if B.nz1(P[0], T[0]) and A.nz2(T[0], Q[0], R[0], S[0]):
            out -= _es("pt,tqrs->pqrs", B.one(P, T), A.two(T, Q, R, S))
    return out


def _g2(A, B, P, Q, R, S, bl):
    """sum_t (A_tr B_pqts - B_tr A_pqts)."""
    out = _z(P, Q, R, S)
    for T in (("o", bl.O), ("v", bl.V)):
        if A.nz1(T[0], R[0]) and B.nz2(P[0], Q[0], T[0], S[0]):
            out += _es("tr,pqts->pqrs", A.one(T, R), B.two(P, Q, T, S))
        if B.nz1(T[0], R[0]) and A.nz2(P[0], Q[0], T[0], S[0]):
            out -= _es("tr,pqts->pqrs", B.one(T, R), A.two(P, Q, T, S))
    return out


def _ph(A, B, P, Q, R, S, bl):
    """X_pqrs = - sum_{t virtual, u occupied} (A_putr B_tqus - B_putr A_tqus)."""
    O, V = ("o", bl.O), ("v", bl.V)
    out = _z(P, Q, R, S)
    if A.nz2(P[0], "o", "v", R[0]) and B.nz2("v", Q[0], "o", S[0]):
        out -= _es("putr,tqus->pqrs", A.two(P, O, V, R), B.two(V, Q, O, S))
    if B.nz2(P[0], "o", "v", R[0]) and A.nz2("v", Q[0], "o", S[0]):
        out += _es("putr,tqus->pqrs", B.two(P, O, V, R), A.two(V, Q, O, S))
    return out


def comm2(A: Op, B: Op, P, Q, R, S, bl: Blocks) -> np.ndarray:
    """Two-body part of [A,B] on pure index blocks P,Q,R,S."""
    O, V = ("o", bl.O), ("v", bl.V)
    # (1-P_pq) sum_t (A_pt B_tqrs - B_pt A_tqrs)
    out = _g1(A, B, P, Q, R, S, bl) - _g1(A, B, Q, P, R, S, bl).transpose(1, 0, 2, 3)
    # -(1-P_rs) sum_t (A_tr B_pqts - B_tr A_pqts)
    out -= _g2(A, B, P, Q, R, S, bl) - _g2(A, B, P, Q, S, R, bl).transpose(0, 1, 3, 2)
    # 1/2 sum_tu (1 - n_t - n_u)(...): only t,u in the same block survive
    for (T, w) in ((V, 0.5), (O, -0.5)):
        if A.nz2(P[0], Q[0], T[0], T[0]) and B.nz2(T[0], T[0], R[0], S[0]):
            out += w * _es("pqtu,turs->pqrs", A.two(P, Q, T, T), B.two(T, T, R, S))
        if B.nz2(P[0], Q[0], T[0], T[0]) and A.nz2(T[0], T[0], R[0], S[0]):
            out -= w * _es("pqtu,turs->pqrs", B.two(P, Q, T, T), A.two(T, T, R, S))
    # (1-P_pq)(1-P_rs) X_pqrs
    out += (_ph(A, B, P, Q, R, S, bl)
            - _ph(A, B, Q, P, R, S, bl).transpose(1, 0, 2, 3)
            - _ph(A, B, P, Q, S, R, bl).transpose(0, 1, 3, 2)
            + _ph(A, B, Q, P, S, R, bl).transpose(1, 0, 3, 2))
    return out


class Commutator(Op):
    """Lazy [A,B] truncated to rank 2; blocks are evaluated on request."""

    def __init__(self, A: Op, B: Op, bl: Blocks):
        self.A, self.B, self.bl = A, B, bl
        self._z = None

    def zero(self):
        if self._z is None:
            self._z = comm0(self.A, self.B, self.bl)
        return self._z

    def one(self, I, J):
        return comm1(self.A, self.B, I, J, self.bl)

    def two(self, I, J, K, L):
        return comm2(self.A, self.B, I, J, K, L, self.bl)


class Dense(Op):
    """Operator held as full dense spin-orbital arrays (small systems)."""

    def __init__(self, x0, x1, x2):
        self.x0, self.x1, self.x2 = x0, x1, x2

    def zero(self):
        return self.x0

    def one(self, I, J):
        return self.x1[np.ix_(I[1], J[1])]

    def two(self, I, J, K, L):
        return self.x2[np.ix_(I[1], J[1], K[1], L[1])]


def to_dense(A: Op, bl: Blocks):
    """Evaluate (x0, x1[N,N], x2[N,N,N,N]) of A over all blocks."""
    N = bl.N
    x1 = np.zeros((N, N))
    x2 = np.zeros((N, N, N, N))
    B = [("o", bl.O), ("v", bl.V)]
    for P in B:
        for Q in B:
            x1[np.ix_(P[1], Q[1])] = A.one(P, Q)
            for R in B:
                for S in B:
                    x2[np.ix_(P[1], Q[1], R[1], S[1])] = A.two(P, Q, R, S)
    return A.zero(), x1, x2


def restrict(A: Op, idx, bl: Blocks):
    """(x0, x1, x2) of A restricted to the spin orbitals idx (any mix of
    blocks); the arrays are indexed in the order of idx."""
    idx = np.asarray(idx, dtype=np.int64)
    pos = {int(k): m for m, k in enumerate(idx)}
    parts = bl.split(idx)
    n = len(idx)
    x1 = np.zeros((n, n))
    x2 = np.zeros((n, n, n, n))

    def loc(P):
        return np.array([pos[int(k)] for k in P[1]])

    for P in parts:
        for Q in parts:
            x1[np.ix_(loc(P), loc(Q))] = A.one(P, Q)
            for R in parts:
                for S in parts:
                    x2[np.ix_(loc(P), loc(Q), loc(R), loc(S))] = A.two(P, Q, R, S)
    return A.zero(), x1, x2
