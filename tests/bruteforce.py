"""Brute-force second quantisation on tiny Fock spaces (tests only).

Every operator here is an explicit sparse matrix on the full Fock space of N
spin orbitals (dimension 2^N), built from Jordan-Wigner annihilators.  Nothing
is truncated or factorised, so these matrices are the exact definitions against
which the oracle's normal-ordered algebra is pinned.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


class FockSpace:
    def __init__(self, N: int):
        self.N = N
        self.dim = 1 << N
        states = np.arange(self.dim)
        self.nel = np.array([bin(s).count("1") for s in states])
        self.ann = []
        for p in range(N):
            rows, cols, vals = [], [], []
            for s in states:
                if (s >> p) & 1:
                    below = bin(s & ((1 << p) - 1)).count("1")
                    rows.append(s ^ (1 << p))
                    cols.append(s)
                    vals.append(-1.0 if below % 2 else 1.0)
            self.ann.append(sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim)))
        self.cre = [a.T.tocsr() for a in self.ann]
        self.I = sp.identity(self.dim, format="csr")

    def ref_state(self, n_occ_so: int) -> int:
        return (1 << n_occ_so) - 1

    def qp_count(self, n_occ_so: int) -> np.ndarray:
        ref = self.ref_state(n_occ_so)
        return np.array([bin(s ^ ref).count("1") for s in range(self.dim)])

    def normal_ordered(self, ops, n_occ_so: int):
        """Matrix of {o_1 ... o_k}; ops = [(p, dagger)], normal order taken
        with respect to the determinant occupying spin orbitals < n_occ_so."""
        def is_qp_creator(p, dag):
            hole = p < n_occ_so
            return dag != hole      # particle creator or hole annihilator
        order = sorted(range(len(ops)), key=lambda k: (0 if is_qp_creator(*ops[k]) else 1, k))
        # sign of the permutation `order`
        perm = list(order)
        sign = 1
        for i in range(len(perm)):
            while perm[i] != i:
                j = perm[i]
                perm[i], perm[j] = perm[j], perm[i]
                sign = -sign
        M = self.I
        for k in order:
            p, dag = ops[k]
            M = M @ (self.cre[p] if dag else self.ann[p])
        return sign * M

    def operator(self, x0, x1, x2, n_occ_so: int, tol=0.0):
        """x0 + sum x1[p,q] {p+ q} + 1/4 sum x2[p,q,r,s] {p+ q+ s r}."""
        N = self.N
        M = x0 * self.I
        for p, q in itertools.product(range(N), repeat=2):
            if abs(x1[p, q]) > tol:
                M = M + x1[p, q] * self.normal_ordered([(p, 1), (q, 0)], n_occ_so)
        for p, q, r, s in itertools.product(range(N), repeat=4):
            if abs(x2[p, q, r, s]) > tol:
                M = M + 0.25 * x2[p, q, r, s] * self.normal_ordered(
                    [(p, 1), (q, 1), (s, 0), (r, 0)], n_occ_so)
        return M.tocsr()

    def E(self, P, Q):
        """Spin-summed E_PQ for spatial orbitals (spin orbital 2P+s)."""
        return self.cre[2 * P] @ self.ann[2 * Q] + self.cre[2 * P + 1] @ self.ann[2 * Q + 1]


def random_antisym(N, rng, scale=1.0):
    x = rng.normal(scale=scale, size=(N, N, N, N))
    x = x - x.transpose(1, 0, 2, 3)
    x = x - x.transpose(0, 1, 3, 2)
    return x / 4.0


def spin_free_hamiltonian(fs: FockSpace, h, eri, n):
    """H = sum h_pq E_pq + 1/2 sum (pq|rs)(E_pq E_rs - d_qr E_ps)."""
    E = [[fs.E(p, q) for q in range(n)] for p in range(n)]
    M = 0 * fs.I
    for p, q in itertools.product(range(n), repeat=2):
        M = M + h[p, q] * E[p][q]
    for p, q, r, s in itertools.product(range(n), repeat=4):
        if eri[p, q, r, s] != 0.0:
            term = E[p][q] @ E[r][s]
            if q == r:
                term = term - E[p][s]
            M = M + 0.5 * eri[p, q, r, s] * term
    return M.tocsr()


def sector_dets(n: int, na: int, nb: int):
    """Determinants (bit strings over 2n spin orbitals, spin orbital 2P+s)
    with na alpha and nb beta electrons."""
    out = []
    for A in itertools.combinations(range(n), na):
        for B in itertools.combinations(range(n), nb):
            b = 0
            for P in A:
                b |= 1 << (2 * P)
            for P in B:
                b |= 1 << (2 * P + 1)
            out.append(b)
    return np.array(sorted(out), dtype=np.int64)


def _apply_string(ops, bits):
    bits = bits.copy()
    sign = np.ones(len(bits))
    ok = np.ones(len(bits), dtype=bool)
    for p, dag in reversed(ops):
        occ = ((bits >> p) & 1).astype(bool)
        ok &= (~occ) if dag else occ
        par = np.bitwise_count(bits & ((1 << p) - 1)) & 1
        sign *= np.where(par == 1, -1.0, 1.0)
        bits ^= 1 << p
    return bits, sign, ok


def sector_hamiltonian(h, eri, n, na, nb, e_core=0.0):
    """Dense H = e_core + sum_{pq,s} h_pq a+_ps a_qs
    + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs on a fixed-(na,nb)
    determinant sector of n spatial orbitals."""
    dets = sector_dets(n, na, nb)
    index = {int(d): k for k, d in enumerate(dets)}
    D = len(dets)
    H = e_core * np.eye(D)

    def add(coef, ops):
        bits, sign, ok = _apply_string(ops, dets)
        cols = np.nonzero(ok)[0]
        rows = np.searchsorted(dets, bits[cols])
        rows = np.minimum(rows, D - 1)
        hit = dets[rows] == bits[cols]
        np.add.at(H, (rows[hit], cols[hit]), coef * sign[cols][hit])

    for p, q in itertools.product(range(n), repeat=2):
        if h[p, q] != 0.0:
            for s in (0, 1):
                add(h[p, q], [(2 * p + s, 1), (2 * q + s, 0)])
    for p, q, r, s_ in itertools.product(range(n), repeat=4):
        if eri[p, q, r, s_] != 0.0:
            for s in (0, 1):
                for t in (0, 1):
                    add(0.5 * eri[p, q, r, s_],
                        [(2 * p + s, 1), (2 * r + t, 1), (2 * s_ + t, 0), (2 * q + s, 0)])
    return H, dets
