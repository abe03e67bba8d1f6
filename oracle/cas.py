"""Determinant-space representation of an active-space Hamiltonian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An active space with n_a spatial orbitals (the first n_occ of them occupied in
Phi) is handled in its 2*n_a local spin orbitals, ordered (P0 alpha, P0 beta,
P1 alpha, ...).  Determinants are bit strings over those local spin orbitals,
|D> = prod_{p ascending, bit p set} a+_p |vac>.  The CAS basis is every
determinant with n_occ alpha and n_occ beta electrons (Sz = 0), i.e. Phi plus
all excitations within the space (the span of P + Q_int of Eq. (6)).

Matrix elements are obtained by applying each normal-ordered operator string
to every basis determinant with Jordan-Wigner signs, so no Slater-Condon rule
or spin coupling formula is assumed.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


def _popcount_below(bits: np.ndarray, p: int) -> np.ndarray:
    return np.bitwise_count(bits & ((1 << p) - 1)).astype(np.int64)


def _apply(ops, dets: np.ndarray):
    """Apply the operator product ops[0] ops[1] ... (rightmost first) to each
    determinant; returns (new bit strings, sign, valid mask)."""
    bits = dets.copy()
    sign = np.ones(len(dets))
    valid = np.ones(len(dets), dtype=bool)
    for p, dag in reversed(ops):
        occ = ((bits >> p) & 1).astype(bool)
        valid &= (~occ) if dag else occ
        par = _popcount_below(bits, p) % 2
        sign = sign * np.where(par == 1, -1.0, 1.0)
        bits = bits ^ (1 << p)
    return bits, sign, valid


def _normal_order(ops, n_ref: int):
    """Reorder a string into normal order w.r.t. the reference that occupies
    local spin orbitals < n_ref: quasi-particle creators (particle a+, hole a)
    to the left.  Returns (sign, reordered ops)."""
    def qp_creator(p, dag):
        return dag != (p < n_ref)
    order = sorted(range(len(ops)), key=lambda k: (0 if qp_creator(*ops[k]) else 1, k))
    perm = list(order)
    sign = 1
    for i in range(len(perm)):
        while perm[i] != i:
            j = perm[i]
            perm[i], perm[j] = perm[j], perm[i]
            sign = -sign
    return sign, [ops[k] for k in order]


class CASBasis:
    """Sz=0 determinant basis of (2*n_occ electrons, n_a orbitals)."""

    def __init__(self, n_occ: int, n_a: int):
        self.n_occ, self.n_a = n_occ, n_a
        self.M = 2 * n_a
        dets = []
        for aocc in itertools.combinations(range(n_a), n_occ):
            for bocc in itertools.combinations(range(n_a), n_occ):
                b = 0
                for P in aocc:
                    b |= 1 << (2 * P)
                for P in bocc:
                    b |= 1 << (2 * P + 1)
                dets.append(b)
        self.dets = np.array(sorted(dets), dtype=np.int64)
        self.index = {int(d): k for k, d in enumerate(self.dets)}
        self.ref = (1 << (2 * n_occ)) - 1
        self.iref = self.index[self.ref]
        self.dim = len(self.dets)

    def _lookup(self, bits):
        return np.array([self.index.get(int(b), -1) for b in bits], dtype=np.int64)

    def string_matrix(self, ops):
        """Sparse (rows, cols, vals) of the normal-ordered string {ops}."""
        sgn, ordered = _normal_order(ops, 2 * self.n_occ)
        bits, sign, valid = _apply(ordered, self.dets)
        cols = np.nonzero(valid)[0]
        rows = self._lookup(bits[valid])
        keep = rows >= 0
        return rows[keep], cols[keep], sgn * sign[valid][keep]

    @functools.cached_property
    def couplings(self):
        """Concatenated sparse entries of every one- and two-body string:
        (rows, cols, vals, term) with term = p*M+q for {p+ q} and
        M^2 + ((p*M+q)*M+r)*M+s for {p+ q+ s r}."""
        M = self.M
        R, C, V, T = [], [], [], []
        for p, q in itertools.product(range(M), repeat=2):
            if p % 2 != q % 2:
                continue
            r, c, v = self.string_matrix([(p, 1), (q, 0)])
            R.append(r); C.append(c); V.append(v); T.append(np.full(len(r), p * M + q))
        for p, q, r_, s in itertools.product(range(M), repeat=4):
            if (p % 2) + (q % 2) != (r_ % 2) + (s % 2):
                continue
            r, c, v = self.string_matrix([(p, 1), (q, 1), (s, 0), (r_, 0)])
            R.append(r); C.append(c); V.append(v)
            T.append(np.full(len(r), M * M + ((p * M + q) * M + r_) * M + s))
        return (np.concatenate(R), np.concatenate(C), np.concatenate(V),
                np.concatenate(T))

    def matrix(self, x0: float, x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
        """<D_I| x0 + sum x1 {p+ q} + 1/4 sum x2 {p+ q+ s r} |D_J>."""
        M = self.M
        rows, cols, vals, term = self.couplings
        coef = np.concatenate([x1.reshape(-1), 0.25 * x2.reshape(-1)])
        w = vals * coef[term]
        H = np.bincount(rows * self.dim + cols, weights=w, minlength=self.dim * self.dim)
        H = H.reshape(self.dim, self.dim)
        H[np.diag_indices(self.dim)] += x0
        return H

    def overlap_string(self, ops, c: np.ndarray) -> float:
        """<ref| ops |c> for a plain (not normal-ordered) operator string."""
        bits, sign, valid = _apply(ops, self.dets)
        hit = valid & (bits == self.ref)
        return float(np.sum(sign[hit] * c[hit]))


@functools.lru_cache(maxsize=None)
def basis(n_occ: int, n_a: int) -> CASBasis:
    return CASBasis(n_occ, n_a)
