"""Algorithm 1 (coverage-driven active-space sampling) and amplitude ownership.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1: start from the minimal coverage set C_min of all tuples
(o1<o2, v1<v2); repeatedly draw n_o occupied and n_v virtual orbitals uniformly
without replacement, discard the candidate if it covers no tuple still in the
remaining set R, otherwise record it with Delta-eps = sum eps_v - sum eps_o and
remove what it covers from R; finally sort by Delta-eps ascending and verify
that the union of coverages equals C_min.

Sampling without replacement uses a partial Fisher-Yates shuffle of the index
list 0..N-1 driven by one uniform u in [0,1) per step:
j = k + floor(u * (N - k)).  The uniforms are passed in (a ``synth.Stream``).
``cap`` stops after that many accepted spaces (a fixed-K workload); the sort
is stable and ties in Delta-eps are broken by the orbital tuples.

Ownership: each amplitude t_i^a (i in O~, a in V~) and each pair
t_ij^ab = t_ji^ba (i,j in O~, a,b in V~) belongs to the first space in the
sorted list that reaches it, so that it is written once per sweep.
"""
from __future__ import annotations

import itertools

import numpy as np


def draw_subset(stream, N: int, k: int):
    idx = list(range(N))
    u = stream.uniform(k)
    for m in range(k):
        j = m + int(np.floor(u[m] * (N - m)))
        idx[m], idx[j] = idx[j], idx[m]
    return tuple(sorted(idx[:k]))


def algorithm1(No: int, Nv: int, no: int, nv: int, eps, stream, cap=None):
    """Returns the sorted list of (occ tuple, vir tuple, delta_eps) with
    absolute orbital indices (virtuals offset by No)."""
    R = set((o1, o2, v1, v2) for o1, o2 in itertools.combinations(range(No), 2)
            for v1, v2 in itertools.combinations(range(No, No + Nv), 2))
    cmin = set(R)
    S = []
    while R and (cap is None or len(S) < cap):
        O = draw_subset(stream, No, no)
        V = tuple(No + x for x in draw_subset(stream, Nv, nv))
        cov = set((o1, o2, v1, v2) for o1, o2 in itertools.combinations(O, 2)
                  for v1, v2 in itertools.combinations(V, 2)) & R
        if not cov:
            continue
        de = float(sum(eps[v] for v in V) - sum(eps[o] for o in O))
        S.append((O, V, de))
        R -= cov
    S.sort(key=lambda s: (s[2], s[0], s[1]))
    if cap is None:
        covered = set()
        for O, V, _ in S:
            covered |= set((o1, o2, v1, v2) for o1, o2 in itertools.combinations(O, 2)
                           for v1, v2 in itertools.combinations(V, 2))
        assert covered == cmin, "Algorithm 1: coverage check failed"
    return S


def enumerate_spaces(No: int, Nv: int, no: int, nv: int, eps):
    """Every (O~, V~) pair, sorted by Delta-eps (used when the whole list is
    small enough to take, as for the 8-orbital workload)."""
    S = []
    for O in itertools.combinations(range(No), no):
        for V in itertools.combinations(range(No, No + Nv), nv):
            S.append((O, V, float(sum(eps[v] for v in V) - sum(eps[o] for o in O))))
    S.sort(key=lambda s: (s[2], s[0], s[1]))
    return S


def ownership(No: int, Nv: int, spaces):
    """owner1[i,a], owner2[i,j,a,b] (virtual indices relative to No); -1 means
    no space reaches the amplitude."""
    owner1 = -np.ones((No, Nv), dtype=np.int32)
    owner2 = -np.ones((No, No, Nv, Nv), dtype=np.int32)
    for k, sp in enumerate(spaces):
        O, V = sp[0], sp[1]
        for i in O:
            for a in V:
                if owner1[i, a - No] < 0:
                    owner1[i, a - No] = k
        for i in O:
            for j in O:
                for a in V:
                    for b in V:
                        if owner2[i, j, a - No, b - No] < 0:
                            owner2[i, j, a - No, b - No] = k
    return owner1, owner2
