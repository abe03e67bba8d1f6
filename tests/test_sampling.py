"""Algorithm 1 and ownership, pinned to numbers the paper prints."""
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import sampling

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_cycle_sizes.txt")


def table1():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, No, Nv, size = line.split()
        rows.append((name, int(No), int(Nv), int(size)))
    return rows


def eps_for(No, Nv, seed=3):
    u = synth.uniform(seed, No + Nv)
    return np.concatenate([np.sort(-2 + 1.5 * u[:No]), np.sort(0.2 + 2.8 * u[No:])])


@pytest.mark.parametrize("row", table1(), ids=lambda r: r[0])
def test_cycle_size_matches_table1(row):
    """A full Algorithm-1 cycle of (3,3) spaces has the paper's size to 5%."""
    name, No, Nv, size = row
    S = sampling.algorithm1(No, Nv, 3, 3, eps_for(No, Nv), synth.Stream(100 + Nv))
    assert abs(len(S) - size) / size < 0.05


def test_minimal_spaces_give_cmin_and_full_space_gives_one():
    No, Nv = 4, 19
    cmin = math.comb(No, 2) * math.comb(Nv, 2)
    S = sampling.algorithm1(No, Nv, 2, 2, eps_for(No, Nv), synth.Stream(7))
    assert len(S) == cmin == 1026
    S = sampling.algorithm1(No, Nv, No, Nv, eps_for(No, Nv), synth.Stream(8))
    assert len(S) == 1


def test_sorted_by_delta_eps_and_coverage_verified():
    No, Nv = 4, 19
    eps = eps_for(No, Nv)
    S = sampling.algorithm1(No, Nv, 3, 3, eps, synth.Stream(9))
    de = [s[2] for s in S]
    assert de == sorted(de)
    for O, V, d in S:
        assert abs(d - (sum(eps[v] for v in V) - sum(eps[o] for o in O))) < 1e-12


def test_parameter_count_matches_paper():
    """1.17e6 parameters for propane (13 occ, 69 virt) = unique spin-orbital
    singles and doubles (same-spin pairs i<j, a<b; opposite spins all)."""
    o, v = 13, 69
    singles = 2 * o * v
    same = 2 * math.comb(o, 2) * math.comb(v, 2)
    opposite = o * o * v * v
    assert singles + same + opposite == 1172379
    assert round((singles + same + opposite) / 1e4) / 100 == 1.17


def test_ownership_unique_first_reacher():
    No, Nv = 5, 12
    eps = eps_for(No, Nv)
    S = sampling.algorithm1(No, Nv, 3, 3, eps, synth.Stream(10), cap=40)
    o1, o2 = sampling.ownership(No, Nv, S)
    # pair symmetry and first-reacher rule
    assert np.array_equal(o2, o2.transpose(1, 0, 3, 2))
    for i, j, a, b in itertools.product(range(No), range(No), range(Nv), range(Nv)):
        reach = [k for k, s in enumerate(S) if i in s[0] and j in s[0]
                 and No + a in s[1] and No + b in s[1]]
        assert o2[i, j, a, b] == (reach[0] if reach else -1)


def test_qubit_count():
    # a (3,3) space needs 2 (3 + 3) = 12 qubits; Table 1 parents 2 (N_o+N_v)
    for name, No, Nv, _ in table1()[:5]:
        assert 2 * (No + Nv) in (46, 80, 114, 182, 228)
