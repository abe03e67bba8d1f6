"""Pins of the oracle's next DUCC truncation, Problem(..., truncation="H"):
Hbar gains 1/2 [[V_N, s]_2, s]_2 (V_N the two-body part of H_N), each pinned
against something other than the oracle's own formulas:

* every block of Hbar against exact Fock-space commutators: the inner
  [V_N, s]_2 against the exact commutator of V_N = H_N - F_N with s, and the
  outer one against the exact commutator of that truncated operator with s,
  on matrix elements whose bra and ket carry at most five quasi-particles
  (the dropped three-body parts need six); planted mistakes (H_N or F_N in
  place of V_N) fail it;
* its order in the interaction: with the two-electron integrals scaled by
  lambda, no occupied-virtual one-electron coupling and MP2 amplitudes (so
  both of order lambda), the new zero-body term is of third order (the F_N
  term it completes is of second order);
* a space that holds every orbital has s = 0: its CAS problem is the bare
  Hamiltonian's full CI, for either truncation.
"""
import itertools

import numpy as np
import pytest

import synth
from bruteforce import FockSpace, sector_hamiltonian, spin_free_hamiltonian
from oracle import qflow, so


def _ext(t1, t2, mask, n, o):
    ext1, ext2 = t1.copy(), t2.copy()
    if mask is None:
        return ext1, ext2
    m = np.zeros(n, bool)
    m[list(mask)] = True
    for i in range(o):
        for a in range(n - o):
            if m[i] and m[o + a]:
                ext1[i, a] = 0
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            if m[i] and m[j] and m[o + a] and m[o + b]:
                ext2[i, j, a, b] = 0
    return ext1, ext2


def _brute_T(fs, n, o, t1, t2):
    T = 0 * fs.I
    for i in range(o):
        for a in range(n - o):
            T = T + t1[i, a] * fs.E(o + a, i)
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            T = T + 0.5 * t2[i, j, a, b] * (fs.E(o + a, i) @ fs.E(o + b, j))
    return T.tocsr()


def _low_qp(fs, nocc, max_qp=5):
    qp = fs.qp_count(nocc)
    return (qp[:, None] + qp[None, :]) <= max_qp


def _hbar_errors(mask):
    n, o = 4, 2
    h, eri = synth.gen_integrals(n, o, 2 * n, 3, b_std=0.05, off_std=0.05)
    pb = qflow.Problem(h, eri, o, truncation="H")
    fs = FockSpace(2 * n)
    nocc = 2 * o
    t1, t2 = synth.random_amplitudes(o, n - o, 9, scale=0.2)
    e1, e2 = _ext(t1, t2, mask, n, o)
    S = (_brute_T(fs, n, o, e1, e2) - _brute_T(fs, n, o, e1, e2).T).toarray()
    H = spin_free_hamiltonian(fs, h, eri, n).toarray()
    F = fs.operator(0.0, so.to_dense(pb.F, pb.bl)[1], np.zeros((2 * n,) * 4), nocc).toarray()
    Hn = H - pb.e_ref * np.eye(fs.dim)
    Vn = Hn - F
    msk = _low_qp(fs, nocc)
    # the inner commutator, truncated by the oracle, against the exact one
    Sop = so.Cluster(pb.bl, t1, t2, mask)
    W = so.to_dense(so.Commutator(pb.VN, Sop, pb.bl), pb.bl)
    MW = fs.operator(*W, nocc).toarray()
    inner = np.abs(((Vn @ S - S @ Vn) - MW)[msk]).max()
    # the whole Hbar: the outer commutator of the truncated W exactly
    C1 = Hn @ S - S @ Hn
    Y = F @ S - S @ F
    exact = H + C1 + 0.5 * (Y @ S - S @ Y) + 0.5 * (MW @ S - S @ MW)
    M = fs.operator(*so.to_dense(qflow.hbar(pb, t1, t2, mask=mask), pb.bl), nocc).toarray()
    scale = max(1.0, np.abs(exact).max())
    return inner / scale, np.abs((exact - M)[msk]).max() / scale, np.abs(MW).max()


@pytest.mark.parametrize("mask", [None, (0, 2, 3), (1, 3)])
def test_v_double_commutator_every_block_matches_exact_commutators(mask):
    inner, outer, wscale = _hbar_errors(mask)
    assert wscale > 1e-2
    assert inner < 1e-12 and outer < 1e-12


@pytest.mark.parametrize("wrong", ["HN", "F"])
def test_v_double_commutator_pin_catches_the_wrong_operator(monkeypatch, wrong):
    init = qflow.Problem.__init__

    def bad(self, *a, **k):
        init(self, *a, **k)
        self.VN = self.HN if wrong == "HN" else self.F
    monkeypatch.setattr(qflow.Problem, "__init__", bad)
    inner, outer, _ = _hbar_errors((0, 2, 3))
    assert max(inner, outer) > 1e-4


def _zero_body_terms(lam):
    n, o = 6, 2
    h, eri = synth.gen_integrals(n, o, 2 * n, 21, b_std=0.08, off_std=0.03)
    h = h.copy()
    h[:o, o:] = h[o:, :o] = 0.0   # f_ia of order lambda, so t1 is too
    pb = qflow.Problem(h, lam * eri, o, truncation="H")
    t1, t2 = qflow.mp2_guess(pb.f, lam * eri, o)
    S = so.Cluster(pb.bl, t1, t2)
    Y = so.Commutator(pb.F, S, pb.bl)
    W = so.Dense(*so.to_dense(so.Commutator(pb.VN, S, pb.bl), pb.bl))
    return 0.5 * so.Commutator(Y, S, pb.bl).zero(), 0.5 * so.Commutator(W, S, pb.bl).zero()


def test_v_double_commutator_is_third_order():
    f1, v1 = _zero_body_terms(0.02)
    f2, v2 = _zero_body_terms(0.01)
    # halving the interaction: the F_N term falls by 4, the V_N term by 8
    assert abs(f1 / f2 - 4.0) < 0.1
    assert abs(v1 / v2 - 8.0) < 0.2
    assert abs(v1) > 1e-12


@pytest.mark.parametrize("truncation", ["F", "H"])
def test_whole_space_is_full_ci_for_either_truncation(truncation):
    n, o = 4, 1
    h, eri = synth.gen_integrals(n, o, 2 * n, 31, b_std=0.08, off_std=0.05)
    pb = qflow.Problem(h, eri, o, truncation=truncation)
    t1, t2 = synth.random_amplitudes(o, n - o, 32, scale=0.1)
    s = qflow.solve_space(pb, t1, t2, (0, 1, 2, 3), 1)
    Hs, _ = sector_hamiltonian(h, eri, n, o, o)
    assert abs(s["E"] - np.linalg.eigvalsh(Hs)[0]) < 1e-10


def test_unknown_truncation_is_rejected():
    h, eri = synth.gen_integrals(4, 2, 8, 3)
    with pytest.raises(ValueError):
        qflow.Problem(h, eri, 2, truncation="V")
