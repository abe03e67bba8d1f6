"""Pins of the oracle's spin-flip sector (reading R15: the Sz = 0 solve is
started from Phi and kept in its even-S sector).

* The spin flip of the CAS basis equals the brute-force product over the
  space's orbitals of the exchange of the two spin orbitals of each,
  1 - n_Pa - n_Pb + a+_Pa a_Pb + a+_Pb a_Pa, on the Jordan-Wigner Fock space;
  a planted mistake (the permutation sign dropped) fails that pin.
* The space matrix of a downfolded (spin-free) Hamiltonian commutes with it.
* With a closed-shell-dominated ground state the sector's lowest eigenvalue is
  the matrix's lowest; where a state of the other sector lies lower (a large
  random pool on 24 orbitals), the oracle keeps Phi's sector and that other
  state is odd under the flip.
"""
import numpy as np
import pytest

import synth
from bruteforce import FockSpace
from oracle import qflow, sampling
from oracle.cas import basis


def brute_flip(n_occ, na):
    fs = FockSpace(2 * na)
    F = fs.I
    for P in range(na):
        a, b = 2 * P, 2 * P + 1
        na_, nb_ = fs.cre[a] @ fs.ann[a], fs.cre[b] @ fs.ann[b]
        F = F @ (fs.I - na_ - nb_ + fs.cre[a] @ fs.ann[b] + fs.cre[b] @ fs.ann[a])
    B = basis(n_occ, na)
    return F.toarray()[np.ix_(B.dets, B.dets)]


@pytest.mark.parametrize("n_occ,na", [(1, 3), (2, 4), (3, 6)])
def test_spin_flip_matches_brute_force(n_occ, na):
    F = qflow.spin_flip(n_occ, na)
    assert np.array_equal(F, brute_flip(n_occ, na))
    assert np.array_equal(F @ F, np.eye(len(F)))


def test_spin_flip_pin_catches_a_dropped_sign():
    good = qflow.spin_flip(3, 6)
    assert not np.array_equal(np.abs(good), good)      # some signs are negative
    assert not np.array_equal(np.abs(good), brute_flip(3, 6))


def test_space_matrix_commutes_with_spin_flip():
    n, o = 8, 3
    h, eri = synth.gen_integrals(n, o, 2 * n, 211, b_std=0.06, off_std=0.04)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = synth.random_amplitudes(o, n - o, 212, scale=0.1)
    for orbs, no in (((0, 1, 3, 4), 2), ((0, 1, 2, 3, 5, 7), 3)):
        Hc = qflow.cas_matrix(*qflow.heff(pb, t1, t2, orbs), no)
        F = qflow.spin_flip(no, len(orbs))
        assert np.abs(Hc @ F - F @ Hc).max() < 1e-12 * np.abs(Hc).max()


def test_sector_lowest_is_the_lowest_for_closed_shell_ground_states():
    h, eri = synth.config_integrals("c1")
    pb = qflow.Problem(h, eri, 3)
    t1, t2 = qflow.mp2_guess(pb.f, eri, 3)
    for occ, vir, _ in sampling.enumerate_spaces(3, 5, 3, 3, pb.eps)[:4]:
        x = qflow.heff(pb, t1, t2, tuple(occ) + tuple(vir))
        E, c, Hc = qflow.solve_cas(*x, 3)
        assert abs(E - np.linalg.eigvalsh(Hc)[0]) < 1e-12
        assert abs(c @ Hc @ c - E) < 1e-12


def test_sector_is_kept_when_the_other_sector_lies_lower():
    n, o = 24, 4
    h, eri = synth.gen_integrals(n, o, 2 * n, 123, b_std=0.04, off_std=0.03)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = synth.random_amplitudes(o, n - o, 124, scale=0.05)
    lists = [(s[0], s[1]) for s in sampling.algorithm1(o, n - o, 3, 3, pb.eps,
                                                       synth.Stream(123), cap=4)]
    found = False
    for occ, vir in lists:
        E, c, Hc = qflow.solve_cas(*qflow.heff(pb, t1, t2, tuple(occ) + tuple(vir)), 3)
        w, U = np.linalg.eigh(Hc)
        F = qflow.spin_flip(3, 6)
        f = F[basis(3, 6).iref, basis(3, 6).iref]
        assert np.abs(F @ c - f * c).max() < 1e-10             # c in Phi's sector
        assert E >= w[0] - 1e-10
        if E > w[0] + 1e-6:
            found = True
            assert np.abs(F @ U[:, 0] + f * U[:, 0]).max() < 1e-8   # the lower one is odd
    assert found
