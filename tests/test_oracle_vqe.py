"""Pins of the UCCSD-VQE solver of the oracle (oracle/vqe.py), each against
something other than itself:

* the generators sum_k theta_k G_k equal T - T^dagger built from spin-summed
  excitation operators on the brute-force Jordan-Wigner Fock space, with the
  pool's convention T = sum t1 E_AI + 1/2 sum t2 E_AI E_BJ (a planted mistake,
  the 1/2 of the equal pairs dropped, fails it);
* the exact gradient equals scipy's Frechet derivative of expm and central
  differences of the energy;
* the energy is variational (never below the lowest eigenvalue of the
  space's sector) and exact for two electrons;
* a Hamiltonian whose ground state is e^{sigma(theta0)} Phi gives back theta0;
* one VQE flow step with a single space holding every orbital of a
  two-electron problem gives the full-CI energy, and the pool it writes
  rebuilds the full-CI vector as e^{sigma} Phi.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import synth
from bruteforce import FockSpace, sector_hamiltonian
from oracle import qflow, sampling, vqe
from oracle.cas import basis


def brute_T(fs, n, o, t1, t2):
    T = 0 * fs.I
    for i in range(o):
        for a in range(n - o):
            T = T + t1[i, a] * fs.E(o + a, i)
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            T = T + 0.5 * t2[i, j, a, b] * (fs.E(o + a, i) @ fs.E(o + b, j))
    return T.toarray()


def _generator_error(n_occ, n_vir, seed):
    na = n_occ + n_vir
    theta = 0.3 * synth.Stream(seed).normal(len(vqe.parameter_list(n_occ, n_vir)))
    A = np.tensordot(theta, vqe.generators(n_occ, n_vir), axes=1)
    t1, t2 = vqe.unpack(theta, n_occ, n_vir)
    fs = FockSpace(2 * na)
    T = brute_T(fs, na, n_occ, t1, t2)
    B = basis(n_occ, na)
    S = (T - T.T)[np.ix_(B.dets, B.dets)]
    return np.abs(A - S).max(), np.abs(S).max()


@pytest.mark.parametrize("n_occ,n_vir", [(1, 3), (2, 2), (2, 3)])
def test_generators_are_the_cluster_operator(n_occ, n_vir):
    err, scale = _generator_error(n_occ, n_vir, 301)
    assert scale > 0.1 and err < 1e-14


def test_generator_pin_catches_a_missing_half(monkeypatch):
    good = vqe.generators

    def bad(n_occ, n_vir):
        G = good(n_occ, n_vir).copy()
        for k, par in enumerate(vqe.parameter_list(n_occ, n_vir)):
            if par[0] == "d" and (par[1], par[3]) == (par[2], par[4]):
                G[k] *= 2.0
        return G
    monkeypatch.setattr(vqe, "generators", bad)
    err, scale = _generator_error(2, 2, 301)
    assert err > 1e-3


def _space_matrix(n, o, seed, orbs, n_occ, scale=0.05):
    h, eri = synth.gen_integrals(n, o, 2 * n, seed, b_std=0.05, off_std=0.03)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = synth.random_amplitudes(o, n - o, seed + 1, scale=scale)
    return qflow.cas_matrix(*qflow.heff(pb, t1, t2, orbs), n_occ)


def test_gradient_is_exact():
    H = _space_matrix(7, 3, 311, (0, 2, 4, 6), 2)
    gens = vqe.generators(2, 2)
    iref = basis(2, 4).iref
    th = 0.2 * synth.Stream(312).normal(len(gens))
    E, g = vqe.energy_gradient(th, H, gens, iref)
    assert abs(E - vqe.energy(th, H, gens, iref)) < 1e-13
    A = np.tensordot(th, gens, axes=1)
    w = H @ scipy.linalg.expm(A)[:, iref]
    gf = np.array([2 * w @ scipy.linalg.expm_frechet(A, G)[1][:, iref] for G in gens])
    assert np.abs(g - gf).max() < 1e-12 * np.abs(g).max()
    h = 1e-5
    for k in range(len(gens)):
        e = np.zeros(len(gens))
        e[k] = h
        fd = (vqe.energy(th + e, H, gens, iref) - vqe.energy(th - e, H, gens, iref)) / (2 * h)
        assert abs(fd - g[k]) < 1e-7


def _sector_lowest(H, n_occ, na):
    F = qflow.spin_flip(n_occ, na)
    B = basis(n_occ, na)
    f = F[B.iref, B.iref]
    w, U = np.linalg.eigh(0.5 * (np.eye(B.dim) + f * F))
    Q = U[:, w > 0.5]
    return np.linalg.eigvalsh(Q.T @ H @ Q)[0]


def test_energy_is_variational_and_exact_for_two_electrons():
    # four electrons: above the space's lowest eigenvalue (but close)
    H = _space_matrix(7, 3, 321, (0, 1, 3, 5), 2)
    s = vqe.solve(H, 2, 2)
    e0 = _sector_lowest(H, 2, 4)
    assert s["gmax"] < 1e-10
    assert e0 - 1e-12 <= s["E"] < e0 + 1e-3
    # two electrons: UCCSD reaches the exact ground state
    H2 = _space_matrix(7, 2, 322, (1, 3, 4, 6), 1)
    s2 = vqe.solve(H2, 1, 3)
    assert abs(s2["E"] - _sector_lowest(H2, 1, 4)) < 1e-10


def test_parameters_of_a_ucc_ground_state_are_recovered():
    gens = vqe.generators(2, 2)
    B = basis(2, 4)
    theta0 = 0.1 * synth.Stream(331).normal(len(gens))
    U = scipy.linalg.expm(np.tensordot(theta0, gens, axes=1))
    d = 1.0 + np.arange(B.dim, dtype=float)
    d[B.iref] = -1.0
    H = U @ np.diag(d) @ U.T
    s = vqe.solve(H, 2, 2, gtol=1e-12)
    assert abs(s["E"] + 1.0) < 1e-12
    assert np.abs(s["theta"] - theta0).max() < 1e-7


def test_whole_space_vqe_flow_step_is_full_ci():
    n, o = 4, 1
    h, eri = synth.gen_integrals(n, o, 2 * n, 341, b_std=0.08, off_std=0.05)
    pb = qflow.Problem(h, eri, o)
    spaces = [((0,), (1, 2, 3))]
    o1, o2 = sampling.ownership(o, n - o, spaces)
    t1, t2 = synth.random_amplitudes(o, n - o, 342, scale=0.05)
    nt1, nt2, E, Em, sols = vqe.flow_step(pb, t1, t2, spaces, o1, o2)
    Hs, dets = sector_hamiltonian(h, eri, n, o, o)
    w, V = np.linalg.eigh(Hs)
    assert abs(Em - w[0]) < 1e-10
    # the pool written back rebuilds the FCI vector: e^{sigma} Phi
    fs = FockSpace(2 * n)
    T = brute_T(fs, n, o, nt1, nt2)
    ref = np.zeros(fs.dim)
    ref[fs.ref_state(2 * o)] = 1.0
    psi = scipy.linalg.expm(T - T.T) @ ref
    fci = np.zeros(fs.dim)
    fci[dets] = V[:, 0]
    assert abs(abs(psi @ fci) - 1.0) < 1e-9
