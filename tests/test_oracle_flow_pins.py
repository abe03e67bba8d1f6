"""Pins of the oracle's flow update and of its MP2 start.

Each reference value here comes from exact second quantisation on a tiny Fock
space (tests/bruteforce.py), never from the oracle's own formulas, and each pin
has a companion test that plants a plausible mistake in the oracle and checks
that the pin then fails:

* the residual Jacobi step of amplitudes no space owns, driven through
  ``flow_step`` with no spaces, reaches the exact zero-residual fixed point
  (the residual projected with dense Fock-space matrices);
* the owned write-back: with one space that holds every orbital, the pool
  after one step equals the intermediate-normalised cluster amplitudes of the
  brute-force full-CI vector (Jordan-Wigner determinants);
* the fixed point does not depend on the start (zero or MP2 pool);
* the MP2 start equals the first-order Rayleigh-Schroedinger wavefunction
  with the diagonal Fock operator as zeroth-order Hamiltonian, and its
  amplitude energy equals the brute-force second-order energy.
"""
import itertools

import numpy as np
import pytest

import synth
from bruteforce import FockSpace, sector_hamiltonian, spin_free_hamiltonian
from oracle import qflow, sampling, so


def small_problem(n, o, seed, b_std=0.05, off_std=0.05):
    return synth.gen_integrals(n, o, 2 * n, seed, b_std=b_std, off_std=off_std)


def brute_T(fs, n, o, t1, t2):
    T = 0 * fs.I
    for i in range(o):
        for a in range(n - o):
            T = T + t1[i, a] * fs.E(o + a, i)
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            T = T + 0.5 * t2[i, j, a, b] * (fs.E(o + a, i) @ fs.E(o + b, j))
    return T.tocsr()


def ref_vector(fs, o):
    r = np.zeros(fs.dim)
    r[fs.ref_state(2 * o)] = 1.0
    return r


def single_det(fs, o, i, a):
    """a+_{a alpha} i_{alpha} Phi (absolute spatial indices)."""
    return (fs.cre[2 * a] @ fs.ann[2 * i]) @ ref_vector(fs, o)


def double_det(fs, o, i, j, a, b):
    """a+_{a alpha} b+_{b beta} j_{beta} i_{alpha} Phi."""
    return (fs.cre[2 * a] @ fs.cre[2 * b + 1] @ fs.ann[2 * j + 1] @ fs.ann[2 * i]) \
        @ ref_vector(fs, o)


def exact_residual(fs, pb, h, eri, t1, t2):
    """max |<X| H + [H,s] + 1/2[[F,s],s] |Phi>| over X = singles and doubles,
    from dense Fock-space matrices (no normal-ordered algebra)."""
    n, o = pb.n, pb.o
    T = brute_T(fs, n, o, t1, t2)
    S = (T - T.T).toarray()
    H = spin_free_hamiltonian(fs, h, eri, n).toarray()
    F = fs.operator(0.0, so.to_dense(pb.F, pb.bl)[1], np.zeros((2 * n,) * 4), 2 * o).toarray()
    Y = F @ S - S @ F
    Xphi = (H + (H @ S - S @ H) + 0.5 * (Y @ S - S @ Y)) @ ref_vector(fs, o)
    r = 0.0
    for i in range(o):
        for a in range(o, n):
            r = max(r, abs(single_det(fs, o, i, a) @ Xphi))
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(o, n), repeat=2):
            r = max(r, abs(double_det(fs, o, i, j, a, b) @ Xphi))
    return r


# --------------------------------------------------------------------------
# (a) no spaces: flow_step is the residual iteration; its fixed point has R=0
# --------------------------------------------------------------------------

def _residual_fixed_point(steps=60):
    n, o = 5, 2
    h, eri = small_problem(n, o, 91, b_std=0.03, off_std=0.02)
    pb = qflow.Problem(h, eri, o)
    v = n - o
    o1 = -np.ones((o, v), np.int32)
    o2 = -np.ones((o, o, v, v), np.int32)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    for _ in range(steps):
        t1, t2, E, Em, _s = qflow.flow_step(pb, t1, t2, [], o1, o2)
        if not (np.all(np.isfinite(t1)) and np.all(np.isfinite(t2))):
            return np.inf, Em, E
    fs = FockSpace(2 * n)
    return exact_residual(fs, pb, h, eri, t1, t2), Em, E


def test_flow_step_without_spaces_reaches_zero_residual():
    r, Em, E = _residual_fixed_point()
    assert len(E) == 0 and np.isnan(Em)
    assert r < 1e-10


def test_zero_residual_pin_catches_a_sign_slip(monkeypatch):
    good = qflow.denominators

    def slipped(eps, o):
        d1, d2 = good(eps, o)
        return d1, -d2
    monkeypatch.setattr(qflow, "denominators", slipped)
    r, _, _ = _residual_fixed_point()
    assert not r < 1e-6


# --------------------------------------------------------------------------
# (b) one space holding every orbital: the write-back is the full-CI vector's
#     cluster amplitudes
# --------------------------------------------------------------------------

def _fci_cluster_amplitudes(h, eri, n, o):
    """t1[i,a], t2[i,j,a,b] (i,a alpha; j,b beta) of the brute-force FCI
    ground state: C = coefficients over c_Phi of the Jordan-Wigner
    determinants a+ i Phi and a+ b+ j i Phi; T1 = C1, T2 = C2 - C1 C1."""
    H, dets = sector_hamiltonian(h, eri, n, o, o)
    w, U = np.linalg.eigh(H)
    fs = FockSpace(2 * n)
    psi = np.zeros(fs.dim)
    psi[dets] = U[:, 0]
    ref = ref_vector(fs, o)
    c0 = ref @ psi
    psi = psi / c0
    v = n - o
    t1 = np.zeros((o, v))
    t2 = np.zeros((o, o, v, v))
    for i in range(o):
        for a in range(v):
            t1[i, a] = single_det(fs, o, i, o + a) @ psi
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(v), repeat=2):
            c2 = double_det(fs, o, i, j, o + a, o + b) @ psi
            t2[i, j, a, b] = c2 - t1[i, a] * t1[j, b]
    return w[0], t1, t2


def _whole_space_write_back_error():
    n, o = 6, 3
    h, eri = small_problem(n, o, 141, b_std=0.1)
    pb = qflow.Problem(h, eri, o)
    spaces = [(tuple(range(o)), tuple(range(o, n)))]
    o1, o2 = sampling.ownership(o, n - o, spaces)
    assert np.all(o1 == 0) and np.all(o2 == 0)
    t1, t2 = synth.random_amplitudes(o, n - o, 142, scale=0.1)
    nt1, nt2, E, Em, _s = qflow.flow_step(pb, t1, t2, spaces, o1, o2)
    e_fci, f1, f2 = _fci_cluster_amplitudes(h, eri, n, o)
    assert abs(Em - e_fci) < 1e-10
    assert np.abs(f2).max() > 1e-2 and np.abs(f1).max() > 1e-3
    return max(np.abs(nt1 - f1).max(), np.abs(nt2 - f2).max())


def test_whole_space_write_back_is_fci_cluster_amplitudes():
    assert _whole_space_write_back_error() < 1e-9


def test_write_back_pin_catches_transposed_doubles(monkeypatch):
    def transposed(t1, t2, sol, k, occ, vir, owner1, owner2, o):
        for I, i in enumerate(occ):
            for A, a in enumerate(vir):
                if owner1[i, a - o] == k:
                    t1[i, a - o] = sol["t1"][I, A]
        for I, i in enumerate(occ):
            for J, j in enumerate(occ):
                for A, a in enumerate(vir):
                    for B, b in enumerate(vir):
                        if owner2[i, j, a - o, b - o] == k:
                            t2[j, i, a - o, b - o] = sol["t2"][I, J, A, B]
    monkeypatch.setattr(qflow, "write_owned", transposed)
    assert _whole_space_write_back_error() > 1e-4


# --------------------------------------------------------------------------
# (c) zero and MP2 starts reach the same fixed point; runs are deterministic
# --------------------------------------------------------------------------

def _fixed_points(max_steps=80):
    n, o = 12, 3
    h, eri = synth.gen_integrals(n, o, 2 * n, 161, b_std=0.03, off_std=0.02)
    pb = qflow.Problem(h, eri, o)
    lists = [(s[0], s[1]) for s in sampling.algorithm1(o, n - o, 2, 2, pb.eps,
                                                       synth.Stream(161), cap=6)]
    o1, o2 = sampling.ownership(o, n - o, lists)
    assert np.any(o2 >= 0) and np.any(o2 < 0)
    starts = [(np.zeros((o, n - o)), np.zeros((o, o, n - o, n - o))),
              qflow.mp2_guess(pb.f, eri, o)]
    out = []
    for t1, t2 in starts:
        for _ in range(max_steps):
            n1, n2, E, Em, _s = qflow.flow_step(pb, t1, t2, lists, o1, o2)
            dt = max(np.abs(n1 - t1).max(), np.abs(n2 - t2).max())
            t1, t2 = n1, n2
            if dt < 1e-12:
                break
        out.append((t1, t2, E, Em, dt))
    return out, (pb, lists, o1, o2)


def test_zero_and_mp2_starts_reach_one_fixed_point():
    (a, b), (pb, lists, o1, o2) = _fixed_points()
    assert a[4] < 1e-11 and b[4] < 1e-11
    assert abs(a[3] - b[3]) < 1e-9
    assert np.abs(a[2] - b[2]).max() < 1e-9
    assert max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) < 1e-9
    # at the fixed point one more step changes t by < 1e-9 and E by < 1e-11,
    # and repeating that step gives the same bits
    n1, n2, E, Em, _ = qflow.flow_step(pb, a[0], a[1], lists, o1, o2)
    m1, m2, E2, Em2, _ = qflow.flow_step(pb, a[0], a[1], lists, o1, o2)
    assert max(np.abs(n1 - a[0]).max(), np.abs(n2 - a[1]).max()) < 1e-9
    assert abs(Em - a[3]) < 1e-11
    assert np.array_equal(n1, m1) and np.array_equal(n2, m2) and Em == Em2


def test_fixed_point_pin_catches_a_missing_write_back(monkeypatch):
    monkeypatch.setattr(qflow, "write_owned", lambda *args: None)
    (a, b), _ = _fixed_points(max_steps=40)
    assert max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) > 1e-4


# --------------------------------------------------------------------------
# (d) MP2 start = first-order Rayleigh-Schroedinger wavefunction
# --------------------------------------------------------------------------

def _first_order_wavefunction(h, eri, n, o):
    """Brute force, zeroth-order H0 = sum_P eps_P (n_P alpha + n_P beta) with
    eps = diag(f): psi1 = sum_X |X> <X|H|Phi> / (E0(Phi) - E0(X)) over every
    determinant X != Phi; returns (fs, psi1, H, ref)."""
    pb = qflow.Problem(h, eri, o)
    fs = FockSpace(2 * n)
    H = spin_free_hamiltonian(fs, h, eri, n)
    ref = ref_vector(fs, o)
    col = H @ ref
    eps_so = np.repeat(pb.eps, 2)
    e0 = np.array([sum(eps_so[p] for p in range(2 * n) if (s >> p) & 1)
                   for s in range(fs.dim)])
    phi = fs.ref_state(2 * o)
    psi1 = np.zeros(fs.dim)
    sector = fs.nel == 2 * o
    for s in np.nonzero(sector)[0]:
        if s != phi:
            psi1[s] = col[s] / (e0[phi] - e0[s])
    return fs, psi1, H, ref, pb


def _mp2_pin_error(n, o, seed, t1, t2):
    h, eri = small_problem(n, o, seed)
    fs, psi1, _, _, _ = _first_order_wavefunction(h, eri, n, o)
    err = 0.0
    for i in range(o):
        for a in range(n - o):
            err = max(err, abs(single_det(fs, o, i, o + a) @ psi1 - t1[i, a]))
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            err = max(err, abs(double_det(fs, o, i, j, o + a, o + b) @ psi1 - t2[i, j, a, b]))
    return err


def test_mp2_guess_is_first_order_wavefunction():
    n, o = 5, 2
    h, eri = small_problem(n, o, 171)
    pb = qflow.Problem(h, eri, o)
    assert np.abs(pb.f[:o, o:]).max() > 1e-2          # singles are present
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    assert _mp2_pin_error(n, o, 171, t1, t2) < 1e-13


def test_mp2_pin_catches_swapped_virtuals():
    n, o = 5, 2
    h, eri = small_problem(n, o, 171)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    assert _mp2_pin_error(n, o, 171, t1, t2.transpose(0, 1, 3, 2)) > 1e-4


def test_mp2_energy_is_second_order_energy():
    """Diagonal Fock matrix (so f_ia = 0): <Phi|H T|Phi> with the MP2
    amplitudes equals sum_X |<X|H|Phi>|^2 / (E0(Phi) - E0(X))."""
    n, o = 5, 2
    h, eri = small_problem(n, o, 181)
    pb0 = qflow.Problem(h, eri, o)
    h = h - (pb0.f - np.diag(np.diag(pb0.f)))          # makes f diagonal
    pb = qflow.Problem(h, eri, o)
    assert np.abs(pb.f - np.diag(np.diag(pb.f))).max() < 1e-14
    fs, psi1, H, ref, _ = _first_order_wavefunction(h, eri, n, o)
    e2 = ref @ (H @ psi1)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    assert np.abs(t1).max() < 1e-15
    T = brute_T(fs, n, o, t1, t2)
    e_amp = ref @ (H @ (T @ ref))
    assert e2 < -1e-4
    assert abs(e_amp - e2) < 1e-13 * max(1.0, abs(e2))
