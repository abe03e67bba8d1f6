"""Pins of the CPU oracle against things other than itself.

Every reference value here comes from exact second quantisation on tiny Fock
spaces (tests/bruteforce.py), closed forms, or numbers the paper prints.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import synth
from bruteforce import FockSpace, random_antisym, sector_hamiltonian, spin_free_hamiltonian
from oracle import qflow, sampling, so
from oracle.cas import basis


def small_problem(n, o, seed, b_std=0.05, off_std=0.05):
    h, eri = synth.gen_integrals(n, o, 2 * n, seed, b_std=b_std, off_std=off_std)
    return h, eri


def brute_T(fs, n, o, t1, t2):
    """T1 + T2 = sum t1[i,a] E_ai + 1/2 sum t2[i,j,a,b] E_ai E_bj."""
    T = 0 * fs.I
    for i in range(o):
        for a in range(n - o):
            T = T + t1[i, a] * fs.E(o + a, i)
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            T = T + 0.5 * t2[i, j, a, b] * (fs.E(o + a, i) @ fs.E(o + b, j))
    return T.tocsr()


def low_qp_mask(fs, nocc_so, max_qp=5):
    qp = fs.qp_count(nocc_so)
    return (qp[:, None] + qp[None, :]) <= max_qp


# --------------------------------------------------------------------------
# commutator algebra
# --------------------------------------------------------------------------

def _commutator_error(seed):
    rng = np.random.default_rng(seed)
    n, o = 4, 2
    N, nocc = 2 * n, 2 * o
    bl = so.Blocks(n, o)
    fs = FockSpace(N)
    A = (rng.normal(), rng.normal(size=(N, N)), random_antisym(N, rng))
    B = (rng.normal(), rng.normal(size=(N, N)), random_antisym(N, rng))
    MA, MB = fs.operator(*A, nocc), fs.operator(*B, nocc)
    exact = (MA @ MB - MB @ MA).toarray()
    Z = so.to_dense(so.Commutator(so.Dense(*A), so.Dense(*B), bl), bl)
    MZ = fs.operator(*Z, nocc).toarray()
    m = low_qp_mask(fs, nocc)
    # elements whose bra and ket carry <= 5 quasi-particles in total see only
    # the 0-, 1- and 2-body parts; the dropped 3-body part needs 6.
    return np.abs((exact - MZ)[m]).max(), np.abs(exact[m]).max()


@pytest.mark.parametrize("seed", [11, 12])
def test_commutator_matches_exact_fock_space(seed):
    err, scale = _commutator_error(seed)
    assert scale > 1.0
    assert err < 1e-12 * scale


def test_commutator_pin_catches_a_dropped_term(monkeypatch):
    # a planted mistake in the oracle (the particle-hole term dropped) must fail
    monkeypatch.setattr(so, "_ph", lambda A, B, P, Q, R, S, bl: so._z(P, Q, R, S))
    err, scale = _commutator_error(11)
    assert err > 1e-3 * scale


# --------------------------------------------------------------------------
# Hamiltonian, reference quantities and the cluster operator
# --------------------------------------------------------------------------

def test_normal_ordered_hamiltonian_is_exact():
    n, o = 4, 2
    h, eri = small_problem(n, o, 7)
    fs = FockSpace(2 * n)
    pb = qflow.Problem(h, eri, o)
    exact = spin_free_hamiltonian(fs, h, eri, n).toarray()
    x = so.to_dense(pb.H, pb.bl)
    M = fs.operator(*x, 2 * o).toarray()
    assert np.abs(exact - M).max() < 1e-12
    # E_ref is the expectation value in Phi; eps are Fock diagonals
    ref = fs.ref_state(2 * o)
    assert abs(exact[ref, ref] - pb.e_ref) < 1e-12


def test_cluster_operator_spin_adaptation():
    n, o = 4, 2
    fs = FockSpace(2 * n)
    t1, t2 = synth.random_amplitudes(o, n - o, 5, scale=0.3)
    bl = so.Blocks(n, o)
    T = brute_T(fs, n, o, t1, t2)
    sigma = (T - T.T).toarray()
    M = fs.operator(*so.to_dense(so.Cluster(bl, t1, t2), bl), 2 * o).toarray()
    assert np.abs(sigma - M).max() < 1e-13


# --------------------------------------------------------------------------
# the downfolded Hamiltonian, every block
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mask", [None, (0, 2, 3), (1, 3)])
def test_hbar_every_block_matches_exact_commutators(mask):
    n, o = 4, 2
    h, eri = small_problem(n, o, 3)
    pb = qflow.Problem(h, eri, o)
    fs = FockSpace(2 * n)
    t1, t2 = synth.random_amplitudes(o, n - o, 9, scale=0.2)
    nocc = 2 * o
    ext_t1, ext_t2 = t1.copy(), t2.copy()
    if mask is not None:
        m = np.zeros(n, bool)
        m[list(mask)] = True
        for i in range(o):
            for a in range(n - o):
                if m[i] and m[o + a]:
                    ext_t1[i, a] = 0
        for i, j in itertools.product(range(o), repeat=2):
            for a, b in itertools.product(range(n - o), repeat=2):
                if m[i] and m[j] and m[o + a] and m[o + b]:
                    ext_t2[i, j, a, b] = 0
    T = brute_T(fs, n, o, ext_t1, ext_t2)
    S = (T - T.T).toarray()
    H = spin_free_hamiltonian(fs, h, eri, n).toarray()
    F = fs.operator(0.0, so.to_dense(pb.F, pb.bl)[1], np.zeros((2 * n,) * 4), nocc).toarray()
    Hn = H - pb.e_ref * np.eye(fs.dim)
    C1 = Hn @ S - S @ Hn
    Y = F @ S - S @ F
    C2 = Y @ S - S @ Y
    exact = H + C1 + 0.5 * C2
    Hb = qflow.hbar(pb, t1, t2, mask=mask)
    M = fs.operator(*so.to_dense(Hb, pb.bl), nocc).toarray()
    msk = low_qp_mask(fs, nocc)
    assert np.abs((exact - M)[msk]).max() < 1e-12 * max(1.0, np.abs(exact).max())


def test_residual_is_exact_projection():
    """R1, R2 and E0 equal <X| H + [H,s] + 1/2[[F,s],s] |Phi> exactly (the
    dropped three-body parts never reach singles or doubles from Phi)."""
    n, o = 4, 2
    h, eri = small_problem(n, o, 21)
    pb = qflow.Problem(h, eri, o)
    fs = FockSpace(2 * n)
    t1, t2 = synth.random_amplitudes(o, n - o, 22, scale=0.2)
    T = brute_T(fs, n, o, t1, t2)
    S = (T - T.T).toarray()
    H = spin_free_hamiltonian(fs, h, eri, n).toarray()
    F = fs.operator(0.0, so.to_dense(pb.F, pb.bl)[1], np.zeros((2 * n,) * 4), 2 * o).toarray()
    Y = F @ S - S @ F
    X = H + (H @ S - S @ H) + 0.5 * (Y @ S - S @ Y)
    ref = np.zeros(fs.dim)
    ref[fs.ref_state(2 * o)] = 1.0
    Xphi = X @ ref
    R1, R2, E0 = qflow.residual(pb, t1, t2)
    assert abs(E0 - ref @ Xphi) < 1e-12
    for i in range(o):
        for a in range(n - o):
            det = (fs.cre[2 * (o + a)] @ fs.ann[2 * i]) @ ref
            assert abs(det @ Xphi - R1[i, a]) < 1e-12
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(n - o), repeat=2):
            det = (fs.cre[2 * (o + a)] @ fs.cre[2 * (o + b) + 1]
                   @ fs.ann[2 * j + 1] @ fs.ann[2 * i]) @ ref
            assert abs(det @ Xphi - R2[i, j, a, b]) < 1e-12


# --------------------------------------------------------------------------
# active-space matrix, eigenproblem, cluster analysis
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,o,occ,vir", [(5, 2, (0, 1), (2, 4)), (5, 3, (0, 2), (3, 4))])
def test_bare_cas_is_projected_hamiltonian(n, o, occ, vir):
    """Zero pool: the space's matrix is H projected on determinants that keep
    the inactive orbitals as in Phi (frozen core, empty external virtuals)."""
    h, eri = small_problem(n, o, 31)
    pb = qflow.Problem(h, eri, o)
    orbs = occ + vir
    x = qflow.heff(pb, np.zeros((o, n - o)), np.zeros((o, o, n - o, n - o)), orbs)
    E_cas = np.linalg.eigvalsh(qflow.cas_matrix(*x, len(occ)))
    H, dets = sector_hamiltonian(h, eri, n, o, o)
    inact_occ = [P for P in range(o) if P not in occ]
    inact_vir = [P for P in range(o, n) if P not in vir]
    keep = np.ones(len(dets), bool)
    for P in inact_occ:
        keep &= ((dets >> (2 * P)) & 1).astype(bool) & ((dets >> (2 * P + 1)) & 1).astype(bool)
    for P in inact_vir:
        keep &= ~((dets >> (2 * P)) & 1).astype(bool) & ~((dets >> (2 * P + 1)) & 1).astype(bool)
    E_ref = np.linalg.eigvalsh(H[np.ix_(keep, keep)])
    assert len(E_ref) == len(E_cas)
    assert np.abs(E_ref - E_cas).max() < 1e-11


def test_whole_space_equals_fci_and_is_stationary():
    """One space holding every orbital: sigma_ext = 0, H_eff = H, so the space
    energy is the full-CI energy whatever the pool holds."""
    n, o = 6, 2
    h, eri = small_problem(n, o, 41)
    pb = qflow.Problem(h, eri, o)
    H, _ = sector_hamiltonian(h, eri, n, o, o)
    e_fci = np.linalg.eigvalsh(H)[0]
    spaces = [(tuple(range(o)), tuple(range(o, n)))]
    o1, o2 = sampling.ownership(o, n - o, spaces)
    t1, t2 = synth.random_amplitudes(o, n - o, 42, scale=0.1)
    for _ in range(2):
        t1, t2, E, Em, _s = qflow.flow_step(pb, t1, t2, spaces, o1, o2)
        assert abs(Em - e_fci) < 1e-10


def test_whole_space_fci_eight_orbitals():
    h, eri = synth.config_integrals("c1")
    pb = qflow.Problem(h, eri, 3)
    H, _ = sector_hamiltonian(h, eri, 8, 3, 3)
    e_fci = np.linalg.eigvalsh(H)[0]
    t1, t2 = synth.random_amplitudes(3, 5, 43, scale=0.05)
    orbs = tuple(range(8))
    E, c, Hc = qflow.solve_cas(*qflow.heff(pb, t1, t2, orbs), 3)
    assert Hc.shape == (3136, 3136)
    assert abs(E - e_fci) < 1e-10


def test_cas_matrix_symmetric_and_heff_four_fold():
    n, o = 6, 3
    h, eri = small_problem(n, o, 51)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = synth.random_amplitudes(o, n - o, 52, scale=0.1)
    x = qflow.heff(pb, t1, t2, (0, 1, 3, 4))
    Hc = qflow.cas_matrix(*x, 2)
    assert np.abs(Hc - Hc.T).max() < 1e-14 * np.abs(Hc).max()
    _, h1, g = qflow.heff_spatial(*x)
    assert np.abs(h1 - h1.T).max() < 1e-14
    assert np.abs(g - g.transpose(1, 0, 3, 2)).max() < 1e-14
    assert np.abs(g - g.transpose(2, 3, 0, 1)).max() < 1e-14
    # not 8-fold in general (dressed blocks break (pr|qs) <-> (rp|qs))
    assert np.abs(g - g.transpose(2, 1, 0, 3)).max() > 1e-6


def test_cluster_analysis_round_trip_and_singlet():
    n_occ, n_vir = 3, 3
    na = n_occ + n_vir
    fs = FockSpace(2 * na)
    t1, t2 = synth.random_amplitudes(n_occ, n_vir, 61, scale=0.15)
    T = brute_T(fs, na, n_occ, t1, t2).toarray()
    ref = np.zeros(fs.dim)
    ref[fs.ref_state(2 * n_occ)] = 1.0
    psi = scipy.linalg.expm(T) @ ref
    B = basis(n_occ, na)
    c = psi[B.dets]
    assert abs(np.linalg.norm(c) - np.linalg.norm(psi)) < 1e-12   # stays in the CAS
    c = c / np.linalg.norm(c)
    r1, r2 = qflow.cluster_analysis(c, n_occ, n_vir)
    assert np.abs(r1 - t1).max() < 1e-13
    assert np.abs(r2 - t2).max() < 1e-13
    # same-spin doubles: C_{i a, j a}^{a a, b a} - (t_i^a t_j^b - t_i^b t_j^a)
    c0 = c[B.iref]
    for I, J in itertools.combinations(range(n_occ), 2):
        for A, Bv in itertools.combinations(range(n_vir), 2):
            i, j = 2 * I, 2 * J
            a, b = 2 * (n_occ + A), 2 * (n_occ + Bv)
            caa = B.overlap_string([(i, 1), (j, 1), (b, 0), (a, 0)], c) / c0
            taa = caa - (t1[I, A] * t1[J, Bv] - t1[I, Bv] * t1[J, A])
            assert abs(taa - (t2[I, J, A, Bv] - t2[I, J, Bv, A])) < 1e-13


# --------------------------------------------------------------------------
# flow-level invariants
# --------------------------------------------------------------------------

def test_no_interaction_limit():
    n, o = 6, 3
    h, _ = small_problem(n, o, 71)
    h[:o, o:] = 0.0
    h[o:, :o] = 0.0
    eri = np.zeros((n,) * 4)
    pb = qflow.Problem(h, eri, o)
    spaces = [((0, 1, 2), (3, 4, 5))]
    o1, o2 = sampling.ownership(o, n - o, spaces)
    t1, t2, E, Em, _s = qflow.flow_step(pb, np.zeros((o, 3)), np.zeros((o, o, 3, 3)), spaces, o1, o2)
    assert abs(Em - pb.e_ref) < 1e-13
    assert np.abs(t1).max() < 1e-13 and np.abs(t2).max() < 1e-13


def test_correlation_energy_second_order_in_coupling():
    n, o = 6, 3
    h, eri = small_problem(n, o, 81)
    h[:o, o:] = 0.0
    h[o:, :o] = 0.0
    spaces = [((0, 1, 2), (3, 4, 5))]
    o1, o2 = sampling.ownership(o, n - o, spaces)
    ecorr = []
    for lam in (0.05, 0.1):
        pb = qflow.Problem(h, lam * eri, o)
        # remove the mean-field shift so only the fluctuation scales
        _, _, E, Em, _s = qflow.flow_step(pb, np.zeros((o, 3)), np.zeros((o, o, 3, 3)), spaces, o1, o2)
        ecorr.append(Em - pb.e_ref)
    assert ecorr[0] < 0 and ecorr[1] < 0
    assert abs(ecorr[1] / ecorr[0] - 4.0) < 0.2


def test_residual_iteration_reaches_zero_residual():
    """No spaces: every amplitude is unowned, the flow is the residual Jacobi
    iteration and its fixed point has R = 0."""
    n, o = 6, 2
    h, eri = small_problem(n, o, 91, b_std=0.03, off_std=0.02)
    pb = qflow.Problem(h, eri, o)
    v = n - o
    o1 = -np.ones((o, v), np.int32)
    o2 = -np.ones((o, o, v, v), np.int32)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    for _ in range(40):
        R1, R2, _ = qflow.residual(pb, t1, t2)
        e = pb.eps
        t1 = t1 - R1 / (e[o:][None, :] - e[:o][:, None])
        t2 = t2 - R2 / (e[o:][None, None, :, None] + e[o:][None, None, None, :]
                        - e[:o][:, None, None, None] - e[:o][None, :, None, None])
    R1, R2, _ = qflow.residual(pb, t1, t2)
    assert max(np.abs(R1).max(), np.abs(R2).max()) < 1e-10


def test_cas_integrals_reproduce_space_spectrum():
    """The vacuum-form integrals of a space, fed to a brute-force determinant
    Hamiltonian, give the spectrum of the space's normal-ordered operator."""
    n, o = 6, 3
    h, eri = small_problem(n, o, 55)
    pb = qflow.Problem(h, eri, o)
    t1, t2 = synth.random_amplitudes(o, n - o, 56, scale=0.1)
    orbs = (0, 2, 3, 5)
    x = qflow.heff(pb, t1, t2, orbs)
    ec, hs, g = qflow.cas_integrals(*x, 2)
    Hb, _ = sector_hamiltonian(hs, g, 4, 2, 2, e_core=ec)
    w1 = np.linalg.eigvalsh(Hb)
    w2 = np.linalg.eigvalsh(qflow.cas_matrix(*x, 2))
    assert np.abs(w1 - w2).max() < 1e-12


def test_diis_reaches_fixed_point_of_linear_iteration():
    """DIIS on x <- M x + c in dimension d: once more than d error vectors
    are held (and no pair was dropped) the errors are linearly dependent and
    the extrapolated vector is the exact fixed point (I - M)^-1 c; before
    the start call the plain iterate is returned unchanged."""
    rng = np.random.default_rng(7)
    d = 4
    Q = np.linalg.qr(rng.standard_normal((d, d)))[0]
    M = Q @ np.diag([0.9, -0.7, 0.5, 0.2]) @ Q.T
    c = rng.standard_normal(d)
    xstar = np.linalg.solve(np.eye(d) - M, c)
    dz = qflow.DIIS(max_vectors=8, start=3)
    x = np.zeros(d)
    for it in range(1, 7):
        xn = M @ x + c
        y = dz.step(xn, xn - x)
        if it < 3:
            assert np.array_equal(y, xn)
        x = y
    assert np.abs(x - xstar).max() < 1e-10
    # without DIIS the same six plain steps are still far from it
    z = np.zeros(d)
    for _ in range(6):
        z = M @ z + c
    assert np.abs(z - xstar).max() > 1e-2


def test_diis_coefficients_minimise_the_error_norm():
    """The returned combination's coefficients sum to one and minimise
    |sum c_i e_i| (checked against a direct constrained least-squares solve),
    and a history of identical errors (singular B) falls back to the newest
    vector."""
    rng = np.random.default_rng(8)
    d, m = 12, 5
    T = rng.standard_normal((m, d))
    E = rng.standard_normal((m, d))
    dz = qflow.DIIS(max_vectors=8, start=1)
    for i in range(m):
        y = dz.step(T[i], E[i])
    # constrained minimum: c = argmin |E^T c| with sum c = 1
    G = E @ E.T
    w = np.linalg.solve(G, np.ones(m))
    c = w / w.sum()
    assert np.abs(y - c @ T).max() < 1e-10
    dz2 = qflow.DIIS(max_vectors=8, start=1)
    e = rng.standard_normal(d)
    for i in range(3):
        y2 = dz2.step(T[i], e)
    assert np.array_equal(y2, T[2])


def test_windowed_sweep_with_one_window_is_the_jacobi_step():
    """A window holding every space reads one pool for all of them: the
    windowed sweep then equals the Jacobi macro-iteration (same solves, same
    owned writes, same residual step); with smaller windows the owned
    amplitudes of the first window still equal the Jacobi ones, while later
    windows see the updated pool."""
    h, eri = synth.gen_integrals(12, 3, 24, 181, b_std=0.04, off_std=0.03)
    pb = qflow.Problem(h, eri, 3)
    lists = [(s[0], s[1]) for s in sampling.algorithm1(3, 9, 2, 2, pb.eps, synth.Stream(181),
                                                       cap=6)]
    o1, o2 = sampling.ownership(3, 9, lists)
    t1, t2 = qflow.mp2_guess(pb.f, eri, 3)
    j1, j2, Ej, Emj, _ = qflow.flow_step(pb, t1, t2, lists, o1, o2)
    w1, w2, Ew, Emw = qflow.flow_sweep_windowed(pb, t1, t2, lists, o1, o2, window=len(lists))
    assert np.array_equal(Ew, Ej) and Emw == Emj
    assert np.array_equal(w1, j1) and np.array_equal(w2, j2)
    g1, g2, Eg, _ = qflow.flow_sweep_windowed(pb, t1, t2, lists, o1, o2, window=2)
    assert np.array_equal(Eg[:2], Ej[:2])
    first = (o2 == 0) | (o2 == 1)
    assert np.array_equal(g2[first], j2[first])
    assert not np.allclose(Eg[2:], Ej[2:], rtol=0, atol=1e-12)
