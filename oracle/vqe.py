"""UCCSD-VQE active-space solver: the paper's solver in place of the CI
eigenvector and its cluster analysis.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (8) at N=1 gives the trial state of active space i as e^{sigma_int(i)}|Phi>
and Eq. (5) its energy E(i) = <Phi| e^{-sigma_int} H_eff(i) e^{sigma_int} |Phi>;
the paper finds sigma_int(i) by a variational quantum eigensolver over a UCCSD
ansatz and writes the optimised parameters back into the amplitude pool
("Numerical Implementation").  Here the ansatz is evaluated exactly in the
space's determinant basis:

* parameters: the space's spin-adapted singles t1[I,A] and doubles
  t2[I,J,A,B] = t2[J,I,B,A] (local indices), i.e. the pool's amplitudes
  restricted to the space; T = sum t1 E_AI + 1/2 sum t2 E_AI E_BJ with
  spin-summed excitation operators E, and sigma_int = T - T^dagger;
* state: psi(theta) = expm(A) e_Phi with A the (real, antisymmetric) matrix
  of sigma_int in the space's Sz = 0 determinant basis (oracle.cas);
* energy: psi^T H psi with H the space's CAS matrix;
* gradient: dE/dtheta_k = 2 w^T L(A, G_k) e_Phi with w = H psi and L the
  Frechet derivative of the matrix exponential, evaluated exactly by the
  Daleckii-Krein formula for a normal matrix A = V diag(mu) V^H:
  L(A, G) = V [(V^H G V) o Phi] V^H with Phi_ij = (e^mu_i - e^mu_j) /
  (mu_i - mu_j) (e^mu_i where mu_i = mu_j), mu = i lam purely imaginary;
* minimiser: BFGS (scipy.optimize.minimize) from a given start (by default
  the pool's own amplitudes of the space), then Newton steps with the
  Hessian from central differences of the exact gradient until the
  gradient's largest entry is below gtol.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg
import scipy.optimize

from .cas import _apply, basis


def parameter_list(n_occ: int, n_vir: int):
    """Unique spin-adapted parameters: ('s', I, A) for every single, then
    ('d', I, J, A, B) for every pair (I, A) <= (J, B) of singles (the doubles
    t2[I,J,A,B] = t2[J,I,B,A] share one parameter)."""
    singles = [(I, A) for I in range(n_occ) for A in range(n_vir)]
    out = [("s", I, A) for I, A in singles]
    for p, (I, A) in enumerate(singles):
        for J, B in singles[p:]:
            out.append(("d", I, J, A, B))
    return out


def _string_matrix(B, ops):
    """Dense matrix of a plain operator product in the CAS basis."""
    bits, sign, valid = _apply(ops, B.dets)
    M = np.zeros((B.dim, B.dim))
    cols = np.nonzero(valid)[0]
    for c in cols:
        r = B.index.get(int(bits[c]), -1)
        if r >= 0:
            M[r, c] += sign[c]
    return M


def excitation(B, P: int, Q: int):
    """Spin-summed E_PQ = sum_s a+_{P s} a_{Q s} (local spatial orbitals)."""
    return _string_matrix(B, [(2 * P, 1), (2 * Q, 0)]) + _string_matrix(B, [(2 * P + 1, 1), (2 * Q + 1, 0)])


def generators(n_occ: int, n_vir: int):
    """Matrices G_k = T_k - T_k^T of sigma_int's parameters (parameter_list
    order): T_k = E_AI for a single; E_AI E_BJ for a pair of distinct singles
    (the two equal terms of 1/2 sum t2 E_AI E_BJ); 1/2 E_AI E_AI for a pair
    of equal ones."""
    na = n_occ + n_vir
    B = basis(n_occ, na)
    E = {}

    def e(A, I):
        if (A, I) not in E:
            E[(A, I)] = excitation(B, n_occ + A, I)
        return E[(A, I)]

    gens = []
    for par in parameter_list(n_occ, n_vir):
        if par[0] == "s":
            _, I, A = par
            T = e(A, I)
        else:
            _, I, J, A, Bv = par
            T = e(A, I) @ e(Bv, J)
            if (I, A) == (J, Bv):
                T = 0.5 * T
        gens.append(T - T.T)
    return np.array(gens)


def pack(t1, t2, n_occ, n_vir):
    """Local amplitudes -> parameter vector."""
    out = []
    for par in parameter_list(n_occ, n_vir):
        out.append(t1[par[1], par[2]] if par[0] == "s" else t2[par[1], par[2], par[3], par[4]])
    return np.array(out)


def unpack(theta, n_occ, n_vir):
    """Parameter vector -> local t1[I,A], t2[I,J,A,B] (t2 pair symmetric)."""
    t1 = np.zeros((n_occ, n_vir))
    t2 = np.zeros((n_occ, n_occ, n_vir, n_vir))
    for x, par in zip(theta, parameter_list(n_occ, n_vir)):
        if par[0] == "s":
            t1[par[1], par[2]] = x
        else:
            _, I, J, A, B = par
            t2[I, J, A, B] = x
            t2[J, I, B, A] = x
    return t1, t2


def energy(theta, H, gens, iref):
    A = np.tensordot(theta, gens, axes=1)
    psi = scipy.linalg.expm(A)[:, iref]
    return float(psi @ H @ psi)


def energy_gradient(theta, H, gens, iref):
    """(E, dE/dtheta) with the exact Frechet derivative (Daleckii-Krein)."""
    A = np.tensordot(theta, gens, axes=1)
    # A real antisymmetric: -iA is Hermitian, A = V diag(i lam) V^H
    lam, V = np.linalg.eigh(-1j * A)
    em = np.exp(1j * lam)
    # divided differences of exp at i lam: exp(i (lam_i + lam_j) / 2) times
    # sin(d / 2) / (d / 2), d = lam_i - lam_j (no cancellation for close or
    # equal eigenvalues)
    Phi = np.exp(0.5j * (lam[:, None] + lam[None, :])) * np.sinc(
        (lam[:, None] - lam[None, :]) / (2.0 * np.pi))
    U = (V * em[None, :]) @ V.conj().T
    psi = U[:, iref].real
    w = H @ psi
    a = V.conj().T @ w
    b = V.conj().T[:, iref]
    M = np.conj(a)[:, None] * Phi * b[None, :]
    K = np.conj(V) @ M @ V.T
    grad = 2.0 * np.real(np.tensordot(gens, K, axes=([1, 2], [0, 1])))
    return float(psi @ w), grad


def solve(H, n_occ, n_vir, theta0=None, gtol=1e-10, maxiter=2000):
    """Minimise the UCCSD energy of the CAS matrix H.  Returns dict(E, theta,
    t1, t2, psi, iters, gmax)."""
    B = basis(n_occ, n_occ + n_vir)
    gens = generators(n_occ, n_vir)
    theta0 = np.zeros(len(gens)) if theta0 is None else np.asarray(theta0, dtype=float)
    res = scipy.optimize.minimize(energy_gradient, theta0, args=(H, gens, B.iref), jac=True,
                                  method="BFGS", options={"gtol": gtol, "maxiter": maxiter})
    theta = res.x
    E, g = energy_gradient(theta, H, gens, B.iref)
    # Newton steps with the Hessian from central differences of the exact
    # gradient, until the gradient is below gtol (BFGS stops early when its
    # line search runs out of precision)
    for _ in range(3):
        if np.abs(g).max() < gtol:
            break
        h = 1e-4
        Hs = np.zeros((len(theta), len(theta)))
        for j in range(len(theta)):
            e = np.zeros(len(theta))
            e[j] = h
            Hs[:, j] = (energy_gradient(theta + e, H, gens, B.iref)[1]
                        - energy_gradient(theta - e, H, gens, B.iref)[1]) / (2 * h)
        theta = theta - np.linalg.solve(0.5 * (Hs + Hs.T), g)
        E, g = energy_gradient(theta, H, gens, B.iref)
    t1, t2 = unpack(theta, n_occ, n_vir)
    psi = scipy.linalg.expm(np.tensordot(theta, gens, axes=1))[:, B.iref]
    return dict(E=E, theta=theta, t1=t1, t2=t2, psi=psi, iters=res.nit,
                gmax=float(np.abs(g).max()))


def solve_space(pb, t1, t2, orbs, n_occ, gtol=1e-10):
    """The VQE solution of one space of the flow: its downfolded Hamiltonian
    from the pool (t1, t2), minimised from the pool's own amplitudes of the
    space; returns the space energy and the local amplitudes to write back."""
    from . import qflow
    x = qflow.heff(pb, t1, t2, orbs)
    H = qflow.cas_matrix(*x, n_occ)
    occ, vir = orbs[:n_occ], orbs[n_occ:]
    o = pb.o
    lt1 = t1[np.ix_(occ, [a - o for a in vir])]
    lt2 = t2[np.ix_(occ, occ, [a - o for a in vir], [a - o for a in vir])]
    n_vir = len(vir)
    s = solve(H, n_occ, n_vir, theta0=pack(lt1, lt2, n_occ, n_vir), gtol=gtol)
    s["c0"] = 1.0            # the write-back does not divide by a reference weight
    s["x"] = x
    return s


def flow_step(pb, t1, t2, spaces, owner1, owner2, unowned="residual", gtol=1e-10):
    """One Jacobi macro-iteration with the VQE solver: every space's amplitudes
    are its optimised parameters (no cluster analysis); ownership, the
    unowned residual step and the mean are those of qflow.flow_step."""
    from . import qflow
    o = pb.o
    sols = [solve_space(pb, t1, t2, tuple(occ) + tuple(vir), len(occ), gtol)
            for (occ, vir) in spaces]
    E = np.array([s["E"] for s in sols])
    nt1, nt2 = t1.copy(), t2.copy()
    if unowned == "residual" and (np.any(owner1 < 0) or np.any(owner2 < 0)):
        R1, R2, _ = qflow.residual(pb, t1, t2)
        d1, d2 = qflow.denominators(pb.eps, o)
        nt1 = np.where(owner1 < 0, t1 - R1 / d1, nt1)
        nt2 = np.where(owner2 < 0, t2 - R2 / d2, nt2)
    for k, (occ, vir) in enumerate(spaces):
        qflow.write_owned(nt1, nt2, sols[k], k, occ, vir, owner1, owner2, o)
    return nt1, nt2, E, qflow.mean_energy(E), sols
