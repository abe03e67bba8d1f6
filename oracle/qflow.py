"""The QFlow method (singles and doubles, N=1 Trotter) in plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the order the paper states them:

* Reference quantities of the closed-shell determinant Phi that fills the
  occupied orbitals O = {0..N_o-1} ("Numerical Implementation", first index
  paragraph): Fock matrix f, reference energy E_ref, orbital energies eps=diag f.
* sigma = T - T^dagger with T = T1 + T2 over singles and doubles (Eq. (1)),
  split per active space into sigma_int(i) (amplitudes whose indices all lie in
  the space) and sigma_ext(i) = sigma - sigma_int(i) (Eq. (3)).
* The downfolded Hamiltonian of Eq. (6) at N=1, where G = exp(sigma_ext)
  (Eq. (7)).  Its similarity transform is expanded as
      Hbar = H + [H_N, sigma_ext]_2 + 1/2 [[F_N, sigma_ext]_2, sigma_ext]_2
  (commutators truncated to 0-, 1- and 2-body parts; F_N the normal-ordered
  Fock operator), then restricted to the orbitals of the space: the projector
  P + Q_int(i) keeps Phi and every determinant excited inside the space.
  The next truncation of the expansion (the paper's route to the remaining
  correlation, closing paragraph of "Results") adds
  1/2 [[V_N, sigma_ext]_2, sigma_ext]_2 (Problem(..., truncation="H")).
* E(i) is the lowest eigenvalue of that active-space matrix in the spin-flip
  sector of Phi (Eq. (5) with the exact active-space ground state standing in
  for the UCCSD-VQE solver), with the eigenvector's reference coefficient
  made positive.
* The eigenvector is mapped back to amplitudes by intermediate-normalised
  cluster analysis: T1 = C1, T2 = C2 - T1^2/2 (in spin orbitals).
* Each amplitude is written by the first space in Delta-epsilon order that
  reaches it (ownership; amplitudes no space reaches take a residual Jacobi
  step t <- t - R/Delta with R = <X|Hbar(sigma)|Phi>).
* One macro-iteration is a Jacobi sweep: every space reads the pool as it was
  at the end of the previous sweep (the barrier at the end of each sweep).
* The flow energy is the unweighted mean of E(i) over the spaces.
"""
from __future__ import annotations

import numpy as np

from . import so
from .cas import basis


# ----------------------------------------------------------------------------
# reference quantities
# ----------------------------------------------------------------------------

def reference(h: np.ndarray, eri: np.ndarray, o: int):
    """f_pq = h_pq + sum_k [2(pq|kk) - (pk|kq)], E_ref = sum_k (h_kk + f_kk),
    eps_p = f_pp (k runs over the occupied orbitals of Phi)."""
    k = np.arange(o)
    f = h + 2.0 * eri[:, :, k, k].sum(axis=2) - eri[:, k, k, :].sum(axis=1)
    e_ref = float(np.sum(h[k, k] + f[k, k]))
    return f, e_ref, np.diag(f).copy()


def mp2_guess(f, eri, o):
    """t_ij^ab = (ia|jb)/(e_i+e_j-e_a-e_b), t_i^a = f_ia/(e_i-e_a)."""
    e = np.diag(f)
    eo, ev = e[:o], e[o:]
    t1 = f[:o, o:] / (eo[:, None] - ev[None, :])
    iajb = eri[:o, o:, :o, o:]                    # (ia|jb) as [i,a,j,b]
    t2 = iajb.transpose(0, 2, 1, 3) / (eo[:, None, None, None] + eo[None, :, None, None]
                                        - ev[None, None, :, None] - ev[None, None, None, :])
    return t1, t2


TRUNCATIONS = ("F", "H")


class Problem:
    """Integrals and reference quantities; `truncation` selects the double
    commutator of the downfolded Hamiltonian: "F" keeps 1/2 [[F_N, s]_2, s]_2
    only, "H" also 1/2 [[V_N, s]_2, s]_2 (V_N = H_N - F_N, the two-body part),
    i.e. 1/2 [[H_N, s]_2, s]_2 in all."""

    def __init__(self, h, eri, o, truncation="F"):
        if truncation not in TRUNCATIONS:
            raise ValueError(f"truncation must be one of {TRUNCATIONS}")
        self.h, self.eri, self.o = h, eri, o
        self.truncation = truncation
        self.n = h.shape[0]
        self.v = self.n - o
        self.f, self.e_ref, self.eps = reference(h, eri, o)
        self.bl = so.Blocks(self.n, o)
        self.H = so.Hamiltonian(self.f, eri, self.e_ref)
        self.HN = so.Hamiltonian(self.f, eri, 0.0)
        self.F = so.Fock(self.f)
        self.VN = so.Hamiltonian(np.zeros_like(self.f), eri, 0.0)


class Sum(so.Op):
    def __init__(self, terms):
        self.terms = terms

    def zero(self):
        return sum(w * A.zero() for w, A in self.terms)

    def one(self, I, J):
        return sum(w * A.one(I, J) for w, A in self.terms)

    def two(self, I, J, K, L):
        return sum(w * A.two(I, J, K, L) for w, A in self.terms)


def hbar(pb: Problem, t1, t2, mask=None) -> so.Op:
    """H + [H_N, s]_2 + 1/2 [[F_N, s]_2, s]_2 with s = sigma (mask None) or
    s = sigma_ext of the space whose spatial orbitals are `mask`; with the
    problem's truncation "H" also + 1/2 [[V_N, s]_2, s]_2, the inner
    commutator truncated to its 0-, 1- and 2-body parts before the outer one
    is taken."""
    S = so.Cluster(pb.bl, t1, t2, mask)
    Y = so.Commutator(pb.F, S, pb.bl)
    terms = [(1.0, pb.H), (1.0, so.Commutator(pb.HN, S, pb.bl)),
             (0.5, so.Commutator(Y, S, pb.bl))]
    if pb.truncation == "H":
        W = so.Dense(*so.to_dense(so.Commutator(pb.VN, S, pb.bl), pb.bl))
        terms.append((0.5, so.Commutator(W, S, pb.bl)))
    return Sum(terms)


def spin_orbitals(orbs):
    return np.array([2 * P + s for P in orbs for s in (0, 1)], dtype=np.int64)


# ----------------------------------------------------------------------------
# per active space
# ----------------------------------------------------------------------------

def heff(pb: Problem, t1, t2, orbs):
    """Normal-ordered (x0, x1, x2) of Eq. (6) at N=1 for the space `orbs`
    (sorted spatial orbitals, occupied first), in its local spin orbitals."""
    Hb = hbar(pb, t1, t2, mask=orbs)
    return so.restrict(Hb, spin_orbitals(orbs), pb.bl)


def heff_spatial(x0, x1, x2):
    """Spin-free view of a singlet operator restricted to a space: x0, the
    alpha-alpha one-body block and the alpha-beta two-body block
    x2[P alpha, Q beta, R alpha, S beta]."""
    return x0, x1[0::2, 0::2].copy(), x2[0::2, 1::2, 0::2, 1::2].copy()


def cas_integrals(x0, x1, x2, n_occ):
    """The space's operator relative to the empty active space,
    Ec + sum h_pq p+ q + 1/4 sum g_pqrs p+ q+ s r (spin orbitals), from its
    normal-ordered form: with k, l over the active occupied spin orbitals,
    {p+ q} = p+ q - d_pq n_p and the two-body contractions give
        h_pq = x1_pq - sum_k x2_pkqk,
        Ec   = x0 - sum_k x1_kk + 1/2 sum_kl x2_klkl.
    Returns the spin-free (Ec, h[P,Q], g[P,Q,R,S] = (PQ|RS)) with
    h = alpha-alpha block and (PQ|RS) = <P alpha R beta | Q alpha S beta>."""
    occ = np.arange(2 * n_occ)
    h = x1 - np.einsum("pkqk->pq", x2[:, occ][:, :, :, occ])
    ec = x0 - np.trace(x1[np.ix_(occ, occ)]) + 0.5 * np.einsum(
        "klkl->", x2[np.ix_(occ, occ, occ, occ)])
    hs = h[0::2, 0::2]
    g = x2[0::2, 1::2, 0::2, 1::2].transpose(0, 2, 1, 3)
    return float(ec), hs.copy(), g.copy()


def cas_matrix(x0, x1, x2, n_occ):
    na = x1.shape[0] // 2
    return basis(n_occ, na).matrix(x0, x1, x2)


def spin_flip(n_occ, na):
    """Matrix of the spin flip in the space's CAS basis: every creator
    a+_{P alpha} exchanged with a+_{P beta} (local spin orbitals 2P <-> 2P+1),
    the product reordered ascending with its permutation sign."""
    B = basis(n_occ, na)
    F = np.zeros((B.dim, B.dim))
    for k, d in enumerate(B.dets):
        occ = [p for p in range(B.M) if (int(d) >> p) & 1]
        new = [p ^ 1 for p in occ]
        order = sorted(range(len(new)), key=lambda i: new[i])
        sign, seen = 1, [False] * len(order)
        for i in range(len(order)):          # parity of the sorting permutation
            if not seen[i]:
                j, cyc = i, 0
                while not seen[j]:
                    seen[j] = True
                    j = order[j]
                    cyc += 1
                if cyc % 2 == 0:
                    sign = -sign
        F[B.index[sum(1 << p for p in new)], k] = sign
    return F


def solve_cas(x0, x1, x2, n_occ):
    """Lowest eigenpair of the active-space matrix within the spin-flip sector
    of Phi (reading R15: Sz = 0 determinants, the solve started from Phi and
    kept in its even-S sector); reference weight > 0.  The downfolded
    operator is spin-free, so the matrix commutes with the spin flip F and
    the sector is the range of the projector (1 + f F)/2, F Phi = f Phi."""
    na = x1.shape[0] // 2
    B = basis(n_occ, na)
    Hc = B.matrix(x0, x1, x2)
    F = spin_flip(n_occ, na)
    f = F[B.iref, B.iref]
    w, U = np.linalg.eigh(0.5 * (np.eye(B.dim) + f * F))
    Q = U[:, w > 0.5]
    e, V = np.linalg.eigh(Q.T @ Hc @ Q)
    c = Q @ V[:, 0]
    if c[B.iref] < 0:
        c = -c
    return float(e[0]), c, Hc


def cluster_analysis(c, n_occ, n_vir):
    """Intermediate-normalised cluster amplitudes of c (local indices).

    C_i^a = <Phi| i+ a |c>/c_Phi and C_ij^ab = <Phi| i+ j+ b a |c>/c_Phi are the
    coefficients of a+ i Phi and a+ b+ j i Phi; T1 = C1 and
    T2 = C2 - (C_i^a C_j^b - C_i^b C_j^a).  Returns spatial t1[i,a] (alpha)
    and t2[i,j,a,b] (i,a alpha; j,b beta)."""
    na = n_occ + n_vir
    B = basis(n_occ, na)
    c0 = c[B.iref]
    occ = [2 * P + s for P in range(n_occ) for s in (0, 1)]
    vir = [2 * P + s for P in range(n_occ, na) for s in (0, 1)]
    M = 2 * na
    C1 = np.zeros((M, M))
    for i in occ:
        for a in vir:
            C1[i, a] = B.overlap_string([(i, 1), (a, 0)], c) / c0
    t1 = np.zeros((n_occ, n_vir))
    t2 = np.zeros((n_occ, n_occ, n_vir, n_vir))
    for I in range(n_occ):
        for A in range(n_vir):
            t1[I, A] = C1[2 * I, 2 * (n_occ + A)]
    for I in range(n_occ):
        for J in range(n_occ):
            for A in range(n_vir):
                for Bv in range(n_vir):
                    i, j = 2 * I, 2 * J + 1
                    a, b = 2 * (n_occ + A), 2 * (n_occ + Bv) + 1
                    c2 = B.overlap_string([(i, 1), (j, 1), (b, 0), (a, 0)], c) / c0
                    t2[I, J, A, Bv] = c2 - (C1[i, a] * C1[j, b] - C1[i, b] * C1[j, a])
    return t1, t2


def solve_space(pb: Problem, t1, t2, orbs, n_occ):
    x0, x1, x2 = heff(pb, t1, t2, orbs)
    E, c, _ = solve_cas(x0, x1, x2, n_occ)
    B = basis(n_occ, len(orbs))
    c0 = c[B.iref]
    lt1, lt2 = cluster_analysis(c, n_occ, len(orbs) - n_occ)
    return dict(E=E, c0=c0, t1=lt1, t2=lt2, x=(x0, x1, x2), c=c)


# ----------------------------------------------------------------------------
# global residual
# ----------------------------------------------------------------------------

def residual(pb: Problem, t1, t2, occ=None, vir=None):
    """R1[i,a] = <Phi_i^a|Hbar(sigma)|Phi> and
    R2[i,j,a,b] = <Phi_{i alpha j beta}^{a alpha b beta}|Hbar(sigma)|Phi>,
    E0 = <Phi|Hbar(sigma)|Phi>.  occ/vir optionally restrict the output to
    subsets of spatial occupied / virtual orbitals (absolute indices)."""
    o, n = pb.o, pb.n
    occ = np.arange(o) if occ is None else np.asarray(occ)
    vir = np.arange(o, n) if vir is None else np.asarray(vir)
    Hb = hbar(pb, t1, t2)
    Ia, Ib = ("o", 2 * occ), ("o", 2 * occ + 1)
    Aa, Ab = ("v", 2 * vir), ("v", 2 * vir + 1)
    R1 = Hb.one(Aa, Ia).T.copy()
    R2 = Hb.two(Aa, Ab, Ia, Ib).transpose(2, 3, 0, 1).copy()
    return R1, R2, Hb.zero()


# ----------------------------------------------------------------------------
# one macro-iteration
# ----------------------------------------------------------------------------

REF_WEIGHT_MIN = 0.1

_SHARED = None


def _one_blas_thread():
    """Worker start-up: one BLAS thread per worker process (the workers
    already spread the spaces over the cores)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass


def _solve_shared(k):
    pb, t1, t2, spaces = _SHARED
    occ, vir = spaces[k]
    return solve_space(pb, t1, t2, tuple(occ) + tuple(vir), len(occ))


def solve_spaces(pb: Problem, t1, t2, spaces, workers=1):
    """solve_space for every space of the list, all from the same pool (the
    Jacobi sweep).  The spaces are independent, so with workers > 1 they are
    spread over forked processes; each solve is the same computation either
    way."""
    if workers <= 1 or len(spaces) < 2:
        return [solve_space(pb, t1, t2, tuple(occ) + tuple(vir), len(occ))
                for (occ, vir) in spaces]
    import multiprocessing
    global _SHARED
    _SHARED = (pb, t1, t2, [(tuple(s[0]), tuple(s[1])) for s in spaces])
    try:
        with multiprocessing.get_context("fork").Pool(workers, initializer=_one_blas_thread) as pool:
            return pool.map(_solve_shared, range(len(spaces)), chunksize=1)
    finally:
        _SHARED = None


def denominators(eps, o):
    """Delta_ia = eps_a - eps_i and Delta_ijab = eps_a + eps_b - eps_i - eps_j
    of the residual step taken by amplitudes no space owns."""
    eo, ev = eps[:o], eps[o:]
    d1 = ev[None, :] - eo[:, None]
    d2 = (ev[None, None, :, None] + ev[None, None, None, :]
          - eo[:, None, None, None] - eo[None, :, None, None])
    return d1, d2


def write_owned(t1, t2, sol, k, occ, vir, owner1, owner2, o):
    """Write the amplitudes space k owns (assignment of each excitation to the
    first space, in Delta-epsilon order, that reaches it) from its local
    cluster amplitudes sol['t1'][I,A], sol['t2'][I,J,A,B] into the pool."""
    for I, i in enumerate(occ):
        for A, a in enumerate(vir):
            if owner1[i, a - o] == k:
                t1[i, a - o] = sol["t1"][I, A]
    for I, i in enumerate(occ):
        for J, j in enumerate(occ):
            for A, a in enumerate(vir):
                for B, b in enumerate(vir):
                    if owner2[i, j, a - o, b - o] == k:
                        t2[i, j, a - o, b - o] = sol["t2"][I, J, A, B]


def mean_energy(E):
    """Unweighted mean of the space energies; NaN when there is no space."""
    return float(np.mean(E)) if len(E) else float("nan")


def flow_step(pb: Problem, t1, t2, spaces, owner1, owner2, unowned="residual", workers=1):
    """One Jacobi macro-iteration.  spaces: list of (occ tuple, vir tuple) of
    absolute spatial orbitals, in Delta-epsilon order.  owner1[i,a] and
    owner2[i,j,a,b] hold the owning space index or -1.  Returns new (t1, t2),
    per-space energies, the mean energy (NaN with no space) and per-space
    solutions.  workers > 1 solves the (independent) spaces in that many
    forked processes."""
    o = pb.o
    sols = solve_spaces(pb, t1, t2, spaces, workers)
    E = np.array([s["E"] for s in sols])
    nt1, nt2 = t1.copy(), t2.copy()
    if unowned == "residual" and (np.any(owner1 < 0) or np.any(owner2 < 0)):
        R1, R2, _ = residual(pb, t1, t2)
        d1, d2 = denominators(pb.eps, o)
        nt1 = np.where(owner1 < 0, t1 - R1 / d1, nt1)
        nt2 = np.where(owner2 < 0, t2 - R2 / d2, nt2)
    for k, (occ, vir) in enumerate(spaces):
        if abs(sols[k]["c0"]) < REF_WEIGHT_MIN:
            continue
        write_owned(nt1, nt2, sols[k], k, occ, vir, owner1, owner2, o)
    return nt1, nt2, E, mean_energy(E), sols


# ----------------------------------------------------------------------------
# DIIS over the amplitude vector (reading R9; the paper itself has none)
# ----------------------------------------------------------------------------

DIIS_MAX_VECTORS = 8
DIIS_START = 3
DIIS_PIVOT_TOL = 1e-14


def _solve_bordered(B, pivot_tol):
    """Solve [B 1; 1^T 0] [c; lam] = [0; 1] by Gaussian elimination with
    partial pivoting.  Returns c, or None when a pivot falls below
    pivot_tol * max|B| (the system is treated as singular)."""
    m = B.shape[0]
    A = np.zeros((m + 1, m + 2))
    A[:m, :m] = B
    A[:m, m] = 1.0
    A[m, :m] = 1.0
    A[m, m + 1] = 1.0
    scale = np.abs(B).max()
    for col in range(m + 1):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if abs(A[piv, col]) < pivot_tol * scale:
            return None
        A[[col, piv]] = A[[piv, col]]
        for r in range(col + 1, m + 1):
            A[r, col:] -= A[r, col] / A[col, col] * A[col, col:]
    x = np.zeros(m + 1)
    for r in range(m, -1, -1):
        x[r] = (A[r, m + 1] - A[r, r + 1:m + 1] @ x[r + 1:]) / A[r, r]
    return x[:m]


class DIIS:
    """Pulay's direct inversion in the iterative subspace on the whole
    amplitude vector.  Each call takes the plainly updated vector t_new and
    its error e = t_new - t_old, keeps the last max_vectors pairs, and from
    the start-th call on returns sum_i c_i t_new_i with the c minimising
    |sum_i c_i e_i| under sum_i c_i = 1 (B_ij = e_i . e_j); when the bordered
    system is singular the oldest pair is dropped and it is solved again."""

    def __init__(self, max_vectors=DIIS_MAX_VECTORS, start=DIIS_START,
                 pivot_tol=DIIS_PIVOT_TOL):
        self.max_vectors, self.start, self.pivot_tol = max_vectors, start, pivot_tol
        self.T, self.E = [], []
        self.calls = 0

    def step(self, t_new, err):
        self.T.append(np.array(t_new, dtype=np.float64))
        self.E.append(np.array(err, dtype=np.float64))
        if len(self.T) > self.max_vectors:
            self.T.pop(0)
            self.E.pop(0)
        self.calls += 1
        if self.calls < self.start:
            return self.T[-1].copy()
        first = 0
        while True:
            Es = self.E[first:]
            m = len(Es)
            if m == 1:
                return self.T[-1].copy()
            B = np.array([[ei @ ej for ej in Es] for ei in Es])
            c = _solve_bordered(B, self.pivot_tol)
            if c is not None:
                return sum(ci * Ti for ci, Ti in zip(c, self.T[first:]))
            first += 1


def pack(t1, t2):
    return np.concatenate([t1.reshape(-1), t2.reshape(-1)])


def unpack(x, o, v):
    return x[:o * v].reshape(o, v).copy(), x[o * v:].reshape(o, o, v, v).copy()


def flow_step_diis(pb: Problem, t1, t2, spaces, owner1, owner2, diis: DIIS,
                   unowned="residual"):
    """One macro-iteration followed by the DIIS extrapolation of the pool."""
    nt1, nt2, E, Em, sols = flow_step(pb, t1, t2, spaces, owner1, owner2, unowned)
    x = diis.step(pack(nt1, nt2), pack(nt1, nt2) - pack(t1, t2))
    xt1, xt2 = unpack(x, pb.o, pb.v)
    return xt1, xt2, E, Em, sols


# ----------------------------------------------------------------------------
# windowed Gauss-Seidel sweep (the paper's process groups taking spaces in
# Delta-epsilon order and updating the pool as they finish)
# ----------------------------------------------------------------------------

def flow_sweep_windowed(pb: Problem, t1, t2, spaces, owner1, owner2, window,
                        unowned="residual"):
    """One sweep over the spaces (Delta-epsilon order) in consecutive windows
    of `window` spaces: each window's spaces are solved with the pool as it
    stands, then their owned amplitudes are written into the pool before the
    next window starts.  The amplitudes no space owns take t <- t - R/Delta
    with R from the pool at the start of the sweep (as in the Jacobi step, so
    a single window reproduces it).  Returns new (t1, t2), per-space energies
    and their mean."""
    o = pb.o
    step_unowned = unowned == "residual" and (np.any(owner1 < 0) or np.any(owner2 < 0))
    if step_unowned:
        R1, R2, _ = residual(pb, t1, t2)
    t1, t2 = t1.copy(), t2.copy()
    E = np.zeros(len(spaces))
    for w0 in range(0, len(spaces), window):
        chunk = list(range(w0, min(w0 + window, len(spaces))))
        sols = {k: solve_space(pb, t1, t2, tuple(spaces[k][0]) + tuple(spaces[k][1]),
                               len(spaces[k][0])) for k in chunk}
        for k in chunk:
            E[k] = sols[k]["E"]
            if abs(sols[k]["c0"]) < REF_WEIGHT_MIN:
                continue
            write_owned(t1, t2, sols[k], k, spaces[k][0], spaces[k][1], owner1, owner2, o)
    if step_unowned:
        d1, d2 = denominators(pb.eps, o)
        t1 = np.where(owner1 < 0, t1 - R1 / d1, t1)
        t2 = np.where(owner2 < 0, t2 - R2 / d2, t2)
    return t1, t2, E, mean_energy(E)
