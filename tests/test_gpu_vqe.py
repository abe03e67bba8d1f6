"""UCCSD-VQE solver of the HIP path (qflow_solve_vqe_batch and flow steps with
QFLOW_SOLVER_VQE) against the oracle's (oracle/vqe.py), through the C ABI.

Both sides minimise the same FP64 energy until the largest gradient entry is
below 1e-10 Eh, by different routes (BFGS with quadrature gradients here;
BFGS and Newton steps with the exact Frechet derivative in the oracle), so
energies agree to 1e-10 Eh and parameters to 1e-7: the gradient bound over
the energy's smallest curvature (of the order of the smallest excitation
energy of the space, 0.1 Eh and more on these problems), with room for the
rounding of the steps.  At a fixed parameter vector (max_iter = 0) the two
energies differ only by rounding: 1e-12 Eh.  The oracle's (3,3) solves take
tens of seconds each, so their results are stored (tests/golden/qflow_vqe.npz,
written by tests/golden/make_golden.py from the oracle alone); the (2,2)
solves, and the oracle's energy and exact gradient at the parameters found
here, are computed live.
"""
import os

import numpy as np
import pytest

import synth
from oracle import qflow, sampling, vqe
from oracle.cas import basis

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_E, TOL_T = 1e-10, 1e-7


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def _problem(n, o, seed):
    h, eri = synth.gen_integrals(n, o, 2 * n, seed, b_std=0.04, off_std=0.03)
    return h, eri, qflow.Problem(h, eri, o)


def _context(h, eri, o):
    import paper_2606_04186_amd as qf
    ctx = qf.Context(0)
    ctx.load_integrals(dev(h), dev(eri), o)
    return ctx


def _spaces(o, v, eps, seed, caps):
    """(2,2) and (3,3) spaces of Algorithm 1, sorted by Delta eps."""
    out = []
    for size, cap in zip((2, 3), caps):
        if cap == 0:
            continue
        S = sampling.algorithm1(o, v, size, size, eps, synth.Stream(seed + size), cap=cap)
        out += [(tuple(s[0]), tuple(s[1]), s[2]) for s in S]
    out.sort(key=lambda s: s[2])
    return [(s[0], s[1]) for s in out]


def _local(t1, t2, occ, vir, o):
    """The pool's amplitudes of one space in the amp layout."""
    vv = [a - o for a in vir]
    lt1 = t1[np.ix_(occ, vv)]
    lt2 = t2[np.ix_(occ, occ, vv, vv)]
    return np.concatenate([lt1.ravel(), lt2.ravel()])


def _amp_len(lists):
    return sum(len(a) * len(b) * (1 + len(a) * len(b)) for a, b in lists)


def _batch(ctx, lists, t1, t2, o, theta0, gtol=1e-10, max_iter=500):
    import paper_2606_04186_amd as qf
    sp = qf.make_spaces(lists)
    hoff = qf.api.offsets(sp, qf.heff_size)
    aoff = qf.api.offsets(sp, qf.amp_size)
    K = len(lists)
    heff = torch.zeros(int(hoff[-1]), dtype=torch.float64, device="cuda")
    ctx.build_heff(sp, dev(t1), dev(t2), heff, hoff)
    th = dev(theta0)
    amp = torch.zeros_like(th)
    energy = torch.zeros(K, dtype=torch.float64, device="cuda")
    iters = torch.zeros(K, dtype=torch.int32, device="cuda")
    status = torch.zeros(K, dtype=torch.int32, device="cuda")
    ctx.solve_vqe_batch(sp, heff, hoff, th, amp, aoff, energy, iters, status, gtol, max_iter)
    torch.cuda.synchronize()
    return aoff, host(energy), host(amp), host(iters), host(status)


def test_vqe_energy_at_the_start_matches_oracle():
    """max_iter = 0 evaluates E(theta0) only: the exponential, the CAS
    product and the parameter layout, without the minimiser."""
    _need_gpu()
    n, o, seed = 16, 4, 701
    h, eri, pb = _problem(n, o, seed)
    t1, t2 = synth.random_amplitudes(o, n - o, seed + 1, scale=0.08)
    lists = _spaces(o, n - o, pb.eps, seed, (4, 3))
    theta0 = np.concatenate([_local(t1, t2, occ, vir, o) for occ, vir in lists])
    ctx = _context(h, eri, o)
    aoff, E, A, it, st = _batch(ctx, lists, t1, t2, o, theta0, max_iter=0)
    for k, (occ, vir) in enumerate(lists):
        no, nv = len(occ), len(vir)
        H = qflow.cas_matrix(*qflow.heff(pb, t1, t2, tuple(occ) + tuple(vir)), no)
        lt = theta0[aoff[k]:aoff[k + 1]]
        th = vqe.pack(lt[:no * nv].reshape(no, nv), lt[no * nv:].reshape(no, no, nv, nv), no, nv)
        e = vqe.energy(th, H, vqe.generators(no, nv), basis(no, no + nv).iref)
        assert abs(E[k] - e) < 1e-12, k
        assert st[k] == -5 and it[k] == 0
        u1, u2 = vqe.unpack(th, no, nv)
        blk = A[aoff[k]:aoff[k + 1]]
        assert np.abs(blk - np.concatenate([u1.ravel(), u2.ravel()])).max() == 0.0, k


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "qflow_vqe.npz")
# (n, o, seed, caps) of the stored oracle runs (tests/golden/make_golden.py vqe)
VQE_FLOW = (16, 4, 731, (5, 2))
VQE_SOLVE = {"pool": (16, 4, 711, (5, 2)), "zero": (24, 4, 712, (4, 2))}


def _stationary(H, no, nv, blk, e_gpu):
    """The oracle's energy and exact gradient at the HIP path's parameters."""
    th = vqe.pack(blk[:no * nv].reshape(no, nv), blk[no * nv:].reshape(no, no, nv, nv), no, nv)
    e, g = vqe.energy_gradient(th, H, vqe.generators(no, nv), basis(no, no + nv).iref)
    assert abs(e - e_gpu) < 1e-12
    assert np.abs(g).max() < 1e-9


@pytest.mark.parametrize("start", ["pool", "zero"])
def test_vqe_solve_matches_oracle(start):
    """Every space against the stored oracle solution; at the parameters
    found here, the oracle's energy and exact gradient (a stationary point of
    the oracle's energy); the (2,2) spaces are also solved live."""
    _need_gpu()
    n, o, seed, caps = VQE_SOLVE[start]
    h, eri, pb = _problem(n, o, seed)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    lists = _spaces(o, n - o, pb.eps, seed, caps)
    if start == "pool":
        theta0 = np.concatenate([_local(t1, t2, occ, vir, o) for occ, vir in lists])
    else:
        theta0 = np.zeros(_amp_len(lists))
    ctx = _context(h, eri, o)
    aoff, E, A, it, st = _batch(ctx, lists, t1, t2, o, theta0)
    gold = np.load(GOLDEN)
    ge, ga = gold[f"solve_{start}_e"], gold[f"solve_{start}_amp"]
    assert len(ge) == len(lists) and len(ga) == len(A)
    assert np.all(st == 0), it
    assert np.abs(E - ge).max() < TOL_E
    assert np.abs(A - ga).max() < TOL_T
    for k, (occ, vir) in enumerate(lists):
        no, nv = len(occ), len(vir)
        H = qflow.cas_matrix(*qflow.heff(pb, t1, t2, tuple(occ) + tuple(vir)), no)
        blk = A[aoff[k]:aoff[k + 1]]
        _stationary(H, no, nv, blk, E[k])
        if no == 2:
            lt = theta0[aoff[k]:aoff[k + 1]]
            th0 = vqe.pack(lt[:4].reshape(2, 2), lt[4:].reshape(2, 2, 2, 2), 2, 2)
            s = vqe.solve(H, 2, 2, theta0=th0)
            assert abs(E[k] - s["E"]) < TOL_E, k
            assert np.abs(blk - np.concatenate([s["t1"].ravel(), s["t2"].ravel()])).max() < TOL_T


def test_vqe_not_converged_status():
    """One BFGS iteration does not reach the gradient bound: status -5."""
    _need_gpu()
    n, o, seed = 16, 4, 721
    h, eri, pb = _problem(n, o, seed)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    lists = _spaces(o, n - o, pb.eps, seed, (3, 1))
    theta0 = np.zeros(_amp_len(lists))
    ctx = _context(h, eri, o)
    _, E, _, it, st = _batch(ctx, lists, t1, t2, o, theta0, max_iter=1)
    assert np.all(st == -5) and np.all(it == 1)


def _flow(n, o, seed, caps, steps, flags_extra=0):
    import paper_2606_04186_amd as qf
    h, eri, pb = _problem(n, o, seed)
    v = n - o
    lists = _spaces(o, v, pb.eps, seed, caps)
    o1, o2 = sampling.ownership(o, v, lists)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    sp = qf.make_spaces(lists)
    ctx = _context(h, eri, o)
    g1, g2 = dev(t1), dev(t2)
    energy = torch.zeros(len(lists), dtype=torch.float64, device="cuda")
    d1, d2 = dev(o1, torch.int32), dev(o2, torch.int32)
    out = []
    for _ in range(steps):
        em, _md = ctx.flow_step(sp, d1, d2, g1, g2, energy, qf.SOLVER_VQE | flags_extra)
        out.append((em, host(energy).copy(), host(g1).copy(), host(g2).copy(),
                    ctx.last_solve(len(lists))[1]))
    return pb, lists, o1, o2, t1, t2, out


def test_vqe_flow_steps_match_oracle():
    """Two Jacobi macro-iterations with the VQE solver on a partly covered
    pool (unowned amplitudes take the residual step), against the stored
    oracle run; the first step's pool is also checked live for the
    amplitudes no space owns (residual step) and those of (2,2) owners."""
    _need_gpu()
    pb, lists, o1, o2, t1, t2, out = _flow(*VQE_FLOW, 2)
    gold = np.load(GOLDEN)
    for step, (em, E, g1, g2, st) in enumerate(out):
        assert np.all(st == 0), step
        assert abs(em - float(gold[f"flow_mean_{step}"])) < TOL_E, step
        assert np.abs(E - gold[f"flow_e_{step}"]).max() < TOL_E, step
        assert np.abs(g1 - gold[f"flow_t1_{step}"]).max() < TOL_T, step
        assert np.abs(g2 - gold[f"flow_t2_{step}"]).max() < TOL_T, step
    # live: the residual step of the unowned amplitudes after the first step
    R1, R2, _ = qflow.residual(pb, t1, t2)
    d1, d2 = qflow.denominators(pb.eps, pb.o)
    em, E, g1, g2, st = out[0]
    assert np.abs(np.where(o1 < 0, g1 - (t1 - R1 / d1), 0.0)).max() < 1e-11
    assert np.abs(np.where(o2 < 0, g2 - (t2 - R2 / d2), 0.0)).max() < 1e-11


def test_vqe_flow_graph_replays_equal_eager():
    import paper_2606_04186_amd as qf
    _need_gpu()
    *_, eager = _flow(16, 4, 741, (4, 1), 3)
    *_, graph = _flow(16, 4, 741, (4, 1), 3, qf.GRAPH)
    assert all(np.all(a[4] == 0) for a in eager)
    for a, b in zip(eager, graph):
        assert a[0] == b[0]
        for x, y in zip(a[1:], b[1:]):
            assert np.array_equal(x, y)


def test_vqe_rejects_unsupported_spaces_and_flags():
    import paper_2606_04186_amd as qf
    _need_gpu()
    n, o = 16, 4
    h, eri, pb = _problem(n, o, 751)
    ctx = _context(h, eri, o)
    lists = [((0, 1, 2, 3), (4, 5, 6, 7))]
    sp = qf.make_spaces(lists)
    hoff = qf.api.offsets(sp, qf.heff_size)
    aoff = qf.api.offsets(sp, qf.amp_size)
    heff = torch.zeros(int(hoff[-1]), dtype=torch.float64, device="cuda")
    th = torch.zeros(int(aoff[-1]), dtype=torch.float64, device="cuda")
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    ione = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(qf.QFlowError) as e:
        ctx.solve_vqe_batch(sp, heff, hoff, th, th, aoff, one, ione, ione)
    assert e.value.code == -8
    v = n - o
    o1, o2 = sampling.ownership(o, v, lists)
    t1, t2 = dev(np.zeros((o, v))), dev(np.zeros((o, o, v, v)))
    d1, d2 = dev(o1, torch.int32), dev(o2, torch.int32)
    with pytest.raises(qf.QFlowError) as e:
        ctx.flow_step(sp, d1, d2, t1, t2, one, qf.SOLVER_VQE)
    assert e.value.code == -8
    ok = qf.make_spaces([((0, 1), (4, 5))])
    with pytest.raises(qf.QFlowError) as e:
        ctx.flow_sweep_windowed(ok, d1, d2, t1, t2, one, 1, qf.SOLVER_VQE)
    assert e.value.code == -8
    with pytest.raises(qf.QFlowError) as e:
        ctx.set_vqe(0.0, 10)
    assert e.value.code == -1
