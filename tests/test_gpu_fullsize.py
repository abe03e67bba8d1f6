"""The 114-orbital workload at full size, in the configuration bench.py
times (K = 4096 (3,3) spaces from Algorithm 1, MP2 start; BF16x3 contractions
replayed as a captured graph, and plain FP64), checked on sampled outputs the
oracle computes one by one: the energy and the owned amplitudes of sampled
spaces (first and last in Delta-eps order), and residual steps of sampled
unowned doubles.

Tolerances: FP64 as in test_gpu_parity (energies 1e-9 Eh, amplitudes 1e-8);
BF16x3 at the mixed-precision target (per-space energies 1e-6 Eh, amplitudes
1e-6, residual steps 1e-4 of the largest sampled step: about 2^-16 per
product).
"""
import numpy as np
import pytest

import synth
from oracle import qflow

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.timeout(600)
def test_full_size_flow_step_sampled_against_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_04186_amd as qf
    cfg = synth.CONFIGS["c4"]
    n, o, K = cfg["n"], cfg["o"], cfg["K"]
    v = n - o
    h, eri = synth.config_integrals("c4")
    dev = torch.device("cuda:0")
    dh, deri = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    ctx_b, ctx_f = qf.Context(0), qf.Context(0)
    ctx_b.load_integrals(dh, deri, o)
    ctx_f.load_integrals(dh, deri, o)
    del dh, deri
    _, eps, _ = ctx_b.reference()
    u = synth.sampling_stream("c4", 0).uniform(64 * K)
    spaces, _, _ = qf.sample_spaces(o, v, 3, 3, eps, u, cap=K)
    assert len(spaces) == K
    o1, o2 = qf.build_owners(o, v, spaces)
    d1, d2 = torch.from_numpy(o1).to(dev), torch.from_numpy(o2).to(dev)
    t1 = torch.zeros(o, v, dtype=torch.float64, device=dev)
    t2 = torch.zeros(o, o, v, v, dtype=torch.float64, device=dev)
    ctx_b.mp2_guess(t1, t2)
    t1h, t2h = t1.cpu().numpy().copy(), t2.cpu().numpy().copy()
    b1, b2, f1, f2 = t1.clone(), t2.clone(), t1.clone(), t2.clone()
    eb = torch.zeros(K, dtype=torch.float64, device=dev)
    ef = torch.zeros(K, dtype=torch.float64, device=dev)
    em_b, _ = ctx_b.flow_step(spaces, d1, d2, b1, b2, eb, qf.BF16X3 | qf.GRAPH)
    em_f, _ = ctx_f.flow_step(spaces, d1, d2, f1, f2, ef, qf.FP64)
    Eb, Ef = eb.cpu().numpy(), ef.cpu().numpy()
    B1, B2, F1, F2 = (x.cpu().numpy() for x in (b1, b2, f1, f2))
    assert abs(em_b - Eb.mean()) < 1e-12 and abs(em_f - Ef.mean()) < 1e-12
    assert np.abs(Eb - Ef).max() < 1e-6

    pb = qflow.Problem(h, eri, o)
    assert np.abs(t1h - qflow.mp2_guess(pb.f, eri, o)[0]).max() < 1e-12
    for k in (0, K - 1):
        s = spaces[k]
        occ = [int(x) for x in s["orb"][:3]]
        vir = [int(x) for x in s["orb"][3:6]]
        sol = qflow.solve_space(pb, t1h, t2h, tuple(occ) + tuple(vir), 3)
        print(f"space {k}: E oracle {sol['E']:.12f} FP64 {Ef[k]:.12f} BF16x3 {Eb[k]:.12f}")
        assert abs(Ef[k] - sol["E"]) < 1e-9
        assert abs(Eb[k] - sol["E"]) < 1e-6
        owned = 0
        for I, i in enumerate(occ):
            for A, a in enumerate(vir):
                if o1[i, a - o] == k:
                    owned += 1
                    assert abs(F1[i, a - o] - sol["t1"][I, A]) < 1e-8
                    assert abs(B1[i, a - o] - sol["t1"][I, A]) < 1e-6
        for I, i in enumerate(occ):
            for J, j in enumerate(occ):
                for A, a in enumerate(vir):
                    for Bv, b in enumerate(vir):
                        if o2[i, j, a - o, b - o] == k:
                            owned += 1
                            ref = sol["t2"][I, J, A, Bv]
                            assert abs(F2[i, j, a - o, b - o] - ref) < 1e-8
                            assert abs(B2[i, j, a - o, b - o] - ref) < 1e-6
        print(f"space {k}: {owned} owned amplitudes checked")
    # unowned doubles: t <- t - R/Delta, R from the oracle on a sub-block
    occ_s, vir_s = [3, 11], [o + 7, o + 64, o + 100]
    R1, R2, _ = qflow.residual(pb, t1h, t2h, occ=occ_s, vir=vir_s)
    e = pb.eps
    rows = []
    for I, i in enumerate(occ_s):
        for J, j in enumerate(occ_s):
            for A, a in enumerate(vir_s):
                for Bv, b in enumerate(vir_s):
                    if o2[i, j, a - o, b - o] < 0:
                        step = R2[I, J, A, Bv] / (e[a] + e[b] - e[i] - e[j])
                        rows.append((i, j, a - o, b - o, t2h[i, j, a - o, b - o] - step, step))
    assert rows
    scale = max(abs(r[5]) for r in rows)
    for i, j, a, b, ref, _ in rows:
        assert abs(F2[i, j, a, b] - ref) < 1e-10
        assert abs(B2[i, j, a, b] - ref) < 1e-4 * scale
    print(f"{len(rows)} unowned doubles checked (largest step {scale:.3e})")


@pytest.mark.timeout(900)
def test_full_size_mixed_classes_sampled_against_oracle():
    """The mixed 114-orbital workload at full size (2048 spaces each of
    (2,2), (3,3) and (4,4) from per-class Algorithm 1 streams, merged in
    Delta-eps order; BF16x3 graph and FP64): per-space energies and owned
    amplitudes of the first space of each size class against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_04186_amd as qf
    cfg = synth.CONFIGS["c5"]
    n, o, K = cfg["n"], cfg["o"], cfg["K"]
    v = n - o
    h, eri = synth.config_integrals("c5")
    dev = torch.device("cuda:0")
    dh, deri = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    ctx_b, ctx_f = qf.Context(0), qf.Context(0)
    ctx_b.load_integrals(dh, deri, o)
    ctx_f.load_integrals(dh, deri, o)
    del dh, deri
    _, eps, _ = ctx_b.reference()
    parts, deltas = [], []
    Kc = K // len(cfg["sizes"])
    for c, (no_c, nv_c) in enumerate(cfg["sizes"]):
        u = synth.sampling_stream("c5", c).uniform(64 * Kc)
        sp_c, de_c, _ = qf.sample_spaces(o, v, no_c, nv_c, eps, u, cap=Kc)
        assert len(sp_c) == Kc
        parts.append(sp_c)
        deltas.append(de_c)
    order = np.argsort(np.concatenate(deltas), kind="stable")
    spaces = np.concatenate(parts)[order]
    o1, o2 = qf.build_owners(o, v, spaces)
    d1, d2 = torch.from_numpy(o1).to(dev), torch.from_numpy(o2).to(dev)
    t1 = torch.zeros(o, v, dtype=torch.float64, device=dev)
    t2 = torch.zeros(o, o, v, v, dtype=torch.float64, device=dev)
    ctx_b.mp2_guess(t1, t2)
    t1h, t2h = t1.cpu().numpy().copy(), t2.cpu().numpy().copy()
    b1, b2, f1, f2 = t1.clone(), t2.clone(), t1.clone(), t2.clone()
    eb = torch.zeros(K, dtype=torch.float64, device=dev)
    ef = torch.zeros(K, dtype=torch.float64, device=dev)
    ctx_b.flow_step(spaces, d1, d2, b1, b2, eb, qf.BF16X3 | qf.GRAPH)
    ctx_f.flow_step(spaces, d1, d2, f1, f2, ef, qf.FP64)
    Eb, Ef = eb.cpu().numpy(), ef.cpu().numpy()
    B1, B2, F1, F2 = (x.cpu().numpy() for x in (b1, b2, f1, f2))
    assert np.abs(Eb - Ef).max() < 1e-6
    pb = qflow.Problem(h, eri, o)
    for size in (2, 3, 4):
        k = int(np.nonzero(spaces["n_o"] == size)[0][0])
        s = spaces[k]
        occ = [int(x) for x in s["orb"][:size]]
        vir = [int(x) for x in s["orb"][size:2 * size]]
        sol = qflow.solve_space(pb, t1h, t2h, tuple(occ) + tuple(vir), size)
        print(f"({size},{size}) space {k}: E oracle {sol['E']:.12f} FP64 {Ef[k]:.12f} "
              f"BF16x3 {Eb[k]:.12f}")
        assert abs(Ef[k] - sol["E"]) < 1e-9
        assert abs(Eb[k] - sol["E"]) < 1e-6
        owned = 0
        for I, i in enumerate(occ):
            for A, a in enumerate(vir):
                if o1[i, a - o] == k:
                    owned += 1
                    assert abs(F1[i, a - o] - sol["t1"][I, A]) < 1e-8
                    assert abs(B1[i, a - o] - sol["t1"][I, A]) < 1e-6
        for I, i in enumerate(occ):
            for J, j in enumerate(occ):
                for A, a in enumerate(vir):
                    for Bv, b in enumerate(vir):
                        if o2[i, j, a - o, b - o] == k:
                            owned += 1
                            ref = sol["t2"][I, J, A, Bv]
                            assert abs(F2[i, j, a - o, b - o] - ref) < 1e-8
                            assert abs(B2[i, j, a - o, b - o] - ref) < 1e-6
        print(f"({size},{size}) space {k}: {owned} owned amplitudes checked")


def _full_cycle(qf, o, v, eps, name):
    nu = 1 << 22
    while True:
        u = synth.sampling_stream(name, 0).uniform(nu)
        try:
            return qf.sample_spaces(o, v, 3, 3, eps, u, cap=0, max_out=nu)[0]
        except qf.QFlowError:
            nu *= 4


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,size", [("c6", 10319), ("c7", 56860)])
def test_full_cycle_at_paper_shapes_sampled_against_oracle(name, size):
    """A full Algorithm 1 cycle at the shapes of the paper's largest
    workloads (4 + 110 orbitals, about 10.3k spaces; 13 + 69, about 56.9k):
    every amplitude is owned, so the pool update is the paper's pure
    owned-amplitude rule.  The first and last spaces' energies and owned
    amplitudes (FP64, and BF16x3 as a captured graph) against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_04186_amd as qf
    cfg = synth.CONFIGS[name]
    n, o = cfg["n"], cfg["o"]
    v = n - o
    h, eri = synth.config_integrals(name)
    dev = torch.device("cuda:0")
    dh, deri = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    ctx_b, ctx_f = qf.Context(0), qf.Context(0)
    ctx_b.load_integrals(dh, deri, o)
    ctx_f.load_integrals(dh, deri, o)
    del dh, deri
    _, eps, _ = ctx_b.reference()
    spaces = _full_cycle(qf, o, v, eps, name)
    K = len(spaces)
    assert abs(K - size) / size < 0.05
    o1, o2 = qf.build_owners(o, v, spaces)
    assert (o1 >= 0).all() and (o2 >= 0).all()
    d1, d2 = torch.from_numpy(o1).to(dev), torch.from_numpy(o2).to(dev)
    t1 = torch.zeros(o, v, dtype=torch.float64, device=dev)
    t2 = torch.zeros(o, o, v, v, dtype=torch.float64, device=dev)
    ctx_b.mp2_guess(t1, t2)
    t1h, t2h = t1.cpu().numpy().copy(), t2.cpu().numpy().copy()
    b1, b2, f1, f2 = t1.clone(), t2.clone(), t1.clone(), t2.clone()
    eb = torch.zeros(K, dtype=torch.float64, device=dev)
    ef = torch.zeros(K, dtype=torch.float64, device=dev)
    ctx_b.flow_step(spaces, d1, d2, b1, b2, eb, qf.BF16X3 | qf.GRAPH)
    ctx_f.flow_step(spaces, d1, d2, f1, f2, ef, qf.FP64)
    Eb, Ef = eb.cpu().numpy(), ef.cpu().numpy()
    B1, B2, F1, F2 = (x.cpu().numpy() for x in (b1, b2, f1, f2))
    assert np.abs(Eb - Ef).max() < 1e-6
    pb = qflow.Problem(h, eri, o)
    for k in (0, K - 1):
        s = spaces[k]
        occ = [int(x) for x in s["orb"][:3]]
        vir = [int(x) for x in s["orb"][3:6]]
        sol = qflow.solve_space(pb, t1h, t2h, tuple(occ) + tuple(vir), 3)
        print(f"{name} space {k} of {K}: E oracle {sol['E']:.12f} FP64 {Ef[k]:.12f} "
              f"BF16x3 {Eb[k]:.12f}")
        assert abs(Ef[k] - sol["E"]) < 1e-9
        assert abs(Eb[k] - sol["E"]) < 1e-6
        for I, i in enumerate(occ):
            for A, a in enumerate(vir):
                if o1[i, a - o] == k:
                    assert abs(F1[i, a - o] - sol["t1"][I, A]) < 1e-8
                    assert abs(B1[i, a - o] - sol["t1"][I, A]) < 1e-6
        for I, i in enumerate(occ):
            for J, j in enumerate(occ):
                for A, a in enumerate(vir):
                    for Bv, b in enumerate(vir):
                        if o2[i, j, a - o, b - o] == k:
                            ref = sol["t2"][I, J, A, Bv]
                            assert abs(F2[i, j, a - o, b - o] - ref) < 1e-8
                            assert abs(B2[i, j, a - o, b - o] - ref) < 1e-6
