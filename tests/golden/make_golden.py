"""Write the oracle's expected values for the larger workloads.

    python tests/golden/make_golden.py c2|c3|c4|vqe|vqe_c4 [--workers W]

Calls only ``oracle`` (the plain FP64 CPU implementation) and ``synth`` (the
seeded inputs); nothing here comes from the HIP path.  The active spaces are
Algorithm 1's, capped at K, on the workload's sampling stream; the pool starts
from MP2; every macro-iteration is the Jacobi sweep with the residual step for
amplitudes no space owns.

* c2 (40 orbitals, 5 occupied, K = 256): 30 macro-iterations.  Stores every
  space's energy and the mean per iteration, and the whole pool after the
  first and the last iteration.
* c3 (82 orbitals, 10 occupied, K = 2048): two macro-iterations.  The first is
  taken in full (every space; its energies are stored); the second only for
  16 sampled spaces spread over the Delta-eps order and the orbital range
  (their energies and local cluster amplitudes), plus the pool on a sampled
  block of doubles (occupied x occupied x virtual x virtual) and its singles
  after each iteration.
* c4 (114 orbitals, 13 occupied, K = 4096): the first macro-iteration for 16
  sampled spaces (energies, local cluster amplitudes) and the pool on a
  sampled block after it.  With --full, the whole first iteration is taken
  and the second one is stored for the sampled spaces as for c3.

* vqe (16 and 24 orbitals, 4 occupied; (2,2) and (3,3) spaces of Algorithm
  1): the UCCSD-VQE solver of oracle.vqe.  Two VQE macro-iterations from MP2
  on 16 orbitals (every space's energy, the mean and the whole pool after
  each), and batch solves of the spaces from the pool's own amplitudes
  (16 orbitals) and from zero (24 orbitals) with their energies and
  parameters.
* vqe_c4 (114 orbitals, K = 4096): the first VQE macro-iteration from MP2 on
  four sampled spaces (their energies and optimised parameters).

Sampled spaces: 16 positions evenly spread over the Delta-eps order, the
first replaced where needed so that the sample holds a space with the first
occupied orbital and one with the last virtual orbital.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import qflow, sampling, vqe  # noqa: E402


def workload(name):
    c = synth.CONFIGS[name]
    n, o, K = c["n"], c["o"], c["K"]
    h, eri = synth.config_integrals(name)
    pb = qflow.Problem(h, eri, o)
    S = sampling.algorithm1(o, n - o, 3, 3, pb.eps, synth.sampling_stream(name), cap=K)
    spaces = [(s[0], s[1]) for s in S]
    assert len(spaces) == K
    o1, o2 = sampling.ownership(o, n - o, spaces)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    orbs = np.array([list(a) + list(b) for a, b in spaces], dtype=np.int32)
    return pb, spaces, o1, o2, t1, t2, orbs


def sample_positions(spaces, n, o):
    K = len(spaces)
    pos = [int(round(x)) for x in np.linspace(0, K - 1, 16)]
    want = [lambda s: 0 in s[0], lambda s: (n - 1) in s[1]]
    for m, cond in enumerate(want):
        if not any(cond(spaces[p]) for p in pos):
            k = next(k for k in range(K) if cond(spaces[k]) and k not in pos)
            pos[1 + m] = k
    return np.array(sorted(set(pos)), dtype=np.int32)


def sample_block(o, n):
    occ = np.array(sorted({0, o // 2, o - 1}), dtype=np.int32)
    vir = np.array(sorted({o, o + (n - o) // 3, o + 2 * (n - o) // 3, n - 1}), dtype=np.int32)
    return occ, vir


def block_of(t1, t2, occ, vir, o):
    return (t1[np.ix_(occ, vir - o)].copy(),
            t2[np.ix_(occ, occ, vir - o, vir - o)].copy())


def local_solutions(sols):
    return (np.array([s["E"] for s in sols]), np.array([s["c0"] for s in sols]),
            np.array([s["t1"] for s in sols]), np.array([s["t2"] for s in sols]))


def make_c2(workers):
    pb, spaces, o1, o2, t1, t2, orbs = workload("c2")
    steps = 30
    e_space = np.zeros((steps, len(spaces)))
    e_mean = np.zeros(steps)
    max_dt = np.zeros(steps)
    out = dict(orbs=orbs)
    for it in range(steps):
        t0 = time.time()
        n1, n2, E, Em, _ = qflow.flow_step(pb, t1, t2, spaces, o1, o2, workers=workers)
        max_dt[it] = max(np.abs(n1 - t1).max(), np.abs(n2 - t2).max())
        t1, t2 = n1, n2
        e_space[it], e_mean[it] = E, Em
        if it == 0:
            out.update(t1_first=t1.copy(), t2_first=t2.copy())
        print(f"c2 step {it}: E_mean {Em:.12f} max|dt| {max_dt[it]:.3e} "
              f"({time.time() - t0:.1f} s)", flush=True)
    out.update(e_space=e_space, e_mean=e_mean, max_dt=max_dt, t1_last=t1, t2_last=t2)
    np.savez_compressed(os.path.join(HERE, "qflow_c2_trajectory.npz"), **out)


def make_two_steps(name, workers, full):
    pb, spaces, o1, o2, t1, t2, orbs = workload(name)
    o, n = pb.o, pb.n
    samp = sample_positions(spaces, n, o)
    bocc, bvir = sample_block(o, n)
    sampled = [spaces[k] for k in samp]
    out = dict(orbs=orbs, samp=samp, block_occ=bocc, block_vir=bvir)
    t0 = time.time()
    if full:
        n1, n2, E, Em, sols = qflow.flow_step(pb, t1, t2, spaces, o1, o2, workers=workers)
        out.update(e_space_1=E, e_mean_1=Em)
        s1 = [sols[k] for k in samp]
    else:
        s1 = qflow.solve_spaces(pb, t1, t2, sampled, workers)
        n1 = n2 = None
    e, c0, lt1, lt2 = local_solutions(s1)
    out.update(e_samp_1=e, c0_samp_1=c0, t1_samp_1=lt1, t2_samp_1=lt2)
    # the pool on the sampled block after the first iteration: owned entries
    # from their owner's solution (the owner may lie outside the sample, so the
    # full step is needed), unowned ones by the residual step
    R1, R2, _ = qflow.residual(pb, t1, t2, occ=bocc, vir=bvir)
    d1, d2 = qflow.denominators(pb.eps, o)
    b1, b2 = block_of(t1, t2, bocc, bvir, o)
    db1, db2 = d1[np.ix_(bocc, bvir - o)], d2[np.ix_(bocc, bocc, bvir - o, bvir - o)]
    un1 = o1[np.ix_(bocc, bvir - o)] < 0
    un2 = o2[np.ix_(bocc, bocc, bvir - o, bvir - o)] < 0
    out.update(block_unowned1_1=un1, block_unowned2_1=un2,
               block_t1_step_1=np.where(un1, b1 - R1 / db1, np.nan),
               block_t2_step_1=np.where(un2, b2 - R2 / db2, np.nan))
    print(f"{name} step 0 done ({time.time() - t0:.1f} s)", flush=True)
    if full:
        f1, f2 = block_of(n1, n2, bocc, bvir, o)
        out.update(block_t1_1=f1, block_t2_1=f2)
        t0 = time.time()
        s2 = qflow.solve_spaces(pb, n1, n2, sampled, workers)
        e, c0, lt1, lt2 = local_solutions(s2)
        out.update(e_samp_2=e, c0_samp_2=c0, t1_samp_2=lt1, t2_samp_2=lt2)
        R1, R2, _ = qflow.residual(pb, n1, n2, occ=bocc, vir=bvir)
        out.update(block_t1_step_2=np.where(un1, f1 - R1 / db1, np.nan),
                   block_t2_step_2=np.where(un2, f2 - R2 / db2, np.nan))
        print(f"{name} step 1 (sampled) done ({time.time() - t0:.1f} s)", flush=True)
    tag = "two_steps" if full else "first_step"
    np.savez_compressed(os.path.join(HERE, f"qflow_{name}_{tag}.npz"), **out)


# (n, o, seed, caps of the (2,2) and (3,3) classes)
VQE_FLOW = (16, 4, 731, (5, 2))
VQE_SOLVE_POOL = (16, 4, 711, (5, 2))
VQE_SOLVE_ZERO = (24, 4, 712, (4, 2))


def vqe_inputs(n, o, seed, caps):
    """Integrals (the stress recipe), the problem, the MP2 pool and the
    spaces: Algorithm 1 per size class on its own stream, merged in Delta-eps
    order."""
    h, eri = synth.gen_integrals(n, o, 2 * n, seed, b_std=0.04, off_std=0.03)
    pb = qflow.Problem(h, eri, o)
    out = []
    for size, cap in zip((2, 3), caps):
        S = sampling.algorithm1(o, n - o, size, size, pb.eps, synth.Stream(seed + size), cap=cap)
        out += [(tuple(s[0]), tuple(s[1]), s[2]) for s in S]
    out.sort(key=lambda s: s[2])
    spaces = [(s[0], s[1]) for s in out]
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    return pb, spaces, t1, t2


def local_amplitudes(t1, t2, occ, vir, o):
    vv = [a - o for a in vir]
    return np.concatenate([t1[np.ix_(occ, vv)].ravel(), t2[np.ix_(occ, occ, vv, vv)].ravel()])


def make_vqe():
    out = {}
    pb, spaces, t1, t2 = vqe_inputs(*VQE_FLOW)
    o, v = pb.o, pb.n - pb.o
    o1, o2 = sampling.ownership(o, v, spaces)
    for it in range(2):
        t0 = time.time()
        t1, t2, E, Em, _ = vqe.flow_step(pb, t1, t2, spaces, o1, o2)
        out.update({f"flow_e_{it}": E, f"flow_mean_{it}": Em, f"flow_t1_{it}": t1,
                    f"flow_t2_{it}": t2})
        print(f"vqe flow step {it}: E_mean {Em:.12f} ({time.time() - t0:.1f} s)", flush=True)
    for tag, case in (("pool", VQE_SOLVE_POOL), ("zero", VQE_SOLVE_ZERO)):
        t0 = time.time()
        pb, spaces, t1, t2 = vqe_inputs(*case)
        E, amp = [], []
        for occ, vir in spaces:
            no, nv = len(occ), len(vir)
            H = qflow.cas_matrix(*qflow.heff(pb, t1, t2, tuple(occ) + tuple(vir)), no)
            th0 = None
            if tag == "pool":
                lt = local_amplitudes(t1, t2, occ, vir, pb.o)
                th0 = vqe.pack(lt[:no * nv].reshape(no, nv), lt[no * nv:].reshape(no, no, nv, nv),
                               no, nv)
            s = vqe.solve(H, no, nv, theta0=th0)
            E.append(s["E"])
            amp.append(np.concatenate([s["t1"].ravel(), s["t2"].ravel()]))
        out.update({f"solve_{tag}_e": np.array(E), f"solve_{tag}_amp": np.concatenate(amp)})
        print(f"vqe solves ({tag}) done ({time.time() - t0:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "qflow_vqe.npz"), **out)


def make_vqe_c4(workers):
    """The 114-orbital workload's first VQE macro-iteration from MP2 on four
    sampled spaces (first, last, and two spread over the Delta-eps order, one
    holding orbital 113): their VQE energies and optimised parameters."""
    pb, spaces, o1, o2, t1, t2, orbs = workload("c4")
    n, o, K = pb.n, pb.o, len(spaces)
    pos = [0, K // 3, 2 * K // 3, K - 1]
    if not any((n - 1) in spaces[k][1] for k in pos):
        pos[2] = next(k for k in range(K) if (n - 1) in spaces[k][1] and k not in pos)
    pos = sorted(set(pos))
    t0 = time.time()
    E, amp = [], []
    for k in pos:
        occ, vir = spaces[k]
        sol = vqe.solve_space(pb, t1, t2, tuple(occ) + tuple(vir), len(occ))
        E.append(sol["E"])
        amp.append(np.concatenate([sol["t1"].ravel(), sol["t2"].ravel()]))
        print(f"c4 vqe space {k}: E {sol['E']:.12f} ({time.time() - t0:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "qflow_c4_vqe_first_step.npz"), orbs=orbs,
                        samp=np.array(pos, dtype=np.int32), e_samp=np.array(E),
                        amp_samp=np.array(amp))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c2", "c3", "c4", "vqe", "vqe_c4"])
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--full", action="store_true",
                    help="c4: take the whole first iteration and the sampled second")
    a = ap.parse_args()
    if a.config == "c2":
        make_c2(a.workers)
    elif a.config == "vqe":
        make_vqe()
    elif a.config == "vqe_c4":
        make_vqe_c4(a.workers)
    elif a.config == "c3":
        make_two_steps("c3", a.workers, True)
    else:
        make_two_steps("c4", a.workers, a.full)


if __name__ == "__main__":
    main()
