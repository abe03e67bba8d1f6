"""The autotuner and the launch choices it sets: every choice gives the same
flow step (to the summation-order rounding of split products), the tuner's
result is one of its candidates, it is written to the JSON cache and applied
from there without timing."""
import itertools
import json

import numpy as np
import pytest

import synth
from oracle import qflow, sampling

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mixed(n, o, seed, eps, caps):
    out = []
    for size, cap in zip((2, 3, 4), caps):
        S = sampling.algorithm1(o, n - o, size, size, eps, synth.Stream(seed + size), cap=cap)
        out += [(tuple(s[0]), tuple(s[1]), s[2]) for s in S]
    out.sort(key=lambda s: s[2])
    return [(s[0], s[1]) for s in out]


def _setup(n=24, o=5, seed=191, caps=(6, 8, 2)):
    import paper_2606_04186_amd as qf
    h, eri = synth.gen_integrals(n, o, 2 * n, seed, b_std=0.04, off_std=0.03)
    pb = qflow.Problem(h, eri, o)
    lists = _mixed(n, o, seed, pb.eps, caps)
    o1, o2 = sampling.ownership(o, n - o, lists)
    t1, t2 = qflow.mp2_guess(pb.f, eri, o)
    ctx = qf.Context(0)
    ctx.load_integrals(torch.from_numpy(h).cuda(), torch.from_numpy(eri).cuda(), o)
    d = dict(sp=qf.make_spaces(lists), o1=torch.from_numpy(o1).cuda(),
             o2=torch.from_numpy(o2).cuda(), t1=t1, t2=t2, pb=pb, lists=lists, o=o)
    return qf, ctx, d


def _step(ctx, d, flags):
    g1, g2 = torch.from_numpy(d["t1"]).cuda(), torch.from_numpy(d["t2"]).cuda()
    e = torch.zeros(len(d["sp"]), dtype=torch.float64, device="cuda")
    em, _ = ctx.flow_step(d["sp"], d["o1"], d["o2"], g1, g2, e, flags)
    return em, e.cpu().numpy(), g1.cpu().numpy(), g2.cpu().numpy()


@pytest.mark.timeout(300)
def test_every_launch_choice_gives_the_same_step():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qf, ctx, d = _setup()
    ref = _step(ctx, d, qf.FP64)
    n1, n2, E, Em, _ = qflow.flow_step(d["pb"], d["t1"], d["t2"], d["lists"],
                                       d["o1"].cpu().numpy(), d["o2"].cpu().numpy())
    assert abs(ref[0] - Em) < 1e-9 and np.abs(ref[2] - n1).max() < 1e-8
    for dav, split, tile, z, blk in itertools.product(
            (qf.api.DAV_PER_CLASS, qf.api.DAV_PERSISTENT), (1, 8, 16), (0, 1, 2),
            (qf.Z_SPACE, qf.Z_DENSE), (512, 1024)):
        ctx.set_tuning(davidson=dav, split_target=split, f64_tile=tile, z_mode=z, block_44=blk)
        for flags in (qf.FP64, qf.FP64 | qf.GRAPH):
            got = _step(ctx, d, flags)
            assert abs(got[0] - ref[0]) < 1e-11
            assert np.abs(got[1] - ref[1]).max() < 1e-11
            assert np.abs(got[2] - ref[2]).max() < 1e-8
            assert np.abs(got[3] - ref[3]).max() < 1e-8
    with pytest.raises(qf.QFlowError):
        ctx.set_tuning(split_target=0)
    with pytest.raises(qf.QFlowError):
        ctx.set_tuning(davidson=2)
    with pytest.raises(qf.QFlowError):
        ctx.set_tuning(block_44=256)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_autotune_chooses_a_candidate_and_caches_it(tmp_path, prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qf, ctx, d = _setup()
    flags = {"fp64": qf.FP64, "bf16x3": qf.BF16X3}[prec] | qf.GRAPH
    g1, g2 = torch.from_numpy(d["t1"]).cuda(), torch.from_numpy(d["t2"]).cuda()
    cache = tmp_path / "tune.json"
    t, rep = ctx.autotune(d["sp"], d["o1"], d["o2"], g1, g2, flags, str(cache))
    print(rep)
    # the caller's pool is untouched
    assert np.array_equal(g1.cpu().numpy(), d["t1"]) and np.array_equal(g2.cpu().numpy(), d["t2"])
    choice = t.as_dict()
    assert choice["davidson"] in (0, 1) and choice["split_target"] in (2, 4, 8)
    assert choice["z_mode"] in (qf.Z_SPACE, qf.Z_DENSE, qf.Z_AUTO)
    assert ctx.get_tuning().as_dict() == choice
    lines = [ln for ln in rep.splitlines() if ln.startswith("davidson=")]
    assert len(lines) >= 5 and "chosen:" in rep
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert f"precision={flags & 15}" in key and "graph=1" in key
    assert {k: val[k] for k in choice} == choice
    # a new context takes the cached entry without timing
    qf2, ctx2, _ = _setup()
    t2, rep2 = ctx2.autotune(d["sp"], d["o1"], d["o2"], g1, g2, flags, str(cache))
    assert rep2.startswith("cached:") and t2.as_dict() == choice
    # and the tuned step is still the oracle's step
    em, E, T1, T2 = _step(ctx2, d, flags)
    n1, n2, Eo, Em, _ = qflow.flow_step(d["pb"], d["t1"], d["t2"], d["lists"],
                                        d["o1"].cpu().numpy(), d["o2"].cpu().numpy())
    tol = 1e-9 if prec == "fp64" else 1e-6
    assert abs(em - Em) < tol and np.abs(E - Eo).max() < tol
    assert np.abs(T2 - n2).max() < (1e-8 if prec == "fp64" else 1e-6)
