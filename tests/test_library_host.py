"""libqflow without a GPU: exported symbols and the host-side logic
(Algorithm 1 and ownership) against the oracle, bit for bit."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import sampling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_04186_amd", "libqflow.so")
HEADER = os.path.join(ROOT, "include", "qflow.h")

needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libqflow.so not built")


def declared_symbols():
    """Function names declared in the header (comments removed first)."""
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return sorted(set(re.findall(r"\b(qflow_[a-z_0-9]+)\s*\(", text)))


@needs_lib
def test_library_exports_every_declared_symbol():
    import ctypes
    L = ctypes.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


@needs_lib
@pytest.mark.parametrize("No,Nv,cap", [(5, 12, 0), (4, 19, 0), (10, 72, 300)])
def test_sampler_matches_oracle(No, Nv, cap):
    from paper_2606_04186_amd import api
    u = synth.uniform(2024 + Nv, 400000)
    eps = np.concatenate([np.sort(-2 + 1.5 * synth.uniform(5, No)),
                          np.sort(0.2 + 2.8 * synth.uniform(6, Nv))])
    sp, de, used = api.sample_spaces(No, Nv, 3, 3, eps, u, cap=cap, max_out=200000)

    class Fixed:
        def __init__(self):
            self.pos = 0

        def uniform(self, k):
            x = u[self.pos:self.pos + k]
            self.pos += k
            return x

    st = Fixed()
    ref = sampling.algorithm1(No, Nv, 3, 3, eps, st, cap=cap or None)
    assert used == st.pos
    assert len(sp) == len(ref)
    for s, r in zip(sp, ref):
        assert tuple(s["orb"][:3]) == r[0] and tuple(s["orb"][3:6]) == r[1]
    assert np.array_equal(de, np.array([r[2] for r in ref]))


@needs_lib
def test_owners_match_oracle():
    from paper_2606_04186_amd import api
    No, Nv = 6, 14
    u = synth.uniform(77, 20000)
    eps = np.linspace(-2, 3, No + Nv)
    sp, _, _ = api.sample_spaces(No, Nv, 3, 3, eps, u, cap=25)
    o1, o2 = api.build_owners(No, Nv, sp)
    lists = [(tuple(s["orb"][:3]), tuple(s["orb"][3:6])) for s in sp]
    r1, r2 = sampling.ownership(No, Nv, lists)
    assert np.array_equal(o1, r1) and np.array_equal(o2, r2)


@needs_lib
def test_sampler_rejects_exhausted_uniforms():
    from paper_2606_04186_amd import api
    with pytest.raises(api.QFlowError):
        api.sample_spaces(4, 19, 3, 3, np.linspace(-1, 1, 23), synth.uniform(1, 50))
