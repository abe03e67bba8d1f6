"""The seeded input generator (shared by the oracle and the HIP path)."""
import numpy as np
import pytest

import synth
from oracle import qflow


def test_splitmix64_published_sequence():
    # first outputs of SplitMix64 seeded with 1234567 (reference C code of
    # Steele, Lea and Flood as distributed with xoshiro/xoroshiro)
    assert list(map(int, synth.splitmix64(1234567, 5))) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_stream_is_counter_based():
    st = synth.Stream(99)
    a = st.uniform(10)
    b = st.uniform(5)
    assert np.array_equal(np.concatenate([a, b]), synth.uniform(99, 15))
    assert a.min() >= 0 and a.max() < 1


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_integrals_symmetry_and_scale(name):
    c = synth.CONFIGS[name]
    h, eri = synth.config_integrals(name)
    n, o = c["n"], c["o"]
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2)]:
        assert np.array_equal(eri, eri.transpose(perm))
    d = np.diag(h)
    assert np.all(np.diff(d[:o]) >= 0) and np.all(np.diff(d[o:]) >= 0)
    assert -2 <= d[:o].min() and d[:o].max() <= -0.5
    assert 0.2 <= d[o:].min() and d[o:].max() <= 3
    pb = qflow.Problem(h, eri, o)
    assert pb.eps[o:].min() - pb.eps[:o].max() > 0.5     # positive gap
    # (pq|pq) >= 0 for a positive semidefinite product of factors
    pq = eri.reshape(n * n, n * n)
    assert np.linalg.eigvalsh(pq).min() > -1e-12


def test_random_amplitudes_pair_symmetry():
    t1, t2 = synth.random_amplitudes(3, 5, 1)
    assert np.array_equal(t2, t2.transpose(1, 0, 3, 2))
