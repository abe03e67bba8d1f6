"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the Quantum Flow method itself: it only
draws random numbers and assembles the synthetic Hamiltonian integrals and
random amplitude pools that both sides consume, so that random number
generation never enters a parity comparison.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), which is counter based: output k
of a stream seeded with s is mix(s + (k+1)*gamma).  Uniforms on [0,1) are
(x >> 11) * 2**-53; normals use the Box-Muller transform.

Integral recipe (synthetic stand-in for the paper's molecular Hamiltonians,
which need basis sets and SCF runs that are not available here):
  * h_pq symmetric; diagonal ~ U(-2,-0.5) for the N_o occupied orbitals and
    ~ U(0.2,3) for the N_v virtual ones, each sorted ascending; off-diagonal
    (p<q) ~ N(0, 0.01).
  * (pq|rs) = sum_L B^L_pq B^L_rs, B^L real symmetric with entries (p<=q)
    ~ N(0, 0.0125) * exp(-|p-q|/8).  The "0.05/4" of the workload statement is
    read as a standard deviation.
  * Occupied orbitals come first (indices 0..N_o-1), virtuals after.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Workload configurations: name -> (n_orb, n_occ, L, K, space sizes, seed index);
# K = 0 runs Algorithm 1 to full coverage
CONFIGS = {
    "c1": dict(n=8, o=3, L=16, K=10, sizes=((3, 3),), idx=1),
    "c2": dict(n=40, o=5, L=80, K=256, sizes=((3, 3),), idx=2),
    "c3": dict(n=82, o=10, L=164, K=2048, sizes=((3, 3),), idx=3),
    "c4": dict(n=114, o=13, L=228, K=4096, sizes=((3, 3),), idx=4),
    "c5": dict(n=114, o=13, L=228, K=6144, sizes=((2, 2), (3, 3), (4, 4)), idx=5),
    # full Algorithm 1 cycles (K = 0: every (o1<o2, v1<v2) tuple covered) at
    # the shapes of the paper's largest workloads: 4 correlated occupied and
    # 110 virtual orbitals (water, cc-pVQZ; about 10.3k spaces) and 13 and 69
    # (propane, cc-pVDZ; about 56.9k spaces)
    "c6": dict(n=114, o=4, L=228, K=0, sizes=((3, 3),), idx=6),
    "c7": dict(n=82, o=13, L=164, K=0, sizes=((3, 3),), idx=7),
}


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Raw 64-bit SplitMix64 outputs number offset..offset+count-1."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles on [0,1): (x >> 11) * 2^-53."""
    x = splitmix64(seed, count, offset)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential reader over one SplitMix64 uniform stream."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def uniform(self, count: int) -> np.ndarray:
        u = uniform(self.seed, count, self.pos)
        self.pos += count
        return u

    def normal(self, count: int) -> np.ndarray:
        """Box-Muller: two uniforms per normal (cosine branch only)."""
        u = self.uniform(2 * count).reshape(count, 2)
        r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
        return r * np.cos(2.0 * np.pi * u[:, 1])


def gen_integrals(n: int, o: int, L: int, seed: int, b_std: float = 0.0125,
                  off_std: float = 0.01):
    """Return (h[n,n], eri[n,n,n,n]) in chemist order (pq|rs), float64."""
    st = Stream(seed)
    v = n - o
    h = np.zeros((n, n))
    d_occ = np.sort(-2.0 + 1.5 * st.uniform(o))
    d_vir = np.sort(0.2 + 2.8 * st.uniform(v))
    h[np.arange(o), np.arange(o)] = d_occ
    h[np.arange(o, n), np.arange(o, n)] = d_vir
    iu = np.triu_indices(n, 1)
    off = off_std * st.normal(len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    ip, iq = np.triu_indices(n, 0)
    damp = np.exp(-np.abs(ip - iq) / 8.0)
    B = np.zeros((L, n, n))
    for l in range(L):
        x = b_std * st.normal(len(ip)) * damp
        B[l][ip, iq] = x
        B[l][iq, ip] = x
    # Products over unique pairs only, then scattered to all eight index
    # permutations, so the stored tensor is exactly 8-fold symmetric.
    Bp = B[:, ip, iq]
    G = Bp.T @ Bp
    G = 0.5 * (G + G.T)
    pair = np.zeros((n, n), dtype=np.int64)
    pair[ip, iq] = np.arange(len(ip))
    pair[iq, ip] = np.arange(len(ip))
    eri = G[pair[:, :, None, None], pair[None, None, :, :]]
    return h, eri


def config_integrals(name: str):
    c = CONFIGS[name]
    return gen_integrals(c["n"], c["o"], c["L"], 1000 + c["idx"])


def sampling_stream(name: str, size_class: int = 0) -> Stream:
    """Uniform stream for active-space sampling of config `name`; a config
    with several space sizes draws each size class (its position in
    `sizes`) from a stream of its own, seeded 2000 + N + 100 * class."""
    return Stream(2000 + CONFIGS[name]["idx"] + 100 * size_class)


def random_amplitudes(o: int, v: int, seed: int, scale: float = 0.05):
    """Random t1[o,v] and t2[o,o,v,v] with t2[i,j,a,b] = t2[j,i,b,a]."""
    st = Stream(seed)
    t1 = scale * st.normal(o * v).reshape(o, v)
    t2 = scale * st.normal(o * o * v * v).reshape(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    return t1, t2
