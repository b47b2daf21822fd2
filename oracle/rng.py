"""Probe vectors for the oracle: Z4 noise and hierarchical probing (FP64 / exact).

Z4 noise (Section 1): every component is drawn uniformly from {1, i, -1, -i}.
Algorithm 1 draws it with MATLAB randi, which is not reproducible, so the
noise index of each component comes from a counter-based generator instead:
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  The i-th output (i = 0, 1, ...) of the stream with
state s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), where mix is the 64-bit
finaliser  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31.

Keys:  K_run = out(seed, run);  hierarchical probing uses K_run for its single
base vector z0;  plain Monte Carlo uses K_j = out(K_run, j) for probe j.
Component n of a vector with key K takes bits 2(n mod 32), 2(n mod 32)+1 of
word out(K, n div 32); the 2-bit value k maps to i^k by table.

Hierarchical probing (Section 1 and Section 5.2): the nested colourings of
the 4D lattice and their Hadamard probing vectors.  The paper only describes
the construction; the colour used here (bit 4l at level l is the parity of
sum_mu floor(x_mu / 2^l); bits 4l+1..4l+3 are floor(x_mu / 2^l) mod 2 for
mu = x, y, z) and the natural Sylvester-Hadamard order
h_j(x) = (-1)^popcount(c(x) & j) are readings.  The first 2^m vectors span the
indicators of the partition by the low m colour bits, so 2, 32 and 512 vectors
are complete colourings ("colour closings", Section 6.3).  The probe is
z = z0 * h_j (Algorithm 1), with the Hadamard sign shared by the 12 components
of a site.

This is plain Python/numpy; uint64 arithmetic wraps modulo 2^64.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_out(state: int, i: int) -> int:
    """The i-th output (0-based) of a SplitMix64 stream started at `state`."""
    return mix64((state + (i + 1) * GOLDEN) & MASK64)


def splitmix64_sequence(state: int, count: int):
    """First `count` outputs of the stream (reference generator: state += gamma; return mix(state))."""
    out = []
    x = state & MASK64
    for _ in range(count):
        x = (x + GOLDEN) & MASK64
        out.append(mix64(x))
    return out


def _words(key: int, nwords: int) -> np.ndarray:
    """out(key, w) for w = 0..nwords-1, vectorised in uint64 numpy arithmetic."""
    with np.errstate(over="ignore"):
        w = np.arange(nwords, dtype=np.uint64)
        z = np.uint64(key) + (w + np.uint64(1)) * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def run_key(seed: int, run: int) -> int:
    return splitmix64_out(seed, run)


def probe_key(seed: int, run: int, hp: bool, j: int) -> int:
    kr = run_key(seed, run)
    return kr if hp else splitmix64_out(kr, j)


def z4_indices(key: int, N: int) -> np.ndarray:
    """2-bit noise index k(n) in {0,1,2,3} for n = 0..N-1 (uint8)."""
    nwords = (N + 31) // 32
    words = _words(key, nwords)
    n = np.arange(N, dtype=np.uint64)
    k = (words[n >> np.uint64(5)] >> (np.uint64(2) * (n & np.uint64(31)))) & np.uint64(3)
    return k.astype(np.uint8)


Z4_TABLE = np.array([1.0 + 0.0j, 0.0 + 1.0j, -1.0 + 0.0j, 0.0 - 1.0j], dtype=np.complex128)


def hp_colour(coords, level_count: int) -> int:
    """Colour bits of one site for levels 0..level_count-1 (pure Python)."""
    c = 0
    for lev in range(level_count):
        q = [coords[mu] >> lev for mu in range(4)]
        c |= ((q[0] + q[1] + q[2] + q[3]) & 1) << (4 * lev)
        c |= (q[0] & 1) << (4 * lev + 1)
        c |= (q[1] & 1) << (4 * lev + 2)
        c |= (q[2] & 1) << (4 * lev + 3)
    return c


def hp_colours(L, level_count: int = 4) -> np.ndarray:
    """Colour of every site in lexicographic order (x fastest), int64."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    xs = [a.ravel().astype(np.int64) for a in (x, y, z, t)]
    c = np.zeros_like(xs[0])
    for lev in range(level_count):
        q = [a >> lev for a in xs]
        c |= ((q[0] + q[1] + q[2] + q[3]) & 1) << (4 * lev)
        c |= (q[0] & 1) << (4 * lev + 1)
        c |= (q[1] & 1) << (4 * lev + 2)
        c |= (q[2] & 1) << (4 * lev + 3)
    return c


def popcount_parity(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.int64).copy()
    par = np.zeros_like(v)
    while np.any(v):
        par ^= v & 1
        v >>= 1
    return par


def hadamard_signs(L, j: int, level_count: int = 4) -> np.ndarray:
    """h_j(x) = (-1)^popcount(c(x) & j) per site (float64 +-1)."""
    if j >= 1 << (4 * level_count):
        raise ValueError("probe index needs more colour levels")
    c = hp_colours(L, level_count)
    return 1.0 - 2.0 * popcount_parity(c & j)


def probe(L, seed: int, run: int, hp: bool, j: int) -> np.ndarray:
    """Probe vector z_j (complex128, length N = 12 V, canonical component order)."""
    V = int(np.prod(L))
    N = 12 * V
    k = z4_indices(probe_key(seed, run, hp, j), N)
    z = Z4_TABLE[k]
    if hp:
        h = hadamard_signs(L, j)
        z = z * np.repeat(h, 12)
    return z


def probes(L, seed: int, run: int, hp: bool, first: int, count: int) -> np.ndarray:
    return np.stack([probe(L, seed, run, hp, first + j) for j in range(count)])
