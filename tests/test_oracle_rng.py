"""Pins of the oracle's probe generator.

- SplitMix64 reproduces its published known-answer values;
- the per-component bit extraction agrees with the scalar generator;
- Z4 indices are uniform and E(z z^H) = I (Section 1's requirement on z);
- Hadamard columns: sum_{j<2^m} h_j(x) h_j(y) = 2^m [c_m(x) == c_m(y)];
- colour closings: with 2, 32 and 512 vectors the same-colour site pairs lie
  at torus Manhattan distances that are multiples of 2, 4 and 8 -- the paper
  states that 32 vectors remove distances 1, 2, 3, 5, 6, 7 (Section 6.2);
- a complete sweep equals z0^H (M_s . A) z0 for any A.
"""
import os

import numpy as np
import pytest

from oracle import rng
from oracle.lattice import site_coords

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def test_splitmix64_known_answers():
    vals = [int(l) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert rng.splitmix64_sequence(1234567, len(vals)) == vals
    assert [rng.splitmix64_out(1234567, i) for i in range(len(vals))] == vals


def test_z4_bits_match_scalar_generator():
    key = rng.probe_key(7, 3, False, 5)
    k = rng.z4_indices(key, 200)
    for n in range(200):
        word = rng.splitmix64_out(key, n // 32)
        assert k[n] == (word >> (2 * (n % 32))) & 3


def test_z4_uniform_and_isotropic():
    N = 64
    s = 4000
    Z = np.stack([rng.Z4_TABLE[rng.z4_indices(rng.probe_key(1, 0, False, j), N)] for j in range(s)])
    C = (Z.T @ Z.conj()) / s          # estimate of E z z^H
    assert np.abs(np.diag(C) - 1).max() < 1e-12
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 5.0 / np.sqrt(s) * 1.5
    counts = np.bincount(rng.z4_indices(rng.probe_key(2, 0, True, 0), 400000), minlength=4)
    exp = 100000
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < 25.0                 # 3 dof, p ~ 2e-5


@pytest.mark.parametrize("m", [1, 4, 5, 8])
def test_hadamard_partition_identity(m):
    L = (4, 4, 4, 8)
    c = rng.hp_colours(L)
    H = np.stack([rng.hadamard_signs(L, j) for j in range(1 << m)])
    G = H.T @ H
    cm = c & ((1 << m) - 1)
    assert np.array_equal(G, (1 << m) * (cm[:, None] == cm[None, :]))


def _torus_dist(a, b, L):
    return sum(min(abs(a[i] - b[i]), L[i] - abs(a[i] - b[i])) for i in range(4))


@pytest.mark.parametrize("L,nbits,modulus", [((4, 4, 4, 4), 1, 2), ((4, 4, 4, 4), 5, 4), ((8, 8, 8, 8), 9, 8)])
def test_colour_closing_distances(L, nbits, modulus):
    c = rng.hp_colours(L) & ((1 << nbits) - 1)
    V = int(np.prod(L))
    rs = np.random.default_rng(0)
    src = rs.choice(V, size=min(V, 40), replace=False)
    coords = [site_coords(n, L) for n in range(V)]
    seen = set()
    for a in src:
        for b in range(V):
            if c[a] == c[b]:
                d = _torus_dist(coords[a], coords[b], L)
                assert d % modulus == 0
                seen.add(d)
    assert 0 in seen and modulus in seen
    if nbits == 5:
        # Section 6.2: 32 probing vectors remove distances 1, 2, 3, 5, 6, 7
        assert not seen & {1, 2, 3, 5, 6, 7}


def test_complete_sweep_is_masked_quadratic_form():
    L = (4, 4, 4, 4)
    V = 256
    N = 12 * V
    rs = np.random.default_rng(1)
    A = rs.standard_normal((N, N)) + 1j * rs.standard_normal((N, N))
    nb = 5
    Z = rng.probes(L, 3, 0, True, 0, 1 << nb)
    t_sweep = np.mean(np.einsum("ja,ab,jb->j", Z.conj(), A, Z))
    z0 = rng.Z4_TABLE[rng.z4_indices(rng.probe_key(3, 0, True, 0), N)]
    cm = np.repeat(rng.hp_colours(L) & ((1 << nb) - 1), 12)
    Am = np.where(cm[:, None] == cm[None, :], A, 0)
    assert abs(t_sweep - z0.conj() @ Am @ z0) <= 1e-10 * abs(t_sweep)
