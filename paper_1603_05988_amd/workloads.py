"""Seeded synthetic inputs: the five lattice workloads and their gauge links.

This module produces *inputs* only (gauge links, random test spinors, the
configuration table).  It holds none of the estimator's arithmetic, so both the
GPU path and the CPU oracle may be fed from it.

The paper's operators are two physical 32^3x64 clover-Wilson ensembles
(Section 6); they are not available, so the workloads use random-link Wilson
operators with the paper's lattice shapes.  Links are U = exp(i*eps*H) with H a
random traceless Hermitian 3x3 matrix with Gaussian entries.

Link layout (canonical, shared by every interface): complex128 array of shape
[4][Lt][Lz][Ly][Lx][3][3], direction mu = 0..3 <-> x, y, z, t, row-major 3x3,
U_mu(x) connects site x to x + mu-hat.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    L: tuple            # (Lx, Ly, Lz, Lt)
    eps: float          # link roughness: U = exp(i eps H)
    seed: int           # link seed, also the probe-noise seed
    mass: float         # bare Wilson mass m in D = (4+m) - hop/2
    k: int              # deflation vectors
    nprobe: int         # probe vectors per run
    batch: int          # right-hand sides per batch
    hp: bool            # hierarchical probing (True) or plain Z4 noise (False)
    tol: float          # relative true-residual target of each solve

    @property
    def V(self) -> int:
        return int(np.prod(self.L))

    @property
    def N(self) -> int:
        return 12 * self.V


# The five workloads.  c1 is the dense-checkable case, c5 the paper-sized one
# (same N = 25,165,824 and k = 1000 as the paper's Section 6 runs, s = 512
# hierarchical-probing vectors = the paper's second colour closing).
WORKLOADS = {
    "c1": Workload("wilson_4^4", (4, 4, 4, 4), 0.3, 0, -0.20, 16, 256, 16, False, 1e-12),
    "c2": Workload("wilson_8^3x16", (8, 8, 8, 16), 0.5, 1, -0.35, 64, 64, 64, False, 1e-8),
    "c3": Workload("wilson_16^3x32", (16, 16, 16, 32), 0.5, 2, -0.38, 200, 256, 16, True, 1e-8),
    "c4": Workload("wilson_8^3x16_nn", (8, 8, 8, 16), 0.5, 1, -0.35, 64, 64, 16, False, 1e-8),
    "c5": Workload("wilson_32^3x64", (32, 32, 32, 64), 0.5, 3, -0.39, 1000, 512, 16, True, 1e-8),
}


def gauge_links(L, eps: float, seed: int, chunk_sites: int = 1 << 20) -> np.ndarray:
    """Random links U = exp(i eps H), H traceless Hermitian with N(0,1) entries.

    Draw order: numpy default_rng(seed) produces standard normals of shape
    [4][Lt][Lz][Ly][Lx][3][3][2] (real, imaginary), consumed in C order in
    chunks; H = (G + G^H)/2 - Tr(.)/3 I; U = Q diag(exp(i eps h)) Q^H from the
    eigendecomposition of H.  Returns complex128 [4][Lt][Lz][Ly][Lx][3][3].
    """
    Lx, Ly, Lz, Lt = L
    nmat = 4 * Lt * Lz * Ly * Lx
    rng = np.random.default_rng(seed)
    out = np.empty((nmat, 3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for s in range(0, nmat, chunk_sites):
        n = min(chunk_sites, nmat - s)
        g = rng.standard_normal((n, 3, 3, 2))
        a = g[..., 0] + 1j * g[..., 1]
        h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
        tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
        h = h - tr[:, None, None] * eye
        w, q = np.linalg.eigh(h)
        ph = np.exp(1j * eps * w)
        out[s:s + n] = (q * ph[:, None, :]) @ np.conj(np.swapaxes(q, -1, -2))
    return out.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def random_spinors(L, nrhs: int, seed: int) -> np.ndarray:
    """Gaussian complex test spinors, canonical layout [rhs][t][z][y][x][spin 4][colour 3]."""
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed)
    shape = (nrhs, Lt, Lz, Ly, Lx, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_gauge_transform(L, seed: int) -> np.ndarray:
    """Random SU(3)-valued (unitary) site matrices g(x), shape [Lt][Lz][Ly][Lx][3][3]."""
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((Lt * Lz * Ly * Lx, 3, 3)) + 1j * rng.standard_normal((Lt * Lz * Ly * Lx, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    return q.reshape(Lt, Lz, Ly, Lx, 3, 3)


def _mix32(x, xp):
    """A 32-bit integer mixer (xor-shift / multiply; Wellons' "lowbias32"
    constants) on non-negative int64 arrays of numpy or torch, kept to 32 bits."""
    m = 0xFFFFFFFF
    x = x & m
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & m
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & m
    x = x ^ (x >> 16)
    return x


def hashed_basis(cols, N: int, seed: int, xp=np, device=None):
    """Synthetic deflation-basis columns with entries (+-1 +- i) * 2^-13, the
    signs hashed from (seed, column, index): exact in BF16 and in every FP32
    partial sum of their products with Z4 probes, so sampled projection
    coefficients can be checked exactly.  cols: column indices; returns a
    complex128 array [len(cols)][N] (numpy, or torch on `device`)."""
    out = []
    for c in cols:
        if xp is np:
            n = np.arange(N, dtype=np.int64)
            key = int(_mix32(seed * 1000003 + int(c), np))
        else:
            n = xp.arange(N, dtype=xp.int64, device=device)
            key = int(_mix32(seed * 1000003 + int(c), np))
        h = _mix32(n ^ key, xp)
        re = 1.0 - 2.0 * (h & 1)
        im = 1.0 - 2.0 * ((h >> 1) & 1)
        if xp is np:
            out.append((re + 1j * im) * 2.0 ** -13)
        else:
            out.append(xp.complex(re.double(), im.double()) * 2.0 ** -13)
    return np.stack(out) if xp is np else xp.stack(out)
