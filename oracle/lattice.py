"""Dense Wilson-Dirac matrix on a small 4D lattice (oracle; FP64).

The paper treats the Dirac matrix only as a discrete differential operator on
a regular 4D lattice with 12 degrees of freedom per site, 4 spin x 3 colour
(Section 1, dilution paragraph), and uses a clover-improved Wilson matrix in
Section 6.  It does not print the operator.  The oracle uses the plain Wilson
form with r = 1 (readings listed with the design notes):

    D psi(x) = (4 + m) psi(x)
               - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
                              + (1 + g_mu) U_mu(x - mu)^dagger psi(x - mu) ]

with a factor -1 on every hop that crosses the t boundary (antiperiodic in t,
periodic in x, y, z).  Chiral basis: g_k = [[0, -i s_k], [i s_k, 0]] for
k = 1, 2, 3 and g_4 = [[0, 1], [1, 0]], so g5 = g1 g2 g3 g4 = diag(1, 1, -1, -1).

Indexing: site n = x + Lx (y + Ly (z + Lz t)); component 12 n + 3 spin + colour.
Canonical spinor arrays are [..][Lt][Lz][Ly][Lx][4][3]; links [4][Lt][Lz][Ly][Lx][3][3].

This module is written for clarity, not speed: explicit 4x4 spin matrices and
a Python loop over sites (small lattices only).
"""
from __future__ import annotations

import numpy as np

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def gamma_matrices():
    """Chiral-basis Euclidean gamma matrices (g_x, g_y, g_z, g_t) and g5."""
    z2 = np.zeros((2, 2), dtype=np.complex128)
    i2 = np.eye(2, dtype=np.complex128)
    g = [np.block([[z2, -1j * s], [1j * s, z2]]) for s in SIGMA]
    g.append(np.block([[z2, i2], [i2, z2]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def volume(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


def site_index(c, L) -> int:
    """Lexicographic site number, x fastest."""
    return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))


def site_coords(n, L):
    x = n % L[0]
    n //= L[0]
    y = n % L[1]
    n //= L[1]
    z = n % L[2]
    t = n // L[2]
    return (x, y, z, t)


def dense_wilson(U: np.ndarray, L, mass: float, t_antiperiodic: bool = True) -> np.ndarray:
    """Dense N x N Wilson-Dirac matrix, N = 12 V.

    U: canonical links [4][Lt][Lz][Ly][Lx][3][3].  Blocks accumulate, so a
    direction of extent 2 (forward and backward neighbour coincide) is handled
    by summing both hops.
    """
    g, _ = gamma_matrices()
    i4 = np.eye(4, dtype=np.complex128)
    V = volume(L)
    N = 12 * V
    D = np.zeros((N, N), dtype=np.complex128)
    D[np.arange(N), np.arange(N)] = 4.0 + mass
    for n in range(V):
        c = site_coords(n, L)
        for mu in range(4):
            c2 = list(c)
            c2[mu] = (c[mu] + 1) % L[mu]
            n2 = site_index(c2, L)
            phase = -1.0 if (t_antiperiodic and mu == 3 and c[3] == L[3] - 1) else 1.0
            u = U[mu, c[3], c[2], c[1], c[0]]
            # forward hop from x to x+mu, and the backward hop from x+mu to x
            D[12 * n:12 * n + 12, 12 * n2:12 * n2 + 12] += -0.5 * phase * np.kron(i4 - g[mu], u)
            D[12 * n2:12 * n2 + 12, 12 * n:12 * n + 12] += -0.5 * phase * np.kron(i4 + g[mu], u.conj().T)
    return D


def gamma5_full(V: int) -> np.ndarray:
    """Diagonal of g5 (x) 1_colour on all N = 12 V components (chiral basis)."""
    _, g5 = gamma_matrices()
    d = np.real(np.diag(g5))
    return np.tile(np.repeat(d, 3), V)


def to_vector(psi: np.ndarray) -> np.ndarray:
    """Canonical [..][Lt][Lz][Ly][Lx][4][3] -> [..][N] (pure reshape)."""
    lead = psi.shape[:-6]
    return psi.reshape(lead + (-1,))


def free_field_singular_values(L, mass: float, t_antiperiodic: bool = True) -> np.ndarray:
    """Closed-form singular values of the free (U = 1) Wilson matrix.

    In momentum space the free operator is M(p) + i sum_mu g_mu sin p_mu with
    M(p) = m + sum_mu (1 - cos p_mu); its singular values are
    sqrt(M^2 + sum sin^2 p), each 12-fold (4 spin x 3 colour, the two
    chiralities pair up).  p_mu = 2 pi n / L_mu, and p_t = (2n + 1) pi / L_t
    for antiperiodic time.  Section 6 completes the measured spectrum with
    this free-field spectrum.
    """
    ps = []
    for mu in range(4):
        n = np.arange(L[mu])
        if mu == 3 and t_antiperiodic:
            ps.append((2 * n + 1) * np.pi / L[mu])
        else:
            ps.append(2 * n * np.pi / L[mu])
    P = np.meshgrid(*ps, indexing="ij")
    M = mass + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    sig = np.sqrt(M ** 2 + s2).ravel()
    return np.sort(np.repeat(sig, 12))


def free_field_trace_inverse(L, mass: float, t_antiperiodic: bool = True) -> float:
    """Closed form Tr D^-1 of the free Wilson matrix: sum_p 12 M(p) / (M(p)^2 + sum sin^2 p)."""
    ps = []
    for mu in range(4):
        n = np.arange(L[mu])
        if mu == 3 and t_antiperiodic:
            ps.append((2 * n + 1) * np.pi / L[mu])
        else:
            ps.append(2 * n * np.pi / L[mu])
    P = np.meshgrid(*ps, indexing="ij")
    M = mass + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    return float(np.sum(12.0 * M / (M ** 2 + s2)))
