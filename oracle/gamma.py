"""Traces Tr(Gamma A^-1) for several spin matrices Gamma over one deflation space
(oracle; FP64; test infrastructure only).

Follows the end of Section 5.2: the split of the trace into a deflated part
and a remainder holds with any inexpensive matrix Gamma multiplied in, the
estimator inserts one Gamma product per probe, and the deflation space (and
its cost) is shared by every Gamma.  With the deflated part P = W M W^H g5 of
D^-1 (the g5 form used for Tr(D^-1) as well):

    Tr(Gamma D^-1) = Tr(Gamma P) + Tr(Gamma (D^-1 - P)),
    T_D(Gamma)     = Tr(Gamma W M W^H g5) = Tr(M W^H g5 Gamma W),
    per probe      z^H Gamma D^-1 z - z^H Gamma P z
                 = z^H Gamma x - (W^H Gamma^H z)^H M (W^H g5 z),    x = D^-1 z.

Reading: Gamma is a 4 x 4 complex spin matrix acting the same way on every
site and colour (the Dirac matrices and their products are the case the
paper has in mind; any such matrix qualifies, Hermitian or not).  Vectors use
the canonical layout, entry n = 12 site + 3 spin + colour.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import lattice


def gamma_full(G: np.ndarray, V: int) -> np.ndarray:
    """The N x N matrix of Gamma on V sites: 1_sites (x) Gamma (x) 1_colour."""
    return np.kron(np.eye(V), np.kron(np.asarray(G, dtype=np.complex128), np.eye(3)))


def gamma_apply(G: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Gamma z for each row z of Z (rows of length 12 V)."""
    Z = np.atleast_2d(Z)
    s = Z.reshape(Z.shape[0], -1, 4, 3)
    return np.einsum("st,bvtc->bvsc", G, s).reshape(Z.shape)


def dirac_basis():
    """The 16 products g_mu1 g_mu2 ... (mu1 < mu2 < ...) of the chiral-basis
    Euclidean gamma matrices, the empty product (identity) first, then by
    number of factors and lexicographically.  Returns (labels, [16][4][4])."""
    g, _ = lattice.gamma_matrices()
    labels, mats = [], []
    for n in range(5):
        for idx in itertools.combinations(range(4), n):
            m = np.eye(4, dtype=np.complex128)
            for mu in idx:
                m = m @ g[mu]
            labels.append("".join("xyzt"[mu] for mu in idx) or "1")
            mats.append(m)
    return labels, np.array(mats)


def gamma_trace_exact(G: np.ndarray, Dinv: np.ndarray, V: int) -> complex:
    """Tr(Gamma D^-1) from the dense inverse."""
    return complex(np.trace(gamma_full(G, V) @ Dinv))


def gamma_deflated_trace(W: np.ndarray, M: np.ndarray, g5diag: np.ndarray, G: np.ndarray) -> complex:
    """T_D(Gamma) = Tr(Gamma W M W^H g5) = Tr(M W^H g5 Gamma W)."""
    GW = gamma_apply(G, W.T).T
    return complex(np.trace(M @ (W.conj().T @ (g5diag[:, None] * GW))))


def gamma_projection(W: np.ndarray, Z: np.ndarray, G: np.ndarray) -> np.ndarray:
    """c1(Gamma) = W^H Gamma^H z for each probe (rows of Z): k x s."""
    return W.conj().T @ gamma_apply(np.conj(np.asarray(G)).T, Z).T


def gamma_quadratic_forms(Z: np.ndarray, X: np.ndarray, G: np.ndarray) -> np.ndarray:
    """z_j^H Gamma x_j for each pair of rows."""
    GX = gamma_apply(G, X)
    return np.einsum("ja,ja->j", np.conj(Z), GX)


def gamma_corrections(W: np.ndarray, M: np.ndarray, g5diag: np.ndarray, Z: np.ndarray, G: np.ndarray) -> np.ndarray:
    """z_j^H Gamma P z_j = c1(Gamma)_j^H M c2_j with c2 = W^H g5 z."""
    c1 = gamma_projection(W, Z, G)
    c2 = W.conj().T @ (g5diag[:, None] * Z.T)
    return np.einsum("ij,ik,kj->j", c1.conj(), M, c2)
