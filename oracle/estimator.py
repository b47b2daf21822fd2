"""Hutchinson trace estimation with deflation and hierarchical probing (oracle; FP64).

Follows:
- Section 1, eq. (1): t = (1/s) sum_j z_j^H A^-1 z_j, unbiased for Tr(A^-1) when
  E(z z^H) = I.
- Section 1, eq. variance: for Z4 noise, Var(t) per sample = ||A~||_F^2, the
  squared Frobenius norm of the off-diagonal part.
- Section 2, eq. deflatedA and Section 5.2: Tr(A^-1) = Tr(A_D^-1) + Tr(A_R^-1);
  the deflated part is evaluated exactly, the remainder by quadratures
  z^H A^-1 z - z^H (deflated part) z.
- Algorithm 1: T_D once, then T_R accumulates z^H y - z^H P z, and the trace
  estimate after j probes is T_R / j + T_D.

Deflation form (reading): with k eigenvectors W of the Hermitian Q = g5 D,
D^-1 = Q^-1 g5, and the deflated part is P = W M W^H g5 with M = (W^H Q W)^-1
(the Galerkin inverse of Q on span W; equal to Lambda^-1 for exact orthonormal
eigenvectors, and to the Rayleigh-Ritz form Y Theta^-1 Y^H in general).  For
exact triplets this equals V Sigma^-1 U^H of Section 5.2.  The estimator stays
unbiased for any W provided T_D = Tr(P) uses the same W and M.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


# --------------------------------------------------------------------------
# exact quantities
# --------------------------------------------------------------------------
def lu_factor(D: np.ndarray):
    return sla.lu_factor(D)


def exact_inverse(D: np.ndarray) -> np.ndarray:
    return sla.lu_solve(sla.lu_factor(D), np.eye(D.shape[0], dtype=D.dtype))


def trace_inverse_lu(D: np.ndarray) -> complex:
    """Tr(D^-1) from an LU factorisation (column by column solve)."""
    return complex(np.trace(exact_inverse(D)))


def trace_inverse_eig(D: np.ndarray) -> complex:
    """Tr(D^-1) = sum 1/eig(D): an independent route for the same number."""
    return complex(np.sum(1.0 / np.linalg.eigvals(D)))


def offdiag_frobenius2(A: np.ndarray) -> float:
    """||A - diag(diag(A))||_F^2 (Section 1, eq. variance)."""
    return float(np.sum(np.abs(A) ** 2) - np.sum(np.abs(np.diag(A)) ** 2))


def masked_offdiag_frobenius2(A: np.ndarray, colours: np.ndarray, nbits: int) -> float:
    """||offdiag(M_s . A)||_F^2 where M_s(a, b) = [c_m(a) == c_m(b)], m = nbits.

    Variance over the Z4 base vector of one complete hierarchical-probing
    sweep over 2^m Hadamard vectors (Section 6.2's masked Frobenius norms).
    `colours` is per component (length N).
    """
    cm = colours & ((1 << nbits) - 1)
    mask = cm[:, None] == cm[None, :]
    B = np.where(mask, A, 0)
    return offdiag_frobenius2(B)


# --------------------------------------------------------------------------
# deflation (Section 5.2; the T_D step of Algorithm 1)
# --------------------------------------------------------------------------
def q_eigenpairs(D: np.ndarray, g5diag: np.ndarray, k: int):
    """k eigenpairs of Q = g5 D with smallest |lambda| (dense eigh)."""
    Q = g5diag[:, None] * D
    Q = 0.5 * (Q + Q.conj().T)
    lam, W = np.linalg.eigh(Q)
    order = np.argsort(np.abs(lam), kind="stable")[:k]
    return lam[order], W[:, order]


def galerkin_M(W: np.ndarray, D: np.ndarray, g5diag: np.ndarray) -> np.ndarray:
    """M = (W^H Q W)^-1 with Q = g5 D."""
    H = W.conj().T @ (g5diag[:, None] * (D @ W))
    return np.linalg.inv(H)


def rayleigh_diag_M(W: np.ndarray, D: np.ndarray, g5diag: np.ndarray) -> np.ndarray:
    """Diagonal M with M_ii = 1 / (w_i^H Q w_i): the Galerkin inverse when W holds
    orthonormal eigenvectors of Q; for other W it defines another valid P."""
    QW = g5diag[:, None] * (D @ W)
    rq = np.einsum("ni,ni->i", W.conj(), QW).real
    return np.diag(1.0 / rq)


def deflated_trace(W: np.ndarray, M: np.ndarray, g5diag: np.ndarray) -> complex:
    """T_D = Tr(P) = Tr(M W^H g5 W)."""
    return complex(np.trace(M @ (W.conj().T @ (g5diag[:, None] * W))))


def deflation_matrix(W: np.ndarray, M: np.ndarray, g5diag: np.ndarray) -> np.ndarray:
    """P = W M W^H g5 (dense)."""
    return (W @ M @ W.conj().T) * g5diag[None, :]


def trace_deflated_svd(D: np.ndarray, k: int):
    """T_D = Tr(V_k Sigma_k^-1 U_k^H) = sum_i u_i^H v_i / sigma_i over the k smallest
    singular triplets of D (Section 5.2, via dense SVD)."""
    U, s, Vh = np.linalg.svd(D)
    idx = np.argsort(s)[:k]
    val = 0.0 + 0.0j
    for i in idx:
        val += np.vdot(U[:, i], Vh[i].conj()) / s[i]
    return complex(val), np.sort(s)


def projection_coefficients(W: np.ndarray, Z: np.ndarray, g5diag: np.ndarray):
    """c1 = W^H z and c2 = W^H g5 z for each probe (rows of Z): k x s matrices."""
    c1 = W.conj().T @ Z.T
    c2 = W.conj().T @ (g5diag[:, None] * Z.T)
    return c1, c2


def deflation_corrections(c1: np.ndarray, c2: np.ndarray, M: np.ndarray) -> np.ndarray:
    """d_j = z_j^H P z_j = c1_j^H M c2_j."""
    return np.einsum("ij,ik,kj->j", c1.conj(), M, c2)


# --------------------------------------------------------------------------
# quadratic forms and estimates (eq. 1, Algorithm 1)
# --------------------------------------------------------------------------
def quadratic_forms(Z: np.ndarray, X: np.ndarray) -> np.ndarray:
    """q_j = z_j^H x_j, each summed with math.fsum (Re and Im separately)."""
    out = np.empty(Z.shape[0], dtype=np.complex128)
    for j in range(Z.shape[0]):
        prod = np.conj(Z[j]) * X[j]
        out[j] = complex(math.fsum(prod.real), math.fsum(prod.imag))
    return out


def running_trace(q: np.ndarray, T_D: complex = 0.0) -> np.ndarray:
    """Algorithm 1: Trace after j probes = T_R / j + T_D."""
    return np.cumsum(q) / np.arange(1, len(q) + 1) + T_D


def sample_statistics(q: np.ndarray):
    """Mean and unbiased (1/(s-1)) sample variances of complex samples.

    var      = mean |q - qbar|^2 (the Z4 variance of eq. variance)
    var_re   = variance of Re q,  var_im = variance of Im q.
    """
    s = len(q)
    mean = complex(np.mean(q))
    if s < 2:
        return mean, float("nan"), float("nan"), float("nan")
    d = q - mean
    var = float(np.sum(np.abs(d) ** 2) / (s - 1))
    var_re = float(np.sum(d.real ** 2) / (s - 1))
    var_im = float(np.sum(d.imag ** 2) / (s - 1))
    return mean, var, var_re, var_im


def hutchinson_enumeration(A: np.ndarray):
    """Exact mean and variance of z^H A z over ALL 4^N Z4 vectors (tiny N only).

    Returns (mean, E|z^H A z - mean|^2) by brute-force enumeration.
    """
    N = A.shape[0]
    vals = np.array([1, 1j, -1, -1j])
    grids = np.meshgrid(*([np.arange(4)] * N), indexing="ij")
    idx = np.stack([g.ravel() for g in grids], axis=1)
    Z = vals[idx]
    q = np.einsum("sa,ab,sb->s", Z.conj(), A, Z)
    mean = q.mean()
    return complex(mean), float(np.mean(np.abs(q - mean) ** 2))


# --------------------------------------------------------------------------
# variance analysis over runs (Sections 6.1-6.3)
# --------------------------------------------------------------------------
def jackknife_error(values: np.ndarray, statistic) -> float:
    """Jackknife standard error of statistic(values) from its leave-one-out
    values: sqrt((R - 1) / R * sum (s_(-r) - mean s_(-))^2) (Section 6.1 quotes
    Jackknife error bars over 40 runs)."""
    R = len(values)
    loo = np.array([statistic(np.delete(values, r)) for r in range(R)])
    return float(np.sqrt((R - 1) / R * np.sum((loo - loo.mean()) ** 2)))


def complex_variance(t: np.ndarray) -> float:
    """Unbiased E|t - tbar|^2 of complex samples."""
    return float(np.sum(np.abs(t - t.mean()) ** 2) / (len(t) - 1))


def hp_run_statistics(q_runs: np.ndarray, s: int, v_stoc: float = 0.0) -> dict:
    """Runs r of Algorithm 1 with the quadratic forms q_runs[r, :] of their
    probes: the estimate after s probes t_r = mean of the first s, the variance
    over runs V_hp(s) with its Jackknife error, and the speedup over plain
    noise R_s = V_stoc / (V_hp(s) s) (Section 6.2)."""
    t = q_runs[:, :s].mean(axis=1)
    V = complex_variance(t)
    out = {"mean": complex(t.mean()), "mean_err": float(np.sqrt(V / len(t))), "var": V,
           "var_err": jackknife_error(t, complex_variance)}
    if v_stoc > 0:
        out["rs"] = v_stoc / (V * s)
        out["rs_err"] = jackknife_error(t, lambda x: v_stoc / (complex_variance(x) * s))
    return out


def playback(W: np.ndarray, D: np.ndarray, g5diag: np.ndarray, Z: np.ndarray, q: np.ndarray, kk: int,
             diagonal: bool = False):
    """Section 6.3's playback: the deflated quadratures q_j - z_j^H P' z_j and
    T_D' = Tr P' of the basis restricted to its leading kk vectors, with the
    Galerkin (or diagonal Rayleigh) M of that smaller basis."""
    if kk == 0:
        return q.copy(), 0.0
    Wk = W[:, :kk]
    M = rayleigh_diag_M(Wk, D, g5diag) if diagonal else galerkin_M(Wk, D, g5diag)
    c1, c2 = projection_coefficients(Wk, Z, g5diag)
    return q - deflation_corrections(c1, c2, M), deflated_trace(Wk, M, g5diag)
