"""Variance theory of deflated Hutchinson estimation (oracle; FP64).

- Theorem 1 (Section 2): with singular triplets (sigma, U, V) of A in
  descending order, Delta_ml = sum_i conj(u_im) v_im u_il conj(v_il), and the
  Z4 variance of the estimator of Tr(A_R) after deflating the k largest
  triplets is  sum_{m>k} sigma_m^2 - sum_{m,l>k} sigma_m sigma_l Delta_ml
  (eq. varAr); the difference to the undeflated variance is eq. vA-vAR.
- The 3x3 example of Section 2 (deflating the largest triplet of a symmetric
  3x3 matrix can raise, keep or lower the variance).
"""
from __future__ import annotations

import numpy as np


def svd_desc(A: np.ndarray):
    """Singular triplets in descending order: A = U diag(s) V^H."""
    U, s, Vh = np.linalg.svd(A)
    return U, s, Vh.conj().T


def delta_matrix(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Delta = (U . conj(V))^H (U . conj(V)) (eq. Delta)."""
    X = U * V.conj()
    return X.conj().T @ X


def variance_deflated_theorem1(A: np.ndarray, k: int) -> float:
    """Right-hand side of eq. varAr for deflation of the k largest triplets."""
    U, s, V = svd_desc(A)
    Dl = delta_matrix(U, V)
    sr = s[k:]
    val = np.sum(sr ** 2) - np.real(sr @ Dl[k:, k:] @ sr)
    return float(val)


def variance_difference_theorem1(A: np.ndarray, k: int) -> float:
    """Right-hand side of eq. vA-vAR."""
    U, s, V = svd_desc(A)
    Dl = delta_matrix(U, V)
    N = len(s)
    val = 0.0
    for m in range(k):
        val += s[m] ** 2 * (1 - np.real(Dl[m, m]))
        for l in range(m + 1, N):
            val -= s[m] * s[l] * np.real(Dl[m, l] + Dl[l, m])
    return float(val)


def deflated_remainder(A: np.ndarray, k: int) -> np.ndarray:
    """A_R = U_2 Sigma_2 V_2^H, i.e. A minus its k largest triplets (eq. deflatedA)."""
    U, s, V = svd_desc(A)
    return (U[:, k:] * s[k:]) @ V[:, k:].conj().T


def example_3x3_ratio(s: float, d: float) -> float:
    """Var(t(A)) / Var(t(A_r)) for the Section 2 example.

    A = U diag(1+2s, 1+s, 1) U^T with U from the QR factorisation of
    [[-1, d, d], [d, 1, 1], [d, 1, -1]]; A_r drops the largest eigenpair.
    A value above 1 means deflation reduced the variance.  The ratio does not
    depend on the column signs of U, so numpy's QR sign convention is fine.
    """
    B = np.array([[-1.0, d, d], [d, 1.0, 1.0], [d, 1.0, -1.0]])
    U, _ = np.linalg.qr(B)
    A = U @ np.diag([1 + 2 * s, 1 + s, 1.0]) @ U.T
    Ar = U[:, 1:] @ np.diag([1 + s, 1.0]) @ U[:, 1:].T
    off = lambda M: np.sum(M ** 2) - np.sum(np.diag(M) ** 2)
    return float(off(A) / off(Ar))
