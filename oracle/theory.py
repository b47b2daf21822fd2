"""Variance theory of deflated Hutchinson estimation (oracle; FP64).

- Theorem 1 (Section 2): with singular triplets (sigma, U, V) of A in
  descending order, Delta_ml = sum_i conj(u_im) v_im u_il conj(v_il), and the
  Z4 variance of the estimator of Tr(A_R) after deflating the k largest
  triplets is  sum_{m>k} sigma_m^2 - sum_{m,l>k} sigma_m sigma_l Delta_ml
  (eq. varAr); the difference to the undeflated variance is eq. vA-vAR.
- The 3x3 example of Section 2 (deflating the largest triplet of a symmetric
  3x3 matrix can raise, keep or lower the variance).
- Theorem 2 (Section 2.1): the expected variance after deflating the k
  largest singular triplets when the singular vectors are random unitary,
  from the mean mu_k and variance V_k of the N - k remaining values; Remark 4
  (k = 0) and the Corollary (when deflation lowers the expected variance).
  Reading for Hermitian matrices: the values are the eigenvalues with their
  signs (the right singular vector of an eigenvalue of negative sign is minus
  the left one, so the cross terms of the proof carry the product of signs);
  for a positive definite matrix they are the singular values, as printed.
- The distance profile W_d of Section 6.2: for sampled rows i, the mean of
  |B_ij|^2 over the entries j whose lattice site lies at torus Manhattan
  distance d from the site of i.
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


# --------------------------------------------------------------------------
# Theorem 2, Remark 4, Corollary (Section 2.1)
# --------------------------------------------------------------------------
def _remaining(values, k: int):
    v = np.asarray(values, dtype=np.float64)
    order = np.argsort(-np.abs(v), kind="stable")
    return v[order][:k], v[order][k:]


def theorem2_expected_variance(values, k: int, hermitian: bool) -> float:
    """E(Var(t(A_R))) after deflating the k values of largest modulus:
    (N - k)(1 - 1/N)(V_k + mu_k^2) for non-Hermitian A, and
    (N - k)(V_k N / (N + 1) + mu_k^2 k / (N + 1)) for Hermitian A."""
    N = len(values)
    _, r = _remaining(values, k)
    if len(r) == 0:
        return 0.0
    mu = float(np.mean(r))
    Vk = float(np.mean((r - mu) ** 2))
    if not hermitian:
        return (N - k) * (1.0 - 1.0 / N) * (Vk + mu ** 2)
    return (N - k) * (Vk * N / (N + 1) + mu ** 2 * k / (N + 1))


def remark4_undeflated(values, hermitian: bool) -> float:
    """k = 0: (N - 1)(V_0 + mu_0^2) non-Hermitian, N^2 V_0 / (N + 1) Hermitian."""
    v = np.asarray(values, dtype=np.float64)
    N = len(v)
    mu, V0 = float(np.mean(v)), float(np.var(v))
    return (N - 1) * (V0 + mu ** 2) if not hermitian else N * N * V0 / (N + 1)


def corollary_hermitian_reduces(values, k: int) -> bool:
    """Deflation lowers the expected variance of a Hermitian A iff
    mu_0^2 - ((N - k) / N)^2 mu_k^2 < (1/N) sum_{i <= k} sigma_i^2."""
    v = np.asarray(values, dtype=np.float64)
    N = len(v)
    top, r = _remaining(v, k)
    mu0, muk = float(np.mean(v)), float(np.mean(r))
    return mu0 ** 2 - ((N - k) / N) ** 2 * muk ** 2 < float(np.sum(top ** 2)) / N


def haar_unitary(N: int, rs) -> np.ndarray:
    """A Haar-distributed N x N unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    Z = (rs.standard_normal((N, N)) + 1j * rs.standard_normal((N, N))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R)
    return Q * (d / np.abs(d))[None, :]


def random_vector_matrix(values, rs, hermitian: bool):
    """(A, A_R-builder) with the given spectrum and Haar singular vectors:
    A = U diag(sigma) V^H with independent U, V, or U diag(lambda) U^H."""
    v = np.asarray(values, dtype=np.float64)
    order = np.argsort(-np.abs(v), kind="stable")
    v = v[order]
    N = len(v)
    U = haar_unitary(N, rs)
    V = U if hermitian else haar_unitary(N, rs)
    A = (U * v) @ V.conj().T

    def remainder(k):
        return (U[:, k:] * v[k:]) @ V[:, k:].conj().T

    return A, remainder


# --------------------------------------------------------------------------
# distance profile W_d (Section 6.2)
# --------------------------------------------------------------------------
def torus_distance(a, b, L) -> int:
    """Manhattan distance of two sites on the periodic lattice."""
    d = 0
    for mu in range(4):
        x = abs(a[mu] - b[mu])
        d += min(x, L[mu] - x)
    return d


def distance_counts(L) -> np.ndarray:
    """m_d: the number of entries (12 per site) at distance d from a site."""
    from .lattice import site_coords, volume
    V = volume(L)
    o = site_coords(0, L)
    m = np.zeros(sum(l // 2 for l in L) + 1, dtype=np.int64)
    for n in range(V):
        m[torus_distance(o, site_coords(n, L), L)] += 12
    return m


def distance_sums(v: np.ndarray, i: int, L) -> np.ndarray:
    """sum of |v_j|^2 over the entries j whose site lies at distance d from the
    site of entry i, for every d (v: one row of B, length 12 V)."""
    from .lattice import site_coords, volume
    V = volume(L)
    si = site_coords(i // 12, L)
    out = np.zeros(sum(l // 2 for l in L) + 1)
    for n in range(V):
        out[torus_distance(si, site_coords(n, L), L)] += float(np.sum(np.abs(v[12 * n:12 * n + 12]) ** 2))
    return out


def distance_profile(B: np.ndarray, rows, L):
    """(W, m): W[a][d] = distance_sums(row rows[a] of B)[d] / m_d; the profile
    W_d of the paper is the mean of W over the sampled rows."""
    m = distance_counts(L)
    W = np.array([distance_sums(B[i], i, L) for i in rows])
    return W / m[None, :], m
