"""Pins of the oracle's estimator, deflation and variance code.

- brute force over all 4^N Z4 vectors (N <= 5): the Hutchinson mean is Tr(A)
  (eq. 1) and the variance is ||offdiag A||_F^2 (eq. variance);
- T_D from eigenvectors of Q = g5 D equals sum u_i^H v_i / sigma_i from the
  SVD (Section 5.2), and M = (W^H Q W)^-1 = Lambda^-1 for exact eigenvectors;
- the exact split Tr D^-1 = T_D + Tr(D^-1 - P) and the deflated variance
  ||offdiag(D^-1 - P)||_F^2 agree with Monte Carlo over the oracle's own
  probes within 5 sigma (a 4th-moment estimate of the error);
- quadratic forms with fsum agree with exact dense values.
"""
import numpy as np
import pytest

from oracle import estimator, lattice, rng
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_brute_force_hutchinson(N):
    rs = np.random.default_rng(N)
    A = rs.standard_normal((N, N)) + 1j * rs.standard_normal((N, N))
    mean, var = estimator.hutchinson_enumeration(A)
    assert abs(mean - np.trace(A)) <= 1e-12 * max(1.0, abs(np.trace(A)))
    assert abs(var - estimator.offdiag_frobenius2(A)) <= 1e-12 * max(1.0, var)


def test_brute_force_sample_statistics_definition():
    q = np.array([1 + 2j, -0.5 + 1j, 3 - 1j, 0.25j])
    mean, var, vre, vim = estimator.sample_statistics(q)
    assert np.isclose(mean, q.mean())
    assert np.isclose(vre, np.var(q.real, ddof=1))
    assert np.isclose(vim, np.var(q.imag, ddof=1))
    assert np.isclose(var, vre + vim)


@pytest.fixture(scope="module")
def c1_dense():
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    D = lattice.dense_wilson(U, w.L, w.mass)
    g5 = lattice.gamma5_full(w.V)
    Dinv = estimator.exact_inverse(D)
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    return w, U, D, g5, Dinv, lam, W


def test_deflated_trace_two_routes(c1_dense):
    w, U, D, g5, Dinv, lam, W = c1_dense
    M = estimator.galerkin_M(W, D, g5)
    assert np.abs(M - np.diag(1.0 / lam)).max() <= 1e-10 * np.abs(1.0 / lam).max()
    T_eig = estimator.deflated_trace(W, M, g5)
    T_svd, s = estimator.trace_deflated_svd(D, w.k)
    assert abs(T_eig - T_svd) <= 1e-12 * abs(T_svd) * 10
    # |lambda| are the k smallest singular values
    assert np.allclose(np.sort(np.abs(lam)), s[:w.k], rtol=1e-10)
    # T_D = sum lambda^-1 w^H g5 w, real
    alt = np.sum((1.0 / lam) * np.einsum("ni,n,ni->i", W.conj(), g5, W))
    assert abs(T_eig - alt) <= 1e-12 * abs(alt)
    assert abs(T_eig.imag) <= 1e-12 * abs(T_eig)


def test_exact_split_and_mc_statistics(c1_dense):
    w, U, D, g5, Dinv, lam, W = c1_dense
    M = estimator.galerkin_M(W, D, g5)
    P = estimator.deflation_matrix(W, M, g5)
    T_D = estimator.deflated_trace(W, M, g5)
    tr = np.trace(Dinv)
    assert abs(tr - (T_D + np.trace(Dinv - P))) <= 1e-12 * abs(tr)
    Z = rng.probes(w.L, w.seed, 0, False, 0, w.nprobe)
    X = Dinv @ Z.T
    q = estimator.quadratic_forms(Z, X.T)
    c1, c2 = estimator.projection_coefficients(W, Z, g5)
    d = estimator.deflation_corrections(c1, c2, M)
    # d_j = z^H P z directly
    assert np.abs(d - np.einsum("ja,ab,jb->j", Z.conj(), P, Z)).max() <= 1e-10 * np.abs(d).max()
    qR = q - d
    s = len(q)
    for samples, exact_tr, A in ((q, tr, Dinv), (qR, tr - T_D, Dinv - P)):
        mean, var, _, _ = estimator.sample_statistics(samples)
        V_exact = estimator.offdiag_frobenius2(A)
        assert abs(mean - exact_tr) <= 5 * np.sqrt(V_exact / s)
        dev = np.abs(samples - exact_tr) ** 2
        sd_var = np.sqrt(np.var(dev, ddof=1) / s)
        assert abs(var - V_exact) <= 5 * sd_var
    # deflating the smallest singular directions lowers this variance
    assert estimator.offdiag_frobenius2(Dinv - P) < estimator.offdiag_frobenius2(Dinv)


def test_quadratic_forms_fsum(c1_dense):
    w, U, D, g5, Dinv, lam, W = c1_dense
    Z = rng.probes(w.L, 5, 1, True, 0, 4)
    X = (Dinv @ Z.T).T
    q = estimator.quadratic_forms(Z, X)
    ref = np.einsum("ja,ab,jb->j", Z.conj(), Dinv, Z)
    assert np.abs(q - ref).max() <= 1e-12 * np.abs(ref).max()
    tr = estimator.running_trace(q, 1.0)
    assert np.isclose(tr[-1], np.mean(q) + 1.0)
