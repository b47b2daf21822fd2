"""Pins of the Tr(Gamma D^-1) oracle (oracle/gamma.py; end of Section 5.2), each
fixed by something other than the oracle's own formulas:

- the Dirac basis: orthonormal under tr(A^H B) / 4, g5 = g_x g_y g_z g_t is
  its last element, and every element squares to +-1;
- full deflation (k = N, every eigenvector of Q = g5 D): P = D^-1, so
  T_D(Gamma) equals Tr(Gamma D^-1) computed from numpy's dense inverse, and
  every probe's deflated quadrature z^H Gamma D^-1 z - z^H Gamma P z is zero,
  for all 16 basis matrices and for a random non-Hermitian Gamma (a
  transposed or unconjugated Gamma in either formula fails here);
- g5 in closed form: Tr(g5 D^-1) = Tr(Q^-1) = sum of 1 / lambda over the
  eigenvalues of Q, and with the k exact eigenpairs of smallest |lambda|,
  T_D(g5) = sum of their 1 / lambda;
- g5-hermiticity D^H = g5 D g5: conj Tr(Gamma D^-1) = Tr(g5 Gamma^H g5 D^-1),
  so Tr(g_mu D^-1) is imaginary and Tr(g5 g_mu D^-1) is real;
- linearity: the deflated quadrature z^H Gamma P z is complex-linear in
  Gamma (an antilinear slip, such as Gamma^T for Gamma^H, breaks it);
- unbiasedness: the mean deflated quadrature over Z4 probes approaches
  Tr(Gamma (D^-1 - P)) within 5 standard errors.
"""
import numpy as np
import pytest

from oracle import estimator, gamma, lattice, rng
from paper_1603_05988_amd.workloads import gauge_links

L_SMALL = (4, 2, 2, 2)
MASS = -0.2


@pytest.fixture(scope="module")
def small():
    U = gauge_links(L_SMALL, 0.4, 11)
    D = lattice.dense_wilson(U, L_SMALL, MASS)
    V = lattice.volume(L_SMALL)
    g5 = lattice.gamma5_full(V)
    Dinv = np.linalg.inv(D)
    return D, Dinv, g5, V


def random_gamma(seed):
    rs = np.random.default_rng(seed)
    return rs.standard_normal((4, 4)) + 1j * rs.standard_normal((4, 4))


def test_dirac_basis():
    labels, B = gamma.dirac_basis()
    assert len(labels) == 16 and labels[0] == "1" and labels[-1] == "xyzt"
    gram = np.einsum("aij,bij->ab", B.conj(), B) / 4
    assert np.abs(gram - np.eye(16)).max() <= 1e-15
    _, g5 = lattice.gamma_matrices()
    assert np.abs(B[-1] - g5).max() == 0
    for m in B:
        sq = m @ m
        assert np.abs(np.abs(sq[0, 0]) - 1) == 0 and np.abs(sq - sq[0, 0] * np.eye(4)).max() == 0


def test_full_deflation_recovers_every_gamma_trace(small):
    D, Dinv, g5, V = small
    N = D.shape[0]
    lam, W = estimator.q_eigenpairs(D, g5, N)
    M = estimator.galerkin_M(W, D, g5)
    _, B = gamma.dirac_basis()
    Z = rng.probes(L_SMALL, 5, 0, False, 0, 6)
    X = Z @ Dinv.T
    for G in list(B) + [random_gamma(1)]:
        exact = np.trace(gamma.gamma_full(G, V) @ Dinv)
        TD = gamma.gamma_deflated_trace(W, M, g5, G)
        assert abs(TD - exact) <= 1e-10 * max(1.0, abs(exact)), (TD, exact)
        q = gamma.gamma_quadratic_forms(Z, X, G)
        d = gamma.gamma_corrections(W, M, g5, Z, G)
        assert np.abs(q - d).max() <= 1e-9 * np.abs(q).max()


def test_g5_closed_forms(small):
    D, Dinv, g5, V = small
    _, g5s = lattice.gamma_matrices()
    Q = g5[:, None] * D
    lam_all = np.linalg.eigvalsh(0.5 * (Q + Q.conj().T))
    exact = gamma.gamma_trace_exact(g5s, Dinv, V)
    assert abs(exact - np.sum(1.0 / lam_all)) <= 1e-10 * abs(exact)
    k = 20
    lam, W = estimator.q_eigenpairs(D, g5, k)
    M = estimator.galerkin_M(W, D, g5)
    TD = gamma.gamma_deflated_trace(W, M, g5, g5s)
    assert abs(TD - np.sum(1.0 / lam)) <= 1e-10 * abs(np.sum(1.0 / lam))


def test_g5_hermiticity(small):
    D, Dinv, g5, V = small
    g, g5s = lattice.gamma_matrices()
    for G in [random_gamma(2), random_gamma(3)]:
        lhs = np.conj(gamma.gamma_trace_exact(G, Dinv, V))
        rhs = gamma.gamma_trace_exact(g5s @ G.conj().T @ g5s, Dinv, V)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    for mu in range(4):
        t_mu = gamma.gamma_trace_exact(g[mu], Dinv, V)
        t_5mu = gamma.gamma_trace_exact(g5s @ g[mu], Dinv, V)
        assert abs(t_mu.real) <= 1e-12 * max(1.0, abs(t_mu))
        assert abs(t_5mu.imag) <= 1e-12 * max(1.0, abs(t_5mu))


def test_corrections_linear_in_gamma(small):
    D, Dinv, g5, V = small
    lam, W = estimator.q_eigenpairs(D, g5, 12)
    M = estimator.galerkin_M(W, D, g5)
    Z = rng.probes(L_SMALL, 6, 0, False, 0, 4)
    G1, G2 = random_gamma(4), random_gamma(5)
    a, b = 0.3 - 1.7j, 2.1 + 0.4j
    lhs = gamma.gamma_corrections(W, M, g5, Z, a * G1 + b * G2)
    rhs = a * gamma.gamma_corrections(W, M, g5, Z, G1) + b * gamma.gamma_corrections(W, M, g5, Z, G2)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()
    td = gamma.gamma_deflated_trace(W, M, g5, a * G1 + b * G2)
    assert abs(td - a * gamma.gamma_deflated_trace(W, M, g5, G1) - b * gamma.gamma_deflated_trace(W, M, g5, G2)) \
        <= 1e-12 * abs(td)


def test_deflated_quadrature_unbiased(small):
    D, Dinv, g5, V = small
    lam, W = estimator.q_eigenpairs(D, g5, 16)
    M = estimator.galerkin_M(W, D, g5)
    P = estimator.deflation_matrix(W, M, g5)
    G = random_gamma(7)
    target = np.trace(gamma.gamma_full(G, V) @ (Dinv - P))
    Z = rng.probes(L_SMALL, 8, 0, False, 0, 3000)
    s = gamma.gamma_quadratic_forms(Z, Z @ Dinv.T, G) - gamma.gamma_corrections(W, M, g5, Z, G)
    err = np.sqrt(np.var(s.real, ddof=1) / len(s) + np.var(s.imag, ddof=1) / len(s))
    assert abs(s.mean() - target) <= 5 * err, (s.mean(), target, err)
