"""Pins of oracle functions that the GPU tests use as references, each fixed by
something other than the function's own formula:

- rayleigh_diag_M: on exact eigenvectors of Q = g5 D it is diag(1 / lambda)
  (closed form: w^H Q w = lambda for unit eigenvectors), its T_D equals
  sum lambda^-1 w^H g5 w and the SVD route sum u^H v / sigma (Section 5.2);
  for one arbitrary vector w, P = w M w^H g5 is the oblique projector with
  P D w = w, and P does not change when w is rescaled;
- galerkin_M: for an arbitrary (non-eigen) block W, P D is a projector onto
  span W: (P D) W = W and (P D)^2 = P D;
- masked_offdiag_frobenius2: the variance over Z4 base vectors of one complete
  hierarchical-probing sweep (Section 6.2's masked Frobenius norm), checked
  against the sample variance of independent runs of the oracle's own HP
  probes (5 sigma, 4th-moment error estimate), with and without deflation;
- running_trace (Algorithm 1, the trace update T_R / j + T_D): constant and
  equal to Tr A when every quadratic form is exact (a diagonal A: z^H A z =
  Tr A for unit-modulus z), equal to Tr A after the complete enumeration of
  all Z4 vectors (exact unbiasedness, eq. 1), and equal to T_D = Tr A at every
  step when the deflated part is A itself (k = N);
- o2_project (the C oracle's projection): a dense W^H z (textbook product).
"""
import numpy as np
import pytest

from oracle import estimator, lattice, rng, stencil
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    D = lattice.dense_wilson(U, w.L, w.mass)
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    return w, D, g5, lam, W


def test_rayleigh_diag_M_on_eigenvectors(c1):
    w, D, g5, lam, W = c1
    M = estimator.rayleigh_diag_M(W, D, g5)
    assert np.abs(M - np.diag(1.0 / lam)).max() <= 1e-10 * np.abs(1.0 / lam).max()
    TD = estimator.deflated_trace(W, M, g5)
    closed = np.sum((1.0 / lam) * np.einsum("ni,n,ni->i", W.conj(), g5, W).real)
    T_svd, _ = estimator.trace_deflated_svd(D, w.k)
    assert abs(TD - closed) <= 1e-12 * abs(closed)
    assert abs(TD - T_svd) <= 1e-10 * abs(T_svd)


def test_rayleigh_diag_M_single_vector_projector(c1):
    w, D, g5, lam, W = c1
    rs = np.random.default_rng(3)
    v = rs.standard_normal((D.shape[0], 1)) + 1j * rs.standard_normal((D.shape[0], 1))
    M = estimator.rayleigh_diag_M(v, D, g5)
    P = estimator.deflation_matrix(v, M, g5)
    assert np.linalg.norm(P @ (D @ v) - v) <= 1e-12 * np.linalg.norm(v)
    # P depends on span(v) only
    P2 = estimator.deflation_matrix(2.5j * v, estimator.rayleigh_diag_M(2.5j * v, D, g5), g5)
    assert np.abs(P2 - P).max() <= 1e-12 * np.abs(P).max()
    # its trace is T_D (Tr P of the dense matrix)
    assert abs(np.trace(P) - estimator.deflated_trace(v, M, g5)) <= 1e-12 * abs(np.trace(P))


def test_galerkin_M_oblique_projector(c1):
    w, D, g5, lam, W = c1
    rs = np.random.default_rng(4)
    X = rs.standard_normal((D.shape[0], 5)) + 1j * rs.standard_normal((D.shape[0], 5))
    M = estimator.galerkin_M(X, D, g5)
    P = estimator.deflation_matrix(X, M, g5)
    PD = P @ D
    assert np.linalg.norm(PD @ X - X) <= 1e-10 * np.linalg.norm(X)
    assert np.abs(PD @ PD - PD).max() <= 1e-10 * np.abs(PD).max()


@pytest.mark.parametrize("deflate", [False, True])
def test_masked_norm_is_the_hp_run_variance(c1, deflate):
    """Runs r = 0..R-1 each sweep the first 2^m hierarchical-probing vectors
    of their own Z4 base vector; the run means scatter with variance
    ||offdiag(M_s . A)||_F^2 (A = D^-1 or D^-1 - P)."""
    w, D, g5, lam, W = c1
    A = estimator.exact_inverse(D)
    if deflate:
        A = A - estimator.deflation_matrix(W, estimator.galerkin_M(W, D, g5), g5)
    m, R = 5, 160
    colours = np.repeat(rng.hp_colours(w.L), 12)
    V_exact = estimator.masked_offdiag_frobenius2(A, colours, m)
    tr = np.trace(A)
    t = np.empty(R, dtype=np.complex128)
    for r in range(R):
        Z = rng.probes(w.L, 77, r, True, 0, 1 << m)
        t[r] = np.mean(np.einsum("ja,ja->j", Z.conj(), Z @ A.T))
    mean, var, _, _ = estimator.sample_statistics(t)
    assert abs(mean - tr) <= 5 * np.sqrt(V_exact / R)
    dev = np.abs(t - tr) ** 2
    assert abs(var - V_exact) <= 5 * np.sqrt(np.var(dev, ddof=1) / R), (var, V_exact)
    # the sweep removes variance: the masked norm is below the plain one
    assert V_exact < estimator.offdiag_frobenius2(A)


def test_running_trace_exact_cases():
    rs = np.random.default_rng(5)
    N = 3
    d = rs.standard_normal(N) + 1j * rs.standard_normal(N)
    Ad = np.diag(d)
    Z = rng.Z4_TABLE[rs.integers(0, 4, size=(40, N))]
    q = np.einsum("ja,ab,jb->j", Z.conj(), Ad, Z)
    assert np.abs(estimator.running_trace(q) - d.sum()).max() <= 1e-13 * abs(d.sum())
    # all 4^N Z4 vectors: the estimate is exactly Tr A
    A = rs.standard_normal((N, N)) + 1j * rs.standard_normal((N, N))
    vals = np.array([1, 1j, -1, -1j])
    grid = np.stack(np.meshgrid(*([np.arange(4)] * N), indexing="ij"), -1).reshape(-1, N)
    Zall = vals[grid]
    qa = np.einsum("ja,ab,jb->j", Zall.conj(), A, Zall)
    assert abs(estimator.running_trace(qa)[-1] - np.trace(A)) <= 1e-12 * abs(np.trace(A))
    # deflating A itself (k = N): T_R stays 0 and the estimate is T_D = Tr A at every step
    Wq, _ = np.linalg.qr(rs.standard_normal((N, N)) + 1j * rs.standard_normal((N, N)))
    g5 = np.ones(N)
    Dm = np.linalg.inv(A)
    M = estimator.galerkin_M(Wq, Dm, g5)
    P = estimator.deflation_matrix(Wq, M, g5)
    TD = estimator.deflated_trace(Wq, M, g5)
    c1_, c2_ = estimator.projection_coefficients(Wq, Z[:10], g5)
    qd = np.einsum("ja,ab,jb->j", Z[:10].conj(), A, Z[:10]) - estimator.deflation_corrections(c1_, c2_, M)
    assert np.abs(P - A).max() <= 1e-10 * np.abs(A).max()
    assert np.abs(estimator.running_trace(qd, TD) - np.trace(A)).max() <= 1e-10 * abs(np.trace(A))


def test_o2_project_matches_dense_product():
    rs = np.random.default_rng(6)
    k, N = 7, 12 * 4 * 4 * 4 * 2
    Wr = rs.standard_normal((k, N)) + 1j * rs.standard_normal((k, N))
    z = rs.standard_normal(N) + 1j * rs.standard_normal(N)
    ref = Wr.conj() @ z
    out = stencil.project(Wr, z)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
