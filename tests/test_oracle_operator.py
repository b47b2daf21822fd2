"""Pins of the oracle's Wilson-Dirac operator against facts fixed independently of it.

- gamma algebra of the chiral basis;
- g5-hermiticity g5 D g5 = D^H (holds for any gauge field);
- free field: singular values and Tr D^-1 from the closed momentum-space form
  (the paper completes its spectrum with the free-field spectrum, Section 6);
- a free-field plane wave is mapped to (M(p) + i sum g_mu sin p_mu) times itself,
  which fixes the hop sign convention and the antiperiodic time boundary;
- gauge covariance D[U^g] = G D[U] G^H fixes where each link enters;
- the dense matrix and the independent C stencil agree, including a lattice
  with an extent-2 direction (forward and backward neighbours coincide);
- Tr D^-1 from LU equals sum 1/eig(D), and is real (g5-hermiticity).
"""
import numpy as np
import pytest

from oracle import estimator, lattice, stencil
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links, random_gauge_transform, random_spinors


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    D = lattice.dense_wilson(U, w.L, w.mass)
    return w, U, D


def test_gamma_algebra():
    g, g5 = lattice.gamma_matrices()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 4), (4, 2, 2, 6)])
def test_gamma5_hermiticity(L):
    U = gauge_links(L, 0.7, 11)
    D = lattice.dense_wilson(U, L, -0.3)
    g5 = lattice.gamma5_full(lattice.volume(L))
    assert np.abs(g5[:, None] * D * g5[None, :] - D.conj().T).max() <= 1e-14


@pytest.mark.parametrize("L,m", [((4, 4, 4, 4), -0.2), ((2, 4, 2, 6), 0.1), ((4, 4, 2, 8), -0.5)])
def test_free_field_spectrum_and_trace(L, m):
    V = lattice.volume(L)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, L[3], L[2], L[1], L[0], 3, 3)).copy()
    D = lattice.dense_wilson(U, L, m)
    s = np.sort(np.linalg.svd(D, compute_uv=False))
    ref = lattice.free_field_singular_values(L, m)
    assert len(s) == 12 * V
    assert np.abs(s - ref).max() <= 1e-12 * ref.max()
    tr = estimator.trace_inverse_lu(D)
    tr_ref = lattice.free_field_trace_inverse(L, m)
    assert abs(tr - tr_ref) <= 1e-10 * abs(tr_ref)


def test_free_field_plane_wave():
    L = (4, 4, 4, 6)
    m = -0.3
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, L[3], L[2], L[1], L[0], 3, 3)).copy()
    D = lattice.dense_wilson(U, L, m)
    g, _ = lattice.gamma_matrices()
    rng = np.random.default_rng(3)
    n = (1, 3, 2, 4)
    p = [2 * np.pi * n[0] / L[0], 2 * np.pi * n[1] / L[1], 2 * np.pi * n[2] / L[2], (2 * n[3] + 1) * np.pi / L[3]]
    u = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    t, z, y, x = np.meshgrid(*[np.arange(L[i]) for i in (3, 2, 1, 0)], indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).ravel()
    psi = (ph[:, None] * u[None, :]).ravel()
    Mp = m + sum(1 - np.cos(pm) for pm in p)
    Dp = Mp * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    expect = (ph[:, None] * (np.kron(Dp, np.eye(3)) @ u)[None, :]).ravel()
    assert np.abs(D @ psi - expect).max() <= 1e-13


def test_gauge_covariance():
    L = (4, 2, 4, 4)
    U = gauge_links(L, 0.9, 5)
    gt = random_gauge_transform(L, 6)
    Ug = np.empty_like(U)
    for mu in range(4):
        shifted = np.roll(gt, -1, axis=3 - mu)   # g(x + mu)
        Ug[mu] = gt @ U[mu] @ np.conj(np.swapaxes(shifted, -1, -2))
    D = lattice.dense_wilson(U, L, 0.05)
    Dg = lattice.dense_wilson(Ug, L, 0.05)
    V = lattice.volume(L)
    G = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    gs = gt.reshape(V, 3, 3)
    for n in range(V):
        G[12 * n:12 * n + 12, 12 * n:12 * n + 12] = np.kron(np.eye(4), gs[n])
    assert np.abs(Dg - G @ D @ G.conj().T).max() <= 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 4), (6, 2, 4, 2)])
def test_dense_matches_c_stencil(L):
    U = gauge_links(L, 0.5, 21)
    D = lattice.dense_wilson(U, L, -0.25)
    psi = random_spinors(L, 1, 4)[0]
    y_dense = D @ psi.ravel()
    y_c = stencil.apply_D(U, L, -0.25, psi).ravel()
    assert np.abs(y_dense - y_c).max() <= 1e-13


def test_trace_two_routes_and_real(c1):
    w, U, D = c1
    t_lu = estimator.trace_inverse_lu(D)
    t_eig = estimator.trace_inverse_eig(D)
    assert abs(t_lu - t_eig) <= 1e-10 * abs(t_lu)
    assert abs(t_lu.imag) <= 1e-10 * abs(t_lu)


def test_c_stencil_bicgstab_solves(c1):
    w, U, D = c1
    b = random_spinors(w.L, 1, 9)[0]
    x, st, it, rr = stencil.solve(U, w.L, w.mass, b, 1e-12, 2000)
    assert st == 0 and rr <= 1e-12
    xd = np.linalg.solve(D, b.ravel())
    assert np.abs(x.ravel() - xd).max() <= 1e-10 * np.abs(xd).max()
