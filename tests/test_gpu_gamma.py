"""GPU parity of the traces Tr(Gamma D^-1) over one deflation space (end of
Section 5.2): dht_gamma_set, dht_trace_gamma_batch and dht_gamma_estimate_get
against the oracle (oracle/gamma.py) on the same seeded probes.

- c1 (4^4, dense inverse): the 16 Dirac-basis matrices and a random complex
  matrix, with FP64, FP32 and BF16 bases (FP64 / FP32 take the generic FP64
  spin-pair projection, BF16 the MFMA one over exact probe codes).  T_D(Gamma)
  to 1e-10 relative (FP64 sums over the stored basis, whatever its storage);
  q = z^H Gamma x to 1e-10 of max |q| (solves to 1e-12); the deflation
  corrections z^H Gamma P z to 1e-10 of max |q| on the FP64 paths, and on the
  MFMA path within the first-order bound of its FP32 chunk sums (each
  spin-pair coefficient W_s^H z_t off by at most 32 * 2^-24 * sum |w|, as in
  the plain projection).
- Gamma = 1 gives dht_trace_batch's q and q_defl.
- ragged batches of 1, 5 and 23 probes (MFMA passes of 16 + 7).
- the running estimates per matrix are the sample statistics of the records,
  with T_D(Gamma) added to the deflated mean.
- c2 (8^3 x 16): a BF16 random basis with the diagonal M, corrections against
  the oracle (M from the C oracle's stencil) on 16 probes.
"""
import numpy as np
import pytest

from oracle import estimator, gamma, lattice, rng, stencil
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_1603_05988_amd import _lib as L
    return L


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def round_storage(W, prec):
    if prec == 0:
        return W
    f = np.stack([W.real, W.imag], axis=-1).astype(np.float32)
    if prec == 2:
        u = f.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        f = u.astype(np.uint32).view(np.float32)
    f = f.astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]


def gammas():
    _, B = gamma.dirac_basis()
    rs = np.random.default_rng(17)
    R = rs.standard_normal((4, 4)) + 1j * rs.standard_normal((4, 4))
    return np.concatenate([B, R[None]])


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    D = lattice.dense_wilson(U, w.L, w.mass)
    ctx = _lib().Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    yield w, D, estimator.exact_inverse(D), g5, W, ctx
    ctx.close()


def mfma_bound(Wr, M, g5, Z, G):
    """First-order bound on |d_gpu - d_ref| from coefficient errors
    e_i = 32 * 2^-24 * sum |w_i| in every spin-pair projection."""
    e = 32 * 2.0 ** -24 * np.abs(Wr).sum(axis=0)
    c1 = gamma.gamma_projection(Wr, Z, G)            # k x s
    c2 = Wr.conj().T @ (g5[:, None] * Z.T)
    v = M @ c2
    g1 = np.abs(G).sum()
    return (g1 * e) @ np.abs(v) + np.abs(c1).T @ (np.abs(M) @ (4 * e)) + 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_gamma_traces_c1(c1, prec):
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    ctx.set_deflation(cuda(W.T), prec)
    Wr = round_storage(W, prec)
    M = estimator.galerkin_M(Wr, D, g5)
    G = gammas()
    td = ctx.gamma_set(G)
    for g in range(len(G)):
        ref = gamma.gamma_deflated_trace(Wr, M, g5, G[g])
        assert abs(td[g] - ref) <= 1e-10 * max(1.0, abs(ref)), (g, td[g], ref)
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    first, n = 3, 16
    q, qd, stats = ctx.trace_gamma_batch(w.seed, 1, False, first, n, prm)
    Z = rng.probes(w.L, w.seed, 1, False, first, n)
    X = Z @ Dinv.T
    for g in range(len(G)):
        q_ref = gamma.gamma_quadratic_forms(Z, X, G[g])
        d_ref = gamma.gamma_corrections(Wr, M, g5, Z, G[g])
        scale = np.abs(q_ref).max()
        assert np.abs(q[g] - q_ref).max() <= 1e-10 * scale, g
        d = q[g] - qd[g]
        if prec == 2:
            bound = mfma_bound(Wr, M, g5, Z, G[g]) + 1e-12 * scale
            assert np.all(np.abs(d - d_ref) <= bound), (g, np.abs(d - d_ref).max(), bound.min())
        else:
            assert np.abs(d - d_ref).max() <= 1e-10 * scale, (g, np.abs(d - d_ref).max())
    # the running estimates are the records' statistics
    for g in (0, 15, 16):
        est = ctx.gamma_estimate(g)
        m, var, _, _ = estimator.sample_statistics(q[g])
        md, vard, _, _ = estimator.sample_statistics(qd[g])
        assert est["n"] == n
        assert abs(complex(est["mean_re"], est["mean_im"]) - m) <= 1e-12 * max(1.0, abs(m))
        assert abs(complex(est["TD_re"], est["TD_im"]) - td[g]) <= 1e-14 * max(1.0, abs(td[g]))
        assert abs(complex(est["mean_defl_re"], est["mean_defl_im"]) - (md + td[g])) <= 1e-10 * max(1.0, abs(m))
        assert abs(est["var_defl"] - vard) <= 1e-8 * max(vard, 1e-300)
    ctx.clear_deflation()


def test_identity_matches_trace_batch(c1):
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    for prec in (0, 2):
        ctx.set_deflation(cuda(W.T), prec)
        ctx.gamma_set(np.eye(4)[None])
        prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
        q, qd, _ = ctx.trace_gamma_batch(w.seed, 0, True, 0, 16, prm)
        recs = ctx.trace_batch(w.seed, 0, True, 0, 16, prm)
        q0 = np.array([r["q"] for r in recs])
        qd0 = np.array([r["q_defl"] for r in recs])
        scale = np.abs(q0).max()
        assert np.abs(q[0] - q0).max() <= 1e-11 * scale
        # the MFMA spin-pair sums (16 pairs) and the plain ones (chirality halves)
        # take different FP32 chunk sums: both sit within the projection's bound
        tol = 1e-11 if prec == 0 else 1e-5
        assert np.abs(qd[0] - qd0).max() <= tol * scale, (prec, np.abs(qd[0] - qd0).max())
        ctx.clear_deflation()


@pytest.mark.parametrize("n", [1, 5, 23])
def test_ragged_batches_bf16(c1, n):
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    ctx.set_deflation(cuda(W.T), L.BF16)
    Wr = round_storage(W, 2)
    M = estimator.galerkin_M(Wr, D, g5)
    G = gammas()[[1, 6, 15, 16]]
    ctx.gamma_set(G)
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10)
    q, qd, stats = ctx.trace_gamma_batch(w.seed, 2, True, 7, n, prm)
    Z = rng.probes(w.L, w.seed, 2, True, 7, n)
    X = Z @ Dinv.T
    for g in range(len(G)):
        q_ref = gamma.gamma_quadratic_forms(Z, X, G[g])
        d_ref = gamma.gamma_corrections(Wr, M, g5, Z, G[g])
        scale = np.abs(q_ref).max()
        assert np.abs(q[g] - q_ref).max() <= 1e-8 * scale
        bound = mfma_bound(Wr, M, g5, Z, G[g]) + 1e-12 * scale
        assert np.all(np.abs((q[g] - qd[g]) - d_ref) <= bound)
    assert all(s["true_resid"] <= 1e-10 for s in stats)
    ctx.clear_deflation()


def test_without_basis_and_errors(c1):
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    ctx.clear_deflation()
    G = gammas()[[0, 4]]
    td = ctx.gamma_set(G)
    assert np.all(td == 0)
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    q, qd, _ = ctx.trace_gamma_batch(w.seed, 3, False, 0, 4, prm)
    assert np.array_equal(q, qd)
    Z = rng.probes(w.L, w.seed, 3, False, 0, 4)
    q_ref = gamma.gamma_quadratic_forms(Z, Z @ Dinv.T, G[1])
    assert np.abs(q[1] - q_ref).max() <= 1e-10 * np.abs(q_ref).max()
    with pytest.raises(RuntimeError):
        ctx.gamma_set(np.zeros((0, 4, 4)))
    bad = np.eye(4, dtype=np.complex128)[None].copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(RuntimeError):
        ctx.gamma_set(bad)
    with pytest.raises(RuntimeError):
        ctx.gamma_estimate(5)


def test_gamma_corrections_c2_bf16_diagonal():
    w = WORKLOADS["c2"]
    L = _lib()
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    N = 12 * w.V
    k = 24
    rs = np.random.default_rng(23)
    W = rs.standard_normal((N, k)) + 1j * rs.standard_normal((N, k))
    W /= np.linalg.norm(W, axis=0)
    ctx.set_deflation(cuda(W.T), L.BF16, diagonal=True)
    Wr = round_storage(W, 2)
    g5 = lattice.gamma5_full(w.V)
    rq = np.array([np.vdot(Wr[:, i], g5 * stencil.apply_D(U, w.L, w.mass, Wr[:, i])).real for i in range(k)])
    M = np.diag(1.0 / rq)
    G = gammas()[[0, 5, 10, 15, 16]]
    td = ctx.gamma_set(G)
    for g in range(len(G)):
        ref = gamma.gamma_deflated_trace(Wr, M, g5, G[g])
        assert abs(td[g] - ref) <= 1e-10 * max(1.0, abs(ref))
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-8)
    q, qd, stats = ctx.trace_gamma_batch(w.seed, 0, True, 0, 16, prm)
    Z = rng.probes(w.L, w.seed, 0, True, 0, 16)
    for g in range(len(G)):
        d_ref = gamma.gamma_corrections(Wr, M, g5, Z, G[g])
        bound = mfma_bound(Wr, M, g5, Z, G[g]) + 1e-12 * np.abs(q[g]).max()
        assert np.all(np.abs((q[g] - qd[g]) - d_ref) <= bound), g
    ctx.close()


def test_two_row_tiles_and_four_slices(c1):
    """k = 40 (two MFMA row tiles of 32, the second padded) and 64 probes (four
    spin-pair passes of 16) with a BF16 basis and a full Galerkin M."""
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    lam, W40 = estimator.q_eigenpairs(D, g5, 40)
    ctx.set_deflation(cuda(W40.T), L.BF16)
    Wr = round_storage(W40, 2)
    M = estimator.galerkin_M(Wr, D, g5)
    G = gammas()[[2, 9, 16]]
    td = ctx.gamma_set(G)
    for g in range(len(G)):
        ref = gamma.gamma_deflated_trace(Wr, M, g5, G[g])
        assert abs(td[g] - ref) <= 1e-10 * max(1.0, abs(ref))
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    q, qd, _ = ctx.trace_gamma_batch(w.seed, 4, False, 0, 64, prm)
    Z = rng.probes(w.L, w.seed, 4, False, 0, 64)
    for g in range(len(G)):
        d_ref = gamma.gamma_corrections(Wr, M, g5, Z, G[g])
        bound = mfma_bound(Wr, M, g5, Z, G[g]) + 1e-12 * np.abs(q[g]).max()
        assert np.all(np.abs((q[g] - qd[g]) - d_ref) <= bound), g
    ctx.clear_deflation()


def test_largest_batch_and_most_matrices(c1):
    """DHT_MAX_BATCH probes in one call (FP64 basis: one generic spin-pair pass over
    256 columns) and DHT_MAX_GAMMA random matrices at once."""
    w, D, Dinv, g5, W, ctx = c1
    L = _lib()
    ctx.set_deflation(cuda(W.T), L.FP64)
    M = estimator.galerkin_M(W, D, g5)
    rs = np.random.default_rng(29)
    G = rs.standard_normal((64, 4, 4)) + 1j * rs.standard_normal((64, 4, 4))
    td = ctx.gamma_set(G)
    for g in (0, 31, 63):
        ref = gamma.gamma_deflated_trace(W, M, g5, G[g])
        assert abs(td[g] - ref) <= 1e-10 * max(1.0, abs(ref))
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    q, qd, stats = ctx.trace_gamma_batch(w.seed, 5, False, 0, 256, prm)
    assert q.shape == (64, 256)
    Z = rng.probes(w.L, w.seed, 5, False, 0, 256)
    X = Z @ Dinv.T
    for g in (0, 17, 63):
        q_ref = gamma.gamma_quadratic_forms(Z, X, G[g])
        d_ref = gamma.gamma_corrections(W, M, g5, Z, G[g])
        scale = np.abs(q_ref).max()
        assert np.abs(q[g] - q_ref).max() <= 1e-10 * scale
        assert np.abs((q[g] - qd[g]) - d_ref).max() <= 1e-10 * scale
    with pytest.raises(RuntimeError):
        ctx.gamma_set(np.zeros((65, 4, 4)))
    ctx.clear_deflation()
