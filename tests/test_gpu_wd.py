"""GPU parity of the distance profile W_d (Section 6.2; dht_distance_profile)
against the oracle (oracle/theory.py, pinned by ring-distance counts, the row
sum rule, the probing mask's pattern and g5-hermiticity).

- c1 (4^4, dense inverse): 17 rows (batches of 16 + 1), B = D^-1 and
  D^-1 - P (FP64 basis, Galerkin M), with and without the mask of 32
  hierarchical-probing vectors; each W[r][d] to 1e-9 of the row's largest
  (solves to 1e-12), the masked distances d % 4 != 0 exactly 0, m_d equal.
- c2 (8^3 x 16): 3 rows with a BF16 random basis and the diagonal M, against
  columns from the C oracle's BiCGStab (1e-12) minus the oracle's deflation
  term, to 1e-7 of the row's largest (mixed-precision solves to 1e-10).
- report: the four profiles of the paper's figure (plain, deflated, 32 HP
  vectors, both) at 8^3 x 16 with 64 eigenvectors of Q, written to
  wd_profile_c2.json in the directory DHT_REPORT_DIR names, if it is set.
"""
import json

import numpy as np
import pytest

from oracle import estimator, lattice, stencil, theory
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links
from reports import write_report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_1603_05988_amd import _lib as L
    return L


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    D = lattice.dense_wilson(U, w.L, w.mass)
    ctx = _lib().Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    yield w, D, ctx
    ctx.close()


@pytest.mark.parametrize("deflate", [False, True])
@pytest.mark.parametrize("hp", [0, 32])
def test_profile_c1(c1, deflate, hp):
    w, D, ctx = c1
    L = _lib()
    N = D.shape[0]
    g5 = lattice.gamma5_full(w.V)
    B = estimator.exact_inverse(D)
    if deflate:
        lam, W = estimator.q_eigenpairs(D, g5, w.k)
        ctx.set_deflation(cuda(W.T), L.FP64)
        B = B - estimator.deflation_matrix(W, estimator.galerkin_M(W, D, g5), g5)
    if hp:
        from oracle import rng
        col = np.repeat(rng.hp_colours(w.L), 12)
        B = np.where((col[:, None] & (hp - 1)) == (col[None, :] & (hp - 1)), B, 0)
    rs = np.random.default_rng(4)
    rows = np.concatenate([[5, 400, 2000, N - 1], rs.choice(N, 13, replace=False)])
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    Wg, m = ctx.distance_profile(rows, prm, deflate=deflate, hp_vectors=hp)
    Wr, mr = theory.distance_profile(B, rows, w.L)
    assert np.array_equal(m, mr)
    for a in range(len(rows)):
        assert np.abs(Wg[a] - Wr[a]).max() <= 1e-9 * Wr[a].max(), (a, np.abs(Wg[a] - Wr[a]).max(), Wr[a].max())
    if hp:
        d = np.arange(Wg.shape[1])
        assert np.all(Wg[:, d % 4 != 0] == 0)
    if deflate:
        ctx.clear_deflation()


def test_profile_c2_bf16_basis():
    w = WORKLOADS["c2"]
    L = _lib()
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    N = 12 * w.V
    k = 20
    rs = np.random.default_rng(5)
    W = rs.standard_normal((N, k)) + 1j * rs.standard_normal((N, k))
    W /= np.linalg.norm(W, axis=0)
    ctx.set_deflation(cuda(W.T), L.BF16, diagonal=True)
    f = np.stack([W.real, W.imag], axis=-1).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    f = u.astype(np.uint32).view(np.float32).astype(np.float64)
    Wr = f[..., 0] + 1j * f[..., 1]
    g5 = lattice.gamma5_full(w.V)
    rq = np.array([np.vdot(Wr[:, i], g5 * stencil.apply_D(U, w.L, w.mass, Wr[:, i])).real for i in range(k)])
    rows = np.array([7, 40000, N - 3])
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10)
    Wg, m = ctx.distance_profile(rows, prm, deflate=True)
    for a, i in enumerate(rows):
        e = np.zeros(N, dtype=np.complex128)
        e[i] = 1.0
        x, status, _, res = stencil.solve(U, w.L, w.mass, e, 1e-12, 20000)
        assert res <= 1e-12
        col = x - Wr @ ((1.0 / rq) * (g5[i] * Wr[i].conj()))
        ref = theory.distance_sums(col, i, w.L) / m
        assert np.abs(Wg[a] - ref).max() <= 1e-7 * ref.max(), (a, np.abs(Wg[a] - ref).max(), ref.max())
    ctx.close()


def test_report_profiles_c2():
    w = WORKLOADS["c2"]
    L = _lib()
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    lam, res, st, td = ctx.eigensolve(w.k, L.FP64, tol=1e-9, max_iter=400, degree=16, seed=11)
    rs = np.random.default_rng(6)
    rows = rs.choice(12 * w.V, 10, replace=False)
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10)
    out = {"lattice": list(w.L), "k": int(w.k), "rows": rows.tolist()}
    for name, defl, hp in (("monte_carlo", False, 0), ("deflation", True, 0), ("hp32", False, 32),
                           ("hp32_deflation", True, 32)):
        Wg, m = ctx.distance_profile(rows, prm, deflate=defl, hp_vectors=hp)
        out[name] = Wg.mean(axis=0).tolist()
    out["m_d"] = m.tolist()
    # squared row norms: deflating (near-)exact eigenvectors removes sigma_m^2 |u_im|^2
    # from every row, and the mask drops entries; the combination is reported
    tot = {n: float(np.dot(out[n], m)) for n in ("monte_carlo", "deflation", "hp32", "hp32_deflation")}
    out["row_norm2"] = tot
    print(json.dumps(out))
    assert tot["deflation"] < tot["monte_carlo"] and tot["hp32"] < tot["monte_carlo"]
    write_report("wd_profile_c2.json", out)
    ctx.close()


def test_profile_c1_fp32_basis_full_M(c1):
    """The deflated profile with an FP32 basis and the Galerkin M of the stored vectors."""
    w, D, ctx = c1
    L = _lib()
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, 12)
    ctx.set_deflation(cuda(W.T), L.FP32)
    f = np.stack([W.real, W.imag], axis=-1).astype(np.float32).astype(np.float64)
    Wr = f[..., 0] + 1j * f[..., 1]
    B = estimator.exact_inverse(D) - estimator.deflation_matrix(Wr, estimator.galerkin_M(Wr, D, g5), g5)
    rows = np.array([0, 1234, 3000])
    Wg, m = ctx.distance_profile(rows, ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12), deflate=True)
    Wref, _ = theory.distance_profile(B, rows, w.L)
    for a in range(len(rows)):
        assert np.abs(Wg[a] - Wref[a]).max() <= 1e-9 * Wref[a].max()
    ctx.clear_deflation()
