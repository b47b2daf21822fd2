"""Parity at the full 32^3x64 size (N = 25,165,824), in the launch configuration
bench.py times (autotuned hop shapes, batches of 16 hierarchical probes, BF16
inner storage with FP64 defect correction, k = 1000 BF16 deflation basis),
on outputs the oracle can compute one by one or on properties that hold at
any size:

- gamma5-hermiticity of the FP64 operator, <phi, D psi> = <D^H phi, psi>,
  on two random fields (relative 1e-12);
- the true relative residual ||z - D x|| / ||z|| of two sampled solutions of
  a 16-probe batch, recomputed by the oracle's C stencil from the oracle's own
  probes (<= 1e-8, the solve tolerance);
- bit-exact projection coefficients W^H z and W^H g5 z for sampled
  (column, probe) pairs: the basis entries are (+-1 +- i) 2^-13, exact in BF16,
  and every partial sum of their products with Z4 probes is exact in FP32 and
  FP64, so the MFMA path must reproduce the oracle's sums exactly;
- q = z^H x of the timed trace_batch path against the oracle's C-stencil
  solve, and the 16 Dirac-matrix quadratic forms z^H Gamma x of the
  Gamma-trace path against the same oracle solves.
"""
import numpy as np
import pytest

from oracle import lattice, rng, stencil
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links, hashed_basis, random_spinors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W5 = WORKLOADS["c5"]


def _lib():
    from paper_1603_05988_amd import _lib as L
    return L


@pytest.fixture(scope="module")
def c5():
    Lb = _lib()
    U = gauge_links(W5.L, W5.eps, W5.seed)
    ctx = Lb.Context(W5.L, W5.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    for prec in (Lb.FP64, Lb.BF16):   # the shapes bench.py times
        ctx.autotune_hop(prec, W5.batch, reps=3)
    yield U, ctx
    ctx.close()


def test_c5_gamma5_hermiticity(c5):
    U, ctx = c5
    Lb = _lib()
    X = random_spinors(W5.L, 2, 17)
    phi = torch.from_numpy(X[0:1]).cuda()
    psi = torch.from_numpy(X[1:2]).cuda()
    Dpsi = ctx.apply(psi, Lb.OP_D, Lb.FP64)
    Dhphi = ctx.apply(phi, Lb.OP_DDAG, Lb.FP64)
    a = torch.vdot(phi.flatten(), Dpsi.flatten()).item()
    b = torch.vdot(Dhphi.flatten(), psi.flatten()).item()
    assert abs(a - b) <= 1e-12 * abs(a), (a, b)


def test_c5_mixed_solve_true_residual_by_oracle(c5):
    U, ctx = c5
    Lb = _lib()
    B = W5.batch
    Z = ctx.make_probes(W5.seed, 0, W5.hp, 0, B)
    prm = ctx.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.BF16, tol=W5.tol, maxiter=5000)
    X, stats, rc = ctx.solve(Z, prm)
    assert all(s["true_resid"] <= W5.tol for s in stats), stats
    del Z
    for r in (0, B - 1):
        z = rng.probe(W5.L, W5.seed, 0, W5.hp, r)
        x = X[r].cpu().numpy().ravel()
        res = z - stencil.apply_D(U, W5.L, W5.mass, x)
        rel = np.linalg.norm(res) / np.linalg.norm(z)
        assert rel <= W5.tol, (r, rel, stats[r])
        assert abs(rel - stats[r]["true_resid"]) <= 1e-3 * W5.tol + 1e-3 * rel


@pytest.fixture(scope="module")
def c5_basis(c5):
    U, ctx = c5
    Lb = _lib()
    k, N = W5.k, W5.N
    ctx.begin_deflation(k, Lb.BF16)
    for j in range(0, k, 32):
        cols = list(range(j, min(k, j + 32)))
        Wb = hashed_basis(cols, N, 11, xp=torch, device="cuda")
        ctx.set_deflation_columns(j, Wb)
        del Wb
    torch.cuda.empty_cache()
    ctx.finalize_deflation(diagonal=True)
    yield U, ctx
    ctx.set_projection_window(0)
    ctx.clear_deflation()


def _check_exact(c1, c2, first, rows):
    g5 = lattice.gamma5_full(W5.V)
    for r in rows:
        z = rng.probe(W5.L, W5.seed, 0, W5.hp, first + r)
        for i in (0, 517, W5.k - 1):
            w = hashed_basis([i], W5.N, 11)[0]
            e1 = np.vdot(w, z)
            e2 = np.vdot(w, g5 * z)
            assert c1[i, r] == e1 and c2[i, r] == e2, (i, first + r, c1[i, r], e1, c2[i, r], e2)


def test_c5_projection_sampled_exact(c5_basis):
    U, ctx = c5_basis
    c1, c2 = ctx.project_probes(W5.seed, 0, W5.hp, 0, W5.batch)
    _check_exact(c1, c2, 0, (0, 7, W5.batch - 1))


def test_c5_projection_window_exact(c5_basis):
    """The 64-probe projection window bench.py times: the batch that opens the
    window and one that reuses it get the exact coefficients of their probes."""
    U, ctx = c5_basis
    Lb = _lib()
    B = W5.batch
    prm = ctx.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.BF16, tol=W5.tol, maxiter=5000)
    ctx.set_projection_window(4 * B)
    for first in (0, 2 * B):
        recs, c1, c2 = ctx.trace_batch(W5.seed, 0, W5.hp, first, B, prm, want_coef=True)
        assert all(r["true_resid"] <= W5.tol for r in recs)
        _check_exact(c1, c2, first, (0, B - 1))
    ctx.set_projection_window(0)


def test_c5_quadratic_forms_vs_oracle_solve(c5_basis):
    """q = z^H x of the timed trace_batch path (BF16 probes, fused z^H x in
    the final residual hops, predicted final check, in-place residual updates,
    64-probe projection window) for two probes of a 32^3x64 batch, against
    z^H x* with x* from the oracle's C-stencil FP64 BiCGStab to 1e-10:
    relative 1e-8 (the tolerance after mixed-precision refinement)."""
    U, ctx = c5_basis
    Lb = _lib()
    B = W5.batch
    prm = ctx.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.BF16, tol=W5.tol, maxiter=5000)
    ctx.set_projection_window(4 * B)
    recs = ctx.trace_batch(W5.seed, 0, W5.hp, B, B, prm)
    ctx.set_projection_window(0)
    for r in (0, B - 1):
        z = rng.probe(W5.L, W5.seed, 0, W5.hp, B + r)
        x, st, it, rr = stencil.solve(U, W5.L, W5.mass, z, 1e-10, 5000)
        assert st == 0 and rr <= 1e-10, (st, it, rr)
        qs = np.vdot(z, x.ravel())
        q = recs[r]["q"]
        print("probe %d: q = %.12e%+.12ei, oracle %.12e%+.12ei, rel %.2e" % (B + r, q.real, q.imag, qs.real,
                                                                            qs.imag, abs(q - qs) / abs(qs)))
        assert abs(q - qs) <= 1e-8 * abs(qs), (r, q, qs)


def test_c5_gamma_traces_vs_oracle_solve(c5_basis):
    """Tr(Gamma D^-1) for the 16 Dirac matrices at the full size, the way bench.py
    times it (one solve per probe, spin-pair projection on the k = 1000 BF16
    basis): z^H Gamma x of two sampled probes against z^H Gamma x* with x* from
    the oracle's C-stencil FP64 BiCGStab to 1e-10, within 1e-8 of |z^H x*|; with
    Gamma = 1 the deflated quadratures equal those of dht_trace_batch on the
    same probes up to the FP32 chunk sums of the two projections."""
    from oracle import gamma
    U, ctx = c5_basis
    Lb = _lib()
    B = W5.batch
    prm = ctx.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.BF16, tol=W5.tol, maxiter=5000)
    _, G = gamma.dirac_basis()
    ctx.gamma_set(G)
    q, qd, stats = ctx.trace_gamma_batch(W5.seed, 0, W5.hp, 3 * B, B, prm)
    assert all(s["true_resid"] <= W5.tol for s in stats)
    for r in (0, B - 1):
        z = rng.probe(W5.L, W5.seed, 0, W5.hp, 3 * B + r)
        x, st, it, rr = stencil.solve(U, W5.L, W5.mass, z, 1e-10, 5000)
        assert st == 0 and rr <= 1e-10, (st, it, rr)
        scale = abs(np.vdot(z, x.ravel()))
        for g in range(16):
            ref = gamma.gamma_quadratic_forms(z[None], x.ravel()[None], G[g])[0]
            assert abs(q[g, r] - ref) <= 1e-8 * scale, (r, g, q[g, r], ref)
    recs = ctx.trace_batch(W5.seed, 0, W5.hp, 3 * B, B, prm)
    qd1 = np.array([rec["q_defl"] for rec in recs])
    q1 = np.array([rec["q"] for rec in recs])
    assert np.abs(q[0] - q1).max() <= 1e-8 * np.abs(q1).max()
    assert np.abs(qd[0] - qd1).max() <= 1e-6 * np.abs(q1).max()
