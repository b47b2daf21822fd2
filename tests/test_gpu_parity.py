"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances: FP64 operator 1e-13 relative (rounding of the stencil sum), FP32
1e-6, BF16 element by element within the rounding model of tests/bounds.py
(8-bit significand on links, spinors and output); FP64 solves give q to
1e-10 relative, mixed-precision solves to 1e-8 (solver residual 1e-8); probe
indices and signs bit-exact.
"""
import numpy as np
import pytest

from bounds import bf16_bound_ratio
from oracle import estimator, lattice, rng, stencil
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links, random_spinors

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
    yield w, U, D, ctx
    ctx.close()


@pytest.fixture(scope="module")
def c1_inv(c1):
    w, U, D, ctx = c1
    return estimator.exact_inverse(D)


@pytest.mark.parametrize("nrhs", [1, 3, 16])
def test_apply_fp64_matches_dense(c1, nrhs):
    w, U, D, ctx = c1
    L = _lib()
    X = random_spinors(w.L, nrhs, 100 + nrhs)
    g5 = lattice.gamma5_full(w.V)
    Xv = X.reshape(nrhs, -1)
    refs = {
        L.OP_D: (D @ Xv.T).T,
        L.OP_DDAG: (D.conj().T @ Xv.T).T,
        L.OP_G5: g5[None, :] * Xv,
        L.OP_Q: (g5[:, None] * D @ Xv.T).T,
    }
    for op, ref in refs.items():
        Y = ctx.apply(cuda(X), op, L.FP64).cpu().numpy().reshape(nrhs, -1)
        err = np.abs(Y - ref).max() / np.abs(ref).max()
        assert err <= 1e-13, (op, err)


def test_apply_fp32(c1):
    w, U, D, ctx = c1
    X = random_spinors(w.L, 16, 7)
    Y = ctx.apply(cuda(X), 0, 1).cpu().numpy().reshape(16, -1)
    ref = (D @ X.reshape(16, -1).T).T
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= 1e-6, err


def test_apply_bf16_elementwise(c1):
    """Every output component within 2u |D||x| + u |Dx| (u = 2^-8, factor
    1.5): a dropped hop, a wrong projector sign or a swapped link would miss
    it by orders of magnitude on the affected components."""
    w, U, D, ctx = c1
    X = random_spinors(w.L, 16, 7)
    Y = ctx.apply(cuda(X), 0, 2).cpu().numpy().reshape(16, -1)
    Xv = X.reshape(16, -1)
    ref = (D @ Xv.T).T
    ratio = bf16_bound_ratio(Y, ref, np.abs(D), np.abs(Xv))
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("L", [(2, 4, 2, 6), (4, 2, 6, 2), (6, 4, 4, 2)])
def test_apply_ragged_lattices(L):
    U = gauge_links(L, 0.8, 3)
    D = lattice.dense_wilson(U, L, -0.1)
    ctx = _lib().Context(L, -0.1)
    ctx.set_gauge(cuda(U))
    X = random_spinors(L, 5, 4)
    Y = ctx.apply(cuda(X), 0, 0).cpu().numpy().reshape(5, -1)
    ref = (D @ X.reshape(5, -1).T).T
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


def test_apply_c2_matches_c_stencil():
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = _lib().Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    X = random_spinors(w.L, 4, 11)
    Y = ctx.apply(cuda(X), 0, 0).cpu().numpy()
    for r in range(4):
        ref = stencil.apply_D(U, w.L, w.mass, X[r])
        assert np.abs(Y[r] - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("hp,first,nrhs", [(False, 0, 16), (True, 0, 32), (True, 250, 6), (False, 1000, 3)])
def test_probe_indices_bit_exact(c1, hp, first, nrhs):
    w, U, D, ctx = c1
    k, s = ctx.probe_indices(w.seed, 3, hp, first, nrhs)
    k = k.cpu().numpy()
    s = s.cpu().numpy()
    for r in range(nrhs):
        j = first + r
        kref = rng.z4_indices(rng.probe_key(w.seed, 3, hp, j), w.N)
        assert np.array_equal(k[r], kref)
        sref = rng.hadamard_signs(w.L, j) if hp else np.ones(w.V)
        assert np.array_equal(s[r].astype(np.float64), sref)
    Z = ctx.make_probes(w.seed, 3, hp, first, nrhs).cpu().numpy().reshape(nrhs, -1)
    Zref = rng.probes(w.L, w.seed, 3, hp, first, nrhs)
    assert np.array_equal(Z, Zref)


def test_probes_c3_hp_high_bits():
    w = WORKLOADS["c3"]
    ctx = _lib().Context(w.L, w.mass)
    k, s = ctx.probe_indices(w.seed, 0, True, 200, 4)
    s = s.cpu().numpy()
    k = k.cpu().numpy()
    for r in range(4):
        assert np.array_equal(s[r].astype(np.float64), rng.hadamard_signs(w.L, 200 + r))
        assert np.array_equal(k[r], rng.z4_indices(rng.probe_key(w.seed, 0, True, 200 + r), w.N))
    ctx.close()


def test_solve_fp64_c1(c1, c1_inv):
    w, U, D, ctx = c1
    L = _lib()
    Z = rng.probes(w.L, w.seed, 0, False, 0, 8)
    X, stats, rc = ctx.solve(cuda(Z.reshape((8,) + ctx._spinor_shape())), ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12))
    X = X.cpu().numpy().reshape(8, -1)
    ref = (c1_inv @ Z.T).T
    assert all(s["true_resid"] <= 1e-12 for s in stats)
    assert np.abs(X - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("inner", [1, 2])
def test_solve_mixed_c1(c1, c1_inv, inner):
    w, U, D, ctx = c1
    L = _lib()
    nrhs = 5
    Z = rng.probes(w.L, w.seed, 1, False, 0, nrhs)
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=inner, tol=1e-10)
    X, stats, rc = ctx.solve(cuda(Z.reshape((nrhs,) + ctx._spinor_shape())), prm)
    X = X.cpu().numpy().reshape(nrhs, -1)
    ref = (c1_inv @ Z.T).T
    assert all(s["true_resid"] <= 1e-10 and s["status"] == 0 for s in stats), stats
    q = np.einsum("ja,ja->j", Z.conj(), X)
    qref = np.einsum("ja,ja->j", Z.conj(), ref)
    assert np.abs(q - qref).max() <= 1e-10 * np.abs(qref).max()


def test_solve_mixed_c2_vs_c_stencil():
    w = WORKLOADS["c2"]
    L = _lib()
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = _lib().Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    nrhs = 4
    Z = rng.probes(w.L, w.seed, 0, False, 0, nrhs)
    Zt = cuda(Z.reshape((nrhs,) + ctx._spinor_shape()))
    for inner in (L.FP32, L.BF16):
        X, stats, rc = ctx.solve(Zt, ctx.params(L.SOLVER_DC_BICGSTAB, inner=inner, tol=1e-8))
        X = X.cpu().numpy().reshape(nrhs, -1)
        for r in range(nrhs):
            xr, st, it, rr = stencil.solve(U, w.L, w.mass, Z[r], 1e-12, 5000)
            assert st == 0
            q = np.vdot(Z[r], X[r])
            qref = np.vdot(Z[r], xr.ravel())
            assert stats[r]["true_resid"] <= 1e-8
            assert abs(q - qref) <= 1e-8 * abs(qref), (inner, r, abs(q - qref) / abs(qref))
    ctx.close()


def round_storage(W, prec):
    """Round a complex128 array as the library stores it: FP32 by IEEE
    round-to-nearest-even, BF16 by RNE of the FP32 value's upper 16 bits."""
    if prec == 0:
        return W
    f = np.stack([W.real, W.imag], axis=-1).astype(np.float32)
    if prec == 2:
        u = f.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        f = u.astype(np.uint32).view(np.float32)
    f = f.astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_deflation_c1(c1, c1_inv, prec):
    w, U, D, ctx = c1
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    TD = ctx.set_deflation(cuda(W.T), prec)
    # the reference takes the same rounded basis, in FP64
    Wr = round_storage(W, prec)
    M = estimator.galerkin_M(Wr, D, g5)
    TD_ref = estimator.deflated_trace(Wr, M, g5)
    assert abs(TD - TD_ref) <= 1e-10 * abs(TD_ref)
    assert np.abs(ctx.deflation_M() - M).max() <= 1e-9 * np.abs(M).max()
    Z = rng.probes(w.L, w.seed, 0, False, 0, 7)
    c1_, c2_ = ctx.project(cuda(Z.reshape((7,) + ctx._spinor_shape())))
    r1, r2 = estimator.projection_coefficients(Wr, Z, g5)
    assert np.abs(c1_ - r1).max() <= 1e-13 * np.abs(r1).max()
    assert np.abs(c2_ - r2).max() <= 1e-13 * np.abs(r2).max()
    ctx.clear_deflation()


def test_trace_batch_c1_mc_and_deflated(c1, c1_inv):
    w, U, D, ctx = c1
    L = _lib()
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    TD = ctx.set_deflation(cuda(W.T), L.FP64)
    ctx.reset_estimate()
    prm = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    recs = []
    for b in range(0, w.nprobe, w.batch):
        recs += ctx.trace_batch(w.seed, 0, False, b, w.batch, prm)
    Z = rng.probes(w.L, w.seed, 0, False, 0, w.nprobe)
    q_ref = np.einsum("ja,ab,jb->j", Z.conj(), c1_inv, Z)
    M = estimator.galerkin_M(W, D, g5)
    c1_, c2_ = estimator.projection_coefficients(W, Z, g5)
    qd_ref = q_ref - estimator.deflation_corrections(c1_, c2_, M)
    q = np.array([r["q"] for r in recs])
    qd = np.array([r["q_defl"] for r in recs])
    scale = np.abs(q_ref).max()
    assert np.abs(q - q_ref).max() <= 1e-10 * scale
    assert np.abs(qd - qd_ref).max() <= 1e-10 * scale
    est = ctx.estimate()
    m, var, vre, vim = estimator.sample_statistics(q_ref)
    md, vard, _, _ = estimator.sample_statistics(qd_ref)
    TD_ref = estimator.deflated_trace(W, M, g5)
    assert est["n"] == w.nprobe
    assert abs(complex(est["mean_re"], est["mean_im"]) - m) <= 1e-10 * abs(m)
    assert abs(complex(est["mean_defl_re"], est["mean_defl_im"]) - (md + TD_ref)) <= 1e-10 * abs(m)
    assert abs(est["var"] - var) <= 1e-8 * var
    assert abs(est["var_re"] - vre) <= 1e-8 * var
    assert abs(est["var_defl"] - vard) <= 1e-8 * var
    ctx.clear_deflation()


@pytest.mark.parametrize("method", ["fp64", "dc_bf16"])
def test_trace_batch_c1_without_deflation(c1, c1_inv, method):
    """Without a deflation basis the batch solves take the probes from a BF16
    field (probe values are exact there; the FP64 hops widen them exactly):
    q matches the exact inverse, and the solve of the same probes handed in
    as an FP64 field, to the solver's tolerance."""
    w, U, D, ctx = c1
    L = _lib()
    ctx.clear_deflation()
    ctx.reset_estimate()
    prm = (ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12) if method == "fp64"
           else ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10))
    n = 2 * w.batch
    recs = []
    for b in range(0, n, w.batch):
        recs += ctx.trace_batch(w.seed, 1, True, b, w.batch, prm)
    Z = rng.probes(w.L, w.seed, 1, True, 0, n)
    q_ref = np.einsum("ja,ab,jb->j", Z.conj(), c1_inv, Z)
    q = np.array([r["q"] for r in recs])
    tol = 1e-10 if method == "fp64" else 1e-8
    scale = np.abs(q_ref).max()
    assert np.abs(q - q_ref).max() <= tol * scale
    X, st, rc = ctx.solve(cuda(Z.reshape((n,) + ctx._spinor_shape())), prm)
    q2 = np.einsum("ja,ja->j", Z.conj(), X.cpu().numpy().reshape(n, -1))
    assert np.abs(q - q2).max() <= tol * scale
    assert ctx.estimate()["n"] == n


@pytest.mark.parametrize("form", [0, 1, 2])
def test_trace_batch_bf16_probe_operands_every_hop_form(c1, c1_inv, form):
    """The FP64 hops that read the probes from BF16 storage (Schur right-hand
    side, odd sites, final residual), forced into each launch form: a trace
    batch matches the exact inverse to the solver's tolerance."""
    w, U, D, ctx = c1
    L = _lib()
    ctx.clear_deflation()
    ctx.reset_estimate()
    ctx.set_hop_config(L.FP64, w.batch, {"form": form, "streaming_stores": 1, "t_chunk": 2 if form == 2 else 0})
    try:
        recs = ctx.trace_batch(w.seed, 2, True, 0, w.batch, ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12))
    finally:
        ctx.set_hop_config(L.FP64, w.batch, None)
    Z = rng.probes(w.L, w.seed, 2, True, 0, w.batch)
    q_ref = np.einsum("ja,ab,jb->j", Z.conj(), c1_inv, Z)
    q = np.array([r["q"] for r in recs])
    assert np.abs(q - q_ref).max() <= 1e-10 * np.abs(q_ref).max()


@pytest.mark.parametrize("method", ["fp64", "dc_bf16"])
def test_solve_zero_right_hand_sides(c1, c1_inv, method):
    """A zero right-hand side has the solution 0 (the solver writes it although
    no correction is ever applied), alone or next to a non-zero one, and the
    non-zero one is solved as usual."""
    w, U, D, ctx = c1
    L = _lib()
    prm = (ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-10) if method == "fp64"
           else ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10))
    shape = (2,) + ctx._spinor_shape()
    # the workspace first holds a non-zero solution, so stale values would show
    Z = cuda(random_spinors(w.L, 2, 5))
    ctx.solve(Z, prm)
    X, st, rc = ctx.solve(torch.zeros(shape, dtype=torch.complex128, device="cuda"), prm)
    assert torch.count_nonzero(X).item() == 0
    assert all(s["true_resid"] == 0.0 for s in st)
    Z[1] = 0
    X, st, rc = ctx.solve(Z, prm)
    assert torch.count_nonzero(X[1]).item() == 0
    x0 = X[0].cpu().numpy().ravel()
    z0 = Z[0].cpu().numpy().ravel()
    assert np.linalg.norm(x0 - c1_inv @ z0) <= 1e-8 * np.linalg.norm(c1_inv @ z0)


def test_bf16_inner_solution_history_ring_wraps():
    """A BF16 inner solve rebuilds its solution from the stored iterations in
    rings (here of 3, forced): a cycle runs longer than that, so the rings
    are flushed into x in the middle of the cycle.  The solution must still
    meet the true-residual tolerance and match FP64."""
    L = _lib()
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    Z = cuda(random_spinors(w.L, 4, 31))
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-9, maxiter=4000, inner_tol=1e-5, history=3)
    X, st, rc = ctx.solve(Z, prm)
    assert all(s["true_resid"] <= 1e-9 for s in st), st
    assert max(s["iters"] / max(1, s["outer"]) for s in st) > 3, st   # longer than a ring
    with pytest.raises(L.DhtError):
        ctx.solve(Z, ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-9, history=17))
    X64, st64, _ = ctx.solve(Z, ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-11, maxiter=4000))
    err = (X - X64).abs().max().item() / X64.abs().max().item()
    assert err <= 1e-7, err
    for r in (0, 3):
        x = X[r].cpu().numpy().ravel()
        z = Z[r].cpu().numpy().ravel()
        res = np.linalg.norm(z - stencil.apply_D(U, w.L, w.mass, x)) / np.linalg.norm(z)
        assert res <= 1e-9, (r, res)
    ctx.close()


def test_invalid_arguments(c1):
    w, U, D, ctx = c1
    L = _lib()
    with pytest.raises(L.DhtError):
        L.Context((3, 4, 4, 4), -0.2)
    with pytest.raises(L.DhtError):
        ctx.trace_batch(0, 0, False, 0, 0, ctx.params())
    with pytest.raises(L.DhtError):
        ctx.project(torch.zeros((1,) + ctx._spinor_shape(), dtype=torch.complex128, device="cuda"))


def test_fault_injection_falls_back(c1, c1_inv):
    w, U, D, ctx = c1
    L = _lib()
    Z = rng.probes(w.L, w.seed, 2, False, 0, 4)
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10, fault_inject=1)
    X, stats, rc = ctx.solve(cuda(Z.reshape((4,) + ctx._spinor_shape())), prm)
    assert all(s["true_resid"] <= 1e-10 for s in stats)
    assert all(s["status"] in (2, 3) for s in stats), stats
    X = X.cpu().numpy().reshape(4, -1)
    ref = (c1_inv @ Z.T).T
    assert np.abs(X - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("k", [12, 20, 33])
def test_deflation_finalize_k_not_power_of_two(c1, c1_inv, k):
    """The FP64 Galerkin finalize processes the basis in blocks of up to 32
    columns padded to a power of two; k = 12, 20 (one padded block) and 33
    (a full block and a ragged one) give M and T_D of the oracle."""
    w, U, D, ctx = c1
    L = _lib()
    g5 = lattice.gamma5_full(w.V)
    lam, W = estimator.q_eigenpairs(D, g5, k)
    rs = np.random.default_rng(k)
    Wp = W + 1e-3 * (rs.standard_normal(W.shape) + 1j * rs.standard_normal(W.shape))   # not eigenvectors
    TD = ctx.set_deflation(cuda(Wp.T), L.FP64)
    M = estimator.galerkin_M(Wp, D, g5)
    TD_ref = estimator.deflated_trace(Wp, M, g5)
    assert abs(TD - TD_ref) <= 1e-10 * abs(TD_ref), (TD, TD_ref)
    assert np.abs(ctx.deflation_M() - M).max() <= 1e-9 * np.abs(M).max()
    ctx.clear_deflation()


def test_unconverged_probes_stay_out_of_the_estimates(c1, c1_inv):
    """A probe whose solve misses the tolerance is reported (status 1) but not
    added to the running estimates; the retried batch then counts once."""
    w, U, D, ctx = c1
    L = _lib()
    ctx.clear_deflation()
    ctx.reset_estimate()
    bad = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12, maxiter=2)
    recs = ctx.trace_batch(w.seed, 3, True, 0, w.batch, bad, allow_not_converged=True)
    assert all(r["status"] == 1 for r in recs), recs
    assert ctx.estimate()["n"] == 0
    good = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=1e-12)
    recs = ctx.trace_batch(w.seed, 3, True, 0, w.batch, good)
    assert ctx.estimate()["n"] == w.batch
    Z = rng.probes(w.L, w.seed, 3, True, 0, w.batch)
    q_ref = np.einsum("ja,ab,jb->j", Z.conj(), c1_inv, Z)
    est = ctx.estimate()
    assert abs(complex(est["mean_re"], est["mean_im"]) - q_ref.mean()) <= 1e-10 * abs(q_ref.mean())


@pytest.mark.parametrize("hook,counter", [(2, "predicted_failed"), (4, "reentries")])
def test_defect_correction_forced_branches(c1, c1_inv, hook, counter):
    """Host-forced conditions drive the defect-correction loop through the
    branch that continues from a stored FP64 residual after a failed
    convergence prediction (hook 2), and through the one that resumes the
    loop when the in-place residual update stopped it on norms its FP64
    residual does not confirm (hook 4).  Both end on the exact inverse."""
    w, U, D, ctx = c1
    L = _lib()
    ctx.clear_deflation()
    ctx.reset_estimate()
    before = ctx.solver_counters()
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-10, fault_inject=hook)
    recs = ctx.trace_batch(w.seed, 4, True, 0, w.batch, prm)
    after = ctx.solver_counters()
    assert after[counter] > before[counter], (before, after)
    assert all(r["true_resid"] <= 1e-10 and r["status"] == 0 for r in recs), recs
    Z = rng.probes(w.L, w.seed, 4, True, 0, w.batch)
    q_ref = np.einsum("ja,ab,jb->j", Z.conj(), c1_inv, Z)
    q = np.array([r["q"] for r in recs])
    assert np.abs(q - q_ref).max() <= 1e-8 * np.abs(q_ref).max()
