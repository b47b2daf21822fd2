"""Every launch shape of the hopping kernel against the dense oracle, and the
autotuner that chooses among them.

The forms (one lane per site with links per lane, staged in LDS or shared
across the 16-lane row of a site; one lane per (x, y, z) column walking t in
chunks, plain or skewed by one slice, rows in y-fastest order or in z blocks,
with links per lane or row-shared, with or without streaming stores,
sweeping the lattice once for all right-hand sides or once per group of them)
accumulate the same 8 neighbour terms in different orders, so each must match
the dense Wilson matrix to the storage precision: FP64 1e-13 relative
(max-norm), FP32 1e-6, BF16 element by element within the rounding model of
tests/bounds.py (2u |D||x| + u |Dx|, u = 2^-8, with a factor 1.5).  The
fused-dot variants used inside BiCGStab are covered by solves in each forced
form.
"""
import json

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


def forms(L, nrhs, rowl=True):
    out = []
    for G in sorted({nrhs, max(1, nrhs // 2), max(1, nrhs // 4)}, reverse=True):
        for nt in (0, 1):
            out.append({"form": 0, "streaming_stores": nt, "t_chunk": 0, "rhs_group": G})
            if G >= 8:
                out.append({"form": 1, "streaming_stores": nt, "t_chunk": 0, "rhs_group": G})
            for form in (2, 5):   # t-marching, plain and skewed
                for tc in range(2, L[3] + 1, 2):
                    if L[3] % tc == 0:
                        out.append({"form": form, "streaming_stores": nt, "t_chunk": tc, "rhs_group": G})
            if G >= 16 and rowl:   # links shared across the 16-lane row of a site (BF16; plain forms otherwise)
                out.append({"form": 3, "streaming_stores": nt, "t_chunk": 0, "rhs_group": G})
                for form in (4, 6):
                    for tc in range(2, L[3] + 1, 2):
                        if L[3] % tc == 0:
                            out.append({"form": form, "streaming_stores": nt, "t_chunk": tc, "rhs_group": G})
    return out


def zforms(L, nrhs, rowl=True):
    """The t-marching forms with their rows walked in z blocks (z_block = 2, 4
    where they divide Lz), at the shortest chunk and streaming stores on."""
    out = []
    tc = min(tc for tc in range(2, L[3] + 1, 2) if L[3] % tc == 0)
    for form in ((2, 5, 4, 6) if nrhs >= 16 and rowl else (2, 5)):
        for zb in (2, 4):
            if L[2] % zb == 0:
                out.append({"form": form, "streaming_stores": 1, "t_chunk": tc, "rhs_group": nrhs, "z_block": zb})
    return out


def err_of(prec, Y, ref, Dabs=None, Xabs=None):
    if prec == 2:
        return bf16_bound_ratio(Y, ref, Dabs, Xabs)
    return np.abs(Y - ref).max() / np.abs(ref).max()


TOL = {0: 1e-13, 1: 1e-6, 2: 1.0}


@pytest.mark.parametrize("L,nrhs", [((4, 4, 4, 4), 16), ((2, 4, 2, 6), 8), ((6, 4, 4, 2), 8), ((4, 2, 6, 4), 32),
                                    ((4, 4, 2, 8), 4)])
def test_every_form_matches_dense(L, nrhs):
    Lb = _lib()
    U = gauge_links(L, 0.6, 5)
    D = lattice.dense_wilson(U, L, -0.2)
    g5 = lattice.gamma5_full(int(np.prod(L)))
    ctx = Lb.Context(L, -0.2)
    ctx.set_gauge(cuda(U))
    X = random_spinors(L, nrhs, 9)
    Xv = X.reshape(nrhs, -1)
    refs = {Lb.OP_D: (D @ Xv.T).T, Lb.OP_DDAG: (D.conj().T @ Xv.T).T, Lb.OP_Q: (g5[:, None] * D @ Xv.T).T}
    Dabs = {Lb.OP_D: np.abs(D), Lb.OP_DDAG: np.abs(D.conj().T), Lb.OP_Q: np.abs(D)}
    Xabs = np.abs(Xv)
    for prec in (0, 1, 2):
        for cfg in forms(L, nrhs) + zforms(L, nrhs):
            ctx.set_hop_config(prec, nrhs, cfg)     # both epilogue classes
            for cls in Lb.HOP_CLASSES:
                got = ctx.hop_config(prec, nrhs, cls)
                assert got["form"] == cfg["form"] and got["streaming_stores"] == cfg["streaming_stores"]
                assert got["rhs_group"] == cfg["rhs_group"] and got["z_block"] == max(1, cfg.get("z_block", 0))
                if cfg["form"] in (2, 4, 5, 6):
                    assert got["t_chunk"] == cfg["t_chunk"]
            for op, ref in refs.items():
                Y = ctx.apply(cuda(X), op, prec).cpu().numpy().reshape(nrhs, -1)
                e = err_of(prec, Y, ref, Dabs[op], Xabs)
                assert e <= TOL[prec], (prec, cfg, op, e)
        ctx.set_hop_config(prec, nrhs, None)
    ctx.close()


@pytest.mark.parametrize("cfg", [{"form": 0, "streaming_stores": 0, "t_chunk": 0},
                                 {"form": 1, "streaming_stores": 1, "t_chunk": 0},
                                 {"form": 2, "streaming_stores": 1, "t_chunk": 2},
                                 {"form": 2, "streaming_stores": 0, "t_chunk": 4},
                                 {"form": 0, "streaming_stores": 1, "t_chunk": 0, "rhs_group": 2},
                                 {"form": 2, "streaming_stores": 1, "t_chunk": 2, "rhs_group": 4},
                                 {"form": 5, "streaming_stores": 1, "t_chunk": 2},
                                 {"form": 5, "streaming_stores": 0, "t_chunk": 4, "rhs_group": 4},
                                 {"form": 2, "streaming_stores": 1, "t_chunk": 2, "z_block": 4},
                                 {"form": 5, "streaming_stores": 1, "t_chunk": 4, "z_block": 2}])
def test_solves_in_every_form(cfg):
    """BiCGStab (FP64, and FP32 inside FP64 defect correction) with the fused
    hop+dot kernels in one forced shape, against the LU inverse."""
    Lb = _lib()
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    Dinv = estimator.exact_inverse(lattice.dense_wilson(U, w.L, w.mass))
    ctx = Lb.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    for prec in (0, 1):
        ctx.set_hop_config(prec, 8, cfg)
    Z = rng.probes(w.L, w.seed, 3, False, 0, 5)
    ref = (Dinv @ Z.T).T
    for prm in (ctx.params(Lb.SOLVER_BICGSTAB_FP64, tol=1e-11, maxiter=2000),
                ctx.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.FP32, tol=1e-10, maxiter=2000)):
        X, stats, rc = ctx.solve(cuda(Z.reshape((5,) + ctx._spinor_shape())), prm)
        X = X.cpu().numpy().reshape(5, -1)
        assert all(s["true_resid"] <= prm.tol for s in stats), (cfg, stats)
        assert np.abs(X - ref).max() <= 1e-8 * np.abs(ref).max(), cfg
    ctx.close()


def test_invalid_shapes_rejected():
    Lb = _lib()
    ctx = Lb.Context((4, 4, 4, 6), -0.2)
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 4, {"form": 1})                          # LDS links need >= 8 RHS
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 2, "t_chunk": 4})           # 4 does not divide Lt = 6
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 2, "t_chunk": 3})           # odd chunk
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 12, {"form": 0})                         # batch not a power of two
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 7})
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 0, "rhs_group": 3})         # group not a power of two
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 0, "rhs_group": 32})        # group larger than the batch
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 1, "rhs_group": 4})         # LDS links need >= 8 RHS per sweep
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 2, "t_chunk": 2, "z_block": 3})   # z block not a power of two
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 5, "t_chunk": 2, "z_block": 8})   # 8 does not divide Lz = 4
    with pytest.raises(Lb.DhtError):
        ctx.set_hop_config(1, 16, {"form": 0, "z_block": 2})                 # z blocks only in the t-marching forms
    with pytest.raises(Lb.DhtError):
        ctx.autotune_hop(1, 16, 2)                                       # no gauge field yet
    ctx.close()


def test_autotune_c2(tmp_path):
    """The tuner times every valid shape on the 8^3x16 operator, rejects none
    (all agree to rounding), installs the fastest, and the operator still
    matches the C stencil afterwards; the table survives a JSON round trip."""
    Lb = _lib()
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = Lb.Context(w.L, w.mass)
    ctx.set_gauge(cuda(U))
    res = {}
    for prec in (0, 1, 2):
        r = ctx.autotune_hop(prec, 16, reps=3)
        res[prec] = r
        assert r["rejected"] == 0 and r["candidates"] == len(forms(w.L, 16, rowl=prec == 2)), r
        assert r["max_rel_diff"] <= {0: 1e-12, 1: 1e-5, 2: 1.6e-2}[prec], r
        for cls, name in Lb.HOP_CLASSES.items():
            assert 0 < r["best_ms"][name] <= r["default_ms"][name] * (1 + 1e-9), r
            assert ctx.hop_config(prec, 16, cls) == r["best"][name]
    X = random_spinors(w.L, 16, 21)
    Y = ctx.apply(cuda(X), 0, 0).cpu().numpy()
    for rr in (0, 15):
        ref = stencil.apply_D(U, w.L, w.mass, X[rr])
        assert np.abs(Y[rr] - ref).max() <= 1e-13 * np.abs(ref).max()
    path = tmp_path / "tune.json"
    ctx.save_tuning(str(path))
    tab = json.load(open(path))
    assert set(tab["entries"]) == {"0:16", "1:16", "2:16"}
    ctx2 = Lb.Context(w.L, w.mass)
    assert ctx2.load_tuning(str(path)) == 3
    for prec in (0, 1, 2):
        for cls, name in Lb.HOP_CLASSES.items():
            assert ctx2.hop_config(prec, 16, cls) == res[prec]["best"][name]
    other = Lb.Context((4, 4, 4, 4), -0.2)
    assert other.load_tuning(str(path)) == 0     # measured on another lattice: ignored
    other.close()
    ctx2.close()
    ctx.close()
