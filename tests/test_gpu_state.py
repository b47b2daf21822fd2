"""Checkpoint / resume of the running estimates and the autotuner's cache
file, through the C ABI.

Splitting an Algorithm-1 run into two processes (save after the first batch,
load into a fresh context, continue) gives exactly the estimates of one
uninterrupted run: the per-probe quadratic forms are deterministic (fixed
reduction orders) and the moments round-trip exactly.  A checkpoint refuses a
context of another lattice or deflation space.
"""
import numpy as np
import pytest

from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_1603_05988_amd import _lib as L
    return L


def _ctx(w, U):
    ctx = _lib().Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    return ctx


def test_checkpoint_resume_is_exact(tmp_path):
    Lb = _lib()
    w = WORKLOADS["c1"]
    U = gauge_links(w.L, w.eps, w.seed)
    prm = Lb.Context.params(Lb.SOLVER_DC_BICGSTAB, inner=Lb.FP32, tol=1e-10, maxiter=2000)
    whole = _ctx(w, U)
    for first in (0, 16):
        whole.trace_batch(w.seed, 0, False, first, 16, prm)
    ref = whole.estimate()
    whole.close()

    a = _ctx(w, U)
    a.trace_batch(w.seed, 0, False, 0, 16, prm)
    path = str(tmp_path / "est.txt")
    a.save_state(path)
    a.close()
    b = _ctx(w, U)
    b.load_state(path)
    b.trace_batch(w.seed, 0, False, 16, 16, prm)
    got = b.estimate()
    for key in ("n", "mean_re", "mean_im", "var", "var_re", "var_im"):
        assert got[key] == ref[key], (key, got[key], ref[key])
    b.close()

    other = _lib().Context((4, 4, 4, 8), w.mass)
    with pytest.raises(Lb.DhtError):
        other.load_state(path)                      # another lattice
    other.close()
    c = _ctx(w, U)
    Wd = torch.randn((4, w.N), dtype=torch.complex128, device="cuda")
    c.set_deflation(Wd / torch.linalg.vector_norm(Wd, dim=1, keepdim=True))
    with pytest.raises(Lb.DhtError):
        c.load_state(path)                          # saved without deflation
    c.close()
    bad = tmp_path / "bad.txt"
    bad.write_text("something else\n")
    d = _ctx(w, U)
    with pytest.raises(Lb.DhtError):
        d.load_state(str(bad))
    d.close()


def test_autotune_cache_file(tmp_path):
    Lb = _lib()
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    cache = str(tmp_path / "tune.txt")
    # a line in the layout without z blocks is skipped, not installed
    with open(cache, "w") as f:
        f.write("hop %d %d %d %d 2 16 0 0 1 0 16 0.1\n" % tuple(w.L))
    a = _ctx(w, U)
    r1 = a.autotune(Lb.BF16, 16, reps=2, cache_path=cache)
    assert r1["candidates"] > 0
    a.close()
    lines = open(cache).read().split("\n")
    assert sum(1 for x in lines if x.startswith("hop2 ")) == len(Lb.HOP_CLASSES)
    b = _ctx(w, U)
    r2 = b.autotune(Lb.BF16, 16, reps=2, cache_path=cache)
    assert r2["candidates"] == 0 and r2["best"] == r1["best"]
    for cls, name in Lb.HOP_CLASSES.items():
        assert b.hop_config(Lb.BF16, 16, cls) == r1["best"][name]
    r3 = b.autotune(Lb.FP32, 16, reps=2, cache_path=cache)     # not cached yet: tuned and appended
    assert r3["candidates"] > 0
    assert sum(1 for x in open(cache).read().split("\n") if x.startswith("hop2 ")) == 2 * len(Lb.HOP_CLASSES)
    b.close()
