"""ctypes wrapper of the plain-C FP64 Wilson stencil oracle (stencil.c).

Test infrastructure only.  `build()` compiles stencil.c with gcc/OpenMP into
oracle/_build/libo2stencil.so.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil.c")
_OUT = os.path.join(_HERE, "_build", "libo2stencil.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_OUT)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.o2_dslash.argtypes = [ip, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        L.o2_dslash.restype = None
        L.o2_bicgstab.argtypes = [ip, ctypes.c_double, ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                  ctypes.c_int, ip, dp]
        L.o2_bicgstab.restype = ctypes.c_int
        L.o2_project.argtypes = [dp, ctypes.c_int, dp, ctypes.c_long, dp]
        L.o2_project.restype = None
        L.o2_num_threads.argtypes = []
        L.o2_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _L(L):
    return (ctypes.c_int * 4)(*[int(v) for v in L])


def apply_D(U: np.ndarray, L, mass: float, psi: np.ndarray, t_antiperiodic: bool = True) -> np.ndarray:
    """D psi for one canonical spinor (any shape with 12 V complex entries)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    lib().o2_dslash(_L(L), float(mass), int(t_antiperiodic), _dp(U), _dp(psi), _dp(out))
    return out


def solve(U: np.ndarray, L, mass: float, b: np.ndarray, tol: float, maxiter: int,
          t_antiperiodic: bool = True):
    """BiCGStab for D x = b.  Returns (x, status, iters, true relative residual)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = lib().o2_bicgstab(_L(L), float(mass), int(t_antiperiodic), _dp(U), _dp(b), _dp(x),
                           float(tol), int(maxiter), ctypes.byref(it), ctypes.byref(rr))
    return x, int(st), int(it.value), float(rr.value)


def project(W: np.ndarray, z: np.ndarray) -> np.ndarray:
    """W^H z with W given as k rows of N complex entries."""
    W = np.ascontiguousarray(W, dtype=np.complex128)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    k, N = W.shape
    out = np.empty(k, dtype=np.complex128)
    lib().o2_project(_dp(W), int(k), _dp(z), int(N), _dp(out))
    return out


def num_threads() -> int:
    return int(lib().o2_num_threads())
