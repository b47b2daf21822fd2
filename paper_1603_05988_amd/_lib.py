"""ctypes binding of libdhtrace.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts torch
tensors to device pointers, numpy arrays to host pointers, and C structs to
Python values.  Importing it on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdhtrace.so")

DHT_OK = 0
DHT_ERR_NOT_CONVERGED = -6
FP64, FP32, BF16 = 0, 1, 2
OP_D, OP_DDAG, OP_G5, OP_Q = 0, 1, 2, 3
SOLVER_BICGSTAB_FP64, SOLVER_DC_BICGSTAB, SOLVER_DC_FGMRES_NN = 0, 1, 2
STATUS_NAMES = {0: "converged", 1: "not_converged", 2: "fallback_fp32", 3: "fallback_fp64"}


class Lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("mass", ctypes.c_double), ("t_antiperiodic", ctypes.c_int)]


class ProbeSpec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("run", ctypes.c_uint64), ("hp", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("inner", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("restart", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("fault_inject", ctypes.c_uint32), ("history", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("true_resid", ctypes.c_double),
                ("status", ctypes.c_int)]


class Record(ctypes.Structure):
    _fields_ = [("q_re", ctypes.c_double), ("q_im", ctypes.c_double), ("qd_re", ctypes.c_double),
                ("qd_im", ctypes.c_double), ("s", SolveStats)]


class EigParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("degree", ctypes.c_int),
                ("guard", ctypes.c_int), ("seed", ctypes.c_uint64)]


class LobpcgParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("block", ctypes.c_int),
                ("precond", ctypes.c_int), ("precond_tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class LobpcgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("q_applications", ctypes.c_int64),
                ("precond_solves", ctypes.c_int64)]


class EigStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("block", ctypes.c_int),
                ("matvecs", ctypes.c_int64)]


class HopConfig(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("streaming_stores", ctypes.c_int), ("t_chunk", ctypes.c_int),
                ("rhs_group", ctypes.c_int), ("z_block", ctypes.c_int)]


def _hop_dict(h) -> dict:
    return {"form": h.form, "streaming_stores": h.streaming_stores, "t_chunk": h.t_chunk,
            "rhs_group": h.rhs_group, "z_block": h.z_block}


class TuneResult(ctypes.Structure):
    _fields_ = [("best", HopConfig * 3), ("best_ms", ctypes.c_double * 3), ("default_ms", ctypes.c_double * 3),
                ("candidates", ctypes.c_int), ("rejected", ctypes.c_int), ("max_rel_diff", ctypes.c_double)]


HOP_SITE, HOP_SITE_LDS, HOP_TMARCH, HOP_SITE_ROWL, HOP_TMARCH_ROWL, HOP_TSKEW, HOP_TSKEW_ROWL = 0, 1, 2, 3, 4, 5, 6
HOP_PLAIN, HOP_FUSED, HOP_FUSED_A = 0, 1, 2
HOP_CLASSES = {HOP_PLAIN: "plain", HOP_FUSED: "fused", HOP_FUSED_A: "fused_a"}
HOP_FORMS = {HOP_SITE: "site", HOP_SITE_LDS: "site_lds", HOP_TMARCH: "tmarch", HOP_SITE_ROWL: "site_rowl",
             HOP_TMARCH_ROWL: "tmarch_rowl", HOP_TSKEW: "tskew", HOP_TSKEW_ROWL: "tskew_rowl"}


class BatchTune(ctypes.Structure):
    _fields_ = [("best_nrhs", ctypes.c_int), ("candidates", ctypes.c_int), ("nrhs", ctypes.c_int * 8),
                ("status", ctypes.c_int * 8), ("rhs_per_s", ctypes.c_double * 8), ("workspace", ctypes.c_size_t * 8)]


class HPVar(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("mean_re", ctypes.c_double), ("mean_im", ctypes.c_double),
                ("mean_err", ctypes.c_double), ("var", ctypes.c_double), ("var_err", ctypes.c_double),
                ("rs", ctypes.c_double), ("rs_err", ctypes.c_double)]


class Thm2(ctypes.Structure):
    _fields_ = [("var_k", ctypes.c_double), ("var_0", ctypes.c_double), ("ratio", ctypes.c_double),
                ("mu_k", ctypes.c_double), ("V_k", ctypes.c_double), ("reduces", ctypes.c_int)]


class Estimate(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean_re", ctypes.c_double), ("mean_im", ctypes.c_double),
                ("mean_defl_re", ctypes.c_double), ("mean_defl_im", ctypes.c_double),
                ("TD_re", ctypes.c_double), ("TD_im", ctypes.c_double),
                ("var", ctypes.c_double), ("var_re", ctypes.c_double), ("var_im", ctypes.c_double),
                ("var_defl", ctypes.c_double), ("var_defl_re", ctypes.c_double), ("var_defl_im", ctypes.c_double)]


# name -> (restype, argtypes); mirrors include/dhtrace.h
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "dht_create": (_i, [ctypes.POINTER(Lattice), _i, _vp, ctypes.POINTER(_vp)]),
    "dht_destroy": (_i, [_vp]),
    "dht_last_error": (ctypes.c_char_p, []),
    "dht_version": (ctypes.c_char_p, []),
    "dht_set_gauge": (_i, [_vp, _vp]),
    "dht_workspace_trim": (_i, [_vp]),
    "dht_workspace_size": (_i, [_vp, _i, ctypes.POINTER(SolverParams), ctypes.POINTER(ctypes.c_size_t)]),
    "dht_set_workspace": (_i, [_vp, _vp, ctypes.c_size_t]),
    "dht_apply": (_i, [_vp, _i, _i, _vp, _vp, _i]),
    "dht_apply_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _i]),
    "dht_make_probes": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, _vp]),
    "dht_probe_indices": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, _vp, _vp]),
    "dht_solve": (_i, [_vp, ctypes.POINTER(SolverParams), _vp, _vp, _i, ctypes.POINTER(SolveStats)]),
    "dht_deflation_begin": (_i, [_vp, _i, _i]),
    "dht_deflation_set": (_i, [_vp, _i, _i, _vp]),
    "dht_deflation_eigensolve": (_i, [_vp, ctypes.POINTER(EigParams), _dp, _dp, ctypes.POINTER(EigStats)]),
    "dht_deflation_lobpcg": (_i, [_vp, ctypes.POINTER(LobpcgParams), _dp, _dp, ctypes.POINTER(LobpcgStats)]),
    "dht_deflation_finalize": (_i, [_vp, _dp]),
    "dht_deflation_get": (_i, [_vp, _i, _i, _vp]),
    "dht_deflation_finalize_diag": (_i, [_vp, _dp]),
    "dht_project_probes": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, _dp, _dp]),
    "dht_set_projection_window": (_i, [_vp, _i]),
    "dht_profile_enable": (_i, [_vp, _i]),
    "dht_profile_reset": (_i, [_vp]),
    "dht_profile_get": (_i, [_vp, _i, ctypes.POINTER(_i64), _dp, _dp]),
    "dht_deflation_get_M": (_i, [_vp, _dp]),
    "dht_deflation_clear": (_i, [_vp]),
    "dht_project": (_i, [_vp, _vp, _i, _dp, _dp]),
    "dht_trace_batch": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, ctypes.POINTER(SolverParams),
                             ctypes.POINTER(Record), _dp]),
    "dht_estimate_get": (_i, [_vp, ctypes.POINTER(Estimate)]),
    "dht_gamma_set": (_i, [_vp, _dp, _i, _dp]),
    "dht_theorem2": (_i, [_i64, _i, _i, ctypes.c_double, ctypes.c_double, _dp, ctypes.POINTER(Thm2)]),
    "dht_distance_profile": (_i, [_vp, ctypes.POINTER(_i64), _i, _i, _i, ctypes.POINTER(SolverParams), _dp,
                                  ctypes.POINTER(_i64)]),
    "dht_trace_gamma_batch": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, ctypes.POINTER(SolverParams),
                                   ctypes.POINTER(Record)]),
    "dht_gamma_estimate_get": (_i, [_vp, _i, ctypes.POINTER(Estimate)]),
    "dht_estimate_reset": (_i, [_vp]),
    "dht_last_timings": (_i, [_vp, _dp, _i]),
    "dht_solver_counters": (_i, [_vp, ctypes.POINTER(_i64), _i]),
    "dht_bench_hop": (_i, [_vp, _i, _i, _i, _i, _dp]),
    "dht_nn_num_weights": (_i64, []),
    "dht_nn_init": (_i, [_vp, _u64]),
    "dht_nn_set_skip": (_i, [_vp, _d]),
    "dht_nn_set_weights": (_i, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "dht_nn_get_weights": (_i, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "dht_nn_forward": (_i, [_vp, _vp, _vp, _i]),
    "dht_nn_grad": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(ctypes.c_float), _dp]),
    "dht_nn_train": (_i, [_vp, _vp, _vp, _i, _i, _i, ctypes.c_float, _dp]),
    "dht_nn_make_pairs": (_i, [_vp, ctypes.POINTER(ProbeSpec), _i64, _i, _i, _vp, _vp, _i, ctypes.POINTER(_i)]),
    "dht_hop_config_set": (_i, [_vp, _i, _i, _i, ctypes.POINTER(HopConfig)]),
    "dht_hop_config_get": (_i, [_vp, _i, _i, _i, ctypes.POINTER(HopConfig)]),
    "dht_autotune_hop": (_i, [_vp, _i, _i, _i, ctypes.POINTER(TuneResult)]),
    "dht_autotune": (_i, [_vp, _i, _i, _i, ctypes.c_char_p, ctypes.POINTER(TuneResult)]),
    "dht_autotune_batch": (_i, [_vp, ctypes.POINTER(ProbeSpec), ctypes.POINTER(SolverParams), ctypes.POINTER(_i), _i,
                                ctypes.c_size_t, _i, ctypes.POINTER(BatchTune)]),
    "dht_autotune_projection": (_i, [_vp, _i, _i, ctypes.POINTER(_i), _dp]),
    "dht_hp_variance": (_i, [_dp, _i, _i, ctypes.POINTER(_i), _i, _d, ctypes.POINTER(HPVar)]),
    "dht_playback": (_i, [_dp, _dp, _i, _i, _dp, _dp, _i, ctypes.POINTER(_i), _i, _dp, _dp]),
    "dht_deflation_get_galerkin": (_i, [_vp, _dp, _dp, ctypes.POINTER(_i)]),
    "dht_state_save": (_i, [_vp, ctypes.c_char_p]),
    "dht_state_load": (_i, [_vp, ctypes.c_char_p]),
}

SOLVER_DC_FGMRES = 3
NN_CHANNELS = (24, 48, 48, 24)

_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises OSError if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError("libdhtrace.so is not built (run __graft_entry__.build()): %s" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def hp_variance(q, s_list, v_stoc: float = 0.0):
    """Run-to-run variance V_hp(s) of the HP estimate with Jackknife errors and
    the speedup R_s over plain noise; q: complex array [runs][probes]."""
    q = np.ascontiguousarray(q, dtype=np.complex128)
    R, S = q.shape
    sl = (ctypes.c_int * len(s_list))(*[int(s) for s in s_list])
    out = (HPVar * len(s_list))()
    check(load().dht_hp_variance(q.view(np.float64).ctypes.data_as(_dp), R, S, sl, len(s_list), float(v_stoc), out))
    return [{f[0]: getattr(o, f[0]) for f in HPVar._fields_} for o in out]


def theorem2(N: int, k: int, hermitian: bool, sum_all: float, sumsq_all: float, top) -> dict:
    """Theorem 2's expected deflated variance (and Remark 4's undeflated one)."""
    top = np.ascontiguousarray(np.asarray(top, dtype=np.float64).reshape(-1))
    out = Thm2()
    check(load().dht_theorem2(int(N), int(k), int(hermitian), float(sum_all), float(sumsq_all),
                              top.ctypes.data_as(_dp) if top.size else None, ctypes.byref(out)))
    return {f[0]: getattr(out, f[0]) for f in Thm2._fields_}


def playback(H, G5, coef, q, k_list, diagonal: bool = False):
    """Deflated quadratures and T_D with the leading kk basis vectors for each kk
    of k_list, from stored coefficients coef [2][k][n] and quadratic forms q [n]."""
    H = np.ascontiguousarray(H, dtype=np.complex128)
    G5 = np.ascontiguousarray(G5, dtype=np.complex128)
    coef = np.ascontiguousarray(coef, dtype=np.complex128)
    q = np.ascontiguousarray(q, dtype=np.complex128)
    k = H.shape[0]
    n = q.shape[0]
    kl = (ctypes.c_int * len(k_list))(*[int(v) for v in k_list])
    qd = np.zeros((len(k_list), n), dtype=np.complex128)
    td = np.zeros(len(k_list), dtype=np.complex128)
    check(load().dht_playback(H.view(np.float64).ctypes.data_as(_dp), G5.view(np.float64).ctypes.data_as(_dp), k,
                              int(diagonal), coef.view(np.float64).ctypes.data_as(_dp),
                              q.view(np.float64).ctypes.data_as(_dp), n, kl, len(k_list),
                              qd.view(np.float64).ctypes.data_as(_dp), td.view(np.float64).ctypes.data_as(_dp)))
    return qd, td


class DhtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dhtrace error %d: %s" % (code, msg))
        self.code = code


def check(rc: int, allow=()):
    if rc != DHT_OK and rc not in allow:
        raise DhtError(rc, load().dht_last_error().decode())
    return rc


def _ptr(t) -> int:
    return int(t.data_ptr())


def _as_f64_view(t):
    """complex128 torch tensor -> its data pointer (must be contiguous, on the GPU)."""
    import torch
    if t.dtype != torch.complex128 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous complex128 CUDA tensor")
    return _ptr(t)


def _np_dp(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Context:
    """One library context: lattice, gauge field, deflation basis, estimator state."""

    def __init__(self, L, mass: float, t_antiperiodic: bool = True, device: int = 0, stream=None):
        import torch
        self.L = tuple(int(v) for v in L)
        self._tuned = {}
        self.V = int(np.prod(self.L))
        self.N = 12 * self.V
        self.mass = float(mass)
        self.device = device
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        lat = Lattice((ctypes.c_int * 4)(*self.L), self.mass, int(t_antiperiodic))
        h = _vp()
        check(load().dht_create(ctypes.byref(lat), device, _vp(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.k = 0

    def close(self):
        if self.h:
            load().dht_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operator ---------------------------------------------------------
    def set_gauge(self, U):
        """U: complex128 CUDA tensor [4][Lt][Lz][Ly][Lx][3][3]."""
        check(load().dht_set_gauge(self.h, _as_f64_view(U)))

    def apply(self, X, op: int = OP_D, prec: int = FP64):
        """op(X) for X of shape [nrhs][Lt][Lz][Ly][Lx][4][3] (complex128 CUDA)."""
        Y = self.torch.empty_like(X)
        nrhs = X.shape[0]
        check(load().dht_apply(self.h, op, prec, _as_f64_view(X), _as_f64_view(Y), nrhs))
        return Y

    def apply_noalloc(self, X, Y, op: int = OP_D, prec: int = FP64):
        """Y = op(X) into a caller tensor Y with no device allocation in the
        library (fixed per-GPU scratch); asynchronous on the context stream."""
        check(load().dht_apply_noalloc(self.h, op, prec, _as_f64_view(X), _as_f64_view(Y), X.shape[0]))
        return Y

    def make_probes(self, seed: int, run: int, hp: bool, first: int, nrhs: int):
        Z = self.torch.empty((nrhs,) + self._spinor_shape(), dtype=self.torch.complex128, device="cuda")
        sp = ProbeSpec(seed, run, int(hp))
        check(load().dht_make_probes(self.h, ctypes.byref(sp), first, nrhs, _as_f64_view(Z)))
        return Z

    def probe_indices(self, seed: int, run: int, hp: bool, first: int, nrhs: int):
        k = self.torch.empty((nrhs, self.N), dtype=self.torch.uint8, device="cuda")
        s = self.torch.empty((nrhs, self.V), dtype=self.torch.int8, device="cuda")
        sp = ProbeSpec(seed, run, int(hp))
        check(load().dht_probe_indices(self.h, ctypes.byref(sp), first, nrhs, _ptr(k), _ptr(s)))
        return k, s

    def _spinor_shape(self):
        Lx, Ly, Lz, Lt = self.L
        return (Lt, Lz, Ly, Lx, 4, 3)

    # -- solver -----------------------------------------------------------
    @staticmethod
    def params(method=SOLVER_BICGSTAB_FP64, inner=FP32, tol=1e-10, maxiter=10000, restart=32,
               inner_tol=0.0, max_outer=0, fault_inject=0, history=0):
        return SolverParams(method, inner, tol, maxiter, restart, inner_tol, max_outer, fault_inject, history)

    def solve(self, Z, prm: SolverParams, allow_not_converged: bool = False):
        X = self.torch.empty_like(Z)
        nrhs = Z.shape[0]
        st = (SolveStats * nrhs)()
        allow = (DHT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        rc = check(load().dht_solve(self.h, ctypes.byref(prm), _as_f64_view(Z), _as_f64_view(X), nrhs, st), allow)
        return X, [dict(iters=s.iters, outer=s.outer, true_resid=s.true_resid, status=s.status) for s in st], rc

    # -- deflation --------------------------------------------------------
    def set_deflation(self, W, prec: int = FP64, block: int = 64, diagonal: bool = False):
        """W: complex128 CUDA tensor [k][N] (or [k][spinor shape]); returns T_D."""
        k = W.shape[0]
        self.begin_deflation(k, prec)
        for j in range(0, k, block):
            n = min(block, k - j)
            self.set_deflation_columns(j, W[j:j + n])
        return self.finalize_deflation(diagonal)

    def begin_deflation(self, k: int, prec: int):
        check(load().dht_deflation_begin(self.h, k, prec))
        self.k = k

    def set_deflation_columns(self, first: int, Wblock):
        Wblock = Wblock.contiguous()
        check(load().dht_deflation_set(self.h, first, Wblock.shape[0], _ptr(Wblock)))

    def eigensolve(self, k: int, prec: int = FP64, tol: float = 1e-10, max_iter: int = 200, degree: int = 16,
                   guard: int = 0, seed: int = 1, finalize: bool = True, allow_not_converged: bool = False):
        """Deflation basis from the library's eigensolver: the k eigenvectors of
        Q = g5 D of smallest |lambda|, stored in `prec`; with finalize, also the
        Galerkin M and T_D.  Returns (lambda, relative residuals, stats, T_D)."""
        self.begin_deflation(k, prec)
        lam = np.zeros(k)
        res = np.zeros(k)
        st = EigStats()
        prm = EigParams(float(tol), int(max_iter), int(degree), int(guard), int(seed))
        rc = load().dht_deflation_eigensolve(self.h, ctypes.byref(prm), _np_dp(lam), _np_dp(res), ctypes.byref(st))
        if rc != 0 and not (allow_not_converged and rc == -6):
            check(rc)
        stats = {f[0]: getattr(st, f[0]) for f in EigStats._fields_}
        stats["status"] = rc
        td = self.finalize_deflation() if finalize else None
        return lam, res, stats, td

    def lobpcg(self, k: int, prec: int = FP64, tol: float = 1e-9, max_iter: int = 500, block: int = 32,
               precond: bool = True, precond_tol: float = 1e-2, seed: int = 1, finalize: bool = True,
               allow_not_converged: bool = False):
        """Deflation basis from the preconditioned block eigensolver (LOBPCG on Q^2
        with locking).  Returns (sigma, relative residuals, stats, T_D)."""
        self.begin_deflation(k, prec)
        sig = np.zeros(k)
        res = np.zeros(k)
        st = LobpcgStats()
        prm = LobpcgParams(float(tol), int(max_iter), int(block), int(precond), float(precond_tol), int(seed))
        rc = load().dht_deflation_lobpcg(self.h, ctypes.byref(prm), _np_dp(sig), _np_dp(res), ctypes.byref(st))
        if rc != 0 and not (allow_not_converged and rc == DHT_ERR_NOT_CONVERGED):
            check(rc)
        stats = {f[0]: getattr(st, f[0]) for f in LobpcgStats._fields_}
        stats["status"] = rc
        td = self.finalize_deflation() if finalize else None
        return sig, res, stats, td

    def deflation_columns(self, first: int, count: int):
        """Stored basis columns (rounded to the storage precision) as a
        complex128 CUDA tensor [count][N]."""
        out = self.torch.empty((count, self.N), dtype=self.torch.complex128, device="cuda")
        check(load().dht_deflation_get(self.h, first, count, _ptr(out)))
        return out

    def finalize_deflation(self, diagonal: bool = False):
        td = np.zeros(2)
        fn = load().dht_deflation_finalize_diag if diagonal else load().dht_deflation_finalize
        check(fn(self.h, _np_dp(td)))
        return complex(td[0], td[1])

    def project_probes(self, seed: int, run: int, hp: bool, first: int, nrhs: int):
        sp = ProbeSpec(seed, run, int(hp))
        c1 = np.zeros(2 * self.k * nrhs)
        c2 = np.zeros(2 * self.k * nrhs)
        check(load().dht_project_probes(self.h, ctypes.byref(sp), first, nrhs, _np_dp(c1), _np_dp(c2)))
        return (c1.view(np.complex128).reshape(self.k, nrhs), c2.view(np.complex128).reshape(self.k, nrhs))

    def set_projection_window(self, nprobes: int):
        """Project up to 64 probes per pass over a BF16 basis inside
        trace_batch (0: each batch on its own); also drops the current window."""
        check(load().dht_set_projection_window(self.h, int(nprobes)))

    # -- instrumentation --------------------------------------------------
    PROF_CLASSES = {"hop_fp64": 0, "hop_fp32": 1, "hop_bf16": 2, "proj_mfma": 3, "proj_generic": 4, "conv": 5, "proj_sp": 6}

    def workspace_size(self, max_nrhs: int, prm: SolverParams) -> int:
        """Device bytes that trace_batch / solve need for batches up to max_nrhs with prm."""
        n = ctypes.c_size_t(0)
        check(load().dht_workspace_size(self.h, int(max_nrhs), ctypes.byref(prm), ctypes.byref(n)))
        return n.value

    def set_workspace(self, buf):
        """Hand over a caller-owned device buffer (a uint8 CUDA tensor of at least
        workspace_size bytes; kept referenced here), or None for library workspace."""
        if buf is None:
            check(load().dht_set_workspace(self.h, None, 0))
            self._workspace = None
            return
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("expected a contiguous CUDA tensor")
        check(load().dht_set_workspace(self.h, _vp(_ptr(buf)), buf.numel() * buf.element_size()))
        self._workspace = buf

    def workspace_trim(self):
        """Free the library-owned workspace (links, basis, weights and estimates stay)."""
        check(load().dht_workspace_trim(self.h))

    def profile(self, on: bool = True):
        check(load().dht_profile_enable(self.h, int(on)))

    def profile_reset(self):
        check(load().dht_profile_reset(self.h))

    def profile_get(self, cls):
        if isinstance(cls, str):
            cls = self.PROF_CLASSES[cls]
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0)
        by = ctypes.c_double(0)
        check(load().dht_profile_get(self.h, cls, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return dict(count=n.value, ms=ms.value, bytes=by.value)

    def deflation_galerkin(self):
        """(H = W^H Q W, G5 = W^H g5 W, diagonal) of the finalized basis."""
        H = np.zeros(2 * self.k * self.k)
        G = np.zeros(2 * self.k * self.k)
        d = ctypes.c_int(0)
        check(load().dht_deflation_get_galerkin(self.h, _np_dp(H), _np_dp(G), ctypes.byref(d)))
        return (H.view(np.complex128).reshape(self.k, self.k), G.view(np.complex128).reshape(self.k, self.k),
                bool(d.value))

    def deflation_M(self):
        M = np.zeros(2 * self.k * self.k)
        check(load().dht_deflation_get_M(self.h, _np_dp(M)))
        return M.view(np.complex128).reshape(self.k, self.k)

    def clear_deflation(self):
        check(load().dht_deflation_clear(self.h))
        self.k = 0

    def project(self, Z):
        nrhs = Z.shape[0]
        c1 = np.zeros(2 * self.k * nrhs)
        c2 = np.zeros(2 * self.k * nrhs)
        check(load().dht_project(self.h, _as_f64_view(Z), nrhs, _np_dp(c1), _np_dp(c2)))
        return (c1.view(np.complex128).reshape(self.k, nrhs), c2.view(np.complex128).reshape(self.k, nrhs))

    # -- Algorithm 1 ------------------------------------------------------
    def trace_batch(self, seed: int, run: int, hp: bool, first: int, nrhs: int, prm: SolverParams,
                    want_coef: bool = False, allow_not_converged: bool = False):
        sp = ProbeSpec(seed, run, int(hp))
        rec = (Record * nrhs)()
        coef = np.zeros(2 * 2 * self.k * nrhs) if (want_coef and self.k) else None
        allow = (DHT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        check(load().dht_trace_batch(self.h, ctypes.byref(sp), first, nrhs, ctypes.byref(prm), rec,
                                     _np_dp(coef) if coef is not None else None), allow)
        out = [dict(q=complex(r.q_re, r.q_im), q_defl=complex(r.qd_re, r.qd_im), iters=r.s.iters,
                    outer=r.s.outer, true_resid=r.s.true_resid, status=r.s.status) for r in rec]
        if coef is not None:
            cc = coef.view(np.complex128).reshape(2, self.k, nrhs)
            return out, cc[0], cc[1]
        return out

    def estimate(self):
        e = Estimate()
        check(load().dht_estimate_get(self.h, ctypes.byref(e)))
        return {f[0]: getattr(e, f[0]) for f in Estimate._fields_}

    def reset_estimate(self):
        check(load().dht_estimate_reset(self.h))

    # -- traces Tr(Gamma D^-1) over the same deflation space ----------------
    def gamma_set(self, gammas) -> np.ndarray:
        """Register spin matrices (array [ng][4][4] complex); returns T_D(Gamma) per matrix."""
        G = np.ascontiguousarray(np.asarray(gammas, dtype=np.complex128).reshape(-1, 4, 4))
        ng = G.shape[0]
        td = np.zeros(max(1, ng), dtype=np.complex128)
        check(load().dht_gamma_set(self.h, _np_dp(G.view(np.float64)), ng, _np_dp(td.view(np.float64))))
        self._ng = ng   # only once the library has accepted them
        return td[:ng]

    def trace_gamma_batch(self, seed: int, run: int, hp: bool, first: int, nrhs: int, prm: SolverParams,
                          allow_not_converged: bool = False):
        """Returns (q [ng][nrhs], q_defl [ng][nrhs], per-probe solve stats)."""
        sp = ProbeSpec(seed, run, int(hp))
        ng = getattr(self, "_ng", 0)
        rec = (Record * max(1, ng * nrhs))()
        allow = (DHT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        check(load().dht_trace_gamma_batch(self.h, ctypes.byref(sp), first, nrhs, ctypes.byref(prm), rec), allow)
        q = np.array([complex(r.q_re, r.q_im) for r in rec[:ng * nrhs]]).reshape(ng, nrhs)
        qd = np.array([complex(r.qd_re, r.qd_im) for r in rec[:ng * nrhs]]).reshape(ng, nrhs)
        stats = [dict(iters=r.s.iters, outer=r.s.outer, true_resid=r.s.true_resid, status=r.s.status)
                 for r in rec[:nrhs]]
        return q, qd, stats

    def distance_profile(self, rows, prm: SolverParams, deflate: bool = False, hp_vectors: int = 0,
                         allow_not_converged: bool = False):
        """(W [nrows][dmax+1], m [dmax+1]): Section 6.2's distance profile of sampled rows."""
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
        nd = sum(l // 2 for l in self.L) + 1
        W = np.zeros((rows.size, nd))
        m = np.zeros(nd, dtype=np.int64)
        allow = (DHT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        check(load().dht_distance_profile(self.h, rows.ctypes.data_as(ctypes.POINTER(_i64)), rows.size, int(deflate),
                                          int(hp_vectors), ctypes.byref(prm), _np_dp(W),
                                          m.ctypes.data_as(ctypes.POINTER(_i64))), allow)
        return W, m

    def gamma_estimate(self, g: int):
        e = Estimate()
        check(load().dht_gamma_estimate_get(self.h, g, ctypes.byref(e)))
        return {f[0]: getattr(e, f[0]) for f in Estimate._fields_}

    def timings(self):
        t = np.zeros(5)
        check(load().dht_last_timings(self.h, _np_dp(t), 5))
        return dict(probes=t[0], solve=t[1], project=t[2], qform=t[3], total=t[4])

    SOLVER_COUNTERS = ("predicted_checks", "predicted_failed", "inplace_updates", "reentries")

    def solver_counters(self):
        out = (_i64 * 4)()
        check(load().dht_solver_counters(self.h, out, 4))
        return dict(zip(self.SOLVER_COUNTERS, list(out)))

    # -- learned preconditioner ------------------------------------------
    @staticmethod
    def _flat_weights(Ws):
        return np.ascontiguousarray(np.concatenate([np.asarray(W, dtype=np.float32).ravel() for W in Ws]))

    @staticmethod
    def _split_weights(flat):
        out, off = [], 0
        for l in range(3):
            cin, cout = NN_CHANNELS[l], NN_CHANNELS[l + 1]
            n = 81 * cout * cin
            out.append(flat[off:off + n].reshape(81, cout, cin).astype(np.float64))
            off += n
        return out

    def nn_init(self, seed: int):
        check(load().dht_nn_init(self.h, seed))

    def nn_set_skip(self, s: float):
        """M(r) = net(r) + s r; s = 1 / (4 + m) for the Jacobi-plus-correction form."""
        check(load().dht_nn_set_skip(self.h, float(s)))

    def nn_set_weights(self, Ws):
        flat = self._flat_weights(Ws)
        check(load().dht_nn_set_weights(self.h, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def nn_get_weights(self):
        flat = np.zeros(load().dht_nn_num_weights(), dtype=np.float32)
        check(load().dht_nn_get_weights(self.h, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return self._split_weights(flat)

    def nn_forward(self, R):
        E = self.torch.empty_like(R)
        check(load().dht_nn_forward(self.h, _as_f64_view(R), _as_f64_view(E), R.shape[0]))
        return E

    def nn_grad(self, R, E):
        flat = np.zeros(load().dht_nn_num_weights(), dtype=np.float32)
        loss = ctypes.c_double(0)
        check(load().dht_nn_grad(self.h, _as_f64_view(R), _as_f64_view(E), R.shape[0],
                                 flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return loss.value, self._split_weights(flat)

    def nn_train(self, R, E, epochs: int = 1, batch: int = 16, lr: float = 1e-3) -> float:
        loss = ctypes.c_double(0)
        check(load().dht_nn_train(self.h, _as_f64_view(R), _as_f64_view(E), R.shape[0], epochs, batch, lr,
                                  ctypes.byref(loss)))
        return loss.value

    def nn_make_pairs(self, seed: int, run: int, hp: bool, first: int, nrhs: int, restart: int, cap: int):
        shape = (cap,) + self._spinor_shape()
        R = self.torch.zeros(shape, dtype=self.torch.complex128, device="cuda")
        E = self.torch.zeros(shape, dtype=self.torch.complex128, device="cuda")
        sp = ProbeSpec(seed, run, int(hp))
        cnt = ctypes.c_int(0)
        check(load().dht_nn_make_pairs(self.h, ctypes.byref(sp), first, nrhs, restart, _as_f64_view(R),
                                       _as_f64_view(E), cap, ctypes.byref(cnt)))
        return R[:cnt.value], E[:cnt.value]

    # ---- launch-shape autotuning -------------------------------------------
    def hop_config(self, prec: int, nrhs: int, epilogue: int = HOP_PLAIN) -> dict:
        h = HopConfig()
        check(load().dht_hop_config_get(self.h, prec, nrhs, epilogue, ctypes.byref(h)))
        return _hop_dict(h)

    def set_hop_config(self, prec: int, nrhs: int, cfg: dict | None, epilogue: int | None = None):
        """Install a hopping-kernel shape for (prec, nrhs) and one epilogue
        class (both when epilogue is None); None restores the default."""
        for cls in (tuple(HOP_CLASSES) if epilogue is None else (epilogue,)):
            if cfg is None:
                check(load().dht_hop_config_set(self.h, prec, nrhs, cls, None))
                continue
            h = HopConfig(int(cfg["form"]), int(cfg.get("streaming_stores", 1)), int(cfg.get("t_chunk", 0)),
                          int(cfg.get("rhs_group", 0)), int(cfg.get("z_block", 0)))
            check(load().dht_hop_config_set(self.h, prec, nrhs, cls, ctypes.byref(h)))

    def autotune_hop(self, prec: int, nrhs: int, reps: int = 10) -> dict:
        """Time every valid hopping-kernel shape for (prec, nrhs), per epilogue
        class, and keep the fastest one whose output matches the default's to
        rounding."""
        r = TuneResult()
        check(load().dht_autotune_hop(self.h, prec, nrhs, reps, ctypes.byref(r)))
        best = {HOP_CLASSES[k]: _hop_dict(r.best[k]) for k in HOP_CLASSES}
        out = {"prec": prec, "nrhs": nrhs, "best": best,
               "best_form": {c: HOP_FORMS[b["form"]] for c, b in best.items()},
               "best_ms": {HOP_CLASSES[k]: r.best_ms[k] for k in HOP_CLASSES},
               "default_ms": {HOP_CLASSES[k]: r.default_ms[k] for k in HOP_CLASSES},
               "candidates": r.candidates, "rejected": r.rejected, "max_rel_diff": r.max_rel_diff}
        self._tuned[(prec, nrhs)] = out
        return out

    def autotune(self, prec: int, nrhs: int, reps: int = 10, cache_path: str | None = None) -> dict:
        """The library's autotuner with its text cache file (shapes reused when
        the file holds this lattice, prec and nrhs)."""
        r = TuneResult()
        cp = cache_path.encode() if cache_path else None
        check(load().dht_autotune(self.h, prec, nrhs, reps, cp, ctypes.byref(r)))
        return {"best": {HOP_CLASSES[k]: _hop_dict(r.best[k]) for k in HOP_CLASSES},
                "best_ms": {HOP_CLASSES[k]: r.best_ms[k] for k in HOP_CLASSES},
                "candidates": r.candidates, "rejected": r.rejected}

    def autotune_batch(self, seed: int, run: int, hp: bool, prm: SolverParams, candidates=(16, 32, 64),
                       mem_budget: int = 0, reps: int = 2) -> dict:
        """Time Algorithm-1 batches of each candidate size (within the memory
        budget) and return the fastest with the per-candidate figures."""
        out = BatchTune()
        cand = (ctypes.c_int * len(candidates))(*candidates)
        sp = ProbeSpec(seed, run, int(hp))
        check(load().dht_autotune_batch(self.h, ctypes.byref(sp), ctypes.byref(prm), cand, len(candidates),
                                        int(mem_budget), int(reps), ctypes.byref(out)))
        names = {0: "invalid", 1: "timed", 2: "over_budget", 3: "failed"}
        return {"best_nrhs": out.best_nrhs,
                "candidates": [{"nrhs": out.nrhs[i], "status": names[out.status[i]],
                                "rhs_per_s": out.rhs_per_s[i], "workspace_bytes": out.workspace[i]}
                               for i in range(out.candidates)]}

    def autotune_projection(self, nrhs: int, reps: int = 3) -> dict:
        w = ctypes.c_int(0)
        ms = ctypes.c_double(0)
        check(load().dht_autotune_projection(self.h, int(nrhs), int(reps), ctypes.byref(w), ctypes.byref(ms)))
        return {"workgroups": w.value, "ms_per_pass": ms.value}

    def save_state(self, path: str):
        """Checkpoint the running estimates."""
        check(load().dht_state_save(self.h, path.encode()))

    def load_state(self, path: str):
        """Resume the running estimates from a checkpoint of the same lattice,
        operator and deflation space."""
        check(load().dht_state_load(self.h, path.encode()))

    def tuning_table(self) -> dict:
        """The shapes installed by autotune_hop / load_tuning, keyed
        "prec:nrhs", with the lattice they were measured on (JSON-ready)."""
        return {"lattice": list(self.L), "entries": {"%d:%d" % k: v for k, v in self._tuned.items()}}

    def save_tuning(self, path: str):
        with open(path, "w") as f:
            json.dump(self.tuning_table(), f, indent=1)

    def load_tuning(self, path: str) -> int:
        """Install the shapes of a saved table if it was measured on this
        lattice; returns the number installed."""
        with open(path) as f:
            tab = json.load(f)
        if list(tab.get("lattice", [])) != list(self.L):
            return 0
        n = 0
        for key, ent in tab.get("entries", {}).items():
            prec, nrhs = (int(v) for v in key.split(":"))
            if any(name not in ent.get("best", {}) for name in HOP_CLASSES.values()):
                continue   # a table from before an epilogue class existed: tune again
            for cls, name in HOP_CLASSES.items():
                self.set_hop_config(prec, nrhs, ent["best"][name], cls)
            self._tuned[(prec, nrhs)] = ent
            n += 1
        return n

    def bench_hop(self, prec: int, nrhs: int, warmup: int = 3, reps: int = 10) -> float:
        ms = ctypes.c_double(0.0)
        check(load().dht_bench_hop(self.h, prec, nrhs, warmup, reps, ctypes.byref(ms)))
        return ms.value
