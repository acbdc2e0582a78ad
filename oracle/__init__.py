"""CPU oracle for the transformed Radau IIA linear solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1701_07181_amd``) and never imports it.

The numerical work lives in ``oracle.c`` (plain FP64 loops); this module only
builds it with gcc and marshals NumPy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

PC_COUPLED, PC_SHIFTED, PC_UNSHIFTED, PC_NONE = 0, 1, 2, 3
PC_NAMES = {"coupled": PC_COUPLED, "uncoupled_shifted": PC_SHIFTED,
            "uncoupled": PC_UNSHIFTED, "none": PC_NONE}


def build(openmp: bool = False) -> str:
    """Compile oracle.c: liboracle.so (plain -O2, single-threaded: the
    library every test uses) or, with openmp, liboracle_omp.so (the same
    source with its OpenMP loops enabled, for the all-cores CPU baseline
    only; its reductions sum in a thread-dependent order)."""
    out = LIB_OMP if openmp else LIB
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared"] + (["-fopenmp"] if openmp else []) + \
          ["-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None
_omp = False


def use_openmp(on: bool = True):
    """Select the OpenMP build for the calls that follow (bench only).  Must
    be called before the first oracle call of the process."""
    global _omp
    if _lib is not None and on != _omp:
        raise RuntimeError("the oracle library is already loaded")
    _omp = on
    # idle threads sleep between the many short parallel loops instead of
    # spinning on the cores the serial parts run on (read by the OpenMP
    # runtime when the library loads)
    if on:
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")


def lib():
    global _lib
    if _lib is None:
        # IRK_ORACLE_LIB: a build of oracle.c made elsewhere (the sanitizer
        # test's instrumented copy), loaded as it is
        path = os.environ.get("IRK_ORACLE_LIB") or (LIB_OMP if _omp else LIB)
        if path in (LIB, LIB_OMP) and (not os.path.exists(path) or
                                       os.path.getmtime(path) < os.path.getmtime(SRC)):
            build(openmp=_omp)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_radau_iia.argtypes = [C.c_int, dp, dp, dp]
        L.orc_inverse.argtypes = [C.c_int, dp, dp]
        L.orc_shifts.argtypes = [C.c_int, dp, C.c_int, dp]
        L.orc_matvec_transformed.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_matvec_untransformed.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_coupled_nnzb.argtypes = [C.c_int, C.c_int, ip]
        L.orc_coupled_nnzb.restype = C.c_long
        L.orc_build_coupled.argtypes = [C.c_void_p, dp, ip, ip, dp]
        L.orc_build_stage.argtypes = [C.c_void_p, C.c_int, C.c_double, ip, ip, dp]
        L.orc_ilu0.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, ip]
        L.orc_ilu0_apply.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, ip, dp, dp]
        L.orc_bsr_matvec.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, dp]
        L.orc_coupled_explicit.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_solve.argtypes = [C.c_void_p, dp, C.c_void_p, dp, dp, C.c_void_p, dp]
        L.orc_pc_apply.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_bf16_from_f32.argtypes = [C.c_float]
        L.orc_bf16_from_f32.restype = C.c_uint16
        L.orc_f16_from_f32.argtypes = [C.c_float]
        L.orc_f16_from_f32.restype = C.c_uint16
        L.orc_f16_block_exponent.argtypes = [C.c_size_t, dp]
        L.orc_f16_block_exponent.restype = C.c_int
        L.orc_quantize_bf16.argtypes = [C.c_size_t, dp, C.POINTER(C.c_uint16)]
        L.orc_quantize_f16_scaled.argtypes = [C.c_size_t, dp, C.c_int, C.POINTER(C.c_uint16)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class _Problem(C.Structure):
    _fields_ = [("s", C.c_int), ("T", C.c_int), ("m", C.c_int), ("nJ", C.c_int),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("J", C.c_void_p), ("M", C.c_void_p), ("dt", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("pc", C.c_int), ("shift_rule", C.c_int), ("restart", C.c_int),
                ("maxit", C.c_int), ("orth", C.c_int), ("rtol", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("converged", C.c_int), ("iters", C.c_int), ("restarts", C.c_int),
                ("status", C.c_int), ("rel_res_true", C.c_double),
                ("rel_res_est", C.c_double)]


class Problem:
    """Holds contiguous copies of a system's arrays and the ctypes struct."""

    def __init__(self, sys, dt: Optional[float] = None, s: Optional[int] = None):
        self.s = int(sys.s if s is None else s)
        self.T, self.m, self.nJ = int(sys.T), int(sys.m), int(sys.nJ)
        self.dt = float(sys.dt if dt is None else dt)
        self.row_ptr = np.ascontiguousarray(sys.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(sys.col_idx, dtype=np.int32)
        self.J = np.ascontiguousarray(sys.J, dtype=np.float64)
        self.M = np.ascontiguousarray(sys.M, dtype=np.float64)
        self.st = _Problem(self.s, self.T, self.m, self.nJ,
                           self.row_ptr.ctypes.data, self.col_idx.ctypes.data,
                           self.J.ctypes.data, self.M.ctypes.data, self.dt)

    @property
    def N(self):
        return self.s * self.T * self.m

    def ptr(self):
        return C.byref(self.st)


# ----------------------------------------------------------------------------
# tableau
# ----------------------------------------------------------------------------

def radau_iia(s: int):
    """(A, b, c) of the s-stage Radau IIA method (App. A construction)."""
    A = np.zeros((s, s)); b = np.zeros(s); c = np.zeros(s)
    rc = lib().orc_radau_iia(s, _d(A), _d(b), _d(c))
    if rc != 0:
        raise ValueError(f"radau_iia({s}) failed")
    return A, b, c


def inverse(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.zeros_like(A)
    if lib().orc_inverse(n, _d(A), _d(out)) != 0:
        raise np.linalg.LinAlgError("singular")
    return out


def shifts(Ainv: np.ndarray, rule: int = 0) -> np.ndarray:
    Ainv = np.ascontiguousarray(Ainv, dtype=np.float64)
    s = Ainv.shape[0]
    a = np.zeros(s)
    lib().orc_shifts(s, _d(Ainv), rule, _d(a))
    return a


# ----------------------------------------------------------------------------
# operators
# ----------------------------------------------------------------------------

def matvec(prob: Problem, Ainv: np.ndarray, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(prob.N)
    Ainv = np.ascontiguousarray(Ainv, dtype=np.float64)
    lib().orc_matvec_transformed(prob.ptr(), _d(Ainv), _d(x), _d(y))
    return y


def matvec_untransformed(prob: Problem, A: np.ndarray, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(prob.N)
    A = np.ascontiguousarray(A, dtype=np.float64)
    lib().orc_matvec_untransformed(prob.ptr(), _d(A), _d(x), _d(y))
    return y


# ----------------------------------------------------------------------------
# generic block matrices and ILU(0)
# ----------------------------------------------------------------------------

class BlockMatrix:
    """Generic block-sparse matrix: nb block rows, m x m row-major blocks."""

    def __init__(self, nb, m, ptr, col, val):
        self.nb, self.m = int(nb), int(m)
        self.ptr = np.ascontiguousarray(ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.dlu = None
        self.dpiv = None

    def copy(self):
        return BlockMatrix(self.nb, self.m, self.ptr.copy(), self.col.copy(), self.val.copy())

    def dense(self) -> np.ndarray:
        m = self.m
        D = np.zeros((self.nb * m, self.nb * m))
        for i in range(self.nb):
            for a in range(self.ptr[i], self.ptr[i + 1]):
                j = self.col[a]
                D[i * m:(i + 1) * m, j * m:(j + 1) * m] = self.val[a]
        return D

    def block(self, i, j):
        for a in range(self.ptr[i], self.ptr[i + 1]):
            if self.col[a] == j:
                return self.val[a]
        return None

    def ilu0(self) -> "BlockMatrix":
        """Factor in place (Alg. 1); returns self."""
        self.dlu = np.zeros((self.nb, self.m, self.m))
        self.dpiv = np.zeros((self.nb, self.m), dtype=np.int32)
        rc = lib().orc_ilu0(self.nb, self.m, _i(self.ptr), _i(self.col), _d(self.val),
                            _d(self.dlu), _i(self.dpiv))
        if rc != 0:
            raise np.linalg.LinAlgError(f"singular pivot at block row {rc - 1}")
        return self

    def apply(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        z = np.zeros_like(v)
        lib().orc_ilu0_apply(self.nb, self.m, _i(self.ptr), _i(self.col), _d(self.val),
                             _d(self.dlu), _i(self.dpiv), _d(v), _d(z))
        return z

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.nb * self.m)
        lib().orc_bsr_matvec(self.nb, self.m, _i(self.ptr), _i(self.col), _d(self.val),
                             _d(x), _d(y))
        return y


def build_coupled(prob: Problem, Ainv: np.ndarray) -> BlockMatrix:
    nnz = lib().orc_coupled_nnzb(prob.s, prob.T, _i(prob.row_ptr))
    nb = prob.s * prob.T
    ptr = np.zeros(nb + 1, dtype=np.int32)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros((nnz, prob.m, prob.m))
    Ainv = np.ascontiguousarray(Ainv, dtype=np.float64)
    lib().orc_build_coupled(prob.ptr(), _d(Ainv), _i(ptr), _i(col), _d(val))
    return BlockMatrix(nb, prob.m, ptr, col, val)


def build_stage(prob: Problem, k: int, diag_coeff: float) -> BlockMatrix:
    nnz = int(prob.row_ptr[-1])
    ptr = np.zeros(prob.T + 1, dtype=np.int32)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros((nnz, prob.m, prob.m))
    lib().orc_build_stage(prob.ptr(), k, float(diag_coeff), _i(ptr), _i(col), _d(val))
    return BlockMatrix(prob.T, prob.m, ptr, col, val)


def coupled_explicit(prob: Problem, Ainv: np.ndarray):
    """Pivot blocks P[s][T] and cross-stage blocks C[s][s][T] of the explicit
    coupled factorization."""
    s, T, m = prob.s, prob.T, prob.m
    P = np.zeros((s, T, m, m))
    Cb = np.zeros((s, s, T, m, m))
    Ainv = np.ascontiguousarray(Ainv, dtype=np.float64)
    rc = lib().orc_coupled_explicit(prob.ptr(), _d(Ainv), _d(P), _d(Cb))
    if rc != 0:
        raise np.linalg.LinAlgError("singular pivot")
    return P, Cb


# ----------------------------------------------------------------------------
# solves
# ----------------------------------------------------------------------------

def pc_apply(prob: Problem, A: np.ndarray, pc: str, v: np.ndarray, shift_rule: int = 0):
    """z = P^{-1} v for one vector [N] or a stack [q, N]."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    nvec = 1 if v.ndim == 1 else v.shape[0]
    z = np.zeros_like(v)
    A = np.ascontiguousarray(A, dtype=np.float64)
    rc = lib().orc_pc_apply(prob.ptr(), _d(A), PC_NAMES[pc], shift_rule, nvec, _d(v), _d(z))
    if rc != 0:
        raise np.linalg.LinAlgError(f"pc_apply failed ({rc})")
    return z


def solve(prob: Problem, A: np.ndarray, rhs: np.ndarray, pc: str = "coupled",
          rtol: float = 1e-10, restart: int = 30, maxit: int = 1000, orth: str = "mgs",
          x0: Optional[np.ndarray] = None, shift_rule: int = 0, history: bool = False):
    """GMRES solve of B W = R.  Returns (x, info dict[, history])."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.zeros(prob.N) if x0 is None else np.array(x0, dtype=np.float64)
    opts = _Opts(PC_NAMES[pc], shift_rule, restart, maxit, 1 if orth == "cgs2" else 0, rtol)
    info = _Info()
    hist = np.zeros(maxit + 1)
    rc = lib().orc_solve(prob.ptr(), _d(A), C.byref(opts), _d(rhs), _d(x), C.byref(info),
                         _d(hist))
    d = dict(status=rc, converged=bool(info.converged), iters=info.iters,
             restarts=info.restarts, rel_res_true=info.rel_res_true,
             rel_res_est=info.rel_res_est)
    if history:
        return x, d, hist[:info.iters].copy()
    return x, d


# ----------------------------------------------------------------------------
# quantizers
# ----------------------------------------------------------------------------

def bf16_bits(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    q = np.zeros(x.size, dtype=np.uint16)
    lib().orc_quantize_bf16(x.size, _d(x), q.ctypes.data_as(C.POINTER(C.c_uint16)))
    return q


def f16_block_exponent(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return int(lib().orc_f16_block_exponent(x.size, _d(x)))


def f16_scaled_bits(x: np.ndarray, e: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    q = np.zeros(x.size, dtype=np.uint16)
    lib().orc_quantize_f16_scaled(x.size, _d(x), int(e), q.ctypes.data_as(C.POINTER(C.c_uint16)))
    return q


def f32_to_bf16_bits(f: float) -> int:
    return int(lib().orc_bf16_from_f32(float(f)))


def f32_to_f16_bits(f: float) -> int:
    return int(lib().orc_f16_from_f32(float(f)))
