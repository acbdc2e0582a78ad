"""Python binding of libirk, the gfx950 solver of the transformed Radau IIA
Newton system  (A^{-1} (x) M - dt diag(J_k)) W = R  (Pazner & Persson,
Sec. 4.3, Eq. big-irk) by restarted GMRES with block ILU(0).

This module only marshals arguments: every step of the solve runs in the HIP
kernels of ``libirk.so`` (built by ``build.py``).  PyTorch provides device
memory and the stream.  If the library is missing this import fails; there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libirk.so")

(OK, ERR_ARG, ERR_NOMEM, ERR_SINGULAR, ERR_NOCONV, ERR_BREAKDOWN, ERR_NONFINITE, ERR_DEVICE, ERR_STATE,
 ERR_INTERNAL) = range(10)
PC = {"coupled": 0, "uncoupled_shifted": 1, "uncoupled": 2, "none": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16s": 3}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python paper_1701_07181_amd/build.py` "
                      "(or __graft_entry__.build()) first")
_L = C.CDLL(LIB_PATH)


class IrkError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_L.irk_status_str(status).decode()} (status {status})")


class _Problem(C.Structure):
    _fields_ = [("s", C.c_int), ("A", C.c_void_p), ("T", C.c_int), ("m", C.c_int),
                ("nnzb", C.c_int), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("J", C.c_void_p), ("nJ", C.c_int), ("M", C.c_void_p), ("dt", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("pc", C.c_int), ("shift_rule", C.c_int), ("alpha", C.c_void_p),
                ("matvec_prec", C.c_int), ("factor_prec", C.c_int), ("restart", C.c_int),
                ("max_iters", C.c_int), ("max_outer", C.c_int), ("rtol", C.c_double),
                ("inner_rtol", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("converged", C.c_int), ("iters", C.c_int), ("outer_iters", C.c_int),
                ("restarts", C.c_int), ("equiv_mults", C.c_int), ("rel_res_true", C.c_double),
                ("rel_res_est", C.c_double), ("bad_element", C.c_int), ("ms_factor", C.c_float),
                ("ms_solve", C.c_float)]


class _Prof(C.Structure):
    _fields_ = [("matvec_count", C.c_int), ("matvec_ms", C.c_double),
                ("matvec32_count", C.c_int), ("matvec32_ms", C.c_double),
                ("pc_count", C.c_int), ("pc_ms", C.c_double),
                ("orth_count", C.c_int), ("orth_ms", C.c_double),
                ("factor_count", C.c_int), ("factor_ms", C.c_double),
                ("dropped", C.c_int), ("untr_count", C.c_int), ("untr_ms", C.c_double)]


class _Rhs(C.Structure):
    _fields_ = [("g", C.c_void_p), ("omega", C.c_double), ("eps", C.c_double)]


class _StepInfo(C.Structure):
    _fields_ = [("converged", C.c_int), ("newton_iters", C.c_int), ("gmres_iters", C.c_int),
                ("equiv_mults", C.c_int), ("factorizations", C.c_int), ("update_norm", C.c_double),
                ("ms", C.c_float)]


class _Tune(C.Structure):
    _fields_ = [("matvec_teams", C.c_int), ("sweep_big_min", C.c_int), ("sweep_teams", C.c_int),
                ("from_cache", C.c_int), ("matvec_us", C.c_float), ("sweep_us", C.c_float),
                ("sweep_big_form", C.c_int), ("sweep_flow", C.c_int),
                ("sweep_chain_max", C.c_int), ("sweep_split", C.c_int)]


_vp = C.c_void_p
_L.irk_status_str.restype = C.c_char_p
_L.irk_status_str.argtypes = [C.c_int]
_L.irk_default_options.argtypes = [C.POINTER(_Options)]
_L.irk_workspace_size.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(C.c_size_t)]
_L.irk_setup.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), _vp, C.c_size_t, _vp, C.POINTER(_vp)]
_L.irk_update_values.argtypes = [_vp, _vp, _vp, C.c_double]
_L.irk_factor_ilu.argtypes = [_vp]
_L.irk_factor_ilu_async.argtypes = [_vp]
_L.irk_gmres_solve.argtypes = [_vp, _vp, _vp, C.POINTER(_Info)]
_L.irk_solve_batched.argtypes = [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.c_int, C.POINTER(_Info)]
_L.irk_solve_batched_noalloc.argtypes = [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.c_int, _vp,
                                         C.POINTER(_Info)]
_L.irk_batch_workspace_size.argtypes = [C.c_int, C.c_longlong, C.POINTER(C.c_size_t)]
_L.irk_batch_create.argtypes = [C.c_int, C.c_longlong, _vp, C.c_size_t, _vp, C.POINTER(_vp)]
_L.irk_batch_admit.argtypes = [_vp, _vp, _vp, _vp, C.c_longlong]
_L.irk_batch_advance.argtypes = [_vp, C.c_int]
_L.irk_batch_retire.argtypes = [_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_int), C.POINTER(_Info), C.c_int, C.POINTER(C.c_int)]
_L.irk_batch_pending.argtypes = [_vp]
_L.irk_batch_destroy.argtypes = [_vp]
_L.irk_apply_operator.argtypes = [_vp, _vp, _vp]
_L.irk_apply_preconditioner.argtypes = [_vp, _vp, _vp]
_L.irk_apply_operator_inner.argtypes = [_vp, _vp, _vp]
_L.irk_apply_operator_untransformed.argtypes = [_vp, C.c_int, _vp, _vp]
_L.irk_apply_preconditioner_inner.argtypes = [_vp, _vp, _vp]
_L.irk_export_factors.argtypes = [_vp, _vp, _vp]
_L.irk_last_bad_element.argtypes = [_vp]
_L.irk_destroy.argtypes = [_vp]
_L.irk_radau_iia.argtypes = [C.c_int, _vp, _vp, _vp]
_L.irk_profile_enable.argtypes = [_vp, C.c_int]
_L.irk_quantize_blocks.argtypes = [_vp, C.c_longlong, C.c_int, C.c_int, _vp, _vp, _vp]
_L.irk_profile_read.argtypes = [_vp, C.POINTER(_Prof)]
_L.irk_autotune.argtypes = [_vp, C.c_int, C.POINTER(_Tune)]
_L.irk_factor_batched.argtypes = [_vp, C.POINTER(_vp), C.c_int, C.POINTER(C.c_int)]
_L.irk_step_workspace_size.argtypes = [_vp, C.POINTER(C.c_size_t)]
_L.irk_radau_step.argtypes = [_vp, C.POINTER(_Rhs), _vp, C.c_double, _vp, _vp, C.c_double, C.c_int,
                              _vp, C.c_size_t, C.POINTER(_StepInfo)]
_L.irk_dirk_tableau.argtypes = [C.c_int, C.POINTER(C.c_int), _vp, _vp, _vp]
_L.irk_dirk_workspace_size.argtypes = [_vp, C.c_int, C.POINTER(C.c_size_t)]
_ip = C.POINTER(C.c_int)
_L.irk_level_schedule.argtypes = [C.c_int, C.c_int, _vp, _vp, _vp, _vp, _ip, _vp, _vp, _ip]
_L.irk_dirk_step.argtypes = [_vp, C.POINTER(_Rhs), C.c_int, _vp, C.c_double, _vp, _vp, C.c_double,
                             C.c_int, _vp, C.c_size_t, C.POINTER(_StepInfo)]

EXPORTED = ["irk_default_options", "irk_workspace_size", "irk_setup", "irk_update_values",
            "irk_factor_ilu", "irk_gmres_solve", "irk_solve_batched", "irk_apply_operator",
            "irk_apply_preconditioner", "irk_export_factors", "irk_last_bad_element",
            "irk_destroy", "irk_status_str", "irk_radau_iia", "irk_profile_enable",
            "irk_profile_read", "irk_quantize_blocks", "irk_batch_workspace_size",
            "irk_batch_create", "irk_batch_admit", "irk_batch_advance", "irk_batch_retire",
            "irk_batch_pending", "irk_batch_destroy", "irk_autotune", "irk_factor_batched",
            "irk_apply_operator_inner", "irk_apply_preconditioner_inner",
            "irk_apply_operator_untransformed", "irk_step_workspace_size", "irk_radau_step",
            "irk_dirk_workspace_size", "irk_dirk_step", "irk_dirk_tableau",
            "irk_solve_batched_noalloc", "irk_level_schedule", "irk_factor_ilu_async"]


def _check(st: int, where: str):
    if st != OK:
        raise IrkError(st, where)


def status_str(st: int) -> str:
    return _L.irk_status_str(st).decode()


def radau_iia(s: int):
    """(A, b, c) of the s-stage Radau IIA method, computed by the library."""
    A = np.zeros((s, s)); b = np.zeros(s); c = np.zeros(s)
    _check(_L.irk_radau_iia(s, A.ctypes.data, b.ctypes.data, c.ctypes.data), "irk_radau_iia")
    return A, b, c


def level_schedule(row_ptr, col_idx):
    """The factorization's and sweeps' level schedule of a BSR pattern, from
    the library: (lvl_fwd, off_fwd, lvl_bwd, off_bwd) as int32 arrays, level
    l of a direction being lvl[off[l]:off[l + 1]].  Raises IrkError for a
    pattern irk_setup would reject."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    T = len(rp) - 1
    lf = np.zeros(T, np.int32); lb = np.zeros(T, np.int32)
    of = np.zeros(T + 1, np.int32); ob = np.zeros(T + 1, np.int32)
    nf = C.c_int(); nb = C.c_int()
    _check(_L.irk_level_schedule(T, len(ci), rp.ctypes.data, ci.ctypes.data, lf.ctypes.data, of.ctypes.data,
                                 C.byref(nf), lb.ctypes.data, ob.ctypes.data, C.byref(nb)),
           "irk_level_schedule")
    return lf, of[:nf.value + 1], lb, ob[:nb.value + 1]


def dirk_tableau(name: str):
    """(A, b, c) of DIRK33 or ESDIRK65 (App. A), from the library."""
    which = {"DIRK33": 0, "ESDIRK65": 1}[name]
    A = np.zeros(64); b = np.zeros(8); c = np.zeros(8)
    st = C.c_int()
    _check(_L.irk_dirk_tableau(which, C.byref(st), A.ctypes.data, b.ctypes.data, c.ctypes.data),
           "irk_dirk_tableau")
    s = st.value
    return A[:s * s].reshape(s, s).copy(), b[:s].copy(), c[:s].copy()


def quantize_blocks(src: torch.Tensor, prec: str):
    """Quantize FP64 blocks [nblk, m, m] (device tensor) with the library's
    factor quantizer.  Returns (values as int16/float32 tensor, exponents or
    None)."""
    src = src.contiguous()
    nblk, m = int(src.shape[0]), int(src.shape[1])
    if prec == "fp32":
        dst = torch.empty(src.shape, dtype=torch.float32, device=src.device)
    else:
        dst = torch.empty(src.shape, dtype=torch.int16, device=src.device)
    ex = torch.zeros(nblk, dtype=torch.int32, device=src.device) if prec == "fp16s" else None
    st = torch.cuda.current_stream(src.device).cuda_stream
    _check(_L.irk_quantize_blocks(src.data_ptr(), nblk, m, PREC[prec], dst.data_ptr(),
                                  ex.data_ptr() if ex is not None else None, _vp(st)),
           "irk_quantize_blocks")
    return dst, ex


@dataclass
class Options:
    pc: str = "coupled"
    shift_rule: int = 0
    alpha: Optional[Sequence[float]] = None
    matvec_prec: str = "fp64"
    factor_prec: str = "fp64"
    restart: int = 30
    max_iters: int = 3000
    max_outer: int = 20
    rtol: float = 1e-10
    inner_rtol: float = 1e-4

    def _c(self):
        o = _Options()
        _L.irk_default_options(C.byref(o))
        o.pc = PC[self.pc]
        o.shift_rule = self.shift_rule
        self._alpha = None
        if self.alpha is not None:
            self._alpha = np.ascontiguousarray(self.alpha, dtype=np.float64)
            o.alpha = self._alpha.ctypes.data
        o.matvec_prec = PREC[self.matvec_prec]
        o.factor_prec = PREC[self.factor_prec]
        o.restart, o.max_iters, o.max_outer = self.restart, self.max_iters, self.max_outer
        o.rtol, o.inner_rtol = self.rtol, self.inner_rtol
        return o


def _info_dict(inf: _Info, status: int) -> dict:
    return dict(status=status, converged=bool(inf.converged), iters=inf.iters,
                outer_iters=inf.outer_iters, restarts=inf.restarts,
                equiv_mults=inf.equiv_mults, rel_res_true=inf.rel_res_true,
                rel_res_est=inf.rel_res_est, bad_element=inf.bad_element,
                ms_factor=inf.ms_factor, ms_solve=inf.ms_solve)


class Solver:
    """One system B W = R on the current CUDA (HIP) device.

    ``system`` needs the attributes s, T, m, nJ, dt, row_ptr, col_idx (host
    int32), J [nJ, nnzb, m, m] and M [T, m, m] (NumPy or torch FP64; moved to
    the device here).  ``A`` is the s x s Butcher matrix (default: Radau IIA
    from the library).  ``workspace_alloc(nbytes)``, if given, supplies the
    device workspace (a uint8 CUDA tensor of at least nbytes bytes, 256-byte
    aligned) in place of a fresh allocation, e.g. a range of a pool that the
    caller manages.
    """

    def __init__(self, system, options: Optional[Options] = None, A=None,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None,
                 s: Optional[int] = None, dt: Optional[float] = None, workspace_alloc=None):
        self.options = options or Options()
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.s = int(system.s if s is None else s)
        self.T, self.m, self.nJ = int(system.T), int(system.m), int(system.nJ)
        self.dt = float(system.dt if dt is None else dt)
        self.N = self.s * self.T * self.m
        self.A = np.ascontiguousarray(radau_iia(self.s)[0] if A is None else A, dtype=np.float64)
        self.row_ptr = np.ascontiguousarray(system.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(system.col_idx, dtype=np.int32)
        J = torch.as_tensor(system.J, dtype=torch.float64)
        M = torch.as_tensor(system.M, dtype=torch.float64)
        with torch.cuda.stream(self.stream):
            self.J = J.to(self.device).contiguous()
            self.M = M.to(self.device).contiguous()
        self._p = _Problem(self.s, self.A.ctypes.data, self.T, self.m, int(self.col_idx.size),
                           self.row_ptr.ctypes.data, self.col_idx.ctypes.data,
                           self.J.data_ptr(), self.nJ, self.M.data_ptr(), self.dt)
        self._o = self.options._c()
        nbytes = C.c_size_t()
        _check(_L.irk_workspace_size(C.byref(self._p), C.byref(self._o), C.byref(nbytes)),
               "irk_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        if workspace_alloc is None:
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        else:
            ws = workspace_alloc(self.workspace_bytes)
            if (not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or ws.device.type != "cuda"
                    or (self.device.index is not None and ws.device.index != self.device.index)
                    or ws.numel() < self.workspace_bytes or ws.data_ptr() % 256):
                raise ValueError("workspace_alloc must return an aligned uint8 tensor of at least "
                                 f"{self.workspace_bytes} bytes on {self.device}")
            self.workspace = ws
        h = _vp()
        _check(_L.irk_setup(C.byref(self._p), C.byref(self._o), self.workspace.data_ptr(),
                            self.workspace_bytes, _vp(self.stream.cuda_stream), C.byref(h)),
               "irk_setup")
        self._h = h
        self.factored = False

    # -- lifecycle --
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L.irk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def update_values(self, J, M, dt: Optional[float] = None):
        with torch.cuda.stream(self.stream):
            self.J = torch.as_tensor(J, dtype=torch.float64).to(self.device).contiguous()
            self.M = torch.as_tensor(M, dtype=torch.float64).to(self.device).contiguous()
        if dt is not None:
            self.dt = float(dt)
        _check(_L.irk_update_values(self._h, self.J.data_ptr(), self.M.data_ptr(), self.dt),
               "irk_update_values")
        self.factored = False

    def factor(self, wait: bool = True):
        """Block ILU(0) factorization (raises IrkError on a singular pivot).
        wait=False: irk_factor_ilu_async (returns at once; a singular pivot
        is raised by the next call that uses the factors)."""
        if not wait:
            _check(_L.irk_factor_ilu_async(self._h), "irk_factor_ilu_async")
            self.factored = True
            return
        st = _L.irk_factor_ilu(self._h)
        if st == ERR_SINGULAR:
            raise IrkError(st, f"irk_factor_ilu (element {_L.irk_last_bad_element(self._h)})")
        _check(st, "irk_factor_ilu")
        self.factored = True

    def _vec(self, v) -> torch.Tensor:
        t = torch.as_tensor(v, dtype=torch.float64)
        if t.device != self.device:
            with torch.cuda.stream(self.stream):
                t = t.to(self.device)
        t = t.contiguous().view(-1)
        if t.numel() != self.N:
            raise ValueError(f"vector of {t.numel()} entries, expected {self.N}")
        return t

    def solve(self, rhs, x0=None, raise_on_error: bool = True):
        """Returns (x, info dict)."""
        b = self._vec(rhs)
        with torch.cuda.stream(self.stream):
            x = torch.zeros(self.N, dtype=torch.float64, device=self.device) if x0 is None \
                else self._vec(x0).clone()
        inf = _Info()
        st = _L.irk_gmres_solve(self._h, b.data_ptr(), x.data_ptr(), C.byref(inf))
        if raise_on_error and st not in (OK, ERR_NOCONV):
            raise IrkError(st, "irk_gmres_solve")
        return x, _info_dict(inf, st)

    def apply_operator(self, x) -> torch.Tensor:
        xv = self._vec(x)
        with torch.cuda.stream(self.stream):
            y = torch.empty_like(xv)
        _check(_L.irk_apply_operator(self._h, xv.data_ptr(), y.data_ptr()), "irk_apply_operator")
        return y

    def apply_preconditioner(self, v) -> torch.Tensor:
        vv = self._vec(v)
        with torch.cuda.stream(self.stream):
            z = torch.empty_like(vv)
        _check(_L.irk_apply_preconditioner(self._h, vv.data_ptr(), z.data_ptr()),
               "irk_apply_preconditioner")
        return z

    def _step_vectors(self, u0, g):
        n = self.T * self.m
        with torch.cuda.stream(self.stream):
            u = torch.as_tensor(u0, dtype=torch.float64).to(self.device).contiguous().view(-1)
            gv = None if g is None else \
                torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous().view(-1)
            u1 = torch.empty(n, dtype=torch.float64, device=self.device)
        if u.numel() != n or (gv is not None and gv.numel() != n):
            raise ValueError(f"vectors of {n} entries expected")
        return u, gv, u1

    def _scratch(self, nbytes: int) -> torch.Tensor:
        if getattr(self, "_step_ws", None) is None or self._step_ws.numel() < nbytes:
            with torch.cuda.stream(self.stream):
                self._step_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._step_ws

    def step(self, u0, t0: float = 0.0, g=None, omega: float = 0.0, eps: float = 0.0, b=None,
             newton_tol: float = 1e-10, max_newton: int = 20, raise_on_error: bool = True):
        """One implicit Runge-Kutta step of M u' = J u + cos(omega t) g - eps u^3
        from (t0, u0) with this solver's dt, by Newton's method on the
        transformed stage equations (irk_radau_step).  Returns (u1, info)."""
        u, gv, u1 = self._step_vectors(u0, g)
        nb = C.c_size_t()
        _check(_L.irk_step_workspace_size(self._h, C.byref(nb)), "irk_step_workspace_size")
        ws = self._scratch(int(nb.value))
        rhs = _Rhs(gv.data_ptr() if gv is not None else None, float(omega), float(eps))
        bw = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        inf = _StepInfo()
        st = _L.irk_radau_step(self._h, C.byref(rhs), bw.ctypes.data if bw is not None else None,
                               float(t0), u.data_ptr(), u1.data_ptr(), float(newton_tol),
                               int(max_newton), ws.data_ptr(), ws.numel(), C.byref(inf))
        if raise_on_error and st != OK:
            raise IrkError(st, "irk_radau_step")
        return u1, dict(status=st, **{f: getattr(inf, f) for f, _ in _StepInfo._fields_})

    def dirk_step(self, A, u0, t0: float = 0.0, g=None, omega: float = 0.0, eps: float = 0.0,
                  newton_tol: float = 1e-10, max_newton: int = 20, raise_on_error: bool = True):
        """One step of the stiffly accurate DIRK tableau A (irk_dirk_step);
        this solver must be a one-stage system whose tableau entry is A's
        implicit diagonal.  Returns (u1, info)."""
        Ad = np.ascontiguousarray(A, dtype=np.float64)
        stages = int(Ad.shape[0])
        u, gv, u1 = self._step_vectors(u0, g)
        nb = C.c_size_t()
        _check(_L.irk_dirk_workspace_size(self._h, stages, C.byref(nb)), "irk_dirk_workspace_size")
        ws = self._scratch(int(nb.value))
        rhs = _Rhs(gv.data_ptr() if gv is not None else None, float(omega), float(eps))
        inf = _StepInfo()
        st = _L.irk_dirk_step(self._h, C.byref(rhs), stages, Ad.ctypes.data, float(t0), u.data_ptr(),
                              u1.data_ptr(), float(newton_tol), int(max_newton), ws.data_ptr(),
                              ws.numel(), C.byref(inf))
        if raise_on_error and st != OK:
            raise IrkError(st, "irk_dirk_step")
        return u1, dict(status=st, **{f: getattr(inf, f) for f, _ in _StepInfo._fields_})

    def apply_operator_untransformed(self, x, form: str = "fused") -> torch.Tensor:
        """y = (I (x) M - dt [a_kl J_k]) x, the untransformed operator
        (form "blocks": one pass over J_k per block of the s x s block
        matrix; "fused": one pass per element row)."""
        xv = self._vec(x)
        with torch.cuda.stream(self.stream):
            y = torch.empty_like(xv)
        f = {"blocks": 0, "fused": 1}[form]
        _check(_L.irk_apply_operator_untransformed(self._h, f, xv.data_ptr(), y.data_ptr()),
               "irk_apply_operator_untransformed")
        return y

    def apply_operator_inner(self, x) -> torch.Tensor:
        """y = B x with the inner-iteration operator (FP32 for a mixed-
        precision solver, FP64 otherwise)."""
        xv = self._vec(x)
        with torch.cuda.stream(self.stream):
            y = torch.empty_like(xv)
        _check(_L.irk_apply_operator_inner(self._h, xv.data_ptr(), y.data_ptr()),
               "irk_apply_operator_inner")
        return y

    def apply_preconditioner_inner(self, v) -> torch.Tensor:
        """z = P^{-1} v with the inner-iteration sweeps (reduced-precision
        factors and FP32 sweeps for a mixed-precision solver)."""
        vv = self._vec(v)
        with torch.cuda.stream(self.stream):
            z = torch.empty_like(vv)
        _check(_L.irk_apply_preconditioner_inner(self._h, vv.data_ptr(), z.data_ptr()),
               "irk_apply_preconditioner_inner")
        return z

    def autotune(self, retime: bool = False) -> dict:
        """Pick the matvec and sweep launch shapes by timing them on this
        system (irk_autotune); needs a factored solver.  Later solvers of the
        same problem class reuse the choice without timing."""
        t = _Tune()
        _check(_L.irk_autotune(self._h, 1 if retime else 0, C.byref(t)), "irk_autotune")
        return {f: getattr(t, f) for f, _ in _Tune._fields_}

    def profile(self, on: bool = True):
        """Turn HIP-event kernel timing on or off (clears recorded intervals)."""
        _check(_L.irk_profile_enable(self._h, 1 if on else 0), "irk_profile_enable")

    def profile_read(self) -> dict:
        """Totals since the last read: counts and milliseconds per kernel class."""
        p = _Prof()
        _check(_L.irk_profile_read(self._h, C.byref(p)), "irk_profile_read")
        return {f: getattr(p, f) for f, _ in _Prof._fields_}

    def export_factors(self, cross: bool = False):
        with torch.cuda.stream(self.stream):
            P = torch.zeros((self.s, self.T, self.m, self.m), dtype=torch.float64, device=self.device)
            Cx = torch.zeros((self.s, self.s, self.T, self.m, self.m), dtype=torch.float64,
                             device=self.device) if cross else None
        _check(_L.irk_export_factors(self._h, P.data_ptr(), Cx.data_ptr() if cross else None),
               "irk_export_factors")
        return (P, Cx) if cross else P


class Batch:
    """Many independent systems iterated together (one launch per phase covers
    every member).  Members are factored Solvers sharing the preconditioner
    kind and precision scheme."""

    def __init__(self, capacity: int, max_elements: int, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(self.device)
        nbytes = C.c_size_t()
        _check(_L.irk_batch_workspace_size(capacity, max_elements, C.byref(nbytes)),
               "irk_batch_workspace_size")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_L.irk_batch_create(capacity, max_elements, self.workspace.data_ptr(),
                                   int(nbytes.value), _vp(self.stream.cuda_stream), C.byref(h)),
               "irk_batch_create")
        self._b = h
        self._keep = {}     # tag -> (solver, rhs, x) kept alive while in the batch
        self.capacity = capacity

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            _L.irk_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, solver: "Solver", rhs, tag: int, x0=None) -> int:
        """Queue a factored solver; returns the status (OK, or ERR_NOMEM when full).
        The right-hand side and the initial guess are staged on the batch's
        stream, so admission never waits for other work on the solver's."""
        with torch.cuda.stream(self.stream):
            b = torch.as_tensor(rhs, dtype=torch.float64).to(solver.device).contiguous().view(-1)
            if b.numel() != solver.N:
                raise ValueError(f"vector of {b.numel()} entries, expected {solver.N}")
            x = torch.zeros(solver.N, dtype=torch.float64, device=solver.device) if x0 is None \
                else torch.as_tensor(x0, dtype=torch.float64).to(solver.device).contiguous().view(-1).clone()
        st = _L.irk_batch_admit(self._b, solver.handle, b.data_ptr(), x.data_ptr(), int(tag))
        if st == OK:
            self._keep[int(tag)] = (solver, b, x)
        return st

    def advance(self, cycles: int = 1):
        _check(_L.irk_batch_advance(self._b, int(cycles)), "irk_batch_advance")

    @property
    def pending(self) -> int:
        return int(_L.irk_batch_pending(self._b))

    def retire(self):
        """List of (tag, x, info dict) of the members that finished."""
        out = []
        while True:
            n = 64
            tags = (C.c_longlong * n)()
            sts = (C.c_int * n)()
            infos = (_Info * n)()
            cnt = C.c_int()
            _check(_L.irk_batch_retire(self._b, tags, sts, infos, n, C.byref(cnt)), "irk_batch_retire")
            for q in range(cnt.value):
                solver, b, x = self._keep.pop(int(tags[q]))
                out.append((int(tags[q]), x, _info_dict(infos[q], int(sts[q]))))
            if cnt.value < n:
                break
        return out


def factor_batched(batch: Batch, solvers: Sequence[Solver]) -> List[int]:
    """Factor several systems together through irk_factor_batched (level l
    of every system in the same launches; the batch must have no members).
    Returns the per-system statuses; raises IrkError for the first system
    with a singular pivot (the others are factored)."""
    n = len(solvers)
    if n == 0:
        return []
    H = (_vp * n)(*[s.handle for s in solvers])
    sts = (C.c_int * n)()
    st = _L.irk_factor_batched(batch._b, H, n, sts)
    for s, q in zip(solvers, sts):
        s.factored = (q == OK)
    if st == ERR_SINGULAR:
        q = next(q for q in range(n) if sts[q] == ERR_SINGULAR)
        raise IrkError(st, f"irk_factor_batched (system {q}, element "
                           f"{_L.irk_last_bad_element(solvers[q].handle)})")
    _check(st, "irk_factor_batched")
    return list(sts)


def solve_batched(batch: Batch, solvers: Sequence[Solver], rhs: Sequence, x0: Optional[Sequence] = None):
    """Solve several systems together through irk_solve_batched.  Returns
    (list of x, list of info dicts, status)."""
    n = len(solvers)
    bs, xs = [], []
    # staged on the batch's stream, which the solve runs on
    with torch.cuda.stream(batch.stream):
        for q, s in enumerate(solvers):
            b = torch.as_tensor(rhs[q], dtype=torch.float64).to(s.device).contiguous().view(-1)
            if b.numel() != s.N:
                raise ValueError(f"vector of {b.numel()} entries, expected {s.N}")
            bs.append(b)
        if x0 is None:
            # one zero-filled allocation, one view per member
            flat = torch.zeros(sum(s.N for s in solvers), dtype=torch.float64, device=batch.device)
            xs = list(torch.split(flat, [s.N for s in solvers]))
        else:
            xs = [torch.as_tensor(x0[q], dtype=torch.float64).to(s.device).contiguous().view(-1).clone()
                  for q, s in enumerate(solvers)]
    H = (_vp * n)(*[s.handle for s in solvers])
    B = (_vp * n)(*[b.data_ptr() for b in bs])
    X = (_vp * n)(*[x.data_ptr() for x in xs])
    infos = (_Info * n)()
    st = _L.irk_solve_batched(batch._b, H, B, X, n, infos)
    return xs, [_info_dict(infos[q], st) for q in range(n)], st


def solve_batched_noalloc(solvers: Sequence[Solver], rhs: Sequence, x: Sequence[torch.Tensor],
                          stream: Optional[torch.cuda.Stream] = None):
    """irk_solve_batched_noalloc: the batched solve with the library's own
    static device scratch (no batch object, no device allocation in the
    call).  rhs and x are device FP64 vectors of each solver's size; x holds
    the initial guesses and receives the solutions.  Returns (info dicts,
    status)."""
    n = len(solvers)
    st_ = stream or torch.cuda.current_stream()
    H = (_vp * n)(*[s.handle for s in solvers])
    B = (_vp * n)(*[int(r.data_ptr()) for r in rhs])
    X = (_vp * n)(*[int(v.data_ptr()) for v in x])
    infos = (_Info * n)()
    st = _L.irk_solve_batched_noalloc(H, B, X, n, _vp(st_.cuda_stream), infos)
    return [_info_dict(infos[q], st) for q in range(n)], st
