"""One implicit Runge-Kutta time step by Newton's method (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy plus the
oracle's own BSR product and GMRES solve; it shares nothing with the HIP
library.

The ODE is the semi-discrete form of Sec. 3, M u' = f(t, u), with the
synthetic right-hand side

    f(t, u) = J u + cos(omega t) g - eps u^3        (u^3 component-wise)

(J the block Jacobian of the linear part, M block diagonal).  Its Jacobian
is J_f(t, u) = J - 3 eps diag(u^2): only the diagonal entries of the
diagonal blocks depend on u.

Sec. 4.1 writes the s stage equations in the variables W = (A (x) I) K as
Eq. modified-IRK,

    G(W) = (A^{-1} (x) M) W - F(t0 + dt c, U0 + dt W) = 0,

solved by Newton's method with the matrix of Eq. big-irk,
A^{-1} (x) M - dt diag(J_1, ..., J_s), J_k = J_f(t0 + c_k dt, u0 + dt w_k),
and the new solution is u1 = u0 + dt (b^T A^{-1} (x) I) W, which is
u0 + dt w_s for the stiffly accurate Radau IIA methods.  Newton stops when
the infinity norm of the update is at most newton_tol (the stopping test
Sec. 5.1.1 states for its Newton iterations).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import BlockMatrix, Problem, inverse, solve


class _StageSystem:
    """The attributes oracle.Problem reads, with one Jacobian per stage."""

    def __init__(self, base, J_stages, dt):
        self.s = J_stages.shape[0]
        self.T, self.m = base.T, base.m
        self.nJ = self.s
        self.dt = dt
        self.row_ptr, self.col_idx, self.M = base.row_ptr, base.col_idx, base.M
        self.J = J_stages


def rhs_f(sys, t: float, u: np.ndarray, g: Optional[np.ndarray], omega: float, eps: float):
    """f(t, u) = J u + cos(omega t) g - eps u^3 with J = sys.J[0]."""
    Jb = BlockMatrix(sys.T, sys.m, sys.row_ptr, sys.col_idx, sys.J[0])
    out = Jb.matvec(u)
    if g is not None:
        out = out + np.cos(omega * t) * g
    if eps != 0.0:
        out = out - eps * u ** 3
    return out


def mass_product(sys, x: np.ndarray) -> np.ndarray:
    """M x for one vector [T*m] (block diagonal)."""
    T, m = sys.T, sys.m
    return np.einsum("tij,tj->ti", sys.M, x.reshape(T, m)).reshape(-1)


def irk_step(sys, A: np.ndarray, b: Optional[np.ndarray], t0: float, u0: np.ndarray, dt: float,
             g: Optional[np.ndarray] = None, omega: float = 0.0, eps: float = 0.0,
             newton_tol: float = 1e-12, max_newton: int = 20, pc: str = "coupled",
             rtol: float = 1e-13, history: bool = False):
    """One step of the s-stage method (A, b) from (t0, u0).  Returns u1 and a
    dict (newton iterations, GMRES iterations, update norms)."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    n = sys.T * sys.m
    c = A.sum(axis=1)                      # c_i = sum_j a_ij (condition C(1))
    Ainv = inverse(A)
    d = np.zeros(s)
    d[-1] = 1.0
    if b is not None:
        d = np.asarray(b, dtype=np.float64) @ Ainv
    Jbase = np.asarray(sys.J[0])
    dpos = np.array([int(np.flatnonzero(sys.col_idx[sys.row_ptr[i]:sys.row_ptr[i + 1]] == i)[0])
                     + int(sys.row_ptr[i]) for i in range(sys.T)])
    W = np.zeros((s, n))
    norms = []
    gm = 0
    converged = False
    for it in range(max_newton):
        U = u0[None, :] + dt * W
        # Newton residual R = -G(W) of Eq. modified-IRK
        R = np.zeros((s, n))
        MW = np.stack([mass_product(sys, W[l]) for l in range(s)])
        for k in range(s):
            R[k] = rhs_f(sys, t0 + c[k] * dt, U[k], g, omega, eps) - Ainv[k] @ MW
        # stage Jacobians J_k = J - 3 eps diag(U_k^2)
        Js = np.repeat(Jbase[None], s, axis=0)
        if eps != 0.0:
            for k in range(s):
                for i in range(sys.T):
                    blk = Js[k, dpos[i]]
                    blk[np.diag_indices(sys.m)] -= 3.0 * eps * U[k, i * sys.m:(i + 1) * sys.m] ** 2
        P = Problem(_StageSystem(sys, np.ascontiguousarray(Js), dt))
        delta, info = solve(P, A, R.reshape(-1), pc=pc, rtol=rtol, maxit=3000, orth="cgs2")
        gm += info["iters"]
        W += delta.reshape(s, n)
        nrm = float(np.abs(delta).max())
        norms.append(nrm)
        if nrm <= newton_tol:
            converged = True
            break
    u1 = u0 + dt * (d @ W)
    out = dict(newton_iters=len(norms), gmres_iters=gm, converged=converged, update_norms=norms)
    return u1, out


def integrate(sys, A, b, u0, t0, t1, nsteps, **kw):
    """nsteps equal steps of irk_step from t0 to t1; returns u(t1)."""
    dt = (t1 - t0) / nsteps
    u = np.array(u0, dtype=np.float64)
    for q in range(nsteps):
        u, _ = irk_step(sys, A, b, t0 + q * dt, u, dt, **kw)
    return u
