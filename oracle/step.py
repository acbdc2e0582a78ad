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

import math
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
    out = dict(newton_iters=len(norms), gmres_iters=gm, equiv_mults=gm * s, converged=converged,
               update_norms=norms)
    return u1, out


def integrate(sys, A, b, u0, t0, t1, nsteps, **kw):
    """nsteps equal steps of irk_step from t0 to t1; returns u(t1)."""
    dt = (t1 - t0) / nsteps
    u = np.array(u0, dtype=np.float64)
    for q in range(nsteps):
        u, _ = irk_step(sys, A, b, t0 + q * dt, u, dt, **kw)
    return u


# ----------------------------------------------------------------------------
# the diagonally implicit comparison methods (Sec. 3, tableaux of App. A)
# ----------------------------------------------------------------------------

def dirk33():
    """DIRK33 (App. A): three-stage, third-order, L-stable, stiffly accurate."""
    t = math.atan(math.sqrt(2.0) / 4.0) / 3.0
    al = 1.0 + math.sqrt(6.0) / 2.0 * math.sin(t) - math.sqrt(2.0) / 2.0 * math.cos(t)
    tau2 = (1.0 + al) / 2.0
    b1 = -(6.0 * al * al - 16.0 * al + 1.0) / 4.0
    b2 = (6.0 * al * al - 20.0 * al + 5.0) / 4.0
    A = np.array([[al, 0.0, 0.0], [tau2 - al, al, 0.0], [b1, b2, al]])
    return A, A[2].copy(), np.array([al, tau2, 1.0])


# ESDIRK65 as printed in App. A (16 significant digits): explicit first
# stage, five implicit stages with the common diagonal 0.2780538411364465.
_ESDIRK65_A = [
    [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
    [0.2780538411364465, 0.2780538411364465, 0.0, 0.0, 0.0, 0.0],
    [0.3137405401502951, 0.4363327154020044, 0.2780538411364465, 0.0, 0.0, 0.0],
    [0.2741986534107860, -0.0164268277321164, 0.0048197082596452, 0.2780538411364465, 0.0, 0.0],
    [-0.2441776975175844, -3.3203529439447852, 0.0477747285706825, 3.2974431145814931,
     0.2780538411364465, 0.0],
    [-0.2786732780227907, 1.8929947094010862, -0.1280948204262490, -1.3574693381380240,
     0.5931888860495311, 0.2780538411364465],
]
_ESDIRK65_C = [0.0, 0.556107682272893, 1.028127096688746, 0.540645375074761, 0.058741042826253, 1.0]


def esdirk65():
    """ESDIRK65 (App. A): six stages (the first explicit), fifth order."""
    A = np.array(_ESDIRK65_A)
    return A, A[5].copy(), np.array(_ESDIRK65_C)


def dirk_step(sys, A: np.ndarray, t0: float, u0: np.ndarray, dt: float,
              g: Optional[np.ndarray] = None, omega: float = 0.0, eps: float = 0.0,
              newton_tol: float = 1e-12, max_newton: int = 20, pc: str = "coupled",
              rtol: float = 1e-13):
    """One step of a stiffly accurate DIRK method (lower-triangular A, b = last
    row, an explicit stage allowed only first with a zero row).

    Stage i solves  M (U_i - u0) = dt sum_{j<i} a_ij F_j + dt a_ii f(t_i, U_i),
    F_j = f(t_j, U_j), by Newton in W = (U_i - u0) / dt: the residual
    f(t_i, u0 + dt W) + (1/a_ii) sum_{j<i} a_ij F_j - (1/a_ii) M W and the
    matrix (1/a_ii) M - dt J_f(U_i), an n x n system of the form of Eq.
    big-irk with s = 1 and A = [[a_ii]] (so the same block ILU(0) and GMRES
    apply).  Stiff accuracy gives u1 = U_s.  Returns u1 and a dict."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    c = A.sum(axis=1)
    n = sys.T * sys.m
    Jbase = np.asarray(sys.J[0])
    dpos = np.array([int(np.flatnonzero(sys.col_idx[sys.row_ptr[i]:sys.row_ptr[i + 1]] == i)[0])
                     + int(sys.row_ptr[i]) for i in range(sys.T)])
    F = np.zeros((s, n))
    U = u0.copy()
    newton = gm = 0
    converged = True
    for i in range(s):
        aii = A[i, i]
        ti = t0 + c[i] * dt
        if aii == 0.0:
            if i != 0 or np.any(A[0] != 0.0):
                raise ValueError("only a first stage with a zero row may be explicit")
            U = u0.copy()
            F[i] = rhs_f(sys, ti, U, g, omega, eps)
            continue
        hist = (A[i, :i] @ F[:i]) / aii if i > 0 else np.zeros(n)
        W = np.zeros(n)
        ok = False
        for it in range(max_newton):
            U = u0 + dt * W
            R = rhs_f(sys, ti, U, g, omega, eps) + hist - mass_product(sys, W) / aii
            J1 = Jbase.copy()
            if eps != 0.0:
                for e in range(sys.T):
                    blk = J1[dpos[e]]
                    blk[np.diag_indices(sys.m)] -= 3.0 * eps * U[e * sys.m:(e + 1) * sys.m] ** 2
            P = Problem(_StageSystem(sys, np.ascontiguousarray(J1[None]), dt))
            delta, info = solve(P, np.array([[aii]]), R, pc=pc, rtol=rtol, maxit=3000, orth="cgs2")
            gm += info["iters"]
            newton += 1
            W += delta
            if float(np.abs(delta).max()) <= newton_tol:
                ok = True
                break
        converged = converged and ok
        U = u0 + dt * W
        F[i] = rhs_f(sys, ti, U, g, omega, eps)
    return U, dict(newton_iters=newton, gmres_iters=gm, equiv_mults=gm, converged=converged)
