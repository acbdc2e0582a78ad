"""Pins of the oracle's Newton time step (Sec. 4.1, Eq. modified-IRK,
u1 = u0 + dt w_s) against what the mathematics fixes:

* linear, unforced M u' = J u: one step is the stability function of Sec. 3
  applied to u0, u1 = Q(Z)^{-1} P(Z) u0 with Z = dt M^{-1} J and (P, Q) the
  (s-1, s) Pade pair of e^z;
* linear with forcing cos(omega t) g: the exact solution comes from the
  matrix exponential of the system augmented by (cos, sin) of omega t, and
  the observed order of accuracy (the rate estimator of Sec. 5.1.2) is the
  2s - 1 of Table 1;
* the nonlinear f with -eps u^3: against a library integrator (SciPy's
  DOP853 at rtol 1e-13), same order 2s - 1; Newton needs more than one
  iteration and its updates shrink quadratically.
"""
import math

import numpy as np
import pytest

import dgsynth
import oracle
from oracle import step as ostep
from tests import dense

scipy_linalg = pytest.importorskip("scipy.linalg")
scipy_integrate = pytest.importorskip("scipy.integrate")


def _pade(s):
    k, j = s - 1, s
    P = [math.factorial(k + j - i) * math.factorial(k)
         / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) for i in range(k + 1)]
    Q = [math.factorial(k + j - i) * math.factorial(j)
         / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-1) ** i
         for i in range(j + 1)]
    return P, Q


def _polym(coef, Z):
    out = np.zeros_like(Z)
    Zp = np.eye(Z.shape[0])
    for c in coef:
        out += c * Zp
        Zp = Zp @ Z
    return out


def _ode(seed, s, m=3, N=4):
    sys = dgsynth.make_system(seed, dgsynth.grid2d(N), m, s, 0.1)
    rng = np.random.default_rng(seed + 1)
    n = sys.T * sys.m
    return sys, rng.standard_normal(n), rng.standard_normal(n)


@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_linear_step_is_pade(s):
    sys, u0, _ = _ode(500 + s, s)
    A, b, _ = oracle.radau_iia(s)
    dt = 0.3
    u1, info = ostep.irk_step(sys, A, None, 0.0, u0, dt, newton_tol=1e-13, rtol=1e-14)
    Md, Jd = dense.dense_M(sys), dense.dense_J(sys)
    Z = dt * np.linalg.solve(Md, Jd)
    P, Q = _pade(s)
    ref = np.linalg.solve(_polym(Q, Z), _polym(P, Z) @ u0)
    assert np.abs(u1 - ref).max() <= 1e-12 * np.abs(ref).max()
    # a linear problem: the first Newton update solves it, the second is at
    # the level of the linear-solve tolerance
    assert info["newton_iters"] <= 2
    # b^T A^{-1} = e_s: passing b changes nothing
    u1b, _ = ostep.irk_step(sys, A, b, 0.0, u0, dt, newton_tol=1e-13, rtol=1e-14)
    assert np.abs(u1b - u1).max() <= 1e-12 * np.abs(ref).max()


def _exact_forced(sys, u0, g, omega, t0, t1):
    Md, Jd = dense.dense_M(sys), dense.dense_J(sys)
    n = Md.shape[0]
    Aug = np.zeros((n + 2, n + 2))
    Aug[:n, :n] = np.linalg.solve(Md, Jd)
    Aug[:n, n] = np.linalg.solve(Md, g)
    Aug[n, n + 1] = -omega
    Aug[n + 1, n] = omega
    y0 = np.concatenate([u0, [math.cos(omega * t0), math.sin(omega * t0)]])
    return (scipy_linalg.expm((t1 - t0) * Aug) @ y0)[:n]


def _rates(errs, dts):
    """r_i = log(e_{i+1} / e_i) / log(dt_{i+1} / dt_i) (Sec. 5.1.2)."""
    return [math.log(errs[q + 1] / errs[q]) / math.log(dts[q + 1] / dts[q])
            for q in range(len(errs) - 1)]


@pytest.mark.parametrize("s", [2, 3])
def test_forced_linear_order(s):
    """Observed order 2s - 1 (3 for RADAU23, 5 for RADAU35, Table 1) against
    the exact solution."""
    sys, u0, g = _ode(600 + s, s)
    A, _, _ = oracle.radau_iia(s)
    omega, t1 = 2.0, 0.8
    ref = _exact_forced(sys, u0, g, omega, 0.0, t1)
    steps = [4, 8, 16]
    errs = []
    for ns in steps:
        u = ostep.integrate(sys, A, None, u0, 0.0, t1, ns, g=g, omega=omega,
                            newton_tol=1e-14, rtol=1e-14)
        errs.append(np.abs(u - ref).max())
    r = _rates(errs, [t1 / q for q in steps])
    assert all(abs(x - (2 * s - 1)) < 0.35 for x in r), (errs, r)


def _scipy_reference(sys, u0, g, omega, eps, t1):
    Md = dense.dense_M(sys)
    Jd = dense.dense_J(sys)

    def rhs(t, u):
        return np.linalg.solve(Md, Jd @ u + math.cos(omega * t) * g - eps * u ** 3)
    sol = scipy_integrate.solve_ivp(rhs, (0.0, t1), u0, method="DOP853", rtol=1e-13, atol=1e-15)
    assert sol.success
    return sol.y[:, -1]


@pytest.mark.parametrize("s", [2, 3])
def test_nonlinear_order_and_newton(s):
    sys, u0, g = _ode(700 + s, s)
    A, _, _ = oracle.radau_iia(s)
    omega, eps, t1 = 2.0, 0.3, 0.8
    ref = _scipy_reference(sys, u0, g, omega, eps, t1)
    steps = [4, 8, 16]
    errs = []
    for ns in steps:
        u = ostep.integrate(sys, A, None, u0, 0.0, t1, ns, g=g, omega=omega, eps=eps,
                            newton_tol=1e-14, rtol=1e-14)
        errs.append(np.abs(u - ref).max())
    r = _rates(errs, [t1 / q for q in steps])
    assert all(abs(x - (2 * s - 1)) < 0.35 for x in r), (errs, r)
    # Newton on the nonlinear stage equations: several iterations, each
    # update at most a constant times the square of the previous one
    _, info = ostep.irk_step(sys, A, None, 0.0, u0, 0.2, g=g, omega=omega, eps=eps,
                             newton_tol=1e-13, rtol=1e-14)
    nr = info["update_norms"]
    assert info["converged"] and info["newton_iters"] >= 3
    assert all(nr[q + 1] < nr[q] for q in range(len(nr) - 1))
    # quadratic convergence: |d_{k+1}| <= K |d_k|^2 with a moderate K
    assert nr[2] <= 1e3 * nr[1] ** 2


def test_wrong_stage_time_is_detected():
    """The stage times c_k = sum_j a_kj enter through the forcing: evaluating
    the forcing at t0 instead makes the error first order, so the order test
    above would catch a dropped c."""
    s = 2
    sys, u0, g = _ode(611, s)
    A, _, _ = oracle.radau_iia(s)
    omega, t1 = 2.0, 0.8
    ref = _exact_forced(sys, u0, g, omega, 0.0, t1)
    # forcing frozen at the step start: shift the tableau's stage times to 0
    # by hand through a constant-in-time forcing per step
    errs = []
    for ns in (4, 8):
        dt = t1 / ns
        u = u0.copy()
        for q in range(ns):
            gq = math.cos(omega * q * dt) * g
            u, _ = ostep.irk_step(sys, A, None, q * dt, u, dt, g=gq, omega=0.0,
                                  newton_tol=1e-14, rtol=1e-14)
        errs.append(np.abs(u - ref).max())
    rate = math.log(errs[1] / errs[0]) / math.log(0.5)
    assert rate < 1.5
