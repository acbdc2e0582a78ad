"""Pins of the DIRK comparison methods (tableaux of App. A, Table 1) and of
the oracle's DIRK step.

* The transcribed tableaux satisfy the Runge-Kutta order conditions (the
  rooted-tree conditions up to order 3 for DIRK33 and 5 for ESDIRK65, to
  rounding), are stiffly accurate with c = row sums, ESDIRK65 has stage
  order 2 (Sec. 3), and both reproduce the leading error coefficients
  printed in Table 1 (tests/golden/table1_dirk_error_constants.txt): the
  coefficient of z^{p+1} in e^z - R(z), the same quantity that gives the
  Radau IIA entries of that table.
* One linear step of the oracle's DIRK equals the dense stability-matrix
  formula u1 = u0 + (b^T (x) Z) (I - A (x) Z)^{-1} (1 (x) u0), Z = dt M^{-1} J.
* Observed order 3 and 5 against the matrix-exponential solution of the
  forced linear problem (rate estimator of Sec. 5.1.2).
"""
import math
import os

import numpy as np
import pytest

import dgsynth
import oracle
from oracle import step as ostep
from tests import dense

scipy_linalg = pytest.importorskip("scipy.linalg")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_dirk_error_constants.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, p, v = line.split()
            out[name] = (int(p), float(v))
    return out


def _conditions(A, b, order):
    """(value, exact) of every rooted-tree order condition up to `order`."""
    c = A.sum(axis=1)
    one = np.ones(len(b))
    Ac, Ac2, AAc = A @ c, A @ c ** 2, A @ (A @ c)
    out = [(b @ one, 1.0)]
    if order >= 2:
        out += [(b @ c, 1 / 2)]
    if order >= 3:
        out += [(b @ c ** 2, 1 / 3), (b @ Ac, 1 / 6)]
    if order >= 4:
        out += [(b @ c ** 3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ Ac2, 1 / 12), (b @ AAc, 1 / 24)]
    if order >= 5:
        out += [(b @ c ** 4, 1 / 5), (b @ (c ** 2 * Ac), 1 / 10), (b @ (c * Ac2), 1 / 15),
                (b @ (c * AAc), 1 / 30), (b @ Ac ** 2, 1 / 20), (b @ (A @ c ** 3), 1 / 20),
                (b @ (A @ (c * Ac)), 1 / 40), (b @ (A @ Ac2), 1 / 60), (b @ (A @ AAc), 1 / 120)]
    return out


def _err_coeff(A, b, p):
    """Coefficient of z^{p+1} in e^z - R(z), R(z) = 1 + sum_q z^{q+1} b^T A^q 1."""
    return 1.0 / math.factorial(p + 1) - b @ np.linalg.matrix_power(A, p) @ np.ones(len(b))


@pytest.mark.parametrize("name", ["DIRK33", "ESDIRK65"])
def test_tableau_order_conditions_and_table1(name):
    A, b, c = ostep.dirk33() if name == "DIRK33" else ostep.esdirk65()
    p, printed = _golden()[name]
    assert np.allclose(np.triu(A, 1), 0.0)                       # diagonally implicit
    assert np.array_equal(b, A[-1]) and c[-1] == 1.0               # stiffly accurate
    assert np.abs(A.sum(axis=1) - c).max() < 1e-14                 # c = row sums
    worst = max(abs(v - e) for v, e in _conditions(A, b, p))
    assert worst < 1e-14, worst
    # not of order p + 1: some condition of the next order fails
    if p + 1 <= 5:
        assert max(abs(v - e) for v, e in _conditions(A, b, p + 1)) > 1e-6
    assert abs(abs(_err_coeff(A, b, p)) - printed) <= 0.005 * printed


def test_dirk33_alpha_is_the_l_stable_root():
    """alpha solves 6 a^3 - 18 a^2 + 9 a - 1 = 0 (the condition that makes the
    three-stage SDIRK of order 3 L-stable) and lies in (1/3, 1/2)."""
    A, _, _ = ostep.dirk33()
    a = A[0, 0]
    assert abs(6 * a ** 3 - 18 * a ** 2 + 9 * a - 1) < 1e-14
    assert 1 / 3 < a < 1 / 2


def test_esdirk65_stage_order_two_and_l_stability():
    A, b, c = ostep.esdirk65()
    assert np.abs((A @ c)[1:] - c[1:] ** 2 / 2).max() < 1e-14      # stage order 2
    # L-stability: R(z) -> 0 as z -> -infinity (like 1/z: |z R(z)| stays bounded)
    for z in (-1e4, -1e6, -1e8):
        R = 1 + z * b @ np.linalg.solve(np.eye(6) - z * A, np.ones(6))
        assert abs(z * R) < 10.0


def _ode(seed, m=3, N=4):
    sys = dgsynth.make_system(seed, dgsynth.grid2d(N), m, 1, 0.1)
    rng = np.random.default_rng(seed + 1)
    n = sys.T * sys.m
    return sys, rng.standard_normal(n), rng.standard_normal(n)


@pytest.mark.parametrize("name", ["DIRK33", "ESDIRK65"])
def test_linear_dirk_step_is_stability_matrix(name):
    A, b, _ = ostep.dirk33() if name == "DIRK33" else ostep.esdirk65()
    sys, u0, _ = _ode(900)
    dt = 0.3
    u1, info = ostep.dirk_step(sys, A, 0.0, u0, dt, newton_tol=1e-13, rtol=1e-14)
    Z = dt * np.linalg.solve(dense.dense_M(sys), dense.dense_J(sys))
    s, n = A.shape[0], Z.shape[0]
    K = np.linalg.solve(np.eye(s * n) - np.kron(A, Z), np.kron(np.ones(s), u0))
    ref = u0 + np.kron(b[None, :], Z) @ K
    assert np.abs(u1 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert info["converged"]


def _exact_forced(sys, u0, g, omega, t1):
    Md, Jd = dense.dense_M(sys), dense.dense_J(sys)
    n = Md.shape[0]
    Aug = np.zeros((n + 2, n + 2))
    Aug[:n, :n] = np.linalg.solve(Md, Jd)
    Aug[:n, n] = np.linalg.solve(Md, g)
    Aug[n, n + 1] = -omega
    Aug[n + 1, n] = omega
    return (scipy_linalg.expm(t1 * Aug) @ np.concatenate([u0, [1.0, 0.0]]))[:n]


@pytest.mark.parametrize("name,order", [("DIRK33", 3), ("ESDIRK65", 5)])
def test_dirk_observed_order(name, order):
    A, _, _ = ostep.dirk33() if name == "DIRK33" else ostep.esdirk65()
    sys, u0, g = _ode(910)
    omega, t1 = 2.0, 0.8
    ref = _exact_forced(sys, u0, g, omega, t1)
    errs, dts = [], []
    for ns in (4, 8, 16):
        dt = t1 / ns
        u = u0.copy()
        for q in range(ns):
            u, _ = ostep.dirk_step(sys, A, q * dt, u, dt, g=g, omega=omega,
                                   newton_tol=1e-14, rtol=1e-14)
        errs.append(np.abs(u - ref).max())
        dts.append(dt)
    rates = [math.log(errs[q + 1] / errs[q]) / math.log(dts[q + 1] / dts[q]) for q in range(2)]
    assert all(abs(r - order) < 0.4 for r in rates), (errs, rates)
