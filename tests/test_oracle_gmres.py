"""Pins of the oracle's full solve: dense LU, the linear-ODE one-step
identity (the stability function of Sec. 3 reached through Eq. big-irk and
u1 = u0 + dt w_s of Sec. 4.1), transformed vs untransformed solutions, and
GMRES properties that hold for any correct implementation."""
import math

import numpy as np
import pytest

import dgsynth
import oracle
from tests import dense


def _pade_pq(s):
    k, j = s - 1, s
    P = [math.factorial(k + j - i) * math.factorial(k)
         / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) for i in range(k + 1)]
    Q = [math.factorial(k + j - i) * math.factorial(j)
         / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-1) ** i
         for i in range(j + 1)]
    return P, Q


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled", "none"])
def test_cfg0_solve_vs_dense_lu(pc):
    sys = dgsynth.config_system("cfg0")
    A, _, _ = oracle.radau_iia(sys.s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    x, info = oracle.solve(P, A, sys.rhs, pc=pc, rtol=1e-12, maxit=3000)
    assert info["converged"] and info["rel_res_true"] <= 1e-12
    xd = np.linalg.solve(dense.dense_B(sys, Ainv), sys.rhs)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_preconditioner_quality_order_cfg0():
    """Qualitative claim of Sec. 5.1.1: coupled <= shifted < unshifted in
    GMRES iterations (parity unpinned: no paper value applies to synthetic
    systems; this only checks the ordering)."""
    sys = dgsynth.config_system("cfg0")
    A, _, _ = oracle.radau_iia(sys.s)
    P = oracle.Problem(sys)
    its = {}
    for pc in ("coupled", "uncoupled_shifted", "uncoupled"):
        _, info = oracle.solve(P, A, sys.rhs, pc=pc, rtol=1e-10)
        its[pc] = info["iters"]
    assert its["coupled"] <= its["uncoupled_shifted"] < its["uncoupled"], its


@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_linear_ode_one_step_is_pade(s):
    """For M u' = J u the transformed Newton system with R = 1_s (x) (J u0)
    is exact in one step, and u1 = u0 + dt w_s = Q(Z)^{-1} P(Z) u0 with
    Z = dt M^{-1} J and (P, Q) the (s-1, s) Pade pair of e^z."""
    sys = dgsynth.make_system(100 + s, dgsynth.grid2d(4), 3, s, 0.3)
    A, _, _ = oracle.radau_iia(s)
    Pr = oracle.Problem(sys)
    n = sys.T * sys.m
    Jd, Md = dense.dense_J(sys), dense.dense_M(sys)
    u0 = np.random.default_rng(s).standard_normal(n)
    R = np.tile(Jd @ u0, s)
    w, info = oracle.solve(Pr, A, R, pc="coupled", rtol=1e-14, maxit=500)
    assert info["converged"]
    u1 = u0 + sys.dt * w[(s - 1) * n:]
    Z = sys.dt * np.linalg.solve(Md, Jd)
    Pc, Qc = _pade_pq(s)
    Pm = sum(c * np.linalg.matrix_power(Z, i) for i, c in enumerate(Pc))
    Qm = sum(c * np.linalg.matrix_power(Z, i) for i, c in enumerate(Qc))
    ref = np.linalg.solve(Qm, Pm @ u0)
    assert np.linalg.norm(u1 - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("s", [2, 3])
def test_transformed_solution_is_A_times_untransformed(s):
    """W = (A (x) I) K where K solves the untransformed Newton system with the
    same right-hand side (Sec. 4.1)."""
    sys = dgsynth.make_system(200 + s, dgsynth.grid2d(4), 3, s, 0.2)
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sys)
    w, info = oracle.solve(P, A, sys.rhs, pc="uncoupled_shifted", rtol=1e-14, maxit=500)
    assert info["converged"]
    K = np.linalg.solve(dense.dense_B_untransformed(sys, A), sys.rhs)
    n = sys.T * sys.m
    W = (A @ K.reshape(s, n)).ravel()
    assert np.linalg.norm(w - W) / np.linalg.norm(W) < 1e-12


def test_exact_preconditioner_one_iteration():
    """r = 0: coupled ILU(0) is an exact LU, so GMRES needs one iteration."""
    sys = dgsynth.make_system(5, dgsynth.isolated_mesh(6), 4, 3, 0.5)
    A, _, _ = oracle.radau_iia(3)
    x, info = oracle.solve(oracle.Problem(sys), A, sys.rhs, pc="coupled", rtol=1e-12)
    assert info["converged"] and info["iters"] == 1


def test_unpreconditioned_full_gmres_terminates():
    """Unrestarted GMRES without preconditioning reaches the solution in at
    most N steps (exact-arithmetic finite termination; here N = 2*4*2 = 16)."""
    sys = dgsynth.make_system(6, dgsynth.path_mesh(4), 2, 2, 0.5)
    A, _, _ = oracle.radau_iia(2)
    N = 2 * 4 * 2
    x, info = oracle.solve(oracle.Problem(sys), A, sys.rhs, pc="none", rtol=1e-11,
                           restart=N, maxit=N + 2)
    assert info["converged"] and info["iters"] <= N


@pytest.mark.parametrize("orth", ["mgs", "cgs2"])
def test_residual_history_monotone_within_cycle(orth):
    sys = dgsynth.config_system("cfg0", dt=1.0)
    A, _, _ = oracle.radau_iia(2)
    x, info, hist = oracle.solve(oracle.Problem(sys), A, sys.rhs, pc="uncoupled",
                                 rtol=1e-10, restart=10, orth=orth, history=True)
    assert info["converged"]
    for c0 in range(0, len(hist), 10):
        h = hist[c0:c0 + 10]
        assert np.all(np.diff(h) <= 1e-15 + 1e-12 * h[:-1])


def test_mgs_and_cgs2_agree():
    sys = dgsynth.config_system("cfg0")
    A, _, _ = oracle.radau_iia(2)
    P = oracle.Problem(sys)
    x1, i1 = oracle.solve(P, A, sys.rhs, pc="coupled", rtol=1e-12, orth="mgs")
    x2, i2 = oracle.solve(P, A, sys.rhs, pc="coupled", rtol=1e-12, orth="cgs2")
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-10


def test_noconv_and_zero_rhs():
    sys = dgsynth.config_system("cfg0")
    A, _, _ = oracle.radau_iia(2)
    P = oracle.Problem(sys)
    x, info = oracle.solve(P, A, sys.rhs, pc="none", rtol=1e-12, maxit=3)
    assert not info["converged"] and info["status"] == 4 and info["iters"] == 3
    x, info = oracle.solve(P, A, np.zeros(P.N), pc="coupled")
    assert info["converged"] and not x.any()
