"""Pins of the oracle's operators (Sec. 4.1, Eq. newton-system-2 and
Eq. big-irk) against dense brute force and the algebraic identity that links
the transformed and untransformed systems."""
import numpy as np
import pytest

import dgsynth
import oracle
from tests import dense


def _sys(s=2, N=4, m=3, nJ=1, seed=7, dt=0.3):
    return dgsynth.make_system(seed, dgsynth.grid2d(N), m, s, dt, nJ=nJ)


@pytest.mark.parametrize("s,nJ", [(1, 1), (2, 1), (3, 1), (3, 3), (4, 4)])
def test_transformed_matvec_vs_dense(s, nJ):
    sys = _sys(s=s, nJ=nJ)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    x = np.random.default_rng(1).standard_normal(P.N)
    y = oracle.matvec(P, Ainv, x)
    yd = dense.dense_B(sys, Ainv) @ x
    np.testing.assert_allclose(y, yd, rtol=0, atol=1e-12 * np.abs(yd).max())


@pytest.mark.parametrize("s,nJ", [(2, 1), (3, 1), (3, 3)])
def test_untransformed_matvec_vs_dense(s, nJ):
    sys = _sys(s=s, nJ=nJ, seed=3)
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sys)
    x = np.random.default_rng(2).standard_normal(P.N)
    y = oracle.matvec_untransformed(P, A, x)
    yd = dense.dense_B_untransformed(sys, A) @ x
    np.testing.assert_allclose(y, yd, rtol=0, atol=1e-12 * np.abs(yd).max())


@pytest.mark.parametrize("s", [2, 3, 4])
def test_transformed_equals_untransformed_times_Ainv(s):
    """With W = (A (x) I) K:  B_tr x = B_untr (A^{-1} (x) I) x  (Sec. 4.1)."""
    sys = _sys(s=s, nJ=s, seed=11, m=5)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    x = np.random.default_rng(4).standard_normal(P.N)
    n = sys.T * sys.m
    xk = (Ainv @ x.reshape(s, n)).ravel()
    y1 = oracle.matvec(P, Ainv, x)
    y2 = oracle.matvec_untransformed(P, A, xk)
    np.testing.assert_allclose(y1, y2, rtol=0, atol=1e-12 * np.abs(y1).max())


def test_single_stage_is_backward_euler_operator():
    """s = 1 (A = [1]) reduces the transformed operator to (M - dt J) x."""
    sys = _sys(s=1, m=4)
    P = oracle.Problem(sys)
    x = np.random.default_rng(5).standard_normal(P.N)
    y = oracle.matvec(P, np.array([[1.0]]), x)
    yd = (dense.dense_M(sys) - sys.dt * dense.dense_J(sys)) @ x
    np.testing.assert_allclose(y, yd, rtol=0, atol=1e-13 * np.abs(yd).max())


def test_shared_J_equals_per_stage_copies():
    """nJ = 1 is the same operator as nJ = s with every J_k equal."""
    sys = _sys(s=3, m=4, seed=9)
    A, _, _ = oracle.radau_iia(3)
    Ainv = oracle.inverse(A)
    P1 = oracle.Problem(sys)
    sys3 = dgsynth.System(**{**sys.__dict__})
    sys3.J = np.repeat(sys.J, 3, axis=0)
    sys3.nJ = 3
    P3 = oracle.Problem(sys3)
    x = np.random.default_rng(6).standard_normal(P1.N)
    np.testing.assert_array_equal(oracle.matvec(P1, Ainv, x), oracle.matvec(P3, Ainv, x))


def test_generator_structure():
    """Periodic grids give sorted rows with the diagonal, r+1 blocks per row,
    a structurally symmetric pattern, and a triangle-free neighbour graph."""
    sys = dgsynth.config_system("cfg0")
    T = sys.T
    assert T == 64 and sys.m == 16 and sys.nnzb == 5 * T
    nb = [set(sys.col_idx[sys.row_ptr[i]:sys.row_ptr[i + 1]]) - {i} for i in range(T)]
    for i in range(T):
        row = sys.col_idx[sys.row_ptr[i]:sys.row_ptr[i + 1]]
        assert list(row) == sorted(row) and i in row
        for j in nb[i]:
            assert i in nb[j]
            assert not (nb[i] & nb[j])          # no triangles
    g3 = dgsynth.grid3d(4)
    assert all(len(n) == 6 for n in g3)
    with pytest.raises(ValueError):
        dgsynth.grid2d(3)
