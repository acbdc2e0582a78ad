"""Pins of the oracle's block ILU(0) (Sec. 4.2.1 Alg. 1-2, Sec. 4.3.1 Alg. 3,
Sec. 4.3.2): the ILU(0) characterization, special cases where it is an exact
LU, the D-ILU structure on triangle-free meshes, and the explicit coupled
form as an independent second implementation."""
import numpy as np
import pytest

import dgsynth
import oracle
from tests import dense


def _sys(s=2, N=4, m=3, nJ=1, seed=7, dt=0.3, mesh=None, permute=True):
    mesh = dgsynth.grid2d(N) if mesh is None else mesh
    return dgsynth.make_system(seed, mesh, m, s, dt, nJ=nJ, permute=permute)


def _pattern_check(B0, F):
    """(L~ U~)_pq == B_pq for every block (p, q) of the pattern: the defining
    property of ILU(0)."""
    L, U = dense.factors_dense(F)
    LU = L @ U
    m = B0.m
    worst = 0.0
    for i in range(B0.nb):
        for a in range(B0.ptr[i], B0.ptr[i + 1]):
            j = B0.col[a]
            d = np.abs(LU[i * m:(i + 1) * m, j * m:(j + 1) * m] - B0.val[a]).max()
            worst = max(worst, d / max(1.0, np.abs(B0.val[a]).max()))
    return worst


@pytest.mark.parametrize("s", [2, 3, 4])
def test_coupled_pattern_invariant(s):
    sys = _sys(s=s, N=4, m=4, nJ=s, seed=20 + s)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    B0 = oracle.build_coupled(P, Ainv)
    np.testing.assert_array_equal(B0.dense(), dense.dense_B(sys, Ainv))
    F = B0.copy().ilu0()
    assert _pattern_check(B0, F) < 1e-13


@pytest.mark.parametrize("shifted", [True, False])
def test_uncoupled_pattern_invariant(shifted):
    s = 3
    sys = _sys(s=s, N=5, m=3, nJ=s, seed=5)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    al = oracle.shifts(Ainv, 0 if shifted else 1)
    P = oracle.Problem(sys)
    for k in range(s):
        B0 = oracle.build_stage(P, k, Ainv[k, k] + al[k])
        Bd = (Ainv[k, k] + al[k]) * dense.dense_M(sys) - sys.dt * dense.dense_J(sys, k)
        np.testing.assert_array_equal(B0.dense(), Bd)
        F = B0.copy().ilu0()
        assert _pattern_check(B0, F) < 1e-13


def test_dilu_structure_triangle_free():
    """On a triangle-free mesh the factors keep every off-diagonal Jacobian
    block: U~_ij = B_ij (j > i) exactly, and L~_ji = B_ji P_i^{-1}; only the
    pivots change (Alg. 2)."""
    s = 2
    sys = _sys(s=s, N=4, m=4, seed=31)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    B0 = oracle.build_coupled(P, Ainv)
    F = B0.copy().ilu0()
    nb, m = B0.nb, B0.m
    for i in range(nb):
        for a in range(B0.ptr[i], B0.ptr[i + 1]):
            j = B0.col[a]
            if j > i:
                np.testing.assert_array_equal(F.val[a], B0.val[a])
            elif j < i:
                Pj = F.block(j, j)
                np.testing.assert_allclose(F.val[a] @ Pj, B0.val[a], atol=1e-13)


def test_path_mesh_uncoupled_is_exact_lu():
    """On a tree (non-periodic chain) in natural order block ILU(0) drops no
    fill, so L~U~ = B exactly and the preconditioner is an exact inverse."""
    s = 2
    sys = _sys(s=s, mesh=dgsynth.path_mesh(7), m=4, seed=3, permute=False)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    B0 = oracle.build_stage(P, 0, Ainv[0, 0])
    F = B0.copy().ilu0()
    L, U = dense.factors_dense(F)
    np.testing.assert_allclose(L @ U, B0.dense(), atol=1e-13)
    v = np.random.default_rng(0).standard_normal(B0.nb * B0.m)
    np.testing.assert_allclose(B0.matvec(F.apply(v)), v, atol=1e-12)


def test_periodic_ring_is_not_exact():
    """A periodic ring is not a tree: ILU(0) drops fill there."""
    s = 1
    ring = [[(e - 1) % 6, (e + 1) % 6] for e in range(6)]
    sys = _sys(s=s, mesh=ring, m=3, seed=4, permute=False)
    P = oracle.Problem(sys)
    B0 = oracle.build_stage(P, 0, 1.0)
    F = B0.copy().ilu0()
    L, U = dense.factors_dense(F)
    assert np.abs(L @ U - B0.dense()).max() > 1e-6


@pytest.mark.parametrize("s", [2, 3])
def test_isolated_elements_coupled_is_exact(s):
    """r = 0: B is block diagonal over elements (stage coupling only); the
    coupled ILU(0) is then an exact LU of every element's s x s block system."""
    sys = _sys(s=s, mesh=dgsynth.isolated_mesh(5), m=3, seed=8)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    B0 = oracle.build_coupled(P, Ainv)
    F = B0.copy().ilu0()
    L, U = dense.factors_dense(F)
    np.testing.assert_allclose(L @ U, B0.dense(), atol=1e-13)


def test_single_element_coupled_is_exact():
    """T = 1: the coupled pattern is full, so ILU(0) is a block LU."""
    s = 4
    sys = _sys(s=s, mesh=[[]], m=5, seed=12, nJ=s)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    B0 = oracle.build_coupled(oracle.Problem(sys), Ainv)
    F = B0.copy().ilu0()
    L, U = dense.factors_dense(F)
    np.testing.assert_allclose(L @ U, B0.dense(), atol=1e-12)


@pytest.mark.parametrize("s", [2, 3, 4])
def test_explicit_coupled_equals_generic(s):
    """The explicit element-local form (pivots P_{k,i}, cross-stage blocks
    C_{kl,i}) reproduces the generic factorization of the coupled matrix."""
    sys = _sys(s=s, N=4, m=4, nJ=s, seed=40 + s)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    F = oracle.build_coupled(P, Ainv).ilu0()
    Pk, Ck = oracle.coupled_explicit(P, Ainv)
    T = sys.T
    for k in range(s):
        for i in range(T):
            np.testing.assert_allclose(Pk[k, i], F.block(k * T + i, k * T + i), atol=1e-12)
            for l in range(s):
                if l == k:
                    continue
                G = F.block(k * T + i, l * T + i)
                if l > k:        # upper factor block
                    np.testing.assert_allclose(Ck[k, l, i], G, atol=1e-12)
                else:            # lower factor block = C_{kl} P_{l}^{-1}
                    np.testing.assert_allclose(Ck[k, l, i], G @ Pk[l, i], atol=1e-12)


def test_literal_alg3_differs_for_three_stages():
    """At s = 3 the factorization changes the cross-stage block C_{23,i}
    (stages 2 and 3, both after the first pivot).  Alg. 3 as printed has no
    such update, so it is not the ILU(0) of the coupled matrix for s >= 3;
    the standard ILU(0) reading (pinned by the pattern invariant above) is
    the one computed."""
    s = 3
    sys = _sys(s=s, N=4, m=4, seed=55)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    Pk, Ck = oracle.coupled_explicit(P, Ainv)
    T = sys.T
    # at least one cross-stage block between stages >= 2 moved away from A^{-1}_kl M
    moved = max(np.abs(Ck[1, 2, i] - Ainv[1, 2] * sys.M[i]).max() for i in range(T))
    assert moved > 1e-3


def test_apply_solves_factored_system():
    s = 3
    sys = _sys(s=s, N=4, m=3, seed=60)
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sys)
    F = oracle.build_coupled(P, Ainv).ilu0()
    L, U = dense.factors_dense(F)
    v = np.random.default_rng(1).standard_normal(P.N)
    z = F.apply(v)
    np.testing.assert_allclose(L @ (U @ z), v, atol=1e-12)
    # pc_apply entry point (coupled) agrees with the BlockMatrix path
    np.testing.assert_allclose(oracle.pc_apply(P, A, "coupled", v), z, rtol=0, atol=1e-14)


def test_singular_pivot_reported():
    sys = _sys(s=1, N=4, m=3, seed=61)
    sys.M[:] = 0.0
    sys.J[:] = 0.0
    P = oracle.Problem(sys)
    B0 = oracle.build_stage(P, 0, 1.0)
    with pytest.raises(np.linalg.LinAlgError):
        B0.ilu0()


# The uncoupled preconditioners on a tree.  Along a non-periodic path in
# natural order the per-stage block ILU(0) is an exact LU, so the stage-
# uncoupled preconditioner of Sec. 4.3.2 must be the exact block-diagonal
# solve  z_k = ((A^{-1}_kk + alpha_k) M - dt J_k)^{-1} v_k.  For s = 2 the
# Radau IIA inverse is A^{-1} = [[3/2, 1/2], [-9/2, 5/2]] (exact rationals),
# so the column-sum shifts of Sec. 4.3.2 are alpha = (9/2, 1/2) and the
# pivot coefficients (6, 3); they are written out here, not taken from the
# oracle.  A dropped shift, a row-sum shift (1/2, 9/2), a wrong stage offset
# or the wrong stage Jacobian fails one of these cases.
S2_AINV_DIAG = (1.5, 2.5)


@pytest.mark.parametrize("nJ", [1, 2])
@pytest.mark.parametrize("pc,alpha", [("uncoupled_shifted", (4.5, 0.5)), ("uncoupled", (0.0, 0.0))])
def test_uncoupled_apply_exact_on_tree(pc, alpha, nJ):
    sys = _sys(s=2, m=3, nJ=nJ, seed=77, dt=0.4, mesh=dgsynth.path_mesh(7), permute=False)
    A, _, _ = oracle.radau_iia(2)
    P = oracle.Problem(sys)
    v = np.random.default_rng(78).standard_normal(P.N)
    z = oracle.pc_apply(P, A, pc, v)
    n = sys.T * sys.m
    for k in range(2):
        Bk = (S2_AINV_DIAG[k] + alpha[k]) * dense.dense_M(sys) - sys.dt * dense.dense_J(sys, k)
        zk = np.linalg.solve(Bk, v[k * n:(k + 1) * n])
        np.testing.assert_allclose(z[k * n:(k + 1) * n], zk, rtol=0, atol=1e-12 * np.abs(zk).max())


def test_uncoupled_shifted_apply_exact_on_tree_three_stages():
    """s = 3 with one Jacobian per stage: the third stage's offset and J_3
    are reached.  Shifts from the column sums of A^{-1}, which the tableau
    pins fix (C(3), B(5), App. A closed forms)."""
    s = 3
    sys = _sys(s=s, m=4, nJ=s, seed=79, dt=0.25, mesh=dgsynth.path_mesh(6), permute=False)
    A, _, _ = oracle.radau_iia(s)
    Ainv = np.linalg.inv(A)
    alpha = [sum(abs(Ainv[j, k]) for j in range(s) if j != k) for k in range(s)]
    P = oracle.Problem(sys)
    v = np.random.default_rng(80).standard_normal(P.N)
    z = oracle.pc_apply(P, A, "uncoupled_shifted", v)
    n = sys.T * sys.m
    for k in range(s):
        Bk = (Ainv[k, k] + alpha[k]) * dense.dense_M(sys) - sys.dt * dense.dense_J(sys, k)
        zk = np.linalg.solve(Bk, v[k * n:(k + 1) * n])
        np.testing.assert_allclose(z[k * n:(k + 1) * n], zk, rtol=0, atol=1e-12 * np.abs(zk).max())
