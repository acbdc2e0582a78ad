"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Kernel-level outputs (operator, factors, preconditioner apply) must agree
with the oracle to 1e-12 relative (FP64 arithmetic, different summation
order and a different pivot inversion method); full solves run both sides to
rtol 1e-12 and must agree to 1e-10 relative, with iteration counts within
one of the oracle's CGS2 GMRES.
"""
import sys

import numpy as np
import pytest

import dgsynth
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _system(s, dim, N, m, nJ=1, seed=11, dt=0.1, mesh=None):
    if mesh is None:
        mesh = dgsynth.grid2d(N) if dim == 2 else dgsynth.grid3d(N)
    return dgsynth.make_system(seed, mesh, m, s, dt, nJ=nJ)


# shapes: several tiles, ragged m, every stage count, shared and per-stage J
OP_CASES = [
    (2, 2, 8, 16, 1),    # the small validation workload's shape
    (3, 2, 4, 5, 1),     # ragged block size
    (1, 2, 4, 7, 1),
    (4, 2, 5, 36, 4),
    (5, 2, 4, 9, 1),
    (3, 2, 6, 64, 3),
    (3, 3, 4, 135, 1),   # 3D hex, m = 135 (p = 2, 5 components)
    (2, 2, 4, 100, 2),
]


def _ids(c):
    return "s%d_%dd_N%d_m%d_nJ%d" % c


@pytest.mark.parametrize("case", OP_CASES, ids=_ids)
def test_operator_parity(case):
    irk = _irk()
    s, dim, N, m, nJ = case
    _say("operator", case)
    sy = _system(s, dim, N, m, nJ)
    sol = irk.Solver(sy, irk.Options(pc="none"))
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    x = np.random.default_rng(5).standard_normal(P.N)
    y = sol.apply_operator(x).cpu().numpy()
    yo = oracle.matvec(P, oracle.inverse(A), x)
    assert _rel(y, yo) < 1e-12
    sol.close()


def _oracle_pivots(sy, pc):
    """Inverse pivot blocks P_{k,i}^{-1} [s][T] from the oracle's generic ILU(0)."""
    s, T, m = sy.s, sy.T, sy.m
    A, _, _ = oracle.radau_iia(s)
    Ainv = oracle.inverse(A)
    P = oracle.Problem(sy)
    out = np.zeros((s, T, m, m))
    if pc == "coupled":
        F = oracle.build_coupled(P, Ainv).ilu0()
        for k in range(s):
            for i in range(T):
                out[k, i] = np.linalg.inv(F.block(k * T + i, k * T + i))
        return out, F
    al = oracle.shifts(Ainv, 0 if pc == "uncoupled_shifted" else 1)
    for k in range(s):
        F = oracle.build_stage(P, k, Ainv[k, k] + al[k]).ilu0()
        for i in range(T):
            out[k, i] = np.linalg.inv(F.block(i, i))
    return out, None


FAC_CASES = [
    ("coupled", (2, 2, 8, 16, 1)),
    ("coupled", (3, 2, 4, 8, 3)),
    ("coupled", (4, 2, 4, 5, 1)),
    ("uncoupled_shifted", (3, 2, 5, 12, 1)),
    ("uncoupled", (2, 2, 4, 7, 2)),
    ("coupled", (3, 3, 4, 135, 1)),
    ("uncoupled_shifted", (3, 2, 6, 64, 1)),
    # the block-size classes of the factorization kernels and their edges:
    # m <= 64 partial tiles / all tiles with a ragged K block, 64 < m <= 128
    # (two row groups per lane), 128 < m <= 160 (three)
    ("coupled", (3, 2, 4, 33, 1)),
    ("coupled", (2, 2, 4, 60, 1)),
    ("uncoupled_shifted", (2, 2, 4, 100, 1)),
    ("coupled", (2, 2, 4, 129, 1)),
    ("uncoupled", (2, 2, 4, 160, 1)),
]


@pytest.mark.parametrize("pc,case", FAC_CASES, ids=lambda v: v if isinstance(v, str) else _ids(v))
def test_factor_parity(pc, case):
    irk = _irk()
    s, dim, N, m, nJ = case
    _say("factor", pc, case)
    sy = _system(s, dim, N, m, nJ, seed=23)
    sol = irk.Solver(sy, irk.Options(pc=pc))
    sol.factor()
    Pg, Cg = sol.export_factors(cross=True)
    Pg = Pg.cpu().numpy()
    Po, F = _oracle_pivots(sy, pc)
    assert _rel(Pg, Po) < 1e-11
    if pc == "coupled" and s > 1:
        Cg = Cg.cpu().numpy()
        T = sy.T
        worst = 0.0
        for k in range(s):
            for l in range(s):
                if l == k:
                    continue
                for i in range(T):
                    G = F.block(k * T + i, l * T + i)
                    ref = G if l > k else G @ F.block(l * T + i, l * T + i)
                    worst = max(worst, np.abs(Cg[k, l, i] - ref).max() / max(np.abs(ref).max(), 1e-300))
        assert worst < 1e-11
    sol.close()


@pytest.mark.parametrize("m", [16, 64, 100, 135])
def test_factor_pivot_ties(m):
    """Pivot blocks whose columns hold equal magnitudes everywhere (random
    +-1 mass blocks, zero Jacobian, so P_{k,i} = A^{-1}_kk M_i): every pivot
    choice is a tie, decided by the first candidate row.  The inverses must
    still match the oracle's."""
    irk = _irk()
    _say("factor ties", m)
    sy = _system(2, 2, 4, m, 1, seed=41)
    rng = np.random.default_rng(43 + m)
    sy.J[:] = 0.0
    for i in range(sy.T):
        while True:             # a well-conditioned sign matrix (redrawn otherwise)
            sy.M[i] = rng.choice([-1.0, 1.0], size=(m, m))
            if np.linalg.cond(sy.M[i]) < 1e4:
                break
    sol = irk.Solver(sy, irk.Options(pc="uncoupled"))
    sol.factor()
    Pg = sol.export_factors(cross=False)
    Po, _ = _oracle_pivots(sy, "uncoupled")
    # condition numbers up to 1e4: the two FP64 inverses agree to ~cond * eps
    assert _rel(Pg.cpu().numpy(), Po) < 1e-10
    sol.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled"])
@pytest.mark.parametrize("case", [(2, 2, 8, 16, 1), (3, 2, 5, 9, 1), (4, 2, 4, 6, 4),
                                  (3, 3, 4, 20, 1)], ids=_ids)
def test_preconditioner_parity(pc, case):
    irk = _irk()
    s, dim, N, m, nJ = case
    _say("pc apply", pc, case)
    sy = _system(s, dim, N, m, nJ, seed=31)
    sol = irk.Solver(sy, irk.Options(pc=pc))
    sol.factor()
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(7).standard_normal(P.N)
    z = sol.apply_preconditioner(v).cpu().numpy()
    zo = oracle.pc_apply(P, A, pc, v)
    assert _rel(z, zo) < 1e-11
    sol.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled", "none"])
def test_cfg0_solve_parity(pc):
    irk = _irk()
    _say("cfg0 solve", pc)
    sy = dgsynth.config_system("cfg0")
    sol = irk.Solver(sy, irk.Options(pc=pc, rtol=1e-12))
    sol.factor()
    x, info = sol.solve(sy.rhs)
    x = x.cpu().numpy()
    A, _, _ = oracle.radau_iia(sy.s)
    xo, io = oracle.solve(oracle.Problem(sy), A, sy.rhs, pc=pc, rtol=1e-12, orth="cgs2", maxit=3000)
    _say("  gpu iters", info["iters"], "oracle iters", io["iters"], "res", info["rel_res_true"])
    assert info["converged"] and info["rel_res_true"] <= 1e-12
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-10
    assert abs(info["iters"] - io["iters"]) <= 1
    assert info["equiv_mults"] == info["iters"] * sy.s
    sol.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
@pytest.mark.parametrize("dt", [0.01, 1.0])
def test_cfg1_shape_small_mesh_parity(pc, dt):
    """The s = 3, m = 64 block shape of the FP64 workload on a 12 x 12 mesh."""
    irk = _irk()
    _say("cfg1-shape solve", pc, dt)
    sy = dgsynth.config_system("cfg1", N=12, dt=dt)
    sol = irk.Solver(sy, irk.Options(pc=pc, rtol=1e-12))
    sol.factor()
    x, info = sol.solve(sy.rhs)
    x = x.cpu().numpy()
    A, _, _ = oracle.radau_iia(sy.s)
    xo, io = oracle.solve(oracle.Problem(sy), A, sy.rhs, pc=pc, rtol=1e-12, orth="cgs2")
    _say("  gpu iters", info["iters"], "oracle iters", io["iters"])
    assert info["converged"]
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-10
    assert abs(info["iters"] - io["iters"]) <= 1
    sol.close()


def test_restart_and_initial_guess():
    """Short restart forces several cycles; a nonzero x0 is honoured."""
    irk = _irk()
    _say("restart / x0")
    sy = dgsynth.config_system("cfg0", dt=1.0)
    sol = irk.Solver(sy, irk.Options(pc="uncoupled", rtol=1e-11, restart=4))
    sol.factor()
    x0 = np.random.default_rng(3).standard_normal(sy.s * sy.T * sy.m)
    x, info = sol.solve(sy.rhs, x0=x0)
    A, _, _ = oracle.radau_iia(sy.s)
    xo, io = oracle.solve(oracle.Problem(sy), A, sy.rhs, pc="uncoupled", rtol=1e-11, restart=4,
                          orth="cgs2", x0=x0)
    assert info["converged"] and info["restarts"] >= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-9
    assert abs(info["iters"] - io["iters"]) <= 2
    sol.close()


def test_deterministic():
    irk = _irk()
    sy = dgsynth.config_system("cfg1", N=8)
    sol = irk.Solver(sy, irk.Options(pc="coupled"))
    sol.factor()
    x1, i1 = sol.solve(sy.rhs)
    x2, i2 = sol.solve(sy.rhs)
    assert i1["iters"] == i2["iters"]
    assert torch.equal(x1, x2)
    sol.close()


UNTR_CASES = [(2, 2, 8, 16, 1), (3, 2, 4, 5, 1), (1, 2, 4, 7, 1), (4, 2, 5, 36, 4),
              (5, 2, 4, 9, 1), (3, 2, 6, 64, 3), (3, 3, 4, 135, 1)]


@pytest.mark.parametrize("form", ["blocks", "fused"])
@pytest.mark.parametrize("case", UNTR_CASES, ids=_ids)
def test_untransformed_operator_parity(form, case):
    """The untransformed operator I (x) M - dt [a_kl J_k] (Eq. newton-system-2)
    against the oracle's, and the transformation identity
    B x = B_untr (A^{-1} (x) I) x between the library's two operators."""
    irk = _irk()
    s, dim, N, m, nJ = case
    _say("untransformed", form, case)
    sy = _system(s, dim, N, m, nJ, seed=13)
    sol = irk.Solver(sy, irk.Options(pc="none"))
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    x = np.random.default_rng(6).standard_normal(P.N)
    y = sol.apply_operator_untransformed(x, form=form).cpu().numpy()
    yo = oracle.matvec_untransformed(P, A, x)
    assert _rel(y, yo) < 1e-12
    Ainv = oracle.inverse(A)
    n = sy.T * sy.m
    xt = (Ainv @ x.reshape(s, n)).reshape(-1)
    yt = sol.apply_operator_untransformed(xt, form=form).cpu().numpy()
    assert _rel(yt, sol.apply_operator(x).cpu().numpy()) < 1e-12
    sol.close()
