"""Element-wise parity of every form of the preconditioner sweeps, and the
method's exact-preconditioner cases, on the GPU.

* The large-level sweep forms (streaming, and prefetching without the
  Jacobian columns) are forced for every level (IRK_SWEEP_BIG=1 and
  IRK_SWEEP_BIG_FORM, read at set-up) and compared with the oracle's
  preconditioner apply element by element, for all three FP64
  preconditioners, block sizes 6 to 135 and 2D/3D meshes.
* Rows with more than 8 lower or upper neighbours (the records keep the
  first 8 columns; the rest are read from the column index) on a complete
  bipartite mesh, which is triangle-free.
* The inner-iteration kernels of the mixed-precision solve (FP32 operator;
  FP32 sweeps with FP32 / BF16 / FP16-scaled factors) against the FP64
  oracle, within bounds derived from the storage precision.
* Exact cases: r = 0 (isolated elements) makes the coupled ILU(0) an exact
  LU of B, so GMRES converges in one iteration to the dense solution; on a
  non-periodic path in natural order (a tree) each stage's ILU(0) is exact,
  so the uncoupled applies equal dense block-diagonal solves.
"""
import sys

import numpy as np
import pytest

import dgsynth
import oracle
from tests import dense

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


def _system(s, dim, N, m, nJ=1, seed=31, dt=0.1):
    mesh = dgsynth.grid2d(N) if dim == 2 else dgsynth.grid3d(N)
    return dgsynth.make_system(seed, mesh, m, s, dt, nJ=nJ)


def _ids(c):
    return "s%d_%dd_N%d_m%d_nJ%d" % c


STREAM_CASES = [(2, 2, 8, 16, 1), (3, 2, 5, 9, 1), (4, 2, 4, 6, 4), (3, 3, 4, 20, 1),
                (3, 2, 6, 64, 1), (3, 3, 4, 135, 1), (2, 2, 5, 100, 2)]


@pytest.mark.parametrize("form", ["streaming", "prefetch_lite"])
@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled"])
@pytest.mark.parametrize("case", STREAM_CASES, ids=_ids)
def test_streaming_form_parity(pc, case, form, monkeypatch):
    """Every level in the large-level form (streaming, or prefetching without
    the Jacobian columns), element-wise against the oracle."""
    irk = _irk()
    monkeypatch.setenv("IRK_SWEEP_BIG", "1")
    if form == "prefetch_lite":
        monkeypatch.setenv("IRK_SWEEP_BIG_FORM", "2")
    s, dim, N, m, nJ = case
    _say("streaming sweep", pc, case)
    sy = _system(s, dim, N, m, nJ)
    sol = irk.Solver(sy, irk.Options(pc=pc))
    sol.factor()
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(7).standard_normal(P.N)
    z = sol.apply_preconditioner(v).cpu().numpy()
    zo = oracle.pc_apply(P, A, pc, v)
    assert _rel(z, zo) < 1e-11
    sol.close()


def _bipartite(a, b):
    """Complete bipartite mesh K_{a,b} numbered leaves, hubs, leaves: the a
    hubs (labels b//2 .. b//2 + a - 1) touch all b leaves, so each hub row
    has b//2 lower and b - b//2 upper blocks.  Bipartite, hence
    triangle-free."""
    lo = b // 2
    hubs = list(range(lo, lo + a))
    leaves = [e for e in range(a + b) if e not in hubs]
    return [leaves if e in hubs else hubs for e in range(a + b)]


@pytest.mark.parametrize("form", ["default", "streaming"])
@pytest.mark.parametrize("pc,s,m", [("coupled", 3, 12), ("uncoupled_shifted", 2, 16),
                                    ("coupled", 2, 64)])
def test_rows_longer_than_record(form, pc, s, m, monkeypatch):
    """Hubs with 10 lower and 10 upper neighbours: rows with more than 8
    lower and upper blocks in the sweeps (and 21 blocks in the matvec)."""
    irk = _irk()
    if form == "streaming":
        monkeypatch.setenv("IRK_SWEEP_BIG", "1")
    mesh = _bipartite(3, 20)
    sy = dgsynth.make_system(91 + m, mesh, m, s, 0.05, permute=False)
    lower = [int(np.sum(sy.col_idx[sy.row_ptr[i]:sy.row_ptr[i + 1]] < i)) for i in range(sy.T)]
    upper = [int(np.sum(sy.col_idx[sy.row_ptr[i]:sy.row_ptr[i + 1]] > i)) for i in range(sy.T)]
    _say("long rows", form, pc, s, m, "max lower", max(lower), "max upper", max(upper))
    assert max(lower) > 8 and max(upper) > 8
    sol = irk.Solver(sy, irk.Options(pc=pc))
    sol.factor()
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(P.N)
    assert _rel(sol.apply_preconditioner(v).cpu().numpy(), oracle.pc_apply(P, A, pc, v)) < 1e-11
    x = rng.standard_normal(P.N)
    assert _rel(sol.apply_operator(x).cpu().numpy(), oracle.matvec(P, oracle.inverse(A), x)) < 1e-12
    sol.close()


# Bounds for the inner (reduced-precision) kernels against the FP64 oracle,
# relative to the largest output entry: the factors are stored with unit
# roundoff u (FP32 2^-24, BF16 2^-8, FP16 2^-11 after the per-block power-
# of-two scale), the arithmetic is FP32 throughout, and an output entry is
# the end of a chain of ~2 L dependent block products (L levels per sweep);
# each product sums (r + 1) m terms whose magnitudes stay within a small
# multiple of the result on these diagonally dominant pivots.  The bounds
# take 16 u for the 16-bit factors and 2^-17 for the FP32 ones (where the
# FP32 arithmetic, not the storage, dominates).
INNER_BOUND = {"fp32": 2.0 ** -17, "bf16": 16 * 2.0 ** -8, "fp16s": 16 * 2.0 ** -11}


@pytest.mark.parametrize("form", ["default", "streaming", "prefetch_lite"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16s"])
@pytest.mark.parametrize("pc,case", [("uncoupled_shifted", (3, 3, 4, 135, 1)),
                                     ("coupled", (3, 2, 6, 64, 1)),
                                     ("coupled", (2, 2, 8, 16, 1))],
                         ids=lambda v: v if isinstance(v, str) else _ids(v))
def test_inner_preconditioner_parity(form, prec, pc, case, monkeypatch):
    irk = _irk()
    if form != "default":
        monkeypatch.setenv("IRK_SWEEP_BIG", "1")
    if form == "prefetch_lite":
        monkeypatch.setenv("IRK_SWEEP_BIG_FORM", "2")
    s, dim, N, m, nJ = case
    sy = _system(s, dim, N, m, nJ, seed=53)
    sol = irk.Solver(sy, irk.Options(pc=pc, matvec_prec="fp32", factor_prec=prec, rtol=1e-8))
    sol.factor()
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(9).standard_normal(P.N)
    z = sol.apply_preconditioner_inner(v).cpu().numpy()
    zo = oracle.pc_apply(P, A, pc, v)
    err = _rel(z, zo)
    _say("inner pc", form, prec, pc, case, f"rel err {err:.2e} bound {INNER_BOUND[prec]:.1e}")
    assert err < INNER_BOUND[prec]
    # the FP64 sweeps of the same handle are unchanged by the stored copies
    assert _rel(sol.apply_preconditioner(v).cpu().numpy(), zo) < 1e-11
    sol.close()


@pytest.mark.parametrize("case", [(3, 2, 6, 64, 1), (3, 3, 4, 135, 1), (2, 2, 4, 36, 2)], ids=_ids)
def test_inner_operator_parity(case):
    """FP32 operator (FP32 copies of J and M, FP32 input) against the FP64
    oracle: one product of (r + 2) m terms per row, bound 2^-17 relative to
    the largest entry."""
    irk = _irk()
    s, dim, N, m, nJ = case
    sy = _system(s, dim, N, m, nJ, seed=54)
    sol = irk.Solver(sy, irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="fp32",
                                     rtol=1e-8))
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    x = np.random.default_rng(10).standard_normal(P.N)
    y = sol.apply_operator_inner(x).cpu().numpy()
    yo = oracle.matvec(P, oracle.inverse(A), x)
    err = _rel(y, yo)
    _say("inner operator", case, f"rel err {err:.2e}")
    assert err < 2.0 ** -17
    sol.close()


@pytest.mark.parametrize("s,m", [(2, 16), (3, 64), (4, 9)])
def test_isolated_elements_coupled_is_exact(s, m):
    """r = 0: B is block diagonal over elements and the stage-coupled block
    ILU(0) of one element's s x s block matrix is its exact LU, so GMRES
    stops after one iteration at the dense solution."""
    irk = _irk()
    sy = dgsynth.make_system(61 + s, dgsynth.isolated_mesh(12), m, s, 0.2)
    sol = irk.Solver(sy, irk.Options(pc="coupled", rtol=1e-12))
    sol.factor()
    x, info = sol.solve(sy.rhs)
    A, _, _ = oracle.radau_iia(s)
    xd = np.linalg.solve(dense.dense_B(sy, np.linalg.inv(A)), sy.rhs)
    err = np.linalg.norm(x.cpu().numpy() - xd) / np.linalg.norm(xd)
    _say("isolated", s, m, "iters", info["iters"], f"err {err:.2e}")
    assert info["converged"] and info["iters"] == 1
    assert err <= 1e-12


# s = 2 Radau IIA: A^{-1} = [[3/2, 1/2], [-9/2, 5/2]], column-sum shifts
# alpha = (9/2, 1/2), written out from the exact rationals.
S2_AINV_DIAG = (1.5, 2.5)


@pytest.mark.parametrize("form", ["default", "streaming"])
@pytest.mark.parametrize("pc,alpha", [("uncoupled_shifted", (4.5, 0.5)), ("uncoupled", (0.0, 0.0))])
def test_tree_uncoupled_apply_is_exact(form, pc, alpha, monkeypatch):
    """Path in natural order: each stage's block ILU(0) is an exact LU, so the
    GPU's apply equals ((A^{-1}_kk + alpha_k) M - dt J_k)^{-1} v_k."""
    irk = _irk()
    if form == "streaming":
        monkeypatch.setenv("IRK_SWEEP_BIG", "1")
    sy = dgsynth.make_system(77, dgsynth.path_mesh(40), 16, 2, 0.4, nJ=2, permute=False)
    sol = irk.Solver(sy, irk.Options(pc=pc))
    sol.factor()
    v = np.random.default_rng(78).standard_normal(2 * sy.T * sy.m)
    z = sol.apply_preconditioner(v).cpu().numpy()
    n = sy.T * sy.m
    for k in range(2):
        Bk = (S2_AINV_DIAG[k] + alpha[k]) * dense.dense_M(sy) - sy.dt * dense.dense_J(sy, k)
        zk = np.linalg.solve(Bk, v[k * n:(k + 1) * n])
        assert _rel(z[k * n:(k + 1) * n], zk) < 1e-12
    sol.close()
