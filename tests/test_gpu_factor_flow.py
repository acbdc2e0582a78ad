"""The dependency-driven factorization (the uncoupled forms, and the coupled
form with m <= 64: runs of consecutive wavefronts in one launch, each task
waiting only for the tasks it reads), synchronous and asynchronous, all
three preconditioner forms, on the GPU, against the factorization with one
launch per wavefront (IRK_FACTOR_FLOW=0 at set-up).

* Bitwise the same factors (pivot inverses and stored cross blocks) as the
  wavefront-per-launch factorization: s = 2, 3, 4, m from 6 to 64 (both
  forms of the four-wave block routines: all tiles for m > 56, masked
  tiles below) and m = 100, 135 (the eight-wave routines, two and three
  row groups; the coupled form keeps one launch per wavefront there),
  2D and 3D meshes, shared and per-stage Jacobians.
* Repeated factorizations on one handle (the epochs grow, the flags are
  never reset) and a value update between them.
* The solve after it: the same iterations and bitwise the same solution
  as after the synchronous factorization.
* A singular pivot is still reported (asynchronous: by the solve).
"""
import numpy as np
import pytest

import dgsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _system(s, dim, N, m, nJ=1, seed=61, dt=0.1):
    mesh = dgsynth.grid2d(N) if dim == 2 else dgsynth.grid3d(N)
    return dgsynth.make_system(seed, mesh, m, s, dt, nJ=nJ)


def _ids(c):
    return "s%d_%dd_N%d_m%d_nJ%d" % c


CASES = [(3, 2, 24, 64, 1), (2, 2, 16, 40, 1), (4, 2, 8, 16, 1), (3, 3, 5, 20, 1), (3, 2, 12, 6, 3),
         (3, 2, 32, 64, 1), (3, 2, 8, 100, 1), (2, 2, 6, 135, 2)]


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_flow_factors_equal_wavefront_factors(case, pc, monkeypatch):
    irk = _irk()
    s, dim, N, m, nJ = case
    print("factor flow", pc, case, flush=True)
    sy = _system(s, dim, N, m, nJ)
    opts = irk.Options(pc=pc)
    monkeypatch.setenv("IRK_FACTOR_FLOW", "0")
    ref = irk.Solver(sy, opts)
    ref.factor()
    pr, cr = ref.export_factors(cross=True)
    xr, ir = ref.solve(sy.rhs)
    monkeypatch.setenv("IRK_FACTOR_FLOW", "1")
    sol = irk.Solver(sy, opts)
    for rep in range(3):
        sol.factor(wait=rep == 1)
        p, c = sol.export_factors(cross=True)
        assert torch.equal(p, pr) and torch.equal(c, cr), rep
    sol.factor(wait=False)
    x, i = sol.solve(sy.rhs)
    assert i["converged"] and i["iters"] == ir["iters"] and torch.equal(x, xr)
    x, i = sol.solve(sy.rhs)          # (a solve with the same factors)
    assert i["iters"] == ir["iters"] and torch.equal(x, xr)
    # a value update between two factorizations
    sy2 = _system(s, dim, N, m, nJ, seed=62, dt=0.3)
    for h in (ref, sol):
        h.update_values(sy2.J, sy2.M, 0.3)
    ref.factor()
    sol.factor(wait=False)
    p2, c2 = sol.export_factors(cross=True)
    pr2, cr2 = ref.export_factors(cross=True)
    assert torch.equal(p2, pr2) and torch.equal(c2, cr2)
    ref.close()
    sol.close()


def test_flow_factor_reports_singular(monkeypatch):
    irk = _irk()
    monkeypatch.setenv("IRK_FACTOR_FLOW", "1")
    sy = dgsynth.config_system("cfg0")
    bad = int(np.flatnonzero(sy.col_idx == 0)[0])
    sy.M[0] = 0.0
    sy.J[:, bad] = 0.0
    sol = irk.Solver(sy, irk.Options(pc="coupled"))
    sol.factor(wait=False)
    x, info = sol.solve(sy.rhs, raise_on_error=False)
    assert info["status"] == irk.ERR_SINGULAR
    with pytest.raises(irk.IrkError) as ei:
        sol.factor()
    assert ei.value.status == irk.ERR_SINGULAR
    sol.close()
