"""Failure handling through the C ABI on the GPU: every error is a status,
never an abort, and the device keeps working afterwards."""
import numpy as np
import pytest

import dgsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def test_singular_pivot_names_the_element():
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    bad = int(np.flatnonzero(sy.col_idx == 0)[0])    # the (0, 0) block
    i = 0
    sy.M[i] = 0.0
    sy.J[:, bad] = 0.0
    sol = irk.Solver(sy, irk.Options(pc="uncoupled"))
    with pytest.raises(irk.IrkError) as ei:
        sol.factor()
    assert ei.value.status == irk.ERR_SINGULAR
    assert "element 0" in str(ei.value)
    with pytest.raises(irk.IrkError) as ei:
        sol.solve(sy.rhs)                 # solve before a successful factorization
    assert ei.value.status == irk.ERR_STATE


def test_nonfinite_rhs_and_zero_rhs():
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    sol = irk.Solver(sy, irk.Options(pc="coupled"))
    sol.factor()
    r = sy.rhs.copy()
    r[5] = np.nan
    x, info = sol.solve(r, raise_on_error=False)
    assert info["status"] == irk.ERR_NONFINITE
    x, info = sol.solve(np.zeros_like(sy.rhs))
    assert info["converged"] and not torch.any(x)
    # still usable afterwards
    x, info = sol.solve(sy.rhs)
    assert info["converged"]


def test_max_iters_returns_noconv_and_iterate():
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    sol = irk.Solver(sy, irk.Options(pc="none", max_iters=3, rtol=1e-12))
    sol.factor()
    x, info = sol.solve(sy.rhs)
    assert info["status"] == irk.ERR_NOCONV and not info["converged"]
    assert info["iters"] == 3 and 0 < info["rel_res_true"] < 1
    assert torch.any(x)


def test_nonfinite_jacobian_is_reported():
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    sy.J[0, 3, 2, 2] = np.inf
    sol = irk.Solver(sy, irk.Options(pc="coupled"))
    with pytest.raises(irk.IrkError) as ei:
        sol.factor()
        sol.solve(sy.rhs)
    assert ei.value.status in (irk.ERR_SINGULAR, irk.ERR_NONFINITE)

