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



def test_async_factor_reports_singular_at_the_solve():
    """irk_factor_ilu_async returns at once; the singular pivot comes back
    from the solve, with the element, and the handle is then not factored."""
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    bad = int(np.flatnonzero(sy.col_idx == 0)[0])
    sy.M[0] = 0.0
    sy.J[:, bad] = 0.0
    sol = irk.Solver(sy, irk.Options(pc="uncoupled"))
    sol.factor(wait=False)
    x, info = sol.solve(sy.rhs, raise_on_error=False)
    assert info["status"] == irk.ERR_SINGULAR
    with pytest.raises(irk.IrkError) as ei:
        sol.solve(sy.rhs)
    assert ei.value.status == irk.ERR_STATE
    # the same through a call that waits for the stream first
    sol.factor(wait=False)
    with pytest.raises(irk.IrkError) as ei:
        sol.apply_preconditioner(sy.rhs)
    assert ei.value.status == irk.ERR_SINGULAR


@pytest.mark.parametrize("chain", ["none", "all"])
@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
def test_async_factor_overlapped_initial_residual(pc, chain, monkeypatch):
    """An asynchronous factorization runs on a second stream; the initial
    residual of the solve that follows runs beside its last wavefronts, and
    the first forward sweep's first launch group (one level, or the chained
    run of streaming levels) once the factors of its levels are final:
    bitwise the same solution as after a synchronous factorization, on a
    mesh whose factorization runs many wavefronts, also when the solve's
    zero initial guess is written (in the handle's stream order, after the
    factorization was enqueued) into memory that held the previous solution;
    a zero right-hand side right after an asynchronous factorization; a
    value update right after one; solves that follow with the same
    factors."""
    irk = _irk()
    print("async overlap", pc, chain, flush=True)
    if chain == "all":
        monkeypatch.setenv("IRK_SWEEP_CHAIN", str(1 << 30))
        monkeypatch.setenv("IRK_SWEEP_BIG", "40")
    sy = dgsynth.config_system("cfg1", N=24)
    a = irk.Solver(sy, irk.Options(pc=pc))
    b = irk.Solver(sy, irk.Options(pc=pc))
    a.factor()
    xa, ia = a.solve(sy.rhs)
    for _ in range(3):
        b.factor(wait=False)
        xb, ib = b.solve(sy.rhs)
        assert ib["converged"] and ib["iters"] == ia["iters"] and torch.equal(xb, xa)
        assert ib["ms_factor"] > 0
        del xb          # (its memory may become the next solve's x)
    b.factor(wait=False)
    b.update_values(sy.J, sy.M, sy.dt)
    b.factor(wait=False)
    xb, ib = b.solve(sy.rhs)
    assert ib["iters"] == ia["iters"] and torch.equal(xb, xa)
    b.factor(wait=False)
    x0, i0 = b.solve(np.zeros_like(sy.rhs))
    assert i0["converged"] and int(torch.count_nonzero(x0)) == 0
    xb, ib = b.solve(sy.rhs)
    assert ib["iters"] == ia["iters"] and torch.equal(xb, xa)
    a.close()
    b.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
def test_async_factor_equals_sync(pc):
    """Same factors, same solve, bitwise, with and without waiting; a value
    update between two asynchronous factorizations is honoured."""
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    a = irk.Solver(sy, irk.Options(pc=pc))
    b = irk.Solver(sy, irk.Options(pc=pc))
    a.factor()
    xa, ia = a.solve(sy.rhs)
    b.factor(wait=False)
    xb, ib = b.solve(sy.rhs)
    assert ia["iters"] == ib["iters"] and torch.equal(xa, xb)
    assert ib["ms_factor"] > 0
    z = b.apply_preconditioner(sy.rhs)
    assert torch.equal(z, a.apply_preconditioner(sy.rhs))
    sy2 = dgsynth.config_system("cfg0", dt=0.3)
    for s_ in (a, b):
        s_.update_values(sy2.J, sy2.M, 0.3)
    a.factor()
    b.factor(wait=False)
    b.factor(wait=False)
    xa, ia = a.solve(sy.rhs)
    xb, ib = b.solve(sy.rhs)
    assert ia["iters"] == ib["iters"] and torch.equal(xa, xb)
    a.close()
    b.close()
