"""The allocation-free batched solve (irk_solve_batched_noalloc) against the
batched solve with a caller-provided batch workspace (irk_solve_batched):
the same kernels on the same data, so the solutions must agree bit for bit
and the iteration counts exactly.  Two calls in a row, the second with a
smaller input (fewer and smaller systems), share the library's static
device array; requests beyond its limits are refused before any work."""
import numpy as np
import pytest

import dgsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _systems(specs):
    out = []
    for (dim, N, m, s, dt, seed) in specs:
        mesh = dgsynth.grid2d(N) if dim == 2 else dgsynth.grid3d(N)
        out.append(dgsynth.make_system(seed, mesh, m, s, dt))
    return out


FIRST = [(2, 8, 16, 2, 0.1, 1), (2, 12, 36, 3, 0.3, 2), (2, 6, 64, 3, 0.05, 3),
         (3, 4, 20, 2, 0.2, 4), (2, 16, 9, 4, 0.5, 5)]
SECOND = [(2, 5, 16, 3, 0.2, 11), (2, 4, 9, 2, 0.7, 12)]


@pytest.mark.parametrize("pc,prec", [("coupled", "fp64"), ("uncoupled_shifted", "fp32")])
def test_noalloc_equals_batched(pc, prec):
    irk = _irk()
    opts = irk.Options(pc=pc, matvec_prec=prec, factor_prec=prec,
                       rtol=1e-10 if prec == "fp64" else 1e-8)
    for call, specs in enumerate((FIRST, SECOND)):
        sys_ = _systems(specs)
        solvers = [irk.Solver(sy, opts) for sy in sys_]
        for so in solvers:
            so.factor()
        rhs = [so._vec(sy.rhs) for so, sy in zip(solvers, sys_)]
        # reference: the batch with its own workspace
        ref_batch = irk.Batch(len(solvers), sum(sy.T for sy in sys_))
        xr, ir, str_ = irk.solve_batched(ref_batch, solvers, rhs)
        assert str_ == irk.OK
        # the allocation-free call
        xs = [torch.zeros(so.N, dtype=torch.float64, device=so.device) for so in solvers]
        torch.cuda.synchronize()
        infos, st = irk.solve_batched_noalloc(solvers, rhs, xs)
        torch.cuda.synchronize()
        print(f"call {call}: {len(solvers)} systems, status {st}, iters "
              f"{[i['iters'] for i in infos]}", flush=True)
        assert st == irk.OK
        for q in range(len(solvers)):
            assert infos[q]["converged"] and infos[q]["iters"] == ir[q]["iters"]
            assert torch.equal(xs[q], xr[q]), (call, q)
        ref_batch.close()
        for so in solvers:
            so.close()


def test_noalloc_rejects_beyond_limits():
    irk = _irk()
    sy = dgsynth.make_system(21, dgsynth.grid2d(4), 4, 2, 0.1)
    so = irk.Solver(sy, irk.Options(pc="coupled"))
    so.factor()
    rhs = so._vec(sy.rhs)
    xs = [torch.zeros(so.N, dtype=torch.float64, device=so.device) for _ in range(65)]
    # 65 members (the same handle repeated: refused on the count first)
    infos, st = irk.solve_batched_noalloc([so] * 65, [rhs] * 65, xs)
    assert st == irk.ERR_ARG
    big = dgsynth.make_system(22, dgsynth.grid2d(182), 4, 2, 0.1)   # 33124 elements
    so2 = irk.Solver(big, irk.Options(pc="coupled"))
    x2 = torch.zeros(so2.N, dtype=torch.float64, device=so2.device)
    infos, st = irk.solve_batched_noalloc([so2], [so2._vec(big.rhs)], [x2])
    assert st == irk.ERR_ARG
    so.close()
    so2.close()
