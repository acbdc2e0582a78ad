"""Autotuned launch shapes (irk_autotune): the timed choice is applied to the
handle and stored per problem class; solves with the chosen shapes match
the default-shape solve (same iterations, FP64 results to 1e-12: only the
matvec's partial sums may combine in another order), batched members with
tuned shapes still equal their solo solves bitwise, and results agree with
the oracle."""
import numpy as np
import pytest

import dgsynth
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _true_res(sy, x):
    A, _, _ = oracle.radau_iia(sy.s)
    P = oracle.Problem(sy)
    r = sy.rhs - oracle.matvec(P, oracle.inverse(A), x)
    return np.linalg.norm(r) / np.linalg.norm(sy.rhs)


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
def test_autotune_fp64(pc):
    irk = _irk()
    print("autotune fp64", pc, flush=True)
    sy = dgsynth.config_system("cfg1", N=12)
    a = irk.Solver(sy, irk.Options(pc=pc, rtol=1e-10))
    a.factor()
    x0, i0 = a.solve(sy.rhs)
    info = a.autotune(retime=True)
    assert info["from_cache"] == 0 and info["matvec_teams"] in (1, 2, 4, 8)
    assert info["sweep_teams"] >= 1 and info["sweep_big_min"] >= 1
    assert info["matvec_us"] > 0 and info["sweep_us"] > 0
    x1, i1 = a.solve(sy.rhs)
    assert i1["converged"] and i1["iters"] == i0["iters"]
    assert float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)) < 1e-12
    assert _true_res(sy, x1.cpu().numpy()) <= 1e-10 * 1.01
    # a second handle of the same class takes the stored choice
    b = irk.Solver(sy, irk.Options(pc=pc, rtol=1e-10))
    b.factor()
    info2 = b.autotune()
    assert info2["from_cache"] == 1
    for k in ("matvec_teams", "sweep_big_min", "sweep_teams"):
        assert info2[k] == info[k]
    x2, i2 = b.solve(sy.rhs)
    assert torch.equal(x2, x1) and i2["iters"] == i1["iters"]
    a.close()
    b.close()


def test_autotune_mixed():
    irk = _irk()
    print("autotune mixed", flush=True)
    sy = dgsynth.make_system(77, dgsynth.grid3d(4), 135, 3, 0.5)
    so = irk.Solver(sy, irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="bf16",
                                    rtol=1e-8))
    so.factor()
    info = so.autotune(retime=True)
    assert info["from_cache"] == 0
    x, i = so.solve(sy.rhs)
    assert i["converged"]
    assert _true_res(sy, x.cpu().numpy()) <= 1e-8 * 1.01
    so.close()


def test_autotune_batch_equals_solo():
    irk = _irk()
    print("autotune batch", flush=True)
    specs = dgsynth.batch_specs(count=8, seed=3300, Nmin=4, Nmax=8, pmax=2)
    systems = [sp.build() for sp in specs]
    opts = irk.Options(pc="uncoupled_shifted", rtol=1e-8, matvec_prec="fp32", factor_prec="fp32")
    solvers = []
    for sy in systems:
        so = irk.Solver(sy, opts)
        so.factor()
        so.autotune(retime=True)
        solvers.append(so)
    solo = [so.solve(sy.rhs) for so, sy in zip(solvers, systems)]
    batch = irk.Batch(capacity=8, max_elements=sum(sy.T for sy in systems))
    xs, infos, st = irk.solve_batched(batch, solvers, [sy.rhs for sy in systems])
    assert st == irk.OK
    for q in range(len(systems)):
        assert infos[q]["iters"] == solo[q][1]["iters"], q
        assert torch.equal(xs[q], solo[q][0]), q
    batch.close()
    for so in solvers:
        so.close()
