"""Batched solves: many independent systems of uneven size, degree, stage
count and time step iterated in the same kernel launches.  Every member's
result must be the same as its solo solve (bitwise: the per-system
arithmetic and reduction order do not depend on the batch), and agree with
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


def _specs(count, seed, Nmax=8, pmax=2):
    return dgsynth.batch_specs(count=count, seed=seed, Nmin=4, Nmax=Nmax, pmax=pmax)


@pytest.mark.parametrize("pc,prec", [("coupled", "fp64"), ("uncoupled_shifted", "fp64"),
                                     ("uncoupled_shifted", "fp32"), ("coupled", "bf16")])
def test_batch_equals_solo(pc, prec):
    irk = _irk()
    specs = _specs(12, 3100)
    systems = [sp.build() for sp in specs]
    mixed = prec != "fp64"
    opts = irk.Options(pc=pc, rtol=1e-8 if mixed else 1e-10,
                       matvec_prec="fp32" if mixed else "fp64", factor_prec=prec)
    solvers = []
    for sy in systems:
        so = irk.Solver(sy, opts)
        so.factor()
        solvers.append(so)
    solo = [so.solve(sy.rhs) for so, sy in zip(solvers, systems)]
    batch = irk.Batch(capacity=16, max_elements=sum(sy.T for sy in systems))
    xs, infos, st = irk.solve_batched(batch, solvers, [sy.rhs for sy in systems])
    assert st == irk.OK
    for q, sy in enumerate(systems):
        xsolo, isolo = solo[q]
        assert infos[q]["converged"] and infos[q]["iters"] == isolo["iters"], (q, infos[q], isolo)
        assert torch.equal(xs[q], xsolo), q
    # spot-check two members against the oracle
    for q in (0, len(systems) - 1):
        sy = systems[q]
        A, _, _ = oracle.radau_iia(sy.s)
        P = oracle.Problem(sy)
        r = sy.rhs - oracle.matvec(P, oracle.inverse(A), xs[q].cpu().numpy())
        assert np.linalg.norm(r) / np.linalg.norm(sy.rhs) <= (1e-8 if mixed else 1e-10) * (1 + 1e-6)
    batch.close()


def test_continuous_admission():
    """Members join while others iterate; every result equals its solo solve."""
    irk = _irk()
    specs = _specs(10, 3200)
    systems = [sp.build() for sp in specs]
    opts = irk.Options(pc="uncoupled_shifted", rtol=1e-10, restart=8)
    solvers = []
    for sy in systems:
        so = irk.Solver(sy, opts)
        so.factor()
        solvers.append(so)
    solo = [so.solve(sy.rhs)[0] for so, sy in zip(solvers, systems)]
    batch = irk.Batch(capacity=4, max_elements=sum(sy.T for sy in systems))
    done = {}
    nxt = 0
    rounds = 0
    while len(done) < len(systems):
        while nxt < len(systems) and batch.admit(solvers[nxt], systems[nxt].rhs, tag=nxt) == irk.OK:
            nxt += 1
        batch.advance(1)
        for tag, x, info in batch.retire():
            assert info["converged"]
            done[tag] = x
        rounds += 1
        assert rounds < 500
    for q in range(len(systems)):
        assert torch.equal(done[q], solo[q]), q
    batch.close()


def test_batch_rejects_mixed_kinds():
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    a = irk.Solver(sy, irk.Options(pc="coupled"))
    b = irk.Solver(sy, irk.Options(pc="uncoupled_shifted"))
    a.factor(); b.factor()
    batch = irk.Batch(capacity=2, max_elements=1000)
    assert batch.admit(a, sy.rhs, tag=0) == irk.OK
    assert batch.admit(b, sy.rhs, tag=1) == irk.ERR_ARG
    assert batch.admit(a, sy.rhs, tag=2) == irk.ERR_ARG    # same handle twice
    batch.advance(100)
    out = batch.retire()
    assert len(out) == 1 and out[0][2]["converged"]
    batch.close()


@pytest.mark.parametrize("pc,prec", [("coupled", "fp64"), ("uncoupled_shifted", "fp32")])
def test_batch_mixed_launch_shapes(pc, prec, monkeypatch):
    """Members with blocks of 16 to 100 rows and levels above and below the
    size at which a sweep level switches from the prefetching to the
    streaming form (lowered here so that small meshes cross it): launches
    group members by elements per workgroup and pad each member to whole
    workgroups; every member still equals its solo solve bitwise."""
    irk = _irk()
    monkeypatch.setenv("IRK_SWEEP_BIG", "12")
    specs = dgsynth.batch_specs(count=8, seed=3300, Nmin=6, Nmax=12, pmax=4)
    systems = [sp.build() for sp in specs]
    assert len({sy.m for sy in systems}) >= 3
    mixed = prec != "fp64"
    opts = irk.Options(pc=pc, rtol=1e-8 if mixed else 1e-10,
                       matvec_prec="fp32" if mixed else "fp64", factor_prec=prec)
    solvers = []
    for sy in systems:
        so = irk.Solver(sy, opts)
        so.factor()
        solvers.append(so)
    solo = [so.solve(sy.rhs) for so, sy in zip(solvers, systems)]
    batch = irk.Batch(capacity=8, max_elements=sum(sy.T for sy in systems))
    xs, infos, st = irk.solve_batched(batch, solvers, [sy.rhs for sy in systems])
    assert st == irk.OK
    for q, sy in enumerate(systems):
        xsolo, isolo = solo[q]
        assert infos[q]["converged"] and infos[q]["iters"] == isolo["iters"], (q, infos[q], isolo)
        assert torch.equal(xs[q], xsolo), q
        A, _, _ = oracle.radau_iia(sy.s)
        r = sy.rhs - oracle.matvec(oracle.Problem(sy), oracle.inverse(A), xs[q].cpu().numpy())
        assert np.linalg.norm(r) / np.linalg.norm(sy.rhs) <= (1e-8 if mixed else 1e-10) * 1.01
    batch.close()
