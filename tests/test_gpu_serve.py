"""Serving: requests of different sizes arrive while others iterate; each
served result equals the result of solving the same system alone (bitwise),
re-used operators are not set up again, and every request completes."""
import numpy as np
import pytest

import dgsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_served_results_equal_solo():
    import paper_1701_07181_amd as irk
    from paper_1701_07181_amd.serve import Request, Server, latency_stats

    stream = dgsynth.serve_requests(16, seed=4100, N2max=10, N3max=4, reuse_frac=0.3)
    opts = irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="fp32",
                       rtol=1e-8, restart=10)
    systems = {}
    reqs = []
    for rid, (spec, reuse_of, rhs_seed) in enumerate(stream):
        op = rid if reuse_of is None else reuse_of
        if op not in systems:
            sy = spec.build()
            sy.J = torch.from_numpy(sy.J).cuda()
            sy.M = torch.from_numpy(sy.M).cuda()
            systems[op] = sy
        sy = systems[op]
        rhs = torch.from_numpy(dgsynth.fresh_rhs(rhs_seed, sy.s, sy.T, sy.m)).cuda()
        reqs.append(Request(rid, op, sy, rhs, arrival=0.002 * rid))
    srv = Server(opts, capacity=4, max_elements=1 << 16, budget_bytes=8 << 30)
    results = srv.run(reqs)
    stats = latency_stats(results)
    srv.close()
    print(stats, flush=True)
    assert len(results) == len(reqs) and stats["converged"] == len(reqs)
    assert stats["reused"] >= 1
    for r in results:
        sy = systems[r.op_id]
        solo = irk.Solver(sy, opts)
        solo.factor()
        x, info = solo.solve(reqs[r.rid].rhs)
        assert info["iters"] == r.info["iters"], (r.rid, info["iters"], r.info["iters"])
        assert torch.equal(x, r.x), r.rid
        solo.close()


def test_served_results_with_evictions():
    """A pool smaller than the operators' workspaces together: idle
    factorizations are evicted and prepared again when asked for; results
    still equal solo solves."""
    import paper_1701_07181_amd as irk
    from paper_1701_07181_amd.serve import Request, Server, latency_stats

    stream = dgsynth.serve_requests(12, seed=4200, N2max=10, N3max=4, reuse_frac=0.4)
    opts = irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="fp32",
                       rtol=1e-8, restart=10)
    systems, reqs = {}, []
    for rid, (spec, reuse_of, rhs_seed) in enumerate(stream):
        op = rid if reuse_of is None else reuse_of
        if op not in systems:
            sy = spec.build()
            sy.J = torch.from_numpy(sy.J).cuda()
            sy.M = torch.from_numpy(sy.M).cuda()
            systems[op] = sy
        sy = systems[op]
        rhs = torch.from_numpy(dgsynth.fresh_rhs(rhs_seed, sy.s, sy.T, sy.m)).cuda()
        reqs.append(Request(rid, op, sy, rhs, arrival=0.003 * rid))
    sizes = []
    for sy in systems.values():
        so = irk.Solver(sy, opts)
        sizes.append(so.workspace_bytes)
        so.close()
    rounded = [-(-n // 256) * 256 for n in sizes]
    budget = max(max(rounded) + 1024, sum(rounded) // 2)     # every operator fits, not all at once
    assert budget < sum(rounded)
    print("operators", len(systems), "largest workspace", max(sizes), "pool", budget, flush=True)
    srv = Server(opts, capacity=2, max_elements=1 << 16, budget_bytes=budget)
    results = srv.run(reqs)
    stats = latency_stats(results)
    evictions = srv.evictions
    assert srv.pool.free_bytes() + sum(-(-n // 256) * 256 for _, n in srv.range_of.values()) == srv.pool.size
    srv.close()
    print(stats, "evictions", evictions, flush=True)
    assert len(results) == len(reqs) and stats["converged"] == len(reqs)
    assert evictions >= 1
    for r in results:
        solo = irk.Solver(systems[r.op_id], opts)
        solo.factor()
        x, info = solo.solve(reqs[r.rid].rhs)
        assert info["iters"] == r.info["iters"], (r.rid, info["iters"], r.info["iters"])
        assert torch.equal(x, r.x), r.rid
        solo.close()


def test_singular_operator_surfaces_and_frees_its_range():
    """A request whose operator has a singular pivot ends the run with the
    library's error; the pool gets the operator's range back."""
    import paper_1701_07181_amd as irk
    from paper_1701_07181_amd.serve import Request, Server

    sy = dgsynth.config_system("cfg0")
    col = int(np.flatnonzero(sy.col_idx == 0)[0])     # the (0, 0) block
    sy.M[0] = 0.0
    sy.J[:, col] = 0.0
    sy.J = torch.from_numpy(sy.J).cuda()
    sy.M = torch.from_numpy(sy.M).cuda()
    rhs = torch.from_numpy(sy.rhs).cuda()
    srv = Server(irk.Options(pc="uncoupled"), capacity=2, max_elements=1 << 12, budget_bytes=1 << 30)
    with pytest.raises(irk.IrkError) as ei:
        srv.run([Request(0, 0, sy, rhs, arrival=0.0)])
    assert ei.value.status == irk.ERR_SINGULAR
    assert srv.pool.free_bytes() == srv.pool.size and not srv.resident
    srv.close()
