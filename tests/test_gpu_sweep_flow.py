"""The single-launch sweeps (every level of a direction in one launch, each
element waiting only for the neighbours it reads), on the GPU.

* Element-wise parity with the oracle's preconditioner apply for all three
  FP64 preconditioners and each form (prefetching, streaming, prefetching
  without the Jacobian columns), block sizes 6 to 135, 2D and 3D meshes;
  and bitwise equality with the level-per-launch kernel of the same form
  (both run the same arithmetic in the same order).
* Rows with more than 8 lower and upper neighbours (waits on flags read
  through the column index).
* Many applications in a row on one handle (the epochs keep growing, the
  flags are never reset) and interleaved handles.
* The inner (FP32 / BF16 / FP16-scaled) sweeps against the FP64 oracle.
* Whole solves and batched solves: same iterations and bitwise the same
  solution as with the level-per-launch sweeps; batch == solo.
* Chaining only the levels below a size (the others one launch per level,
  publishing their flags for the chained launch that follows): bitwise the
  same as no chaining, for several thresholds.
The choice is fixed per handle at set-up through IRK_SWEEP_FLOW (1: the
default form, 10 + form: that form; 0: level per launch) and
IRK_SWEEP_CHAIN (levels of fewer elements chained).
"""
import sys

import numpy as np
import pytest

import dgsynth
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOW_FORMS = {"prefetch": "11", "streaming": "10", "prefetch_lite": "12"}


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


def _solver(irk, sy, opts, monkeypatch, flow, big=None, chain="0"):
    monkeypatch.setenv("IRK_SWEEP_FLOW", flow)
    monkeypatch.setenv("IRK_SWEEP_CHAIN", chain)
    if big is not None:
        monkeypatch.setenv("IRK_SWEEP_BIG", big)
    else:
        monkeypatch.delenv("IRK_SWEEP_BIG", raising=False)
    sol = irk.Solver(sy, opts)
    sol.factor()
    return sol


CASES = [(2, 2, 8, 16, 1), (3, 2, 5, 9, 1), (4, 2, 4, 6, 4), (3, 3, 4, 20, 1),
         (3, 2, 6, 64, 1), (3, 3, 4, 135, 1), (2, 2, 5, 100, 2)]


@pytest.mark.parametrize("form", list(FLOW_FORMS))
@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted", "uncoupled"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_flow_parity(pc, case, form, monkeypatch):
    irk = _irk()
    s, dim, N, m, nJ = case
    _say("flow sweep", form, pc, case)
    sy = _system(s, dim, N, m, nJ)
    opts = irk.Options(pc=pc)
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(7).standard_normal(P.N)
    zo = oracle.pc_apply(P, A, pc, v)
    sol = _solver(irk, sy, opts, monkeypatch, FLOW_FORMS[form])
    z = sol.apply_preconditioner(v)
    assert _rel(z.cpu().numpy(), zo) < 1e-11
    # the level-per-launch kernel of the same form gives the same bits
    big = "1" if form != "prefetch" else str(1 << 30)
    ref = _solver(irk, sy, opts, monkeypatch, "0", big=big)
    if form == "prefetch_lite":
        monkeypatch.setenv("IRK_SWEEP_BIG_FORM", "2")
        ref.close()
        ref = _solver(irk, sy, opts, monkeypatch, "0", big="1")
    zr = ref.apply_preconditioner(v)
    assert torch.equal(z, zr)
    ref.close()
    sol.close()


def _bipartite(a, b):
    """Complete bipartite mesh K_{a,b} numbered leaves, hubs, leaves (each hub
    row has b//2 lower and b - b//2 upper blocks); triangle-free."""
    lo = b // 2
    hubs = list(range(lo, lo + a))
    leaves = [e for e in range(a + b) if e not in hubs]
    return [leaves if e in hubs else hubs for e in range(a + b)]


@pytest.mark.parametrize("form", ["prefetch", "streaming"])
@pytest.mark.parametrize("pc,s,m", [("coupled", 3, 12), ("uncoupled_shifted", 2, 16), ("coupled", 2, 64)])
def test_flow_rows_longer_than_record(form, pc, s, m, monkeypatch):
    irk = _irk()
    sy = dgsynth.make_system(91 + m, _bipartite(3, 20), m, s, 0.05, permute=False)
    sol = _solver(irk, sy, irk.Options(pc=pc), monkeypatch, FLOW_FORMS[form])
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(8).standard_normal(P.N)
    err = _rel(sol.apply_preconditioner(v).cpu().numpy(), oracle.pc_apply(P, A, pc, v))
    _say("flow long rows", form, pc, s, m, f"rel err {err:.2e}")
    assert err < 1e-11
    sol.close()


def test_flow_repeated_and_interleaved(monkeypatch):
    """Fifty applications alternating between two handles that share nothing
    but the process-wide epoch counter: every result equals the first."""
    irk = _irk()
    sa = _system(3, 2, 6, 16, seed=41)
    sb = _system(2, 3, 4, 20, seed=42)
    a = _solver(irk, sa, irk.Options(pc="coupled"), monkeypatch, "1")
    b = _solver(irk, sb, irk.Options(pc="uncoupled_shifted"), monkeypatch, "1")
    rng = np.random.default_rng(43)
    va = rng.standard_normal(3 * sa.T * sa.m)
    vb = rng.standard_normal(2 * sb.T * sb.m)
    za0 = a.apply_preconditioner(va).clone()
    zb0 = b.apply_preconditioner(vb).clone()
    for it in range(25):
        assert torch.equal(a.apply_preconditioner(va), za0), it
        assert torch.equal(b.apply_preconditioner(vb), zb0), it
    A, _, _ = oracle.radau_iia(3)
    assert _rel(za0.cpu().numpy(), oracle.pc_apply(oracle.Problem(sa), A, "coupled", va)) < 1e-11
    a.close()
    b.close()


INNER_BOUND = {"fp32": 2.0 ** -17, "bf16": 16 * 2.0 ** -8, "fp16s": 16 * 2.0 ** -11}


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16s"])
@pytest.mark.parametrize("pc,case", [("uncoupled_shifted", (3, 3, 4, 135, 1)),
                                     ("coupled", (3, 2, 6, 64, 1))],
                         ids=lambda v: v if isinstance(v, str) else _ids(v))
def test_flow_inner_parity(prec, pc, case, monkeypatch):
    """Reduced-precision sweeps (bounds as for the level-per-launch forms:
    storage unit roundoff times 16, 2^-17 for FP32)."""
    irk = _irk()
    s, dim, N, m, nJ = case
    sy = _system(s, dim, N, m, nJ, seed=53)
    opts = irk.Options(pc=pc, matvec_prec="fp32", factor_prec=prec, rtol=1e-8)
    sol = _solver(irk, sy, opts, monkeypatch, "1")
    A, _, _ = oracle.radau_iia(s)
    P = oracle.Problem(sy)
    v = np.random.default_rng(9).standard_normal(P.N)
    zo = oracle.pc_apply(P, A, pc, v)
    err = _rel(sol.apply_preconditioner_inner(v).cpu().numpy(), zo)
    _say("flow inner", prec, pc, case, f"rel err {err:.2e}")
    assert err < INNER_BOUND[prec]
    assert _rel(sol.apply_preconditioner(v).cpu().numpy(), zo) < 1e-11
    sol.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
def test_flow_solve_equals_level_solve(pc, monkeypatch):
    """A whole GMRES solve: same iterations, bitwise the same solution."""
    irk = _irk()
    sy = _system(3, 2, 10, 16, seed=44)
    opts = irk.Options(pc=pc, rtol=1e-10)
    ref = _solver(irk, sy, opts, monkeypatch, "0", big="1")   # streaming, level per launch
    xr, ir = ref.solve(sy.rhs)
    sol = _solver(irk, sy, opts, monkeypatch, "10")          # streaming, one launch
    x, info = sol.solve(sy.rhs)
    _say("flow solve", pc, info["iters"], ir["iters"])
    assert info["converged"] and info["iters"] == ir["iters"]
    assert torch.equal(x, xr)
    A, _, _ = oracle.radau_iia(3)
    r = sy.rhs - oracle.matvec(oracle.Problem(sy), oracle.inverse(A), x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(sy.rhs) <= 1e-10 * (1 + 1e-6)
    sol.close()
    ref.close()


@pytest.mark.parametrize("mode", ["flow", "chain"])
@pytest.mark.parametrize("pc,prec", [("coupled", "fp64"), ("uncoupled_shifted", "fp32")])
def test_flow_batch_equals_solo(pc, prec, mode, monkeypatch):
    """Uneven members (different block sizes, so different records per
    workgroup) merged into chained launches (flow: one form for every level;
    chain: every level chained in its own form); every member equals its
    solo solve bitwise."""
    irk = _irk()
    if mode == "flow":
        monkeypatch.setenv("IRK_SWEEP_FLOW", "1")
        monkeypatch.setenv("IRK_SWEEP_CHAIN", "0")
    else:
        monkeypatch.setenv("IRK_SWEEP_FLOW", "0")
        monkeypatch.setenv("IRK_SWEEP_CHAIN", str(1 << 30))
    specs = dgsynth.batch_specs(count=10, seed=3300, Nmin=4, Nmax=8, pmax=2)
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
    for q in range(len(systems)):
        xsolo, isolo = solo[q]
        assert infos[q]["converged"] and infos[q]["iters"] == isolo["iters"], (q, infos[q], isolo)
        assert torch.equal(xs[q], xsolo), q
    batch.close()
    for so in solvers:
        so.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
@pytest.mark.parametrize("case", [(3, 2, 12, 16, 1), (2, 3, 5, 20, 2), (3, 2, 8, 64, 1)], ids=_ids)
def test_chained_levels_equal_level_launches(pc, case, monkeypatch):
    """Levels below a threshold chained (the rest one launch per level):
    bitwise equal to no chaining, for thresholds that chain none, some and
    all levels; large levels in the streaming form (IRK_SWEEP_BIG) so that
    a sweep mixes forms and launch kinds."""
    irk = _irk()
    s, dim, N, m, nJ = case
    sy = _system(s, dim, N, m, nJ, seed=45)
    opts = irk.Options(pc=pc)
    v = np.random.default_rng(46).standard_normal(s * sy.T * sy.m)
    ref = _solver(irk, sy, opts, monkeypatch, "0", big="12", chain="0")
    zr = ref.apply_preconditioner(v)
    A, _, _ = oracle.radau_iia(s)
    assert _rel(zr.cpu().numpy(), oracle.pc_apply(oracle.Problem(sy), A, pc, v)) < 1e-11
    for chain in ("8", "12", "20", str(1 << 30)):
        sol = _solver(irk, sy, opts, monkeypatch, "0", big="12", chain=chain)
        z = sol.apply_preconditioner(v)
        _say("chained", pc, case, chain)
        assert torch.equal(z, zr), chain
        for _ in range(3):
            assert torch.equal(sol.apply_preconditioner(v), zr), chain
        sol.close()
    x, info = ref.solve(sy.rhs)
    sol = _solver(irk, sy, opts, monkeypatch, "0", big="12", chain="16")
    x2, info2 = sol.solve(sy.rhs)
    assert info2["iters"] == info["iters"] and torch.equal(x, x2)
    sol.close()
    ref.close()


@pytest.mark.parametrize("pc", ["coupled", "uncoupled_shifted"])
@pytest.mark.parametrize("case", [(3, 2, 12, 16, 1), (2, 3, 5, 20, 2), (3, 2, 8, 64, 1)], ids=_ids)
def test_split_streaming_levels(pc, case, monkeypatch):
    """Streaming levels below IRK_SWEEP_SPLIT at half the elements per
    workgroup: element-wise parity with the oracle; chained launches (whose
    workgroups then differ in elements per workgroup) bitwise equal to one
    launch per level with the same split; a solve converges to the same
    iterations as without the split."""
    irk = _irk()
    s, dim, N, m, nJ = case
    sy = _system(s, dim, N, m, nJ, seed=47)
    opts = irk.Options(pc=pc)
    v = np.random.default_rng(48).standard_normal(s * sy.T * sy.m)
    A, _, _ = oracle.radau_iia(s)
    zo = oracle.pc_apply(oracle.Problem(sy), A, pc, v)
    lv = irk.level_schedule(sy.row_ptr, sy.col_idx)
    sizes = sorted({int(b - a) for off in (lv[1], lv[3]) for a, b in zip(off[:-1], off[1:])})
    _say("split", pc, case, "level sizes", sizes)
    plain = _solver(irk, sy, opts, monkeypatch, "0", big="8", chain="0")
    x0, info0 = plain.solve(sy.rhs)
    plain.close()
    for split in (str(sizes[len(sizes) // 2] + 1), str(1 << 30)):
        monkeypatch.setenv("IRK_SWEEP_SPLIT", split)
        ref = _solver(irk, sy, opts, monkeypatch, "0", big="8", chain="0")
        zr = ref.apply_preconditioner(v)
        assert _rel(zr.cpu().numpy(), zo) < 1e-11, split
        sol = _solver(irk, sy, opts, monkeypatch, "0", big="8", chain=str(1 << 30))
        _say("split chained", pc, case, split)
        for _ in range(3):
            assert torch.equal(sol.apply_preconditioner(v), zr), split
        x, info = sol.solve(sy.rhs)
        assert info["converged"] and info["iters"] == info0["iters"]
        assert float(torch.linalg.norm(x - x0) / torch.linalg.norm(x0)) < 1e-11
        sol.close()
        ref.close()
