"""Batched factorization (irk_factor_batched): level l of many handles in the
same launches gives the same factors as factoring each handle alone
(bitwise: the same kernels do the same work per element), for handles of
every kernel class, preconditioner form and precision scheme; a singular
pivot is reported for its own handle only; groups larger than the batch are
split."""
import numpy as np
import pytest

import dgsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _specs():
    S = dgsynth.Spec
    return [S(2, 5, 1, 4, 3, 0.1, (8100, 0)),      # m = 16
            S(2, 6, 2, 4, 2, 0.5, (8100, 1)),      # m = 36
            S(2, 4, 3, 4, 4, 0.05, (8100, 2)),     # m = 64
            S(2, 4, 4, 4, 3, 0.2, (8100, 3)),      # m = 100
            S(3, 4, 2, 5, 2, 0.3, (8100, 4)),      # m = 135
            S(2, 7, 1, 4, 2, 1.0, (8100, 5))]      # m = 16


OPTS = {
    "coupled": dict(pc="coupled"),
    "uncoupled_shifted": dict(pc="uncoupled_shifted"),
    "uncoupled": dict(pc="uncoupled"),
    "mixed_bf16": dict(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="bf16", rtol=1e-8),
}


def _pair(sy, opts):
    irk = _irk()
    return irk.Solver(sy, irk.Options(**opts)), irk.Solver(sy, irk.Options(**opts))


@pytest.mark.parametrize("form", list(OPTS))
def test_batched_factors_equal_solo(form):
    irk = _irk()
    systems = [sp.build() for sp in _specs()]
    pairs = [_pair(sy, OPTS[form]) for sy in systems]
    elems = sum(sy.T for sy in systems)
    batch = irk.Batch(len(systems), elems)
    sts = irk.factor_batched(batch, [a for a, _ in pairs])
    assert sts == [irk.OK] * len(systems)
    for (a, b), sy in zip(pairs, systems):
        b.factor()
        coupled = form == "coupled"
        fa, fb = a.export_factors(cross=coupled), b.export_factors(cross=coupled)
        if coupled:
            assert torch.equal(fa[0], fb[0]) and torch.equal(fa[1], fb[1]), sy.name
        else:
            assert torch.equal(fa, fb), sy.name
        xa, ia = a.solve(sy.rhs)
        xb, ib = b.solve(sy.rhs)
        assert ia["converged"] and ia["iters"] == ib["iters"] and torch.equal(xa, xb), sy.name
    for a, b in pairs:
        a.close(); b.close()
    batch.close()


def test_batched_factor_mixed_forms_and_groups():
    """Handles of different forms, block classes and Jacobian sharing in one
    call, in a batch of capacity 2 (four groups)."""
    irk = _irk()
    systems = [sp.build() for sp in _specs()] + [dgsynth.config_system("cfg0", nJ=2)]
    forms = list(OPTS) + ["coupled", "uncoupled", "coupled"]     # the last one: J per stage
    pairs = [_pair(sy, OPTS[f]) for sy, f in zip(systems, forms)]
    batch = irk.Batch(2, max(sy.T for sy in systems) * 2)
    irk.factor_batched(batch, [a for a, _ in pairs])
    for (a, b), f in zip(pairs, forms):
        b.factor()
        assert torch.equal(a.export_factors(), b.export_factors()), f
    for a, b in pairs:
        a.close(); b.close()
    batch.close()


def test_batched_factor_singular_is_per_handle():
    irk = _irk()
    bad_sy = dgsynth.config_system("cfg0")
    col = int(np.flatnonzero(bad_sy.col_idx == 0)[0])     # the (0, 0) block
    bad_sy.M[0] = 0.0
    bad_sy.J[:, col] = 0.0
    good_sy = dgsynth.config_system("cfg0")
    opts = irk.Options(pc="uncoupled")
    good, bad, good2 = irk.Solver(good_sy, opts), irk.Solver(bad_sy, opts), irk.Solver(good_sy, opts)
    batch = irk.Batch(4, 3 * good_sy.T)
    with pytest.raises(irk.IrkError) as ei:
        irk.factor_batched(batch, [good, bad, good2])
    assert ei.value.status == irk.ERR_SINGULAR
    assert "system 1, element 0" in str(ei.value)
    assert good.factored and good2.factored and not bad.factored
    x, info = good.solve(good_sy.rhs)
    assert info["converged"]
    with pytest.raises(irk.IrkError) as ei:
        bad.solve(bad_sy.rhs)
    assert ei.value.status == irk.ERR_STATE
    # the flags are cleared by the next call: the good handles factor again
    irk.factor_batched(batch, [good, good2])
    for s in (good, bad, good2):
        s.close()
    batch.close()
