"""Mixed precision on the GPU: the factor quantizer matches the oracle's bit
for bit on the same inputs, and the FP32-operator / reduced-precision-factor
solves inside the FP64 refinement loop reach an FP64 true relative residual
of 1e-8 (checked with the oracle's FP64 operator), with the error against
the oracle's FP64 solution reported."""
import sys

import numpy as np
import pytest

import dgsynth
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _irk():
    import paper_1701_07181_amd as irk
    return irk


def _blocks(seed, nblk, m):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nblk, m, m)) * 10.0 ** rng.uniform(-6, 6, (nblk, 1, 1))
    x[0] = 0.0                                  # zero block
    x[1, 0, :4] = [1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, 2.0 ** -30, -65504.0]   # ties, tiny
    x[2] *= 1e-300 / np.abs(x[2]).max()         # exponent clamp
    return x


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16s"])
@pytest.mark.parametrize("m", [16, 64, 135])
def test_quantizer_bit_parity(prec, m):
    irk = _irk()
    x = _blocks(11 + m, 12, m)
    q, ex = irk.quantize_blocks(torch.from_numpy(x).cuda(), prec)
    q = q.cpu().numpy()
    for b in range(x.shape[0]):
        if prec == "fp32":
            ref = x[b].astype(np.float32)
            np.testing.assert_array_equal(q[b].view(np.uint32), ref.view(np.uint32))
        elif prec == "bf16":
            ref = oracle.bf16_bits(x[b])
            np.testing.assert_array_equal(q[b].ravel().view(np.uint16), ref)
        else:
            e = oracle.f16_block_exponent(x[b])
            assert int(ex[b].item()) == e
            ref = oracle.f16_scaled_bits(x[b], e)
            np.testing.assert_array_equal(q[b].ravel().view(np.uint16), ref)


CASES = [("cfg2-shape 3D N=4 m=135", dict(s=3, dim=3, N=4, m=135, dt=0.5)),
         ("cfg1-shape 2D N=8 m=64", dict(s=3, dim=2, N=8, m=64, dt=0.1)),
         ("s=4 2D N=6 m=36", dict(s=4, dim=2, N=6, m=36, dt=0.3))]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16s"])
@pytest.mark.parametrize("pc", ["uncoupled_shifted", "coupled"])
@pytest.mark.parametrize("name,c", CASES, ids=[c[0] for c in CASES])
def test_mixed_precision_solve(name, c, pc, prec):
    irk = _irk()
    mesh = dgsynth.grid2d(c["N"]) if c["dim"] == 2 else dgsynth.grid3d(c["N"])
    sy = dgsynth.make_system(77, mesh, c["m"], c["s"], c["dt"])
    sol = irk.Solver(sy, irk.Options(pc=pc, matvec_prec="fp32", factor_prec=prec, rtol=1e-8,
                                     inner_rtol=1e-4))
    sol.factor()
    x, info = sol.solve(sy.rhs)
    x = x.cpu().numpy()
    A, _, _ = oracle.radau_iia(sy.s)
    P = oracle.Problem(sy)
    r = sy.rhs - oracle.matvec(P, oracle.inverse(A), x)
    rel = np.linalg.norm(r) / np.linalg.norm(sy.rhs)
    xo, io = oracle.solve(P, A, sy.rhs, pc=pc, rtol=1e-12)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"{name} {pc} {prec}: inner iters {info['iters']} outer {info['outer_iters']} "
          f"(oracle FP64 {io['iters']}), true rel res {rel:.2e}, rel err vs FP64 oracle {err:.2e}",
          flush=True)
    assert info["converged"] and info["rel_res_true"] <= 1e-8
    assert rel <= 1e-8 * (1 + 1e-6)
    assert err <= 1e-6
    sol.close()


def test_mixed_beats_nothing_on_error_paths():
    """Mixed precision needs a preconditioner (rejected without one)."""
    irk = _irk()
    sy = dgsynth.config_system("cfg0")
    with pytest.raises(irk.IrkError):
        irk.Solver(sy, irk.Options(pc="none", matvec_prec="fp32", factor_prec="fp32"))
