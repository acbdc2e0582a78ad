"""Host-only checks of the C-ABI library: it loads without a GPU, exports
every entry point declared in include/irk.h, and its host-side tableau
construction agrees with the oracle's independent one."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1701_07181_amd", "libirk.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "irk.h")).read()
    return sorted(set(re.findall(r"\b(irk_[a-z_]+)\s*\(", src)))


def test_library_exports_header_symbols():
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert "irk_setup" in names and "irk_gmres_solve" in names and "irk_factor_ilu" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import paper_1701_07181_amd as irk
    assert sorted(irk.EXPORTED) == _declared()


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 8])
def test_library_tableau_matches_oracle(s):
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import paper_1701_07181_amd as irk
    A, b, c = irk.radau_iia(s)
    Ao, bo, co = oracle.radau_iia(s)
    np.testing.assert_allclose(c, co, rtol=0, atol=1e-15)
    np.testing.assert_allclose(A, Ao, rtol=0, atol=5e-14)
    np.testing.assert_allclose(b, bo, rtol=0, atol=5e-14)


def test_library_rejects_bad_tableau_size():
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import paper_1701_07181_amd as irk
    with pytest.raises(irk.IrkError):
        irk.radau_iia(0)
    assert irk.status_str(irk.ERR_SINGULAR) == "singular pivot block"
