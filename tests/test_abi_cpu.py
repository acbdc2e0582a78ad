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


def _problem(irk, sy, **kw):
    import ctypes as C
    A = np.ascontiguousarray(oracle.radau_iia(sy.s)[0])
    rp = np.ascontiguousarray(sy.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(sy.col_idx, dtype=np.int32)
    p = irk._Problem(kw.get("s", sy.s), A.ctypes.data, sy.T, sy.m, int(ci.size), rp.ctypes.data,
                     ci.ctypes.data, 0x1000, kw.get("nJ", 1), 0x1000, kw.get("dt", sy.dt))
    return p, (A, rp, ci)


def test_host_argument_checks():
    """Argument errors are found on the host, before any device work."""
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import ctypes as C
    import dgsynth
    import paper_1701_07181_amd as irk
    sy = dgsynth.config_system("cfg0")
    o = irk.Options()._c()
    nb = C.c_size_t()
    p, keep = _problem(irk, sy)
    assert irk._L.irk_workspace_size(C.byref(p), C.byref(o), C.byref(nb)) == irk.OK and nb.value > 0
    for kw in ({"dt": 0.0}, {"dt": -1.0}, {"nJ": 3}, {"s": 6}, {"s": 0}):
        p, keep = _problem(irk, sy, **kw)
        assert irk._L.irk_workspace_size(C.byref(p), C.byref(o), C.byref(nb)) == irk.ERR_ARG, kw
    p, keep = _problem(irk, sy)
    for field, val in (("restart", 0), ("restart", 65), ("max_iters", 0), ("rtol", 0.0)):
        o2 = irk.Options()._c()
        setattr(o2, field, val)
        assert irk._L.irk_workspace_size(C.byref(p), C.byref(o2), C.byref(nb)) == irk.ERR_ARG, field
    o3 = irk.Options(pc="none", matvec_prec="fp32", factor_prec="fp32")._c()
    assert irk._L.irk_workspace_size(C.byref(p), C.byref(o3), C.byref(nb)) == irk.ERR_ARG


@pytest.mark.parametrize("bad", ["unsorted", "no_diag", "asymmetric", "triangle"])
def test_setup_rejects_bad_patterns(bad):
    """Pattern checks run in irk_setup before the workspace is touched."""
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import ctypes as C
    import dgsynth
    import paper_1701_07181_amd as irk
    if bad == "triangle":
        tri = [[(e + 1) % 3, (e + 2) % 3] for e in range(3)]     # 3 mutually adjacent elements
        sy = dgsynth.make_system(1, tri, 4, 2, 0.1)
    else:
        sy = dgsynth.config_system("cfg0")
    ci = sy.col_idx.copy()
    rp = sy.row_ptr.copy()
    if bad == "unsorted":
        ci[rp[3]], ci[rp[3] + 1] = ci[rp[3] + 1], ci[rp[3]]
    elif bad == "no_diag":
        row = 5
        d = int(np.flatnonzero(ci[rp[row]:rp[row + 1]] == row)[0]) + rp[row]
        ci[d] = [c for c in range(sy.T) if c not in ci[rp[row]:rp[row + 1]]][0]
        ci[rp[row]:rp[row + 1]] = np.sort(ci[rp[row]:rp[row + 1]])
    elif bad == "asymmetric":
        row = 7
        seg = ci[rp[row]:rp[row + 1]]
        j = [c for c in range(sy.T) if c not in seg and c != row][0]
        seg[int(np.flatnonzero(seg != row)[0])] = j     # row 7 drops a neighbour, gains j
        ci[rp[row]:rp[row + 1]] = np.sort(seg)
    sy.col_idx = ci
    p, keep = _problem(irk, sy)
    o = irk.Options()._c()
    h = C.c_void_p()
    st = irk._L.irk_setup(C.byref(p), C.byref(o), C.c_void_p(0x1000), 1 << 40, None, C.byref(h))
    assert st == irk.ERR_ARG and not h.value


def test_setup_rejects_small_workspace():
    """A workspace below irk_workspace_size is refused before any device work."""
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import ctypes as C
    import dgsynth
    import paper_1701_07181_amd as irk
    sy = dgsynth.config_system("cfg0")
    p, keep = _problem(irk, sy)
    o = irk.Options(pc="coupled")._c()
    nb = C.c_size_t()
    assert irk._L.irk_workspace_size(C.byref(p), C.byref(o), C.byref(nb)) == irk.OK
    h = C.c_void_p()
    st = irk._L.irk_setup(C.byref(p), C.byref(o), C.c_void_p(0x1000), nb.value - 1, None, C.byref(h))
    assert st == irk.ERR_NOMEM and not h.value


@pytest.mark.parametrize("bad", ["jump_past_end", "decreasing", "last_not_nnzb"])
def test_setup_rejects_malformed_row_ptr(bad):
    """The whole row pointer is validated before any col_idx entry is read:
    a row pointer that jumps past nnzb (here 1000 with nnzb = 5) must come
    back as an argument error, not as a read beyond col_idx."""
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import ctypes as C
    import paper_1701_07181_amd as irk
    T, m, s = 4, 4, 2
    if bad == "jump_past_end":
        rp = np.array([0, 1000, 5, 5, 5], dtype=np.int32)
    elif bad == "decreasing":
        rp = np.array([0, 3, 2, 4, 5], dtype=np.int32)
    else:
        rp = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    ci = np.array([0, 1, 2, 3, 0], dtype=np.int32)
    A = np.ascontiguousarray(oracle.radau_iia(s)[0])
    p = irk._Problem(s, A.ctypes.data, T, m, 5, rp.ctypes.data, ci.ctypes.data, 0x1000, 1,
                     0x1000, 0.1)
    o = irk.Options()._c()
    h = C.c_void_p()
    st = irk._L.irk_setup(C.byref(p), C.byref(o), C.c_void_p(0x1000), 1 << 40, None, C.byref(h))
    assert st == irk.ERR_ARG and not h.value


@pytest.mark.parametrize("name", ["DIRK33", "ESDIRK65"])
def test_library_dirk_tableau_matches_oracle(name):
    if not os.path.exists(LIB):
        pytest.skip("libirk.so not built")
    import paper_1701_07181_amd as irk
    from oracle import step as ostep
    A, b, c = irk.dirk_tableau(name)
    Ao, bo, co = ostep.dirk33() if name == "DIRK33" else ostep.esdirk65()
    np.testing.assert_allclose(A, Ao, rtol=0, atol=1e-15)
    np.testing.assert_allclose(b, bo, rtol=0, atol=1e-15)
    np.testing.assert_allclose(c, co, rtol=0, atol=1e-14)
