"""Pins of the oracle's Radau IIA tableau against what the paper and the
mathematics fix (Sec. 3, Table 1; Sec. 4.1; App. A)."""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _closed_forms():
    out = {}
    with open(os.path.join(GOLD, "radau_closed_forms.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, what, r, c, expr = line.split()
            val = eval(expr, {"sqrt": math.sqrt, "__builtins__": {}})
            out.setdefault(name, []).append((what, int(r), None if c == "-" else int(c), val))
    return out


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_simplifying_conditions(s):
    """C(s): sum_j a_ij c_j^(q-1) = c_i^q / q (q <= s); B(2s-1): sum b_i
    c_i^(q-1) = 1/q (q <= 2s-1).  Radau IIA has order 2s-1 and stage order s
    (Sec. 3)."""
    A, b, c = oracle.radau_iia(s)
    for q in range(1, s + 1):
        np.testing.assert_allclose(A @ c ** (q - 1), c ** q / q, rtol=0, atol=2e-15)
    for q in range(1, 2 * s):
        assert abs(b @ c ** (q - 1) - 1.0 / q) < 2e-15
    # order is exactly 2s-1: B(2s) fails
    assert abs(b @ c ** (2 * s - 1) - 1.0 / (2 * s)) > 1e-7


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_stiffly_accurate(s):
    """c_s = 1 and b is the last row of A (Radau right quadrature), hence
    b^T A^{-1} = (0,...,0,1) (Sec. 4.1)."""
    A, b, c = oracle.radau_iia(s)
    assert c[-1] == 1.0
    np.testing.assert_array_equal(b, A[-1])
    e = b @ oracle.inverse(A)
    np.testing.assert_allclose(e, np.eye(s)[-1], atol=5e-14)
    assert np.all(np.diff(c) > 0) and c[0] > 0


def test_closed_forms_app_a():
    """RADAU23 and RADAU35 as printed in App. A (RADAU35 row 2 sign-corrected)."""
    cf = _closed_forms()
    for name, s in (("RADAU23", 2), ("RADAU35", 3)):
        A, b, c = oracle.radau_iia(s)
        for what, r, col, val in cf[name]:
            got = {"A": lambda: A[r, col], "b": lambda: b[r], "c": lambda: c[r]}[what]()
            assert abs(got - val) < 3e-16 * max(1.0, abs(val)) * 8, (name, what, r, col, got, val)


def test_printed_radau35_row2_violates_C3():
    """The literal printed row 2 of RADAU35 fails C(1) (its sum is not c_2):
    this is why the fixture carries the corrected signs."""
    s6 = math.sqrt(6)
    literal = np.array([37 / 225 - 169 * s6 / 1800, 11 / 45 - 7 * s6 / 360, -2 / 225 - s6 / 75])
    c2 = 2 / 5 + s6 / 10
    assert abs(literal.sum() - c2) > 0.5
    A, _, c = oracle.radau_iia(3)
    assert abs(A[1].sum() - c[1]) < 1e-15


def _pade(s, z):
    """(s-1, s) Pade approximant of e^z (textbook formula)."""
    k, j = s - 1, s
    P = sum(math.factorial(k + j - i) * math.factorial(k)
            / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
            for i in range(k + 1))
    Q = sum(math.factorial(k + j - i) * math.factorial(j)
            / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
            for i in range(j + 1))
    return P / Q


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_stability_function_is_pade(s):
    """R(z) = 1 + z b^T (I - zA)^{-1} 1 equals the (s-1, s) Pade approximant
    of e^z, which is what makes Radau IIA L-stable (Sec. 3)."""
    A, b, c = oracle.radau_iia(s)
    for z in (-1.0, -10.0, -0.5 + 2j, 0.3, -1000.0, 5j):
        R = 1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))
        assert abs(R - _pade(s, z)) < 1e-13 * max(1.0, abs(_pade(s, z)))
    # L-stability: R(z) -> 0 as z -> -inf
    z = -1e8
    assert abs(1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))) < 1e-7


def test_error_constants_table1():
    """Leading error coefficient (e^z - R(z)) / z^(2s) at z -> 0 equals
    s!(s-1)!/((2s)!(2s-1)!) and matches Table 1 to its three printed digits."""
    rows = []
    with open(os.path.join(GOLD, "table1_error_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                s, v = line.split()
                rows.append((int(s), float(v)))
    for s, printed in rows:
        A, b, c = oracle.radau_iia(s)
        closed = math.factorial(s) * math.factorial(s - 1) / (
            math.factorial(2 * s) * math.factorial(2 * s - 1))
        # from the tableau: R(z) = 1 + sum_q z^(q+1) b^T A^q 1, so the z^(2s)
        # coefficient of e^z - R(z) is 1/(2s)! - b^T A^(2s-1) 1
        coef = 1.0 / math.factorial(2 * s) - b @ np.linalg.matrix_power(A, 2 * s - 1) @ np.ones(s)
        assert abs(abs(coef) - closed) < 1e-9 * closed + 1e-16
        assert float(f"{closed:.2e}") == printed


def test_s2_inverse_and_shifts():
    """From the printed RADAU23: A^{-1} = [[3/2, 1/2], [-9/2, 5/2]] (det A = 1/6),
    eigenvalues 2 +- i sqrt(2); column-sum shifts alpha = (9/2, 1/2) and
    shifted diagonal coefficients (6, 3) (Sec. 4.3.2)."""
    A, b, c = oracle.radau_iia(2)
    Ainv = oracle.inverse(A)
    np.testing.assert_allclose(Ainv, [[1.5, 0.5], [-4.5, 2.5]], atol=2e-15)
    ev = np.sort_complex(np.linalg.eigvals(Ainv))
    np.testing.assert_allclose(ev, [2 - 1j * math.sqrt(2), 2 + 1j * math.sqrt(2)], atol=1e-14)
    al = oracle.shifts(Ainv, 0)
    np.testing.assert_allclose(al, [4.5, 0.5], atol=2e-15)
    np.testing.assert_allclose(np.diag(Ainv) + al, [6.0, 3.0], atol=2e-15)
    np.testing.assert_array_equal(oracle.shifts(Ainv, 1), [0.0, 0.0])
    np.testing.assert_allclose(oracle.shifts(Ainv, 2), [0.5, 4.5], atol=2e-15)


@pytest.mark.parametrize("n", [1, 3, 7])
def test_dense_inverse(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    Ai = oracle.inverse(A)
    np.testing.assert_allclose(A @ Ai, np.eye(n), atol=1e-13)
    # a matrix that needs row pivoting
    P = np.eye(n)[::-1].copy()
    if n > 1:
        Ai = oracle.inverse(P)
        np.testing.assert_array_equal(Ai, P.T)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.inverse(np.zeros((n, n)))
