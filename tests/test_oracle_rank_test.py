"""Pins of the rank test of Section 3 on cases where its relative clause
decides: dependent iff ||Gamma_r|| < eps or ||Gamma_r|| < eps ||Gamma||.

Every case has two rows.  The first, e_1, starts the basis.  The second row's
rejection against span(e_1) is its tail (entries 2..m), so ||Gamma_r|| and
||Gamma|| are known in closed form and the expected decision follows from the
definition alone:

  REL_DEPENDENT   (1000, 1/2, 0, 0), eps = 1e-3: ||Gamma_r|| = 1/2 passes the
                  absolute clause (1/2 >= eps) but 1/2 < eps ||Gamma|| ~ 1.0000001,
                  so the row is dependent (rank stays 1).  Dropping the
                  relative clause makes it independent.
  REL_BETWEEN     (1000, 2, 0, 0), eps = 1e-3: 2 >= eps ||Gamma|| ~ 1.000002, so
                  independent (rank 2).  A relative clause with ||Gamma||^2
                  (eps ||Gamma||^2 ~ 1000) would call it dependent.
  REL_EQUAL       (3, 1, 1, 1), eps = 1/2: ||Gamma_r|| = sqrt(3) and
                  eps ||Gamma|| = sqrt(12)/2 = sqrt(3) exactly (also in IEEE
                  double: sqrt(12) = 2 sqrt(3) after rounding, and the halving is
                  exact).  The comparison is strict, so the row is independent;
                  a test with <= calls it dependent.

Each case runs through the Python oracle in floats and in exact rationals
(with the same, exactly converted eps) and through the C oracle.  The
mutation tests plant the three slips in both oracles.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref_c, rg_ref

CASES = {
    "REL_DEPENDENT": ([[1, 0, 0, 0], [1000, 0.5, 0, 0]], 1e-3, [True, False]),
    "REL_BETWEEN": ([[1, 0, 0, 0], [1000, 2, 0, 0]], 1e-3, [True, True]),
    "REL_EQUAL": ([[1, 0, 0, 0], [3, 1, 1, 1]], 0.5, [True, True]),
}
TARGETS = [1.0, 2.0]


@pytest.fixture(scope="module", autouse=True)
def _built():
    ref_c.build()


def python_float_decisions(mod, rows, eps):
    st = mod.solve_stream(rows, TARGETS, eps=eps)
    return st.decisions


def python_exact_decisions(mod, rows, eps):
    st = mod.RGState(len(rows[0]), Fraction(0))
    for row, y in zip(rows, TARGETS):
        mod.update_least_squares(st, [Fraction(v) for v in row], Fraction(y), Fraction(eps))
    return st.decisions


def c_decisions(rows, eps, lib_path=None):
    A = np.array(rows, dtype=np.float64)
    *_, dec = ref_c.solve(A, np.array(TARGETS), eps=eps, decisions=True, lib_path=lib_path)
    return [bool(d) for d in dec]


def test_closed_form_norms():
    """The norms the cases rely on, from their definitions."""
    for name, (rows, eps, _) in CASES.items():
        g = np.array(rows[1], dtype=np.float64)
        gr = g.copy()
        gr[0] = 0.0  # rejection from span(e_1)
        st = rg_ref.solve_stream(rows[:1], TARGETS[:1], eps=eps)
        assert st.C == [[1.0, 0.0, 0.0, 0.0]] and st.Ct == [[1.0, 0.0, 0.0, 0.0]]
        nr, ng = np.sqrt(gr @ gr), np.sqrt(g @ g)
        assert nr >= eps, name  # the absolute clause never decides these cases
        if name == "REL_EQUAL":
            assert nr == eps * ng
        elif name == "REL_DEPENDENT":
            assert nr < eps * ng
        else:
            assert eps * ng < nr < eps * ng * ng


@pytest.mark.parametrize("name", sorted(CASES))
def test_python_float(name):
    rows, eps, want = CASES[name]
    assert python_float_decisions(rg_ref, rows, eps) == want


@pytest.mark.parametrize("name", sorted(CASES))
def test_python_exact(name):
    rows, eps, want = CASES[name]
    assert python_exact_decisions(rg_ref, rows, eps) == want


@pytest.mark.parametrize("name", sorted(CASES))
def test_c_oracle(name):
    rows, eps, want = CASES[name]
    assert c_decisions(rows, eps) == want


def test_dependent_row_gives_rank_one_least_squares():
    """REL_DEPENDENT: with the second row taken as dependent the solution is
    the least-squares fit inside span(e_1): x = (y1 + 1000 y2) / (1 + 1000^2) e_1."""
    rows, eps, _ = CASES["REL_DEPENDENT"]
    st = rg_ref.solve_stream(rows, TARGETS, eps=eps)
    x1 = (1.0 + 1000.0 * 2.0) / (1.0 + 1000.0 ** 2)
    assert np.allclose(st.X, [x1, 0.0, 0.0, 0.0], rtol=1e-13, atol=1e-16)
    xc, r, *_ = ref_c.solve(np.array(rows, float), np.array(TARGETS), eps=eps)
    assert r == 1 and np.allclose(xc, st.X, rtol=1e-13, atol=1e-16)
