"""Negative pins of ``penrose_residuals``: matrices that satisfy only some of
the four Penrose equations (introduction: A X A = A, X A X = X, (A X)^T = A X,
(X A)^T = X A) must give non-zero residuals exactly where an equation fails,
with values known in closed form.  Exact rational arithmetic throughout."""
import inspect
import types
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import rg_ref


def _frac(a):
    return np.array([[F(v) for v in row] for row in a], dtype=object)


def _pinv_exact(A):
    """A^+ of a small integer matrix from the exact rational oracle: x = A^+ e_i
    for every unit target e_i (the minimum-norm least-squares solution)."""
    n = len(A)
    cols = [rg_ref.lstsq_exact(A, [int(i == j) for i in range(n)])[0] for j in range(n)]
    return np.array([[cols[j][k] for j in range(n)] for k in range(len(A[0]))], dtype=object)


A_INT = [[1, 2, 0], [2, 4, 0], [0, 1, 1], [1, 3, 1]]  # rank 2 (row 2 = 2 row 1, row 4 = row 1 + row 3)


def test_moore_penrose_inverse_has_zero_residuals():
    Ap = _pinv_exact(A_INT)
    assert rg_ref.penrose_residuals(_frac(A_INT), Ap) == [0, 0, 0, 0]


def test_doubled_pinv_fails_exactly_the_first_two():
    """X = 2 A^+: A X A - A = A and X A X - X = 2 A^+, while A X = 2 A A^+ and
    X A = 2 A^+ A stay symmetric."""
    A = _frac(A_INT)
    Ap = _pinv_exact(A_INT)
    r = rg_ref.penrose_residuals(A, 2 * Ap)
    assert r[0] == max(abs(v) for v in A.ravel())
    assert r[1] == 2 * max(abs(v) for v in Ap.ravel())
    assert r[2] == 0 and r[3] == 0


def test_generalized_inverse_fails_only_the_symmetries():
    """A = [[1, 0], [0, 0]] and X = [[1, 1], [1, 1]]: A X A = A and X A X = X
    hold, but A X = [[1, 1], [0, 0]] and X A = [[1, 0], [1, 0]] are not
    symmetric; each symmetry residual is 1."""
    A = _frac([[1, 0], [0, 0]])
    X = _frac([[1, 1], [1, 1]])
    assert rg_ref.penrose_residuals(A, X) == [0, 0, 1, 1]


def test_transposed_roles_fail_differently():
    """A = [[1, 1]] (1 x 2), X = [[1], [0]]: A X = [[1]] is symmetric and
    A X A = A, but X A = [[1, 1], [0, 0]] is not symmetric and X A X = X holds."""
    A = _frac([[1, 1]])
    X = _frac([[1], [0]])
    assert rg_ref.penrose_residuals(A, X) == [0, 0, 0, 1]


def test_float_perturbation_is_seen():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 4)) @ rng.standard_normal((4, 5))
    Ap = np.linalg.pinv(A)
    assert max(rg_ref.penrose_residuals(A, Ap)) < 1e-12
    E = np.zeros_like(Ap)
    E[2, 3] = 1e-3
    assert min(rg_ref.penrose_residuals(A, Ap + E)[:2]) > 1e-5


PENROSE_MUTATIONS = {
    "all_zero": ("return [abs(np.asarray(r)).max() if r.size else 0 for r in (r1, r2, r3, r4)]",
                 "return [0, 0, 0, 0]"),
    "first_equation_skips_A": ("r1 = A.dot(ApA) - A", "r1 = ApA - ApA"),
    "third_is_fourth": ("r3 = AAp.T - AAp", "r3 = ApA.T - ApA"),
    "second_wrong_product": ("r2 = Ap.dot(AAp) - Ap", "r2 = Ap.dot(AAp).dot(AAp) - Ap"),
}


@pytest.mark.parametrize("name", sorted(PENROSE_MUTATIONS))
def test_penrose_mutation_is_caught(name):
    old, new = PENROSE_MUTATIONS[name]
    src = inspect.getsource(rg_ref)
    assert src.count(old) == 1, old
    mod = types.ModuleType("rg_ref_penrose_mutant")
    exec(compile(src.replace(old, new), "rg_ref_penrose_mutant", "exec"), mod.__dict__)
    caught = False
    for t in (test_doubled_pinv_fails_exactly_the_first_two, test_generalized_inverse_fails_only_the_symmetries,
              test_transposed_roles_fail_differently):
        saved = rg_ref.penrose_residuals
        try:
            rg_ref.penrose_residuals = mod.penrose_residuals
            t()
        except AssertionError:
            caught = True
        finally:
            rg_ref.penrose_residuals = saved
    assert caught
