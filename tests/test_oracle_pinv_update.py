"""Pins of the oracle's maintained pseudoinverse (Theorems 2 and 3,
``track_pinv``), each independent of the update formula it checks:

- exact Fraction runs: the four Penrose equations hold exactly (they define
  A^+ uniquely), the maintained factor satisfies B C = A exactly, and
  A^+ Y equals the exact least-squares solver's x;
- the closed form of the Corollary's example [I_n; 1^T]:
  A^+ = [I - 1 1^T / (n + 1), 1 / (n + 1)];
- the orthogonal variant (alpha = 1) gives the same A^+ as the base
  factorization exactly (A^+ is unique), with its own B and C;
- FP64 runs agree with the SVD pseudoinverse at the planted rank.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import rg_ref


def _int_lowrank(rng, n, m, r, lo=-3, hi=4):
    """n x m integer matrix of rank <= r (product of integer factors), with
    zero rows, a repeated row and a sum of two rows mixed in."""
    A = rng.integers(lo, hi, size=(n, r)) @ rng.integers(lo, hi, size=(r, m))
    if n >= 6:
        A[2] = 0
        A[4] = A[1]
        A[5] = A[0] + A[3]
    return [[int(v) for v in row] for row in A]


def _frac(M):
    return np.array([[Fraction(v) for v in row] for row in M], dtype=object)


CASES = [(9, 5, 2), (12, 7, 4), (10, 4, 4), (6, 8, 3), (14, 6, 6), (7, 3, 1)]


@pytest.mark.parametrize("n,m,r", CASES)
def test_exact_penrose_factor_and_solution(n, m, r):
    rng = np.random.default_rng([n, m, r])
    A = _int_lowrank(rng, n, m, r)
    Y = [int(v) for v in rng.integers(-5, 6, size=n)]
    st = rg_ref.solve_stream(A, Y, exact=True, track_pinv=True)
    Af = _frac(A)
    Ap = np.array(st.Ap, dtype=object)
    assert Ap.shape == (m, n)
    assert all(v == 0 for v in rg_ref.penrose_residuals(Af, Ap))
    Bm = np.array(st.B, dtype=object).reshape(n, st.r)
    Cm = np.array(st.C, dtype=object).reshape(st.r, m)
    assert (Bm.dot(Cm) == Af).all()
    x_exact, r_exact = rg_ref.lstsq_exact(A, Y)
    assert st.r == r_exact
    assert list(Ap.dot(np.array([Fraction(v) for v in Y], dtype=object))) == list(x_exact)
    assert st.X == list(x_exact)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_closed_form_identity_plus_ones_row(n):
    """[I_n; 1^T]: the first n rows are independent, the last is dependent
    (Theorem 3 case); every entry of A^+ changes on that row."""
    A = [[1 if i == j else 0 for j in range(n)] for i in range(n)] + [[1] * n]
    st = rg_ref.solve_stream(A, [0] * (n + 1), exact=True, track_pinv=True)
    q = Fraction(1, n + 1)
    want = [[(1 if i == j else 0) - q for j in range(n)] + [q] for i in range(n)]
    assert st.Ap == want
    assert st.decisions == [True] * n + [False]


@pytest.mark.parametrize("n,m,r", CASES[:4])
def test_orthogonal_variant_same_pinv(n, m, r):
    rng = np.random.default_rng([7, n, m, r])
    A = _int_lowrank(rng, n, m, r)
    Y = [0] * n
    base = rg_ref.solve_stream(A, Y, exact=True, track_pinv=True)
    orth = rg_ref.solve_stream(A, Y, exact=True, variant="orthogonal", track_pinv=True)
    assert orth.Ap == base.Ap
    Bm = np.array(orth.B, dtype=object).reshape(n, orth.r)
    Cm = np.array(orth.C, dtype=object).reshape(orth.r, m)
    assert (Bm.dot(Cm) == _frac(A)).all()


@pytest.mark.parametrize("variant", ["base", "orthogonal", "orthonormal"])
def test_float_vs_svd_pinv(variant):
    rng = np.random.default_rng(3)
    n, m, r = 40, 12, 5
    A = rng.standard_normal((n, r)) @ rng.standard_normal((r, m))
    A[7] = A[3]
    st = rg_ref.solve_stream(A.tolist(), [0.0] * n, eps=1e-9, variant=variant, track_pinv=True)
    assert st.r == r
    Ap = np.array(st.Ap)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Asvd = Vt[:r].T @ np.diag(1.0 / s[:r]) @ U[:, :r].T
    assert np.linalg.norm(Ap - Asvd) <= 1e-10 * np.linalg.norm(Asvd)
    assert np.abs(np.array(st.B) @ np.array(st.C) - A).max() <= 1e-12 * np.abs(A).max()
