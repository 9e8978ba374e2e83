"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is either
a hand-derived fixture (tests/golden), a closed form, an independent exact
solver (row-space normal equations, no recursion), an identity the
pseudoinverse must satisfy, or a library SVD.
"""
import json
import os
import random
from fractions import Fraction as F
from math import comb

import numpy as np
import pytest

from oracle import rg_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _frac(p):
    return F(p[0], p[1])


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_worked_example_every_row():
    """Hand-derived iterates of Algorithm 1 on a 4 x 2 example."""
    g = _load("worked_example_m2.json")
    st = rg_ref.RGState(g["m"], F(0))
    for i, (row, y) in enumerate(zip(g["rows"], g["y"])):
        indep = rg_ref.update_least_squares(st, [F(v) for v in row], F(y), 0)
        assert indep == g["independent"][i]
        assert st.r == g["rank_after_each_row"][i]
        assert st.X == [_frac(p) for p in g["x_after_each_row"][i]]
    assert st.C == [[_frac(p) for p in row] for row in g["final_C"]]
    assert st.Ct == [[_frac(p) for p in row] for row in g["final_Ct"]]
    assert st.Pinv == [[_frac(p) for p in row] for row in g["final_Pinv"]]


def test_min_norm_example():
    g = _load("min_norm_m3.json")
    st = rg_ref.solve_stream(g["rows"], g["y"], exact=True)
    assert st.X == [_frac(p) for p in g["x"]]
    assert st.r == g["rank"]
    x, r = rg_ref.lstsq_exact(g["rows"], g["y"])
    assert x == [_frac(p) for p in g["x"]] and r == g["rank"]


def _planted(rng, n, m, r, p_dup=0.2, p_comb=0.15, p_zero=0.05, lo=-3, hi=3):
    """Tiny integer matrix of rank <= r with duplicates, +-1 combinations of
    earlier rows and zero rows."""
    W = [[rng.randint(lo, hi) for _ in range(m)] for _ in range(r)]
    rows = []
    for i in range(n):
        u = rng.random()
        if i >= 1 and u < p_dup:
            rows.append(list(rows[rng.randrange(i)]))
        elif i >= 2 and u < p_dup + p_comb:
            j, k = rng.sample(range(i), 2)
            s = rng.choice([-1, 1])
            rows.append([a + s * b for a, b in zip(rows[j], rows[k])])
        elif u < p_dup + p_comb + p_zero:
            rows.append([0] * m)
        else:
            z = [rng.randint(-2, 2) for _ in range(r)]
            rows.append([sum(z[k] * W[k][j] for k in range(r)) for j in range(m)])
    Y = [rng.randint(-9, 9) for _ in range(n)]
    return rows, Y


@pytest.mark.parametrize("seed", range(40))
def test_fraction_run_equals_exact_solver(seed):
    """Bit-exact x_n and rank: Algorithm 1 over rationals vs the row-space
    normal-equation solver (which uses no recursion)."""
    rng = random.Random(seed)
    m = rng.randint(1, 7)
    n = rng.randint(1, 18)
    r = rng.randint(1, min(m, 5))
    A, Y = _planted(rng, n, m, r)
    st = rg_ref.solve_stream(A, Y, exact=True)
    x, rank = rg_ref.lstsq_exact(A, Y)
    assert st.r == rank
    assert st.X == x


@pytest.mark.parametrize("seed", range(12))
def test_invariants_after_every_row(seed):
    """Ct C^T = I_r, Pinv (B^T B) = I_r with B = A Ct^T, x = C^T Ct x
    (x in the row space), A^T (A x - Y) = 0, rank grows by at most one."""
    rng = random.Random(1000 + seed)
    m, n, r = rng.randint(2, 6), rng.randint(4, 14), rng.randint(1, 4)
    A, Y = _planted(rng, n, m, min(r, m))
    st = rg_ref.RGState(m, F(0))
    prev = 0
    for i in range(n):
        rg_ref.update_least_squares(st, [F(v) for v in A[i]], F(Y[i]), 0)
        k = st.r
        assert k - prev in (0, 1)
        prev = k
        for a in range(k):
            for b in range(k):
                assert sum(st.Ct[a][j] * st.C[b][j] for j in range(m)) == (1 if a == b else 0)
        Ai = A[:i + 1]
        B = [[sum(F(row[j]) * st.Ct[a][j] for j in range(m)) for a in range(k)] for row in Ai]
        BtB = [[sum(B[t][a] * B[t][b] for t in range(len(Ai))) for b in range(k)] for a in range(k)]
        for a in range(k):
            for b in range(k):
                assert sum(st.Pinv[a][c] * BtB[c][b] for c in range(k)) == (1 if a == b else 0)
        w = [sum(st.C[a][j] * st.X[j] for j in range(m)) for a in range(k)]
        assert [sum(st.Ct[a][j] * w[a] for a in range(k)) for j in range(m)] == st.X
        res = [sum(F(row[j]) * st.X[j] for j in range(m)) - Y[t] for t, row in enumerate(Ai)]
        assert all(sum(F(Ai[t][j]) * res[t] for t in range(len(Ai))) == 0 for j in range(m))


@pytest.mark.parametrize("seed", range(10))
def test_penrose_exact(seed):
    """Theorem 1 applied to the final factors gives the Moore-Penrose inverse:
    all four Penrose equations hold exactly in rationals."""
    rng = random.Random(2000 + seed)
    m, n, r = rng.randint(2, 6), rng.randint(3, 10), rng.randint(1, 4)
    A, Y = _planted(rng, n, m, min(r, m))
    st = rg_ref.solve_stream(A, Y, exact=True)
    Ap = rg_ref.pinv_from_state([[F(v) for v in row] for row in A], st)
    res = rg_ref.penrose_residuals(np.array([[F(v) for v in row] for row in A], dtype=object),
                                   np.array(Ap, dtype=object))
    assert all(v == 0 for v in res)


def _pascal(n):
    return [[comb(i + j, i) for j in range(n)] for i in range(n)]


def _pascal_inverse(n):
    """P(n) = L L^T with L[i][j] = C(i, j); L^-1[i][j] = (-1)^(i-j) C(i, j),
    so P(n)^-1 = L^-T L^-1 (integers)."""
    Li = [[(-1) ** (i - j) * comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)]
    return [[sum(Li[k][i] * Li[k][j] for k in range(n)) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_pascal_exact_inverse(n):
    """Section 4.2: the rational rank-Greville run returns the exact inverse
    of the Pascal matrices."""
    P = _pascal(n)
    st = rg_ref.solve_stream(P, [0] * n, exact=True)
    assert st.r == n
    Ap = rg_ref.pinv_from_state([[F(v) for v in row] for row in P], st)
    assert Ap == [[F(v) for v in row] for row in _pascal_inverse(n)]


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_identity_plus_ones_row(n):
    """Footnote example after Theorem 3: A = I_n, then Gamma = (1,...,1).
    Closed forms: x_n = Y; with the extra row, A^T A = I + 1 1^T whose inverse
    is I - 1 1^T/(n+1), so x = (I - 1 1^T/(n+1)) (Y + y 1); and every entry
    of the pseudoinverse [I | 0] changes."""
    rng = random.Random(n)
    Y = [F(rng.randint(-5, 5)) for _ in range(n)]
    y = F(rng.randint(-5, 5))
    A = [[1 if i == j else 0 for j in range(n)] for i in range(n)]
    st = rg_ref.solve_stream(A, Y, exact=True)
    assert st.X == Y
    Ap0 = rg_ref.pinv_from_state(A, st)
    rg_ref.update_least_squares(st, [F(1)] * n, y, 0)
    v = [Y[j] + y for j in range(n)]
    s = sum(v)
    assert st.X == [v[j] - s / (n + 1) for j in range(n)]
    Ap1 = rg_ref.pinv_from_state(A + [[1] * n], st)
    for j in range(n):
        for i in range(n):
            assert Ap1[j][i] != Ap0[j][i]
        assert Ap1[j][n] != 0


def test_single_row_closed_form():
    """One row: x = Gamma y / ||Gamma||^2 (Theorem 4 with X_0 = 0)."""
    G = [F(3), F(-1), F(2)]
    st = rg_ref.solve_stream([G], [F(7)], exact=True)
    n2 = sum(v * v for v in G)
    assert st.X == [v * 7 / n2 for v in G]


def test_zero_rows_are_noops():
    """A zero row leaves x and the rank unchanged (dependent branch with
    gamma = 0); an all-zero input keeps x = 0 (A_0^+ = 0)."""
    st = rg_ref.solve_stream([[0, 0, 0]] * 3, [1, 2, 3], exact=True)
    assert st.r == 0 and st.X == [0, 0, 0]
    st = rg_ref.solve_stream([[1, 2, 0], [0, 0, 0], [0, 1, 1]], [1, 5, 2], exact=True)
    st2 = rg_ref.solve_stream([[1, 2, 0], [0, 1, 1]], [1, 2], exact=True)
    assert st.X == st2.X and st.r == st2.r == 2


def test_full_column_rank_normal_equations():
    """Full column rank: x = (A^T A)^-1 A^T Y (FP64, normal equations)."""
    rng = np.random.default_rng(5)
    A = rng.integers(-4, 5, size=(12, 5)).astype(float)
    Y = rng.standard_normal(12)
    st = rg_ref.solve_stream(A.tolist(), Y.tolist())
    assert st.r == 5
    x = np.linalg.solve(A.T @ A, A.T @ Y)
    assert np.allclose(st.X, x, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_float_run_vs_truncated_svd(seed):
    """FP64 Algorithm 1 vs the truncated-SVD solution at the planted rank."""
    from paper_2106_11594_amd import workloads as W
    s = W.single_f64(n=120, m=24, r=6, seed=seed)
    st = rg_ref.solve_stream(s.A.tolist(), s.Y.tolist(), eps=1e-10)
    assert st.r == 6
    x = rg_ref.lstsq_svd(s.A, s.Y, rank=6)
    assert np.linalg.norm(np.array(st.X) - x) <= 1e-10 * np.linalg.norm(x)
    Ap = np.array(rg_ref.pinv_from_state(s.A.tolist(), st))
    res = rg_ref.penrose_residuals(s.A, Ap)
    assert max(res) < 1e-9 * max(1.0, abs(s.A).max())


def test_default_eps_formula():
    """Section 3: eps = (m^2 r + m r + m) eps_M."""
    assert rg_ref.default_eps(10, 3, 1.0) == 100 * 3 + 30 + 10
    assert rg_ref.default_eps(64, 0, 2.0 ** -52) == 64 * 2.0 ** -52
