"""The stability study of Section 4.2 on the CPU: the two measures
(stability factor, residual error) against closed forms, the test-matrix
generators against the condition numbers the paper's tables print, and the
oracle's FP64 rank-Greville run against the rank-Greville columns of those
tables (tests/golden/stability_tables.json, values as printed in the paper).

The paper's runs used NumPy sums and its own seeds; the oracle sums in
another order and the USV family uses our seeds, so the measures are compared
within a factor of 30 (an order of magnitude and a half), except where the
paper's value is set by kappa eps_M ~ 1 (Pascal n = 10), which must agree to
10 %.  The condition numbers do not depend on any of that and must agree to
the three digits printed."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import rg_ref
from paper_2106_11594_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stability_tables.json")))


def _close3(a, b):
    return abs(a - b) <= 0.006 * abs(b)


def test_measures_closed_forms():
    A = np.diag([1.0, 2.0, 4.0])
    Ap = np.diag([1.0, 0.5, 0.25])
    assert rg_ref.stability_factor(Ap, Ap, A) == 0.0
    assert rg_ref.residual_error(Ap, A) == 0.0
    E = np.zeros((3, 3))
    E[1, 2] = 1e-10
    # ||E||_2 = 1e-10, ||A^+||_2 = 1, kappa_2 = 4
    assert np.isclose(rg_ref.stability_factor(Ap + E, Ap, A), 1e-10 / (2.0 ** -52 * 1.0 * 4.0), rtol=1e-12)
    # (A^+ + E) A - I = E A: only entry (1, 2) = 4e-10, so the 2-norm is 4e-10;
    # ||A||_2 = 4 and ||A^+ + E||_2 = 1 (the perturbation leaves the largest singular value)
    assert np.isclose(rg_ref.residual_error(Ap + E, A), 4e-10 / (4.0 * 1.0), rtol=1e-6)
    # rectangular: A (3 x 2) with orthonormal columns scaled by 3, A^+ = A^T / 9
    Q = np.array([[1.0, 0.0], [0.0, 0.6], [0.0, 0.8]]) * 3.0
    assert rg_ref.residual_error(Q.T / 9.0, Q) < 1e-15


@pytest.mark.parametrize("k", range(4))
def test_pascal_kappa_and_oracle_measures(k):
    g = GOLD["pascal"]
    n = g["n"][k]
    P = W.pascal(n)
    assert _close3(np.linalg.cond(P), g["kappa"][k])
    ex = rg_ref.solve_stream(P.tolist(), [0] * n, exact=True, track_pinv=True)
    Pinv = np.array([[float(v) for v in row] for row in ex.Ap])
    assert np.array_equal(Pinv @ P, np.eye(n))  # the exact inverse (integers)
    st = rg_ref.solve_stream(P.tolist(), [0.0] * n, track_pinv=True)
    e = rg_ref.stability_factor(np.array(st.Ap), Pinv, P)
    res = rg_ref.residual_error(np.array(st.Ap), P)
    if n == 10:
        assert abs(e - g["e_rank_greville"][k]) <= 0.1 * g["e_rank_greville"][k]
    else:
        assert g["e_rank_greville"][k] / 30 <= e <= 30 * g["e_rank_greville"][k]
    assert g["res_rank_greville"][k] / 30 <= res <= 30 * g["res_rank_greville"][k]


@pytest.mark.parametrize("k", range(3))
def test_usv_kappa_and_oracle_measures(k):
    g = GOLD["usv"]
    n = g["n"][k]
    A, U, S, V = W.usv(n, g["rows_per_col"])
    assert A.shape == (5 * n, n)
    assert _close3(np.linalg.cond(A), g["kappa"][k])
    ref = (V / S) @ U.T  # (U S V^T)^+ = V S^-1 U^T
    assert np.allclose(ref, np.linalg.pinv(A), rtol=1e-10, atol=1e-13)
    st = rg_ref.solve_stream(A.tolist(), [0.0] * A.shape[0], eps=g["eps"], track_pinv=True)
    assert st.r == n
    e = rg_ref.stability_factor(np.array(st.Ap), ref, A)
    res = rg_ref.residual_error(np.array(st.Ap), A)
    assert g["e_rank_greville"][k] / 30 <= e <= 30 * g["e_rank_greville"][k]
    assert g["res_rank_greville"][k] / 30 <= res <= 30 * g["res_rank_greville"][k]


@pytest.mark.parametrize("k", range(7))
def test_kahan_kappa_and_oracle_residual(k):
    g = GOLD["kahan"]
    c = g["c"][k]
    K = W.kahan(g["n"], c)
    assert _close3(np.linalg.cond(K), g["kappa"][k]) or k >= 5  # past 1e16 the FP64 SVD itself is approximate
    if k < 4:
        st = rg_ref.solve_stream(K.tolist(), [0.0] * g["n"], eps=1e-25, track_pinv=True)
        assert st.r == g["n"]
        res = rg_ref.residual_error(np.array(st.Ap), K)
        assert g["res_rank_greville"][k] / 30 <= res <= 30 * g["res_rank_greville"][k]


def test_kahan_definition_small():
    """K(c, s) for n = 3 written out: rows s^i (e_i - c sum_{j>i} e_j)."""
    c = 0.6
    s = 0.8
    K = W.kahan(3, c)
    want = np.array([[1.0, -c, -c], [0.0, s, -c * s], [0.0, 0.0, s * s]])
    assert np.allclose(K, want, rtol=0, atol=1e-15)
