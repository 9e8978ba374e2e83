"""Pins of the oracle's orthogonal rank factorization variants (Section 2.2).

orthogonal (alpha = 1) stays rational, so it is pinned exactly: over
Fractions it must give the exact minimum-norm least-squares solution and
rank of the independent row-space solver, the same decisions as the base
factorization, mutually orthogonal rows of C, Ct C^T = I and
Pinv (B^T B) = I with B = A Ct^T after every row.  orthonormal
(alpha = 1 / ||Gamma_r||) takes square roots, so it is pinned in FP64: C C^T = I,
Ct = C, Pinv (B^T B) = I, and x equal to the base run and to the truncated SVD
solution.  Mistakes planted in a copy of the variant branch must trip these
pins.
"""
import inspect
import random
import types
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import rg_ref
from tests.test_oracle_exact import _planted


def _bt_b(A, st):
    m, k = st.m, st.r
    B = [[sum(row[j] * st.Ct[a][j] for j in range(m)) for a in range(k)] for row in A]
    return [[sum(B[t][a] * B[t][b] for t in range(len(A))) for b in range(k)] for a in range(k)]


@pytest.mark.parametrize("seed", range(30))
def test_orthogonal_fraction_equals_exact_solver(seed):
    rng = random.Random(5000 + seed)
    m = rng.randint(1, 7)
    n = rng.randint(1, 18)
    r = rng.randint(1, min(m, 5))
    A, Y = _planted(rng, n, m, r)
    st = rg_ref.solve_stream(A, Y, exact=True, variant="orthogonal")
    base = rg_ref.solve_stream(A, Y, exact=True)
    x, rank = rg_ref.lstsq_exact(A, Y)
    assert st.r == rank and st.X == x
    assert st.decisions == base.decisions


@pytest.mark.parametrize("seed", range(10))
def test_orthogonal_invariants_after_every_row(seed):
    rng = random.Random(6000 + seed)
    m, n, r = rng.randint(2, 6), rng.randint(4, 14), rng.randint(1, 4)
    A, Y = _planted(rng, n, m, min(r, m))
    st = rg_ref.RGState(m, F(0), "orthogonal")
    for i in range(n):
        rg_ref.update_least_squares(st, [F(v) for v in A[i]], F(Y[i]), 0)
        k = st.r
        for a in range(k):
            assert sum(st.C[a][j] * st.C[a][j] for j in range(m)) > 0
            for b in range(k):
                if a != b:
                    assert sum(st.C[a][j] * st.C[b][j] for j in range(m)) == 0
                assert sum(st.Ct[a][j] * st.C[b][j] for j in range(m)) == (1 if a == b else 0)
        Ai = [[F(v) for v in row] for row in A[:i + 1]]
        BtB = _bt_b(Ai, st)
        for a in range(k):
            for b in range(k):
                assert sum(st.Pinv[a][c] * BtB[c][b] for c in range(k)) == (1 if a == b else 0)


def _orthonormal_pins(mod, seeds=range(4)):
    """FP64 pins of the orthonormal variant against module ``mod``; returns the
    worst deviations (x vs base, x vs SVD, C C^T - I, Ct - C, Pinv B^T B - I)."""
    from paper_2106_11594_amd import workloads as W
    worst = np.zeros(5)
    for seed in seeds:
        s = W.single_f64(n=90, m=20, r=6, seed=seed)
        A, Y = s.A.tolist(), s.Y.tolist()
        st = mod.solve_stream(A, Y, eps=1e-10, variant="orthonormal")
        base = rg_ref.solve_stream(A, Y, eps=1e-10)
        xs = rg_ref.lstsq_svd(s.A, s.Y, rank=6)
        C, Ct, P = np.array(st.C), np.array(st.Ct), np.array(st.Pinv)
        B = s.A @ Ct.T
        dev = [np.linalg.norm(np.array(st.X) - np.array(base.X)) / np.linalg.norm(base.X),
               np.linalg.norm(np.array(st.X) - xs) / np.linalg.norm(xs),
               np.abs(C @ C.T - np.eye(st.r)).max(),
               np.abs(Ct - C).max(),
               np.abs(P @ (B.T @ B) - np.eye(st.r)).max()]
        if st.r != 6:
            dev[0] = np.inf
        worst = np.maximum(worst, dev)
    return worst


def test_orthonormal_float_pins():
    worst = _orthonormal_pins(rg_ref)
    assert worst[0] <= 1e-11 and worst[1] <= 1e-10
    assert worst[2] <= 1e-13 and worst[3] <= 1e-13 and worst[4] <= 1e-9


def test_orthonormal_is_not_rational():
    with pytest.raises(ValueError):
        rg_ref.solve_stream([[1, 2]], [1], exact=True, variant="orthonormal")


VARIANT_MUTATIONS = {
    "border_sign": ("st.Pinv[i] + [-alpha * zeta[i]]", "st.Pinv[i] + [alpha * zeta[i]]"),
    "corner_no_alpha2": ("[alpha * alpha * ((z + 1) + gz)]", "[((z + 1) + gz)]"),
    "corner_no_one": ("[alpha * alpha * ((z + 1) + gz)]", "[alpha * alpha * gz]"),
    "dual_row_no_alpha": ("[v / (alpha * nrm2) for v in Gamma_r]", "[v / nrm2 for v in Gamma_r]"),
    "basis_raw_row": ("st.C.append([alpha * v for v in Gamma_r])", "st.C.append([alpha * v for v in Gamma])"),
    "alpha_squared_norm": ("(z + 1) / math.sqrt(nrm2)", "(z + 1) / nrm2"),
}


def _mutant(old, new):
    src = inspect.getsource(rg_ref)
    assert src.count(old) == 1, old
    mod = types.ModuleType("rg_ref_variant_mutant")
    exec(compile(src.replace(old, new), "rg_ref_variant_mutant", "exec"), mod.__dict__)
    return mod


def _orthogonal_exact_pin(mod):
    for seed in range(12):
        rng = random.Random(7000 + seed)
        m, n = rng.randint(2, 7), rng.randint(3, 18)
        A, Y = _planted(rng, n, m, rng.randint(1, min(m, 5)))
        try:
            st = mod.solve_stream(A, Y, exact=True, variant="orthogonal")
        except ZeroDivisionError:
            return False
        x, rank = rg_ref.lstsq_exact(A, Y)
        if st.r != rank or st.X != x:
            return False
    return True


@pytest.mark.parametrize("name", sorted(VARIANT_MUTATIONS))
def test_variant_mutation_is_caught(name):
    mod = _mutant(*VARIANT_MUTATIONS[name])
    exact_ok = _orthogonal_exact_pin(mod)
    w = _orthonormal_pins(mod, seeds=range(2))
    float_ok = w[0] <= 1e-11 and w[1] <= 1e-10 and w[2] <= 1e-13 and w[3] <= 1e-13 and w[4] <= 1e-9
    assert not (exact_ok and float_ok), name
