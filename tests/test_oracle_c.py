"""The plain FP64 C oracle against the pinned Python oracle and closed forms."""
import random
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import ref_c, rg_ref
from paper_2106_11594_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    ref_c.build()


@pytest.mark.parametrize("seed", range(6))
def test_c_matches_python_float(seed):
    """Same Algorithm 1 in C and in Python floats: identical decisions,
    results equal to rounding."""
    s = W.single_f64(n=150, m=20, r=5, seed=seed)
    x, r, C, Ct, P, dec = ref_c.solve(s.A, s.Y, eps=1e-10, decisions=True)
    st = rg_ref.solve_stream(s.A.tolist(), s.Y.tolist(), eps=1e-10)
    assert r == st.r == 5
    assert list(dec.astype(bool)) == st.decisions
    assert np.array_equal(C, np.array(st.C))
    assert np.allclose(x, st.X, rtol=1e-12, atol=1e-13)
    assert np.allclose(Ct, np.array(st.Ct), rtol=1e-10, atol=1e-12)
    assert np.allclose(P, np.array(st.Pinv), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("seed", range(10))
def test_c_matches_exact_solver(seed):
    rng = random.Random(seed)
    m, n = rng.randint(2, 7), rng.randint(3, 16)
    Wm = [[rng.randint(-3, 3) for _ in range(m)] for _ in range(rng.randint(1, m))]
    A = []
    for _ in range(n):
        z = [rng.randint(-2, 2) for _ in Wm]
        A.append([sum(z[k] * Wm[k][j] for k in range(len(Wm))) for j in range(m)])
    Y = [rng.randint(-9, 9) for _ in range(n)]
    x_ex, r_ex = rg_ref.lstsq_exact(A, Y)
    x, r, *_ = ref_c.solve(np.array(A, float), np.array(Y, float))
    assert r == r_ex
    xe = np.array([float(v) for v in x_ex])
    assert np.linalg.norm(x - xe) <= 1e-9 * max(1.0, np.linalg.norm(xe))


def test_c_default_eps_and_svd():
    s = W.single_f64(n=400, m=64, r=16)
    x, r, *_ = ref_c.solve(s.A, s.Y, eps=-1.0)
    assert r == 16
    xs = rg_ref.lstsq_svd(s.A, s.Y, rank=16)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_c_incremental_push_equals_one_push():
    s = W.single_f64(n=300, m=32, r=8)
    a = ref_c.Stream(32, eps=1e-10)
    a.push(s.A[:100], s.Y[:100])
    a.push(s.A[100:], s.Y[100:])
    b = ref_c.Stream(32, eps=1e-10)
    b.push(s.A, s.Y)
    assert a.rank == b.rank
    assert np.array_equal(a.x, b.x)


def test_c_capacity_overflow():
    s = W.single_f64(n=100, m=16, r=6)
    st = ref_c.Stream(16, cap=4, eps=1e-10)
    with pytest.raises(OverflowError):
        st.push(s.A, s.Y)
    assert st.rank == 4


def test_c_batch_matches_single():
    bt = W.batched(B=24, m_hi=48, n_scale=0.5, dtype="f64")
    X, x_off, rank, status, used = ref_c.solve_batch(bt.ms, bt.row_ptr, bt.a_off, bt.A, bt.Y, eps=1e-8,
                                                     nthreads=4)
    assert used >= 1 and (status == 0).all()
    for b in range(bt.B):
        A, Y = bt.stream(b)
        x, r, *_ = ref_c.solve(A, Y, eps=1e-8)
        assert r == rank[b] == min(bt.rs[b], A.shape[0])
        assert np.array_equal(x, X[x_off[b]:x_off[b] + bt.ms[b]])
