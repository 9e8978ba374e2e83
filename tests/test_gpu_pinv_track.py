"""rg_pinv_track: the pseudoinverse maintained row by row (Theorem 2 for
independent rows, Theorem 3 for dependent rows), against the oracle's
recursive A^+ (track_pinv) on the same seeded rows, the SVD pseudoinverse at
the planted rank and the four Penrose equations.

Tolerances (FP64 on both sides, same recursion, different summation order):
1e-9 relative in Frobenius norm for A^+ and x against the oracle, 1e-8 against
the SVD pseudoinverse (planted bases with condition numbers of order 10-100,
so n rows of rounding at 2^-52 stay far below either bound); rank exact."""
import numpy as np
import pytest

from oracle import rg_ref
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(seed, n, m, r, dup=False, zero=False):
    rng = np.random.default_rng(seed)
    A = W.lowrank_rows(rng, m, r, n)
    if dup and n > 4:
        A[n - 1] = A[1]
    if zero and n > 3:
        A[2] = 0.0
    Y, _ = W.targets(rng, A)
    return np.ascontiguousarray(A, dtype=np.float64), np.ascontiguousarray(Y, dtype=np.float64)


def _run(As, Ys, r_max=None):
    import torch
    from paper_2106_11594_amd import rg
    Ad = torch.from_numpy(np.stack(As)).cuda()
    Yd = torch.from_numpy(np.stack(Ys)).cuda()
    Ap, X, rank, flags = rg.pinv_track(Ad, Yd, r_max=r_max)
    torch.cuda.synchronize()
    return Ap.cpu().numpy(), X.cpu().numpy(), rank.cpu().numpy(), flags.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check_against_oracle(A, Y, Ap, X, rank, planted):
    st = rg_ref.solve_stream(A, Y, track_pinv=True)
    assert rank == st.r == planted
    assert _rel(Ap, np.array(st.Ap, dtype=np.float64).reshape(Ap.shape)) < 1e-9
    assert _rel(X, np.array(st.X)) < 1e-9
    ref = rg_ref.lstsq_svd(A, np.eye(A.shape[0]), rank=planted)
    assert _rel(Ap, ref) < 1e-8
    res = rg_ref.penrose_residuals(A, Ap)
    assert max(res) < 1e-8, res


def test_batch_vs_oracle_svd_penrose():
    n, m, r = 40, 12, 5
    probs = [_problem(11, n, m, r), _problem(12, n, m, r, dup=True), _problem(13, n, m, r, zero=True)]
    Ap, X, rank, flags = _run([p[0] for p in probs], [p[1] for p in probs])
    assert (flags == 0).all()
    for b, (A, Y) in enumerate(probs):
        _check_against_oracle(A, Y, Ap[b], X[b], rank[b], r)


@pytest.mark.parametrize("n,m,r", [(300, 64, 16), (80, 300, 20), (10, 30, 10), (50, 8, 8), (1, 5, 1)])
def test_shapes_vs_oracle(n, m, r):
    A, Y = _problem(100 + n + m, n, m, r, dup=True)
    Ap, X, rank, flags = _run([A], [Y])
    assert flags[0] == 0
    _check_against_oracle(A, Y, Ap[0], X[0], rank[0], int(np.linalg.matrix_rank(A)))


def test_no_rows():
    import torch
    from paper_2106_11594_amd import rg
    A = torch.zeros((2, 0, 6), dtype=torch.float64, device="cuda")
    Y = torch.zeros((2, 0), dtype=torch.float64, device="cuda")
    Ap, X, rank, flags = rg.pinv_track(A, Y, r_max=3)
    torch.cuda.synchronize()
    assert Ap.shape == (2, 6, 0)
    assert (rank.cpu() == 0).all() and (flags.cpu() == 0).all()
    assert (X.cpu() == 0).all()


def test_rank_capacity_and_nonfinite_flags():
    from paper_2106_11594_amd import rg
    A, Y = _problem(7, 30, 10, 5)
    _, _, rank, flags = _run([A], [Y], r_max=3)
    assert flags[0] == rg.FLAG_RANK_CAPACITY and rank[0] == 3
    A2 = A.copy()
    A2[9, 4] = np.nan
    st = rg_ref.solve_stream(A[:9], Y[:9])
    _, _, rank, flags = _run([A, A2], [Y, Y])
    assert flags[0] == 0 and rank[0] == 5
    assert flags[1] == rg.FLAG_NONFINITE and rank[1] == st.r
