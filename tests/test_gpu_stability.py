"""The pseudoinverse maintained row by row on the GPU (rg_pinv_track, FP64)
in the stability study of Section 4.2, and its multi-right-hand-side form.

Stability: for the Pascal matrices P(4..10) (default threshold), U S V^T
(5n x n, n = 10, 15, 20, eps 1e-8) and the Kahan matrices K(c, s) (n = 100,
c = 0.10 .. 0.25, eps 1e-25), the GPU's stability factor and residual error
(the measures of Section 4.2, computed by the oracle's functions) must be
within a factor 30 of the rank-Greville values the paper prints
(tests/golden/stability_tables.json) and of the oracle's FP64 run on the same
matrix; the rank must be full.  The factor 30 covers summation orders: the
paper's NumPy sums, the oracle's plain loops and the GPU's wave reductions
round differently, and these measures are amplified rounding errors.

Multiple right-hand sides: every column of X takes the same gain per row, so
a q-column run equals q one-column runs bit for bit; with Y = I_n the
solution is A^+ itself; a non-finite target in any column flags the problem.
"""
import json
import os

import numpy as np
import pytest

from oracle import rg_ref
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stability_tables.json")))


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _gpu_pinv(A, eps=None, Y=None):
    import torch
    from paper_2106_11594_amd import rg
    n = A.shape[0]
    Yt = torch.zeros(n, dtype=torch.float64) if Y is None else torch.from_numpy(np.ascontiguousarray(Y))
    Ap, X, rank, flags = rg.pinv_track(torch.from_numpy(np.ascontiguousarray(A)).cuda(), Yt.cuda(), eps=eps)
    torch.cuda.synchronize()
    return Ap.cpu().numpy(), X.cpu().numpy(), int(rank.cpu()), int(flags.cpu())


def _within(v, ref, f=30.0):
    return ref / f <= v <= ref * f


@pytest.mark.parametrize("k", range(4))
def test_pascal(k):
    g = GOLD["pascal"]
    n = g["n"][k]
    P = W.pascal(n)
    ex = rg_ref.solve_stream(P.tolist(), [0] * n, exact=True, track_pinv=True)
    Pinv = np.array([[float(v) for v in row] for row in ex.Ap])
    Ap, _, rank, flags = _gpu_pinv(P)
    st = rg_ref.solve_stream(P.tolist(), [0.0] * n, track_pinv=True)
    e, res = rg_ref.stability_factor(Ap, Pinv, P), rg_ref.residual_error(Ap, P)
    e_o, res_o = rg_ref.stability_factor(np.array(st.Ap), Pinv, P), rg_ref.residual_error(np.array(st.Ap), P)
    print("Pascal n=%d: e %.3g (oracle %.3g, paper %.3g), res %.3g (oracle %.3g, paper %.3g)"
          % (n, e, e_o, g["e_rank_greville"][k], res, res_o, g["res_rank_greville"][k]), flush=True)
    assert flags == 0 and rank == n
    assert _within(e, g["e_rank_greville"][k]) and _within(e, e_o)
    assert _within(res, g["res_rank_greville"][k]) and _within(res, res_o)


@pytest.mark.parametrize("k", range(3))
def test_usv(k):
    g = GOLD["usv"]
    n = g["n"][k]
    A, U, S, V = W.usv(n, g["rows_per_col"])
    ref = (V / S) @ U.T
    Ap, _, rank, flags = _gpu_pinv(A, eps=g["eps"])
    st = rg_ref.solve_stream(A.tolist(), [0.0] * A.shape[0], eps=g["eps"], track_pinv=True)
    e, res = rg_ref.stability_factor(Ap, ref, A), rg_ref.residual_error(Ap, A)
    e_o, res_o = rg_ref.stability_factor(np.array(st.Ap), ref, A), rg_ref.residual_error(np.array(st.Ap), A)
    print("USV n=%d: e %.3g (oracle %.3g, paper %.3g), res %.3g (oracle %.3g, paper %.3g)"
          % (n, e, e_o, g["e_rank_greville"][k], res, res_o, g["res_rank_greville"][k]), flush=True)
    assert flags == 0 and rank == n
    assert _within(e, g["e_rank_greville"][k]) and _within(e, e_o)
    assert _within(res, g["res_rank_greville"][k]) and _within(res, res_o)


@pytest.mark.parametrize("k", range(4))
def test_kahan(k):
    g = GOLD["kahan"]
    c, n = g["c"][k], g["n"]
    K = W.kahan(n, c)
    Ap, _, rank, flags = _gpu_pinv(K, eps=1e-25)
    st = rg_ref.solve_stream(K.tolist(), [0.0] * n, eps=1e-25, track_pinv=True)
    res, res_o = rg_ref.residual_error(Ap, K), rg_ref.residual_error(np.array(st.Ap), K)
    print("Kahan c=%.2f: res %.3g (oracle %.3g, paper %.3g)" % (c, res, res_o, g["res_rank_greville"][k]),
          flush=True)
    assert flags == 0 and rank == n
    assert _within(res, g["res_rank_greville"][k]) and _within(res, res_o)


def test_multiple_rhs_equal_single_columns_and_identity_gives_pinv():
    import torch
    from paper_2106_11594_amd import rg
    rng = np.random.default_rng(3)
    B, n, m, r, q = 4, 60, 24, 9, 5
    A = np.stack([W.lowrank_rows(rng, m, r, n) for _ in range(B)])
    A[1, 7] = A[1, 2]
    Y = rng.standard_normal((B, n, q))
    Ad = torch.from_numpy(A).cuda()
    Ap, X, rank, flags = rg.pinv_track(Ad, torch.from_numpy(Y).cuda())
    torch.cuda.synchronize()
    assert (flags.cpu() == 0).all() and (rank.cpu() == r).all()
    Xn = X.cpu().numpy()
    assert Xn.shape == (B, m, q)
    for c in range(q):
        _, Xc, _, _ = rg.pinv_track(Ad, torch.from_numpy(np.ascontiguousarray(Y[:, :, c])).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(Xc.cpu().numpy(), Xn[:, :, c]), c
    # against the oracle: X = A^+ Y with A^+ from the oracle's FP64 run
    for b in range(B):
        st = rg_ref.solve_stream(A[b].tolist(), [0.0] * n, track_pinv=True)
        ref = np.array(st.Ap) @ Y[b]
        assert np.linalg.norm(Xn[b] - ref) <= 1e-9 * np.linalg.norm(ref), b
    # Y = I_n: the solution is the pseudoinverse
    I = torch.eye(n, dtype=torch.float64).expand(B, n, n).contiguous().cuda()
    Ap2, X2, _, _ = rg.pinv_track(Ad, I)
    torch.cuda.synchronize()
    assert np.allclose(X2.cpu().numpy(), Ap2.cpu().numpy(), rtol=1e-11, atol=1e-13)
    # a non-finite target in one column flags the problem
    Y2 = Y.copy()
    Y2[2, 30, 3] = np.nan
    _, _, rank3, flags3 = rg.pinv_track(Ad, torch.from_numpy(Y2).cuda())
    torch.cuda.synchronize()
    f3 = flags3.cpu().numpy()
    assert f3[2] == rg.FLAG_NONFINITE and (np.delete(f3, 2) == 0).all()
