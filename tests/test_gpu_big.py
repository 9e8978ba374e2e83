"""One large stream over the whole GPU (single-stream handles with m >= 512
that no on-chip class holds): the edge cases of the per-row kernel chain
against the oracle and against the one-workgroup generic kernel
(RG_OPT_GENERIC_KERNEL) on the same rows.

Tolerances: FP64 1e-11 relative; FP32 the bound used everywhere (1e-5 for
kappa(C) <= 1e3, else 0.1 kappa 2^-23)."""
import numpy as np
import pytest

from oracle import ref_c
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _tol(dtype, C):
    if dtype == "f64":
        return 1e-11
    kap = float(np.linalg.cond(C)) if C.shape[0] else 1.0
    return 1e-5 if kap <= 1e3 else 0.1 * kap * 2.0 ** -23


def _solve(A, Y, dtype, eps, r_max=None, chunks=None, flags=0):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float64 if dtype == "f64" else torch.float32
    At = torch.from_numpy(np.ascontiguousarray(A)).to("cuda", td)
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to("cuda", td)
    h = rg.Solver(A.shape[1], r_max=r_max, dtype=dtype, eps=eps, flags=flags)
    bounds = [0] + list(chunks or []) + [A.shape[0]]
    for c0, c1 in zip(bounds[:-1], bounds[1:]):
        if c1 > c0:
            h.push_rows(At[c0:c1].contiguous(), Yt[c0:c1].contiguous())
    x = h.solution().double().cpu().numpy()
    r, f = h.rank(), h.flags()
    h.close()
    return x, r, f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_big_vs_oracle_and_generic_with_incremental_pushes(dtype):
    s = W.large_stream(n=700, m=640, r=48, dtype=dtype, seed=11)
    chunks = [1, 2, 65, 130, 131, 400]  # pushes of 1 .. 269 rows
    xb, rb, fb = _solve(s.A, s.Y, dtype, s.eps, chunks=chunks)
    xg, rg_, fg = _solve(s.A, s.Y, dtype, s.eps, flags=0x2)
    xo, ro, Co, *_ = ref_c.solve(s.A, s.Y, eps=s.eps)
    tol = _tol(dtype, Co)
    print("%s: rank %d/%d/%d, big %.2e, generic %.2e" % (dtype, rb, rg_, ro, _rel(xb, xo), _rel(xg, xo)), flush=True)
    assert fb == fg == 0 and rb == rg_ == ro == 48
    assert _rel(xb, xo) <= tol and _rel(xg, xo) <= tol


def test_big_nonfinite_row_and_target():
    s = W.large_stream(n=300, m=512, r=32, dtype="f64", seed=12)
    A = s.A.copy()
    A[120, 7] = np.nan
    x, r, f = _solve(A, s.Y, "f64", s.eps)
    xo, ro, *_ = ref_c.solve(s.A[:120], s.Y[:120], eps=s.eps)
    assert f == 0x1 and r == ro
    assert _rel(x, xo) <= 1e-11
    Y = s.Y.copy()
    Y[40] = np.inf
    x, r, f = _solve(s.A, Y, "f64", s.eps, chunks=[17])
    xo, ro, *_ = ref_c.solve(s.A[:40], s.Y[:40], eps=s.eps)
    assert f == 0x1 and r == ro
    assert _rel(x, xo) <= 1e-11


def test_big_rank_capacity_and_zero_rows():
    rng = np.random.default_rng(13)
    A0 = W.lowrank_rows(rng, 600, 40, 260)  # the first 40 rows are independent
    Y0, _ = W.targets(rng, A0)
    x, r, f = _solve(A0, Y0, "f64", 1e-8, r_max=25)
    xo, ro, *_ = ref_c.solve(A0[:25], Y0[:25], eps=1e-8, cap=25)
    assert f == 0x2 and r == ro == 25  # row 25 is independent at r = r_max: flagged, nothing after it applied
    assert _rel(x, xo) <= 1e-11
    s = W.large_stream(n=260, m=600, r=40, dtype="f64", seed=13)
    A, Y = s.A.copy(), s.Y.copy()
    A[:5] = 0.0  # a zero first row (rank 0) and more zero rows
    Y[:5] = 0.0
    A[100:110] = 0.0
    Y[100:110] = 0.0
    x, r, f = _solve(A, Y, "f64", s.eps)
    xo, ro, *_ = ref_c.solve(A, Y, eps=s.eps)
    assert f == 0 and r == ro == 40
    assert _rel(x, xo) <= 1e-11
