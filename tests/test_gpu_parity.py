"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
  FP64 streams: same decisions (rank and the accepted rows C, compared bit for
    bit), x within 1e-11 relative.  Both sides run Algorithm 1 in IEEE double;
    only summation order and the coordinate form x = Ct^T w differ, which moves
    x by a few ulps times the condition of the basis (kappa(C) <= ~1e3 here).
  FP32 streams: same decisions (rank and C bit for bit: C holds raw input
    rows, exactly representable).  In the blocked on-chip classes (dual basis
    in factored form H^-1 C with H^-1 = (C C^T)^-1 in FP64) x is within
    max(1e-5, kappa(C)^2 2^-52) relative (tests/gpu_util.f32_tol): the
    projections are FP64 arithmetic on exact rows, perturbed by about
    2^-52 kappa(C)^2, and x is rounded to FP32 on output.  Streams too large
    for them (capacity above 128 or m above 256) run in the generic kernel
    with an explicit FP32 dual basis: 1e-5 for kappa(C) <= 1e3, else
    0.1 kappa(C) 2^-23.
"""
import json
import os

import numpy as np
import pytest

from oracle import ref_c
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -23


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ref_c.build()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0)


def _f32_tol(C, m=None, r_max=None):
    from tests.gpu_util import f32_tol, factored
    return f32_tol(C, factored=True if m is None else factored(m, r_max))


def _single(A, Y, dtype, eps=None, r_max=None, chunks=None, flags=0):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float32 if dtype == "f32" else torch.float64
    s = rg.Solver(A.shape[1], r_max=r_max, dtype=dtype, eps=eps, flags=flags)
    At = torch.from_numpy(np.ascontiguousarray(A)).to("cuda", td)
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to("cuda", td)
    bounds = chunks or [0, A.shape[0]]
    for a, b in zip(bounds[:-1], bounds[1:]):
        s.push_rows(At[a:b].contiguous(), Yt[a:b].contiguous())
    x = s.solution().double().cpu().numpy()
    return x, s


def _state(s_or_batch, b=0):
    from paper_2106_11594_amd import rg
    st = s_or_batch.get_state() if isinstance(s_or_batch, rg.Solver) else s_or_batch.get_state(b)
    return [t.double().cpu().numpy() for t in st]


@pytest.mark.parametrize("n", [700, 2000])
def test_single_f64_vs_oracle(n):
    s = W.single_f64(n=n)
    x, h = _single(s.A, s.Y, "f64", eps=s.eps)
    xo, ro, Co, Cto, Po = ref_c.solve(s.A, s.Y, eps=s.eps)
    assert h.rank() == ro == 16 and h.flags() == 0
    C, Ct, P, w = _state(h)
    assert np.array_equal(C, Co)
    assert _rel(x, xo) <= 1e-12  # the plain FP64 stream's bar
    assert _rel(Ct, Cto) <= 1e-10 and _rel(P, Po) <= 1e-10


def test_single_f64_default_eps():
    s = W.single_f64(n=500, m=48, r=12, seed=3)
    x, h = _single(s.A, s.Y, "f64")
    xo, ro, *_ = ref_c.solve(s.A, s.Y, eps=-1.0)
    assert h.rank() == ro == 12
    assert _rel(x, xo) <= 1e-11


@pytest.mark.parametrize("seed", [0, 1])
def test_single_f32_vs_oracle(seed):
    s = W.single_f64(n=1200, m=96, r=24, seed=seed)
    A32 = s.A.astype(np.float32).astype(np.float64)
    Y32 = s.Y.astype(np.float32).astype(np.float64)
    x, h = _single(A32, Y32, "f32", eps=1e-3)
    xo, ro, Co, *_ = ref_c.solve(A32, Y32, eps=1e-3)
    assert h.rank() == ro == 24 and h.flags() == 0
    C, *_ = _state(h)
    assert np.array_equal(C, Co)
    tol, kap = _f32_tol(Co, 96, 96)
    assert _rel(x, xo) <= tol, (kap, _rel(x, xo))


def test_worked_example_f64():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_m2.json")))
    A = np.array(g["rows"], float)
    Y = np.array(g["y"], float)
    x, h = _single(A, Y, "f64", eps=1e-12)
    assert h.rank() == 2
    assert np.allclose(x, [20 / 11, 12 / 11], rtol=1e-14, atol=1e-15)
    C, Ct, P, w = _state(h)
    assert np.array_equal(C, [[1, 0], [1, 1]])
    assert np.allclose(Ct, [[1, -1], [0, 1]], atol=1e-15)
    assert np.allclose(P, np.array([[2, 1], [1, 6]]) / 11, atol=1e-15)
    assert np.allclose(w, [20 / 11, 32 / 11], atol=1e-14)


def test_min_norm_example():
    x, h = _single(np.array([[1, 1, 0], [2, 2, 0]], float), np.array([2.0, 2.0]), "f64", eps=1e-12)
    assert h.rank() == 1
    assert np.allclose(x, [0.6, 0.6, 0.0], rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_edge_cases(dtype):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float32 if dtype == "f32" else torch.float64
    # k = 0 push and the empty state
    s = rg.Solver(5, dtype=dtype)
    s.push_rows(torch.empty((0, 5), device="cuda", dtype=td), torch.empty(0, device="cuda", dtype=td))
    assert s.rank() == 0 and np.all(s.solution().cpu().numpy() == 0)
    # zero rows are no-ops
    x, h = _single(np.zeros((4, 5)), np.arange(4.0), dtype)
    assert h.rank() == 0 and np.all(x == 0) and h.flags() == 0
    # m = 1
    x, h = _single(np.array([[2.0], [0.0], [-1.0]]), np.array([4.0, 3.0, 1.0]), dtype, eps=1e-6)
    assert h.rank() == 1 and abs(x[0] - (8.0 - 1.0) / 5.0) < 1e-6
    # single row closed form x = Gamma y / ||Gamma||^2
    G = np.array([[3.0, -1.0, 2.0, 0.5]])
    x, h = _single(G, np.array([7.0]), dtype)
    assert h.rank() == 1 and np.allclose(x, G[0] * 7.0 / (G[0] @ G[0]), rtol=1e-6)
    # full column rank: normal equations
    rng = np.random.default_rng(4)
    A = rng.integers(-4, 5, size=(40, 6)).astype(float)
    Y = rng.integers(-9, 9, size=40).astype(float)
    x, h = _single(A, Y, dtype, eps=1e-4 if dtype == "f32" else 1e-10)
    assert h.rank() == 6
    assert _rel(x, np.linalg.solve(A.T @ A, A.T @ Y)) <= (1e-5 if dtype == "f32" else 1e-12)
    # exact duplicates only
    x, h = _single(np.tile([[1.0, 2.0, 2.0]], (5, 1)), np.arange(5.0), dtype)
    assert h.rank() == 1 and np.allclose(x, np.array([1, 2, 2]) * 2.0 / 9.0, rtol=1e-6)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sticky_flags(dtype):
    from paper_2106_11594_amd import rg
    s = W.single_f64(n=60, m=16, r=6)
    # rank capacity: r_max = 3 < rank 6
    x, h = _single(s.A, s.Y, dtype, r_max=3)
    assert h.rank() == 3 and h.flags() == rg.FLAG_RANK_CAPACITY
    # a NaN row stops the stream; rows before it stay applied
    A = s.A.copy()
    A[30, 2] = np.nan
    x, h = _single(A, s.Y, dtype)
    assert h.flags() == rg.FLAG_NONFINITE
    x2, h2 = _single(s.A[:30], s.Y[:30], dtype)
    assert h.rank() == h2.rank() and np.array_equal(x, x2)
    # reset clears the flag; the state is empty again
    h.reset()
    assert h.flags() == 0 and h.rank() == 0
    Y = s.Y.copy()
    Y[5] = np.inf
    x, h = _single(s.A, Y, dtype)
    assert h.flags() == rg.FLAG_NONFINITE


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_incremental_equals_one_push_and_deterministic(dtype):
    """Pushing the rows in pieces gives the one-push result: with blocks,
    which end at a push boundary, up to rounding; bit for bit when every row
    is taken alone (RG_OPT_ROW_BY_ROW).  Repeating a push sequence repeats
    the bits."""
    from paper_2106_11594_amd import rg
    s = W.single_f64(n=900, m=80, r=20, seed=9)
    chunks = [0, 1, 17, 300, 301, 900]
    x1, h1 = _single(s.A, s.Y, dtype)
    x2, h2 = _single(s.A, s.Y, dtype, chunks=chunks)
    x3, h3 = _single(s.A, s.Y, dtype)
    assert h1.rank() == h2.rank() == h3.rank() == 20
    assert np.array_equal(x1, x3)
    assert _rel(x2, x1) <= (1e-11 if dtype == "f64" else 1e-5)
    xa, _ = _single(s.A, s.Y, dtype, flags=rg.OPT_ROW_BY_ROW)
    xb, _ = _single(s.A, s.Y, dtype, chunks=chunks, flags=rg.OPT_ROW_BY_ROW)
    assert np.array_equal(xa, xb)


def _batch_check(bt, dtype, eps, flags=0):
    from tests.gpu_util import run_batch
    xs, ranks, fl, h = run_batch(bt, dtype, eps=eps, flags=flags)
    assert (fl == 0).all()
    Xo, xoff, ro, st, _ = ref_c.solve_batch(bt.ms, bt.row_ptr, bt.a_off, bt.A, bt.Y, eps=eps, nthreads=8)
    assert (st == 0).all()
    worst = 0.0
    for b in range(bt.B):
        A, Y = bt.stream(b)
        assert ranks[b] == ro[b] == min(int(bt.rs[b]), A.shape[0]), b
        xo = Xo[xoff[b]:xoff[b] + bt.ms[b]]
        if dtype == "f64":
            assert _rel(xs[b], xo) <= 1e-11, b
        else:
            _, _, Co, *_ = ref_c.solve(A, Y, eps=eps)
            C, *_ = _state(h, b)
            assert np.array_equal(C, Co), b
            tol, kap = _f32_tol(Co, bt.ms[b], bt.ms[b])  # default capacity r_max = m
            assert _rel(xs[b], xo) <= tol, (b, kap, _rel(xs[b], xo))
        worst = max(worst, _rel(xs[b], xo))
    return worst


def test_batched_f32_vs_oracle():
    bt = W.batched(B=48, n_scale=0.3, dtype="f32")
    _batch_check(bt, "f32", 1e-3)


def test_batched_f64_vs_oracle():
    bt = W.batched(B=32, m_hi=160, n_scale=0.3, dtype="f64")
    _batch_check(bt, "f64", 1e-8)


def test_batched_generic_kernel_matches():
    from paper_2106_11594_amd import rg
    bt = W.batched(B=24, n_scale=0.25, dtype="f32", seed=1)
    _batch_check(bt, "f32", 1e-3, flags=rg.OPT_GENERIC_KERNEL)


def test_batched_largest_classes():
    """Shapes at the top of the on-chip kernel's range (m = 256 with ranks up
    to 128 and capacities up to 132), checked against the oracle."""
    from paper_2106_11594_amd import rg
    from tests.gpu_util import to_device
    shapes = [(256, 128, 300, 132), (256, 120, 260, 128), (200, 96, 240, 100), (64, 30, 90, 34)]
    streams = []
    for idx, (m, r, n, _) in enumerate(shapes):
        rng = np.random.default_rng(100 + idx)
        A = W.lowrank_rows(rng, m, r, n)
        Y, _ = W.targets(rng, A)
        streams.append((A, Y.astype(np.float32).astype(np.float64)))
    ms, ns, row_ptr, a_off, A, Y = W.pack(streams, 1e-3, "f32")
    bt = W.Batch(ms, np.array([s[1] for s in shapes], np.int32), ns, row_ptr, a_off, A, Y, 1e-3, "f32")
    caps = np.array([s[3] for s in shapes], np.int32)
    Ad, Yd, rp, ao = to_device(bt, "f32")
    h = rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3)
    h.push(Ad, Yd, rp, ao)
    x = h.solution().double().cpu().numpy()
    ranks, fl = h.rank(), h.flags()
    for b, (m, r, n, cap) in enumerate(shapes):
        Ab, Yb = bt.stream(b)
        xo, ro, Co, *_ = ref_c.solve(Ab, Yb, eps=1e-3, cap=cap)
        assert fl[b] == 0 and ranks[b] == ro == r
        C, *_ = _state(h, b)
        assert np.array_equal(C, Co)
        tol, kap = _f32_tol(Co, m, cap)
        assert _rel(x[h.x_off[b]:h.x_off[b] + m], xo) <= tol, (b, kap)
