"""The blocked variant (rows applied up to 16 at a time on the matrix cores:
runs of dependent rows as one Woodbury update, runs of independent rows as
one block append) against the dependent-blocks-only path
(RG_OPT_DEPENDENT_BLOCKS_ONLY), the row-by-row path (RG_OPT_ROW_BY_ROW) and
the oracle, on stream shapes that use the blocked kernel's variants,
including the rows where a block has to stop: a row of the other kind inside
a block, a non-finite row, the rank capacity, zero rows, rows just on either
side of the rank threshold and ragged tails."""
import numpy as np
import pytest

from oracle import ref_c
from paper_2106_11594_amd import workloads as W

# (m, r_max) pairs that select each variant of the blocked kernel
VARIANT_SHAPES = [(100, 44), (120, 100), (170, 60), (190, 120), (250, 40), (256, 128)]


def _rel(x, xo):
    return float(np.linalg.norm(x - xo) / max(np.linalg.norm(xo), 1e-300))


def _kappa_tol(C):
    from tests.gpu_util import f32_tol
    return f32_tol(C, factored=True)


def _solve(A, Y, r_max, flags=0, chunks=None):
    import torch
    from paper_2106_11594_amd import rg
    Ad = torch.from_numpy(np.ascontiguousarray(A, np.float32)).cuda()
    Yd = torch.from_numpy(np.ascontiguousarray(Y, np.float32)).cuda()
    h = rg.Solver(A.shape[1], r_max=r_max, dtype="f32", eps=1e-3, flags=flags)
    bounds = [0] + list(chunks or []) + [A.shape[0]]
    for c0, c1 in zip(bounds[:-1], bounds[1:]):
        if c1 > c0:
            h.push_rows(Ad[c0:c1].contiguous(), Yd[c0:c1].contiguous())
    x = h.solution().double().cpu().numpy()
    r, f = h.rank(), h.flags()
    h.close()
    return x, r, f


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.gpu
@pytest.mark.parametrize("m,r_max", VARIANT_SHAPES)
def test_variant_blocked_vs_row_by_row_and_oracle(m, r_max):
    from paper_2106_11594_amd import rg
    rng = np.random.default_rng(m * 7 + r_max)
    r = r_max - 4
    A = W.lowrank_rows(rng, m, r, 3 * m + 37)  # ragged: not a multiple of 16 past the rank
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A), _f32(Y)
    xb, rb, fb = _solve(A, Y, r_max)
    xd, rd, fd = _solve(A, Y, r_max, flags=rg.OPT_DEPENDENT_BLOCKS_ONLY)
    xr, rr, fr = _solve(A, Y, r_max, flags=rg.OPT_ROW_BY_ROW)
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-3, cap=r_max)
    tol, kap = _kappa_tol(Co)
    print("m=%d r_max=%d: rank %d/%d/%d/%d, kappa %.3g, blocked %.2e, dependent blocks only %.2e, row-by-row %.2e, "
          "blocked vs row-by-row %.2e" % (m, r_max, rb, rd, rr, ro, kap, _rel(xb, xo), _rel(xd, xo), _rel(xr, xo),
                                          _rel(xb, xr)), flush=True)
    assert fb == fd == fr == 0
    assert rb == rd == rr == ro == r
    assert _rel(xb, xo) <= tol and _rel(xd, xo) <= tol and _rel(xr, xo) <= tol
    assert _rel(xb, xr) <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("m,r_max", [(150, 60), (240, 110)])
def test_copies_and_combinations_stop_blocks(m, r_max):
    """Copies and two-row combinations among fresh rows: independent rows
    land inside blocks, which must stop there."""
    from paper_2106_11594_amd import rg
    s = W.large_stream(n=4 * r_max, m=m, r=r_max - 6, p_dup=0.3, p_comb=0.2, dtype="f32")
    xb, rb, fb = _solve(s.A, s.Y, r_max, chunks=[37, 101])
    xr, rr, fr = _solve(s.A, s.Y, r_max, flags=rg.OPT_ROW_BY_ROW)
    xo, ro, Co, *_ = ref_c.solve(s.A, s.Y, eps=1e-3, cap=r_max)
    tol, kap = _kappa_tol(Co)
    assert fb == fr == 0 and rb == rr == ro
    assert _rel(xb, xo) <= tol and _rel(xr, xo) <= tol


@pytest.mark.gpu
def test_nonfinite_row_inside_a_block():
    rng = np.random.default_rng(11)
    A = W.lowrank_rows(rng, 180, 40, 150)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A).copy(), _f32(Y)
    A[97, 13] = np.nan  # past the rank, in the middle of a block
    x, r, f = _solve(A, Y, 48)
    xo, ro, *_ = ref_c.solve(A[:97], Y[:97], eps=1e-3, cap=48)
    assert f == 0x1 and r == ro == 40
    assert _rel(x, xo) <= 1e-5


@pytest.mark.gpu
def test_nonfinite_target_inside_a_block():
    rng = np.random.default_rng(12)
    A = W.lowrank_rows(rng, 200, 50, 160)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A), _f32(Y).copy()
    Y[120] = np.inf
    x, r, f = _solve(A, Y, 64)
    xo, ro, *_ = ref_c.solve(A[:120], Y[:120], eps=1e-3, cap=64)
    assert f == 0x1 and r == ro == 50
    assert _rel(x, xo) <= 1e-5


@pytest.mark.gpu
def test_rank_capacity_in_blocked_variant():
    rng = np.random.default_rng(13)
    A = W.lowrank_rows(rng, 200, 90, 200)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A), _f32(Y)
    x, r, f = _solve(A, Y, 70)
    xo, ro, *_ = ref_c.solve(A[:70], Y[:70], eps=1e-3, cap=70)
    assert f == 0x2 and r == 70
    assert _rel(x, xo) <= 1e-5


@pytest.mark.gpu
def test_zero_rows_and_incremental_pushes():
    rng = np.random.default_rng(14)
    A = W.lowrank_rows(rng, 130, 30, 200)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A).copy(), _f32(Y).copy()
    A[60:75] = 0.0
    Y[60:75] = 0.0
    x1, r1, f1 = _solve(A, Y, 40)
    x2, r2, f2 = _solve(A, Y, 40, chunks=[1, 31, 32, 47, 63, 64, 150, 199])
    xo, ro, *_ = ref_c.solve(A, Y, eps=1e-3, cap=40)
    assert f1 == f2 == 0 and r1 == r2 == ro == 30
    assert _rel(x1, xo) <= 1e-5 and _rel(x2, xo) <= 1e-5


@pytest.mark.gpu
@pytest.mark.parametrize("m,r_max", [(120, 50), (200, 100)])
def test_nonfinite_row_among_independent_rows(m, r_max):
    """A NaN inside the run of independent rows: the block append stops before
    it, the rows before it are applied, the stream is flagged."""
    rng = np.random.default_rng(m + 21)
    A = W.lowrank_rows(rng, m, r_max - 4, 2 * m)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A).copy(), _f32(Y)
    A[21, 5] = np.nan  # inside the second block of independent rows
    x, r, f = _solve(A, Y, r_max)
    xo, ro, *_ = ref_c.solve(A[:21], Y[:21], eps=1e-3, cap=r_max)
    assert f == 0x1 and r == ro == 21
    assert _rel(x, xo) <= 1e-5


@pytest.mark.gpu
def test_zero_and_repeated_rows_among_independent_rows():
    """Zero rows and exact copies inside the run of independent rows end the
    block append; the dependent rows between runs go through the Woodbury
    blocks; the rank and solution follow the oracle."""
    rng = np.random.default_rng(31)
    A = W.lowrank_rows(rng, 180, 60, 300)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A).copy(), _f32(Y).copy()
    A[5:9] = 0.0
    Y[5:9] = 0.0
    A[20] = A[3]
    A[33] = A[17]
    x, r, f = _solve(A, Y, 64)
    xr, rr, fr = _solve(A, Y, 64, flags=0x8)
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-3, cap=64)
    tol, _ = _kappa_tol(Co)
    assert f == fr == 0 and r == rr == ro == 60
    assert _rel(x, xo) <= tol and _rel(xr, xo) <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("delta,indep", [(1e-2, True), (1e-5, False)])
def test_rows_either_side_of_the_rank_threshold(delta, indep):
    """Early rows that are a combination of earlier rows plus a perturbation of
    relative size delta: 1e-2 is independent and 1e-5 dependent at eps 1e-3,
    wherever the row falls in a block."""
    rng = np.random.default_rng(41)
    m, r0 = 150, 40
    A = W.lowrank_rows(rng, m, r0, 200)
    A = A.copy()
    for k in (7, 18, 30):  # inside the first, second and third blocks
        comb = A[k - 3] - 0.5 * A[k - 5]
        e = rng.standard_normal(m)
        A[k] = comb + delta * np.linalg.norm(comb) * e / np.linalg.norm(e)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A), _f32(Y)
    from paper_2106_11594_amd import rg
    x, r, f = _solve(A, Y, 64)
    xr, rr, fr = _solve(A, Y, 64, flags=rg.OPT_ROW_BY_ROW)
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-3, cap=64)
    kap = float(np.linalg.cond(Co))
    print("delta %.0e: rank %d/%d/%d, kappa %.3g, blocked %.2e, row-by-row %.2e"
          % (delta, r, rr, ro, kap, _rel(x, xo), _rel(xr, xo)), flush=True)
    assert f == fr == 0 and r == rr == ro
    assert (r > r0) == indep
    # Rows 1e-2 from the span of the earlier ones raise kappa(C) to a few
    # hundred, well inside the range where the factored dual basis holds 1e-5.
    assert _rel(x, xo) <= 1e-5 and _rel(xr, xo) <= 1e-5


@pytest.mark.gpu
@pytest.mark.parametrize("m,cap", [(100, 37), (250, 120)])
def test_rank_fills_the_capacity_exactly(m, cap):
    """The planted rank equals the capacity: the last block append ends exactly
    at r_max and no flag is raised; the later (dependent) rows apply."""
    rng = np.random.default_rng(m + cap)
    A = W.lowrank_rows(rng, m, cap, cap + 90)
    Y, _ = W.targets(rng, A)
    A, Y = _f32(A), _f32(Y)
    x, r, f = _solve(A, Y, cap)
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-3, cap=cap)
    tol, _ = _kappa_tol(Co)
    assert f == 0 and r == ro == cap
    assert _rel(x, xo) <= tol


@pytest.mark.gpu
def test_persistent_grid_equals_one_workgroup_per_stream():
    """The persistent grid (workgroups taking streams from a queue) and one
    workgroup per stream run the same per-stream arithmetic: bit-equal x,
    equal ranks and flags, on a batch that covers every blocked variant."""
    from paper_2106_11594_amd import rg
    from tests.gpu_util import run_batch
    bt = W.batched(B=160, n_scale=0.3, dtype="f32", seed=11)
    caps = np.minimum(bt.ms, np.minimum(bt.rs + 4, 128)).astype(np.int32)
    xa, ra, fa, ha = run_batch(bt, "f32", r_max=caps, eps=1e-3)
    xb, rb, fb, hb = run_batch(bt, "f32", r_max=caps, eps=1e-3, flags=rg.OPT_ONE_WG_PER_STREAM)
    assert len(set(ha.classes()) & {3, 4, 5, 6, 7, 8}) >= 4
    assert (ra == rb).all() and (fa == fb).all() and (fa == 0).all()
    for b in range(bt.B):
        assert np.array_equal(xa[b], xb[b]), b


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_certified_skip_vs_explicit_rejections(dtype):
    """Blocks whose rows are all dependent beyond doubt (the bound on
    ||Gamma||^2 - gamma^T v below the threshold with its rounding error
    included) skip the explicit rejections; RG_OPT_EXPLICIT_REJECTIONS forms
    them anyway.  On 49 streams of the batched workload, most of whose rows
    come after the rank has filled, both give the oracle's rank and x within
    rounding of each other and within the factored form's bound of the
    oracle."""
    from paper_2106_11594_amd import rg
    from tests.gpu_util import run_batch
    bt = W.batched(streams=np.arange(7, 4096, 85), dtype=dtype)
    xs, r1, f1, _ = run_batch(bt, dtype)
    xe, r2, f2, _ = run_batch(bt, dtype, flags=rg.OPT_EXPLICIT_REJECTIONS)
    assert (f1 == 0).all() and (f2 == 0).all()
    worst = between = 0.0
    for k in range(bt.B):
        A, Y = bt.stream(k)
        xo, ro, Co, *_ = ref_c.solve(A, Y, eps=bt.eps)
        assert r1[k] == r2[k] == ro, k
        tol = _kappa_tol(Co)[0] if dtype == "f32" else max(1e-11, float(np.linalg.cond(Co)) ** 2 * 2.0 ** -52)
        e1, e2, eb = _rel(xs[k], xo), _rel(xe[k], xo), _rel(xs[k], xe[k])
        assert e1 <= tol and e2 <= tol, (k, e1, e2, tol)
        assert eb <= tol, (k, eb)
        worst, between = max(worst, e1, e2), max(between, eb)
    print("%s: worst vs oracle %.2e, between the modes %.2e" % (dtype, worst, between), flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("m,r", [(240, 72), (240, 88), (180, 88), (240, 104)])
def test_rank_tiles_split_over_simds(m, r):
    """Streams whose rank fills 5 (r = 72) or 6 (r = 88) row tiles of 16 in the
    RMAX = 128 variants: the waves past the last tile take pieces of the inner
    dimension of V = Gamma C^T and G = V H^-1, which meet in LDS; 7 tiles
    (r = 104) are not split.  Six streams per case, blocked against row by
    row and against the FP64 oracle: ranks exact, x within the FP32 bound."""
    from paper_2106_11594_amd import rg
    from tests.gpu_util import run_batch
    rng = np.random.default_rng(1000 * m + r)
    streams = []
    for k in range(6):
        A = _f32(W.lowrank_rows(rng, m, r, 3 * m + 37 + 11 * k))
        Y, _ = W.targets(rng, A)
        streams.append((A, _f32(Y)))
    ms, ns, row_ptr, a_off, Ap, Yp = W.pack(streams, 1e-3, "f32")
    bt = W.Batch(ms, np.full(6, r, np.int32), ns, row_ptr, a_off, Ap, Yp, 1e-3, "f32", {})
    r_max = np.full(6, r + 4, np.int32)
    xb, rb, fb, hb = run_batch(bt, "f32", r_max=r_max, eps=1e-3)
    cls = hb.classes()
    hb.close()
    assert all(rg.class_info(int(c))[0] == 128 for c in cls), cls  # an RMAX = 128 variant
    xr, rr, fr, hr = run_batch(bt, "f32", r_max=r_max, eps=1e-3, flags=rg.OPT_ROW_BY_ROW)
    hr.close()
    assert (fb == 0).all() and (fr == 0).all()
    for b, (A, Y) in enumerate(streams):
        xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-3, cap=r + 4)
        tol, kap = _kappa_tol(Co)
        assert rb[b] == rr[b] == ro == r, b
        assert _rel(xb[b], xo) <= tol and _rel(xr[b], xo) <= tol, (b, kap, _rel(xb[b], xo))
        assert _rel(xb[b], xr[b]) <= tol, b
