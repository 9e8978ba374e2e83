"""Kernel size classes and placement rules: the host-side calls (no GPU) and,
on the GPU, streams forced into larger classes than the default one still
match the oracle."""
import numpy as np
import pytest

from oracle import ref_c
from paper_2106_11594_amd import workloads as W


def test_class_table_is_consistent():
    from paper_2106_11594_amd import rg
    n = rg.class_count()
    assert n >= 2
    shapes = [rg.class_info(c) for c in range(n)]
    for c, (rcap, mcap, threads) in enumerate(shapes):
        assert rcap > 0 and mcap > 0 and threads % 64 == 0
        assert not rg.class_fits(c, mcap + 1, 1)
        assert not rg.class_fits(c, mcap, rcap + 1)


def test_f64_class_shape():
    """The FP64 on-chip class follows the FP32 classes: rank capacity 64,
    m up to 128, 256 threads; it takes no placement rules."""
    from paper_2106_11594_amd import rg
    c = rg.class_count()
    assert rg.class_info(c) == (64, 128, 256)
    assert rg.class_fits(c, 128, 64) and rg.class_fits(c, 1, 1)
    assert not rg.class_fits(c, 129, 1) and not rg.class_fits(c, 64, 65)
    with pytest.raises(RuntimeError):
        rg.class_info(c + 1)
    with pytest.raises(RuntimeError):
        rg.set_class_rules([(64, 12, c)])


def test_class_rule_validation():
    from paper_2106_11594_amd import rg
    with pytest.raises(RuntimeError):
        rg.set_class_rules([(64, 12, rg.class_count())])
    with pytest.raises(RuntimeError):
        rg.set_class_rules([(64, 12, -2)])
    with pytest.raises(RuntimeError):
        rg.class_info(-1)
    rg.set_class_rules([(64, 12, 0), (256, 128, -1)])
    rg.set_class_rules([])


@pytest.mark.gpu
@pytest.mark.parametrize("cls", [0, 1, 2, 3, 5, 8, -1])
def test_forced_class_matches_oracle(cls):
    from paper_2106_11594_amd import rg
    from tests.gpu_util import run_batch
    if cls in (0, 1, 2):
        # the row-by-row classes hold r_max <= 12 (class 0): planted ranks 4..8
        rng = np.random.default_rng(50 + cls)
        streams, rs = [], []
        for b in range(12):
            m, r = int(rng.integers(16, 61)), int(rng.integers(4, 9))
            A = W.lowrank_rows(rng, m, r, int(rng.integers(m, 4 * m)))
            Y, _ = W.targets(rng, A)
            streams.append((A, Y.astype(np.float32).astype(np.float64)))
            rs.append(r)
        ms, ns, row_ptr, a_off, A, Y = W.pack(streams, 1e-3, "f32")
        bt = W.Batch(ms, np.array(rs, np.int32), ns, row_ptr, a_off, A, Y, 1e-3, "f32")
    else:
        bt = W.batched(B=12, m_lo=16, m_hi=60, n_scale=0.3, dtype="f32", seed=5)
    r_max = np.minimum(bt.ms, bt.rs + 4).astype(np.int32)
    if cls >= 0:
        assert all(rg.class_fits(cls, int(m), int(c)) for m, c in zip(bt.ms, r_max))
    rg.set_class_rules([(1 << 30, 1 << 30, cls)])
    try:
        xs, ranks, flags, h = run_batch(bt, "f32", r_max=r_max, eps=1e-3)
    finally:
        rg.set_class_rules([])
    Xo, xoff, ro, st, _ = ref_c.solve_batch(bt.ms, bt.row_ptr, bt.a_off, bt.A, bt.Y, eps=1e-3, caps=r_max)
    assert (flags == 0).all()
    for b in range(bt.B):
        assert ranks[b] == ro[b]
        xo = Xo[xoff[b]:xoff[b] + bt.ms[b]]
        assert np.linalg.norm(xs[b] - xo) <= 1e-5 * np.linalg.norm(xo), (cls, b)
