"""The boundary's contract on the GPU, through the C ABI:

  - the relative clause of the Section 3 rank test decides the same cases as
    in the oracle pins (tests/test_oracle_rank_test.py) in every kernel
    family: FP64 streams (generic kernel), FP32 small streams (row-by-row
    on-chip kernel), FP32 larger streams (blocked kernel, with and without
    blocks);
  - status codes: a flagged stream refuses pushes with RG_E_STATE once the host
    has seen the flag, rg_check / rg_batch_status map the flags to
    RG_E_NONFINITE, RG_E_RANK_CAPACITY; rg_reset clears them;
  - a caller-provided workspace gives the same results bit for bit as the
    library's own allocation and is rejected when too small or misaligned;
  - rg_batch_check_layout accepts a packed layout and rejects broken ones;
  - rg_pinv_track with eps = 0 (the exact test) on a small integer matrix
    with a zero row and an exact duplicate matches the oracle's exact
    rational run: rank exactly, A^+ and x to FP64 rounding.
"""
import numpy as np
import pytest

from oracle import rg_ref
from paper_2106_11594_amd import workloads as W
from tests import test_oracle_rank_test as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _pad(rows, m):
    out = np.zeros((len(rows), m))
    for i, row in enumerate(rows):
        out[i, :len(row)] = row
    return out


def _solver_rank(A, Y, dtype, eps, m, r_max=None, flags=0):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float32 if dtype == "f32" else torch.float64
    s = rg.Solver(m, r_max=r_max, dtype=dtype, eps=eps, flags=flags)
    s.push_rows(torch.from_numpy(A).to("cuda", td), torch.from_numpy(Y).to("cuda", td))
    r, f = s.rank(), s.flags()
    x = s.solution().double().cpu().numpy()
    s.close()
    return r, f, x


# (dtype, m, r_max, option bits): FP64 generic kernel, FP32 row-by-row on-chip
# kernel (m = 4), FP32 blocked kernel (m = 100, r_max = 44) in blocks and row by row
FAMILIES = [("f64", 4, None, 0), ("f32", 4, None, 0), ("f32", 100, 44, 0), ("f32", 100, 44, 0x8)]


@pytest.mark.parametrize("fam", FAMILIES, ids=["f64-generic", "f32-rowkernel", "f32-blocked", "f32-blocked-rows"])
@pytest.mark.parametrize("name", sorted(R.CASES))
def test_relative_clause_decides(name, fam):
    dtype, m, r_max, flags = fam
    rows, eps, want = R.CASES[name]
    A = _pad(rows, m)
    Y = np.array(R.TARGETS)
    r, f, x = _solver_rank(A, Y, dtype, eps, m, r_max, flags)
    assert f == 0
    assert r == sum(want), (name, fam)
    st = rg_ref.solve_stream(A.tolist(), Y.tolist(), eps=eps)
    assert st.decisions == want
    tol = 1e-12 if dtype == "f64" else 1e-6
    assert np.linalg.norm(x - np.array(st.X)) <= tol * np.linalg.norm(st.X)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_status_codes_single(dtype):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float32 if dtype == "f32" else torch.float64
    s = W.single_f64(n=60, m=16, r=6)
    A = torch.from_numpy(s.A).to("cuda", td)
    Y = torch.from_numpy(s.Y).to("cuda", td)
    eps = 1e-3 if dtype == "f32" else 1e-8
    h = rg.Solver(16, dtype=dtype, eps=eps)
    h.push_rows(A[:20].contiguous(), Y[:20].contiguous())
    assert h.check() == rg.OK
    bad = A[20:30].clone()
    bad[3, 1] = float("nan")
    h.push_rows(bad, Y[20:30].contiguous())   # enqueued: the host has not seen the flag yet
    assert h.check() == rg.E_NONFINITE
    with pytest.raises(rg.RGError) as e:
        h.push_rows(A[30:40].contiguous(), Y[30:40].contiguous())
    assert e.value.code == rg.E_STATE
    h.reset()
    h.push_rows(A.contiguous(), Y.contiguous())
    assert h.check() == rg.OK and h.rank() == 6
    h.close()
    c = rg.Solver(16, r_max=3, dtype=dtype, eps=eps)
    c.push_rows(A.contiguous(), Y.contiguous())
    assert c.check() == rg.E_RANK_CAPACITY and c.rank() == 3
    with pytest.raises(rg.RGError) as e:
        c.push_rows(A[:5].contiguous(), Y[:5].contiguous())
    assert e.value.code == rg.E_STATE
    c.close()


def test_batch_status_and_layout_check():
    import torch
    from paper_2106_11594_amd import rg
    from tests.gpu_util import to_device
    bt = W.batched(B=6, m_hi=96, n_scale=0.3, dtype="f32", seed=3)
    A, Y, rp, ao = to_device(bt, "f32")
    A[int(bt.a_off[2]) + 5] = float("inf")  # stream 2, first row
    caps = np.minimum(bt.ms, bt.rs + 4).astype(np.int32)
    caps[4] = 2                              # stream 4 runs out of rank capacity
    h = rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3)
    h.check_layout(A, Y, rp, ao)
    h.push(A, Y, rp, ao)
    st = h.status()
    want = np.zeros(bt.B, np.int32)
    want[2], want[4] = rg.E_NONFINITE, rg.E_RANK_CAPACITY
    assert (st == want).all(), st
    # broken layouts: decreasing row pointers, overlapping rows, rows past the end
    for mutate in ("decreasing", "overlap", "past_end"):
        rp2, ao2 = rp.clone(), ao.clone()
        if mutate == "decreasing":
            rp2[3] = rp2[2] - 1
        elif mutate == "overlap":
            ao2[1] = ao2[0] + 1
        else:
            ao2[bt.B - 1] = A.numel() - 1
        with pytest.raises(rg.RGError) as e:
            h.check_layout(A, Y, rp2, ao2)
        assert e.value.code == rg.E_INVALID, mutate
    h.close()


def test_caller_workspace_matches_library_allocation():
    import torch
    from paper_2106_11594_amd import rg
    from tests.gpu_util import to_device
    bt = W.batched(B=40, n_scale=0.3, dtype="f32", seed=8)
    A, Y, rp, ao = to_device(bt, "f32")
    caps = np.minimum(bt.ms, bt.rs + 4).astype(np.int32)
    nbytes = rg.workspace_bytes(bt.ms, caps, "f32")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    outs = []
    for work in (None, ws[:nbytes]):
        h = rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3, workspace=work)
        h.plan(bt.ns)
        h.push(A, Y, rp, ao)
        outs.append((h.solution().cpu(), h.rank()))
        h.close()
    assert torch.equal(outs[0][0], outs[1][0]) and (outs[0][1] == outs[1][1]).all()
    for bad in (ws[:nbytes - 8], ws[4:nbytes + 4]):
        with pytest.raises(rg.RGError) as e:
            rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3, workspace=bad)
        assert e.value.code == rg.E_INVALID


def test_pinv_track_exact_test_with_zero_and_duplicate_rows():
    import torch
    from paper_2106_11594_amd import rg
    # mutually orthogonal basis rows with power-of-two squared norms keep every
    # projection dyadic, so the FP64 rejections of the copy, the combination
    # and the zero row are exactly zero, as the exact test needs
    A = np.array([[1, 1, 0, 0], [0, 0, 0, 0], [1, -1, 1, 1], [1, 1, 0, 0], [2, 0, 1, 1], [0, 0, 1, -1]], float)
    Y = np.array([1, 2, -1, 3, 0, 5], float)
    st = rg_ref.solve_stream(A.tolist(), Y.tolist(), exact=True, track_pinv=True)
    Ap, X, rank, flags = rg.pinv_track(torch.from_numpy(A).cuda(), torch.from_numpy(Y).cuda(), eps=0.0)
    torch.cuda.synchronize()
    assert int(flags.cpu()) == 0 and int(rank.cpu()) == st.r == 3
    Ap_ex = np.array([[float(v) for v in row] for row in st.Ap])
    X_ex = np.array([float(v) for v in st.X])
    assert np.allclose(Ap.cpu().numpy(), Ap_ex, rtol=1e-13, atol=1e-14)
    assert np.allclose(X.cpu().numpy(), X_ex, rtol=1e-13, atol=1e-14)
