"""rg_pinv_track_noalloc (workspace in the library's fixed device array, no
allocation in the call) against rg_pinv_track (caller workspace) through the
C ABI: the same kernel on the same inputs, so every output must be equal bit
for bit.  Two calls in a row, the second on a smaller problem, so the second
call runs on whatever the first left in the shared array.  A request larger
than the array is refused before any device work."""
import numpy as np
import pytest

from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problems(seed, B, n, m, r):
    rng = np.random.default_rng(seed)
    As, Ys = [], []
    for b in range(B):
        A = W.lowrank_rows(rng, m, r, n)
        if b % 2 == 1:
            A[n - 1] = A[1]   # an exact copy
            A[3] = 0.0        # a zero row
        Y, _ = W.targets(rng, A)
        As.append(A)
        Ys.append(Y)
    return np.stack(As), np.stack(Ys)


def _compare(seed, B, n, m, r, r_max):
    import torch
    from paper_2106_11594_amd import rg
    A, Y = _problems(seed, B, n, m, r)
    Ad = torch.from_numpy(A).cuda()
    Yd = torch.from_numpy(Y).cuda()
    Ap0, X0, rank0, flags0 = rg.pinv_track(Ad, Yd, r_max=r_max)
    Ap = torch.full((B, m, n), float("nan"), dtype=torch.float64, device="cuda")
    X = torch.full((B, m), float("nan"), dtype=torch.float64, device="cuda")
    rank = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    flags = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    rg.pinv_track_noalloc(Ad, Yd, Ap, X, rank, flags, r_max=r_max)
    torch.cuda.synchronize()
    assert torch.equal(rank, rank0) and torch.equal(flags, flags0)
    assert (rank.cpu().numpy() == r).all() and (flags.cpu().numpy() == 0).all()
    assert torch.equal(Ap, Ap0) and torch.equal(X, X0)


def test_noalloc_equals_workspace_entry_point_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _compare(31, B=8, n=120, m=48, r=12, r_max=20)
    _compare(32, B=3, n=30, m=10, r=4, r_max=6)   # smaller: runs on the first call's leftovers


def test_noalloc_rejects_requests_beyond_the_array():
    import ctypes
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_11594_amd import rg
    cap = rg.pinv_track_noalloc_max_bytes()
    assert cap == 32 << 20
    B, n, m, r_max = 64, 2048, 64, 32
    assert rg.pinv_track_workspace_bytes(B, n, m, r_max) > cap
    dummy = ctypes.c_void_p(256)
    code = rg.lib().rg_pinv_track_noalloc(dummy, dummy, B, n, m, r_max, -1.0, dummy, dummy, dummy, dummy, None)
    assert code == rg.E_UNSUPPORTED
