"""The batched push (reset + push + solution) captured in a HIP graph: every
replay equals the eager result bit for bit (the kernels are deterministic),
with eager work and synchronisations between replays, and the replayed result
matches the FP64 oracle (rank exactly, x within 1e-5 relative: these streams
run in the blocked classes, whose factored dual basis holds that bound).
Both the persistent grid (default) and one workgroup per stream are
captured."""
import numpy as np
import pytest

from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("flags", [0, 0x80], ids=["persistent", "one-wg-per-stream"])
def test_graph_replay_matches_eager_and_oracle(flags):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from oracle import ref_c
    from paper_2106_11594_amd import rg
    from tests.gpu_util import to_device
    bt = W.batched(B=96, n_scale=0.4, dtype="f32", seed=5)
    A, Y, rp, ao = to_device(bt, "f32")
    s = torch.cuda.Stream()
    caps = np.minimum(bt.ms, bt.rs + 4)
    with torch.cuda.stream(s):
        h = rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3, stream=s, flags=flags)
        h.plan(bt.ns)
        x = torch.empty(h.n_x, dtype=torch.float32, device="cuda")
        h.reset()
        h.push(A, Y, rp, ao)
        h.solution(x)
    s.synchronize()
    eager = x.clone()
    ranks = h.rank()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.reset()
        h.push(A, Y, rp, ao)
        h.solution(x)
    for rep in range(4):
        x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, eager), rep
        assert (h.rank() == ranks).all()
        # eager work between replays
        h.reset()
        with torch.cuda.stream(s):
            h.push(A, Y, rp, ao)
            h.solution(x)
        s.synchronize()
        assert torch.equal(x, eager)
    Xo, xoff, ro, st, _ = ref_c.solve_batch(bt.ms, bt.row_ptr, bt.a_off, bt.A, bt.Y, eps=1e-3, caps=caps)
    g.replay()
    torch.cuda.synchronize()
    xr = x.double().cpu().numpy()
    assert (h.rank() == ro).all() and (st == 0).all()
    for b in range(bt.B):
        xo = Xo[xoff[b]:xoff[b] + bt.ms[b]]
        assert np.linalg.norm(xr[xoff[b]:xoff[b] + bt.ms[b]] - xo) <= 1e-5 * np.linalg.norm(xo), b
