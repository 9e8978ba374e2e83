"""The batched push (reset + push + solution) captured in a HIP graph: every
replay equals the eager result bit for bit (the kernels are deterministic),
with eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_11594_amd import rg
    from tests.gpu_util import to_device
    bt = W.batched(B=96, n_scale=0.4, dtype="f32", seed=5)
    A, Y, rp, ao = to_device(bt, "f32")
    s = torch.cuda.Stream()
    caps = np.minimum(bt.ms, bt.rs + 4)
    with torch.cuda.stream(s):
        h = rg.Batch(bt.ms, r_max=caps, dtype="f32", eps=1e-3, stream=s)
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
