"""Helpers for the GPU tests: move a workload batch to the device and run
the HIP path through the C ABI binding."""
import numpy as np


def to_device(bt, dtype):
    import torch
    td = torch.float32 if dtype == "f32" else torch.float64
    A = torch.from_numpy(np.ascontiguousarray(bt.A)).to(device="cuda", dtype=td)
    Y = torch.from_numpy(np.ascontiguousarray(bt.Y)).to(device="cuda", dtype=td)
    rp = torch.from_numpy(bt.row_ptr).cuda()
    ao = torch.from_numpy(bt.a_off).cuda()
    return A, Y, rp, ao


def run_batch(bt, dtype, r_max=None, eps=None, flags=0, plan=True):
    """Push every stream of ``bt`` from the empty state; return (x, ranks,
    flags, batch handle) with x split per stream (float64 numpy)."""
    import torch
    from paper_2106_11594_amd import rg
    A, Y, rp, ao = to_device(bt, dtype)
    h = rg.Batch(bt.ms, r_max=r_max, dtype=dtype, eps=eps, flags=flags)
    if plan:
        h.plan(bt.ns)
    h.push(A, Y, rp, ao)
    x = h.solution().double().cpu().numpy()
    torch.cuda.synchronize()
    xs = [x[h.x_off[b]:h.x_off[b] + bt.ms[b]] for b in range(bt.B)]
    return xs, h.rank(), h.flags(), h
