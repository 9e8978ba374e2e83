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


EPS32 = 2.0 ** -23


def f32_tol(C, factored=True):
    """(bound, kappa(C)) for the relative error of an FP32 stream's x against
    the FP64 oracle, C the oracle's accepted rows.

    factored=True (the blocked on-chip classes, which keep the dual basis as
    H^-1 C with H^-1 = (C C^T)^-1 in FP64): every projection is FP64
    arithmetic on exact FP32 rows, perturbed to first order by about
    2^-52 kappa(C)^2, and x is rounded to FP32 on output; the bound is
    max(1e-5, kappa^2 2^-52), i.e. 1e-5 up to kappa(C) = 2e5.
    factored=False (the row-by-row classes and the generic kernel, which keep
    an FP32 dual basis): first order kappa(C) 2^-23; 1e-5 for kappa <= 1e3 and
    0.1 kappa 2^-23 above, the constant three times the worst ratio seen in an
    FP64 emulation of that arithmetic."""
    kap = float(np.linalg.cond(C)) if C.shape[0] else 1.0
    if factored:
        return max(1e-5, kap * kap * 2.0 ** -52), kap
    return (1e-5 if kap <= 1e3 else 0.1 * kap * EPS32), kap


def factored(m, r_max):
    """Whether a stream of m regressors and rank capacity r_max runs in a
    blocked on-chip class (dual basis in factored form) under the default
    placement; otherwise it runs in the generic kernel with an explicit FP32
    dual basis."""
    from paper_2106_11594_amd import rg
    return any(rg.class_fits(c, int(m), int(r_max)) for c in range(3, rg.class_count()))
