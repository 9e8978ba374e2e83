"""The on-chip class for FP64 streams (class rg_class_count(): the blocked
kernel with C and the rows in FP64, m <= 128, r_max <= 64), taken by the
stream of a one-stream FP64 handle.  Its blocks project their rejections
twice, so that the rank decision holds at FP64 tolerances (eps 1e-8 here, on
Gaussian rows, rows drawn from spectra down to 1e-2 and 1e-3, and streams of
the FP64 batched workload): the ranks must equal the oracle's and the
global-memory kernel's
(RG_OPT_GENERIC_KERNEL), and x must be within the factored form's bound
max(1e-11, kappa(C)^2 2^-52) of the FP64 oracle.  FP64 streams of batches run
in the global-memory kernel."""
import numpy as np
import pytest

from oracle import ref_c
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def _spectrum_rows(rng, m, r, n, smin):
    U, _ = np.linalg.qr(rng.standard_normal((r, r)))
    V, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Wm = (U * np.logspace(0.0, np.log10(smin), r)) @ V.T
    return rng.standard_normal((n, r)) @ Wm


def _solve(A, Y, r_max, eps, flags=0, chunks=()):
    import torch
    from paper_2106_11594_amd import rg
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    h = rg.Solver(A.shape[1], r_max=r_max, dtype="f64", eps=eps, flags=flags)
    bounds = [0] + list(chunks) + [A.shape[0]]
    for c0, c1 in zip(bounds[:-1], bounds[1:]):
        if c1 > c0:
            h.push_rows(At[c0:c1].contiguous(), Yt[c0:c1].contiguous())
    x = h.solution().double().cpu().numpy()
    r, f = h.rank(), h.flags()
    h.close()
    return x, r, f


def _check(A, Y, r, eps, chunks):
    from paper_2106_11594_amd import rg
    m = A.shape[1]
    cap = min(m, 64)
    h = rg.Batch(np.array([m], np.int32), r_max=np.array([cap], np.int32), dtype="f64", eps=eps)
    assert int(h.classes()[0]) == rg.class_count()
    h.close()
    x, rk, f = _solve(A, Y, cap, eps, chunks=chunks)
    xg, rkg, fg = _solve(A, Y, cap, eps, flags=rg.OPT_GENERIC_KERNEL)
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=eps, cap=cap)
    kap = float(np.linalg.cond(Co))
    tol = max(1e-11, kap * kap * 2.0 ** -52)
    err = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
    print("m %d r %d: rank %d/%d/%d, kappa %.2g, rel err %.2e (bound %.1e)" % (m, r, rk, rkg, ro, kap, err, tol),
          flush=True)
    assert f == fg == 0
    assert rk == rkg == ro == r
    assert err <= tol


@pytest.mark.parametrize("m,r,n,smin", [(64, 16, 400, 1.0), (40, 12, 90, 1e-2), (96, 32, 300, 1e-3)])
def test_f64_class_ranks_and_solution(m, r, n, smin):
    rng = np.random.default_rng(71 + m)
    A = W.lowrank_rows(rng, m, r, n) if smin == 1.0 else _spectrum_rows(rng, m, r, n, smin)
    A[n // 3] = A[n // 3 - 1]       # an exact copy
    A[n // 2] = A[2] - 0.5 * A[5]    # a combination of earlier rows
    Y, _ = W.targets(rng, A)
    _check(A, Y, r, 1e-8, chunks=(1, 17, n // 2))


def test_f64_class_on_batched_workload_streams():
    """Streams of the FP64 batched workload (m <= 128, planted rank <= 64),
    each alone in a handle: the rank decisions that need the second
    projection of the rejections."""
    bt = W.batched(streams=np.arange(7, 4096, 85), dtype="f64")
    done = 0
    for k in range(bt.B):
        A, Y = bt.stream(k)
        if A.shape[1] > 128 or bt.rs[k] > 64:
            continue
        _check(A, Y, int(bt.rs[k]), bt.eps, chunks=(A.shape[0] // 3,))
        done += 1
    assert done >= 8


def test_f64_batches_stay_in_the_generic_kernel():
    from paper_2106_11594_amd import rg
    h = rg.Batch(np.array([64, 40], np.int32), dtype="f64", eps=1e-10)
    assert (h.classes() == -1).all()
    h.close()
    h = rg.Batch(np.array([64, 40], np.int32), dtype="f32", eps=1e-3)
    assert (h.classes() >= 0).all() and (h.classes() < rg.class_count()).all()
    h.close()


@pytest.mark.parametrize("opt", ["OPT_ROW_BY_ROW", "OPT_DEPENDENT_BLOCKS_ONLY", "OPT_EXPLICIT_REJECTIONS"])
def test_f64_class_reference_paths(opt):
    """The FP64 class's row mode (every row alone) and its dependent-blocks-only
    and explicit-rejection paths against the oracle; row by row, pushes in
    pieces repeat the one-push bits."""
    from paper_2106_11594_amd import rg
    flag = getattr(rg, opt)
    rng = np.random.default_rng(91)
    m, r, n = 72, 20, 330
    A = W.lowrank_rows(rng, m, r, n)
    A[40] = A[39]
    A[200] = A[3] + A[7]
    Y, _ = W.targets(rng, A)
    h = rg.Batch(np.array([m], np.int32), r_max=np.array([48], np.int32), dtype="f64", eps=1e-10, flags=flag)
    assert int(h.classes()[0]) == rg.class_count()
    h.close()
    x1, r1, f1 = _solve(A, Y, 48, 1e-10, flags=flag)
    x2, r2, f2 = _solve(A, Y, 48, 1e-10, flags=flag, chunks=(1, 2, 90, 91, 250))
    xo, ro, Co, *_ = ref_c.solve(A, Y, eps=1e-10, cap=48)
    assert f1 == f2 == 0 and r1 == r2 == ro == r
    tol = max(1e-11, float(np.linalg.cond(Co)) ** 2 * 2.0 ** -52)
    assert np.linalg.norm(x1 - xo) <= tol * np.linalg.norm(xo)
    assert np.linalg.norm(x2 - xo) <= tol * np.linalg.norm(xo)
    if opt == "OPT_ROW_BY_ROW":
        assert np.array_equal(x1, x2)


def test_f64_class_adjoint_and_pinv():
    """A one-problem FP64 solve runs in the FP64 class (factored form); its
    adjoint and its pseudoinverse against the FP64 references."""
    import torch
    from oracle import adjoint_ref as G
    from paper_2106_11594_amd import rg
    from paper_2106_11594_amd.rg import rg_solve
    rng = np.random.default_rng(93)
    m, r, n = 24, 5, 40
    A = W.lowrank_rows(rng, m, r, n)
    Y, _ = W.targets(rng, A)
    xt = rng.standard_normal(m)
    At = torch.tensor(A[None], dtype=torch.float64, device="cuda", requires_grad=True)
    Yt = torch.tensor(Y[None], dtype=torch.float64, device="cuda", requires_grad=True)
    x = rg_solve(At, Yt, eps=1e-8)
    (0.5 * ((x - torch.tensor(xt[None], device="cuda")) ** 2).sum()).backward()
    xr = G.solve_rank(A, Y, r)
    rA, rY = G.grad_closed_form(A, Y, xr - xt, r)
    dA, dY = At.grad[0].cpu().numpy(), Yt.grad[0].cpu().numpy()
    assert np.linalg.norm(dA - rA) <= 1e-9 * np.linalg.norm(rA)
    assert np.linalg.norm(dY - rY) <= 1e-9 * np.linalg.norm(rY)
    h = rg.Batch(np.array([m], np.int32), dtype="f64", eps=1e-8)
    assert int(h.classes()[0]) == rg.class_count()
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    rp = torch.tensor([0, n], dtype=torch.int64).cuda()
    ao = torch.tensor([0], dtype=torch.int64).cuda()
    h.push(Ad.reshape(-1), Yd, rp, ao)
    Ap = h.pinv(Ad.reshape(-1), rp, ao).double().cpu().numpy().reshape(m, n)
    assert int(h.rank()[0]) == r
    h.close()
    Asvd = np.linalg.pinv(A, rcond=1e-9)
    assert np.linalg.norm(Ap - Asvd) <= 1e-10 * np.linalg.norm(Asvd)
