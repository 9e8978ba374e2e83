"""The adjoint kernel behind torch.autograd against FP64 references.

Tolerances: the pinned reference gradient (oracle/adjoint_ref.py, checked
against central finite differences in the CPU suite) is evaluated in FP64 on
the same inputs; FP64 GPU runs must agree to 1e-9 relative, FP32 runs to 1e-4
relative (the target bound; FP32 state moves x and the factors by
O(kappa(C) 2^-23) ~ 1e-5 on these inputs).  Directional derivatives are also
checked directly against FP64 central differences through the rank-r
truncated SVD solve (h = 1e-6).
"""
import numpy as np
import pytest

from oracle import adjoint_ref as G
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _problems(B, m, r, n, seed):
    out = []
    for b in range(B):
        rng = np.random.default_rng([seed, b])
        A = W.lowrank_rows(rng, m, r, n)
        Y, _ = W.targets(rng, A)
        out.append((A, Y, rng.standard_normal(m)))
    return out


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-9), ("f32", 1e-4)])
def test_adjoint_vs_reference(dtype, tol):
    import torch
    from paper_2106_11594_amd.rg import rg_solve
    B, m, r, n = 6, 24, 5, 40
    probs = _problems(B, m, r, n, 1)
    td = torch.float64 if dtype == "f64" else torch.float32
    A = torch.tensor(np.stack([p[0] for p in probs]), dtype=td, device="cuda", requires_grad=True)
    Y = torch.tensor(np.stack([p[1] for p in probs]), dtype=td, device="cuda", requires_grad=True)
    xt = torch.tensor(np.stack([p[2] for p in probs]), dtype=td, device="cuda")
    x = rg_solve(A, Y, eps=1e-8 if dtype == "f64" else 1e-3)
    loss = 0.5 * ((x - xt) ** 2).sum()
    loss.backward()
    dA, dY = A.grad.double().cpu().numpy(), Y.grad.double().cpu().numpy()
    for b, (Ab, Yb, xtb) in enumerate(probs):
        Ab = Ab.astype(np.float32).astype(np.float64) if dtype == "f32" else Ab
        Yb = Yb.astype(np.float32).astype(np.float64) if dtype == "f32" else Yb
        xr = G.solve_rank(Ab, Yb, r)
        rA, rY = G.grad_closed_form(Ab, Yb, xr - xtb, r)
        assert _rel(dA[b], rA) <= tol, (b, _rel(dA[b], rA))
        assert _rel(dY[b], rY) <= tol, (b, _rel(dY[b], rY))
        # element by element, against the largest entry of the reference
        assert np.abs(dA[b] - rA).max() <= tol * np.abs(rA).max(), b
        assert np.abs(dY[b] - rY).max() <= tol * np.abs(rY).max(), b


def test_adjoint_vs_finite_differences():
    import torch
    from paper_2106_11594_amd.rg import rg_solve
    B, m, r, n = 4, 16, 4, 30
    probs = _problems(B, m, r, n, 2)
    A = torch.tensor(np.stack([p[0] for p in probs]), dtype=torch.float64, device="cuda", requires_grad=True)
    Y = torch.tensor(np.stack([p[1] for p in probs]), dtype=torch.float64, device="cuda", requires_grad=True)
    xt = torch.tensor(np.stack([p[2] for p in probs]), dtype=torch.float64, device="cuda")
    x = rg_solve(A, Y, eps=1e-8)
    (0.5 * ((x - xt) ** 2).sum()).backward()
    dA, dY = A.grad.cpu().numpy(), Y.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    for b, (Ab, Yb, xtb) in enumerate(probs):
        loss = lambda xx: 0.5 * float(np.sum((xx - xtb) ** 2))
        dirs = [(rng.standard_normal(Ab.shape), rng.standard_normal(Yb.shape)) for _ in range(6)]
        fd = G.grad_fd(Ab, Yb, loss, r, directions=dirs)
        an = np.array([np.sum(dA[b] * d) + np.sum(dY[b] * e) for d, e in dirs])
        assert np.abs(fd - an).max() <= 1e-4 * max(1.0, np.abs(an).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_vs_finite_differences_m64(dtype):
    """Directional derivatives of a larger problem (m = 64, r = 12, n = 150)
    against FP64 central differences through the rank-r solve of the values
    the device received (FP32-rounded for the FP32 run): 1e-4 relative."""
    import torch
    from paper_2106_11594_amd.rg import rg_solve
    B, m, r, n = 2, 64, 12, 150
    probs = _problems(B, m, r, n, 3)
    td = torch.float64 if dtype == "f64" else torch.float32
    A = torch.tensor(np.stack([p[0] for p in probs]), dtype=td, device="cuda", requires_grad=True)
    Y = torch.tensor(np.stack([p[1] for p in probs]), dtype=td, device="cuda", requires_grad=True)
    xt = torch.tensor(np.stack([p[2] for p in probs]), dtype=td, device="cuda")
    x = rg_solve(A, Y, eps=1e-8 if dtype == "f64" else 1e-3)
    (0.5 * ((x - xt) ** 2).sum()).backward()
    dA, dY = A.grad.double().cpu().numpy(), Y.grad.double().cpu().numpy()
    rng = np.random.default_rng(11)
    for b, (Ab, Yb, xtb) in enumerate(probs):
        if dtype == "f32":
            Ab = Ab.astype(np.float32).astype(np.float64)
            Yb = Yb.astype(np.float32).astype(np.float64)
            xtb = xtb.astype(np.float32).astype(np.float64)
        loss = lambda xx: 0.5 * float(np.sum((xx - xtb) ** 2))
        dirs = [(rng.standard_normal(Ab.shape), rng.standard_normal(Yb.shape)) for _ in range(4)]
        fd = G.grad_fd(Ab, Yb, loss, r, directions=dirs)
        an = np.array([np.sum(dA[b] * d) + np.sum(dY[b] * e) for d, e in dirs])
        err = np.abs(fd - an).max() / max(1.0, np.abs(fd).max())
        print("%s problem %d: directional derivatives within %.2e of FD" % (dtype, b, err), flush=True)
        assert err <= 1e-4


def test_grad_batch_workload_sampled():
    """The differentiable batched workload (B=1024, m=128, r=32, n=512, FP32):
    forward ranks exact, and dL/dA, dL/dY of sampled problems within 1e-4 of
    the FP64 reference gradient."""
    import torch
    from paper_2106_11594_amd.rg import rg_solve
    bt = W.grad_batch()
    B, m, n = bt.B, 128, 512
    A = torch.tensor(bt.A.reshape(B, n, m), dtype=torch.float32, device="cuda", requires_grad=True)
    Y = torch.tensor(bt.Y.reshape(B, n), dtype=torch.float32, device="cuda", requires_grad=True)
    xt = torch.tensor(bt.extra["x_target"], dtype=torch.float32, device="cuda")
    x = rg_solve(A, Y, eps=1e-3, r_max=36)
    (0.5 * ((x - xt) ** 2).sum()).backward()
    dA, dY = A.grad.double().cpu().numpy(), Y.grad.double().cpu().numpy()
    worst = 0.0
    for b in list(range(0, B, 97)) + [B - 1]:
        Ab, Yb = bt.stream(b)
        xr = G.solve_rank(Ab, Yb, 32)
        rA, rY = G.grad_closed_form(Ab, Yb, xr - bt.extra["x_target"][b], 32)
        worst = max(worst, _rel(dA[b], rA), _rel(dY[b], rY))
    assert worst <= 1e-4, worst
