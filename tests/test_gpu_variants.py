"""The orthogonal rank factorization variants (Section 2.2: RG_OPT_ORTHOGONAL,
alpha = 1, and RG_OPT_ORTHONORMAL, alpha = 1 / ||Gamma_r||) on the GPU.

Against the oracle's variant runs on small streams (x, rank, and the factors'
defining properties read back from the device), and on larger streams with
copies and two-row combinations against the C oracle of the base
factorization: every factorization of A gives the same x_n = A^+ Y and rank.
The adjoint works from any factorization, so its gradient must equal the base
run's.  Tolerances: FP64 1e-11 relative on the small streams, 1e-9 on the
larger ones; FP32 the bound used everywhere (1e-5 for kappa(C) <= 1e3, else
0.1 kappa 2^-23).
"""
import numpy as np
import pytest

from oracle import ref_c, rg_ref
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = [("orthogonal", 0x20), ("orthonormal", 0x40)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _f32_tol(C):
    kap = float(np.linalg.cond(C)) if C.shape[0] else 1.0
    return 1e-5 if kap <= 1e3 else 0.1 * kap * 2.0 ** -23


def _run(A, Y, dtype, eps, flags, r_max=None):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float64 if dtype == "f64" else torch.float32
    h = rg.Batch(np.array([A.shape[1]], np.int32), r_max=None if r_max is None else np.array([r_max], np.int32),
                 dtype=dtype, eps=eps, flags=flags)
    At = torch.from_numpy(np.ascontiguousarray(A)).to("cuda", td)
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to("cuda", td)
    rp = torch.tensor([0, A.shape[0]], dtype=torch.int64, device="cuda")
    ao = torch.zeros(1, dtype=torch.int64, device="cuda")
    h.push(At.view(-1), Yt, rp, ao)
    x = h.solution().double().cpu().numpy()
    C, Ct, P, w = [t.double().cpu().numpy() for t in h.get_state(0)]
    r, f = int(h.rank()[0]), int(h.flags()[0])
    return x, r, f, C, Ct, P, h


@pytest.mark.parametrize("variant,flag", VARIANTS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_variant_vs_oracle_variant(variant, flag, dtype):
    s = W.single_f64(n=300, m=64, r=16, seed=21)
    A, Y = s.A, s.Y
    eps = 1e-10 if dtype == "f64" else 1e-3
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    st = rg_ref.solve_stream(A.tolist(), Y.tolist(), eps=eps, variant=variant)
    x, r, f, C, Ct, P, _ = _run(A, Y, dtype, eps, flag)
    assert f == 0 and r == st.r == 16
    tol = 1e-11 if dtype == "f64" else _f32_tol(np.array(st.C))
    assert _rel(x, np.array(st.X)) <= tol
    # defining properties of the factors
    G = C @ C.T
    ftol = 1e-12 if dtype == "f64" else 1e-5
    assert np.abs(G - np.diag(np.diag(G))).max() <= ftol * np.abs(G).max()
    assert np.abs(Ct @ C.T - np.eye(r)).max() <= (1e-10 if dtype == "f64" else 1e-4)
    if variant == "orthonormal":
        assert np.array_equal(C, Ct)
        assert np.abs(G - np.eye(r)).max() <= ftol
    B = A @ Ct.T
    assert np.abs(P @ (B.T @ B) - np.eye(r)).max() <= (1e-8 if dtype == "f64" else 1e-2)


@pytest.mark.parametrize("variant,flag", VARIANTS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_variant_larger_stream_vs_base_oracle(variant, flag, dtype):
    """m = 512, planted rank 64, 1500 rows with 10 % copies and 5 % two-row
    combinations: same rank and x as the base Algorithm 1 (C oracle)."""
    s = W.large_stream(n=1500, m=512, r=64, dtype=dtype, seed=4)
    xo, ro, Co, *_ = ref_c.solve(s.A, s.Y, eps=s.eps)
    x, r, f, *_ = _run(s.A, s.Y, dtype, s.eps, flag)
    print("%s %s: rank %d (oracle %d), rel %.2e" % (variant, dtype, r, ro, _rel(x, xo)), flush=True)
    assert f == 0 and r == ro == 64
    assert _rel(x, xo) <= (1e-9 if dtype == "f64" else _f32_tol(Co))


@pytest.mark.parametrize("variant,flag", VARIANTS)
def test_variant_batch_vs_base_oracle(variant, flag):
    from tests.gpu_util import run_batch
    bt = W.batched(B=24, n_scale=0.3, dtype="f32", seed=8)
    xs, ranks, fl, h = run_batch(bt, "f32", eps=1e-3, flags=flag)
    Xo, xoff, ro, st, _ = ref_c.solve_batch(bt.ms, bt.row_ptr, bt.a_off, bt.A, bt.Y, eps=1e-3, nthreads=8)
    assert (fl == 0).all() and (ranks == ro).all()
    for b in range(bt.B):
        A, Y = bt.stream(b)
        _, _, Co, *_ = ref_c.solve(A, Y, eps=1e-3)
        assert _rel(xs[b], Xo[xoff[b]:xoff[b] + bt.ms[b]]) <= _f32_tol(Co), b


@pytest.mark.parametrize("variant,flag", VARIANTS)
def test_variant_adjoint_equals_base(variant, flag):
    """dL/dA and dL/dY from a variant factorization equal the base run's."""
    import torch
    B, n, m, r = 6, 80, 24, 5
    probs = []
    for b in range(B):
        rng = np.random.default_rng([77, b])
        A = W.lowrank_rows(rng, m, r, n)
        Y, _ = W.targets(rng, A)
        probs.append((A, Y))
    ms = np.full(B, m, np.int32)
    A = torch.tensor(np.concatenate([a.reshape(-1) for a, _ in probs]), dtype=torch.float64, device="cuda")
    Y = torch.tensor(np.concatenate([y for _, y in probs]), dtype=torch.float64, device="cuda")
    rp = torch.arange(0, (B + 1) * n, n, dtype=torch.int64, device="cuda")
    ao = torch.arange(0, B * n * m, n * m, dtype=torch.int64, device="cuda")
    g = torch.tensor(np.random.default_rng(5).standard_normal(B * m), dtype=torch.float64, device="cuda")
    from paper_2106_11594_amd import rg
    out = []
    for fl in (0, flag):
        h = rg.Batch(ms, dtype="f64", eps=1e-10, flags=fl)
        h.push(A, Y, rp, ao)
        dA, dY = h.adjoint(A, Y, rp, ao, g)
        out.append((dA.cpu().numpy(), dY.cpu().numpy(), h.rank()))
        h.close()
    assert (out[0][2] == out[1][2]).all() and (out[0][2] == r).all()
    assert _rel(out[1][0], out[0][0]) <= 1e-9 and _rel(out[1][1], out[0][1]) <= 1e-9
