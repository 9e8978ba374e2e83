"""rg_batch_pinv: A^+ of every stream from the maintained factorisation
(Theorem 1), against the oracle's Theorem 1 product on its own state, the SVD
pseudoinverse at the planted rank, and the four Penrose equations.
Tolerances: FP64 1e-10 relative (entries of A^+ in Frobenius norm), Penrose
residuals 1e-8; FP32 1e-4 relative (well-conditioned planted bases)."""
import numpy as np
import pytest

from oracle import rg_ref
from paper_2106_11594_amd import workloads as W

pytestmark = pytest.mark.gpu


def _batch(dtype):
    rng = np.random.default_rng(91)
    streams, ranks = [], []
    for m, r, n in [(8, 3, 15), (24, 6, 40), (40, 10, 60), (17, 17, 30), (33, 5, 9)]:
        A = W.lowrank_rows(rng, m, r, n)
        Y, _ = W.targets(rng, A)
        streams.append((A, Y))
        ranks.append(min(r, n))
    ms, ns, row_ptr, a_off, A, Y = W.pack(streams, 1e-3, dtype)
    return streams, ranks, ms, ns, row_ptr, a_off, A, Y


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pinv_vs_oracle_svd_and_penrose(dtype):
    import torch
    from paper_2106_11594_amd import rg
    streams, ranks, ms, ns, row_ptr, a_off, A, Y = _batch(dtype)
    td = torch.float64 if dtype == "f64" else torch.float32
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to("cuda", td)
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).to("cuda", td)
    rp = torch.from_numpy(row_ptr).cuda()
    ao = torch.from_numpy(a_off).cuda()
    eps = 1e-10 if dtype == "f64" else 1e-3
    h = rg.Batch(ms, dtype=dtype, eps=eps)
    h.push(Ad, Yd, rp, ao)
    Ap = h.pinv(Ad, rp, ao).double().cpu().numpy()
    assert (h.rank() == np.array(ranks)).all()
    for b, (Ab, Yb) in enumerate(streams):
        m, n = Ab.shape[1], Ab.shape[0]
        Ag = Ap[a_off[b]:a_off[b] + m * n].reshape(m, n)
        # the values the device received (FP32-rounded for FP32 runs); SVD cut above their noise floor
        Ab_run = A[a_off[b]:a_off[b] + m * n].reshape(n, m).astype(np.float32 if dtype == "f32" else np.float64)
        Ab_run = Ab_run.astype(np.float64)
        Asvd = np.linalg.pinv(Ab_run, rcond=1e-9 if dtype == "f64" else 1e-4)
        rel = np.linalg.norm(Ag - Asvd) / np.linalg.norm(Asvd)
        if dtype == "f64":
            st = rg_ref.solve_stream(Ab_run.tolist(), [0.0] * n, eps=eps)
            Ao = np.array(rg_ref.pinv_from_state(Ab_run.tolist(), st))
            assert np.linalg.norm(Ag - Ao) <= 1e-10 * np.linalg.norm(Ao), b
            assert rel <= 1e-10, (b, rel)
            res = rg_ref.penrose_residuals(Ab_run, Ag)
            assert max(res) <= 1e-8 * max(1.0, np.abs(Ab_run).max()), (b, res)
        else:
            assert rel <= 1e-4, (b, rel)
    h.close()
