"""Seeded synthetic inputs for the rank-Greville streams.

This module only draws and packs numbers: it holds none of the method's
arithmetic, so the oracle tests and the HIP-path tests can both use it.

The paper times from-scratch solves on products of Gaussian factors
(Section 4.1: a rank-r pseudo-random matrix obtained as the product of N(0,1)
matrices, entries standardised).  We keep that structure, A = Z W with
W (r x m) and Z (n x r), with one change: W and Z are drawn N(0,1) and
rounded to the dyadic grid 2^-5.  Every entry of A is then exactly
representable in FP32 and FP64 (|entries| < 2^14 is checked), A has exact
rank r in both precisions, and the FP32 and FP64 paths consume identical
values.  Targets are y = A x* + N(0, sigma^2), formed in FP64 and then
rounded to the run dtype (the oracle reads the rounded values).

Workloads (sizes as named):
  single_f64     m=64, r=16, n=2000, FP64, rank tolerance 1e-10
  large_stream   m=2048, r=256, n=20000; 10% exact duplicates of earlier rows
                 and 5% exact +-1 combinations of two distinct earlier rows
  batched        B=4096 streams, m~U{16..256}, r~U{4..m/2}, n~U{m..8m}
  stress         m=1024, W = U diag(s) V^T, s log-spaced 1..1e-6,
                 n=50000, rows formed in FP64 and rounded to FP32
  grad_batch     B=1024, m=128, r=32, n=512, plus x_target ~ N(0, I_128)
Every size can be scaled down for tests.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2106115940
GRID = 32.0  # quantisation grid 2^-5


def _q(x):
    return np.round(x * GRID) / GRID


def _rng(tag, *sub):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, tag, *sub])))


def _check_exact(A):
    if A.size and float(np.abs(A).max()) >= 2.0 ** 14:
        raise ValueError("generated rows leave the exactly representable range")


def lowrank_rows(rng, m, r, n):
    """n rows of a rank-r product Z W with quantised N(0,1) factors (exact)."""
    W = _q(rng.standard_normal((r, m)))
    Z = _q(rng.standard_normal((n, r)))
    A = Z @ W
    _check_exact(A)
    return A


def targets(rng, A, sigma=1e-3, xstar=None):
    m = A.shape[1]
    if xstar is None:
        xstar = rng.standard_normal(m)
    return A @ xstar + sigma * rng.standard_normal(A.shape[0]), xstar


@dataclass
class Stream:
    """One stream: rows A (n x m, float64 holding run-dtype values), Y (n)."""
    A: np.ndarray
    Y: np.ndarray
    r_true: int
    eps: float = -1.0
    dtype: str = "f64"
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return self.A.shape[1]

    @property
    def n(self):
        return self.A.shape[0]


def _round(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == "f32" else x


def single_f64(n=2000, m=64, r=16, seed=0):
    rng = _rng(0, seed)
    A = lowrank_rows(rng, m, r, n)
    Y, _ = targets(rng, A)
    return Stream(A, Y, r, eps=1e-10, dtype="f64")


def large_stream(n=20000, m=2048, r=256, p_dup=0.10, p_comb=0.05, dtype="f64", seed=0):
    """Rows W^T z, except (from the third row on) that with probability
    p_dup a row copies a uniformly chosen earlier row and with probability
    p_comb it is Gamma_j +- Gamma_k for two distinct earlier rows.  Targets of
    copies get fresh noise."""
    rng = _rng(1, seed)
    W = _q(rng.standard_normal((r, m)))
    Z = _q(rng.standard_normal((n, r)))
    base = Z @ W
    A = np.empty((n, m))
    kind = rng.random(n)
    for i in range(n):
        if i >= 2 and kind[i] < p_dup:
            A[i] = A[rng.integers(0, i)]
        elif i >= 2 and kind[i] < p_dup + p_comb:
            j, k = rng.choice(i, size=2, replace=False)
            A[i] = A[j] + (1.0 if rng.random() < 0.5 else -1.0) * A[k]
        else:
            A[i] = base[i]
    _check_exact(A)
    Y, xs = targets(rng, A)
    return Stream(A, _round(Y, dtype), r, eps=(1e-3 if dtype == "f32" else 1e-8), dtype=dtype)


def stress(n=50000, m=1024, r=128, seed=0):
    """W = U diag(s) V^T with orthonormal U (r x r), V (m x r) from QR of
    Gaussians and s = logspace(0, -6, r); rows W^T z in FP64 rounded to FP32."""
    rng = _rng(3, seed)
    U, _ = np.linalg.qr(rng.standard_normal((r, r)))
    V, _ = np.linalg.qr(rng.standard_normal((m, r)))
    s = np.logspace(0.0, -6.0, r)
    W = (U * s) @ V.T
    Z = rng.standard_normal((n, r))
    A = (Z @ W).astype(np.float32).astype(np.float64)
    Y, _ = targets(rng, A)
    return Stream(A, _round(Y, "f32"), r, eps=1e-3, dtype="f32")


@dataclass
class Batch:
    """B independent streams packed back to back.

    A_packed: concatenation of each stream's rows (row-major n_b x m_b);
    stream b starts at element a_off[b].  Y_packed: concatenated targets;
    stream b's rows are row_ptr[b] .. row_ptr[b+1]-1.  Values are float64
    holding run-dtype values."""
    ms: np.ndarray
    rs: np.ndarray
    ns: np.ndarray
    row_ptr: np.ndarray
    a_off: np.ndarray
    A: np.ndarray
    Y: np.ndarray
    eps: float
    dtype: str
    extra: dict = field(default_factory=dict)

    @property
    def B(self):
        return int(self.ms.shape[0])

    def stream(self, b):
        m = int(self.ms[b])
        i0, i1 = int(self.row_ptr[b]), int(self.row_ptr[b + 1])
        A = self.A[self.a_off[b]:self.a_off[b] + (i1 - i0) * m].reshape(i1 - i0, m)
        return A, self.Y[i0:i1]

    @property
    def x_off(self):
        off = np.zeros(self.B, dtype=np.int64)
        off[1:] = np.cumsum(self.ms[:-1].astype(np.int64))
        return off


def pack(streams, eps, dtype, store=np.float64):
    ms = np.array([s[0].shape[1] for s in streams], dtype=np.int32)
    ns = np.array([s[0].shape[0] for s in streams], dtype=np.int64)
    row_ptr = np.zeros(len(streams) + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(ns)
    sizes = ns * ms
    a_off = np.zeros(len(streams), dtype=np.int64)
    a_off[1:] = np.cumsum(sizes[:-1])
    A = np.empty(int(sizes.sum()), dtype=store)
    Y = np.empty(int(ns.sum()), dtype=store)
    for b, (Ab, Yb) in enumerate(streams):
        A[a_off[b]:a_off[b] + sizes[b]] = Ab.reshape(-1)
        Y[row_ptr[b]:row_ptr[b + 1]] = Yb
    return ms, ns, row_ptr, a_off, A, Y


def batched_shapes(B=4096, m_lo=16, m_hi=256, seed=0):
    """Per-stream (m, r, n): m ~ U{m_lo..m_hi}, r ~ U{4..m/2}, n ~ U{m..8m}."""
    rng = _rng(2, seed, 0)
    ms = rng.integers(m_lo, m_hi + 1, size=B)
    rs = np.array([rng.integers(4, max(4, m // 2) + 1) for m in ms])
    ns = np.array([rng.integers(m, 8 * m + 1) for m in ms])
    return ms.astype(np.int32), rs.astype(np.int32), ns.astype(np.int64)


def batched(B=4096, m_lo=16, m_hi=256, n_scale=1.0, seed=0, dtype="f32", store=np.float64, streams=None):
    """Uneven independent streams, each with its own W, Z, x* and noise.
    ``streams`` (optional) restricts generation to a subset of indices: the
    per-stream generators are independent, so any subset reproduces exactly
    the same rows as the full batch."""
    ms, rs, ns = batched_shapes(B, m_lo, m_hi, seed)
    ns = np.maximum(1, np.round(ns * n_scale)).astype(np.int64)
    idx = np.arange(B) if streams is None else np.asarray(streams)
    out = []
    for b in idx:
        rng = _rng(2, seed, 1 + int(b))
        A = lowrank_rows(rng, int(ms[b]), int(rs[b]), int(ns[b]))
        Y, _ = targets(rng, A)
        out.append((A, _round(Y, dtype)))
    eps = 1e-3 if dtype == "f32" else 1e-8
    pms, pns, row_ptr, a_off, A, Y = pack(out, eps, dtype, store)
    return Batch(pms, rs[idx], pns, row_ptr, a_off, A, Y, eps, dtype, {"index": idx})


def grad_batch(B=1024, m=128, r=32, n=512, seed=0, store=np.float64):
    """Equal-shape problems for the differentiable solve, plus x_target."""
    out = []
    xt = np.empty((B, m))
    for b in range(B):
        rng = _rng(4, seed, b)
        A = lowrank_rows(rng, m, r, n)
        Y, _ = targets(rng, A)
        out.append((A, _round(Y, "f32")))
        xt[b] = rng.standard_normal(m)
    ms, ns, row_ptr, a_off, A, Y = pack(out, 1e-3, "f32", store)
    bt = Batch(ms, np.full(B, r, np.int32), ns, row_ptr, a_off, A, Y, 1e-3, "f32")
    bt.extra["x_target"] = xt
    return bt


# --------------------------------------------------------------------------
# Test matrices of the stability study (Section 4.2).  Generators only: the
# pseudoinverse references are computed by the callers.
# --------------------------------------------------------------------------

def pascal(n):
    """Symmetric Pascal matrix P(n): P[i][j] = binomial(i + j, i) (integers)."""
    from math import comb
    return np.array([[comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)


def kahan(n, c):
    """Kahan matrix K(c, s), s = sqrt(1 - c^2): upper triangular,
    K[i][i] = s^i, K[i][j] = -c s^i for j > i."""
    s = np.sqrt(1.0 - c * c)
    K = np.triu(-c * np.ones((n, n)), 1) + np.eye(n)
    return (s ** np.arange(n))[:, None] * K


def usv(n, rows_per_col=5, seed=0):
    """U S V^T with U (5n x n) and V (n x n) random column-orthogonal (QR of
    Gaussians) and S = diag(2^(k/2)), k = 0..n-1; returns (A, U, S, V)."""
    rng = _rng(5, n, seed)
    U, _ = np.linalg.qr(rng.standard_normal((rows_per_col * n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S = 2.0 ** (np.arange(n) / 2.0)
    return (U * S) @ V.T, U, S, V


def gaussian(rows, cols, seed=0):
    """N(0, 1) matrix (the random family R_N)."""
    return _rng(6, rows, cols, seed).standard_normal((rows, cols))
