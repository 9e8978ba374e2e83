"""Writes the expected values of the two single-stream workloads that are too
slow for the oracle to recompute inside a test:

  large_stream_f64.npz, large_stream_f32.npz
      m = 2048, r = 256, n = 20000 (10 % copies, 5 % two-row combinations),
      run by the FP64 C oracle on the same input values the GPU receives
      (FP64 targets, eps 1e-8; FP32-rounded targets, eps 1e-3).  Stored: x,
      rank, the decision count and kappa(C) of the accepted rows.
  stress_f32.npz
      m = 1024, r = 128, n = 50000, singular values 1 .. 1e-6, FP32 inputs,
      eps 1e-3: x and the rank after every 5000 rows.

Only the oracle and the seeded input generators are called.

    python tests/golden/make_large_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref_c  # noqa: E402
from paper_2106_11594_amd import workloads as W  # noqa: E402

CHECK_EVERY = 5000


def kappa_of_accepted(A, dec):
    C = A[dec.astype(bool)]
    return float(np.linalg.cond(C)) if C.shape[0] else 1.0


def large(dtype):
    s = W.large_stream(dtype=dtype)
    t = time.time()
    x, r, _, _, _, dec = ref_c.solve(s.A, s.Y, eps=s.eps, decisions=True)
    print("large_stream %s: rank %d, %d rows, %.1f s" % (dtype, r, s.A.shape[0], time.time() - t), flush=True)
    np.savez(os.path.join(HERE, "large_stream_%s.npz" % dtype), x=x, rank=np.int64(r),
             independent=np.int64(dec.sum()), kappa=np.float64(kappa_of_accepted(s.A, dec)), eps=np.float64(s.eps))


def stress():
    s = W.stress()
    n, m = s.A.shape
    st = ref_c.Stream(m, cap=m, eps=s.eps)
    xs, ranks, kap = [], [], []
    acc = np.zeros(n, dtype=bool)
    t = time.time()
    for c0 in range(0, n, CHECK_EVERY):
        dec = st.push(s.A[c0:c0 + CHECK_EVERY], s.Y[c0:c0 + CHECK_EVERY], decisions=True)
        acc[c0:c0 + CHECK_EVERY] = dec.astype(bool)
        xs.append(st.x)
        ranks.append(st.rank)
        kap.append(kappa_of_accepted(s.A, acc))
    st.close()
    print("stress: ranks %s, %.1f s" % (ranks, time.time() - t), flush=True)
    np.savez(os.path.join(HERE, "stress_f32.npz"), x=np.array(xs), rank=np.array(ranks, dtype=np.int64),
             kappa=np.array(kap), check_every=np.int64(CHECK_EVERY), eps=np.float64(s.eps))


if __name__ == "__main__":
    ref_c.build()
    stress()
    large("f64")
    large("f32")
