"""Write c2_worst_kappa.json: the 20 streams of the batched workload (B = 4096,
m ~ U{16..256}, r ~ U{4..m/2}, n ~ U{m..8m}) whose accepted-row matrix C has
the largest condition number, with that condition number and the oracle's
rank.  C and the rank come from the FP64 C oracle at eps = 1e-3 and the
benchmark's rank capacity min(r + 4, 128, m); the rows from the seeded
generator.  Only oracle/ and the input generator are called.

  python tests/golden/make_worst_kappa.py
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref_c  # noqa: E402
from paper_2106_11594_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c2_worst_kappa.json")


def _cap(m, r):
    return int(min(m, r + 4, max(r, 128)))


def _kappa(b):
    ms, rs, _ = W.batched_shapes()
    bt = W.batched(streams=[b])
    A, Y = bt.stream(0)
    _, r, C, *_ = ref_c.solve(A, Y, eps=1e-3, cap=_cap(int(ms[b]), int(rs[b])))
    return b, float(np.linalg.cond(C)) if r else 1.0, int(r)


def main():
    ms, rs, ns = W.batched_shapes()
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_kappa, range(len(ms)), chunksize=16)
    res.sort(key=lambda t: -t[1])
    top = res[:20]
    rec = {"workload": "batched B=4096 (seed 0), eps 1e-3, rank capacity min(r + 4, 128, m)",
           "streams": [t[0] for t in top], "kappa": [t[1] for t in top], "rank": [t[2] for t in top],
           "m": [int(ms[t[0]]) for t in top], "n": [int(ns[t[0]]) for t in top]}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT, ["%d:%.3g" % (b, k) for b, k, _ in top])


if __name__ == "__main__":
    main()
