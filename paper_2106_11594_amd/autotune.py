"""Measured placement of FP32 streams on the kernel size classes.

For every (m, r_max) bucket the tuner builds a batch of synthetic streams of
that shape (low-rank Gaussian rows, as in the batched workload), pushes it
once per candidate class with every stream forced into that class, and keeps
the class with the highest row-update throughput.  The result is a list of
placement rules (m_hi, r_max_hi, class) for rg_set_class_rules, saved as JSON.

    python -m paper_2106_11594_amd.autotune [--out FILE] [--streams 512]

Needs a GPU.  bench.py installs the rules from the default file when it is
present.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "class_rules.json")

# bucket edges: the column and rank capacities at which the classes change
M_EDGES = [16, 64, 128, 192, 256]
R_EDGES = [0, 12, 32, 36, 64, 80, 128]


def _bucket_batch(rng_seed, B, m_lo, m_hi, r_lo, r_hi, n_scale):
    """B streams with m in (m_lo, m_hi], rank capacity in (r_lo, r_hi] and
    n ~ U{m..8m} * n_scale rows (at least r_max + 16)."""
    from . import workloads as W
    rng = np.random.default_rng(rng_seed)
    streams, rmax = [], []
    for _ in range(B):
        m = int(rng.integers(m_lo + 1, m_hi + 1))
        cap_hi = min(r_hi, m)
        cap_lo = max(r_lo + 1, 5)
        if cap_lo > cap_hi:
            return None
        cap = int(rng.integers(cap_lo, cap_hi + 1))
        r = max(1, cap - 4)
        n = max(cap + 16, int(rng.integers(m, 8 * m + 1) * n_scale))
        A = W.lowrank_rows(rng, m, r, n)
        Y, _ = W.targets(rng, A)
        streams.append((A, Y.astype(np.float32).astype(np.float64)))
        rmax.append(cap)
    ms, ns, row_ptr, a_off, A, Y = W.pack(streams, 1e-3, "f32")
    return ms, np.array(rmax, np.int32), ns, row_ptr, a_off, A.astype(np.float32), Y.astype(np.float32)


def _time_class(cls, batch, reps=2):
    """Row-updates per second of the batch with every stream in class cls."""
    import torch
    from . import rg
    ms, rmax, ns, row_ptr, a_off, A, Y = batch
    rg.set_class_rules([(1 << 30, 1 << 30, cls)])
    try:
        h = rg.Batch(ms, r_max=rmax, dtype="f32", eps=1e-3, flags=rg.OPT_SERIAL_CLASSES)
    finally:
        rg.set_class_rules([])
    dev = torch.device("cuda")
    Ad, Yd = torch.from_numpy(A).to(dev), torch.from_numpy(Y).to(dev)
    rp, ao = torch.from_numpy(row_ptr).to(dev), torch.from_numpy(a_off).to(dev)
    h.plan(ns)
    h.reset()
    h.push(Ad, Yd, rp, ao)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.reset()
        h.push(Ad, Yd, rp, ao)
    e1.record()
    torch.cuda.synchronize()
    ms_per = e0.elapsed_time(e1) / reps
    ok = bool((h.flags() == 0).all())
    h.close()
    return int(ns.sum()) / (ms_per * 1e-3), ms_per, ok


def tune(streams=512, n_scale=0.25, seed=7, log=print):
    """Measure every bucket; returns (rules, records)."""
    from . import rg
    ncls = rg.class_count()
    rules, records = [], []
    for mi in range(1, len(M_EDGES)):
        m_lo, m_hi = M_EDGES[mi - 1], M_EDGES[mi]
        for ri in range(1, len(R_EDGES)):
            r_lo, r_hi = R_EDGES[ri - 1], R_EDGES[ri]
            cap_hi = min(r_hi, m_hi)
            if cap_hi <= r_lo:
                continue
            cands = [c for c in range(ncls) if rg.class_fits(c, m_hi, cap_hi)]
            if not cands:
                continue
            batch = _bucket_batch(seed + 100 * mi + ri, streams, m_lo, m_hi, r_lo, r_hi, n_scale)
            if batch is None:
                continue
            best = None
            for c in cands:
                rate, ms_per, ok = _time_class(c, batch)
                rec = {"m": [m_lo, m_hi], "r_max": [r_lo, r_hi], "class": c, "shape": rg.class_info(c),
                       "rows_per_s": rate, "ms": ms_per, "ok": ok}
                records.append(rec)
                log("m (%3d,%3d] r_max (%3d,%3d] class %d %-16s %8.3f ms  %.3g rows/s%s"
                    % (m_lo, m_hi, r_lo, r_hi, c, rg.class_info(c), ms_per, rate, "" if ok else "  FLAGS"))
                if ok and (best is None or rate > best[1]):
                    best = (c, rate)
            if best is not None:
                rules.append([m_hi, r_hi, best[0]])
    return rules, records


def save(rules, records, path=DEFAULT_PATH):
    import torch
    with open(path, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "rules": rules, "records": records}, f, indent=1)


def load(path=DEFAULT_PATH):
    """Rules from a tuning file, or None when there is none."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return [tuple(r) for r in json.load(f)["rules"]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--streams", type=int, default=512)
    ap.add_argument("--n-scale", type=float, default=0.25)
    args = ap.parse_args()
    t0 = time.time()
    rules, records = tune(args.streams, args.n_scale, log=lambda s: print(s, flush=True))
    save(rules, records, args.out)
    print("wrote %d rules to %s in %.0f s" % (len(rules), args.out, time.time() - t0), flush=True)


if __name__ == "__main__":
    sys.exit(main())
