"""Offline tuner of the batched C-A launch (lra_cur_batched).

Blocks are binned by their larger dimension.  For every bin and the rank,
this times each compiled register-panel variant (items per lane x wavefronts
per workgroup, enough item slots for the bin) and the LDS-panel kernel on
seeded far-field blocks of that bin (K_ij = 1/|x_i - y_j|, FP32, rows and
columns uniform up to the bin's bound, the larger above the previous bound),
and writes the fastest variant per bin to ``tuning/batch_rules_<arch>.json``.
``build.py`` turns that file into the library's built-in bin table.  Every
variant computes the same results (only the launch shape differs), so the
tuner compares time alone.

    python -m paper_1710_07946_amd.tune_batched [--blocks 1024] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BINS = [128, 256, 512, 1024]
VARIANTS = [(2, 1), (2, 2), (2, 4), (2, 8)]
RANK, SWEEPS, SEED = 16, 3, 1000


def bin_shapes(lo: int, hi: int, count: int, seed: int):
    """Rows and columns uniform in [16, hi], redrawn until the larger exceeds lo."""
    g = np.random.default_rng(seed)
    ms, ns = [], []
    while len(ms) < count:
        m, n = int(g.integers(16, hi + 1)), int(g.integers(16, hi + 1))
        if max(m, n) > lo:
            ms.append(m)
            ns.append(n)
    return np.array(ms, np.int64), np.array(ns, np.int64)


def lds_limit(lra, torch, base, desc) -> bool:
    """Whether the LDS-panel kernel accepts this bin (its panel fits on chip)."""
    lra.lra_batch_set_rules([(1 << 20, RANK, 0, 0)])
    try:
        lra.lra_cur_batched(base, desc[:1], RANK, 1, SEED)
        torch.cuda.synchronize()
        return True
    except lra.LraError:
        return False


def time_rules(lra, torch, base, desc, rules, reps: int) -> float:
    lra.lra_batch_set_rules(rules)
    out = lra.lra_cur_batched(base, desc, RANK, SWEEPS, SEED)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lra.lra_cur_batched(base, desc, RANK, SWEEPS, SEED, out=out)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    bad = [i for i in out.info() if i["status"] != 0]
    if bad:
        raise RuntimeError("tuning blocks failed: %s" % bad[:2])
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=1024, help="blocks per bin")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    import paper_1710_07946_amd as lra
    from paper_1710_07946_amd import workloads

    lra.load()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    rules, report = [], []
    lo = 0
    for hi in BINS:
        count = args.blocks if hi <= 1024 else max(64, args.blocks // 4)
        shapes = bin_shapes(lo, hi, count, 7000 + hi)
        base, desc = workloads.fmm_batch_device(count, "cuda", block_seed0=8000000 + hi * 10000, shapes=shapes)
        torch.cuda.synchronize()
        times = {}
        for P, W in VARIANTS:
            if 64 * P * W < hi:
                continue
            times["%dx%d" % (P, W)] = time_rules(lra, torch, base, desc, [(hi, RANK, P, W)], args.reps)
            print("bin %4d  items_per_lane %d waves %d  %.3f ms" % (hi, P, W, times["%dx%d" % (P, W)]), flush=True)
        if lds_limit(lra, torch, base, desc):
            times["lds"] = time_rules(lra, torch, base, desc, [(1 << 20, RANK, 0, 0)], args.reps)
            print("bin %4d  LDS panel kernel       %.3f ms" % (hi, times["lds"]), flush=True)
        best = min(times, key=times.get)
        P, W = (0, 0) if best == "lds" else (int(best.split("x")[0]), int(best.split("x")[1]))
        rules.append({"max_dim": hi, "r": RANK, "items_per_lane": P, "waves": W})
        report.append({"max_dim": hi, "blocks": count, "ms": times, "chosen": best})
        lo = hi
        del base
        torch.cuda.empty_cache()
    lra.lra_batch_set_rules([])
    out = args.out or os.path.join(HERE, "tuning", "batch_rules_%s.json" % arch)
    with open(out, "w") as f:
        json.dump({"arch": arch, "dtype": "fp32", "rank": RANK, "sweeps": SWEEPS,
                   "measured": time.strftime("%Y-%m-%d"), "rules": rules, "timings": report}, f, indent=1)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
