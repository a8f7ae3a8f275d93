"""Autotuner for the batched-circuit kernel: team size per size bucket.

    python -m paper_2408_00384_amd.autotune [--batch 4096] [--reps 3]

For every size bucket (max n 64 / 128 / 256) it draws that bucket's share of a
batch of the batched workload's distribution (n uniform in [8, 256], so the
bucket's share of the n range; depth uniform in [n, 4n], 4 shots), times every
compiled team size on them (HIP events around
the persistent launch, median of several runs, after checking that all team
sizes give identical outcome bytes), and writes the fastest choice per bucket
to tuning/batch_gfx950.json, which BatchPlan reads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _binding as B
from .batch import BUCKETS, TUNING_PATH, BatchPlan
from .device import Context


def bucket_circuits(maxn: int, count: int, seed: int = 17):
    from inputs import batch_circuit
    lo = 8 if maxn == BUCKETS[0] else BUCKETS[BUCKETS.index(maxn) - 1] + 1
    rng = np.random.Generator(np.random.PCG64([seed, maxn]))
    ns = rng.integers(lo, maxn + 1, size=count)
    depths = rng.integers(ns, 4 * ns + 1)
    return [batch_circuit(i, ns, depths, seed=seed + maxn, shots=4) for i in range(count)]


def time_plan(plan, reps: int) -> float:
    plan.run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(plan.ctx.stream)
        plan.run()
        e1.record(plan.ctx.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def bucket_share(maxn: int, batch: int) -> int:
    """Circuits of a `batch`-circuit workload with n uniform in [8, 256] that
    fall in the bucket: the choice is a throughput one (many circuits per CU
    at once), so the bucket is timed at its real size, not on a small sample."""
    lo = 8 if maxn == BUCKETS[0] else BUCKETS[BUCKETS.index(maxn) - 1] + 1
    return max(1, round(batch * (maxn - lo + 1) / (BUCKETS[-1] - 8 + 1)))


def autotune(batch: int = 4096, reps: int = 3, out_path: str = TUNING_PATH):
    stream = torch.cuda.Stream()
    ctx = Context(0, stream)
    rec = {"device": torch.cuda.get_device_name(0), "created": time.strftime("%Y-%m-%d %H:%M:%S"),
           "batch": batch, "circuits_per_bucket": {}, "reps": reps, "timings_ms": {}, "best": {}}
    for maxn in BUCKETS:
        circs = bucket_circuits(maxn, bucket_share(maxn, batch))
        rec["circuits_per_bucket"][str(maxn)] = len(circs)
        teams = [t for (t, m) in B.BATCH_CONFIGS if m == maxn]
        ref = None
        timings = {}
        for team in teams:
            with torch.cuda.stream(stream):
                plan = BatchPlan(ctx, circs, teams={maxn: team})
                ms = time_plan(plan, reps)
                outs = plan.outcomes()
            st = plan.status()
            if st["rejected"] or st["anomalies"]:
                raise RuntimeError("batch kernel reported %s (team %d, maxn %d)" % (st, team, maxn))
            if ref is None:
                ref = outs
            elif not all(np.array_equal(a, b) for a, b in zip(ref, outs)):
                raise RuntimeError("team sizes disagree for maxn %d" % maxn)
            timings[str(team)] = ms
            plan.close()
            print("maxn %3d team %3d: %.3f ms (%d circuits)" % (maxn, team, ms, len(circs)),
                  file=sys.stderr, flush=True)
        best = min(timings, key=timings.get)
        rec["timings_ms"][str(maxn)] = timings
        rec["best"][str(maxn)] = {"team": int(best), "ms": timings[best]}
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--batch", type=int, default=4096, help="circuits of the whole batch (split over buckets)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TUNING_PATH)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    rec = autotune(args.batch, args.reps, args.out)
    print(json.dumps(rec["best"]))


if __name__ == "__main__":
    main()
