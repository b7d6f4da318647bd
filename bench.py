#!/usr/bin/env python3
"""Benchmark: LearnedSort 2.0 keys/s on one MI355X.

Default workload: 200,000,000 float64 keys, Zipf(s=1.2) picks among 100,000
distinct values each drawn lognormal(0, 2) (more than 95% repeats), seeded.
A step is one complete sort of one copy of that array (sample, train,
partition rounds, base case, fills, touch-up), inputs resident in HBM.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (algorithmic bytes / its HIP-event time, against 8 TB/s) and the CPU
oracle timed on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "keys/sec sorted (1 MI355X) + % HBM roofline; served p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(ROOT, "paper_2107_03290_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2107_03290_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_workload(name: str, n: int | None):
    import workloads as W
    if name == "zipf_lognormal":
        n = n or 200_000_000
        return W.zipf_lognormal(n, seed=2), "zipf_lognormal_f64", n
    if name == "uniform":
        n = n or 1_000_000
        return W.uniform_1e9grid(n, seed=1), "uniform_1e9grid_f64", n
    if name == "mixed_u64":
        n = n or 1_000_000_000
        return W.mixed_u64(n, seed=3), "mixed_u64", n
    raise SystemExit("unknown workload " + name)


def to_device(a: np.ndarray, torch):
    w = a.view(np.uint64) if a.dtype == np.float64 else a
    t = torch.empty(a.size, dtype=torch.int64, device="cuda:0")
    step = 1 << 26
    for lo in range(0, a.size, step):
        t[lo:lo + step].copy_(torch.from_numpy(w[lo:lo + step].view(np.int64)))
    return t.view(torch.float64) if a.dtype == np.float64 else t


def cpu_baseline(a: np.ndarray, sample: int):
    import oracle
    oracle.build(force=False)
    s = a[:sample].copy()
    t0 = time.perf_counter()
    oracle.sort(s, s_max=4096)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": "first %d keys of the same array, single-threaded C oracle (recursive mode), %.1f s"
                      % (sample, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf_lognormal")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--fanout", type=int, default=0)
    ap.add_argument("--leaves", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--base", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=200_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verify", action="store_true", help="check the sorted output against numpy")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the sort runs on a single MI355X and this build has no "
              "multi-GPU path (see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_03290_amd as ls

    t_gen = time.perf_counter()
    keys, wname, n = make_workload(args.workload, args.n)
    t_gen = time.perf_counter() - t_gen
    print("workload %s n=%d generated in %.1f s" % (wname, n, t_gen), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    pristine = to_device(keys, torch)
    K, Wm = args.steps, args.warmup
    work = [torch.empty_like(pristine) for _ in range(K)]
    S = ls.Sorter(0)
    kw = {}
    for k, v in (("fanout", args.fanout), ("leaves", args.leaves), ("tile", args.tile),
                 ("base_threshold", args.base)):
        if v:
            kw[k] = v
    p = ls.params(flags=ls.FLAG_PROFILE, **kw)
    stream = torch.cuda.current_stream(dev)

    for i in range(Wm):
        work[0].copy_(pristine)
        S.sort_(work[0], p)
    torch.cuda.synchronize()
    if args.verify:
        from tests.helpers import expected_sorted
        got = work[0].view(torch.int64).cpu().numpy().view(np.uint64)
        if not np.array_equal(got, expected_sorted(keys)):
            raise SystemExit("verification failed")
        print("verified against numpy", file=sys.stderr, flush=True)
    for w in work:
        w.copy_(pristine)
    torch.cuda.synchronize()
    S.profile_reset()
    stats = []

    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(K):
        S.sort_(work[i], p)
        stats.append(S.last_stats())
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / K
    value = n * K / (gpu_ms / 1e3)

    prof = S.profile()
    dom = max(("hist", "scatter", "base", "fill", "train"), key=lambda k: prof[k][0])
    ms, launches, byt = prof[dom]
    achieved = (byt / launches) / ((ms / launches) / 1e3) / 1e9 if launches else 0.0
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (dom, wname))
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if tj.get("kernel_source") == kernel_source_hash():
            traffic = tj.get("bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if keys.dtype == np.float64 else "u64",
        "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": wname, "n": n, "fanout": p.fanout, "leaves": p.leaves, "tile": p.tile,
                   "base_threshold": p.base_threshold, "sample_rate": p.sample_rate},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": byt / launches if launches else 0.0,
                     "avg_launch_ms": ms / launches if launches else 0.0},
        "kernel_ms_per_step": {k: prof[k][0] / K for k in prof},
        "kernel_GBps": {k: (prof[k][2] / (prof[k][0] / 1e3) / 1e9 if prof[k][0] else 0.0) for k in prof},
        "pipeline": stats[-1],
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(keys, min(args.cpu_sample, n))
    print(json.dumps(line), flush=True)
    S.close()


if __name__ == "__main__":
    main()
