#!/usr/bin/env python3
"""Benchmark: LearnedSort 2.0 keys/s on one MI355X.

Default workload: 1,000,000,000 uint64 keys (8 GB), equal thirds of
round(N(2^40, 2^36)), round(Exp(scale 2^30)) and U[0, 2^64) mod 10,000 at
shuffled positions, seeded: the largest single-array configuration, with
recursion below level 1.  A step is one complete sort of one copy of that
array (sample, train, partition rounds, base case, fills, touch-up), inputs
resident in HBM.  Other workloads: --workload zipf_lognormal (2e8 f64,
Zipf-duplicates), uniform (1e6 f64), segments, served, sweep.

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


def cpu_library_sort(a: np.ndarray, sample: int):
    """numpy's default sort (one thread) on the order-preserving words of the
    same sample: a comparison-sort reference beside the oracle."""
    w = np.ascontiguousarray(a[:sample]).view(np.uint64)
    if a.dtype == np.float64:
        sign = np.uint64(1 << 63)
        w = np.where(w & sign, ~w, w | sign)
    else:
        w = w.copy()
    t0 = time.perf_counter()
    w.sort(kind="quicksort")
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "keys/s", "cores": 1, "kind": "numpy sort on order words",
            "sample": "first %d keys, %.1f s" % (sample, dt)}


def roofline(prof: dict, wname: str) -> dict:
    """Roofline entry of the dominant kernel class: algorithmic bytes per
    launch over the average launch time (HIP events on the sort's stream).
    Algorithmic bytes are the method's: the histogram reads 8 B per key, the
    scatter reads 8 B per key of a progressing range and writes 8 B per key
    outside all-equal buckets, the base case reads and writes 8 B per key."""
    dom = max(("hist", "scatter", "base", "fill", "train"), key=lambda k: prof[k][0])
    ms, launches, byt = prof[dom]
    achieved = (byt / launches) / ((ms / launches) / 1e3) / 1e9 if launches else 0.0
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (dom, wname))
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if tj.get("kernel_source") == kernel_source_hash():
            traffic = tj.get("bytes_per_launch")
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": byt / launches if launches else 0.0,
            "avg_launch_ms": ms / launches if launches else 0.0}


DOMINANT_CANDIDATES = ("hist", "scatter", "base", "fill", "train")


PROFILED_STEPS = 2


def profiled_warmup(S, ls, run, steps):
    """Run `steps` untimed warm-up steps, then PROFILED_STEPS untimed steps
    with every kernel class timed.  Returns their per-step kernel breakdown
    and the dominant class, whose launches alone get HIP events in the timed
    steps: an event pair costs the stream a few microseconds at each class
    boundary, so timing every class inside the timed region would slow the
    step being measured."""
    import torch
    for _ in range(steps):
        run(ls.FLAG_PROFILE)
    torch.cuda.synchronize()
    S.profile_reset()
    for _ in range(PROFILED_STEPS):
        run(ls.FLAG_PROFILE)
    torch.cuda.synchronize()
    prof = S.profile()
    S.profile_reset()
    dom = max(DOMINANT_CANDIDATES, key=lambda k: prof[k][0])
    breakdown = {k: prof[k][0] / PROFILED_STEPS for k in prof}
    gbps = {k: (prof[k][2] / (prof[k][0] / 1e3) / 1e9 if prof[k][0] else 0.0) for k in prof}
    flags = ls.FLAG_PROFILE | ls.FLAG_PROFILE_ONLY(ls.KERNEL_CLASSES.index(dom))
    return breakdown, gbps, dom, flags


def pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else 0.0


def bench_segments(args, torch, ls):
    """10,000 f64 arrays (log-uniform sizes 1,024..4,194,304, four families)
    sorted as one batch with autotuned parameters, against one plain sort
    call per array on the same GPU.  Both must give identical bits."""
    import workloads as W
    spec = W.segment_spec(count=args.segments)
    t0 = time.perf_counter()
    keys = W.segments(spec)
    off = spec.offsets
    n = int(off[-1])
    print("segments: %d arrays, %d keys generated in %.1f s" % (off.size - 1, n, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    pristine = to_device(keys, torch)
    work = torch.empty_like(pristine)
    S = ls.Sorter(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    best, results = S.autotune([pristine], offsets=off, reps=1)
    t_tune = time.perf_counter() - t0
    print("autotune: fanout %d tile %d base %d (%.1f s)" % (best.fanout, best.tile, best.base_threshold, t_tune),
          file=sys.stderr, flush=True)

    def run(flags):
        work.copy_(pristine)
        S.sort_segments_(work, off, p=ls.params(fanout=best.fanout, tile=best.tile,
                                                base_threshold=best.base_threshold, flags=flags))

    breakdown, gbps, dom, flags = profiled_warmup(S, ls, run, args.warmup)
    tuned = ls.params(fanout=best.fanout, tile=best.tile, base_threshold=best.base_threshold, flags=flags)
    K = args.steps
    ms_b = []
    for _ in range(K):
        work.copy_(pristine)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.sort_segments_(work, off, p=tuned)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_b.append(e0.elapsed_time(e1))
    prof = S.profile()
    stats = S.last_stats()
    # plain: one call per array, default parameters, same stream
    plain = pristine.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(off.size - 1):
        S.sort_(plain[int(off[i]):int(off[i + 1])])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    same = bool(torch.equal(work.view(torch.int64), plain.view(torch.int64)))
    if not same:
        raise SystemExit("batched and plain results differ")
    ms = sum(ms_b) / K
    line = {
        "metric": METRIC, "value": n / (ms / 1e3), "unit": "keys/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": "segments_%d_f64" % (off.size - 1), "keys": n, "fanout": best.fanout,
                   "tile": best.tile or "auto (4096; 8192, or 12288 with <= 512 leaves, in rounds of >= 2^25 keys)",
                   "base_threshold": best.base_threshold, "autotune_s": t_tune},
        "plain": {"value": n / (ms_p / 1e3), "unit": "keys/s", "ms": ms_p,
                  "calls": int(off.size - 1), "params": "defaults"},
        "batched_over_plain": ms_p / ms,
        "identical_to_plain": same,
        "roofline": roofline(prof, "segments_%d_f64" % (off.size - 1)),
        "kernel_ms_per_step": breakdown,
        "kernel_ms_source": "%d untimed steps after the warm-up with every kernel class timed; the timed "
                            "steps time the dominant class (%s) only" % (PROFILED_STEPS, dom),
        "pipeline": stats,
        "autotune": results,
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        want = args.cpu_sample if args.cpu_sample > 0 else 500_000_000   # about 25 s of oracle work
        take = int(np.searchsorted(off, min(want, n), side="right")) - 1
        take = max(take, 1)
        t0 = time.perf_counter()
        for i in range(take):
            oracle.sort(keys[int(off[i]):int(off[i + 1])].copy(), s_max=4096)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": int(off[take]) / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
                                "sample": "first %d arrays (%d keys), single-threaded C oracle, %.1f s"
                                          % (take, int(off[take]), dt)}
    print(json.dumps(line), flush=True)
    S.close()


def bench_served(args, torch, ls):
    """A stream of f64 / u64 sort requests (sizes log-uniform 1,024..2^26,
    duplicate ratio U(0, 0.99)) served by the continuous-batching server
    against one-request-at-a-time plain sorting, first as a burst (all
    requests queued at once: throughput), then with Poisson arrivals at 80%
    of the plain rate (latency).

    Request i sorts a copy of distinct request i mod D (D generated ones)
    made in work slot i mod Q just before it is submitted (plain: just before
    it is sorted), so the stream can be longer than device memory holds; a
    slot is reused once its request completes.  The copy is part of every
    request on both paths.  Every served result is compared with the plain
    result of the same request in an untimed pass."""
    import threading
    import workloads as W
    from concurrent.futures import ThreadPoolExecutor
    R, D, Q = args.requests, min(args.requests, args.distinct), min(args.requests, args.ring)
    spec = W.request_spec()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:
        reqs = list(ex.map(lambda i: W.request_keys(spec, i), range(D)))
    sizes = [reqs[i % D].size for i in range(R)]
    total = int(sum(sizes))
    print("served: %d requests over %d distinct ones, %d keys in all (generated in %.1f s)" %
          (R, D, total, time.perf_counter() - t0), file=sys.stderr, flush=True)
    # graph mode (LS_FLAG_GRAPH): requests and batches of up to 2^22 keys run
    # as replays of captured graphs, on the plain path and in the server
    gp = ls.params(flags=ls.FLAG_GRAPH if args.graph == "on" else 0)
    pristine = [to_device(a, torch) for a in reqs]
    biggest = max(a.size for a in reqs)
    slots = [torch.empty(biggest, dtype=torch.int64, device="cuda:0") for _ in range(Q)]
    S = ls.Sorter(0)

    def slot_view(i):
        src = pristine[i % D]
        v = slots[i % Q][:src.numel()]
        return src, (v.view(torch.float64) if src.dtype == torch.float64 else v)

    # plain results (the reference of every request) and warm-up
    ref = []
    for src in pristine:
        t = src.clone()
        S.sort_(t, gp)
        ref.append(t)
    torch.cuda.synchronize()

    def run_plain(arrival):
        lat = []
        start = time.perf_counter()
        for i in range(R):
            now = time.perf_counter() - start
            if now < arrival[i]:
                time.sleep(arrival[i] - now)
            src, dst = slot_view(i)
            dst.copy_(src)
            S.sort_(dst, gp)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - start - arrival[i])
        return time.perf_counter() - start, lat

    def run_served(arrival, check=False):
        srv = ls.Server(0, hbm_budget=args.budget_gb << 30, max_inflight=args.inflight, p=gp)
        tickets, lat, bad = [None] * R, [0.0] * R, []
        sub_t = [0.0] * R
        start = time.perf_counter()
        stream = torch.cuda.Stream()

        def finish(j):
            lat[j] = sub_t[j] - arrival[j] + srv.wait(tickets[j])
            if check:
                _, out = slot_view(j)
                if not torch.equal(out.view(torch.int64), ref[j % D].view(torch.int64)):
                    bad.append(j)

        def submitter():
            with torch.cuda.stream(stream):
                for i in range(R):
                    if i >= Q:
                        finish(i - Q)             # its slot is needed again
                    now = time.perf_counter() - start
                    if now < arrival[i]:
                        time.sleep(arrival[i] - now)
                    sub_t[i] = time.perf_counter() - start
                    src, dst = slot_view(i)
                    dst.copy_(src)
                    stream.synchronize()
                    tickets[i] = srv.submit(dst)
                for j in range(max(0, R - Q), R):
                    finish(j)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        if bad:
            raise SystemExit("served and plain results differ for requests %s" % bad[:10])
        return wall, lat, st

    burst = [0.0] * R
    wp, lp = run_plain(burst)
    ws, lsv, st_b = run_served(burst)
    mu = R / wp                                # plain requests per second
    lam = 0.8 * mu
    arrival = list(np.asarray(spec.arrival_s[:R]) * (1000.0 / lam))   # spec drawn at 1000 req/s
    arrival = [a - arrival[0] for a in arrival]
    wp2, lp2 = run_plain(arrival)
    ws2, ls2, st_p = run_served(arrival)
    run_served(burst, check=True)              # untimed: every served result equals the plain one
    for j in range(min(D, 8)):                 # and the plain results equal the definition
        raw = pristine[j].view(torch.int64)
        if pristine[j].dtype == torch.float64:
            want = library_sorted_words(raw, torch)
        else:
            sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=raw.device)
            want = torch.sort(raw ^ sign)[0] ^ sign
        if not torch.equal(ref[j].view(torch.int64), want):
            raise SystemExit("plain result %d differs from torch.sort" % j)
    line = {
        "metric": METRIC, "value": total / ws, "unit": "keys/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": ws * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+u64", "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": "served_%d_requests" % R, "distinct_requests": D, "work_slots": Q,
                   "keys": total, "budget_gb": args.budget_gb, "max_inflight": args.inflight,
                   "graph": args.graph == "on"},
        "burst": {"served_keys_per_s": total / ws, "plain_keys_per_s": total / wp,
                  "served_p50_s": pct(lsv, 50), "served_p99_s": pct(lsv, 99),
                  "plain_p50_s": pct(lp, 50), "plain_p99_s": pct(lp, 99), "batches": st_b["batches"],
                  "peak_accounted_bytes": st_b["peak_bytes"]},
        "poisson": {"rate_per_s": lam, "plain_rate_per_s": mu,
                    "served_keys_per_s": total / ws2, "plain_keys_per_s": total / wp2,
                    "served_p50_s": pct(ls2, 50), "served_p99_s": pct(ls2, 99),
                    "plain_p50_s": pct(lp2, 50), "plain_p99_s": pct(lp2, 99), "batches": st_p["batches"]},
        "identical_to_plain": True,
    }
    print(json.dumps(line), flush=True)
    S.close()


# The paper's synthetic workloads (Sec. 6.1 list; Sec. 6.4 scalability on Std
# Normal and TwoDups from 1M to 1B doubles; Fig. 6 Zipf skew 0.50 - 0.99).
SWEEP_POINTS = ([("normal", n) for n in (10 ** 6, 10 ** 7, 10 ** 8, 10 ** 9)] +
                [("two_dups", n) for n in (10 ** 6, 10 ** 7, 10 ** 8, 10 ** 9)] +
                [("zipf%.2f" % s, 10 ** 8) for s in (0.5, 0.6, 0.7, 0.8, 0.9, 0.99)] +
                [(f, 10 ** 8) for f in ("root_dups", "mix_gauss", "chi_square", "exponential", "lognormal",
                                        "uniform")])


def library_sorted_words(t, torch):
    """The definition of the result, computed independently of the library:
    torch.sort (a radix sort) of the order words, turned back into the raw
    words of the keys.  t: int64 view of the f64 keys."""
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=t.device)
    neg = t < 0
    ordw = torch.where(neg, ~t, t | sign)          # totalOrder word (unsigned order)
    srt, _ = torch.sort(ordw ^ sign)               # signed order of (word ^ sign) = unsigned order of word
    srt = srt ^ sign
    return torch.where(srt < 0, srt & ~sign, ~srt)


def bench_sweep(args, torch, ls):
    """One JSON row per point of SWEEP_POINTS: keys/s of whole sorts (inputs
    resident in HBM, a fresh copy per timed sort, copies outside the events)
    and an exact check of the output against a library sort of the same keys
    on the device."""
    import workloads as W
    S = ls.Sorter(0)
    stream = torch.cuda.current_stream()
    points = SWEEP_POINTS
    if args.sweep_max_n:
        points = [(f, n) for f, n in points if n <= args.sweep_max_n]
    for fam, n in points:
        t0 = time.perf_counter()
        keys = W.paper_family_large(fam, n, seed=7)
        gen_s = time.perf_counter() - t0
        pristine = to_device(keys, torch)
        del keys
        work = torch.empty_like(pristine)
        want = library_sorted_words(pristine.view(torch.int64), torch)
        ms = []
        for step in range(args.warmup + args.steps):
            work.copy_(pristine)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            S.sort_(work)
            e1.record(stream)
            torch.cuda.synchronize()
            if step >= args.warmup:
                ms.append(e0.elapsed_time(e1))
        exact = bool(torch.equal(work.view(torch.int64), want))
        dups = int((want[1:] == want[:-1]).sum()) / n
        m = sum(ms) / len(ms)
        print(json.dumps({"metric": METRIC, "workload": "sweep", "family": fam, "n": n, "value": n / (m / 1e3),
                          "unit": "keys/s", "ms_per_sort": m, "steps": args.steps, "dtype": "f64",
                          "duplicate_ratio": dups, "exact_vs_library_sort": exact, "pipeline": S.last_stats(),
                          "generated_s": gen_s}), flush=True)
        del pristine, work, want
        torch.cuda.empty_cache()
        if not exact:
            raise SystemExit("sweep point %s n=%d differs from the library sort" % (fam, n))
    S.close()


# The spill-bucket ablation (LearnedSort 1.0, Sec. 3 / Fig. 2): Std Normal
# (no duplicates) and Zipf skews up to 0.99 at 10^8 keys.
LS1_POINTS = [("normal", 10 ** 8)] + [("zipf%.2f" % s, 10 ** 8) for s in (0.5, 0.7, 0.9, 0.99)]


def bench_ls1(args, torch, ls):
    """One JSON row per LS1_POINTS entry: keys/s of LearnedSort 2.0 (sort_)
    against the spill-bucket design of LearnedSort 1.0 (sort_ls1_, slack
    0.1) on the same keys, with the spilled share and LS1's phases; both
    results checked bit for bit against a library sort on the device."""
    import workloads as W
    S = ls.Sorter(0)
    stream = torch.cuda.current_stream()
    points = LS1_POINTS
    if args.sweep_max_n:
        points = [(f, n) for f, n in points if n <= args.sweep_max_n]
    for fam, n in points:
        keys = W.paper_family_large(fam, n, seed=7)
        pristine = to_device(keys, torch)
        del keys
        work = torch.empty_like(pristine)
        want = library_sorted_words(pristine.view(torch.int64), torch)
        row = {"metric": METRIC, "workload": "ls1_ablation", "family": fam, "n": n, "unit": "keys/s",
               "dtype": "f64", "duplicate_ratio": int((want[1:] == want[:-1]).sum()) / n, "slack": 0.1}
        for mode in ("ls2", "ls1"):
            ms, st = [], None
            for step in range(args.warmup + args.steps):
                work.copy_(pristine)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if mode == "ls2":
                    S.sort_(work)
                else:
                    st = S.sort_ls1_(work, slack=0.1)
                e1.record(stream)
                torch.cuda.synchronize()
                if step >= args.warmup:
                    ms.append(e0.elapsed_time(e1))
            exact = bool(torch.equal(work.view(torch.int64), want))
            m = sum(ms) / len(ms)
            row[mode] = {"value": n / (m / 1e3), "ms_per_sort": m, "exact_vs_library_sort": exact}
            if st:
                row[mode].update({"spilled_frac": st["spilled"] / n, "capacity": st["capacity"],
                                  "ms_phases_last_sort": {k: st[k] for k in ("ms_partition", "ms_bucket_sorts",
                                                                             "ms_spill_sort", "ms_merge")}})
            if not exact:
                raise SystemExit("ls1 ablation %s n=%d: %s differs from the library sort" % (fam, n, mode))
        row["value"] = row["ls2"]["value"]
        row["ls1_over_ls2"] = row["ls1"]["value"] / row["ls2"]["value"]
        print(json.dumps(row), flush=True)
        del pristine, work, want
        torch.cuda.empty_cache()
    S.close()


KERNEL_CLASS_OF = (("k_upload", "upload"), ("k_train", "train"), ("k_hist", "hist"), ("k_scan", "scan"),
                   ("k_classify", "classify"),
                   ("k_layout", "classify"), ("k_round_init", "classify"), ("k_scatter", "scatter"),
                   ("k_base", "base"), ("k_fill", "fill"), ("k_touchup", "touchup"))


def kernel_class(name: str):
    for pat, cls in KERNEL_CLASS_OF:
        if pat in name:
            return cls
    return None


SQ_COLUMNS = ("SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_INSTS_LDS",
              "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_WAIT_ANY", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
              "SQ_INSTS_SALU", "SQ_ACTIVE_INST_VALU")


def summarize_sq(args):
    """profiles/sq_counters_<workload>.txt from the databases of two rocprofv3
    --pmc passes (8 SQ counters each): per kernel the counters summed over its
    dispatches, and the ratios that say what bounds it."""
    import sqlite3
    per = {}
    for pi, db in enumerate(args.summarize_sq):
        con = sqlite3.connect(db)
        for name, cname, v in con.execute("select name, counter_name, counter_value from pmc_events"):
            short = name.split("(")[0].replace("void ", "").replace("lsort::", "")
            if kernel_class(name) in (None, "upload", "scan") or (pi and cname == "SQ_WAVES"):
                continue    # (both passes count the waves: the first one's are kept)
            d = per.setdefault(short, {})
            d[cname] = d.get(cname, 0.0) + v
    lines = ["# rocprofv3 SQ counters: %s" % args.workload_name, "",
             "commands (two passes, 8 SQ counters each; sums over every dispatch of the run):"]
    lines += ["  " + c for c in args.sq_commands if c]
    lines += ["", "%-30s" % "kernel" + "".join("%14s" % c.replace("SQ_", "")[:13] for c in SQ_COLUMNS)]
    for k in sorted(per, key=lambda k: -per[k].get("SQ_WAVE_CYCLES", 0.0)):
        d = per[k]
        lines.append("%-30s" % k[:30] + "".join("%14.3g" % d.get(c, 0.0) for c in SQ_COLUMNS))
    lines += ["", "derived (per kernel):"]
    for k in sorted(per, key=lambda k: -per[k].get("SQ_WAVE_CYCLES", 0.0)):
        d = per[k]
        w = d.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        lds = d.get("SQ_INSTS_LDS", 0.0) or 1.0
        lines.append("  %-28s VALU/LDS %.2f, bank-conflict cycles per LDS instruction %.2f, any wait %.0f%% and "
                     "LDS-issue wait %.0f%% of wave cycles, VALU instructions per wave %.0f" % (
                         k[:28], d.get("SQ_INSTS_VALU", 0.0) / lds, d.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds,
                         100 * d.get("SQ_WAIT_ANY", 0.0) / w, 100 * d.get("SQ_WAIT_INST_LDS", 0.0) / w,
                         d.get("SQ_INSTS_VALU", 0.0) / (d.get("SQ_WAVES", 0.0) or 1.0)))
    path = os.path.join(ROOT, "profiles", "sq_counters_%s.txt" % args.workload_name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path)


def summarize_profiles(args):
    """Turn rocprofv3 databases (a kernel trace, and optionally one FETCH_SIZE
    and one WRITE_SIZE pass) of a bench run into the text summaries kept in
    profiles/.  HBM traffic is calibrated against the device-to-device copy of
    the pristine input that every step makes (a copy of known size)."""
    import sqlite3
    wname = args.workload_name
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    con = sqlite3.connect(args.summarize_trace)
    rows = con.execute("select name, duration from kernels").fetchall()
    per = {}
    for name, dur in rows:
        cls = kernel_class(name) or ("copy" if "copyBuffer" in name else None)
        short = name.split("(")[0].replace("void ", "").replace("lsort::", "")
        d = per.setdefault((cls, short), [0, 0.0])
        d[0] += 1
        d[1] += dur
    lines = ["# rocprofv3 kernel trace: %s" % wname, "",
             "command: " + args.trace_command, "",
             "%-34s %-9s %6s %12s %12s" % ("kernel", "class", "calls", "total_us", "avg_us")]
    cls_tot = {}
    for (cls, short), (n, tot) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append("%-34s %-9s %6d %12.1f %12.2f" % (short[:34], cls or "-", n, tot / 1e3, tot / n / 1e3))
        if cls:
            c = cls_tot.setdefault(cls, [0, 0.0])
            c[0] += n
            c[1] += tot
    lines += ["", "per class (all launches of the class):",
              "%-9s %6s %12s %12s" % ("class", "calls", "total_us", "avg_us")]
    for cls, (n, tot) in sorted(cls_tot.items(), key=lambda kv: -kv[1][1]):
        lines.append("%-9s %6d %12.1f %12.2f" % (cls, n, tot / 1e3, tot / n / 1e3))
    path = os.path.join(out_dir, "kernels_%s.txt" % wname)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path)
    if not (args.summarize_fetch and args.summarize_write):
        return

    def counter(db, cname):
        c = sqlite3.connect(db)
        res = {}
        for name, did, v in c.execute("select name, dispatch_id, counter_value from pmc_events "
                                      "where counter_name = ?", (cname,)):
            res.setdefault(did, [name, 0.0])[1] += v
        return res

    fetch = counter(args.summarize_fetch, "FETCH_SIZE")
    write = counter(args.summarize_write, "WRITE_SIZE")
    copy_bytes = float(args.copy_bytes)

    def scale(vals):
        # the largest device copy is the n*8-byte restore of the pristine input
        kib = max(v for name, v in vals.values() if "copyBuffer" in name)
        return copy_bytes / (kib * 1024.0), kib

    fs, fkib = scale(fetch)
    ws, wkib = scale(write)
    cls = args.traffic_kernel
    fsel = [v for name, v in fetch.values() if kernel_class(name) == cls]
    wsel = [v for name, v in write.values() if kernel_class(name) == cls]
    fb = sum(fsel) * 1024.0 * fs / len(fsel)
    wb = sum(wsel) * 1024.0 * ws / len(wsel)
    tj = {"kernel": cls, "workload": wname, "kernel_source": kernel_source_hash(),
          "launches": len(fsel), "fetch_kib_per_launch": sum(fsel) / len(fsel),
          "write_kib_per_launch": sum(wsel) / len(wsel),
          "copy_bytes": copy_bytes, "copy_fetch_kib": fkib, "copy_write_kib": wkib,
          "fetch_scale": fs, "write_scale": ws,
          "bytes_per_launch": fb + wb, "read_bytes_per_launch": fb, "write_bytes_per_launch": wb,
          "commands": [args.fetch_command, args.write_command]}
    path = os.path.join(out_dir, "traffic_%s_%s.json" % (cls, wname))
    with open(path, "w") as f:
        json.dump(tj, f, indent=1)
        f.write("\n")
    print("wrote", path, json.dumps({k: tj[k] for k in ("fetch_scale", "write_scale", "bytes_per_launch")}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize-trace", help="rocprofv3 database of a --kernel-trace run of this script")
    ap.add_argument("--summarize-fetch", help="rocprofv3 database of a --pmc FETCH_SIZE run")
    ap.add_argument("--summarize-write", help="rocprofv3 database of a --pmc WRITE_SIZE run")
    ap.add_argument("--summarize-sq", nargs=2, help="rocprofv3 databases of the two SQ counter passes")
    ap.add_argument("--sq-commands", nargs=2, default=["", ""])
    ap.add_argument("--workload-name", default="mixed_u64")
    ap.add_argument("--traffic-kernel", default="scatter")
    ap.add_argument("--copy-bytes", type=float, default=8e9)
    ap.add_argument("--trace-command", default="")
    ap.add_argument("--fetch-command", default="")
    ap.add_argument("--write-command", default="")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed_u64")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--fanout", type=int, default=0)
    ap.add_argument("--leaves", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--base", type=int, default=0)
    ap.add_argument("--sample-cap", type=int, default=-1, help="cap on a model's sample (-1: library default)")
    ap.add_argument("--cpu-sample", type=int, default=0, help="keys the CPU oracle sorts (0: the whole array)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verify", action="store_true", help="check the sorted output against numpy")
    ap.add_argument("--inplace", action="store_true",
                    help="in-place partition rounds (fragments and block permutation; no key-sized scratch)")
    ap.add_argument("--segments", type=int, default=10_000, help="arrays of the segments workload")
    ap.add_argument("--requests", type=int, default=5000, help="requests of the served workload")
    ap.add_argument("--distinct", type=int, default=256, help="served workload: distinct requests generated")
    ap.add_argument("--ring", type=int, default=64, help="served workload: work slots (requests outstanding)")
    ap.add_argument("--sweep-max-n", type=int, default=0, help="sweep workload: skip points above this size")
    ap.add_argument("--budget-gb", type=int, default=200)
    ap.add_argument("--inflight", type=int, default=2, help="served workload: batches in flight at once")
    ap.add_argument("--graph", choices=("on", "off"), default="off",
                    help="served workload: run requests and batches of up to 2^22 keys as graph replays")
    args = ap.parse_args()
    if args.summarize_sq:
        summarize_sq(args)
    if args.summarize_trace:
        summarize_profiles(args)
    if args.summarize_sq or args.summarize_trace:
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the sort runs on a single MI355X; there is no multi-GPU path "
              "(sharding would sample per GPU, all-reduce the level-0 histogram and exchange keys once)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_03290_amd as ls

    if args.workload == "segments":
        return bench_segments(args, torch, ls)
    if args.workload == "served":
        return bench_served(args, torch, ls)
    if args.workload == "sweep":
        return bench_sweep(args, torch, ls)
    if args.workload == "ls1":
        return bench_ls1(args, torch, ls)

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
    if args.sample_cap >= 0:
        kw["sample_cap"] = args.sample_cap
    if wname == "mixed_u64" and not args.leaves and not args.inplace:
        # tuned for this workload: 512 leaves sort it as fast as 1024 with
        # the same tiles, and leave LDS room for the 12,288-key scatter tile
        kw["leaves"] = 512
    stream = torch.cuda.current_stream(dev)
    extra = ls.FLAG_INPLACE if args.inplace else 0

    def run(flags):
        work[0].copy_(pristine)
        S.sort_(work[0], ls.params(flags=flags | extra, **kw))

    breakdown, gbps, dom, flags = profiled_warmup(S, ls, run, Wm)
    p = ls.params(flags=flags | extra, **kw)
    if args.verify:
        # against torch.sort on the device (the definition of the result,
        # computed without the library)
        raw = pristine.view(torch.int64)
        if keys.dtype == np.uint64:
            sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
            want = torch.sort(raw ^ sign)[0] ^ sign
        else:
            want = library_sorted_words(raw, torch)
        if not torch.equal(work[0].view(torch.int64), want):
            raise SystemExit("verification failed")
        del want
        torch.cuda.empty_cache()
        print("verified against torch.sort", file=sys.stderr, flush=True)
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
    roof = roofline(prof, wname)
    # reference rate for the roofline: the runtime's device-to-device copy of
    # the same n * 8 bytes (read and written once, as the scatter does),
    # timed after the timed region
    cms = []
    for _ in range(3):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        work[0].copy_(pristine)
        c1.record(stream)
        torch.cuda.synchronize()
        cms.append(c0.elapsed_time(c1))
    copy_gbs = 2.0 * n * 8 / (min(cms) / 1e3) / 1e9
    roof["copy_GBps"] = copy_gbs
    roof["frac_of_copy"] = roof["achieved"] / copy_gbs
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
        "config": {"workload": wname, "n": n, "fanout": p.fanout, "leaves": p.leaves,
                   "tile": p.tile or "auto (4096; 8192, or 12288 with <= 512 leaves, in rounds of >= 2^25 keys)",
                   "base_threshold": p.base_threshold, "sample_rate": p.sample_rate, "sample_cap": p.sample_cap},
        "roofline": roof,
        "kernel_ms_per_step": breakdown,
        "kernel_GBps": gbps,
        "kernel_ms_source": "%d untimed steps after the warm-up with every kernel class timed; the timed "
                            "steps time the dominant class (%s) only" % (PROFILED_STEPS, dom),
        "pipeline": stats[-1],
        "wall_s_timed": wall,
        "context_device_bytes": S.device_bytes(),
    }
    if args.inplace:
        # the in-place rounds time the fragment pass in the histogram's class
        # and the block permutation with the gather in the scatter's
        line["config"]["partition"] = "in-place (Alg. 1 fragments, then block permutation and gather)"
        line["config"]["class_names"] = {"hist": "fragments (k_ip_frag)",
                                         "scatter": "plan + permutation + gather (k_ip_plan/permute/gather)"}
        line["extra_device_frac"] = S.device_bytes() / (n * 8.0)
    if not args.no_cpu_baseline:
        take = min(args.cpu_sample, n) if args.cpu_sample > 0 else n
        line["cpu_baseline"] = cpu_baseline(keys, take)
        line["cpu_library_sort"] = cpu_library_sort(keys, take)
    print(json.dumps(line), flush=True)
    S.close()


if __name__ == "__main__":
    main()
