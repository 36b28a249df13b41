"""Benchmark: find & upsert throughput of the cache-semantic hash table over load factors.

Workload (one GPU): the 2^26-slot table (2^19 buckets x 128), dim-32 fp32 rows, dual-bucket
mode, LRU scores, batches of 2^20 uniform random u64 keys.  Four tables are pre-filled (untimed)
to load factors 0.50 / 0.75 / 0.90 / 1.00.  One step runs, on every table:
  find of 2^20 resident keys (100 % hit), find of 2^20 keys at 50 % hit, insert_or_assign of
  2^20 fresh keys, then (below full load) erase of those keys so the load factor stays put.
`value` counts the find and upsert keys of a step (not the erases) over the wall time of the
whole step, erases included.  Inputs are resident in device memory before timing starts.

Also reported: per-op rates from HIP events, per-batch latency percentiles, the HBM roofline
of the find kernel from its algorithmic bytes, and the sequential CPU oracle timed on a sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2603_17168_amd import cskv  # noqa: E402
from paper_2603_17168_amd.workload import keys as gen_keys, randint, value_rows  # noqa: E402

METRIC = "find & upsert B-KV/s at load 0.5–1.0, % of HBM peak; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
K_B, F_B, L_B, S_B = 8, 1, 128, 64  # input key, found flag, digest line, DRAM access granule


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def find_bytes_per_key(dim: int, hit: bool, load: float) -> float:
    """Algorithmic bytes of one find (dual mode), counting every hit as a b1 hit (a lower bound):
    hit  = key + digest line + key granule + row read + row write + flag
    miss = key + two digest lines + expected false-positive key granules + flag."""
    V = 4 * dim
    if hit:
        return K_B + L_B + S_B + 2 * V + F_B
    return K_B + 2 * L_B + load * 0.5 * S_B + F_B


class Level:
    def __init__(self, table, load, resident_keys):
        self.t = table
        self.target = load
        self.resident = resident_keys


def fill(t: cskv.Table, target: float, batch: int, dim: int, key_stream: int, start: int, dev):
    """Insert fresh-key batches until size >= target * capacity (or 2x capacity offered)."""
    cap = t.capacity
    offered = start
    while True:
        n = batch
        k = gen_keys(key_stream, n, offered, device=dev)
        v = value_rows(11, k, dim)
        t.insert_or_assign(k, v, want_status=False)
        offered += n
        size = t.size()
        if size >= target * cap or offered >= 2 * cap:
            return offered, size


def clone(src: cskv.Table) -> cskv.Table:
    dst = cskv.Table(src.capacity, src.dim, mode=src.mode, policy=src.policy, device=src.device)
    dst.storage.copy_(src.storage)
    dst.clock = src.clock
    return dst


def autotune(t, q100, q50, fresh, rows, outs, found, status, erased, reps=3):
    """Pick find group/prefetch and route group by HIP-event timing on sample batches."""
    def timed(fn):
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return min(ts)

    best = None
    for g in (4, 8, 16):
        for pre in (0, 1):
            t.set_tuning(find_group=g, find_prefetch_b2=pre)
            ms = timed(lambda: (t.find(q100, values_out=outs, found_out=found, want_scores=False),
                                t.find(q50, values_out=outs, found_out=found, want_scores=False)))
            log(f"autotune find group {g} prefetch {pre}: {ms:.3f} ms")
            if best is None or ms < best[0]:
                best = (ms, g, pre)
    tuning = {"find_group": best[1], "find_prefetch_b2": best[2]}
    t.set_tuning(**tuning)
    best_r = None
    for g in (8, 16):
        t.set_tuning(route_group=g)
        ms = timed(lambda: (t.insert_or_assign(fresh, rows, status_out=status), t.erase(fresh, erased_out=erased)))
        log(f"autotune route group {g}: {ms:.3f} ms")
        if best_r is None or ms < best_r[0]:
            best_r = (ms, g)
    tuning["route_group"] = best_r[1]
    return tuning


def cpu_baseline(loads, sample_log2_cap=22, batch=1 << 18):
    """Sequential C oracle (one thread) on a sample: a 2^22-slot dual LRU table filled to each
    load factor (untimed), then the step's three ops on 2^18-key batches, timed."""
    import oracle
    from paper_2603_17168_amd.workload import as_u64

    cap = 1 << sample_log2_cap
    o = oracle.Oracle(cap // 128, 128, oracle.DUAL, oracle.LRU)
    offered = 0
    tot_keys = 0
    tot_s = 0.0
    rng = np.random.default_rng(0)
    for lam in loads:
        while o.size() < lam * cap and offered < 2 * cap:
            k = as_u64(gen_keys(3, batch, offered))
            o.upsert(k, np.zeros(batch, np.uint64))
            offered += batch
        res = o.export()[0]
        q100 = res[rng.integers(0, res.size, batch)]
        q50 = np.concatenate([res[rng.integers(0, res.size, batch // 2)], as_u64(gen_keys(998, batch // 2))])
        fresh = as_u64(gen_keys(997, batch, offered))
        t0 = time.perf_counter()
        o.find(q100)
        o.find(q50)
        o.upsert(fresh, np.zeros(batch, np.uint64))
        tot_s += time.perf_counter() - t0
        tot_keys += 3 * batch
        if lam < 1.0:
            o.erase(fresh)
    return {"value": tot_keys / tot_s / 1e6, "unit": "M-KV/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential C oracle, 2^{sample_log2_cap}-slot dual LRU table filled to loads {loads}; "
                      f"per load one find (100% hit), one find (50% hit) and one insert_or_assign of "
                      f"2^{int(np.log2(batch))} keys; {tot_s:.1f} s timed"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2-capacity", type=int, default=26)
    ap.add_argument("--dim", type=int, default=32)
    ap.add_argument("--log2-batch", type=int, default=20)
    ap.add_argument("--loads", type=str, default="0.5,0.75,0.9,1.0")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see the sharding notes); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cap = 1 << args.log2_capacity
    dim = args.dim
    batch = 1 << args.log2_batch
    loads = [float(x) for x in args.loads.split(",")]

    # ---------------- setup (untimed): tables at each load factor, query sets
    base = cskv.Table(cap, dim, mode="dual", policy="lru", device=dev)
    levels = []
    offered = 0
    for lam in loads:
        offered, size = fill(base, lam, batch, dim, 1, offered, dev)
        t = clone(base)
        k, _, _, _ = t.export(with_values=False)
        levels.append(Level(t, lam, k))
        log(f"setup: load {lam:.2f} -> size {size} ({size / cap:.4f}), offered {offered}")
    del base
    torch.cuda.synchronize()

    n_steps_total = args.warmup + args.steps
    q100, q50, fresh, fresh_rows = [], [], [], []
    for li, lv in enumerate(levels):
        r = lv.resident
        idx = randint(100 + li, batch, r.numel(), device=dev)
        q100.append(r[idx])
        idx2 = randint(200 + li, batch // 2, r.numel(), device=dev)
        miss = gen_keys(900, batch // 2, li * batch, device=dev)
        perm = torch.argsort(randint(300 + li, batch, 1 << 40, device=dev))
        q50.append(torch.cat([r[idx2], miss])[perm])
        fk = gen_keys(500 + li, batch * n_steps_total, 0, device=dev).view(n_steps_total, batch)
        fresh.append(fk)
    rows = value_rows(12, gen_keys(600, batch, 0, device=dev), dim)
    outs = torch.empty((batch, dim), dtype=torch.float32, device=dev)
    found = torch.empty(batch, dtype=torch.uint8, device=dev)
    status = torch.empty(batch, dtype=torch.uint8, device=dev)
    erased = torch.empty(batch, dtype=torch.uint8, device=dev)
    for lv in levels:
        lv.t.workspace(cskv.OP_INSERT_OR_ASSIGN, batch)
        lv.t.workspace(cskv.OP_ERASE, batch)
    torch.cuda.synchronize()

    # autotune launch shapes (results do not depend on them) on the first table
    tuning = autotune(levels[0].t, q100[0], q50[0], gen_keys(700, batch, 0, device=dev), rows, outs, found, status,
                      erased)
    for lv in levels:
        lv.t.set_tuning(**tuning)
    log(f"tuning: {tuning}")

    ev = {}

    def rec(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        ev.setdefault(name, []).append(e)

    def step(s, timed):
        for li, lv in enumerate(levels):
            t = lv.t
            if timed:
                rec(f"f100_{li}_a")
            t.find(q100[li], values_out=outs, found_out=found, want_scores=False)
            if timed:
                rec(f"f100_{li}_b")
            t.find(q50[li], values_out=outs, found_out=found, want_scores=False)
            if timed:
                rec(f"f50_{li}_b")
            t.insert_or_assign(fresh[li][s], rows, status_out=status)
            if timed:
                rec(f"ups_{li}_b")
            if lv.target < 1.0:
                t.erase(fresh[li][s], erased_out=erased)

    for s in range(args.warmup):
        step(s, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, n_steps_total):
        step(s, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    kv_per_step = len(levels) * 3 * batch
    value = kv_per_step * args.steps / wall / 1e9
    per_op = {}
    find_ms, find_bytes, lat = [], [], {"find": [], "upsert": []}
    for li, lv in enumerate(levels):
        a, b1, b2, b3 = ev[f"f100_{li}_a"], ev[f"f100_{li}_b"], ev[f"f50_{li}_b"], ev[f"ups_{li}_b"]
        f100 = [x.elapsed_time(y) for x, y in zip(a, b1)]
        f50 = [x.elapsed_time(y) for x, y in zip(b1, b2)]
        ups = [x.elapsed_time(y) for x, y in zip(b2, b3)]
        lam = lv.resident.numel() / cap
        per_op[f"{lv.target:.2f}"] = {
            "load": round(lam, 4),
            "find_hit100_bkvs": round(batch / np.median(f100) / 1e6, 3),
            "find_hit50_bkvs": round(batch / np.median(f50) / 1e6, 3),
            "insert_or_assign_bkvs": round(batch / np.median(ups) / 1e6, 3),
        }
        lat["find"] += f100 + f50
        lat["upsert"] += ups
        find_ms += f100 + f50
        find_bytes += [batch * find_bytes_per_key(dim, True, lam)] * len(f100)
        find_bytes += [batch * 0.5 * (find_bytes_per_key(dim, True, lam) + find_bytes_per_key(dim, False, lam))] * len(f50)
    achieved = float(np.sum(find_bytes) / (np.sum(find_ms) / 1e3) / 1e9)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "B-KV/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"plain table at scale: capacity 2^{args.log2_capacity} slots (2^{args.log2_capacity - 7} "
                               f"buckets x 128), dim {dim} fp32, dual-bucket, LRU, 2^{args.log2_batch}-key batches of "
                               f"uniform u64 keys; per load: find 100% hit, find 50% hit, insert_or_assign fresh keys",
                   "capacity": cap, "dim": dim, "batch": batch, "loads": loads, "mode": "dual", "policy": "lru"},
        "per_op": per_op,
        "latency_ms": {k: {"p50": round(float(np.percentile(v, 50)), 4), "p99": round(float(np.percentile(v, 99)), 4)}
                       for k, v in lat.items() if v},
        "tuning": tuning,
        "roofline": {"bound": "hbm", "kernel": f"k_find<{tuning['find_group']},{bool(tuning['find_prefetch_b2'])}>", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the sequential oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(loads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
