"""Autotuner for the table's launch shapes (results never depend on them).

For each batch-size class it times, with HIP events on the device, the candidate shapes of
- a program's merged find run: lanes per key (4/8/16), loading both candidate digest lines at
  once or b2 after a miss, and the grid (one lane group per key, or a persistent grid of k
  blocks per compute unit);
- the upsert routing kernel's lanes per key;
and keeps the fastest.  `apply` sets the tuned shape for a batch of n keys before it is added to
a program (or issued as a single call).
"""
from __future__ import annotations

import torch

from . import cskv

CLASSES = [("small", 0, 1 << 13), ("medium", 1 << 13, 1 << 17), ("large", 1 << 17, 1 << 62)]
CLASS_SIZE = {"small": 1 << 12, "medium": 1 << 15, "large": 1 << 20}
FIND_SHAPES = [(g, pre, bpc) for g in (4, 8, 16) for pre in (0, 1) for bpc in (0, 4, 8)]
ROUTE_SHAPES = (4, 8, 16)


def size_class(n: int) -> str:
    for name, lo, hi in CLASSES:
        if lo <= n < hi:
            return name
    return CLASSES[-1][0]


def _timed(fn, reps: int = 3) -> float:
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_find(table: cskv.Table, queries_by_class: dict, log=None) -> dict:
    """queries_by_class: class name -> int64 key tensor on the device (a typical find batch)."""
    out = {}
    dev = table.device
    for cls, q in queries_by_class.items():
        n = q.numel()
        vals = torch.empty((n, table.dim), dtype=torch.float32, device=dev)
        found = torch.empty(n, dtype=torch.uint8, device=dev)
        best = None
        for g, pre, bpc in FIND_SHAPES:
            table.set_tuning(find_group=g, find_prefetch_b2=pre, find_blocks_per_cu=bpc)
            prog = cskv.Program(table)
            prog.add_find(q, vals, found)
            prog.finalize()
            ms = _timed(prog.launch)
            if log:
                log(f"autotune find[{cls}] group {g} prefetch {pre} blocks/CU {bpc}: {ms * 1e3:.1f} us")
            if best is None or ms < best[0]:
                best = (ms, g, pre, bpc)
        out[cls] = {"find_group": best[1], "find_prefetch_b2": best[2], "find_blocks_per_cu": best[3]}
    return out


def tune_route(table: cskv.Table, fresh_by_class: dict, log=None) -> dict:
    """fresh_by_class: class name -> fresh (absent) keys; each trial inserts them and erases them
    again, so the table ends as it started unless a trial evicted a resident (possible at high
    load: one call routes all its keys against the same snapshot and can overfill a bucket);
    callers that need the table unchanged snapshot its storage around the tuning."""
    out = {}
    dev = table.device
    for cls, k in fresh_by_class.items():
        n = k.numel()
        vals = torch.zeros((n, table.dim), dtype=torch.float32, device=dev)
        st = torch.empty(n, dtype=torch.uint8, device=dev)
        er = torch.empty(n, dtype=torch.uint8, device=dev)
        sc = torch.ones(n, dtype=torch.int64, device=dev)
        best = None
        for g in ROUTE_SHAPES:
            table.set_tuning(route_group=g)

            def trial():
                table.insert_or_assign(k, vals, sc, status_out=st)
                table.erase(k, erased_out=er)

            ms = _timed(trial)
            if log:
                log(f"autotune route[{cls}] group {g}: {ms * 1e3:.1f} us")
            if best is None or ms < best[0]:
                best = (ms, g)
        out[cls] = {"route_group": best[1]}
    return out


def merge(*parts: dict) -> dict:
    res = {}
    for p in parts:
        for cls, cfg in p.items():
            res.setdefault(cls, {}).update(cfg)
    return res


def apply(table: cskv.Table, tuning: dict, n: int):
    cfg = tuning.get(size_class(n))
    if cfg:
        table.set_tuning(**cfg)
