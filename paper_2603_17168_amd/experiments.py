"""Eviction-quality experiments of the paper (Exp. 3c, 3d and 4) on seeded synthetic streams.

Each protocol drives a table through a minimal interface, so that the same protocol runs on the
GPU table (``GpuTable``) and, in the tests, on the sequential oracle:

    upsert(keys, scores | None) -> status u8[n]      insert_or_assign
    find(keys) -> found u8[n]                        contains
    size() -> int

Keys and scores are int64 tensors (u64 bit patterns) on the generation device ``dev``; results
come back on the table's device and are moved to ``dev``.

Protocol choices (the paper gives the metrics and the headline parameters; the rest is chosen
here):

* A universe of U = 10 x capacity keys, key of rank r = ``keys_at(stream, r)``; Zipf(alpha)
  ranks.  With this universe LFU's hit ratio sits at the static optimum H(C)/H(U) that the
  paper's LFU column shows (31 % at alpha = 0.5, 88 % at alpha = 0.99 for C = 128 M).
* Scores by step: CUSTOM gets the index of the upsert call (a recency score, so that it orders
  entries exactly as the LRU clock does), LRU the table clock, LFU +1 per occurrence.
* first_eviction (Exp. 4): fresh uniform keys in batches (all keys of a batch share one score);
  the load factor before the first batch in which a key evicts or is refused.  The resolution
  is batch / capacity (a batch's keys are placed per bucket in key order, not in batch order,
  so a position inside the batch does not mark a sequential point).
* zipf_ingestion (Exp. 3c, 4): the table is first filled to load 1.0 with fresh filler keys
  (batches of the same size and scoring), then `capacities` x capacity Zipf keys arrive in
  batches; each batch is looked up, then upserted.  The hit ratio counts the lookups after the
  first capacity of Zipf keys.  Top-N retention (recency scores): the share of the N =
  capacity highest-scored keys offered (each key's score = its last upsert call) that are
  resident at the end; keys tied at the boundary score count up to the remaining budget.
* admission_burst (Exp. 3d): an LFU table fed Zipf(0.99) batches until load >= 0.96, then a
  burst of capacity / 4 fresh keys with increment s in one call; the shares of the burst that
  took free slots, displaced residents or were rejected, and the hit ratio of a fixed
  Zipf(0.99) query set of the universe before and after the burst.
"""
from __future__ import annotations

import torch

from . import cskv
from .workload import Zipf, keys as gen_keys, keys_at

INSERTED, INSERTED_EVICT, REJECTED = cskv.ST_INSERTED, cskv.ST_INSERTED_EVICT, cskv.ST_REJECTED
UNIVERSE_FACTOR = 10


class GpuTable:
    """The experiment interface over a cskv.Table (value rows of dim 4, all zero)."""

    def __init__(self, capacity: int, mode: str, policy: str, device="cuda", subrounds: int = 1):
        self.t = cskv.Table(capacity, 4, mode=mode, policy=policy, device=device)
        if subrounds != 1:
            self.t.set_route_subrounds(subrounds)
        self._zero = torch.zeros((0, 4), dtype=torch.float32, device=self.t.device)

    def _rows(self, n):
        if self._zero.shape[0] < n:
            self._zero = torch.zeros((n, 4), dtype=torch.float32, device=self.t.device)
        return self._zero[:n]

    def upsert(self, keys, scores=None):
        kd = keys.to(self.t.device)
        sd = None if scores is None else scores.to(self.t.device)
        return self.t.insert_or_assign(kd, self._rows(kd.numel()), sd)

    def find(self, keys):
        return self.t.contains(keys.to(self.t.device))

    def size(self):
        return self.t.size()


def _scores(policy: str, n: int, step: int, dev):
    if policy == "custom":
        return torch.full((n,), step, dtype=torch.int64, device=dev)
    if policy == "lfu":
        return torch.ones(n, dtype=torch.int64, device=dev)
    return None


def first_eviction(table, capacity: int, batch: int, stream: int = 61, dev="cpu") -> float:
    """Load factor before the first batch of fresh keys in which a key evicts or is refused."""
    offered = 0
    step = 0
    while offered < 4 * capacity:
        n = min(batch, 4 * capacity - offered)
        size_before = table.size()
        step += 1
        st = table.upsert(gen_keys(stream, n, offered, dev), torch.full((n,), step, dtype=torch.int64, device=dev))
        offered += n
        if bool((st != INSERTED).any()):
            return size_before / capacity
    return 1.0


def _retention(table, last_u, last_f, stream, filler_stream, n_top, dev, chunk=1 << 22):
    """Share of the n_top highest-scored offered keys that are resident (ties at the boundary
    score fill the remaining budget)."""
    top = int(max(int(last_u.max()), int(last_f.max()) if last_f.numel() else 0))
    hist = torch.bincount(last_u, minlength=top + 1) + torch.bincount(last_f, minlength=top + 1)
    hist[0] = 0  # never offered
    above = torch.flip(torch.cumsum(torch.flip(hist, [0]), 0), [0])  # keys with score >= s
    n_top = min(n_top, int(above[1]))
    if n_top == 0:
        return 1.0
    s_n = int(torch.nonzero(above >= n_top)[-1, 0])  # the boundary score
    strict = int(above[s_n + 1]) if s_n + 1 <= top else 0
    hits_strict = hits_tie = 0
    for group, stream_id in ((last_u, stream), (last_f, filler_stream)):
        for sel, is_tie in ((group > s_n, False), (group == s_n, True)):
            idx = torch.nonzero(sel).flatten()
            for c in range(0, idx.numel(), chunk):
                f = table.find(keys_at(stream_id, idx[c:c + chunk])).to(dev)
                if is_tie:
                    hits_tie += int(f.sum())
                else:
                    hits_strict += int(f.sum())
    return (hits_strict + min(hits_tie, n_top - strict)) / n_top


def zipf_ingestion(table, capacity: int, alpha: float, policy: str, batch: int, capacities: int = 5,
                   stream: int = 62, seed: int = 63, dev="cpu", retention: bool = False) -> dict:
    U = UNIVERSE_FACTOR * capacity
    z = Zipf(alpha, U)
    filler_stream = stream + 1
    step = 0
    # fill to load 1.0 with fresh filler keys
    n_fill = 0
    fill_cap = 4 * capacity
    last_f = torch.zeros(fill_cap if retention else 0, dtype=torch.int64, device=dev)
    while table.size() < capacity and n_fill < fill_cap:
        n = min(batch, fill_cap - n_fill)
        step += 1
        table.upsert(gen_keys(filler_stream, n, n_fill, dev), _scores(policy, n, step, dev))
        if retention:
            last_f[n_fill:n_fill + n] = step
        n_fill += n
    load_filled = table.size() / capacity
    # sustained Zipf ingestion
    last_u = torch.zeros(U + 1 if retention else 0, dtype=torch.int64, device=dev)
    total = capacities * capacity
    warm = capacity
    hits = torch.zeros((), dtype=torch.int64, device=dev)
    looks = 0
    done = 0
    while done < total:
        n = min(batch, total - done)
        ranks = z.sample_device(seed * 1_000_003 + done, n, dev)
        k = keys_at(stream, ranks)
        f = table.find(k).to(dev)
        if done >= warm:
            hits += f.sum()
            looks += n
        step += 1
        table.upsert(k, _scores(policy, n, step, dev))
        if retention:
            last_u[ranks] = step
        done += n
    out = {"hit_ratio": int(hits) / looks if looks else 0.0, "load_filled": load_filled,
           "load": table.size() / capacity}
    if retention:
        out["top_n_retention"] = _retention(table, last_u, last_f[:n_fill], stream, filler_stream, capacity, dev)
    return out


def admission_burst(table, capacity: int, burst_increment: int, batch: int, stream: int = 64, seed: int = 65,
                    dev="cpu") -> dict:
    U = UNIVERSE_FACTOR * capacity
    z = Zipf(0.99, U)
    done = 0
    while table.size() < 0.96 * capacity and done < 64 * capacity:
        n = batch
        table.upsert(keys_at(stream, z.sample_device(seed * 1_000_003 + done, n, dev)),
                     torch.ones(n, dtype=torch.int64, device=dev))
        done += n
    load = table.size() / capacity
    q = keys_at(stream, z.sample_device(seed * 1_000_003 - 1, 4 * batch, dev))
    before = float(table.find(q).to(dev).float().mean())
    nb = max(1, capacity // 4)
    burst = gen_keys(stream + 1, nb, 0, dev)
    st = table.upsert(burst, torch.full((nb,), burst_increment, dtype=torch.int64, device=dev)).to(dev)
    after = float(table.find(q).to(dev).float().mean())
    share = lambda s: float((st == s).float().mean())
    return {"load_before": load, "free_slot_inserts": share(INSERTED), "evicting_admissions": share(INSERTED_EVICT),
            "rejected": share(REJECTED), "hit_before": before, "hit_after": after,
            "delta_hit_pp": 100.0 * (after - before)}


def main():
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description="eviction-quality experiments on the GPU table (one JSON line)")
    ap.add_argument("--log2-capacity", type=int, default=27, help="table of Exp. 3c and 4")
    ap.add_argument("--burst-log2-capacity", type=int, default=24, help="table of Exp. 3d")
    ap.add_argument("--batch", type=int, default=1 << 20, help="keys per call of the ingestion experiments")
    ap.add_argument("--capacities", type=int, default=5, help="Zipf keys ingested, in table capacities")
    ap.add_argument("--alphas", default="0.5,0.75,0.99,1.25")
    args = ap.parse_args()
    cap = 1 << args.log2_capacity
    dev = "cuda"
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    res = {"capacity": cap, "batch": args.batch, "ingested_capacities": args.capacities,
           "universe": UNIVERSE_FACTOR * cap}
    res["first_eviction_load"] = {}
    for m in ("single", "dual"):
        res["first_eviction_load"][m] = round(first_eviction(GpuTable(cap, m, "custom"), cap, max(1, cap // 1024),
                                                             dev=dev), 4)
        log(f"first eviction {m}: {res['first_eviction_load'][m]}")
    # snapshot routing: every key of a call sees the occupancies from before the call, so larger
    # calls in dual mode overflow earlier
    res["first_eviction_dual_by_batch"] = {}
    for lb in range(args.log2_capacity - 13, args.log2_capacity - 5, 2):
        res["first_eviction_dual_by_batch"][str(1 << lb)] = round(
            first_eviction(GpuTable(cap, "dual", "custom"), cap, 1 << lb, dev=dev), 4)
    log(f"first eviction dual by batch: {res['first_eviction_dual_by_batch']}")
    # route sub-rounds at the ingestion batch size: each chunk sees the occupancies the chunks
    # before it left
    res["first_eviction_dual_by_subrounds"] = {
        str(r): round(first_eviction(GpuTable(cap, "dual", "custom", subrounds=r), cap, args.batch, dev=dev), 4)
        for r in (1, 2, 4, 8, 16)}
    log(f"first eviction dual at batch {args.batch} by sub-rounds: {res['first_eviction_dual_by_subrounds']}")
    res["zipf0.99_lru"] = {}
    for m in ("single", "dual"):
        r = zipf_ingestion(GpuTable(cap, m, "lru"), cap, 0.99, "lru", args.batch, args.capacities, dev=dev,
                           retention=True)
        res["zipf0.99_lru"][m] = {k: round(v, 4) for k, v in r.items()}
        log(f"zipf 0.99 lru {m}: {r}")
    res["hit_ratio_single"] = {}
    for pol in ("lru", "lfu", "custom"):
        res["hit_ratio_single"][pol] = {}
        for a in [float(x) for x in args.alphas.split(",")]:
            r = zipf_ingestion(GpuTable(cap, "single", pol), cap, a, pol, args.batch, args.capacities, dev=dev)
            res["hit_ratio_single"][pol][str(a)] = round(r["hit_ratio"], 4)
            log(f"hit ratio single {pol} alpha {a}: {r}")
    bcap = 1 << args.burst_log2_capacity
    res["admission_burst"] = {"capacity": bcap}
    for inc in (1, 10 ** 9):
        r = admission_burst(GpuTable(bcap, "dual", "lfu"), bcap, inc, max(1, bcap // 128), dev=dev)
        res["admission_burst"][str(inc)] = {k: round(v, 4) for k, v in r.items()}
        log(f"admission burst s={inc}: {r}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
