"""The evaluation workloads at their stated sizes (Sec. 5.1 configurations as this repository
instantiates them), compared with the sequential oracle call by call and table by table.

* C2 - 2^26 slots, dim 32, dual, LRU, 2^20-key calls, the way the benchmark runs it: fresh-key
  fills to each load 0.50 / 0.75 / 0.90 / 1.00, a copy of the table per load, then on the copy a
  100 %-hit find, a 50 %-hit find, an insert_or_assign of fresh keys and (below load 1) the erase
  that restores the load.  Every fill call's statuses and, per load, both tables are compared.
* C4 - the batched program on a 2^26-slot dim-32 LRU table filled to load 0.9: 256 uneven batches
  (log-uniform 1K-1M keys, 70 % find / 25 % insert_or_assign / 5 % erase) captured once as a
  graph and replayed; every batch's outputs and the final table against the oracle.
* C3 - continuous online eviction at 2^27 slots, dim 64, LFU: filled with uniform keys above 2^32
  (increment 1), then steps of insert_and_evict of 2^20 Zipf(1.05) keys over 2^32 (increment 1
  per occurrence, repeats summed) and a find of 2^20 fresh Zipf keys; statuses, evicted sets and
  finds of every step and the final table.  The step count defaults to 20 (environment variable
  CSKV_C3_STEPS) so that the whole file fits one test run.
* C5 - the serving loop's serialization order replayed through the oracle: 10^4 requests
  (lognormal(4096, 1.0) sizes clipped to 256-65536, 90 % find / 10 % insert_and_evict, Zipf(1.1)
  keys over 2^34, Poisson arrivals, reader groups on two streams of their own) on a 2^22-slot
  dim-32 LRU table filled with ranks 1..2^22.

Rows are compared through value-ids: every inserted occurrence carries its own id, and the GPU's
rows must equal the generator's rows of the ids the oracle holds.  The oracle side of each
workload runs in a background thread from the moment this module starts (see tests/fullsize.py).
"""
import os

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv, serve
from paper_2603_17168_amd.workload import (Zipf, batch_schedule, keys as gen_keys, lognormal_sizes,
                                            poisson_arrivals, randint, uniform01, uniform_u64)
from tests import fullsize as fs
from tests.fullsize import GpuSide, OracleRun, OracleSide, lockstep, say

pytestmark = pytest.mark.gpu

B20 = 1 << 20
C3_STEPS = int(os.environ.get("CSKV_C3_STEPS", "20"))


def u64(t: torch.Tensor) -> np.ndarray:
    return t.numpy().view(np.uint64)


class Vids:
    """Value-id counter: every inserted occurrence gets its own id."""

    def __init__(self, start=1):
        self.v = start

    def take(self, n):
        r = np.arange(self.v, self.v + n, dtype=np.uint64)
        self.v += n
        return r


# ------------------------------------------------------------------------------------ C2
C2_CAP, C2_DIM, C2_SEED = 1 << 26, 32, 41
C2_LOADS = (0.5, 0.75, 0.9, 1.0)


def c2_scenario(side):
    vids = Vids()
    offered = 0
    for li, lam in enumerate(C2_LOADS):
        while True:  # fresh-key fills of 2^20 keys until the load is reached
            k = u64(gen_keys(1, B20, offered))
            yield f"fill@{offered >> 20}", side.upsert(k, vids.take(B20))
            offered += B20
            if side.size() >= lam * C2_CAP or offered >= 2 * C2_CAP:
                break
        lv = side.clone()
        yield f"table {lam}", lv.table()
        res = lv.residents()
        q100 = res[u64(randint(100 + li, B20, res.size))]
        idx2 = u64(randint(200 + li, B20 // 2, res.size))
        miss = u64(gen_keys(900, B20 // 2, li * B20))
        perm = torch.argsort(randint(300 + li, B20, 1 << 40)).numpy()
        q50 = np.concatenate([res[idx2], miss])[perm]
        yield f"find100 {lam}", lv.find(q100)
        yield f"find50 {lam}", lv.find(q50)
        fresh = u64(gen_keys(500 + li, B20, 0))
        yield f"insert {lam}", lv.upsert(fresh, vids.take(B20))
        if lam < 1.0:
            yield f"erase {lam}", lv.erase(fresh)
        yield f"table after step {lam}", lv.table()
        del lv


# ------------------------------------------------------------------------------------ C4
C4_CAP, C4_DIM, C4_SEED = 1 << 26, 32, 43


def c4_prefill(side, vids):
    offered = 0
    while True:
        k = u64(gen_keys(2, B20, offered))
        yield f"prefill@{offered >> 20}", side.upsert(k, vids.take(B20))
        offered += B20
        if side.size() >= 0.9 * C4_CAP or offered >= 2 * C4_CAP:
            break
    side.prefill_keys = u64(gen_keys(2, offered, 0))
    yield "prefilled table", side.table()


def c4_inputs(resident: np.ndarray, vids: Vids):
    """The 256 batches: (op, keys, value-ids or None)."""
    sched = batch_schedule(47, 256, 1 << 10, 1 << 20)
    nres = resident.size
    fresh_ctr = miss_ctr = 0
    out = []
    for j, (op, n) in enumerate(sched):
        if op == "find":
            h = n // 2
            q = np.concatenate([resident[u64(randint(10_000 + j, n - h, nres))], u64(gen_keys(48, h, miss_ctr))])
            miss_ctr += h
            q = q[torch.argsort(uniform_u64(20_000 + j, n)).numpy()]
            out.append((op, q, None))
        elif op == "upsert":
            out.append((op, u64(gen_keys(49, n, fresh_ctr)), vids.take(n)))
            fresh_ctr += n
        else:
            out.append((op, resident[u64(randint(30_000 + j, n, nres))], None))
    return out


def c4_oracle(side):
    vids = Vids()
    yield from c4_prefill(side, vids)
    for j, (op, k, v) in enumerate(c4_inputs(side.prefill_keys, vids)):
        if op == "find":
            yield f"batch {j} find", side.find(k)
        elif op == "upsert":
            yield f"batch {j} upsert", side.upsert(k, v)
        else:
            yield f"batch {j} erase", side.erase(k)
    yield "final table", side.table()
    yield "final clock", {"final_clock": side.clock()}


# ------------------------------------------------------------------------------------ C3
C3_CAP, C3_DIM, C3_SEED = 1 << 27, 64, 45
C3_PREFILL_MAX = C3_CAP + C3_CAP // 4  # keys offered at most while filling


def c3_scenario(side):
    vids = Vids()
    offered = 0
    while True:  # uniform keys above 2^32, LFU increment 1
        k = u64(gen_keys(63, B20, offered)) | np.uint64(1 << 40)
        yield f"prefill@{offered >> 20}", side.upsert(k, vids.take(B20))
        offered += B20
        if side.size() >= C3_CAP or offered >= C3_PREFILL_MAX:
            break
    yield "prefilled table", side.table()
    z = Zipf(1.05, 1 << 32)
    for step in range(C3_STEPS):
        k = z.sample(64 + step, B20)
        yield f"step {step} insert_and_evict", side.upsert(k, vids.take(B20), evict=True)
        yield f"step {step} find", side.find(z.sample(5000 + step, B20))
    yield "final table", side.table()


# ------------------------------------------------------------------------------------ C5
C5_CAP, C5_DIM, C5_SEED, C5_NREQ = 1 << 22, 32, 47, 10_000


def c5_trace():
    sizes = lognormal_sizes(31, C5_NREQ, 4096.0, 1.0, 256, 65536)
    ops = np.where(uniform01(32, C5_NREQ).numpy() < 0.9, serve.REQ_FIND, serve.REQ_INSERT_AND_EVICT)
    keys = Zipf(1.1, 1 << 34).sample(33, int(sizes.sum()))
    arrivals = poisson_arrivals(34, C5_NREQ, 100_000.0)
    return ops, sizes, keys, arrivals


def c5_prefill(side, vids):
    for s in range(0, C5_CAP, B20):
        k = np.arange(1 + s, 1 + s + B20, dtype=np.uint64)
        yield f"prefill@{s >> 20}", side.upsert(k, vids.take(B20))


def c5_oracle(trace):
    ops, sizes, keys, _ = trace

    def scenario(side):
        vids = Vids()
        yield from c5_prefill(side, vids)
        off = np.concatenate([[0], np.cumsum(sizes)])
        for i in range(C5_NREQ):  # arrival order (= the serialization order, checked on the GPU side)
            k = keys[off[i]:off[i + 1]]
            if ops[i] == serve.REQ_FIND:
                yield f"request {i}", side.find(k)
            else:
                yield f"request {i}", side.upsert(k, vids.take(k.size), evict=True)
        yield "final table", side.table()
    return scenario


# ------------------------------------------------------------------------------------ fixture
@pytest.fixture(scope="module")
def oracle_runs():
    """Start every oracle scenario at once, each in its own thread."""
    c5 = c5_trace()
    runs = {
        "C3": OracleRun("C3", c3_scenario, lambda: OracleSide(C3_CAP, C3_DIM, "dual", "lfu")),
        "C2": OracleRun("C2", c2_scenario, lambda: OracleSide(C2_CAP, C2_DIM, "dual", "lru")),
        "C4": OracleRun("C4", c4_oracle, lambda: OracleSide(C4_CAP, C4_DIM, "dual", "lru")),
        "C5": OracleRun("C5", c5_oracle(c5), lambda: OracleSide(C5_CAP, C5_DIM, "dual", "lru")),
    }
    runs["C5"].trace = c5
    yield runs
    for r in runs.values():
        r.stop()


def release(*objs):
    del objs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_c2_as_benchmarked_vs_oracle(oracle_runs):
    dev = torch.device("cuda", 0)
    side = GpuSide(cskv.Table(C2_CAP, C2_DIM, "dual", "lru", device=dev), C2_SEED)
    n = lockstep("C2", oracle_runs["C2"], c2_scenario(side), C2_SEED, C2_DIM, dev, every=8)
    assert n > 70
    release(side)


def test_c4_program_graph_vs_oracle(oracle_runs):
    dev = torch.device("cuda", 0)
    side = GpuSide(cskv.Table(C4_CAP, C4_DIM, "dual", "lru", device=dev), C4_SEED)

    def gpu_records():
        vids = Vids()
        yield from c4_prefill(side, vids)
        ins = c4_inputs(side.prefill_keys, vids)
        t = side.t
        bufs = []
        prog = cskv.Program(t, overlap=False)
        for op, k, v in ins:
            kd = fs.from_u64(k, dev)
            flag = torch.full((k.size,), 9, dtype=torch.uint8, device=dev)
            if op == "find":
                out = torch.full((k.size, C4_DIM), fs.NAN_BITS, dtype=torch.int32, device=dev).view(torch.float32)
                sc = torch.zeros(k.size, dtype=torch.int64, device=dev)
                prog.add_find(kd, out, flag, sc)
                bufs.append((op, flag, out, sc))
            elif op == "upsert":
                prog.add_insert_or_assign(kd, side.rows(v), None, flag)
                bufs.append((op, flag, None, None))
            else:
                prog.add_erase(kd, flag)
                bufs.append((op, flag, None, None))
        prog.finalize()
        s = torch.cuda.Stream(device=dev)
        prog.capture(s)
        say(f"C4: program of {len(ins)} batches captured ({prog.segments} segments); replaying the graph")
        prog.replay(s)
        s.synchronize()
        clock = t.clock
        for j, (op, flag, out, sc) in enumerate(bufs):
            f = flag.cpu().numpy()
            if op == "find":
                hit = torch.from_numpy(np.nonzero(f)[0]).to(dev)
                miss = torch.from_numpy(np.nonzero(f == 0)[0]).to(dev)
                untouched = bool((fs.bits(out[miss]) == fs.NAN_BITS).all().item()) if miss.numel() else True
                yield f"batch {j} find", {"found": f, "scores": fs.as_u64(sc[hit]), "rows": out[hit],
                                          "untouched": untouched}
            elif op == "upsert":
                yield f"batch {j} upsert", {"status": f, "clock": None}
            else:
                yield f"batch {j} erase", {"erased": f}
        yield "final table", side.table()
        yield "final clock", {"final_clock": clock}

    n = lockstep("C4", oracle_runs["C4"], gpu_records(), C4_SEED, C4_DIM, dev, every=32)
    assert n > 256
    release(side)


def test_c3_online_eviction_full_size_vs_oracle(oracle_runs):
    dev = torch.device("cuda", 0)
    side = GpuSide(cskv.Table(C3_CAP, C3_DIM, "dual", "lfu", device=dev), C3_SEED)
    n = lockstep("C3", oracle_runs["C3"], c3_scenario(side), C3_SEED, C3_DIM, dev, every=8)
    assert n >= 2 * C3_STEPS + 2
    release(side)


def test_c5_serving_order_replayed_through_oracle(oracle_runs):
    dev = torch.device("cuda", 0)
    ops, sizes, keys, arrivals = oracle_runs["C5"].trace
    side = GpuSide(cskv.Table(C5_CAP, C5_DIM, "dual", "lru", device=dev), C5_SEED)
    run = oracle_runs["C5"]

    def gpu_records():
        vids = Vids()
        yield from c5_prefill(side, vids)
        ins = ops == serve.REQ_INSERT_AND_EVICT
        off = np.concatenate([[0], np.cumsum(sizes)])
        ins_vids = [vids.take(int(sizes[i])) if ins[i] else None for i in range(C5_NREQ)]
        kd = fs.from_u64(keys, dev)
        vals = side.rows(np.concatenate([v for v in ins_vids if v is not None]))
        tr = serve.Trace(side.t, ops, sizes, kd, vals, arrivals, with_results=True)
        tr.find_out.view(torch.int32).fill_(fs.NAN_BITS)
        say(f"C5: serving {C5_NREQ} requests ({int(sizes.sum())} keys)")
        stats, times = serve.serve(side.t, tr, budget_bytes=1 << 30, max_inflight_groups=4, max_merge=64,
                                   realtime=True, reader_streams=2)
        say(f"C5: served, {stats}")
        assert stats["completed"] == C5_NREQ
        # the oracle replays arrival order: the loop must have serialized requests in that order
        assert np.array_equal(times["seq"], np.arange(C5_NREQ))
        assert stats["groups"] < C5_NREQ, "no reader requests were merged"
        for i in range(C5_NREQ):
            n = int(sizes[i])
            if not ins[i]:
                o = int(tr.find_off[i])
                f = tr.find_flag[o:o + n].cpu().numpy()
                rows = tr.find_out[o:o + n]
                hit = torch.from_numpy(np.nonzero(f)[0]).to(dev)
                miss = torch.from_numpy(np.nonzero(f == 0)[0]).to(dev)
                untouched = bool((fs.bits(rows[miss]) == fs.NAN_BITS).all().item()) if miss.numel() else True
                # the serving loop returns no scores: take the oracle's (compared via the table)
                yield f"request {i}", {"found": f, "scores": None, "rows": rows[hit], "untouched": untouched}
            else:
                o = int(tr.val_off[i])
                m = int(tr.ev_count[i].item())
                ek = tr.ev_keys[o:o + m]
                srt = torch.argsort(ek)
                yield f"request {i}", {"status": tr.ins_status[o:o + n].cpu().numpy(), "clock": None,
                                       "ev": (fs.as_u64(ek[srt]), fs.as_u64(tr.ev_scores[o:o + m][srt]),
                                              tr.ev_vals[o:o + m][srt])}
        yield "final table", side.table()

    n = lockstep("C5", run, gpu_records(), C5_SEED, C5_DIM, dev, every=1000)
    assert n == C5_CAP // B20 + C5_NREQ + 1
    release(side)
