"""Lock-step GPU-vs-oracle comparison for workloads too large to check call by call in one thread.

A *scenario* is a generator function ``scenario(side)`` that issues one deterministic call
sequence through ``side`` and yields ``(label, record)`` after every call it wants compared.  It is
run twice: on :class:`OracleSide` (the sequential C oracle) in a background thread, which starts
when the test module is set up and runs ahead while other tests use the GPU, and on
:class:`GpuSide` (the HIP table through the C-ABI binding) in the test itself.  :func:`lockstep`
pairs the two record streams and compares them element by element:

* statuses, found masks and erased flags - exactly;
* evicted sets - keys, scores and rows, each side sorted by key;
* rows - the GPU's rows against rows generated from the oracle's value-ids (never from keys,
  so that a row written by the wrong occurrence of a repeated key shows up);
* tables - the whole table, sorted by key: keys, scores, bucket of each entry, rows.

Inputs that depend on the table (queries drawn from the resident set) are drawn by each side from
its own sorted resident keys, so they coincide exactly when the tables do (and the tables are
compared before such a draw).  The oracle thread calls into C through ctypes, which releases the
GIL, so several oracle scenarios and the GPU side run concurrently.
"""
from __future__ import annotations

import queue
import sys
import threading
import time

import numpy as np
import torch

import oracle
from paper_2603_17168_amd.workload import as_u64, from_u64, value_rows

MODE = {"single": oracle.SINGLE, "dual": oracle.DUAL}
POLICY = {"custom": oracle.CUSTOM, "lru": oracle.LRU, "lfu": oracle.LFU}
NAN_BITS = 0x7FC0DEAD
ROW_CHUNK = 1 << 22


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(t: torch.Tensor) -> torch.Tensor:
    return t.contiguous().view(torch.int32)


class OracleSide:
    """The sequential C oracle behind the scenario interface (numpy in, numpy records out)."""

    kind = "oracle"

    def __init__(self, capacity: int, dim: int, mode: str, policy: str, ora=None):
        self.capacity, self.dim, self.mode, self.policy = capacity, dim, mode, policy
        self.o = ora if ora is not None else oracle.Oracle(capacity // 128, 128, MODE[mode], POLICY[policy])

    def clone(self) -> "OracleSide":
        return OracleSide(self.capacity, self.dim, self.mode, self.policy, self.o.clone())

    def size(self) -> int:
        return self.o.size()

    def clock(self) -> int:
        return self.o.clock

    def upsert(self, keys, vids, scores=None, evict=False, want=True):
        st, ek, ev, es = self.o.upsert(keys, vids, scores)
        if not want:
            return None
        rec = {"status": st, "clock": self.o.clock}
        if evict:
            o = np.argsort(ek.view(np.int64), kind="stable")
            rec["ev"] = (ek[o], es[o], ev[o])
        return rec

    def find(self, keys):
        f, v, s = self.o.find(keys)
        hit = np.nonzero(f)[0]
        return {"found": f, "scores": s[hit], "rows": v[hit]}

    def erase(self, keys):
        return {"erased": self.o.erase(keys)}

    def residents(self) -> np.ndarray:
        """Resident keys in ascending order of their int64 bit patterns (the GPU side's order)."""
        k, _, _, _ = self.o.export()
        return np.sort(k.view(np.int64)).view(np.uint64)

    def table(self):
        k, v, s, b = self.o.export()
        o = np.argsort(k.view(np.int64), kind="stable")
        return {"table": (k[o], s[o], b[o], v[o])}


class GpuSide:
    """The HIP table (through the binding) behind the scenario interface; rows are generated on
    the device from value-ids with the shared row generator."""

    kind = "gpu"

    def __init__(self, table, seed: int):
        self.t = table
        self.dim = table.dim
        self.seed = seed
        self.dev = table.device

    def clone(self) -> "GpuSide":
        from paper_2603_17168_amd import cskv
        src = self.t
        dst = cskv.Table(src.capacity, src.dim, mode=src.mode, policy=src.policy, device=src.device)
        dst.storage.copy_(src.storage)
        dst.set_tuning(**{k: v for k, v in src.get_tuning().items() if k != "find_digest"})
        dst.clock = src.clock
        return GpuSide(dst, self.seed)

    def rows(self, vids) -> torch.Tensor:
        v = from_u64(np.asarray(vids, dtype=np.uint64), self.dev)
        return value_rows(self.seed, v, self.dim)

    def size(self) -> int:
        return self.t.size()

    def clock(self) -> int:
        return self.t.clock

    def upsert(self, keys, vids, scores=None, evict=False, want=True):
        kd = from_u64(keys, self.dev)
        vd = self.rows(vids)
        sd = None if scores is None else from_u64(scores, self.dev)
        if evict:
            st, ek, ev, es, cnt = self.t.insert_and_evict(kd, vd, sd)
        else:
            st = self.t.insert_or_assign(kd, vd, sd, want_status=want)
        if not want:
            return None
        rec = {"status": st.cpu().numpy(), "clock": self.t.clock}
        if evict:
            m = int(cnt.item())
            o = torch.argsort(ek[:m])
            rec["ev"] = (as_u64(ek[:m][o]), as_u64(es[:m][o]), ev[:m][o])
        return rec

    def find(self, keys):
        kd = from_u64(keys, self.dev)
        n = kd.numel()
        out = torch.full((n, self.dim), NAN_BITS, dtype=torch.int32, device=self.dev).view(torch.float32)
        vals, found, sc = self.t.find(kd, values_out=out)
        f = found.cpu().numpy()
        hit = torch.from_numpy(np.nonzero(f)[0]).to(self.dev)
        miss = torch.from_numpy(np.nonzero(f == 0)[0]).to(self.dev)
        untouched = bool((bits(vals[miss]) == NAN_BITS).all().item()) if miss.numel() else True
        return {"found": f, "scores": as_u64(sc[hit]), "rows": vals[hit], "untouched": untouched}

    def erase(self, keys):
        return {"erased": self.t.erase(from_u64(keys, self.dev)).cpu().numpy()}

    def residents(self) -> np.ndarray:
        k, _, _, _ = self.t.export(with_values=False)
        return as_u64(torch.sort(k)[0])

    def table(self):
        k, v, s, sl = self.t.export(with_values=True)
        o = torch.argsort(k)
        return {"table": (k[o], s[o], sl[o], v[o])}


def _rows_equal(got: torch.Tensor, vids: np.ndarray, seed: int, dim: int, dev) -> bool:
    for c in range(0, vids.size, ROW_CHUNK):
        v = from_u64(vids[c:c + ROW_CHUNK], dev)
        if not torch.equal(bits(got[c:c + ROW_CHUNK]), bits(value_rows(seed, v, dim))):
            return False
    return True


def compare(label: str, g: dict, o: dict, seed: int, dim: int, dev):
    """Element-by-element comparison of one GPU record with the oracle's record of the same call."""
    if "status" in o:
        gs, os_ = g["status"], o["status"]
        if not np.array_equal(gs, os_):
            bad = np.nonzero(gs != os_)[0]
            raise AssertionError(f"{label}: status differs at {bad[:8]} (gpu {gs[bad[:8]]}, oracle {os_[bad[:8]]}), "
                                 f"{bad.size} of {gs.size}")
        if g["clock"] is not None:  # None: calls inside one graph replay (only the final clock is observable)
            assert g["clock"] == o["clock"], f"{label}: clock gpu {g['clock']} oracle {o['clock']}"
    if "ev" in o:
        gk, gsc, grows = g["ev"]
        ok, osc, ovid = o["ev"]
        assert gk.size == ok.size, f"{label}: evicted count gpu {gk.size} oracle {ok.size}"
        assert np.array_equal(gk, ok), f"{label}: evicted keys differ"
        assert np.array_equal(gsc, osc), f"{label}: evicted scores differ"
        assert _rows_equal(grows, ovid, seed, dim, dev), f"{label}: evicted rows differ"
    if "found" in o:
        if not np.array_equal(g["found"], o["found"]):
            bad = np.nonzero(g["found"] != o["found"])[0]
            raise AssertionError(f"{label}: found mask differs at {bad[:8]} (gpu {g['found'][bad[:8]]}, "
                                 f"oracle {o['found'][bad[:8]]}), {bad.size} of {g['found'].size}")
        if g["scores"] is not None:  # None: the call returned no scores
            assert np.array_equal(g["scores"], o["scores"]), f"{label}: found scores differ"
        assert _rows_equal(g["rows"], o["rows"], seed, dim, dev), f"{label}: found rows differ"
        assert g["untouched"], f"{label}: rows of missing keys were written"
    if "final_clock" in o:
        assert g["final_clock"] == o["final_clock"], f"{label}: gpu {g['final_clock']} oracle {o['final_clock']}"
    if "erased" in o:
        assert np.array_equal(g["erased"], o["erased"]), f"{label}: erased flags differ"
    if "table" in o:
        gk, gs, gsl, gv = g["table"]
        ok, os_, ob, ov = o["table"]
        assert gk.numel() == ok.size, f"{label}: table size gpu {gk.numel()} oracle {ok.size}"
        assert torch.equal(gk, from_u64(ok, dev)), f"{label}: table keys differ"
        assert torch.equal(gs, from_u64(os_, dev)), f"{label}: table scores differ"
        assert torch.equal(gsl // 128, from_u64(ob, dev)), f"{label}: an entry sits in another bucket"
        assert torch.unique(gsl).numel() == gsl.numel(), f"{label}: two entries share a slot"
        assert _rows_equal(gv, ov, seed, dim, dev), f"{label}: table rows differ"


class OracleRun:
    """A scenario running on the oracle in a daemon thread; its records queue up in order."""

    def __init__(self, name: str, scenario, side_factory):
        self.name = name
        self.q: queue.Queue = queue.Queue()
        self.t0 = time.time()
        self.halt = threading.Event()
        self.th = threading.Thread(target=self._run, args=(scenario, side_factory), daemon=True, name=name)
        self.th.start()

    def _run(self, scenario, side_factory):
        try:
            for lab, rec in scenario(side_factory()):
                if self.halt.is_set():
                    return
                self.q.put((lab, rec))
            self.q.put(("__end__", None))
        except BaseException as e:  # surfaced in the test thread
            self.q.put(("__error__", e))

    def stop(self, timeout: float = 300.0):
        """Ends the scenario after its current oracle call (a run whose records no test consumed
        must not outlive the test session: native code still running at interpreter exit aborts it)."""
        self.halt.set()
        while True:  # drain, so that a producer blocked on nothing keeps going to its next check
            try:
                self.q.get_nowait()
            except queue.Empty:
                break
        self.th.join(timeout)

    def records(self):
        while True:
            lab, rec = self.q.get()
            if lab == "__error__":
                raise AssertionError(f"oracle scenario {self.name} failed: {rec!r}") from rec
            if lab == "__end__":
                return
            yield lab, rec


def lockstep(name: str, run: OracleRun, gpu_records, seed: int, dim: int, dev, every: int = 1) -> int:
    """Compare the GPU scenario's records with the oracle run's, one pair at a time."""
    n = 0
    ora = run.records()
    for lab, g in gpu_records:
        try:
            olab, o = next(ora)
        except StopIteration:
            raise AssertionError(f"{name}: the oracle scenario ended before {lab}")
        assert lab == olab, f"{name}: record {n} is {lab} on the GPU and {olab} in the oracle"
        compare(f"{name}/{lab}", g, o, seed, dim, dev)
        n += 1
        if n % every == 0:
            say(f"{name}: {lab} equal ({time.time() - run.t0:.0f} s since the oracle started)")
    for lab, _ in ora:
        raise AssertionError(f"{name}: the GPU scenario ended before the oracle's {lab}")
    return n
