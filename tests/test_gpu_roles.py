"""GPU tests of the table role lock (Sec. 3.5, the reader / updater / inserter groups and their
compatibility table): calls issued from one host thread on different streams execute in issue
order when their roles conflict, and the concurrent-caller driver (several host threads, one
stream each) leaves the table the oracle computes for the same calls in sequence."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, from_u64, keys as gen_keys, value_rows
from tests.parity import Twin, bits

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["triple_group", "reader_writer"])
def test_conflicting_calls_follow_issue_order_across_streams(mode):
    say(f"issue order across streams, lock {mode}")
    dim = 16
    t = cskv.Table(1 << 22, dim, "dual", "custom")
    t.set_lock_mode(mode)
    assert t.lock_mode == mode
    n = 1 << 20
    k = gen_keys(90, n, 0, device="cuda")
    r1 = value_rows(1, torch.arange(n), dim).cuda()
    r2 = value_rows(2, torch.arange(n), dim).cuda()
    sc = torch.arange(n, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s1):  # inserter on s1, then a reader on s2: sees every key
            t.insert_or_assign(k, r1, sc)
        with torch.cuda.stream(s2):
            v, f, _ = t.find(k)
        with torch.cuda.stream(s1):  # updater on s1, then a reader on s2: sees the new rows
            t.assign(k, r2, sc + 1)
        with torch.cuda.stream(s2):
            v2, f2, sc2 = t.find(k)
        with torch.cuda.stream(s1):  # reader on s1, then an inserter on s2: the reader ran first
            v3, f3, _ = t.find(k)
        with torch.cuda.stream(s2):
            er = t.erase(k)
        with torch.cuda.stream(s1):  # reader after the erase on s1: nothing left
            f4 = t.contains(k)
        torch.cuda.synchronize()
        assert bool((f == 1).all()) and torch.equal(bits(v), bits(r1)), "reader overtook the inserter"
        assert bool((f2 == 1).all()) and torch.equal(bits(v2), bits(r2)), "reader overtook the updater"
        assert torch.equal(sc2, sc + 1)
        assert bool((f3 == 1).all()) and torch.equal(bits(v3), bits(r2)), "inserter overtook the reader"
        assert bool((er == 1).all()) and bool((f4 == 0).all()), "reader overtook the erase"
        assert t.size() == 0


def test_lock_mode_arguments():
    t = cskv.Table(128 * 8, 8, "dual", "lru")
    assert t.lock_mode == "none"
    for m in ("triple_group", "reader_writer", "none"):
        t.set_lock_mode(m)
        assert t.lock_mode == m
    with pytest.raises(cskv.CskvError):
        cskv._check(cskv.lib().cskv_set_lock_mode(t._h, 3), "cskv_set_lock_mode")


@pytest.mark.parametrize("mode", ["triple_group", "reader_writer", "none"])
def test_concurrent_callers_match_sequential_oracle(mode):
    """Readers find keys A, updaters assign disjoint key sets B_t, inserters insert then erase
    fresh key sets C_i, all at once from their own threads and streams (CUSTOM scores, low load,
    no eviction): the final table is the oracle's after the same calls in sequence, and every
    reader saw A unchanged.  Without a lock (one inserter then) the roles touch disjoint keys and
    slots, so the result holds there too; the lock modes must not change it."""
    say(f"concurrent callers, lock {mode}")
    dim = 8
    tw = Twin(1 << 16, dim, "dual", "custom", seed=5)
    tw.gpu.set_lock_mode(mode)
    rng = np.random.default_rng(5)
    A = as_u64(gen_keys(91, 4096))
    B = [as_u64(gen_keys(92, 1024, 1024 * i)) for i in range(3)]
    # two inserters only under a lock: without one, concurrent inserters could claim one slot
    C = [as_u64(gen_keys(93, 1024, 1024 * i)) for i in range(1 if mode == "none" else 2)]
    tw.upsert(A, rng.integers(0, 100, A.size).astype(np.uint64))
    for b in B:
        tw.upsert(b, rng.integers(0, 100, b.size).astype(np.uint64))
    tw.check_table()
    exp_a = tw.gpu.find(from_u64(A, "cuda"))[0].clone()
    specs = []
    readers = []
    for i in range(3):
        out = torch.empty((A.size, dim), dtype=torch.float32, device="cuda")
        fl = torch.empty(A.size, dtype=torch.uint8, device="cuda")
        readers.append((out, fl))
        specs.append({"op": "find", "calls": 10, "keys": from_u64(A, "cuda"), "values_out": out, "flags": fl})
    upd = []
    for b in B:
        vids = tw._vids(b.size)
        s = rng.integers(0, 1000, b.size).astype(np.uint64)
        upd.append((b, vids, s))
        specs.append({"op": "assign", "calls": 5, "keys": from_u64(b, "cuda"), "values": tw.rows(vids).cuda(),
                      "scores": from_u64(s, "cuda"), "flags": torch.empty(b.size, dtype=torch.uint8, device="cuda")})
    ins = []
    for c in C:
        vids = tw._vids(c.size)
        s = rng.integers(0, 1000, c.size).astype(np.uint64)
        ins.append((c, vids, s))
        specs.append({"op": "insert_erase", "calls": 6, "keys": from_u64(c, "cuda"), "values": tw.rows(vids).cuda(),
                      "scores": from_u64(s, "cuda"), "flags": torch.empty(c.size, dtype=torch.uint8, device="cuda")})
    ms = cskv.run_threads(tw.gpu, specs)
    assert ms > 0
    for b, vids, s in upd:
        for _ in range(5):
            tw.ora.assign(b, vids, s)
    for c, vids, s in ins:
        for _ in range(3):
            tw.ora.upsert(c, vids, s)
            tw.ora.erase(c)
    torch.cuda.synchronize()
    for out, fl in readers:
        assert bool((fl == 1).all()) and torch.equal(bits(out), bits(exp_a)), "a reader saw A change"
    tw.check_table()


@pytest.mark.parametrize("overlap", [0, 1])
def test_program_holds_the_table_as_one_call(overlap):
    """A program with writes is one inserter call under the lock: a find issued on another stream
    after the launch (or after a graph replay) sees every key the program inserted."""
    say(f"program under the lock, overlap {overlap}")
    dim = 8
    t = cskv.Table(1 << 20, dim, "dual", "custom")
    t.set_lock_mode("triple_group")
    n = 1 << 16
    keys = [gen_keys(95, n, i * n, device="cuda") for i in range(4)]
    rows = [value_rows(5 + i, torch.arange(n), dim).cuda() for i in range(4)]
    sc = torch.ones(n, dtype=torch.int64, device="cuda")
    st = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(4)]
    pr = cskv.Program(t, overlap=overlap)
    for i in range(4):
        pr.add_insert_or_assign(keys[i], rows[i], sc, st[i])
    pr.finalize()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    pr.launch(s1)
    with torch.cuda.stream(s2):
        v, f, _ = t.find(keys[3])
    torch.cuda.synchronize()
    assert bool((f == 1).all()) and torch.equal(bits(v), bits(rows[3])), "a reader overtook the program"
    with torch.cuda.stream(s2):
        t.erase(torch.cat(keys))
    pr.capture(s1)
    pr.replay(s1)
    with torch.cuda.stream(s2):
        f2 = t.contains(keys[2])
    torch.cuda.synchronize()
    assert bool((f2 == 1).all()), "a reader overtook the replay"
