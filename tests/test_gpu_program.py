"""Batched programs (merged reader runs, serialization points, hipGraph capture/replay) give
exactly the results of the same calls issued one by one, and of the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2603_17168_amd import autotune, cskv
from paper_2603_17168_amd.workload import (as_u64, batch_schedule, keys as gen_keys, program_inputs,
                                            value_rows)
from tests.parity import bits

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def clone(src: cskv.Table) -> cskv.Table:
    dst = cskv.Table(src.capacity, src.dim, mode=src.mode, policy=src.policy, device=src.device)
    dst.storage.copy_(src.storage)
    torch.cuda.synchronize()
    return dst


def run_calls(t, ops):
    for d in ops:
        if d["op"] == "find":
            t.find(d["keys"], values_out=d["out"], found_out=d["flag"], want_scores=False)
        elif d["op"] == "upsert":
            t.insert_or_assign(d["keys"], d["values"], status_out=d["flag"])
        else:
            t.erase(d["keys"], erased_out=d["flag"])


def build_program(t, ops, tuning=None, overlap=True):
    p = cskv.Program(t, overlap=overlap)
    for d in ops:
        if tuning:
            autotune.apply(t, tuning, d["n"])
        if d["op"] == "find":
            p.add_find(d["keys"], d["out"], d["flag"])
        elif d["op"] == "upsert":
            p.add_insert_or_assign(d["keys"], d["values"], None, d["flag"])
        else:
            p.add_erase(d["keys"], d["flag"])
    return p.finalize()


def fresh_outputs(ops):
    res = []
    for d in ops:
        e = dict(d)
        if "out" in d:
            e["out"] = torch.full_like(d["out"], -7.0)
        e["flag"] = torch.full_like(d["flag"], 9)
        res.append(e)
    return res


def same_outputs(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x["flag"], y["flag"]), x["op"]
        if "out" in x:
            hit = x["flag"].bool()
            assert torch.equal(bits(x["out"][hit]), bits(y["out"][hit]))


def table_digest(t):
    k, v, s, sl = t.export()
    o = torch.argsort(k)
    return k[o], bits(v[o]), s[o], sl[o] // 128


def same_tables(a, b):
    for x, y in zip(table_digest(a), table_digest(b)):
        assert torch.equal(x, y)


def prefilled(capacity, dim, n_prefill, stream=1):
    t = cskv.Table(capacity, dim, mode="dual", policy="lru")
    batch = 1 << 14
    for s in range(0, n_prefill, batch):
        m = min(batch, n_prefill - s)
        k = gen_keys(stream, m, s, device="cuda")
        t.insert_or_assign(k, value_rows(3, k, dim), want_status=False)
    torch.cuda.synchronize()
    return t


def test_program_segments_merge_reader_runs():
    t = cskv.Table(128 * 64, 8, "dual", "lru")
    k = gen_keys(5, 100, device="cuda")
    v = [torch.zeros((100, 8), dtype=torch.float32, device="cuda") for _ in range(6)]
    f = [torch.empty(100, dtype=torch.uint8, device="cuda") for _ in range(6)]
    p = cskv.Program(t, overlap=True)
    p.add_find(k, v[0], f[0])
    p.add_find(k, v[1], f[1])
    p.add_insert_or_assign(k, v[5])
    p.add_find(k, v[2], f[2])
    p.add_erase(k)
    p.add_find(k, v[3], f[3])
    p.add_find(k, v[4], f[4])
    p.add_find(k[:0], v[0][:0], f[0][:0])  # empty batches vanish
    p.finalize()
    assert p.segments == 5
    # find run, upsert (prep, route, apply: no status), find run, erase (probe, clear), find run
    assert p.phases == 8
    with pytest.raises(cskv.CskvError):
        p.add_find(k, v[0], f[0])  # closed after finalize


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_program_aliasing_buffers_keep_call_order(overlap):
    """Ops that share buffers: two finds into the same outputs split the reader run (the second
    one's results remain); a find's output rows are the values of a later upsert (read after
    write); an erase whose flags reuse an upsert's status buffer (write after write).  Eager
    launch and graph replay both equal the calls issued one by one."""
    cap, dim = 1 << 14, 8
    base = prefilled(cap, dim, 9000)
    a = gen_keys(1, 3000, 0, device="cuda")      # resident
    b = gen_keys(1, 3000, 3000, device="cuda")   # resident, other rows
    fresh = gen_keys(60, 3000, device="cuda")
    out = torch.zeros((3000, dim), dtype=torch.float32, device="cuda")
    fl = torch.empty(3000, dtype=torch.uint8, device="cuda")
    st = torch.empty(3000, dtype=torch.uint8, device="cuda")

    def run(t, prog=None):
        out.fill_(-7.0)
        fl.fill_(9)
        st.fill_(9)
        torch.cuda.synchronize()
        if prog is None:
            t.find(a, values_out=out, found_out=fl, want_scores=False)
            t.find(b, values_out=out, found_out=fl, want_scores=False)
            t.insert_or_assign(fresh, out, status_out=st)
            t.erase(b, erased_out=st)
        else:
            prog()
        torch.cuda.synchronize()
        return out.clone(), fl.clone(), st.clone()

    ref_t = clone(base)
    ref = run(ref_t)
    assert bool((ref[1] == 1).all()) and bool((ref[2] <= 1).all())  # st ends as the erase's flags

    def make(t):
        p = cskv.Program(t, overlap=overlap)
        p.add_find(a, out, fl)
        p.add_find(b, out, fl)
        p.add_insert_or_assign(fresh, out, None, st)
        p.add_erase(b, st)
        return p.finalize()

    t1 = clone(base)
    p1 = make(t1)
    assert p1.segments == 4
    got = run(t1, p1.launch)
    for x, y in zip(ref, got):
        assert torch.equal(bits(x) if x.dtype == torch.float32 else x, bits(y) if y.dtype == torch.float32 else y)
    same_tables(ref_t, t1)
    t2 = clone(base)
    p2 = make(t2)
    s = torch.cuda.Stream()
    p2.capture(s)
    got = run(t2, lambda: (p2.replay(s), s.synchronize()))
    for x, y in zip(ref, got):
        assert torch.equal(bits(x) if x.dtype == torch.float32 else x, bits(y) if y.dtype == torch.float32 else y)
    same_tables(ref_t, t2)


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_program_matches_calls_and_oracle(overlap):
    """48 uneven batches (16..4096 keys, 70/25/5 find/upsert/erase) on a 2^15-slot table: the
    eager calls are checked against the oracle call by call; the program launched eagerly and
    the captured graph replayed must give the same outputs and the same table."""
    cap, dim = 1 << 15, 8
    base = prefilled(cap, dim, 24000)
    ora = oracle.Oracle(cap // 128, 128, oracle.DUAL, oracle.LRU)
    pk = as_u64(gen_keys(1, 24000))
    for s in range(0, 24000, 1 << 14):
        ora.upsert(pk[s:s + (1 << 14)], pk[s:s + (1 << 14)])  # value id = key: rows = value_rows(3, key)
    resident = gen_keys(1, 24000, device="cuda")
    sched = batch_schedule(7, 48, 16, 4096)
    ops = program_inputs(sched, dim, resident, fresh_stream=40, miss_stream=41, seed=3, device="cuda")
    t_prog, t_graph = clone(base), clone(base)
    # eager calls, oracle-checked (value ids of the oracle are the keys themselves: rows = f(key))
    run_calls(base, ops)
    torch.cuda.synchronize()
    for d in ops:
        kk = as_u64(d["keys"])
        if d["op"] == "find":
            f, vid, _ = ora.find(kk)
            assert np.array_equal(d["flag"].cpu().numpy(), f)
            hit = np.nonzero(f)[0]
            if hit.size:
                got = bits(d["out"].cpu()[torch.from_numpy(hit)])
                exp = bits(value_rows(3, torch.from_numpy(vid[hit].view(np.int64)), dim))
                # prefilled rows use seed 3 and value-id = key; upserted rows use the same rule
                assert torch.equal(got, exp)
        elif d["op"] == "upsert":
            st = ora.upsert(kk, kk)[0]
            assert np.array_equal(d["flag"].cpu().numpy(), st)
        else:
            assert np.array_equal(d["flag"].cpu().numpy(), ora.erase(kk))
    assert base.clock == ora.clock
    # the same schedule as one program, and as a captured graph
    ops_p = fresh_outputs(ops)
    prog = build_program(t_prog, ops_p, overlap=overlap)
    prog.launch()
    torch.cuda.synchronize()
    same_outputs(ops, ops_p)
    same_tables(base, t_prog)
    ops_g = fresh_outputs(ops)
    prog_g = build_program(t_graph, ops_g, overlap=overlap)
    s = torch.cuda.Stream()
    prog_g.capture(s)
    prog_g.replay(s)
    s.synchronize()
    same_outputs(ops, ops_g)
    same_tables(base, t_graph)
    assert t_graph.clock == ora.clock


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_graph_replays_are_repeatable(overlap):
    """Replay a captured program several times from the same starting table (restored eagerly
    between replays): every replay must reproduce the eager program's outputs and table."""
    cap, dim = 1 << 15, 8
    base = prefilled(cap, dim, 30000)
    resident = gen_keys(1, 30000, device="cuda")
    sched = batch_schedule(8, 32, 32, 2048)
    ops = program_inputs(sched, dim, resident, fresh_stream=42, miss_stream=43, seed=3, device="cuda")
    ref = clone(base)
    run_calls(ref, ops)
    snap = base.storage.clone()
    ops_g = fresh_outputs(ops)
    prog = build_program(base, ops_g, overlap=overlap)
    s = torch.cuda.Stream()
    prog.capture(s)
    for rep in range(3):
        say(f"replay {rep}")
        base.storage.copy_(snap)
        for d in ops_g:
            d["flag"].fill_(9)
        torch.cuda.synchronize()
        prog.replay(s)
        s.synchronize()
        same_outputs(ops, ops_g)
        same_tables(ref, base)


def test_autotuned_program_matches_untuned():
    """Per-size-class launch shapes chosen by the autotuner change no result."""
    cap, dim = 1 << 16, 16
    base = prefilled(cap, dim, 40000)
    resident = gen_keys(1, 40000, device="cuda")
    q = {"small": resident[:3000], "medium": resident[:20000]}
    fr = {"small": gen_keys(77, 3000, device="cuda"), "medium": gen_keys(78, 15000, device="cuda")}
    tuning = autotune.merge(autotune.tune_find(base, q), autotune.tune_route(base, fr))
    assert set(tuning) == {"small", "medium"}
    sched = batch_schedule(9, 40, 64, 30000)
    ops = program_inputs(sched, dim, resident, fresh_stream=44, miss_stream=45, seed=3, device="cuda")
    a, b = clone(base), clone(base)
    a.set_tuning(find_group=8, find_prefetch_b2=0, find_blocks_per_cu=0, route_group=8)
    run_calls(a, ops)
    ops_t = fresh_outputs(ops)
    p = build_program(b, ops_t, tuning)
    p.launch()
    torch.cuda.synchronize()
    same_outputs(ops, ops_t)
    same_tables(a, b)
