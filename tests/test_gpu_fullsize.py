"""The bench's C2 shape at full size (2^26 slots, dim 32, dual, LRU, 2^20-key calls), in every
launch shape the autotuner may pick, checked by properties that hold at any size: every row is
bit-exact with the row generator, every score is the LRU clock of the key's insert call, every
entry sits in one of its key's two candidate buckets (hash written out here from the MurmurHash3
finalizer), statuses and sizes follow from the batch contents, and evicted keys leave."""
import sys

import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import keys as gen_keys, value_rows
from tests.hashkeys import C1, C2

pytestmark = pytest.mark.gpu

CAP, DIM, B = 1 << 26, 32, 1 << 20
NB = CAP // 128


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _s64(x):
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= 1 << 63 else x


def _lsr(x, k):
    return (x >> k) & ((1 << (64 - k)) - 1)


def candidates(keys):
    """(b1, b2) of int64 keys: h = fmix64(k), b1 = h mod B, b2 = (h >> 40) mod B."""
    h = keys ^ _lsr(keys, 33)
    h = h * _s64(C1)
    h = h ^ _lsr(h, 33)
    h = h * _s64(C2)
    h = h ^ _lsr(h, 33)
    return h & (NB - 1), _lsr(h, 40) & (NB - 1)


def bits(t):
    return t.contiguous().view(torch.int32)


SHAPES = [(g, pre, pairs) for g in (4, 8, 16) for pre in (0, 1) for pairs in (0, 1)]


def test_c2_full_size_properties():
    dev = torch.device("cuda", 0)
    t = cskv.Table(CAP, DIM, "dual", "lru", device=dev)
    say("C2 full size: fill to load 0.5")
    for c in range(32):
        k = gen_keys(1, B, c * B, device=dev)
        st = t.insert_or_assign(k, value_rows(11, k, DIM))
        assert bool((st == cskv.ST_INSERTED).all()), f"call {c}: a fresh key below first eviction not inserted"
    assert t.size() == 32 * B and t.clock == 32
    resident = gen_keys(1, 32 * B, 0, device=dev)

    say("placement of every entry")
    ek, _, es, sl = t.export(with_values=False)
    assert ek.numel() == 32 * B
    assert torch.equal(torch.sort(ek)[0], torch.sort(resident)[0]), "the table does not hold exactly the inserted keys"
    b1, b2 = candidates(ek)
    bk = sl // 128
    assert bool(((bk == b1) | (bk == b2)).all()), "an entry outside its key's candidate buckets"
    assert torch.unique(sl).numel() == sl.numel()
    del ek, es, sl, b1, b2, bk

    g = torch.Generator(device=dev)
    g.manual_seed(7)
    idx = torch.randint(0, 32 * B, (B,), device=dev, generator=g)
    q100 = resident[idx]
    fresh = gen_keys(2, B // 2, 0, device=dev)
    q50 = torch.cat([q100[: B // 2], fresh])
    want100 = bits(value_rows(11, q100, DIM))
    for shape in SHAPES:
        say(f"finds in shape group {shape[0]} prefetch {shape[1]} pairs {shape[2]}")
        t.set_tuning(find_group=shape[0], find_prefetch_b2=shape[1], find_pairs=shape[2])
        v, f, s = t.find(q100)
        assert bool((f == 1).all())
        assert torch.equal(bits(v), want100), "a found row differs from its generator"
        assert torch.equal(s, idx // B + 1), "a score differs from its insert call's clock"
        v, f, _ = t.find(q50)
        assert bool((f[: B // 2] == 1).all()) and bool((f[B // 2:] == 0).all())
        assert torch.equal(bits(v[: B // 2]), want100[: B // 2])
        c = t.contains(q50)
        assert torch.equal(c, f)

    say("insert and erase of fresh keys at load 0.5")
    nk = gen_keys(3, B, 0, device=dev)
    st = t.insert_or_assign(nk, value_rows(12, nk, DIM))
    assert bool((st == cskv.ST_INSERTED).all()) and t.size() == 33 * B
    er = t.erase(nk)
    assert bool((er == 1).all()) and t.size() == 32 * B
    assert not bool(t.contains(nk).any())

    say("fill to load 1.0")
    c = 32
    while t.size() < CAP and c < 128:
        k = gen_keys(1, B, c * B, device=dev)
        st = t.insert_or_assign(k, value_rows(11, k, DIM))
        assert bool(((st == cskv.ST_INSERTED) | (st == cskv.ST_INSERTED_EVICT)).all())
        c += 1
    assert t.size() == CAP
    say("insert_and_evict of fresh keys into the full table")
    clock = t.clock  # one tick per non-empty upsert call (the erase did not tick)
    assert clock == c + 1
    nk = gen_keys(4, B, 0, device=dev)
    st, ek, ev, es, cnt = t.insert_and_evict(nk, value_rows(13, nk, DIM))
    m = int(cnt.item())
    # every fresh key carries this call's clock, above every resident score: all admitted
    assert bool((st == cskv.ST_INSERTED_EVICT).all()) and m == B and t.size() == CAP
    assert bool((es[:m] <= clock).all()), "an evicted score is not older than this call"
    assert not bool(t.contains(ek[:m]).any()), "an evicted key is still resident"
    v, f, s = t.find(nk)
    assert bool((f == 1).all()) and torch.equal(bits(v), bits(value_rows(13, nk, DIM)))
    assert bool((s == clock + 1).all())
    # evicted rows are the rows their keys were inserted with
    assert torch.equal(bits(ev[:m]), bits(value_rows(11, ek[:m], DIM)))


def test_c4_full_size_program_properties():
    """C4 at full size (2^26 slots, dim 32, LRU prefilled to 0.9; 256 batches of 1K-1M keys,
    70/25/5 find / insert_or_assign / erase, shapes autotuned per size class) as one program:
    never-inserted keys are never found, every found row is its key's generator row (prefill and
    upserts share it), fresh keys are admitted, the size follows the statuses, and the program's
    outputs equal plain calls'."""
    from paper_2603_17168_amd import autotune as tuner
    from paper_2603_17168_amd.workload import batch_schedule, program_inputs
    dev = torch.device("cuda", 0)
    say("C4 full size: prefill to 0.9")
    t = cskv.Table(CAP, DIM, "dual", "lru", device=dev)
    c = 0
    while t.size() < 0.9 * CAP:
        k = gen_keys(2, B, c * B, device=dev)
        t.insert_or_assign(k, value_rows(11, k, DIM), want_status=False)
        c += 1
    size0 = t.size()
    resident = gen_keys(2, size0, 0, device=dev)
    sched = batch_schedule(21, 256, 1 << 10, 1 << 20)
    ops = program_inputs(sched, DIM, resident, fresh_stream=22, miss_stream=23, seed=11, device=dev)
    q = {s: resident[: tuner.CLASS_SIZE[s]] for s in ("small", "medium", "large")}
    fr = {s: gen_keys(24, tuner.CLASS_SIZE[s], 0, device=dev) for s in ("small", "medium", "large")}
    tuning = tuner.merge(tuner.tune_find(t, q), tuner.tune_route(t, fr))
    # the route tuner's 2^20-key trials may evict a resident now and then (snapshot routing
    # overfills a bucket at this load); conservation counts from the table it leaves
    size0 = t.size()
    snap = t.storage.clone()
    say("plain calls")
    for d in ops:
        tuner.apply(t, tuning, d["n"])
        if d["op"] == "find":
            t.find(d["keys"], values_out=d["out"], found_out=d["flag"], want_scores=False)
        elif d["op"] == "upsert":
            t.insert_or_assign(d["keys"], d["values"], status_out=d["flag"])
        else:
            t.erase(d["keys"], erased_out=d["flag"])
    torch.cuda.synchronize()
    size_plain = t.size()
    ref = [(d["flag"].clone(), d["out"].clone() if "out" in d else None) for d in ops]
    say("the same schedule as one program")
    t.storage.copy_(snap)
    pr = cskv.Program(t, overlap=0)
    for d in ops:
        tuner.apply(t, tuning, d["n"])
        if d["op"] == "find":
            d["out"].zero_()
            pr.add_find(d["keys"], d["out"], d["flag"])
        elif d["op"] == "upsert":
            pr.add_insert_or_assign(d["keys"], d["values"], None, d["flag"])
        else:
            pr.add_erase(d["keys"], d["flag"])
    pr.finalize()
    pr.launch()
    torch.cuda.synchronize()
    assert t.size() == size_plain
    gained = 0
    for d, (flag, out) in zip(ops, ref):
        assert torch.equal(d["flag"], flag), d["op"]
        if d["op"] == "find":
            assert torch.equal(bits(d["out"]), bits(out))
            hit = d["flag"].bool()
            miss_stream_keys = ~torch.isin(d["keys"], resident)
            assert not bool((hit & miss_stream_keys).any()), "a never-inserted key was found"
            assert torch.equal(bits(d["out"][hit]), bits(value_rows(11, d["keys"][hit], DIM))), "a found row differs"
        elif d["op"] == "upsert":
            st = d["flag"]
            assert bool(((st == cskv.ST_INSERTED) | (st == cskv.ST_INSERTED_EVICT)).all()), "a fresh key not admitted"
            gained += int((st == cskv.ST_INSERTED).sum())
        else:
            gained -= torch.unique(d["keys"][d["flag"].bool()]).numel()
    assert t.size() == size0 + gained, "the size does not follow the statuses"
