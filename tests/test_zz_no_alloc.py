"""The allocation-free insert_or_assign (a fixed device array of the library as its workspace)
against cskv_insert_or_assign with a caller workspace: two tables with the same starting
contents take the same calls, one through each entry point, twice in a row with the second
call smaller; statuses and whole-table contents must be equal, and a batch above the limit is
refused before anything runs."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, from_u64, keys as gen_keys, permutation, uniform_u64, value_rows

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def clone(src):
    dst = cskv.Table(src.capacity, src.dim, mode=src.mode, policy=src.policy)
    dst.storage.copy_(src.storage)
    torch.cuda.synchronize()
    return dst


def contents(t):
    """(keys, buckets, scores, value bits) of every entry, sorted by key."""
    k, v, s, sl = t.export()
    o = torch.argsort(k)
    return k[o], (sl[o] // t.bucket_size), s[o], v[o].view(torch.int32)


def assert_same_table(a, b):
    ka, ba, sa, va = contents(a)
    kb, bb, sb, vb = contents(b)
    assert torch.equal(ka, kb)
    assert torch.equal(ba, bb)
    assert torch.equal(sa, sb)
    assert torch.equal(va, vb)
    assert a.clock == b.clock


def batch(seed, n, pool, policy, dev):
    """n occurrences: residents of pool and fresh keys, some repeated, shuffled."""
    fresh = as_u64(gen_keys(seed, n))
    distinct = np.concatenate([pool[: n // 3], fresh[: n - n // 3]]) if pool is not None else fresh
    reps = (as_u64(uniform_u64(seed + 1, distinct.size)) % np.uint64(3)).astype(np.int64) + 1
    k = np.repeat(distinct, reps)[:n]
    k = k[permutation(seed + 2, k.size).numpy()]
    scores = None
    if policy == "custom":
        scores = from_u64((as_u64(uniform_u64(seed + 3, k.size)) >> np.uint64(40)) + np.uint64(1), dev)
    elif policy == "lfu":
        scores = from_u64((as_u64(uniform_u64(seed + 4, k.size)) % np.uint64(4)) + np.uint64(1), dev)
    kd = from_u64(k, dev)
    return kd, value_rows(seed + 5, kd, 8), scores


@pytest.mark.parametrize("policy", ["custom", "lru", "lfu"])
@pytest.mark.parametrize("cap", [1 << 14, 1 << 22])  # full table (evictions, refusals) / roomy table
def test_noalloc_equals_workspace_entry_point(policy, cap):
    dev = torch.device("cuda:0")
    ref = cskv.Table(cap, 8, mode="dual", policy=policy)
    k0, v0, s0 = batch(300, 20000, None, policy, dev)
    ref.insert_or_assign(k0, v0, s0, want_status=False)
    torch.cuda.synchronize()
    got = clone(ref)
    pool = as_u64(k0.cpu())
    for call, n in enumerate([cskv.NOALLOC_MAX_KEYS, 5000]):  # the second call smaller
        k, v, s = batch(310 + 10 * call, n, pool, policy, dev)
        say(f"noalloc {policy} cap {cap} call {call}: n {k.numel()}")
        st_ref = ref.insert_or_assign(k, v, s)
        st = torch.full((k.numel(),), 0xEE, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(dev)
        got.insert_or_assign_noalloc(k, v, s, status_out=st)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
        assert torch.equal(st, st_ref)
        assert_same_table(got, ref)
        hist = np.bincount(st.cpu().numpy(), minlength=6)[1:5]
        say(f"  statuses (updated, inserted, evicting, refused) {hist.tolist()}, size {got.size()}")
        if cap == 1 << 14:
            assert hist[2] + hist[3] > 0  # the full table evicts or refuses
        pool = as_u64(k.cpu())


@pytest.mark.parametrize("policy", ["lru", "lfu"])
def test_noalloc_with_route_subrounds(policy):
    """Route sub-rounds (the call's keys applied in 4 chunks) take the global-dedupe path with its
    rank arrays, which the fixed array must also hold: same results as the workspace entry point
    on two calls, the second smaller."""
    dev = torch.device("cuda:0")
    ref = cskv.Table(1 << 15, 8, mode="dual", policy=policy)
    ref.set_route_subrounds(4)
    k0, v0, s0 = batch(500, 20000, None, policy, dev)
    ref.insert_or_assign(k0, v0, s0, want_status=False)
    torch.cuda.synchronize()
    got = clone(ref)
    got.set_route_subrounds(4)
    pool = as_u64(k0.cpu())
    for call, n in enumerate([cskv.NOALLOC_MAX_KEYS, 3000]):
        k, v, s = batch(510 + 10 * call, n, pool, policy, dev)
        say(f"noalloc sub-rounds {policy} call {call}: n {k.numel()}")
        st_ref = ref.insert_or_assign(k, v, s)
        st = torch.full((k.numel(),), 0xEE, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        got.insert_or_assign_noalloc(k, v, s, status_out=st)
        torch.cuda.synchronize()
        assert torch.equal(st, st_ref)
        assert_same_table(got, ref)
        pool = as_u64(k.cpu())


def test_noalloc_refuses_batches_above_the_limit():
    dev = torch.device("cuda:0")
    t = cskv.Table(1 << 14, 8, mode="dual", policy="lru")
    k, v, _ = batch(400, 1000, None, "lru", dev)
    t.insert_or_assign_noalloc(k, v)
    torch.cuda.synchronize()
    size, clock = t.size(), t.clock
    big = from_u64(as_u64(gen_keys(401, cskv.NOALLOC_MAX_KEYS + 1)), dev)
    with pytest.raises(cskv.CskvError):
        t.insert_or_assign_noalloc(big, value_rows(402, big, 8))
    torch.cuda.synchronize()
    assert t.size() == size and t.clock == clock  # nothing ran
    assert cskv.lib().cskv_noalloc_scratch_bytes() == 12 << 20
