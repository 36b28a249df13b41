"""Oracle parity on shapes that only full-size runs would otherwise reach: launch grids that are
capped (slow per-bucket apply, export), so that only tables or batches larger than the cap make
a block take a second tile; keys repeated across many input blocks on a large table; and a
bucket crowded with more distinct keys than the slow apply's LDS merge table holds.  Each case is
checked against the oracle call by call and by whole-table exports (rows through value-ids)."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd.workload import as_u64, keys as gen_keys, permutation, uniform_u64
from tests.hashkeys import keys_for
from tests.parity import Twin

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("policy", ["custom", "lfu", "lru"])
def test_repeated_keys_on_2e17_buckets(policy):
    """2^24 slots (2^17 buckets): calls whose keys repeat (each distinct key 1-4 times, shuffled,
    residents and fresh keys mixed), so that most repeated keys reach their bucket from several
    input blocks and the apply merges their entries all over a large table."""
    cap = 1 << 24
    tw = Twin(cap, 4, "dual", policy, seed=51)
    base = as_u64(gen_keys(70, 1 << 18))
    say(f"repeated keys, 2^17 buckets, {policy}: fill")
    sc = (np.arange(base.size, dtype=np.uint64) % 1000) + 1
    tw.upsert(base, sc if policy != "lru" else None)
    for call in range(3):
        fresh = as_u64(gen_keys(71 + call, 1 << 17))
        distinct = np.concatenate([base[call::3][: 1 << 16], fresh])  # residents (updates) and fresh keys
        reps = (as_u64(uniform_u64(80 + call, distinct.size)) % np.uint64(4)).astype(np.int64) + 1
        k = np.repeat(distinct, reps)
        k = k[permutation(90 + call, k.size).numpy()]
        scores = None
        if policy == "custom":
            scores = as_u64(uniform_u64(95 + call, k.size)) >> np.uint64(40)
        elif policy == "lfu":
            scores = (as_u64(uniform_u64(97 + call, k.size)) % np.uint64(5)) + np.uint64(1)
        st = tw.upsert(k, scores, evict=(call == 1))
        assert (st == 1).sum() > 0 and (st == 2).sum() > 0
        tw.check_table()
        say(f"  call {call}: {k.size} occurrences of {distinct.size} keys, table equal")


def test_crowded_buckets_beyond_one_slow_grid():
    """8192 buckets each receiving about 24 operations in one call (more than the fast path's 16),
    twice: more crowded buckets than one pass of the slow apply's grid, with inserts into free
    slots, then evictions and rejections."""
    nb = 8192
    tw = Twin(nb * 128, 8, "dual", "custom", seed=52)
    for call in range(4):
        n = nb * 24
        k = as_u64(gen_keys(100 + call, n))
        s = (as_u64(uniform_u64(110 + call, n)) >> np.uint64(44)) + np.uint64(1)
        st = tw.upsert(k, s, evict=(call % 2 == 1))
        tw.check_table()
        say(f"  call {call}: statuses {np.bincount(st, minlength=6)[1:5]}, size {tw.ora.size()}")
    tw.find(as_u64(gen_keys(100, 1 << 16)))


def test_export_beyond_one_grid():
    """Export of a 2^27-slot (2^20-bucket) table, more buckets than one pass of the export grid
    covers; sparse contents keep the oracle quick."""
    tw = Twin(1 << 27, 4, "dual", "lru", seed=53)
    for call in range(2):
        tw.upsert(as_u64(gen_keys(120 + call, 1 << 20)))
    tw.erase(as_u64(gen_keys(120, 1 << 18)))
    tw.check_table()
    tw.export_if(2)


@pytest.mark.parametrize("policy", ["custom", "lfu"])
@pytest.mark.parametrize("distinct", [400, 600])
def test_crowded_bucket_merge_table_and_fallback(policy, distinct):
    """One bucket receives every key of the batch, each key from several blocks of 2048 input
    positions, so the slow apply merges one entry per block and key: 400 distinct keys fit its LDS
    merge table, 600 overflow it and merge through the call's dedupe set instead.  The bucket is
    filled first, then takes the crowded batch with evictions, against the oracle."""
    nb = 8
    tw = Twin(nb * 128, 4, "single", policy, seed=54)
    fill = np.array(keys_for(3, 3, nb, 128, salt0=1 << 12), dtype=np.uint64)
    sc = np.arange(1, 129, dtype=np.uint64) * np.uint64(10)
    tw.upsert(fill, sc if policy == "custom" else None)
    ks = np.array(keys_for(3, 3, nb, distinct, salt0=1 << 13), dtype=np.uint64)
    reps = 12 if distinct == 400 else 8  # 4800 positions: every key in at least two input blocks
    batch = np.concatenate([ks if r % 2 == 0 else ks[::-1] for r in range(reps)])
    if policy == "custom":
        scores = (as_u64(uniform_u64(130 + distinct, batch.size)) % np.uint64(2000)) + np.uint64(1)
    else:
        scores = (as_u64(uniform_u64(131 + distinct, batch.size)) % np.uint64(3)) + np.uint64(1)
    say(f"crowded bucket, {policy}, {distinct} distinct keys in {batch.size} positions")
    st = tw.upsert(batch, scores, evict=True)
    assert (st == 3).sum() > 0 and (st == 4).sum() > 0
    tw.check_table()
    tw.find(np.concatenate([fill, ks]))
