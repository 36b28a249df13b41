"""Pins of the route sub-round setting against the one-round batch semantics: a call with r
sub-rounds cuts its distinct keys, ordered by last occurrence, into chunks (rank q in chunk
q * r // N) and equals the sequence of r ordinary calls that each carry exactly the occurrences
of one chunk's keys (CUSTOM and LFU scores; an LRU call ticks its clock once, so it is left out).
With r >= N every key is its own call, in last-occurrence order."""
import random

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1


def chunks_of(keys, r):
    last = {}
    for i, k in enumerate(keys):
        if k not in (0, M64):
            last[k] = i
    by_last = sorted(last, key=lambda k: last[k])
    n = len(by_last)
    return [set(k for q, k in enumerate(by_last) if q * r // n == c) for c in range(r)] if n else []


def state(o):
    k, v, s, b = o.export()
    return sorted(zip(k.tolist(), v.tolist(), s.tolist(), b.tolist()))


@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LFU])
@pytest.mark.parametrize("r", [2, 3, 5, 64])
@pytest.mark.parametrize("evict", [False, True])
def test_subrounds_equal_a_sequence_of_calls(policy, r, evict):
    for seed in range(20):
        rng = random.Random(seed * 131 + r + policy)
        B, S = rng.choice([(1, 4), (2, 4), (4, 8)])
        a = oracle.Oracle(B, S, oracle.DUAL, policy)
        b = oracle.Oracle(B, S, oracle.DUAL, policy)
        a.set_subrounds(r)
        universe = [rng.getrandbits(64) | 1 for _ in range(B * S * 2)] + [0, M64]
        vid = 1
        for step in range(8):
            n = rng.randint(0, 3 * S)
            keys = np.array([rng.choice(universe) for _ in range(n)], dtype=np.uint64)
            vids = np.arange(vid, vid + n, dtype=np.uint64)
            vid += n
            sc = np.array([rng.randint(0, 30) if policy == oracle.CUSTOM else rng.choice([1, 2, 7])
                           for _ in range(n)], dtype=np.uint64)
            st_a, ek_a, ev_a, es_a = a.upsert(keys, vids, sc)
            st_b = np.full(n, 5, dtype=np.uint8)  # reserved keys: INVALID_KEY
            ev_b = []
            for ch in chunks_of(keys.tolist(), r):
                idx = np.array([i for i, k in enumerate(keys.tolist()) if k in ch], dtype=np.int64)
                s_, ek, ev, es = b.upsert(keys[idx], vids[idx], sc[idx])
                st_b[idx] = s_
                ev_b += list(zip(ek.tolist(), ev.tolist(), es.tolist()))
            assert np.array_equal(st_a, st_b), (seed, step)
            if evict:
                assert sorted(zip(ek_a.tolist(), ev_a.tolist(), es_a.tolist())) == sorted(ev_b)
            assert state(a) == state(b), (seed, step)


def test_subrounds_one_is_the_default_and_bounds_are_checked():
    o = oracle.Oracle(2, 4, oracle.DUAL, oracle.CUSTOM)
    with pytest.raises(ValueError):
        o.set_subrounds(0)
    with pytest.raises(ValueError):
        o.set_subrounds(65)
    o.set_subrounds(1)


def test_many_subrounds_place_a_large_batch_better():
    """Snapshot routing sends every key of a batch by the occupancies from before the batch, so
    a large batch of fresh keys into an empty dual table piles onto b1 (ties go to b1) and
    overflows; 64 sub-rounds refresh the occupancies and place all of it (the trade-off the
    setting exists for).  A few sub-rounds are not monotone in between: each chunk still routes
    against one snapshot."""
    placed = {}
    for r in (1, 64):
        o = oracle.Oracle(64, 128, oracle.DUAL, oracle.CUSTOM)
        o.set_subrounds(r)
        rng = np.random.default_rng(3)
        n = int(0.95 * 64 * 128)
        keys = rng.integers(1, 1 << 62, n, dtype=np.uint64)
        st = o.upsert(keys, np.arange(n, dtype=np.uint64), np.full(n, 1, dtype=np.uint64))[0]
        placed[r] = float((st == 2).mean())
    assert placed[1] < 0.99 and placed[64] == 1.0
