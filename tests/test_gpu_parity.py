"""GPU parity: the HIP table, called through the C-ABI, against the sequential oracle, bit for bit
(statuses, found masks, rows, scores, evicted sets, per-bucket table contents)."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, keys as gen_keys, randint, uniform_u64
from tests.hashkeys import key_for
from tests.parity import Twin

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_keys(stream, n, start=0):
    return as_u64(gen_keys(stream, n, start))


def test_c1_config_full_flow():
    """Plain table, 2^18 slots (2048 x 128), dim 8, CUSTOM score = batch step: 16 insert batches
    of 2^14 fresh keys to full load, a 2^16-key find at 50 % hit, 4 more insert_and_evict
    batches past capacity; a twin run with insert_or_assign must end in the same table."""
    say("c1: capacity 2^18 dim 8 dual custom")
    tw = Twin(1 << 18, 8, "dual", "custom", seed=1)
    twin2 = Twin(1 << 18, 8, "dual", "custom", seed=1)
    bs = 1 << 14
    for t in range(1, 17):
        k = np_keys(1, bs, (t - 1) * bs)
        sc = np.full(bs, t, dtype=np.uint64)
        tw.upsert(k, sc)
        twin2.upsert(k, sc)
        tw.check_table()
    say("c1: size", tw.ora.size())
    resident = tw.ora.export()[0]
    rng = np.random.default_rng(2)
    hit = rng.choice(resident, 1 << 15, replace=False)
    miss = np_keys(2, 1 << 15)
    q = np.concatenate([hit, miss])[rng.permutation(1 << 16)]
    of = tw.find(q)
    assert of.sum() == 1 << 15
    for t in range(17, 21):
        k = np_keys(1, bs, (t - 1) * bs)
        sc = np.full(bs, t, dtype=np.uint64)
        tw.upsert(k, sc, evict=True)
        twin2.upsert(k, sc, evict=False)
        tw.check_table()
    twin2.check_table()


@pytest.mark.parametrize("mode", ["single", "dual"])
@pytest.mark.parametrize("policy", ["custom", "lru", "lfu"])
def test_random_mixed_small_tables(mode, policy):
    """Random upsert / insert_and_evict / erase / find batches with duplicates and reserved
    words on small tables that fill, overflow and drain; whole-table parity after each call."""
    say(f"mixed: mode {mode} policy {policy}")
    for seed, nb in [(1, 4), (2, 16), (3, 64)]:
        rng = np.random.default_rng(seed * 100 + len(mode) + len(policy))
        tw = Twin(nb * 128, 16, mode, policy, seed=seed)
        universe = np_keys(10 + seed, nb * 128 * 3)
        universe = np.concatenate([universe, np.array([0, M64], dtype=np.uint64)])
        for step in range(24):
            n = int(rng.integers(0, nb * 128))
            k = rng.choice(universe, n)
            r = rng.random()
            if r < 0.6:
                if policy == "custom":
                    sc = rng.integers(0, 50, n).astype(np.uint64)
                elif policy == "lfu":
                    sc = rng.choice(np.array([1, 1, 2, 7], dtype=np.uint64), n) if rng.random() < 0.7 else None
                else:
                    sc = None
                tw.upsert(k, sc, evict=bool(rng.random() < 0.5))
            elif r < 0.8:
                tw.erase(k)
            else:
                tw.find(k)
            tw.check_table()


def test_one_bucket_floods():
    """Hundreds of distinct keys aimed at one bucket (b1 == b2): the bucket must keep exactly
    the best 128 by (score, key), whatever the batch size (up to 3 selection chunks and beyond)."""
    nb = 8
    for m, seed in [(100, 1), (129, 2), (200, 3), (700, 4)]:
        say(f"flood: {m} keys into bucket 3")
        tw = Twin(nb * 128, 8, "dual", "custom", seed=seed)
        rng = np.random.default_rng(seed)
        k = np.array([key_for(3, 3, nb, salt=1 + i) for i in range(m)], dtype=np.uint64)
        sc = rng.integers(0, 40, m).astype(np.uint64)
        tw.upsert(k, sc)
        tw.check_table()
        k2 = np.array([key_for(3, 3, nb, salt=5000 + i) for i in range(m)], dtype=np.uint64)
        tw.upsert(np.concatenate([k2, k[: m // 3]]), rng.integers(0, 60, m + m // 3).astype(np.uint64), evict=True)
        tw.check_table()


def test_digest_collisions_and_equal_candidates():
    """Distinct keys with the same bucket and the same 8-bit digest, and keys whose two
    candidates coincide, in single and dual tables."""
    nb = 16
    for mode in ["single", "dual"]:
        say(f"digest collisions: {mode}")
        tw = Twin(nb * 128, 8, mode, "custom", seed=7)
        ks = [key_for(5, 5, nb, salt=1 + i, digest=0x33) for i in range(150)]
        ks += [key_for(5, 9, nb, salt=900 + i, digest=0x33) for i in range(150)]
        ks += [key_for(9, 5, nb, salt=1900 + i, digest=0x33) for i in range(60)]
        k = np.array(ks, dtype=np.uint64)
        rng = np.random.default_rng(1)
        for rep in range(3):
            sel = rng.permutation(k.size)[: 200]
            tw.upsert(k[sel], rng.integers(0, 100, sel.size).astype(np.uint64), evict=True)
            tw.check_table()
            tw.find(k)
        tw.erase(k[::3])
        tw.check_table()
        tw.find(k)


def test_dual_phase_d2_full_tables():
    """Fill every bucket, then stream fresh keys so that all routing is phase D2 with LRU
    scores (many equal minima broken by key)."""
    say("d2: lru full table")
    nb = 64
    tw = Twin(nb * 128, 8, "dual", "lru", seed=3)
    k = np_keys(30, nb * 128 * 2)
    for s in range(0, k.size, 1024):
        tw.upsert(k[s:s + 1024])
    tw.check_table()
    for rep in range(6):
        tw.upsert(np_keys(31, 3000, rep * 3000), evict=True)
        tw.check_table()


def test_lfu_zipf_like_duplicates():
    """A few keys repeated thousands of times in one batch (LFU sums, last-writer rows)."""
    say("lfu duplicates")
    tw = Twin(32 * 128, 8, "dual", "lfu", seed=4)
    rng = np.random.default_rng(5)
    hot = np_keys(40, 50)
    cold = np_keys(41, 6000)
    for rep in range(4):
        k = np.concatenate([rng.choice(hot, 20000), rng.choice(cold, 3000)])[rng.permutation(23000)]
        tw.upsert(k, None, evict=True)
        tw.check_table()
    sat = np.array([(1 << 63), (1 << 63), 5], dtype=np.uint64)
    tw.upsert(np.array([hot[0], hot[0], hot[1]], dtype=np.uint64), sat)
    tw.check_table()


@pytest.mark.parametrize("pairs", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 257, 4099])
def test_ragged_batch_sizes(n, pairs):
    tw = Twin(64 * 128, 12, "dual", "lru", seed=n)
    tw.gpu.set_tuning(find_pairs=pairs)
    k = np_keys(50, n)
    tw.upsert(k, evict=True)
    tw.find(np.concatenate([k, np_keys(51, n)]))
    tw.erase(k[: (n + 1) // 2])
    tw.check_table()
    tw.upsert(np.zeros(0, dtype=np.uint64))  # empty batch: no-op, no clock tick
    tw.check_table()


@pytest.mark.parametrize("dim", [4, 8, 32, 64, 128, 132, 1020, 1024])
def test_value_dims(dim):
    say(f"dim {dim}")
    tw = Twin(32 * 128, dim, "dual", "custom", seed=dim)
    tw.gpu.set_tuning(find_pairs=dim % 8 == 0)
    rng = np.random.default_rng(dim)
    for rep in range(3):
        k = np_keys(60, 6000, rep * 2000)
        tw.upsert(k, rng.integers(0, 9, k.size).astype(np.uint64), evict=True)
        tw.find(np_keys(60, 9000))
    tw.check_table()


@pytest.mark.parametrize("dim", [4, 32, 64, 128])
@pytest.mark.parametrize("n_upd,n_ins", [(1, 1), (2, 2), (6, 9), (10, 30)])
def test_update_then_evict_in_one_call(dim, n_upd, n_ins):
    """A full bucket receives, in one call, updates that lower some residents' scores below all
    others and inserts with higher scores: the victims are the entries just updated, and the
    evicted rows must be the rows those updates wrote (Alg. 2 runs on the bucket as the updates
    left it).  Sizes cover the register-held row path (few operations) and the loop path."""
    say(f"update-then-evict: dim {dim}, {n_upd} updates, {n_ins} inserts")
    nb = 8
    tw = Twin(nb * 128, dim, "dual", "custom", seed=dim + n_ins)
    res = np.array([key_for(3, 3, nb, salt=1 + i) for i in range(128)], dtype=np.uint64)
    tw.upsert(res, np.arange(10, 138, dtype=np.uint64))
    tw.check_table()
    upd = res[[5 + 7 * i for i in range(n_upd)]]
    ins = np.array([key_for(3, 3, nb, salt=900 + i) for i in range(n_ins)], dtype=np.uint64)
    keys = np.concatenate([ins[: n_ins // 2], upd, ins[n_ins // 2:]])
    sc = np.concatenate([np.arange(500, 500 + n_ins // 2), np.arange(1, 1 + n_upd),
                         np.arange(600, 600 + n_ins - n_ins // 2)]).astype(np.uint64)
    st = tw.upsert(keys, sc, evict=True)
    assert (st[n_ins // 2: n_ins // 2 + n_upd] == cskv.ST_UPDATED).all()
    tw.check_table()


@pytest.mark.parametrize("policy", ["custom", "lru", "lfu"])
def test_full_bucket_call_sequences(policy):
    """Many small calls on full buckets: a few inserts above and below the residents' scores
    (evicting or rejected), calls with many inserts, updates beside an insert, assign_scores and
    erases followed by refills, each followed by whole-table parity with the oracle (the bucket
    minimum cached for routing must follow every change)."""
    say(f"full-bucket sequences: {policy}")
    nb = 4
    tw = Twin(nb * 128, 8, "dual", policy, seed=7)
    rng = np.random.default_rng(len(policy))
    salt = [1]
    owner = {}  # key -> its bucket (both candidates of every key here are the same bucket)

    def fresh(b, n):
        k = np.array([key_for(b, b, nb, salt=salt[0] + i) for i in range(n)], dtype=np.uint64)
        salt[0] += n
        owner.update((int(x), b) for x in k)
        return k

    def residents_of(b):
        return np.array([x for x in tw.ora.export()[0] if owner.get(int(x)) == b], dtype=np.uint64)

    def scores(n, lo, hi):
        if policy == "custom":
            return rng.integers(lo, hi, n).astype(np.uint64)
        if policy == "lfu":
            return rng.integers(1, 4, n).astype(np.uint64)
        return None

    for b in (1, 2):
        tw.upsert(fresh(b, 128), scores(128, 100, 1000))
    tw.check_table()
    for step in range(60):
        b = 1 + step % 2
        r = rng.random()
        if r < 0.55:  # a few inserts
            k = fresh(b, int(rng.integers(1, 7)))
            tw.upsert(k, scores(k.size, 0, 1200), evict=bool(rng.random() < 0.5))
        elif r < 0.65:  # many inserts
            k = fresh(b, int(rng.integers(7, 16)))
            tw.upsert(k, scores(k.size, 0, 1200), evict=True)
        elif r < 0.75:  # updates of residents (plus an insert) in one call
            mine = residents_of(b)
            k = np.concatenate([rng.choice(mine, 2, replace=False), fresh(b, 1)])
            tw.upsert(k, scores(k.size, 0, 1200))
        elif r < 0.85 and policy != "lru":  # assign_scores: scores change in place
            mine = residents_of(b)
            k = rng.choice(mine, 3, replace=False)
            tw.assign(k, scores(k.size, 0, 1200), with_values=False)
        else:  # erase, then refill to full
            mine = residents_of(b)
            k = rng.choice(mine, int(rng.integers(1, 4)), replace=False)
            tw.erase(k)
            tw.upsert(fresh(b, k.size), scores(k.size, 500, 1500))
        tw.check_table()


@pytest.mark.parametrize("policy", ["custom", "lru", "lfu"])
@pytest.mark.parametrize("evict", [False, True])
def test_repeated_keys_take_last_occurrence(policy, evict):
    """Keys repeated three times in one call, far apart, with different values and scores: some
    resident (updates), some fresh (inserts). The call must act as the key's last occurrence
    (its row; CUSTOM: its score; LFU: the sum of the increments, added to a resident's score),
    every occurrence reporting that operation's status; whole-table parity after each call."""
    say(f"repeated keys: {policy}, evict {evict}")
    nb = 32  # 4096 slots: the later calls also evict
    tw = Twin(nb * 128, 16, "dual", policy, seed=3)
    rng = np.random.default_rng(5)
    resident = np_keys(70, 3000)
    tw.upsert(resident, rng.integers(1, 50, resident.size).astype(np.uint64) if policy != "lru" else None)
    tw.check_table()
    for step in range(4):
        fresh = np_keys(71, 400, step * 400)
        again = rng.choice(resident, 300, replace=False)
        base = np.concatenate([fresh, again])
        keys = np.concatenate([base, rng.permutation(base), rng.permutation(base)])
        if policy == "custom":
            sc = rng.integers(0, 100, keys.size).astype(np.uint64)
        elif policy == "lfu":
            sc = rng.integers(1, 5, keys.size).astype(np.uint64)
        else:
            sc = None
        tw.upsert(keys, sc, evict=evict)
        tw.check_table()


def test_api_errors_on_gpu():
    t = cskv.Table(128 * 16, 8, "dual", "custom")
    k = torch.ones(4, dtype=torch.int64, device="cuda")
    v = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(cskv.CskvError):
        t.insert_or_assign(k, v, None)  # CUSTOM needs scores
    with pytest.raises(cskv.CskvError):
        t.export(5, 3)
    bad = torch.zeros(4 * 8 + 1, dtype=torch.float32, device="cuda")[1:].view(4, 8)  # misaligned rows
    with pytest.raises(cskv.CskvError):
        t.insert_or_assign(k, bad, k)
    lib = cskv.lib()
    assert lib.cskv_table_bytes(128 * 3, 128, 8) == 0  # 3 buckets: not a power of two
    assert lib.cskv_table_bytes(128 * 4, 64, 8) == 0
    assert lib.cskv_table_bytes(128 * 4, 128, 6) == 0


@pytest.mark.parametrize("group", [4, 8, 16])
def test_find_without_digest_matches(group):
    """The digest ablation (Exp. 3a) scans every stored key of a candidate bucket; it must give
    the oracle's results, including after erases that leave stale keys in freed slots and keys
    re-inserted elsewhere in the same bucket."""
    say(f"find without digest, group {group}")
    nb = 8
    tw = Twin(nb * 128, 8, "dual", "custom", seed=group)
    tw.gpu.set_tuning(find_group=group, find_digest=0)
    assert tw.gpu.get_tuning()["find_digest"] == 0
    rng = np.random.default_rng(group)
    k = np.array([key_for(3, 3, nb, salt=1 + i) for i in range(100)], dtype=np.uint64)
    tw.upsert(k, rng.integers(0, 9, k.size).astype(np.uint64))
    tw.erase(k[:50])
    tw.find(k)
    other = np.array([key_for(3, 3, nb, salt=1000 + i) for i in range(60)], dtype=np.uint64)
    tw.upsert(other, rng.integers(0, 9, other.size).astype(np.uint64))  # takes the freed slots
    tw.upsert(k[:50], rng.integers(0, 9, 50).astype(np.uint64))  # back in, other slots
    tw.find(np.concatenate([k, other, np_keys(81, 500)]))
    for rep in range(4):
        tw.upsert(np_keys(80, 3000, rep * 1000), rng.integers(0, 20, 3000).astype(np.uint64), evict=True)
        tw.erase(np_keys(80, 400, rep * 900))
        tw.find(np_keys(80, 6000))
    tw.check_table()
    with pytest.raises(cskv.CskvError):
        tw.gpu.set_tuning(find_digest=2)


def test_launch_shapes_do_not_change_results():
    """Every tuning variant (probe lanes per key, b2 prefetch, route lanes) gives bit-identical
    outputs and tables, and matches the oracle."""
    say("tuning variants")
    for fg, pre, rg, pairs in [(4, 0, 8, 0), (8, 1, 16, 0), (16, 1, 4, 0), (16, 0, 16, 0), (4, 0, 8, 1),
                               (8, 1, 8, 1), (16, 0, 4, 1)]:
        tw = Twin(64 * 128, 8, "dual", "lru", seed=9)
        tw.gpu.set_tuning(find_group=fg, find_prefetch_b2=pre, route_group=rg, find_pairs=pairs)
        got = tw.gpu.get_tuning()
        assert (got["find_group"], got["route_group"], got["find_prefetch_b2"]) == (fg, rg, pre)
        for rep in range(4):
            tw.upsert(np_keys(70, 5000, rep * 3000), evict=True)
            tw.find(np_keys(70, 20000))
            tw.erase(np_keys(70, 500, rep * 700))
        tw.check_table()
    with pytest.raises(cskv.CskvError):
        tw.gpu.set_tuning(find_group=5)


@pytest.mark.parametrize("policy", ["custom", "lfu", "lru"])
def test_cached_minimum_after_update_only_calls(policy):
    """A full bucket's cached minimum (score, key) through calls the apply may finish without
    reading the bucket's lines: updates that leave the minimum the smallest entry, updates of the
    minimum's own key, (CUSTOM) updates to a smaller score or to the minimum's score with a
    smaller key, and calls whose inserts cannot beat the minimum.  After each call one insert that
    just beats the true minimum shows which entry the table evicts; everything against the oracle."""
    nb = 4
    tw = Twin(nb * 128, 8, "dual", policy, seed=17)
    salt = [1 << 16]

    def fresh(n):
        k = np.array([key_for(1, 1, nb, salt=salt[0] + i) for i in range(n)], dtype=np.uint64)
        salt[0] += n
        return k

    def bucket():
        k, _, s, _ = tw.ora.export()
        return k, s

    def minimum():
        k, s = bucket()
        o = np.lexsort((k, s))
        return k[o[0]], s[o[0]], k[o[1]]

    def sc(vals):
        return None if policy == "lru" else np.asarray(vals, dtype=np.uint64)

    fill = fresh(128)
    tw.upsert(fill, sc(np.arange(100, 228) if policy == "custom" else np.ones(128)))
    tw.check_table()

    def probe():
        # one insert scoring just above the minimum evicts exactly the minimum
        mk, ms, _ = minimum()
        tw.upsert(fresh(1), sc([int(ms) + 1]), evict=True)
        tw.check_table()

    for step in range(4):
        mk, ms, second = minimum()
        k, s = bucket()
        other = k[(k != mk) & (k != second)][step]
        # an update that leaves the minimum the smallest entry
        tw.upsert(np.array([other], dtype=np.uint64), sc([int(ms) + 50]))
        tw.check_table()
        probe()
        # an update of the minimum's own key
        mk, ms, _ = minimum()
        tw.upsert(np.array([mk], dtype=np.uint64), sc([int(ms) + 7]))
        tw.check_table()
        probe()
        if policy == "custom":
            # a resident lowered below the minimum, then one set to the minimum's score with a smaller key
            mk, ms, _ = minimum()
            k, s = bucket()
            tw.upsert(np.array([k[k != mk][0]], dtype=np.uint64), sc([max(int(ms) - 3, 1)]))
            tw.check_table()
            probe()
            mk, ms, _ = minimum()
            k, s = bucket()
            smaller = k[k < mk]
            if smaller.size:
                tw.upsert(np.array([smaller[0]], dtype=np.uint64), sc([int(ms)]))
                tw.check_table()
                probe()
        # inserts that cannot beat the minimum, beside an update of another resident
        mk, ms, _ = minimum()
        k, s = bucket()
        weak = fresh(3)
        if policy == "lru":
            tw.upsert(np.concatenate([weak, k[k != mk][:1]]), None, evict=True)  # LRU inserts always win
        else:
            tw.upsert(np.concatenate([weak, k[k != mk][:1]]), sc([int(ms)] * 3 + [int(ms) + 9]), evict=True)
        tw.check_table()
        probe()
