"""Pins of the oracle against facts fixed outside it: hand-derived cases of the paper's
algorithms, textbook reductions (a dictionary, a bounded top-S heap), brute force over batch
orders, the paper's admission-burst table, Prop. 3's order statistic, and load-factor facts."""
import itertools
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from oracle import pyoracle
from tests.hashkeys import key_for

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


def _state(o):
    k, v, s, b = o.export()
    out = {}
    for kk, vv, ss, bb in zip(k.tolist(), v.tolist(), s.tolist(), b.tolist()):
        out.setdefault(int(bb), []).append((int(kk), int(ss), int(vv)))
    return {b: sorted(x) for b, x in out.items()}


def _check_invariants(o):
    k, v, s, b = o.export()
    keys = k.tolist()
    assert len(set(keys)) == len(keys), "duplicate key in table"
    for kk, bb in zip(keys, b.tolist()):
        assert int(bb) in o.candidates(kk), "key outside its candidate buckets"
    for bb in range(o.B):
        assert o.bucket_count(bb) <= o.S


# ---------------------------------------------------------------- hand-derived cases
def _load_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("impl", ["c", "py"])
def test_hand_derived_cases(case, impl):
    B = case["n_buckets"]
    labels = sorted(case["buckets"])
    # distinct keys with the wanted candidates, then sorted so label order == key order
    key = {}
    for i, lb in enumerate(labels):
        # the i-th label gets a key in the i-th sixteenth of the 64-bit range
        b1, b2 = case["buckets"][lb]
        salt = 1
        while True:
            k = key_for(b1, b2, n_buckets=max(B, 2), salt=salt)
            if k >> 60 == i:
                break
            salt += 1
        key[lb] = k
    lab = {v: k for k, v in key.items()}
    if impl == "c":
        t = oracle.Oracle(B, case["bucket_size"], case["mode"], case["policy"])
    else:
        t = pyoracle.PyTable(B, case["bucket_size"], case["mode"], case["policy"])
    for lb in labels:
        b1, b2 = case["buckets"][lb]
        cand = (t.candidates(key[lb]))
        exp = (b1, b2 if case["mode"] == 2 else b1) if B > 1 else (0, 0)
        assert tuple(cand) == exp
    for step in case["steps"]:
        op = step["op"]
        if op == "upsert":
            ks = [key[x] for x in step["keys"]]
            if impl == "c":
                st, ek, ev, es = t.upsert(ks, step["vids"], step["scores"])
                st = st.tolist()
                evicted = sorted((lab[int(a)], int(c), int(b)) for a, b, c in zip(ek, ev, es))
            else:
                st, evp = t.upsert(ks, step["vids"], step["scores"])
                evicted = sorted((lab[a], c, b) for a, c, b in evp)
            assert st == step["status"], step
            assert evicted == sorted(tuple(e) for e in step["evicted"]), step
        elif op == "find":
            ks = [key[x] for x in step["keys"]]
            if impl == "c":
                f, v, s = t.find(ks)
                got = [[int(s[i]), int(v[i])] if f[i] else None for i in range(len(ks))]
                assert f.tolist() == step["found"]
            else:
                got = [list(r) if r is not None else None for r in t.find(ks)]
            assert got == step["rows"]
        elif op == "erase":
            ks = [key[x] for x in step["keys"]]
            er = t.erase(ks)
            assert [int(x) for x in (er.tolist() if impl == "c" else er)] == step["erased"]
        elif op == "table":
            state = _state(t) if impl == "c" else t.export()
            got = {str(b): sorted([lab[k], s, v] for k, s, v in ents) for b, ents in state.items()}
            exp = {b: sorted(e) for b, e in step["table"].items()}
            assert got == exp


# ---------------------------------------------------------------- dictionary reduction
@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
def test_below_capacity_is_a_dictionary(policy, mode):
    """With no bucket ever full the table is an ordinary map with last-writer-wins batches."""
    rng = random.Random(policy * 10 + mode)
    B, S = 64, 128
    o = oracle.Oracle(B, S, mode, policy)
    universe = [rng.getrandbits(64) | 2 for _ in range(1500)]
    model = {}  # key -> (score, vid)
    clock = 0
    vid = 0
    for _ in range(60):
        r = rng.random()
        n = rng.randint(0, 120)
        ks = [rng.choice(universe) for _ in range(n)]
        if r < 0.55:
            vids = list(range(vid, vid + n))
            vid += n
            sc = [rng.randint(0, 1000) for _ in range(n)] if policy != oracle.LRU else None
            st = o.upsert(ks, vids, sc)[0].tolist()
            if n:
                clock += 1
            before = dict(model)
            for i, k in enumerate(ks):
                exp_st = oracle.UPDATED if k in before else oracle.INSERTED
                assert st[i] == exp_st
            last = {k: i for i, k in enumerate(ks)}
            tot = {}
            for i, k in enumerate(ks):
                tot[k] = tot.get(k, 0) + (sc[i] if sc else 1)
            for k, i in last.items():
                if policy == oracle.CUSTOM:
                    s = sc[i]
                elif policy == oracle.LRU:
                    s = clock
                else:
                    s = before.get(k, (0,))[0] + tot[k]
                model[k] = (s, vids[i])
        elif r < 0.75:
            er = o.erase(ks).tolist()
            before = set(model)
            assert er == [int(k in before) for k in ks]
            for k in ks:
                model.pop(k, None)
        else:
            f, v, s = o.find(ks)
            for i, k in enumerate(ks):
                assert bool(f[i]) == (k in model)
                if k in model:
                    assert (int(s[i]), int(v[i])) == model[k]
        assert o.size() == len(model)
        _check_invariants(o)


# ---------------------------------------------------------------- bounded top-S heap
@pytest.mark.parametrize("S", [4, 16, 128])
def test_single_mode_bucket_keeps_top_s_offered(S):
    """Single mode, each key with one fixed distinct score: after any sequence of batches each
    bucket holds exactly the S highest-scored keys ever offered to it (a bounded min-heap keeps
    the top S of everything offered, whatever the order)."""
    rng = random.Random(S)
    B = 8
    o = oracle.Oracle(B, S, oracle.SINGLE, oracle.CUSTOM)
    pool = rng.sample(range(1, 10 ** 9), 40 * S)
    score_of = {k: rng.getrandbits(40) * 4096 + i for i, k in enumerate(pool)}  # distinct
    offered = {b: set() for b in range(B)}
    for _ in range(30):
        ks = [rng.choice(pool) for _ in range(rng.randint(1, 3 * S))]
        st, ek, ev, es = o.upsert(ks, [0] * len(ks), [score_of[k] for k in ks])
        for k in ks:
            offered[o.candidates(k)[0]].add(k)
        state = _state(o)
        for b in range(B):
            top = sorted(offered[b], key=lambda k: -score_of[k])[:S]
            assert sorted(x[0] for x in state.get(b, [])) == sorted(top)
        # statuses agree with the heap: a key inserted by this batch is never evicted by it,
        # a refused key is not resident (an updated resident may be displaced in the batch)
        resident = {x[0] for ents in state.values() for x in ents}
        for k, s_ in zip(ks, st.tolist()):
            if s_ == oracle.REJECTED:
                assert k not in resident
            elif s_ in (oracle.INSERTED, oracle.INSERTED_EVICT):
                assert k in resident


# ---------------------------------------------------------------- batch-order brute force
@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
@pytest.mark.parametrize("B,S", [(1, 4), (2, 4), (2, 8)])
def test_result_independent_of_order_of_distinct_keys(mode, policy, B, S):
    rng = random.Random(B * 100 + S + policy * 7 + mode)
    for trial in range(3):
        pre = [rng.getrandbits(64) | 1 for _ in range(rng.randint(0, B * S))]
        pre_sc = [rng.randint(1, 9) for _ in pre]
        batch = rng.sample([rng.getrandbits(64) | 1 for _ in range(20)] + pre, 6)
        sc = {k: rng.randint(0, 10) for k in batch}
        vid = {k: 1000 + i for i, k in enumerate(batch)}
        results = set()
        for perm in itertools.permutations(batch):
            o = oracle.Oracle(B, S, mode, policy)
            if pre:
                o.upsert(pre, list(range(len(pre))), pre_sc if policy != oracle.LRU else None)
            st, ek, ev, es = o.upsert(list(perm), [vid[k] for k in perm],
                                      [sc[k] for k in perm] if policy != oracle.LRU else None)
            by_key = tuple(sorted(zip(perm, st.tolist())))
            evs = tuple(sorted(zip(ek.tolist(), es.tolist(), ev.tolist())))
            tab = tuple(sorted((b, tuple(v)) for b, v in _state(o).items()))
            results.add((by_key, evs, tab))
        assert len(results) == 1


# ---------------------------------------------------------------- admission burst (Exp. 3d)
def _full_table(B, S, mode, rng, lo=2, hi=10 ** 6):
    o = oracle.Oracle(B, S, mode, oracle.CUSTOM)
    keys, scores = [], []
    for b in range(B):
        for j in range(S):
            keys.append(key_for(b, b, B, salt=1 + j * 131 + b * 7))
            scores.append(rng.randint(lo, hi))
    st = o.upsert(keys, list(range(len(keys))), scores)[0]
    assert (st == oracle.INSERTED).all() and o.size() == B * S
    return o, keys


@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
def test_admission_burst_table(mode):
    """The paper's admission ablation: a burst of score-1 keys into a full table is fully
    rejected and leaves the hit rate unchanged; a burst of score-1e9 keys is fully admitted."""
    rng = random.Random(mode)
    B, S = 256, 128
    o, resident = _full_table(B, S, mode, rng)
    before = _state(o)
    burst = [rng.getrandbits(64) | 1 for _ in range(B * S // 4)]
    st = o.upsert(burst, [0] * len(burst), [1] * len(burst))[0]
    assert (st == oracle.REJECTED).all()  # 0 % admitted
    assert _state(o) == before  # +0.00 pp hit rate
    assert o.find(resident)[0].all()
    st = o.upsert(burst, [1] * len(burst), [10 ** 9] * len(burst))[0]
    assert (st == oracle.INSERTED_EVICT).all()  # 100 % admitted
    assert o.find(burst)[0].all()
    assert o.size() == B * S


# ---------------------------------------------------------------- Prop. 3
def test_prop3_dual_choice_halves_expected_evicted_score():
    """Full buckets of n=128 i.i.d. U[0,1) scores: evicting the lower bucket minimum of two
    candidates gives E = 1/(2n+1), one candidate gives 1/(n+1) (Prop. 3)."""
    rng = random.Random(42)
    B, S = 1024, 128
    scale = float(1 << 52)
    means = {}
    for mode in (oracle.SINGLE, oracle.DUAL):
        ev_scores = []
        for rep in range(3):
            o = oracle.Oracle(B, S, mode, oracle.CUSTOM)
            keys, sc = [], []
            for b in range(B):
                for j in range(S):
                    keys.append(key_for(b, b, B, salt=1 + j * 131 + rep * 17))
                    sc.append(rng.getrandbits(52))
            o.upsert(keys, [0] * len(keys), sc)
            # probes: distinct candidate pairs, pairwise disjoint so no bucket is hit twice
            perm = list(range(B))
            rng.shuffle(perm)
            probes = []
            for q in range(0, B - 1, 2):
                b1, b2 = perm[q], perm[q + 1]
                probes.append(key_for(b1, b2, B, salt=(1 << 19) + q))
            if mode == oracle.SINGLE:
                probes = probes[: B // 2]
            st, ek, ev, es = o.upsert(probes, [0] * len(probes), [1 << 60] * len(probes))
            assert (st == oracle.INSERTED_EVICT).all()
            ev_scores += (es.astype(np.float64) / scale).tolist()
        means[mode] = np.mean(ev_scores)
    n = 128
    e_single, e_dual = 1 / (n + 1), 1 / (2 * n + 1)
    # sd of a minimum of m uniforms ~ 1/(m+1); ~1500 samples -> sd of the mean ~ 2.6 % of it
    assert abs(means[oracle.SINGLE] - e_single) < 0.12 * e_single
    assert abs(means[oracle.DUAL] - e_dual) < 0.12 * e_dual
    assert 0.4 < means[oracle.DUAL] / means[oracle.SINGLE] < 0.6


# ---------------------------------------------------------------- load-factor facts
def test_single_mode_first_eviction_matches_bucket_counting():
    """Single mode: the first non-INSERTED status comes exactly with the first key that is the
    (S+1)-th distinct key of its bucket; the load factor there is near the paper's ~0.63 for
    128-slot buckets (balls into bins)."""
    B, S = 1 << 12, 128
    o = oracle.Oracle(B, S, oracle.SINGLE, oracle.CUSTOM)
    rng = np.random.default_rng(9)
    keys = np.unique(rng.integers(1, 2 ** 63, size=B * S, dtype=np.uint64))
    keys = keys[rng.permutation(keys.size)]
    b1 = np.array([o.candidates(int(k))[0] for k in keys])
    # first index where some bucket count reaches S+1
    counts = np.zeros(B, dtype=np.int64)
    first = None
    for i, b in enumerate(b1):
        counts[b] += 1
        if counts[b] == S + 1:
            first = i
            break
    assert first is not None
    batch = 64
    got = None
    for s in range(0, keys.size, batch):
        st = o.upsert(keys[s:s + batch], np.zeros(min(batch, keys.size - s), np.uint64),
                      np.full(min(batch, keys.size - s), 1 << 40, np.uint64))[0]
        bad = np.nonzero(st != oracle.INSERTED)[0]
        if bad.size:
            got = s + int(bad[0])
            break
    assert got == first
    lam = first / (B * S)
    assert 0.5 < lam < 0.7


def test_dual_mode_first_eviction_near_capacity():
    """Dual mode with load-balanced placement (phase D1) and small batches first evicts near
    full load; the paper reports 0.977 at 2^20 buckets."""
    B, S = 1 << 10, 128
    o = oracle.Oracle(B, S, oracle.DUAL, oracle.CUSTOM)
    rng = np.random.default_rng(3)
    keys = np.unique(rng.integers(1, 2 ** 63, size=B * S, dtype=np.uint64))
    keys = keys[rng.permutation(keys.size)]
    batch = 16
    first = None
    for s in range(0, keys.size, batch):
        kb = keys[s:s + batch]
        st = o.upsert(kb, np.zeros(kb.size, np.uint64), np.full(kb.size, 7, np.uint64))[0]
        if (st != oracle.INSERTED).any():
            first = s + int(np.nonzero(st != oracle.INSERTED)[0][0])
            break
    lam = (first if first is not None else keys.size) / (B * S)
    assert lam > 0.93


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
def test_conservation_and_invariants(mode, policy):
    rng = random.Random(mode * 3 + policy)
    B, S = 16, 8
    o = oracle.Oracle(B, S, mode, policy)
    universe = [rng.getrandbits(64) | 1 for _ in range(600)] + [0, M64]
    for _ in range(80):
        n = rng.randint(0, 60)
        ks = [rng.choice(universe) for _ in range(n)]
        size0 = o.size()
        if rng.random() < 0.8:
            sc = [rng.randint(0, 50) for _ in range(n)] if policy != oracle.LRU else None
            present = set(int(k) for k in o.export()[0].tolist())
            st, ek, ev, es = o.upsert(ks, list(range(n)), sc)
            st = st.tolist()
            uniq = {}
            for k, s_ in zip(ks, st):
                if k in (0, M64):
                    assert s_ == oracle.INVALID_KEY
                    continue
                assert uniq.setdefault(k, s_) == s_  # every occurrence reports one status
                assert s_ in (oracle.UPDATED, oracle.INSERTED, oracle.INSERTED_EVICT, oracle.REJECTED)
                assert (s_ == oracle.UPDATED) == (k in present)
            ins = sum(1 for s_ in uniq.values() if s_ in (oracle.INSERTED, oracle.INSERTED_EVICT))
            assert o.size() == size0 + ins - len(ek)
            assert sum(1 for s_ in uniq.values() if s_ == oracle.INSERTED_EVICT) == len(ek)
            # evicted keys were residents before the batch and are gone now
            assert set(int(k) for k in ek.tolist()) <= present
            assert not o.find(ek)[0].any()
        else:
            er = o.erase(ks)
            assert o.size() == size0 - len({k for k, e in zip(ks, er.tolist()) if e})
        _check_invariants(o)


def test_lru_bucket_keeps_most_recent():
    """Single mode, LRU, no erase: whenever a bucket is full, its minimum score is at least
    the latest score of every key that was dropped from it (evicted or refused)."""
    rng = random.Random(1)
    B, S = 4, 8
    o = oracle.Oracle(B, S, oracle.SINGLE, oracle.LRU)
    universe = [rng.getrandbits(64) | 1 for _ in range(200)]
    dropped = {b: 0 for b in range(B)}
    for step in range(200):
        ks = [rng.choice(universe) for _ in range(rng.randint(1, 12))]
        st, ek, ev, es = o.upsert(ks, [0] * len(ks))
        c = o.clock
        for k, s_ in zip(ks, st.tolist()):
            if s_ == oracle.REJECTED:
                b = o.candidates(k)[0]
                dropped[b] = max(dropped[b], c)
        for k, s_ in zip(ek.tolist(), es.tolist()):
            b = o.candidates(k)[0]
            dropped[b] = max(dropped[b], s_)
        state = _state(o)
        for b, ents in state.items():
            if len(ents) == S:
                assert min(e[1] for e in ents) >= dropped[b]


def test_reserved_words_and_empty_batches():
    o = oracle.Oracle(4, 4, oracle.DUAL, oracle.LRU)
    st = o.upsert([0, M64, 5], [1, 2, 3])[0]
    assert st.tolist() == [oracle.INVALID_KEY, oracle.INVALID_KEY, oracle.INSERTED]
    assert o.find([0, M64, 5])[0].tolist() == [0, 0, 1]
    assert o.erase([0, M64]).tolist() == [0, 0]
    c = o.clock
    o.upsert([], [])
    assert o.clock == c
    with pytest.raises(ValueError):
        oracle.Oracle(3, 4)
    cu = oracle.Oracle(4, 4, oracle.DUAL, oracle.CUSTOM)
    with pytest.raises(ValueError):
        cu.upsert([1], [1], None)
