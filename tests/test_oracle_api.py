"""Pins of the oracle's reader / updater / find_or_insert calls (the rest of the API named by
Sec. 3.5's role list and Sec. 4.1): a dictionary model below capacity, equivalences with the
pinned find / upsert / export, and at capacity the statement that find_or_insert is an upsert
that never overwrites a resident value."""
import random

import numpy as np
import pytest

import oracle
from oracle import pyoracle

M64 = (1 << 64) - 1


def _state(o):
    k, v, s, b = o.export()
    return sorted(zip(k.tolist(), s.tolist(), v.tolist(), b.tolist()))


@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
def test_api_below_capacity_is_a_dictionary(policy, mode):
    """No bucket ever fills: contains / assign / assign_scores / find_or_insert act on an
    ordinary map (last occurrence wins, LFU increments summed, LRU clock one tick per call)."""
    rng = random.Random(31 * policy + mode)
    o = oracle.Oracle(64, 128, mode, policy)
    universe = [rng.getrandbits(64) | 2 for _ in range(1200)]
    model = {}  # key -> [score, vid]
    clock, vid = 0, 0
    for _ in range(80):
        r = rng.random()
        n = rng.randint(0, 100)
        ks = [rng.choice(universe) for _ in range(n)]
        sc = [rng.randint(0, 500) for _ in range(n)] if policy != oracle.LRU else None
        vids = list(range(vid, vid + n))
        vid += n
        last = {k: i for i, k in enumerate(ks)}
        tot = {}
        for i, k in enumerate(ks):
            tot[k] = tot.get(k, 0) + (sc[i] if sc else 1)
        if n:
            clock += policy == oracle.LRU and r >= 0.15
        if r < 0.15:
            assert o.contains(ks).tolist() == [int(k in model) for k in ks]
            f, b = o.locate(ks)
            for i, k in enumerate(ks):
                assert f[i] == (k in model)
                if k in model:
                    assert int(b[i]) in o.candidates(k)
        elif r < 0.45:
            with_values = r < 0.3
            found = o.assign(ks, vids if with_values else None, sc)
            assert found.tolist() == [int(k in model) for k in ks]
            for k, i in last.items():
                if k not in model:
                    continue
                if policy == oracle.CUSTOM:
                    model[k][0] = sc[i]
                elif policy == oracle.LRU:
                    model[k][0] = clock
                else:
                    model[k][0] = model[k][0] + tot[k]
                if with_values:
                    model[k][1] = vids[i]
        else:
            st, out = o.find_or_insert(ks, vids, sc)
            before = {k: list(v) for k, v in model.items()}
            for k, i in last.items():
                if k in before:
                    if policy == oracle.CUSTOM:
                        model[k][0] = sc[i]
                    elif policy == oracle.LRU:
                        model[k][0] = clock
                    else:
                        model[k][0] = model[k][0] + tot[k]
                else:
                    s = sc[i] if policy == oracle.CUSTOM else clock if policy == oracle.LRU else tot[k]
                    model[k] = [s, vids[i]]
            for i, k in enumerate(ks):
                assert st[i] == (oracle.UPDATED if k in before else oracle.INSERTED)
                assert int(out[i]) == model[k][1]
        got = {k: [s, v] for k, s, v, _ in _state(o)}
        assert got == model
        assert o.clock == clock


@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
def test_find_or_insert_is_upsert_keeping_resident_values(policy):
    """At and beyond capacity (evictions, rejections): from equal tables, find_or_insert leaves
    the same keys, scores and statuses as insert_or_assign of the same batch; resident keys keep
    their value-ids instead of taking the batch's, and each occurrence returns its key's value-id
    from before the call if the key was resident, else the batch's (its last occurrence's)."""
    rng = random.Random(7 + policy)
    for trial in range(60):
        B, S = 4, 8
        a = oracle.Oracle(B, S, oracle.DUAL, policy)
        b = oracle.Oracle(B, S, oracle.DUAL, policy)
        universe = [rng.getrandbits(64) | 2 for _ in range(70)]
        for step in range(rng.randint(0, 5)):  # the same prefill on both
            n = rng.randint(1, 30)
            ks = [rng.choice(universe) for _ in range(n)]
            sc = [rng.randint(0, 30) for _ in range(n)] if policy != oracle.LRU else None
            a.upsert(ks, [100 * step + i for i in range(n)], sc)
            b.upsert(ks, [100 * step + i for i in range(n)], sc)
        assert _state(a) == _state(b)
        vid_before = {k: v for k, _, v, _ in _state(a)}
        n = rng.randint(1, 40)
        ks = [rng.choice(universe) for _ in range(n)]
        vids = [10_000 + i for i in range(n)]
        sc = [rng.randint(0, 30) for _ in range(n)] if policy != oracle.LRU else None
        st_b = b.upsert(ks, vids, sc)[0]
        st_a, out = a.find_or_insert(ks, vids, sc)
        assert st_a.tolist() == st_b.tolist()
        sa, sb = _state(a), _state(b)
        assert [(k, s, bb) for k, s, _, bb in sa] == [(k, s, bb) for k, s, _, bb in sb]
        va = {k: v for k, _, v, _ in sa}
        vb = {k: v for k, _, v, _ in sb}
        for k in va:
            assert va[k] == vid_before.get(k, vb[k])
        last = {k: i for i, k in enumerate(ks)}
        for i, k in enumerate(ks):
            assert int(out[i]) == (vid_before[k] if k in vid_before else vids[last[k]])
        assert a.clock == b.clock


def test_contains_equals_find_flags_and_export_if_filters_export():
    rng = random.Random(5)
    o = oracle.Oracle(16, 8, oracle.DUAL, oracle.CUSTOM)
    ks = [rng.getrandbits(64) | 2 for _ in range(300)]
    o.upsert(ks, list(range(300)), [rng.randint(0, 100) for _ in range(300)])
    q = ks[:150] + [rng.getrandbits(64) | 2 for _ in range(50)] + [0, M64]
    assert o.contains(q).tolist() == o.find(q)[0].tolist()
    k, v, s, b = o.export()
    for thr in (0, 1, 37, 100, 101, M64):
        kk, vv, ss, bb = o.export_if(thr)
        sel = s >= np.uint64(thr)
        assert sorted(zip(kk.tolist(), ss.tolist(), vv.tolist(), bb.tolist())) == \
            sorted(zip(k[sel].tolist(), s[sel].tolist(), v[sel].tolist(), b[sel].tolist()))


def test_api_reserved_words_and_empty_calls():
    o = oracle.Oracle(4, 8, oracle.DUAL, oracle.LRU)
    o.upsert([5, 6], [1, 2])
    c0 = o.clock
    assert o.contains([0, M64, 5]).tolist() == [0, 0, 1]
    assert o.assign([0, M64, 7], [9, 9, 9]).tolist() == [0, 0, 0]
    assert o.clock == c0 + 1
    assert o.assign([], None).tolist() == [] and o.clock == c0 + 1
    st, out = o.find_or_insert([0, 5, M64], [3, 4, 5])
    assert st.tolist() == [oracle.INVALID_KEY, oracle.UPDATED, oracle.INVALID_KEY]
    assert int(out[1]) == 1
