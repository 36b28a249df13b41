"""The C oracle and the literal Python oracle, written independently, agree on random tiny runs."""
import random

import numpy as np
import pytest

import oracle
from oracle import pyoracle

M64 = (1 << 64) - 1


def _c_state(o):
    k, v, s, b = o.export()
    out = {}
    for kk, vv, ss, bb in zip(k.tolist(), v.tolist(), s.tolist(), b.tolist()):
        out.setdefault(int(bb), []).append((int(kk), int(ss), int(vv)))
    return {b: sorted(x) for b, x in out.items()}


def _run(seed, B, S, mode, policy, n_batches=25, subrounds=1):
    rng = random.Random(seed)
    c = oracle.Oracle(B, S, mode, policy)
    p = pyoracle.PyTable(B, S, mode, policy)
    c.set_subrounds(subrounds)
    p.subrounds = subrounds
    universe = [rng.getrandbits(64) | 1 for _ in range(B * S * 2)]
    universe += [0, M64]  # reserved words show up as invalid keys
    vid = 0
    for step in range(n_batches):
        op = rng.random()
        n = rng.randint(0, 3 * S)
        keys = [rng.choice(universe) for _ in range(n)]
        if op < 0.6:
            vids = list(range(vid, vid + n))
            vid += n
            if policy == oracle.CUSTOM:
                scores = [rng.randint(0, 40) for _ in range(n)]
            elif policy == oracle.LFU:
                scores = [rng.choice([1, 1, 2, 5, M64]) for _ in range(n)] if rng.random() < 0.7 else None
            else:
                scores = None
            st_c, ek, ev, es = c.upsert(keys, vids, scores)
            st_p, evp = p.upsert(keys, vids, scores)
            assert st_c.tolist() == st_p, (seed, step)
            assert sorted(zip(ek.tolist(), es.tolist(), ev.tolist())) == sorted(evp)
        elif op < 0.68:
            vids = list(range(vid, vid + n))
            vid += n
            if policy == oracle.CUSTOM:
                scores = [rng.randint(0, 40) for _ in range(n)]
            elif policy == oracle.LFU:
                scores = [rng.choice([1, 2, M64]) for _ in range(n)] if rng.random() < 0.7 else None
            else:
                scores = None
            if rng.random() < 0.5:
                st_c, out_c = c.find_or_insert(keys, vids, scores)
                st_p, out_p = p.find_or_insert(keys, vids, scores)
                assert st_c.tolist() == st_p, (seed, step)
                assert [int(x) for x, k in zip(out_c, keys) if k not in (0, M64)] == [x for x in out_p if x is not None]
            else:
                with_values = rng.random() < 0.5
                f_c = c.assign(keys, vids if with_values else None, scores)
                f_p = p.assign(keys, vids if with_values else None, scores)
                assert f_c.tolist() == [int(x) for x in f_p]
        elif op < 0.8:
            er_c = c.erase(keys)
            er_p = p.erase(keys)
            assert er_c.tolist() == [int(x) for x in er_p]
        elif op < 0.85:
            assert c.contains(keys).tolist() == [int(x) for x in p.contains(keys)]
            fb, bk = c.locate(keys)
            for i, r in enumerate(p.locate(keys)):
                assert fb[i] == (r is not None) and (r is None or int(bk[i]) == r)
            thr = rng.randint(0, 40)
            kk, vv, ss, bb = c.export_if(thr)
            got = {}
            for a_, b_, c_, d_ in zip(kk.tolist(), ss.tolist(), vv.tolist(), bb.tolist()):
                got.setdefault(int(d_), []).append((int(a_), int(b_), int(c_)))
            assert {b: sorted(x) for b, x in got.items()} == p.export_if(thr)
        else:
            f, v, s = c.find(keys)
            fp = p.find(keys)
            for i, r in enumerate(fp):
                assert f[i] == (r is not None)
                if r is not None:
                    assert (int(s[i]), int(v[i])) == r
        assert _c_state(c) == p.export()
        assert c.size() == p.size()
        assert c.clock == p.clock


@pytest.mark.parametrize("mode", [oracle.SINGLE, oracle.DUAL])
@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
@pytest.mark.parametrize("shape", [(1, 4), (2, 4), (4, 8), (8, 16)])
def test_c_and_python_oracles_agree(mode, policy, shape):
    B, S = shape
    for seed in range(6):
        _run(1000 * seed + 17 * B + S + 5 * policy + mode, B, S, mode, policy)


@pytest.mark.parametrize("subrounds", [2, 3, 64])
@pytest.mark.parametrize("policy", [oracle.CUSTOM, oracle.LRU, oracle.LFU])
def test_c_and_python_oracles_agree_with_subrounds(policy, subrounds):
    for seed in range(4):
        for B, S in [(2, 4), (4, 8)]:
            _run(7000 * seed + 31 * subrounds + 5 * policy + B, B, S, oracle.DUAL, policy, subrounds=subrounds)


def test_lfu_saturates():
    c = oracle.Oracle(1, 4, oracle.SINGLE, oracle.LFU)
    p = pyoracle.PyTable(1, 4, oracle.SINGLE, oracle.LFU)
    keys = [5, 5, 5]
    sc = [M64 - 1, 1, 7]
    assert c.upsert(keys, [1, 2, 3], sc)[0].tolist() == p.upsert(keys, [1, 2, 3], sc)[0]
    f, v, s = c.find([5])
    assert int(s[0]) == M64 and int(v[0]) == 3
    assert p.find([5])[0] == (M64, 3)
    c.upsert([5], [4], [9])
    assert int(c.find([5])[2][0]) == M64
