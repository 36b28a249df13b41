"""GPU parity of the rest of the API (Sec. 3.5's role list, Sec. 4.1): contains, find_ptr,
assign, assign_scores, find_or_insert and export_if, through the C-ABI, against the oracle bit
for bit, mixed with the upsert / erase / find calls on small tables that fill, overflow and
drain (whole-table parity after every call)."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, keys as gen_keys
from tests.hashkeys import key_for
from tests.parity import Twin

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_keys(stream, n, start=0):
    return as_u64(gen_keys(stream, n, start))


def _scores(rng, policy, n):
    if policy == "custom":
        return rng.integers(0, 50, n).astype(np.uint64)
    if policy == "lfu":
        return rng.choice(np.array([1, 1, 2, 7, M64], dtype=np.uint64), n) if rng.random() < 0.7 else None
    return None


@pytest.mark.parametrize("mode", ["single", "dual"])
@pytest.mark.parametrize("policy", ["custom", "lru", "lfu"])
def test_api_random_mixed(mode, policy):
    say(f"api mixed: mode {mode} policy {policy}")
    for seed, nb in [(1, 4), (2, 16), (3, 64)]:
        rng = np.random.default_rng(seed * 1000 + len(mode) + 7 * len(policy))
        tw = Twin(nb * 128, 16, mode, policy, seed=seed)
        universe = np.concatenate([np_keys(30 + seed, nb * 128 * 3), np.array([0, M64], dtype=np.uint64)])
        for step in range(30):
            n = int(rng.integers(0, nb * 128))
            k = rng.choice(universe, n)
            r = rng.random()
            if r < 0.3:
                tw.upsert(k, _scores(rng, policy, n), evict=bool(rng.random() < 0.5))
            elif r < 0.5:
                tw.find_or_insert(k, _scores(rng, policy, n))
            elif r < 0.65:
                tw.assign(k, _scores(rng, policy, n), with_values=bool(rng.random() < 0.5))
            elif r < 0.75:
                tw.erase(k)
            elif r < 0.85:
                tw.contains(k)
            elif r < 0.95:
                tw.find_ptr(k)
            else:
                tw.export_if(int(rng.integers(0, 60)) if policy != "lru" else tw.ora.clock)
            tw.check_table()


def test_find_or_insert_floods_one_bucket():
    """Hundreds of keys (half of them resident, with duplicates) aimed at one bucket: the slow
    path keeps resident rows, returns them, and returns every rejected key's own row."""
    nb = 8
    for m, seed in [(60, 1), (300, 2)]:
        say(f"find_or_insert flood: {m} keys into bucket 5")
        tw = Twin(nb * 128, 8, "dual", "custom", seed=seed)
        rng = np.random.default_rng(seed)
        k = np.array([key_for(5, 5, nb, salt=1 + i) for i in range(m)], dtype=np.uint64)
        tw.upsert(k[: m // 2], rng.integers(0, 30, m // 2).astype(np.uint64))
        tw.check_table()
        q = np.concatenate([k, k[: m // 3], k[m // 2: m // 2 + 10]])
        tw.find_or_insert(q, rng.integers(0, 60, q.size).astype(np.uint64))
        tw.check_table()


def test_assign_keeps_structure_and_voids_cached_minima():
    """assign on a full table changes no key and no bucket; lowering a bucket's minimum with
    assign_scores (custom policy) must be seen by the next routing in phase D2."""
    nb = 16
    say("assign on a full table")
    tw = Twin(nb * 128, 8, "dual", "custom", seed=4)
    rng = np.random.default_rng(4)
    k = np_keys(40, nb * 128 * 2)
    tw.upsert(k, rng.integers(100, 200, k.size).astype(np.uint64))
    tw.check_table()
    res = tw.ora.export()[0]
    tw.assign(res[: res.size // 2], rng.integers(0, 5, res.size // 2).astype(np.uint64), with_values=False)
    tw.check_table()
    tw.assign(res, rng.integers(0, 300, res.size).astype(np.uint64), with_values=True)
    tw.check_table()
    tw.upsert(np_keys(41, nb * 128), rng.integers(50, 250, nb * 128).astype(np.uint64), evict=True)
    tw.check_table()


def test_api_errors_and_empty_calls():
    t = cskv.Table(128 * 4, 8, "dual", "custom")
    k = torch.tensor([5, 6], dtype=torch.int64, device="cuda")
    v = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(cskv.CskvError):
        t.assign(k, v)  # custom policy needs scores
    with pytest.raises(cskv.CskvError):
        t.find_or_insert(k, v)  # custom policy needs scores
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert t.contains(e).numel() == 0
    t.assign_scores(e, e)
    out, st = t.find_or_insert(e, torch.empty((0, 8), dtype=torch.float32, device="cuda"), e)
    assert out.numel() == 0 and st.numel() == 0
    torch.cuda.synchronize()
