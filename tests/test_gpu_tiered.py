"""GPU parity of tiered value storage (Sec. 3.6 key-value separation, Sec. 4.2 HBM watermark):
value rows past hbm_value_rows live in pinned host memory reached through its device alias.
Every call must give the oracle's results bit for bit whatever the split (no rows in HBM, a
split inside a bucket, half the buckets), and find_ptr must address the right row in each
region."""
import sys

import numpy as np
import pytest

from paper_2603_17168_amd.workload import as_u64, keys as gen_keys
from tests.parity import Twin

pytestmark = pytest.mark.gpu
M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_keys(stream, n, start=0):
    return as_u64(gen_keys(stream, n, start))


@pytest.mark.parametrize("split", ["none_in_hbm", "inside_a_bucket", "half"])
@pytest.mark.parametrize("mode,policy", [("dual", "custom"), ("single", "lru"), ("dual", "lfu")])
def test_tiered_mixed_calls(split, mode, policy):
    nb = 32
    cap = nb * 128
    hbm = {"none_in_hbm": 0, "inside_a_bucket": 1000, "half": cap // 2}[split]
    say(f"tiered: {split} ({hbm} rows in HBM), {mode} {policy}")
    tw = Twin(cap, 16, mode, policy, seed=3, hbm_value_rows=hbm)
    assert tw.gpu.hbm_value_rows == hbm and tw.gpu.host_values is not None
    rng = np.random.default_rng(hbm + len(mode) + len(policy))
    universe = np.concatenate([np_keys(60, cap * 3), np.array([0, M64], dtype=np.uint64)])

    def scores(n):
        if policy == "custom":
            return rng.integers(0, 50, n).astype(np.uint64)
        if policy == "lfu":
            return rng.integers(1, 4, n).astype(np.uint64)
        return None

    for step in range(24):
        n = int(rng.integers(1, cap))
        k = rng.choice(universe, n)
        r = step % 6
        if r == 0:
            tw.upsert(k, scores(n), evict=bool(step % 12 == 0))
        elif r == 1:
            tw.find(k)
        elif r == 2:
            tw.find_or_insert(k, scores(n))
        elif r == 3:
            tw.assign(k, scores(n), with_values=True)
        elif r == 4:
            tw.find_ptr(k)
        else:
            tw.erase(k[: n // 4])
        tw.check_table()
