"""Oracle parity on the largest table the library accepts: 2^24 buckets of 128 slots (2^31 slots,
dim 4, 71 GB of HBM), so that slot indices reach 2^31 - 1 and row offsets pass 2^31 elements.
The first and last buckets are filled past capacity through both of their candidate roles
(evictions and refusals), random keys land all over the table, and every call is compared with
the oracle, then the whole table (exported, with rows through value-ids)."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd.workload import as_u64, keys as gen_keys, uniform_u64
from tests.hashkeys import keys_for
from tests.parity import Twin

pytestmark = pytest.mark.gpu

NB = 1 << 24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge_keys(count: int, digest: int) -> np.ndarray:
    """Keys whose candidate buckets are the table's last two, its first and last, and its
    second-last and first (both choices at the ends of the index range)."""
    pairs = [(NB - 1, NB - 2), (0, NB - 1), (NB - 2, 0)]
    ks = []
    for b1, b2 in pairs:
        ks += keys_for(b1, b2, NB, count, salt0=1, digest=digest)
    return np.array(ks, dtype=np.uint64)


def test_largest_table():
    say("largest table: 2^24 buckets, dim 4")
    tw = Twin(NB * 128, 4, "dual", "custom", seed=83)
    first = edge_keys(100, 0x5A)  # 300 keys into the three buckets at the ends (384 slots)
    tw.upsert(first, np.arange(1000, 1000 + first.size, dtype=np.uint64), evict=True)
    rnd = as_u64(gen_keys(310, 1 << 20))
    tw.upsert(rnd, (as_u64(uniform_u64(311, rnd.size)) >> np.uint64(44)) + np.uint64(1))
    say("  filled: edge keys and 2^20 random keys")
    # the end buckets overflow: higher scores evict the smallest residents, lower ones are refused
    more = edge_keys(100, 0x3C)
    sc = np.where(np.arange(more.size) % 2 == 0, 5000 + np.arange(more.size), 1 + np.arange(more.size) % 7)
    st = tw.upsert(more, sc.astype(np.uint64), evict=True)
    assert (st == 3).sum() > 0, "no eviction in the end buckets"
    misses = as_u64(gen_keys(312, 1 << 16))
    tw.find(np.concatenate([first, more, rnd[: 1 << 18], misses]))
    tw.erase(np.concatenate([first[::3], rnd[::5]]))
    tw.find(np.concatenate([first, more, rnd[: 1 << 16]]))
    say("  calls equal; whole-table export")
    tw.check_table()
    say("  table equal")
    del tw
    torch.cuda.empty_cache()
