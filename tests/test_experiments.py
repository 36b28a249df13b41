"""The eviction-quality protocols (Exp. 3c, 3d, 4) on the oracle (CPU: the protocols show what
the paper's mechanisms imply) and on the GPU table (gpu: every metric equals the oracle's)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2603_17168_amd import experiments as ex
from paper_2603_17168_amd.workload import as_u64, keys as gen_keys

CAP = 1 << 14  # 128 buckets of 128 slots
BATCH = CAP // 128  # the paper's ratio: 1 M keys per call into 128 M slots


class OracleTable:
    """The experiment interface over the sequential oracle (value-ids all zero)."""

    def __init__(self, capacity, mode, policy):
        self.o = oracle.Oracle(capacity // 128, 128, {"single": oracle.SINGLE, "dual": oracle.DUAL}[mode],
                               {"custom": oracle.CUSTOM, "lru": oracle.LRU, "lfu": oracle.LFU}[policy])

    def upsert(self, keys, scores=None):
        k = as_u64(keys)
        st = self.o.upsert(k, np.zeros(k.size, dtype=np.uint64), None if scores is None else as_u64(scores))[0]
        return torch.from_numpy(st)

    def find(self, keys):
        return torch.from_numpy(self.o.contains(as_u64(keys)))

    def size(self):
        return self.o.size()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_first_eviction_dual_fills_further():
    """Dual-bucket placement (Sec. 3.4, phase D1) defers the first eviction from the birthday
    bound of one candidate bucket to nearly full (Exp. 4)."""
    single = ex.first_eviction(OracleTable(CAP, "single", "custom"), CAP, BATCH)
    dual = ex.first_eviction(OracleTable(CAP, "dual", "custom"), CAP, BATCH)
    assert 0.5 < single < 0.9 < dual < 1.0


def test_first_eviction_single_is_the_first_overfull_bucket():
    """Single mode: the first eviction comes with the first key whose bucket already holds 128
    keys; the protocol reports the load before the batch holding that key."""
    keys = as_u64(gen_keys(61, 2 * CAP))
    o = oracle.Oracle(CAP // 128, 128, oracle.SINGLE, oracle.CUSTOM)
    count = np.zeros(CAP // 128, dtype=np.int64)
    for i, k in enumerate(keys):
        b = o.candidates(int(k))[0]
        if count[b] == 128:
            break
        count[b] += 1
    batch = 16
    assert ex.first_eviction(OracleTable(CAP, "single", "custom"), CAP, batch) == (i // batch) * batch / CAP


def test_zipf_ingestion_policies():
    """At load 1.0 under Zipf ingestion (Exp. 3c): the hit ratio rises with the skew; CUSTOM with
    recency scores equals LRU exactly (the same order of entries); LFU stays at or below the
    static optimum, the probability mass of the C most popular ranks."""
    r = {}
    for pol in ("lru", "lfu", "custom"):
        for a in (0.5, 0.99, 1.25):
            r[pol, a] = ex.zipf_ingestion(OracleTable(CAP, "single", pol), CAP, a, pol, BATCH)
            assert r[pol, a]["load_filled"] == 1.0 and r[pol, a]["load"] == 1.0
    for pol in ("lru", "lfu"):
        assert r[pol, 0.5]["hit_ratio"] < r[pol, 0.99]["hit_ratio"] < r[pol, 1.25]["hit_ratio"]
    for a in (0.5, 0.99, 1.25):
        assert r["custom", a] == r["lru", a]
        k = np.arange(1, ex.UNIVERSE_FACTOR * CAP + 1, dtype=np.float64) ** -a
        assert 0.0 < r["lfu", a]["hit_ratio"] <= k[:CAP].sum() / k.sum() + 0.01


def test_dual_bucket_raises_top_n_retention():
    """Score-based bucket choice (phase D2) keeps more of the highest-scored keys than one
    candidate bucket (Exp. 4)."""
    s = ex.zipf_ingestion(OracleTable(CAP, "single", "lru"), CAP, 0.99, "lru", BATCH, retention=True)
    d = ex.zipf_ingestion(OracleTable(CAP, "dual", "lru"), CAP, 0.99, "lru", BATCH, retention=True)
    assert 0.8 < s["top_n_retention"] < d["top_n_retention"] <= 1.0
    assert d["top_n_retention"] > 0.97


def test_admission_burst_depends_on_increment():
    """A burst of fresh keys with a unit increment into a warmed LFU table displaces nobody (the
    admission gate of Alg. 2 rejects ties with the bucket minimum); with a huge increment every
    key is admitted and the hit ratio falls (Exp. 3d)."""
    low = ex.admission_burst(OracleTable(CAP, "dual", "lfu"), CAP, 1, BATCH)
    high = ex.admission_burst(OracleTable(CAP, "dual", "lfu"), CAP, 10 ** 9, BATCH)
    assert low["load_before"] >= 0.96 and low["load_before"] == high["load_before"]
    assert low["hit_before"] == high["hit_before"]
    assert low["evicting_admissions"] == 0.0 and low["hit_after"] == low["hit_before"]
    assert low["free_slot_inserts"] + low["rejected"] == 1.0
    assert high["rejected"] == 0.0
    assert high["hit_after"] < high["hit_before"]


@pytest.mark.gpu
def test_experiments_gpu_equal_oracle():
    """The protocols on the GPU table give the oracle's metrics exactly (inputs generated on the
    CPU for both; the table is bit-exact with the oracle, so every status, hit and size agrees)."""
    for mode in ("single", "dual"):
        say(f"first_eviction {mode}")
        assert ex.first_eviction(ex.GpuTable(CAP, mode, "custom"), CAP, BATCH) == \
            ex.first_eviction(OracleTable(CAP, mode, "custom"), CAP, BATCH)
    for mode, pol, a, ret in [("dual", "lru", 0.99, True), ("single", "lru", 0.99, True),
                              ("single", "lfu", 0.75, False), ("single", "custom", 1.25, False)]:
        say(f"zipf_ingestion {mode} {pol} {a}")
        g = ex.zipf_ingestion(ex.GpuTable(CAP, mode, pol), CAP, a, pol, BATCH, capacities=2, retention=ret)
        o = ex.zipf_ingestion(OracleTable(CAP, mode, pol), CAP, a, pol, BATCH, capacities=2, retention=ret)
        assert g == o
    for inc in (1, 10 ** 9):
        say(f"admission_burst {inc}")
        assert ex.admission_burst(ex.GpuTable(CAP, "dual", "lfu"), CAP, inc, BATCH) == \
            ex.admission_burst(OracleTable(CAP, "dual", "lfu"), CAP, inc, BATCH)
