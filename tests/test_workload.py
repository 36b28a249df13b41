"""The seeded generators follow their stated distributions (CPU)."""
import math

import numpy as np

from paper_2603_17168_amd.workload import (Zipf, batch_schedule, keys, lognormal_sizes, poisson_arrivals,
                                            value_rows)


def test_keys_distinct_and_valid():
    k = keys(3, 200000).numpy().view(np.uint64)
    assert np.unique(k).size == k.size
    assert not np.isin(k, np.array([0, 2 ** 64 - 1], dtype=np.uint64)).any()
    k2 = keys(4, 200000).numpy().view(np.uint64)
    assert np.intersect1d(k, k2).size == 0


def test_value_rows_exact_and_bounded():
    r = value_rows(1, keys(1, 1000), 32).numpy()
    assert (r >= -1).all() and (r < 1).all()
    # every element is a multiple of 2**-23 (exactly representable)
    assert np.all(np.round(r.astype(np.float64) * 2 ** 23) == r.astype(np.float64) * 2 ** 23)


def test_zipf_rank_frequencies():
    a, N = 1.1, 1 << 34
    z = Zipf(a, N).sample(9, 400000)
    norm = sum(k ** -a for k in range(1, 200001)) + ((N + 0.5) ** (1 - a) - 200000.5 ** (1 - a)) / (1 - a)
    for r in range(1, 6):
        p = r ** -a / norm
        f = np.mean(z == r)
        assert abs(f - p) < 5 * math.sqrt(p * (1 - p) / z.size)


def test_sizes_and_arrivals():
    s = lognormal_sizes(1, 100000, 4096.0, 1.0, 256, 65536)
    assert s.min() >= 256 and s.max() <= 65536
    assert abs(np.median(s) / 4096.0 - 1) < 0.03
    t = poisson_arrivals(2, 100000, 1000.0)
    gaps = np.diff(t)
    assert abs(gaps.mean() * 1000.0 - 1) < 0.02 and abs(gaps.std() / gaps.mean() - 1) < 0.03


def test_batch_schedule_mix():
    sch = batch_schedule(5, 20000, 1 << 10, 1 << 20)
    ops = np.array([o for o, _ in sch])
    sizes = np.array([n for _, n in sch])
    assert abs(np.mean(ops == "find") - 0.70) < 0.02 and abs(np.mean(ops == "erase") - 0.05) < 0.01
    assert sizes.min() >= 1 << 10 and sizes.max() <= 1 << 20
    lg = np.log(sizes)
    assert abs(lg.mean() - (math.log(1 << 10) + math.log(1 << 20)) / 2) < 0.1
