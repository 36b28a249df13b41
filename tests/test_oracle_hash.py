"""Pins of the oracle's bucket hash (MurmurHash3 fmix64 reading of Sec. 3.1/3.2)."""
import random

import numpy as np

import oracle
from oracle import pyoracle
from tests.hashkeys import fmix64_inverse, key_for


def test_fmix64_zero_is_fixed_point():
    # xor-shifts and multiplications all map 0 to 0
    assert oracle.fmix64(0) == 0


def test_fmix64_round_trips_through_independent_inverse():
    rng = random.Random(7)
    for _ in range(2000):
        x = rng.getrandbits(64)
        assert fmix64_inverse(oracle.fmix64(x)) == x
        assert oracle.fmix64(fmix64_inverse(x)) == x


def test_python_and_c_oracles_hash_alike():
    rng = random.Random(11)
    for _ in range(500):
        x = rng.getrandbits(64)
        assert pyoracle.fmix64(x) == oracle.fmix64(x)


def test_fmix64_avalanche():
    # a finalizer meant for hashing flips about half of the output bits per input bit
    rng = random.Random(3)
    flips = []
    for _ in range(300):
        x = rng.getrandbits(64)
        hx = oracle.fmix64(x)
        for b in range(64):
            flips.append(bin(hx ^ oracle.fmix64(x ^ (1 << b))).count("1"))
    assert abs(np.mean(flips) - 32.0) < 0.5


def test_candidate_buckets_follow_bit_fields():
    B = 1 << 10
    o = oracle.Oracle(B, 8, oracle.DUAL, oracle.CUSTOM)
    rng = random.Random(5)
    for _ in range(200):
        b1, b2 = rng.randrange(B), rng.randrange(B)
        k = key_for(b1, b2, B, salt=rng.getrandbits(20))
        assert o.candidates(k) == (b1, b2)
    s = oracle.Oracle(B, 8, oracle.SINGLE, oracle.CUSTOM)
    k = key_for(3, 9, B, salt=1)
    assert s.candidates(k) == (3, 3)


def test_bucket_distribution_uniform():
    # chi-square of b1 over sequential keys: fmix64 spreads even consecutive integers
    B = 256
    o = oracle.Oracle(B, 8, oracle.DUAL, oracle.CUSTOM)
    n = 256 * 200
    counts = np.zeros(B)
    counts2 = np.zeros(B)
    for k in range(1, n + 1):
        b1, b2 = o.candidates(k)
        counts[b1] += 1
        counts2[b2] += 1
    exp = n / B
    for c in (counts, counts2):
        chi2 = ((c - exp) ** 2 / exp).sum()
        # 255 dof: mean 255, sd ~22.6; 6 sd margin
        assert chi2 < 255 + 6 * 22.6
