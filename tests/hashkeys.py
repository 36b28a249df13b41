"""Test-side helpers: construct keys that land in chosen buckets with chosen digests.

The bucket hash is MurmurHash3's 64-bit finalizer, a bijection on 64-bit words.  Its inverse
is written here from its structure (two odd multipliers, invertible mod 2**64, and xor-shifts
by 33 >= 32, each its own inverse), not from the oracle, so a round trip through the oracle's
hash pins the oracle's constants and shifts.
"""
from __future__ import annotations

M64 = (1 << 64) - 1
C1 = 0xFF51AFD7ED558CCD
C2 = 0xC4CEB9FE1A85EC53
C1_INV = pow(C1, -1, 1 << 64)
C2_INV = pow(C2, -1, 1 << 64)


def _xs33(x: int) -> int:
    return x ^ (x >> 33)


def fmix64_inverse(h: int) -> int:
    x = _xs33(h & M64)
    x = (x * C2_INV) & M64
    x = _xs33(x)
    x = (x * C1_INV) & M64
    return _xs33(x)


def hash_word(b1: int, b2: int, digest: int, salt: int, n_buckets: int) -> int:
    """A 64-bit hash value whose low bits give b1, bits 32..39 the digest, bits 40.. give b2."""
    assert n_buckets & (n_buckets - 1) == 0 and n_buckets <= (1 << 24)
    lb = n_buckets.bit_length() - 1
    assert lb <= 24
    # low lb bits = b1; bits [lb, 32) free -> salt; bits 32..39 digest; bits 40.. = b2 + salt hi
    h = b1 & (n_buckets - 1)
    h |= (salt & ((1 << (32 - lb)) - 1)) << lb
    h |= (digest & 0xFF) << 32
    hi = (b2 & (n_buckets - 1)) | ((salt >> (32 - lb)) << lb)
    h |= (hi & ((1 << 24) - 1)) << 40
    return h & M64


def key_for(b1: int, b2: int, n_buckets: int, salt: int, digest: int = 0x5A) -> int:
    """A user key whose candidate buckets are (b1, b2) (dual mode; single mode uses b1)."""
    while True:
        k = fmix64_inverse(hash_word(b1, b2, digest, salt, n_buckets))
        if k not in (0, M64):
            return k
        salt += 1 << 20


def keys_for(b1: int, b2: int, n_buckets: int, count: int, salt0: int = 1, digest: int = 0x5A):
    return [key_for(b1, b2, n_buckets, salt0 + i, digest) for i in range(count)]
