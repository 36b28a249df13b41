"""CPU oracles of the cache-semantic hash table (arxiv 2603.17168).

TEST INFRASTRUCTURE ONLY: imported by the tests, the GPU smoke check and the benchmark's
CPU-baseline leg.  The product path (the HIP library and its binding) never imports it.

``Oracle`` wraps the sequential C oracle (``cskv_oracle.c``, built into ``libcskv_oracle.so``
by ``oracle/build.py``) with numpy arrays; ``pyoracle.PyTable`` is the literal Python version
for tiny cases.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcskv_oracle.so")

SINGLE, DUAL = 1, 2
CUSTOM, LRU, LFU = 0, 1, 2
UPDATED, INSERTED, INSERTED_EVICT, REJECTED, INVALID_KEY = 1, 2, 3, 4, 5

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    U64 = ctypes.c_uint64
    lib.ora_create.restype = P
    lib.ora_create.argtypes = [U64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
    lib.ora_destroy.argtypes = [P]
    lib.ora_clone.restype = P
    lib.ora_clone.argtypes = [P]
    lib.ora_clock.restype = U64
    lib.ora_clock.argtypes = [P]
    lib.ora_size.restype = U64
    lib.ora_size.argtypes = [P]
    lib.ora_bucket_count.restype = ctypes.c_uint32
    lib.ora_bucket_count.argtypes = [P, U64]
    lib.ora_fmix64.restype = U64
    lib.ora_fmix64.argtypes = [U64]
    lib.ora_b1.restype = U64
    lib.ora_b1.argtypes = [P, U64]
    lib.ora_b2.restype = U64
    lib.ora_b2.argtypes = [P, U64]
    lib.ora_find.argtypes = [P, U64, P, P, P, P]
    lib.ora_upsert.restype = ctypes.c_long
    lib.ora_upsert.argtypes = [P, U64, P, P, P, P, P, P, P]
    lib.ora_erase.argtypes = [P, U64, P, P]
    lib.ora_export.restype = U64
    lib.ora_export.argtypes = [P, U64, U64, P, P, P, P]
    lib.ora_contains.argtypes = [P, U64, P, P]
    lib.ora_locate.argtypes = [P, U64, P, P, P]
    lib.ora_assign.restype = ctypes.c_long
    lib.ora_assign.argtypes = [P, U64, P, P, P, P]
    lib.ora_find_or_insert.restype = ctypes.c_long
    lib.ora_find_or_insert.argtypes = [P, U64, P, P, P, P, P]
    lib.ora_export_if.restype = U64
    lib.ora_export_if.argtypes = [P, U64, U64, U64, P, P, P, P]
    lib.ora_stats.argtypes = [P, P]
    lib.ora_set_subrounds.restype = ctypes.c_int
    lib.ora_set_subrounds.argtypes = [P, ctypes.c_uint32]
    lib.ora_reset_stats.argtypes = [P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def fmix64(k: int) -> int:
    return int(_load().ora_fmix64(int(k)))


class Oracle:
    """Sequential C oracle.  Keys/scores/value-ids are numpy uint64 arrays."""

    def __init__(self, n_buckets: int, bucket_size: int = 128, mode: int = DUAL, policy: int = CUSTOM):
        self.lib = _load()
        self.h = self.lib.ora_create(n_buckets, bucket_size, mode, policy)
        if not self.h:
            raise ValueError("invalid oracle table arguments")
        self.B, self.S, self.mode, self.policy = n_buckets, bucket_size, mode, policy

    def clone(self) -> "Oracle":
        """An independent copy of the whole table state."""
        c = Oracle.__new__(Oracle)
        c.lib = self.lib
        c.h = self.lib.ora_clone(self.h)
        if not c.h:
            raise MemoryError("oracle clone failed")
        c.B, c.S, c.mode, c.policy = self.B, self.S, self.mode, self.policy
        return c

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.ora_destroy(self.h)
            self.h = None

    @property
    def clock(self) -> int:
        return int(self.lib.ora_clock(self.h))

    def size(self) -> int:
        return int(self.lib.ora_size(self.h))

    def bucket_count(self, b: int) -> int:
        return int(self.lib.ora_bucket_count(self.h, b))

    def candidates(self, key: int):
        return int(self.lib.ora_b1(self.h, int(key))), int(self.lib.ora_b2(self.h, int(key)))

    def find(self, keys):
        keys = _u64(keys)
        n = keys.size
        found = np.zeros(n, dtype=np.uint8)
        vids = np.zeros(n, dtype=np.uint64)
        scores = np.zeros(n, dtype=np.uint64)
        self.lib.ora_find(self.h, n, _p(keys), _p(found), _p(vids), _p(scores))
        return found, vids, scores

    def upsert(self, keys, vids, scores=None):
        """insert_or_assign / insert_and_evict.  Returns (status u8[n], ev_keys, ev_vids, ev_scores)."""
        keys = _u64(keys)
        vids = _u64(vids)
        n = keys.size
        sc = None if scores is None else _u64(scores)
        status = np.zeros(n, dtype=np.uint8)
        ek = np.zeros(max(n, 1), dtype=np.uint64)
        ev = np.zeros(max(n, 1), dtype=np.uint64)
        es = np.zeros(max(n, 1), dtype=np.uint64)
        r = self.lib.ora_upsert(self.h, n, _p(keys), _p(vids), _p(sc), _p(status), _p(ek), _p(ev), _p(es))
        if r < 0:
            raise ValueError("oracle upsert rejected its arguments")
        return status, ek[:r].copy(), ev[:r].copy(), es[:r].copy()

    def erase(self, keys):
        keys = _u64(keys)
        erased = np.zeros(keys.size, dtype=np.uint8)
        self.lib.ora_erase(self.h, keys.size, _p(keys), _p(erased))
        return erased

    def export(self, b0: int = 0, b1: int | None = None):
        """(keys, vids, scores, buckets) of all entries in buckets [b0, b1)."""
        b1 = self.B if b1 is None else b1
        cap = max(1, (b1 - b0) * self.S)
        k = np.zeros(cap, dtype=np.uint64)
        v = np.zeros(cap, dtype=np.uint64)
        s = np.zeros(cap, dtype=np.uint64)
        b = np.zeros(cap, dtype=np.uint64)
        c = int(self.lib.ora_export(self.h, b0, b1, _p(k), _p(v), _p(s), _p(b)))
        return k[:c], v[:c], s[:c], b[:c]

    def contains(self, keys):
        keys = _u64(keys)
        found = np.zeros(keys.size, dtype=np.uint8)
        self.lib.ora_contains(self.h, keys.size, _p(keys), _p(found))
        return found

    def locate(self, keys):
        """(found u8[n], bucket u64[n]) - the bucket of each resident key (0 where absent)."""
        keys = _u64(keys)
        found = np.zeros(keys.size, dtype=np.uint8)
        buckets = np.zeros(keys.size, dtype=np.uint64)
        self.lib.ora_locate(self.h, keys.size, _p(keys), _p(found), _p(buckets))
        return found, buckets

    def assign(self, keys, vids=None, scores=None):
        """assign (vids given) or assign_scores (vids None); returns found u8[n]."""
        keys = _u64(keys)
        v = None if vids is None else _u64(vids)
        sc = None if scores is None else _u64(scores)
        found = np.zeros(keys.size, dtype=np.uint8)
        if self.lib.ora_assign(self.h, keys.size, _p(keys), _p(v), _p(sc), _p(found)) < 0:
            raise ValueError("oracle assign rejected its arguments")
        return found

    def find_or_insert(self, keys, vids, scores=None):
        """Returns (status u8[n], out_vids u64[n])."""
        keys = _u64(keys)
        vids = _u64(vids)
        sc = None if scores is None else _u64(scores)
        status = np.zeros(keys.size, dtype=np.uint8)
        out = np.zeros(keys.size, dtype=np.uint64)
        if self.lib.ora_find_or_insert(self.h, keys.size, _p(keys), _p(vids), _p(sc), _p(status), _p(out)) < 0:
            raise ValueError("oracle find_or_insert rejected its arguments")
        return status, out

    def export_if(self, min_score: int, b0: int = 0, b1: int | None = None):
        """(keys, vids, scores, buckets) of the entries in buckets [b0, b1) with score >= min_score."""
        b1 = self.B if b1 is None else b1
        cap = max(1, (b1 - b0) * self.S)
        k = np.zeros(cap, dtype=np.uint64)
        v = np.zeros(cap, dtype=np.uint64)
        s = np.zeros(cap, dtype=np.uint64)
        b = np.zeros(cap, dtype=np.uint64)
        c = int(self.lib.ora_export_if(self.h, b0, b1, int(min_score), _p(k), _p(v), _p(s), _p(b)))
        return k[:c], v[:c], s[:c], b[:c]

    def set_subrounds(self, r: int):
        """Route sub-rounds per upsert call (1..64; 1 = the whole batch routes at once)."""
        if self.lib.ora_set_subrounds(self.h, int(r)) != 0:
            raise ValueError("subrounds must be 1..64")

    def stats(self):
        out = np.zeros(9, dtype=np.uint64)
        self.lib.ora_stats(self.h, _p(out))
        names = ["hit1", "hit2", "miss", "upd", "ins", "evict", "rej", "invalid", "d2_routes"]
        return dict(zip(names, (int(x) for x in out)))

    def reset_stats(self):
        self.lib.ora_reset_stats(self.h)
