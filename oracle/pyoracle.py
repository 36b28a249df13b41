"""Literal pure-Python oracle of the cache-semantic hash table (arxiv 2603.17168), for tiny cases.

TEST INFRASTRUCTURE ONLY.  It is written independently of the C oracle (``cskv_oracle.c``) so
that the two cross-check each other; it shares nothing with the HIP library.

Each bucket is a dict ``key -> [score, value_id]``.  The steps follow the paper's algorithms:

* ``find``: Alg. 1 (digest-accelerated find) without the digest filter, which cannot change the
  answer: the key's bucket is searched, and in dual mode (Sec. 3.4) the second candidate too.
* ``upsert``: Alg. 2 (upsert with bucket-local admission and eviction) driven by Alg. 3 (score-based
  dual-bucket choice, phases D1 and D2), under the batch order described in ``cskv_oracle.c``:
  one operation per distinct key (last occurrence wins), routing against the table as it was
  before the batch, then per bucket the updates followed by the inserts in (score desc, key asc)
  order, admission strictly above the bucket's minimum, victim = smallest (score, key).
"""
from __future__ import annotations

EMPTY = 0
LOCKED = (1 << 64) - 1
M64 = (1 << 64) - 1

SINGLE, DUAL = 1, 2
CUSTOM, LRU, LFU = 0, 1, 2
UPDATED, INSERTED, INSERTED_EVICT, REJECTED, INVALID_KEY = 1, 2, 3, 4, 5


def fmix64(k: int) -> int:
    """MurmurHash3's 64-bit finalizer (Appleby)."""
    k &= M64
    k ^= k >> 33
    k = (k * 0xFF51AFD7ED558CCD) & M64
    k ^= k >> 33
    k = (k * 0xC4CEB9FE1A85EC53) & M64
    k ^= k >> 33
    return k


class PyTable:
    def __init__(self, n_buckets: int, bucket_size: int, mode: int = DUAL, policy: int = CUSTOM):
        assert n_buckets > 0 and n_buckets & (n_buckets - 1) == 0
        self.B = n_buckets
        self.S = bucket_size
        self.mode = mode
        self.policy = policy
        self.clock = 0
        self.subrounds = 1  # route sub-rounds per upsert call
        self.buckets = [dict() for _ in range(n_buckets)]

    # --- hashing (Sec. 3.2; second hash of Alg. 3) ---
    def candidates(self, k: int):
        h = fmix64(k)
        b1 = h % self.B
        b2 = (h >> 40) % self.B if self.mode == DUAL else b1
        return b1, b2

    def _where(self, k: int):
        b1, b2 = self.candidates(k)
        if k in self.buckets[b1]:
            return b1
        if k in self.buckets[b2]:
            return b2
        return None

    # --- Alg. 1 ---
    def find(self, keys):
        out = []
        for k in keys:
            if k in (EMPTY, LOCKED):
                out.append(None)
                continue
            b = self._where(k)
            out.append(None if b is None else tuple(self.buckets[b][k]))  # (score, vid)
        return out

    @staticmethod
    def _min_entry(bucket: dict):
        # smallest (score, key) of a full bucket
        return min((sv[0], k) for k, sv in bucket.items())

    # --- Alg. 3 driving Alg. 2, one batch ---
    def upsert(self, keys, vids, scores=None):
        """Returns (status list, evicted list of (key, score, vid))."""
        st, ev, _ = self._upsert(keys, vids, scores, keep_found=False)
        return st, ev

    def find_or_insert(self, keys, vids, scores=None):
        """insert_or_assign in which a resident key keeps its value (its score is updated).
        Returns (status list, value-id per occurrence: the key's value if it was resident before
        the call, else its last occurrence's value-id; None for reserved keys)."""
        st, _, out = self._upsert(keys, vids, scores, keep_found=True)
        return st, [None if k in (EMPTY, LOCKED) else out[k] for k in keys]

    def _upsert(self, keys, vids, scores, keep_found):
        n = len(keys)
        if n == 0:
            return [], [], {}
        if self.policy == LRU:
            self.clock += 1
        # one operation per distinct key
        last, inc, order = {}, {}, []
        for i, k in enumerate(keys):
            if k in (EMPTY, LOCKED):
                continue
            if k not in last:
                order.append(k)
                inc[k] = 0
            last[k] = i
            if self.policy == LFU:
                inc[k] = min(M64, inc[k] + (scores[i] if scores is not None else 1))
        s_new = {}
        for k in order:
            if self.policy == CUSTOM:
                s_new[k] = scores[last[k]]
            elif self.policy == LRU:
                s_new[k] = self.clock
            else:
                s_new[k] = inc[k]
        # sub-rounds: operations ordered by their key's last occurrence, rank q in chunk q*r//N;
        # each chunk routes against the table the chunks before it left
        by_last = sorted(order, key=lambda x: last[x])
        r = self.subrounds
        status, out = {}, {}
        evicted = []
        for c in range(r):
            chunk = [k for q, k in enumerate(by_last) if q * r // len(by_last) == c]
            # routing sees the table before the chunk
            snap_len = [len(b) for b in self.buckets]
            snap_min = {}
            updates, inserts = [], {}
            for k in chunk:
                b = self._where(k)
                if b is not None:
                    updates.append((b, k))
                    continue
                b1, b2 = self.candidates(k)
                if b1 == b2:
                    tgt = b1
                elif snap_len[b1] < self.S or snap_len[b2] < self.S:  # phase D1: load
                    tgt = b1 if snap_len[b1] <= snap_len[b2] else b2
                else:  # phase D2: the lower minimum (score, key)
                    for b in (b1, b2):
                        if b not in snap_min:
                            snap_min[b] = self._min_entry(self.buckets[b])
                    tgt = b2 if snap_min[b2] < snap_min[b1] else b1
                inserts.setdefault(tgt, []).append(k)
            for b, k in updates:
                ent = self.buckets[b][k]
                if self.policy == LFU:
                    ent[0] = min(M64, ent[0] + inc[k])
                else:
                    ent[0] = s_new[k]
                if not keep_found:
                    ent[1] = vids[last[k]]
                out[k] = ent[1]
                status[k] = UPDATED
            for b in sorted(inserts):
                bucket = self.buckets[b]
                for k in sorted(inserts[b], key=lambda x: (-s_new[x], x)):
                    out[k] = vids[last[k]]
                    if len(bucket) < self.S:
                        bucket[k] = [s_new[k], vids[last[k]]]
                        status[k] = INSERTED
                        continue
                    mscore, mkey = self._min_entry(bucket)
                    if s_new[k] > mscore:
                        sc, vid = bucket.pop(mkey)
                        evicted.append((mkey, sc, vid))
                        bucket[k] = [s_new[k], vids[last[k]]]
                        status[k] = INSERTED_EVICT
                    else:
                        status[k] = REJECTED
        st = [INVALID_KEY if k in (EMPTY, LOCKED) else status[k] for k in keys]
        return st, evicted, out

    # --- readers and updaters of Sec. 3.5's role list ---
    def contains(self, keys):
        return [k not in (EMPTY, LOCKED) and self._where(k) is not None for k in keys]

    def locate(self, keys):
        """bucket of each resident key, None where absent"""
        return [None if k in (EMPTY, LOCKED) else self._where(k) for k in keys]

    def assign(self, keys, vids=None, scores=None):
        """assign (vids given) / assign_scores (vids None): resident keys only, last occurrence
        wins, LFU increments summed; returns per-occurrence residency."""
        if not keys:
            return []
        if self.policy == LRU:
            self.clock += 1
        last, inc = {}, {}
        for i, k in enumerate(keys):
            if k in (EMPTY, LOCKED):
                continue
            last[k] = i
            if self.policy == LFU:
                inc[k] = min(M64, inc.get(k, 0) + (scores[i] if scores is not None else 1))
        for k, i in last.items():
            b = self._where(k)
            if b is None:
                continue
            ent = self.buckets[b][k]
            if self.policy == CUSTOM:
                ent[0] = scores[i]
            elif self.policy == LRU:
                ent[0] = self.clock
            else:
                ent[0] = min(M64, ent[0] + inc[k])
            if vids is not None:
                ent[1] = vids[i]
        return self.contains(keys)

    def export_if(self, min_score: int):
        return {b: sorted((k, sv[0], sv[1]) for k, sv in bk.items() if sv[0] >= min_score)
                for b, bk in enumerate(self.buckets) if any(sv[0] >= min_score for sv in bk.values())}

    def erase(self, keys):
        present = [k not in (EMPTY, LOCKED) and self._where(k) is not None for k in keys]
        for k, p in zip(keys, present):
            if p:
                b = self._where(k)
                if b is not None:
                    del self.buckets[b][k]
        return present

    def size(self):
        return sum(len(b) for b in self.buckets)

    def export(self):
        """{bucket: sorted list of (key, score, vid)}"""
        return {b: sorted((k, sv[0], sv[1]) for k, sv in bk.items())
                for b, bk in enumerate(self.buckets) if bk}
