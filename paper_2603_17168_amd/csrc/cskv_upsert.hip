// Upsert kernels of the cache-semantic hash table (insert_or_assign / insert_and_evict) for
// CDNA4 (gfx950, wave64): Alg. 2 (in-line upsert with admission control and eviction) inside
// Alg. 3 (score-based dual-bucket choice), under the deterministic batch order of cskv.h.
//
// A plain call (one route round) is a fixed sequence on one stream:
//   dedupe   block-local, in LDS: each block of 2048 input positions keeps one representative per
//            key, its last occurrence in the block (and, for LFU, the block's sum of the key's
//            increments); no global atomic per key.  The same launch clears the call's zeroed
//            scratch (dedupe set, overflow keys, counters), which it does not read
//   route    G lanes per representative, against the table as it was before the call: update slot
//            if present in b1/b2, else target by phase D1 (occupancy, b1 on a tie) or D2 (the
//            smaller cached bucket minimum (score, key)).  One atomic on the target's counter
//            (inserts in the low half, updates in the high half) gives the operation its place
//            in the bucket's list and, for an insert, its arrival rank r among the bucket's
//            inserts: while r is below the bucket's number of free slots before the call, the
//            insert writes its key, score and row at once into the r-th of those free slots
//            (a direct insert).  Digest bytes are not written here, so every key of the call
//            sees the digest lines, occupancies and free-slot order of the table before it.
//            Routing depends only on the key and that table, so the representatives of a key
//            repeated across blocks all land in the same bucket's list.
//            Routing also writes each representative's status as far as it knows it (UPDATED,
//            INSERTED for a direct insert).
//   commit   (calls of more than 16384 keys) one thread per bucket: a bucket that received only
//            direct inserts of distinct keys and keeps a free slot is finished by writing their
//            digest bytes
//   apply    16 lanes per bucket (8 slots each), 16 buckets per 256-thread block, for the buckets
//            the commit left.  The entries of one key are merged first: the one with the largest
//            input position (the key's last occurrence) wins, LFU increments are summed.  A bucket
//            that received only inserts, no more than its free slots, just has the digest bytes of
//            its direct inserts written.
//            Otherwise: updates, then inserts ranked by (score desc, key asc): the first ones (as
//            many as there were free slots) are inserted, the rest compete with the smallest
//            residents by (score, key) - strict admission.  Slot positions are not observable,
//            so a direct insert keeps the slot it took; the inserts still waiting in the list
//            take the victims' slots and the free slots given up by merged or refused direct
//            inserts and by direct inserts that evicted; victims are copied out first
//   slow     one wave per bucket that received more than 16 operations: the same rules, with the
//            entries of a key merged through the call's dedupe set and the best 128 inserts kept
//            in LDS
//   finish   per-occurrence status (from its representative)
// Route sub-rounds and the phased (overlapped) programs dedupe the whole call first through a
// global set (one CAS per occurrence, k_dedupe) and route only each key's last occurrence.
// Every write to a table slot's key/score/digest in the apply kernels is made by the lane that
// owns the slot, and every 16-byte chunk c of a row by lane c mod (lanes), so writes that must
// follow one another (an update, then the eviction of the same entry) are ordered by program
// order.
#include <hip/hip_runtime.h>

#include "cskv_device.h"
#include "cskv_internal.h"

namespace cskv {

constexpr int GA = 16;            // lanes per bucket in the fast apply kernel
constexpr int SPL = kSlots / GA;  // slots per lane
constexpr uint64_t kGold = 0x9E3779B97F4A7C15ull;

// group minimum of (score, key) pairs under (score asc, key asc), by the DPP exchange steps of
// the group reductions (G <= 16)
template <int S>
__device__ __forceinline__ void min_pair_step(uint64_t& s, uint64_t& k) {
    const uint64_t os = dpp_xchg<S>(s), ok = dpp_xchg<S>(k);
    const bool take = os < s || (os == s && ok < k);
    s = take ? os : s;
    k = take ? ok : k;
}

template <int G>
__device__ __forceinline__ void gmin_pair(uint64_t& s, uint64_t& k) {
    static_assert(G == 16, "16-lane groups");
    min_pair_step<0>(s, k);
    min_pair_step<1>(s, k);
    min_pair_step<2>(s, k);
    min_pair_step<3>(s, k);
}

__device__ __forceinline__ uint64_t scratch_hash(uint64_t x, int logP) { return (fmix64(x) * kGold) >> (64 - logP); }

__device__ __forceinline__ uint64_t overflow_key(uint32_t b, uint32_t r) { return ((uint64_t)b << 32) + r + 1; }

struct Entry {
    uint64_t key;
    uint64_t score;          // CUSTOM / LRU: the operation's score; LFU: its increment (sum)
    uint64_t w;              // dedupe slot (or representative position) << 32 | input position
    uint8_t slot;            // update: the resident slot; direct insert: the free slot it took
    uint8_t dg;              // the key's digest, computed once by routing
    uint8_t kind;            // OpKind
    uint8_t nfree;           // inserts: free slots of the bucket before the call
};

__device__ __forceinline__ Entry load_entry(const OpEntry* p) {
    const ulonglong2* q = reinterpret_cast<const ulonglong2*>(p);
    const ulonglong2 a = q[0], c = q[1];
    Entry e;
    e.key = a.x;
    e.score = a.y;
    e.w = c.x;
    e.slot = (uint8_t)c.y;
    e.dg = (uint8_t)(c.y >> 8);
    e.kind = (uint8_t)(c.y >> 16);
    e.nfree = (uint8_t)(c.y >> 24);
    return e;
}

__device__ __forceinline__ void store_entry(OpEntry* p, uint64_t key, uint64_t score, uint64_t w, uint32_t slot,
                                            uint32_t dg, uint32_t kind, uint32_t nfree) {
    ulonglong2* q = reinterpret_cast<ulonglong2*>(p);
    q[0] = make_ulonglong2(key, score);
    q[1] = make_ulonglong2(w, (unsigned long long)((slot & 0xFFu) | ((dg & 0xFFu) << 8) | ((kind & 0xFFu) << 16) |
                                                   ((nfree & 0xFFu) << 24)));
}

__device__ __forceinline__ Entry fetch_entry(const UpsertWs& w, uint32_t b, uint32_t r) {
    if (r < w.cap) return load_entry(w.il + (size_t)b * w.cap + r);
    const uint64_t ok = overflow_key(b, r);
    uint64_t q = scratch_hash(ok, w.logP);
    for (uint64_t probes = 0; probes < w.P && w.okey[q] != ok; ++probes) q = (q + 1) & (w.P - 1);
    return load_entry(w.ol + q);
}

// operations routed to a bucket by the running call (inserts + updates)
__device__ __forceinline__ uint32_t routed_ops(uint64_t c) { return (uint32_t)c + (uint32_t)(c >> 32); }

// the dedupe-set slot of key k: claims a free slot for a new key (CAS), else finds the key's slot
__device__ __forceinline__ uint64_t set_slot(const UpsertWs& w, uint64_t k) {
    const uint64_t mask = w.P - 1;
    uint64_t x = scratch_hash(k, w.logP);
    for (uint64_t probes = 0; probes < w.P; ++probes) {
        const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&w.dd[x].key), 0ull,
                                                 (unsigned long long)k);
        if (old == 0ull || old == k) break;
        x = (x + 1) & mask;
    }
    return x;
}

// ------------------------------------------------------------------------------------------
// block-local dedupe: 2048 input positions per 512-thread block, an LDS hash table of 4096 keys
// (48 KB; 96 KB with the LFU sums).  Each occurrence records the position of its key's last
// occurrence in the block (its representative); a representative gets the block's (saturating)
// LFU sum of the key's increments.  The larger the block, the fewer representatives a key that
// repeats all over the batch sends to its bucket.
constexpr int kLocalThreads = 512;
constexpr int kLocalKeys = 2048;
constexpr int kLocalHashBits = 12;
constexpr int kLocalHash = 1 << kLocalHashBits;

template <bool LFU>
__global__ void __launch_bounds__(kLocalThreads) k_local_dedupe(UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                                      const uint64_t* __restrict__ scores, uint64_t* ev_count,
                                                      uint4* zero, size_t zero16) {
    __shared__ unsigned long long hk[kLocalHash];
    __shared__ uint32_t hl[kLocalHash];
    __shared__ unsigned long long hi[LFU ? kLocalHash : 1];
    __shared__ uint32_t hs[LFU ? kLocalHash : 1];
    const int tid = threadIdx.x;
    for (int j = tid; j < kLocalHash; j += kLocalThreads) {
        hk[j] = 0ull;
        hl[j] = 0u;
        if constexpr (LFU) {
            hi[j] = 0ull;
            hs[j] = 0u;
        }
    }
    if (blockIdx.x == 0 && tid == 0 && ev_count) *ev_count = 0;
    // the call's zeroed scratch (dedupe set, overflow keys, counters), which this pass does not use
    for (size_t z = (size_t)blockIdx.x * kLocalThreads + tid; z < zero16; z += (size_t)gridDim.x * kLocalThreads)
        zero[z] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kLocalKeys;
    constexpr int PER = kLocalKeys / kLocalThreads;
    int hslot[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t li = (uint32_t)(q * kLocalThreads + tid);
        const uint64_t i = base + li;
        hslot[q] = -1;
        if (i >= n) continue;
        const uint64_t k = keys[i];
        if (reserved_key(k)) continue;
        uint32_t h = (uint32_t)((fmix64(k) * kGold) >> (64 - kLocalHashBits));
        for (int probes = 0; probes < kLocalHash; ++probes) {
            const unsigned long long old = atomicCAS(&hk[h], 0ull, (unsigned long long)k);
            if (old == 0ull) break;
            if (old == k) break;
            h = (h + 1) & (kLocalHash - 1);
        }
        hslot[q] = (int)h;
        atomicMax(&hl[h], li + 1);
        if constexpr (LFU) {
            const unsigned long long inc = scores ? scores[i] : 1ull;
            const unsigned long long old = atomicAdd(&hi[h], inc);
            if (old + inc < old) atomicOr(&hs[h], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint64_t i = base + (uint32_t)(q * kLocalThreads + tid);
        if (i >= n) continue;
        if (hslot[q] < 0) {
            w.slot_of[i] = kNoSlot;
            continue;
        }
        const uint64_t rep = base + hl[hslot[q]] - 1;
        w.slot_of[i] = (uint32_t)rep;
        if constexpr (LFU)
            if (rep == i) w.rinc[i] = hs[hslot[q]] ? ~0ull : hi[hslot[q]];
    }
}

// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dedupe(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                                const uint64_t* __restrict__ scores, uint64_t* ev_count) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && ev_count) *ev_count = 0;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (reserved_key(k)) {
        w.slot_of[i] = kNoSlot;
        return;
    }
    // one atomic per distinct key: the occurrence that claims the entry records its index with a
    // plain store; later occurrences of the key raise `last` with atomicMax
    const uint64_t mask = w.P - 1;
    uint64_t p = scratch_hash(k, w.logP);
    for (uint64_t probes = 0; probes < w.P; ++probes) {
        const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&w.dd[p].key), 0ull,
                                                 (unsigned long long)k);
        if (old == 0ull) {
            w.dd[p].claim = (uint32_t)(i + 1);
            break;
        }
        if (old == k) {
            atomicMax(&w.dd[p].last, (uint32_t)(i + 1));
            w.ctr[kCtrDup] = 1;  // later passes read the set only when some key repeats
            break;
        }
        p = (p + 1) & mask;
    }
    w.slot_of[i] = (uint32_t)p;
    if (t.policy == 2) {  // LFU: saturating sum of the increments
        const uint64_t inc = scores ? scores[i] : 1ull;
        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(w.inc + p), (unsigned long long)inc);
        if (old + inc < old) atomicOr(w.sat + p, 1u);
    }
}

// ------------------------------------------------------------------------------------------
// route sub-rounds: the distinct keys, ordered by the index of their last occurrence, are cut
// into `rounds` chunks (rank q goes to chunk q * rounds / N); each chunk is routed and applied
// against the table the chunks before it left.  The ranks come from a three-kernel scan of the
// last-occurrence flags (block counts, one block scanning them, in-block offsets by ballot).
__device__ __forceinline__ bool last_occurrence(const UpsertWs& w, uint64_t i, bool dups) {
    const uint32_t p = w.slot_of[i];
    if (p == kNoSlot) return false;
    if (!dups) return true;
    const DedupeEntry de = w.dd[p];
    return (de.claim > de.last ? de.claim : de.last) == (uint32_t)(i + 1);
}

__global__ void __launch_bounds__(256) k_rank_count(UpsertWs w, uint64_t n) {
    __shared__ uint32_t part[4];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool dups = w.ctr[kCtrDup] != 0;
    const uint64_t bal = __ballot(i < n && last_occurrence(w, i, dups));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) w.bsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ void __launch_bounds__(256) k_rank_scan(UpsertWs w, uint64_t nblk) {
    __shared__ uint32_t buf[256];
    uint32_t carry = 0;
    for (uint64_t base = 0; base < nblk; base += 256) {
        const uint64_t j = base + threadIdx.x;
        const uint32_t v = j < nblk ? w.bsum[j] : 0u;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive scan in LDS
            const uint32_t x = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
            __syncthreads();
            buf[threadIdx.x] += x;
            __syncthreads();
        }
        if (j < nblk) w.bsum[j] = carry + buf[threadIdx.x] - v;  // exclusive offsets
        carry += buf[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) w.ctr[kCtrDistinct] = carry;
}

__global__ void __launch_bounds__(256) k_rank_write(UpsertWs w, uint64_t n) {
    __shared__ uint32_t part[4];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool dups = w.ctr[kCtrDup] != 0;
    const bool f = i < n && last_occurrence(w, i, dups);
    const uint64_t bal = __ballot(f);
    const int lane = threadIdx.x & 63;
    if (lane == 0) part[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = w.bsum[blockIdx.x];
    for (int q = 0; q < (int)(threadIdx.x >> 6); ++q) off += part[q];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (f) w.rank[i] = off + (uint32_t)__popcll(bal & below);
}

// ------------------------------------------------------------------------------------------
// LOCAL: the block-local dedupe ran before; each representative routes (its block's last
// occurrence of the key, with the block's LFU sum).  Otherwise the global dedupe pass ran before
// (sub-rounds, phased programs), and only each key's last occurrence routes.
template <int G, bool LOCAL>
__global__ void __launch_bounds__(256) k_route(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                               const float* __restrict__ vals, const uint64_t* __restrict__ scores) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int lane = glane<G>();
    if (i >= n) return;
    uint32_t p;
    bool dups = false;
    if constexpr (LOCAL) {
        if (w.slot_of[i] != (uint32_t)i) return;  // not its block's representative of the key
        p = (uint32_t)i;
    } else {
        p = w.slot_of[i];
        if (p == kNoSlot) return;
        dups = w.ctr[kCtrDup] != 0;  // else every occurrence is its key's last and only one
        if (dups) {
            const DedupeEntry de = w.dd[p];
            if ((de.claim > de.last ? de.claim : de.last) != (uint32_t)(i + 1)) return;  // not the last occurrence
        }
        if (w.rounds > 1) {  // only the keys of this sub-round's chunk
            const uint64_t nd = w.ctr[kCtrDistinct];
            if ((uint64_t)w.rank[i] * (uint64_t)w.rounds / nd != (uint64_t)w.round) return;
        }
    }
    const uint64_t k = keys[i];
    const uint64_t clock = *t.clock + 1;  // LRU: this call's clock (advanced after routing)
    const KeyHash h = hash_key(t, k);
    const bool two = h.b2 != h.b1;
    LineSeg<G> s1, s2;
    s1.load(t.dig + (size_t)h.b1 * kSlots, lane);
    if (two) s2.load(t.dig + (size_t)h.b2 * kSlots, lane);  // an insert needs both occupancies
    uint64_t inc = 0;  // LFU: the increment this operation carries
    if (t.policy == 2) {
        if constexpr (LOCAL) inc = w.rinc[i];
        else inc = dups ? (w.sat[p] ? ~0ull : w.inc[p]) : (scores ? scores[i] : 1ull);
    }
    int slot = verify<G>(t, h.b1, s1.match(h.dg), k, lane);
    uint32_t tgt = h.b1;
    if (slot < 0 && two) {
        slot = verify<G>(t, h.b2, s2.match(h.dg), k, lane);
        tgt = h.b2;
    }
    // the operation's score: CUSTOM the caller's, LRU the call's clock, LFU the increment (the
    // apply adds it to a resident's score)
    const uint64_t ns = t.policy == 0 ? scores[i] : (t.policy == 1 ? clock : inc);
    const bool upd = slot >= 0;  // UPDATE in place (Alg. 2, found)
    uint32_t em = 0;             // inserts: this lane's share of the target's free slots (before the call)
    int nfree = 0;
    if (!upd) {  // INSERT: candidate choice (Alg. 3)
        tgt = h.b1;
        const uint32_t em1 = s1.empty_mask();
        em = em1;
        if (two) {
            const uint32_t em2 = s2.empty_mask();
            const int occ1 = kSlots - gsum_i<G>(__popc(em1));
            const int occ2 = kSlots - gsum_i<G>(__popc(em2));
            if (occ1 < kSlots || occ2 < kSlots) {  // phase D1: less occupied, b1 on a tie
                if (occ2 < occ1) {
                    tgt = h.b2;
                    em = em2;
                }
            } else {  // phase D2: smaller minimum (score, key)
                uint64_t m1s = t.bmin[2 * (size_t)h.b1], m1k = t.bmin[2 * (size_t)h.b1 + 1];
                uint64_t m2s = t.bmin[2 * (size_t)h.b2], m2k = t.bmin[2 * (size_t)h.b2 + 1];
                if (m1k == 0) bucket_min<G>(t, h.b1, lane, m1s, m1k);
                if (m2k == 0) bucket_min<G>(t, h.b2, lane, m2s, m2k);
                if (m2s < m1s || (m2s == m1s && m2k < m1k)) {
                    tgt = h.b2;
                    em = em2;
                }
            }
        }
        nfree = gsum_i<G>(__popc(em));
    }
    unsigned long long old = 0;
    if (lane == 0) {
        old = atomicAdd(reinterpret_cast<unsigned long long*>(t.cnt + tgt), upd ? (1ull << 32) : 1ull);
        if (w.list_mode) {  // newly touched buckets: one cursor atomic per wave, not per bucket
            const bool first = old == 0;
            const uint64_t bal = __ballot(first);  // over the active group leaders of this wave
            if (bal) {
                const int me = threadIdx.x & 63;
                const int leader = __ffsll((unsigned long long)bal) - 1;
                uint32_t base = 0;
                if (me == leader) base = atomicAdd(w.ctr + kCtrTouched, (uint32_t)__popcll(bal));
                base = (uint32_t)__shfl((int)base, leader);
                if (first) w.touched[base + __popcll(bal & ((1ull << me) - 1))] = tgt;
            }
        }
    }
    const uint32_t ir = (uint32_t)__shfl((int)(uint32_t)old, 0, G);          // arrival rank among the inserts
    const uint32_t r = ir + (uint32_t)__shfl((int)(uint32_t)(old >> 32), 0, G);  // place in the bucket's list
    const bool direct = !upd && ir < (uint32_t)nfree;
    int eslot = slot;
    if (direct) eslot = nth_free<G>(em, (int)ir, lane);  // the ir-th free slot, in slot order
    if (lane == 0) {
        const uint64_t wv = ((uint64_t)p << 32) | (uint32_t)i;
        const uint32_t kind = upd ? kOpUpdate : (direct ? kOpDirect : kOpListed);
        // local dedupe: the status as far as routing knows it, in input order (an update's is final;
        // the apply kernels rewrite the others' unless the commit pass finishes the bucket)
        if constexpr (LOCAL) w.sstat[i] = upd ? 1 : (direct ? 2 : 0);
        const uint32_t es = eslot >= 0 ? (uint32_t)eslot : 0u;
        if (r < w.cap) {
            store_entry(w.il + (size_t)tgt * w.cap + r, k, ns, wv, es, h.dg, kind, (uint32_t)nfree);
        } else {
            const uint64_t ok = overflow_key(tgt, r);
            uint64_t q = scratch_hash(ok, w.logP);
            for (uint64_t probes = 0; probes < w.P; ++probes) {
                const unsigned long long o2 = atomicCAS(reinterpret_cast<unsigned long long*>(w.okey + q), 0ull,
                                                        (unsigned long long)ok);
                if (o2 == 0ull) break;
                q = (q + 1) & (w.P - 1);
            }
            store_entry(w.ol + q, k, ns, wv, es, h.dg, kind, (uint32_t)nfree);
        }
    }
    if (direct) {  // key, score and row now; the digest byte in the apply pass
        const size_t e = (size_t)tgt * kSlots + eslot;
        if (lane == 0) {
            t.keys[e] = k;
            t.scores[e] = ns;
        }
        copy_row<G>(t.row(e), vals + i * t.dim, t.dim, lane);
    }
}

// ------------------------------------------------------------------------------------------
// commit pass: one thread per bucket (or per touched-list position).  A bucket whose operations
// are all direct inserts of distinct keys that leave it with a free slot is finished here: its
// keys, scores and rows are in place, so only the digest bytes remain (and the statuses, unless
// routing wrote them); its counter is cleared, so the fast apply that follows skips it.  Any
// other bucket (an update, a listed insert, a key with entries from two input blocks, a bucket
// that fills up, more than 16 operations, find_or_insert) is left to the apply kernels, which
// rewrite all its statuses.  A bucket whose cached minimum is set was full when last written and
// most likely still is, so its entries are not read.
constexpr int kLiteMax = 8;                 // operations of a bucket that one thread commits
constexpr uint64_t kCommitMinKeys = 16384;  // calls with fewer keys skip the commit pass

__global__ void __launch_bounds__(256) k_apply_commit(TableView t, UpsertWs w) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = w.list_mode ? (uint64_t)w.ctr[kCtrTouched] : t.nbuckets;
    if (j >= total || w.out) return;
    const uint32_t b = w.list_mode ? w.touched[j] : (uint32_t)j;
    const uint64_t c = t.cnt[b];
    const uint32_t ni = (uint32_t)c, nu = (uint32_t)(c >> 32);
    if (ni == 0 || nu != 0 || ni > (uint32_t)kLiteMax || t.bmin[2 * (size_t)b + 1] != 0) return;
    bool ok = true;
    uint64_t k[kLiteMax];
    uint32_t sd[kLiteMax];  // slot | digest << 8
#pragma unroll
    for (int r = 0; r < kLiteMax; ++r) {
        k[r] = 0;
        sd[r] = 0;
        if (ok && r < (int)ni) {
            const Entry e = fetch_entry(w, b, (uint32_t)r);
            ok = e.kind == kOpDirect && (uint32_t)e.nfree > ni;
            k[r] = e.key;
            sd[r] = (uint32_t)e.slot | ((uint32_t)e.dg << 8);
            if (!w.local) w.sstat[e.w >> 32] = 2;  // INSERTED (the apply kernels rewrite it if need be)
        }
    }
#pragma unroll
    for (int r = 1; r < kLiteMax; ++r)
#pragma unroll
        for (int q = 0; q < r; ++q) ok = ok && !(r < (int)ni && k[q] == k[r]);
    if (!ok) return;
    const size_t eb = (size_t)b * kSlots;
#pragma unroll
    for (int r = 0; r < kLiteMax; ++r)
        if (r < (int)ni) t.dig[eb + (sd[r] & 0xFFu)] = (uint8_t)(sd[r] >> 8);
    t.cnt[b] = 0;
}

// ------------------------------------------------------------------------------------------
// fast apply: one 16-lane group per bucket with 1..16 operations
constexpr int kApplyGroups = 16;  // buckets (16-lane groups) per 256-thread block

// the lane's 8 slots of the bucket's score line (into registers) and key line (into LDS)
__device__ __forceinline__ void load_lines(const TableView& t, size_t eb, int lane, uint64_t (&sc)[SPL], uint64_t* kc) {
    const ulonglong2* sp = reinterpret_cast<const ulonglong2*>(t.scores + eb + lane * SPL);
    const ulonglong2* kp = reinterpret_cast<const ulonglong2*>(t.keys + eb + lane * SPL);
#pragma unroll
    for (int z = 0; z < SPL / 2; ++z) {
        const ulonglong2 v = sp[z], u = kp[z];
        sc[2 * z] = v.x;
        sc[2 * z + 1] = v.y;
        kc[2 * z] = u.x;
        kc[2 * z + 1] = u.y;
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_apply_fast(TableView t, UpsertWs w, const float* __restrict__ vals, EvictOut ev) {
    __shared__ uint32_t s_nev[kApplyGroups];
    __shared__ uint32_t s_off[kApplyGroups];
    __shared__ unsigned long long s_base;
    __shared__ uint8_t s_pool[kApplyGroups][GA];  // per group: slots handed to the listed inserts that rank first
    __shared__ uint64_t s_keys[kApplyGroups][kSlots];
    const int g = threadIdx.x / GA;
    const int lane = threadIdx.x % GA;
    const int gshift = (threadIdx.x & 63) & ~(GA - 1);
    uint64_t bb = (uint64_t)blockIdx.x * kApplyGroups + g;
    if (w.list_mode) bb = bb < w.ctr[kCtrTouched] ? w.touched[bb] : t.nbuckets;
    const uint32_t b = (uint32_t)bb;
    uint32_t ni = 0, nu = 0;
    if (bb < t.nbuckets) {
        const uint64_t c = t.cnt[b];
        ni = (uint32_t)c;
        nu = (uint32_t)(c >> 32);
    }
    uint32_t m = ni + nu;
    if (m > (uint32_t)kFastMax) {
        if (lane == 0) w.slow[atomicAdd(w.ctr + kCtrSlow, 1u)] = b;
        m = ni = nu = 0;
    }
    const size_t eb = (size_t)b * kSlots;

    // state carried over the block barrier
    Entry e{0, 0, 0, 0, 0, kOpUpdate, 0};
    bool is_upd = false, is_ins = false, is_direct = false, admitted = false, evicts = false;
    bool merged = false;  // an entry of a key whose later occurrence another entry carries
    int win = 0;          // the lane holding this key's winning entry
    int q = 0;            // rank of an insert among the bucket's inserts, (score desc, key asc)
    int new_slot = -1;    // slot of an admitted insert (a direct insert keeps its own)
    int vslot = -1, evi = 0;
    uint64_t vkey = 0, vscore = 0;
    uint32_t upd_bits = 0, ins_bits = 0;
    int nfree = 0;
    // a bucket that ends full: its scores (this call's updates applied) in registers and its keys in
    // LDS, each lane holding its own 8 slots of both
    uint64_t sc[SPL];
    uint64_t* kc = s_keys[g] + lane * SPL;
    bool full_after = false;
    uint32_t nev = 0;

    if (m > 0) {
        const bool has = lane < (int)m;
        if (has) e = fetch_entry(w, b, (uint32_t)lane);
        // merge the entries of one key (representatives of blocks that both held it): the largest
        // input position wins, LFU increments add up
        const uint32_t pos = (uint32_t)e.w;
        uint32_t best = pos;
        win = lane;
        uint64_t incsum = e.score;
        for (int x = 0; x < (int)m; ++x) {
            const uint64_t kx = __shfl(e.key, x, GA);
            const uint32_t px = (uint32_t)__shfl((int)pos, x, GA);
            const uint64_t sx = __shfl(e.score, x, GA);
            if (has && x != lane && kx == e.key) {
                incsum = sat_add(incsum, sx);
                if (px > best) {
                    best = px;
                    win = x;
                }
            }
        }
        merged = has && win != lane;
        const bool live = has && !merged;
        if (live && t.policy == 2) e.score = incsum;  // LFU: the key's whole increment
        is_upd = live && e.kind == kOpUpdate;
        is_ins = live && e.kind != kOpUpdate;
        is_direct = live && e.kind == kOpDirect;
        if (is_upd && t.policy == 2) e.score = sat_add(t.scores[eb + e.slot], e.score);
        upd_bits = (uint32_t)((__ballot(is_upd) >> gshift) & 0xFFFFu);
        ins_bits = (uint32_t)((__ballot(is_ins) >> gshift) & 0xFFFFu);
        const int nins = __popc(ins_bits);
        const bool any_merged = ((__ballot(merged) >> gshift) & 0xFFFFu) != 0;
        // free slots before the call: carried by every insert, else read from the digest line
        nfree = gmax_i<GA>(has && e.kind != kOpUpdate ? (int)e.nfree : -1);
        const bool plain = nu == 0 && (int)ni <= nfree;  // only inserts, all of them direct
        uint32_t taken = 0;  // free slots before the call (now holding direct inserts) are never victims
        if (!plain && nfree != 0) {
            const uint2 dv = *reinterpret_cast<const uint2*>(t.dig + eb + lane * SPL);
            taken = match4(dv.x, 0u) | (match4(dv.y, 0u) << 4);
            nfree = gsum_i<GA>(__popc(taken));
        }
        full_after = nins >= nfree;
        int want = nins - nfree;  // inserts beyond the free slots: they compete for victims
        // A bucket that was full keeps its cached minimum (score, key) when every update leaves that
        // entry the smallest (no update of the minimum's own key, none to a smaller pair) and no
        // insert scores above it (strict admission refuses them all): then its score and key lines
        // are not read and its cached minimum stands.  (Under LRU a call's inserts always score above
        // the residents, so only buckets without inserts are checked.)
        if (nfree == 0 && (want == 0 || t.policy != 1)) {
            const uint64_t ms = t.bmin[2 * (size_t)b], mk = t.bmin[2 * (size_t)b + 1];
            if (mk != 0) {
                const bool keeps = !is_upd || (e.key != mk && (e.score > ms || (e.score == ms && e.key > mk)));
                const bool kept = ((__ballot(!keeps) >> gshift) & 0xFFFFu) == 0u;
                const uint64_t top = ~gmin_u64<GA>(is_ins ? ~e.score : ~0ull);  // the best insert score
                if (kept && (want == 0 || top <= ms)) {
                    want = 0;
                    full_after = false;
                }
            }
        }
        if (want > 0) {
            for (int x = 0; x < (int)m; ++x) {
                const uint64_t sx = __shfl(e.score, x, GA);
                const uint64_t kx = __shfl(e.key, x, GA);
                q += (int)(((ins_bits >> x) & 1u) && (sx > e.score || (sx == e.score && kx < e.key)));
            }
        }
        if (full_after) {  // scores and keys of the bucket (direct inserts included), updates applied
            load_lines(t, eb, lane, sc, kc);
            for (uint32_t ub = upd_bits; ub; ub &= ub - 1) {
                const int x = __ffs(ub) - 1;
                const int us = __shfl((int)e.slot, x, GA);
                const uint64_t usc = __shfl(e.score, x, GA);
#pragma unroll
                for (int z = 0; z < SPL; ++z)
                    if ((us >> 3) == lane && (us & 7) == z) sc[z] = usc;
            }
        }
        // victims for the inserts ranked nfree, nfree+1, ... (strict admission, Alg. 2)
        for (int v = 0; v < want; ++v) {
            const uint32_t rb = (uint32_t)((__ballot(is_ins && q == nfree + v) >> gshift) & 0xFFFFu);
            const int rl = __ffs(rb) - 1;
            const uint64_t s_in = __shfl(e.score, rl, GA);
            // smallest resident by (score, key) among the slots not yet taken; the lane's keys are
            // read from LDS two at a time and compared without branches
            uint64_t ls = ~0ull, lk = ~0ull;
            int lslot = -1;
            const ulonglong2* kp2 = reinterpret_cast<const ulonglong2*>(kc);
#pragma unroll
            for (int q2 = 0; q2 < SPL / 2; ++q2) {
                const ulonglong2 kk = kp2[q2];
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int z = 2 * q2 + hh;
                    const uint64_t kz = hh ? kk.y : kk.x;
                    const bool better = (((taken >> z) & 1u) == 0u) & ((sc[z] < ls) | ((sc[z] == ls) & (kz < lk)));
                    ls = better ? sc[z] : ls;
                    lk = better ? kz : lk;
                    lslot = better ? lane * SPL + z : lslot;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            uint64_t gm = ls, gk = lk;
            gmin_pair<GA>(gm, gk);
            if (!(s_in > gm)) break;  // rejected, and so is every later insert
            const uint32_t ob = (uint32_t)((__ballot(lslot >= 0 && ls == gm && lk == gk) >> gshift) & 0xFFFFu);
            const int ol = __ffs(ob) - 1;
            const int vsl = __shfl(lslot, ol, GA);
            if (lane == ol) taken |= 1u << (vsl & 7);
            if (lane == rl) {
                vslot = vsl;
                vkey = gk;
                vscore = gm;
                evi = v;
                evicts = true;
            }
            ++nev;
        }
        admitted = is_ins && (q < nfree || evicts);
        if (is_direct && admitted) new_slot = e.slot;
        if (want > 0 || any_merged) {
            // Slots are not observable, so a direct insert keeps the free slot it took.  The
            // listed inserts that rank among the first nfree take, in rank order, the slots that
            // direct entries give up (a merged or refused one its own free slot, an evicting one
            // its victim's slot); a listed insert that evicts takes its victim's slot.  Slots
            // given up and not taken stay free.
            const bool dmerged = merged && e.kind == kOpDirect;
            const bool gives = (is_direct && (!admitted || evicts)) || dmerged;
            const bool needs = is_ins && !is_direct && q < nfree;
            const int gkey = dmerged ? 1024 + lane : q;  // order of the given-up slots
            const uint32_t gm_ = (uint32_t)((__ballot(gives) >> gshift) & 0xFFFFu);
            const uint32_t nm_ = (uint32_t)((__ballot(needs) >> gshift) & 0xFFFFu);
            int gi = 0, ki = 0;
            for (int x = 0; x < (int)m; ++x) {
                const int qx = __shfl(q, x, GA);
                const int gx = __shfl(gkey, x, GA);
                gi += (int)(((gm_ >> x) & 1u) && gx < gkey);
                ki += (int)(((nm_ >> x) & 1u) && qx < q);
            }
            if (gives) s_pool[g][gi] = (uint8_t)(admitted ? vslot : e.slot);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();  // the group is inside one wave: its LDS accesses stay in order
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (needs) new_slot = s_pool[g][ki];
            if (is_ins && !is_direct && evicts) new_slot = vslot;
        }
    }

    // eviction output positions: one atomic per block
    if (ev.count) {
        if (lane == 0) s_nev[g] = nev;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int z = 0; z < kApplyGroups; ++z) {
                s_off[z] = tot;
                tot += s_nev[z];
            }
            s_base = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(ev.count), (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
    }
    if (m == 0) return;
    const uint64_t ev_base = ev.count ? s_base + s_off[g] : 0ull;

    // statuses (a merged entry takes its key's) and evicted (key, score)
    const int st = is_upd ? 1 : (is_ins ? (q < nfree ? 2 : (evicts ? 3 : 4)) : 0);
    const int wst = __shfl(st, win, GA);
    if ((int)lane < (int)m) w.sstat[e.w >> 32] = (uint8_t)wst;
    if (evicts && ev.keys) {
        ev.keys[ev_base + evi] = vkey;
        ev.scores[ev_base + evi] = vscore;
    }
    // slot metadata, by the owning lane: updates first, then admitted inserts (a direct insert's key
    // and score are in place already, its score only rewritten when merged entries added LFU
    // increments)
    for (uint32_t ub = upd_bits; ub; ub &= ub - 1) {
        const int x = __ffs(ub) - 1;
        const int us = __shfl((int)e.slot, x, GA);
        const uint64_t usc = __shfl(e.score, x, GA);
        if ((us >> 3) == lane) t.scores[eb + us] = usc;
    }
    for (uint32_t ib = ins_bits; ib; ib &= ib - 1) {
        const int x = __ffs(ib) - 1;
        const int ns = __shfl(new_slot, x, GA);
        if (ns < 0) continue;
        const bool dir = __shfl((int)is_direct, x, GA) != 0;
        const uint64_t nk = __shfl(e.key, x, GA);
        const uint64_t nsc = __shfl(e.score, x, GA);
        const int nd = __shfl((int)e.dg, x, GA);
        if ((ns >> 3) == lane) {
            if (!dir) t.keys[eb + ns] = nk;
            if (!dir || t.policy == 2) t.scores[eb + ns] = nsc;
            t.dig[eb + ns] = (uint8_t)nd;
            if (full_after) {
#pragma unroll
                for (int z = 0; z < SPL; ++z)
                    if ((ns & 7) == z) {
                        sc[z] = nsc;
                        kc[z] = nk;
                    }
            }
        }
    }
    // rows: chunk c of every row by lane c mod 16; updates (the winning entry's row), then the
    // victims' rows copied out, then the listed inserts.  find_or_insert (w.out set) keeps a resident
    // row and returns it for every entry of the key; every insert's entries return the key's row.
    const uint32_t chunks = t.dim >> 2;
    for (uint32_t ub = upd_bits; ub; ub &= ub - 1) {
        const int x = __ffs(ub) - 1;
        const int us = __shfl((int)e.slot, x, GA);
        const uint32_t pos = (uint32_t)__shfl((int)(uint32_t)e.w, x, GA);
        uint4* dst = reinterpret_cast<uint4*>(t.row(eb + us));
        if (!w.out) {
            const uint4* src = reinterpret_cast<const uint4*>(vals + (size_t)pos * t.dim);
            for (uint32_t c = lane; c < chunks; c += GA) dst[c] = src[c];
        }
    }
    if (w.out) {
        for (int x = 0; x < (int)m; ++x) {
            const int wx = __shfl(win, x, GA);
            const bool uw = __shfl((int)is_upd, wx, GA) != 0;
            const uint32_t pos = (uint32_t)__shfl((int)(uint32_t)e.w, x, GA);
            const uint32_t wpos = (uint32_t)__shfl((int)(uint32_t)e.w, wx, GA);
            const int us = __shfl((int)e.slot, wx, GA);
            uint4* o = reinterpret_cast<uint4*>(w.out + (size_t)pos * t.dim);
            const uint4* src = uw ? reinterpret_cast<const uint4*>(t.row(eb + us))
                                  : reinterpret_cast<const uint4*>(vals + (size_t)wpos * t.dim);
            for (uint32_t c = lane; c < chunks; c += GA) o[c] = src[c];
        }
    }
    if (nev && ev.vals) {
        for (uint32_t ib = ins_bits; ib; ib &= ib - 1) {
            const int x = __ffs(ib) - 1;
            if (!__shfl((int)evicts, x, GA)) continue;
            const int vs = __shfl(vslot, x, GA);
            const int xi = __shfl(evi, x, GA);
            const uint4* src = reinterpret_cast<const uint4*>(t.row(eb + vs));
            uint4* out = reinterpret_cast<uint4*>(ev.vals + (ev_base + xi) * t.dim);
            for (uint32_t c = lane; c < chunks; c += GA) out[c] = src[c];
        }
    }
    for (uint32_t ib = ins_bits; ib; ib &= ib - 1) {
        const int x = __ffs(ib) - 1;
        const int ns = __shfl(new_slot, x, GA);
        if (ns < 0 || __shfl((int)is_direct, x, GA)) continue;
        const uint32_t pos = (uint32_t)__shfl((int)(uint32_t)e.w, x, GA);
        uint4* dst = reinterpret_cast<uint4*>(t.row(eb + ns));
        const uint4* src = reinterpret_cast<const uint4*>(vals + (size_t)pos * t.dim);
        for (uint32_t c = lane; c < chunks; c += GA) dst[c] = src[c];
    }
    // cached minimum of a full bucket (exact; every slot is occupied now)
    if (full_after) {
        uint64_t ls = ~0ull, lk = ~0ull;
        const ulonglong2* kp2 = reinterpret_cast<const ulonglong2*>(kc);
#pragma unroll
        for (int q2 = 0; q2 < SPL / 2; ++q2) {
            const ulonglong2 kk = kp2[q2];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int z = 2 * q2 + hh;
                const uint64_t kz = hh ? kk.y : kk.x;
                const bool better = (sc[z] < ls) | ((sc[z] == ls) & (kz < lk));
                ls = better ? sc[z] : ls;
                lk = better ? kz : lk;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        gmin_pair<GA>(ls, lk);
        if (lane == 0) {
            t.bmin[2 * (size_t)b] = ls;
            t.bmin[2 * (size_t)b + 1] = lk;
        }
    }
    if (lane == 0) t.cnt[b] = 0;
}

// ------------------------------------------------------------------------------------------
// slow apply: one wave per bucket with more than 16 operations
// the merge table of one crowded bucket's keys in the slow apply (LDS); a bucket with more distinct
// keys than it holds merges through the call's dedupe set in HBM instead
constexpr int kSlowKeys = 512;

__device__ __forceinline__ uint32_t slow_hash(uint64_t k) { return (uint32_t)((fmix64(k) * kGold) >> (64 - 9)); }

// A crowded bucket's list positions past the inline ones live in the hashed overflow table; the
// merge pass finds their slots (the probes of 8 positions per lane issued together) and keeps them
// in LDS for the bucket's later passes, which then load each entry with one access.
constexpr int kSlowBatch = 8;
constexpr uint32_t kSlowStage = 1024;

__device__ __forceinline__ Entry staged_entry(const UpsertWs& w, uint32_t b, uint32_t r, const uint32_t* qst, bool staged) {
    if (r < w.cap) return load_entry(w.il + (size_t)b * w.cap + r);
    if (staged) return load_entry(w.ol + qst[r]);
    return fetch_entry(w, b, r);
}

// the merge-table slot of key k, claimed if new; -1 if the table is full
__device__ __forceinline__ int slow_claim(unsigned long long* hk, uint64_t k) {
    uint32_t h = slow_hash(k);
    for (int probes = 0; probes < kSlowKeys; ++probes) {
        const unsigned long long old = atomicCAS(&hk[h], 0ull, (unsigned long long)k);
        if (old == 0ull || old == k) return (int)h;
        h = (h + 1) & (kSlowKeys - 1);
    }
    return -1;
}

// the merge-table slot of key k, which is present
__device__ __forceinline__ int slow_find(const unsigned long long* hk, uint64_t k) {
    uint32_t h = slow_hash(k);
    for (int probes = 0; probes < kSlowKeys && hk[h] != k; ++probes) h = (h + 1) & (kSlowKeys - 1);
    return (int)h;
}

__global__ void __launch_bounds__(64) k_apply_slow(TableView t, UpsertWs w, const float* __restrict__ vals, EvictOut ev) {
    __shared__ unsigned long long hk[kSlowKeys];  // merge table: key, largest position + 1, LFU sum
    __shared__ uint32_t hl[kSlowKeys];
    __shared__ unsigned long long hi[kSlowKeys];
    __shared__ uint32_t hs[kSlowKeys];
    __shared__ int hfull;
    __shared__ uint64_t cs[192], ck[192], cw[192];  // insert candidates: score, key, w
    __shared__ uint8_t cd[192];                     // and the free slot a direct insert took (0xFF: listed)
    __shared__ uint64_t ns_[128], nk_[128], nw_[128];
    __shared__ uint8_t nd_[128], cst[128];
    __shared__ uint64_t S_[128], K_[128];           // residents by slot (updates applied)
    __shared__ uint64_t rs[128], rk[128];           // smallest residents in (score, key) order
    __shared__ uint8_t rslot[128], dslot[128], uflag[128], nflag[128], gave[128], plist[128];
    __shared__ uint64_t newk[128], news[128];
    __shared__ unsigned long long ev_base_s;
    __shared__ uint32_t qst[kSlowStage];            // overflow-table slots of the list positions

    const int lane = threadIdx.x;
    // routing has read the clock (every sub-round of the call reads the same value)
    if (blockIdx.x == 0 && lane == 0 && t.policy == 1 && w.round == w.rounds - 1) *t.clock += 1;
    const uint32_t nslow = w.ctr[kCtrSlow];
    const uint32_t chunks = t.dim >> 2;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (uint32_t si = blockIdx.x; si < nslow; si += gridDim.x) {
        const uint32_t b = w.slow[si];
        const uint32_t m = routed_ops(t.cnt[b]);
        const size_t eb = (size_t)b * kSlots;

        // residents: the slots occupied before the call (a direct insert's slot still has a zero digest)
        const bool o0 = t.dig[eb + lane] != 0;
        const bool o1 = t.dig[eb + lane + 64] != 0;
        S_[lane] = o0 ? t.scores[eb + lane] : ~0ull;
        K_[lane] = o0 ? t.keys[eb + lane] : ~0ull;
        S_[lane + 64] = o1 ? t.scores[eb + lane + 64] : ~0ull;
        K_[lane + 64] = o1 ? t.keys[eb + lane + 64] : ~0ull;
        uflag[lane] = uflag[lane + 64] = 0;
        nflag[lane] = nflag[lane + 64] = 0;
        gave[lane] = gave[lane + 64] = 0;
        const int occ = __popcll(__ballot(o0)) + __popcll(__ballot(o1));
        const int nfree = kSlots - occ;

        // block-local dedupe leaves one entry per key and input block: merge a key's entries (largest
        // position + 1 wins, LFU increments summed, saturating) in the LDS merge table, or, when the
        // bucket has more distinct keys than it holds, through the call's dedupe set
        bool any_merged = false;
        bool in_lds = true;
        const bool staged = w.local && m <= kSlowStage;
        if (w.local) {
            for (int j = lane; j < kSlowKeys; j += 64) {
                hk[j] = 0ull;
                hl[j] = 0u;
                hi[j] = 0ull;
                hs[j] = 0u;
            }
            if (lane == 0) hfull = 0;
            __syncthreads();
            for (uint32_t c0 = 0; c0 < m; c0 += 64 * kSlowBatch) {
                uint64_t q[kSlowBatch], got[kSlowBatch];
#pragma unroll
                for (int u = 0; u < kSlowBatch; ++u) {  // first probes of every overflow position
                    const uint32_t r = c0 + 64 * u + lane;
                    q[u] = 0;
                    got[u] = 0;
                    if (r < m && r >= w.cap) {
                        q[u] = scratch_hash(overflow_key(b, r), w.logP);
                        got[u] = w.okey[q[u]];
                    }
                }
                Entry eu[kSlowBatch];
#pragma unroll
                for (int u = 0; u < kSlowBatch; ++u) {
                    const uint32_t r = c0 + 64 * u + lane;
                    eu[u] = Entry{0, 0, 0, 0, 0, kOpUpdate, 0};
                    if (r >= m) continue;
                    if (r < w.cap) {
                        eu[u] = load_entry(w.il + (size_t)b * w.cap + r);
                        continue;
                    }
                    const uint64_t ok = overflow_key(b, r);
                    for (uint64_t probes = 0; probes < w.P && got[u] != ok; ++probes) {
                        q[u] = (q[u] + 1) & (w.P - 1);
                        got[u] = w.okey[q[u]];
                    }
                    if (staged) qst[r] = (uint32_t)q[u];
                    eu[u] = load_entry(w.ol + q[u]);
                }
#pragma unroll
                for (int u = 0; u < kSlowBatch; ++u) {
                    if (c0 + 64 * u + lane >= m) continue;
                    const Entry& e = eu[u];
                    const int x = slow_claim(hk, e.key);
                    if (x < 0) {
                        hfull = 1;
                        continue;
                    }
                    atomicMax(&hl[x], (uint32_t)e.w + 1u);
                    if (t.policy == 2) {
                        const unsigned long long old = atomicAdd(&hi[x], (unsigned long long)e.score);
                        if (old + e.score < old) atomicOr(&hs[x], 1u);
                    }
                }
            }
            __syncthreads();
            in_lds = hfull == 0;
            if (!in_lds) {
                for (uint32_t c0 = 0; c0 < m; c0 += 64) {
                    if (c0 + lane >= m) continue;
                    const Entry e = staged_entry(w, b, c0 + lane, qst, staged);
                    const uint64_t x = set_slot(w, e.key);
                    atomicMax(&w.dd[x].last, (uint32_t)e.w + 1u);
                    if (t.policy == 2) {
                        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(w.minc + x),
                                                                 (unsigned long long)e.score);
                        if (old + e.score < old) atomicOr(w.sat + x, 1u);
                    }
                }
                __threadfence();
            }
        }
        __syncthreads();

        // stream the operations: a key's winning entry is applied (updates at once, inserts reduced
        // to the best 128); an entry merged into another gives up the free slot it took, if any
        int nbest = 0;
        for (uint32_t c0 = 0; c0 < m; c0 += 64) {
            const bool has = c0 + lane < m;
            Entry e{0, 0, 0, 0, 0, kOpUpdate, 0};
            if (has) e = staged_entry(w, b, c0 + lane, qst, staged);
            bool live = has;
            if (has && w.local) {
                if (in_lds) {
                    const int x = slow_find(hk, e.key);
                    live = hl[x] == (uint32_t)e.w + 1u;
                    if (live && t.policy == 2) e.score = hs[x] ? ~0ull : hi[x];
                } else {
                    const uint64_t x = set_slot(w, e.key);
                    live = atomicOr(&w.dd[x].last, 0u) == (uint32_t)e.w + 1u;
                    if (live && t.policy == 2) e.score = atomicOr(w.sat + x, 0u) ? ~0ull : atomicAdd(reinterpret_cast<unsigned long long*>(w.minc + x), 0ull);
                }
                if (!live && e.kind == kOpDirect) gave[e.slot] = 1;
            }
            any_merged = any_merged || __ballot(has && !live) != 0;
            const bool upd = live && e.kind == kOpUpdate;
            const bool ins = live && e.kind != kOpUpdate;
            if (upd) {
                S_[e.slot] = t.policy == 2 ? sat_add(S_[e.slot], e.score) : e.score;
                uflag[e.slot] = 1;
                w.sstat[e.w >> 32] = 1;  // UPDATED
            }
            for (uint64_t ub = __ballot(upd); ub; ub &= ub - 1) {
                const int x = __ffsll((unsigned long long)ub) - 1;
                const int us = __shfl((int)e.slot, x);
                const uint32_t pos = (uint32_t)__shfl((int)(uint32_t)e.w, x);
                uint4* dst = reinterpret_cast<uint4*>(t.row(eb + us));
                if (w.out) {  // find_or_insert: the resident row stays and is returned
                    uint4* o = reinterpret_cast<uint4*>(w.out + (size_t)pos * t.dim);
                    for (uint32_t c = lane; c < chunks; c += 64) o[c] = dst[c];
                } else {
                    const uint4* src = reinterpret_cast<const uint4*>(vals + (size_t)pos * t.dim);
                    for (uint32_t c = lane; c < chunks; c += 64) dst[c] = src[c];
                }
            }
            const uint64_t ib = __ballot(ins);
            if (w.out) {  // find_or_insert: every insert returns its own row
                for (uint64_t z = ib; z; z &= z - 1) {
                    const int x = __ffsll((unsigned long long)z) - 1;
                    const uint32_t pos = (uint32_t)__shfl((int)(uint32_t)e.w, x);
                    uint4* o = reinterpret_cast<uint4*>(w.out + (size_t)pos * t.dim);
                    const uint4* src = reinterpret_cast<const uint4*>(vals + (size_t)pos * t.dim);
                    for (uint32_t c = lane; c < chunks; c += 64) o[c] = src[c];
                }
            }
            const int cn = __popcll(ib);
            if (ins) {
                const int at = nbest + __popcll(ib & below);
                cs[at] = e.score;
                ck[at] = e.key;
                cw[at] = e.w;
                cd[at] = e.kind == kOpDirect ? e.slot : (uint8_t)0xFF;
            }
            __syncthreads();
            const int tot = nbest + cn;
            int r[3];
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                const int j = lane + 64 * z;
                r[z] = -1;
                if (j < tot) {
                    const uint64_t s = cs[j], k = ck[j];
                    int rr = 0;
                    for (int x = 0; x < tot; ++x) {
                        const uint64_t sx = cs[x];
                        rr += (sx > s) || (sx == s && ck[x] < k);
                    }
                    r[z] = rr;
                }
            }
            __syncthreads();
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                const int j = lane + 64 * z;
                if (j < tot) {
                    if (r[z] < 128) {
                        ns_[r[z]] = cs[j];
                        nk_[r[z]] = ck[j];
                        nw_[r[z]] = cw[j];
                        nd_[r[z]] = cd[j];
                    } else {
                        w.sstat[cw[j] >> 32] = 4;  // REJECTED: 128 better inserts target this bucket
                        if (cd[j] != 0xFF) gave[cd[j]] = 1;  // a refused direct insert gives up its slot
                    }
                }
            }
            __syncthreads();
            nbest = min(tot, 128);
            for (int j = lane; j < nbest; j += 64) {
                cs[j] = ns_[j];
                ck[j] = nk_[j];
                cw[j] = nw_[j];
                cd[j] = nd_[j];
            }
            __syncthreads();
        }

        // the smallest residents, in (score asc, key asc) order
        const int need = nbest - nfree;
        if (need > 0) {
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                const int sl = lane + 64 * z;
                if (!(z ? o1 : o0)) continue;
                const uint64_t s = S_[sl], k = K_[sl];
                int rr = 0;
                for (int x = 0; x < kSlots; ++x) {
                    const uint64_t sx = S_[x];
                    rr += (sx < s) || (sx == s && K_[x] < k);  // free slots sort last (~0, ~0)
                }
                if (rr < need) {
                    rs[rr] = s;
                    rk[rr] = k;
                    rslot[rr] = (uint8_t)sl;
                }
            }
        }
        __syncthreads();

        // decisions: candidate j is inserted (j < nfree), or competes with the (j-nfree)-th
        // smallest resident; a direct insert keeps the free slot it took and gives it up when
        // refused, or gives up its victim's slot when it evicts; listed inserts take victims'
        // slots, and the ones ranked below nfree take the given-up slots
        bool adm[2];
        uint8_t st[2];
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int j = lane + 64 * z;
            adm[z] = false;
            st[z] = 0;
            if (j < nbest) {
                const bool dir = cd[j] != 0xFF;
                dslot[j] = 0xFF;
                if (j < nfree) {
                    adm[z] = true;
                    st[z] = 2;  // INSERTED
                    if (dir) dslot[j] = cd[j];
                } else {
                    const int v = j - nfree;
                    if (v < occ && cs[j] > rs[v]) {
                        adm[z] = true;
                        st[z] = 3;  // INSERTED_EVICT
                        if (dir) {
                            dslot[j] = cd[j];
                            gave[rslot[v]] = 1;
                        } else {
                            dslot[j] = rslot[v];
                        }
                    } else {
                        st[z] = 4;  // REJECTED
                        if (dir) gave[cd[j]] = 1;
                    }
                }
                cst[j] = st[z];
            }
        }
        __syncthreads();
        // given-up slots in slot order, handed to the listed inserts ranked below nfree in rank order
        {
            const bool g0 = gave[lane] != 0, g1 = gave[lane + 64] != 0;
            const uint64_t b0 = __ballot(g0), b1 = __ballot(g1);
            if (g0) plist[__popcll(b0 & below)] = (uint8_t)lane;
            if (g1) plist[__popcll(b0) + __popcll(b1 & below)] = (uint8_t)(lane + 64);
        }
        __syncthreads();
        {
            const bool w0 = lane < nbest && lane < nfree && cd[lane] == 0xFF;
            const bool w1 = lane + 64 < nbest && lane + 64 < nfree && cd[lane + 64] == 0xFF;
            const uint64_t b0 = __ballot(w0), b1 = __ballot(w1);
            if (w0) dslot[lane] = plist[__popcll(b0 & below)];
            if (w1) dslot[lane + 64] = plist[__popcll(b0) + __popcll(b1 & below)];
        }
        const int nadm = __popcll(__ballot(adm[0])) + __popcll(__ballot(adm[1]));
        const int nev = nadm > nfree ? nadm - nfree : 0;
        if (lane == 0)
            ev_base_s = (ev.count && nev) ? atomicAdd(reinterpret_cast<unsigned long long*>(ev.count), (unsigned long long)nev)
                                          : 0ull;
        __syncthreads();
        const uint64_t ev_base = ev_base_s;
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int j = lane + 64 * z;
            if (j >= nbest) continue;
            w.sstat[cw[j] >> 32] = st[z];
            if (!adm[z]) continue;
            if (st[z] == 3 && ev.keys) {
                const uint64_t x = ev_base + (uint64_t)(j - nfree);
                ev.keys[x] = rk[j - nfree];
                ev.scores[x] = rs[j - nfree];
            }
            nflag[dslot[j]] = 1;
            newk[dslot[j]] = ck[j];
            news[dslot[j]] = cs[j];
        }
        // entries merged into another one: the key's status (UPDATED, a candidate's, or REJECTED when
        // 128 better inserts crowded it out) and, for find_or_insert, the key's row
        if (any_merged) {
            for (uint32_t c0 = 0; c0 < m; c0 += 64) {
                if (c0 + lane >= m) continue;
                const Entry e = staged_entry(w, b, c0 + lane, qst, staged);
                const uint32_t last = in_lds ? hl[slow_find(hk, e.key)] : atomicOr(&w.dd[set_slot(w, e.key)].last, 0u);
                if (last == (uint32_t)e.w + 1u) continue;  // the key's winning entry
                uint8_t s = 4;
                if (e.kind == kOpUpdate) {
                    s = 1;
                } else {
                    for (int j = 0; j < nbest; ++j)
                        if (ck[j] == e.key) s = cst[j];
                }
                w.sstat[e.w >> 32] = s;
                if (w.out) {
                    const uint4* src = e.kind == kOpUpdate ? reinterpret_cast<const uint4*>(t.row(eb + e.slot))
                                                           : reinterpret_cast<const uint4*>(vals + (size_t)(last - 1u) * t.dim);
                    uint4* o = reinterpret_cast<uint4*>(w.out + (size_t)(uint32_t)e.w * t.dim);
                    for (uint32_t c = 0; c < chunks; ++c) o[c] = src[c];
                }
            }
        }
        // rows: chunk c by lane c mod 64; the victims' rows copied out first, then the listed inserts
        if (ev.vals) {
            for (int v = 0; v < nev; ++v) {
                const uint4* src = reinterpret_cast<const uint4*>(t.row(eb + rslot[v]));
                uint4* out = reinterpret_cast<uint4*>(ev.vals + (ev_base + (uint64_t)v) * t.dim);
                for (uint32_t c = lane; c < chunks; c += 64) out[c] = src[c];
            }
        }
        for (int j = 0; j < nadm; ++j) {
            if (cd[j] != 0xFF) continue;  // a direct insert's row is in place
            uint4* dst = reinterpret_cast<uint4*>(t.row(eb + dslot[j]));
            const uint4* src = reinterpret_cast<const uint4*>(vals + (size_t)(uint32_t)cw[j] * t.dim);
            for (uint32_t c = lane; c < chunks; c += 64) dst[c] = src[c];
        }
        __syncthreads();
        // slot metadata by the owning lane; the minimum of the full bucket
        uint64_t lm = ~0ull, lk = ~0ull;
        const bool full = nadm >= nfree;
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int sl = lane + 64 * z;
            if (nflag[sl]) {
                t.keys[eb + sl] = newk[sl];
                t.scores[eb + sl] = news[sl];
                t.dig[eb + sl] = (uint8_t)hash_key(t, newk[sl]).dg;
                S_[sl] = news[sl];
                K_[sl] = newk[sl];
            } else if (uflag[sl]) {
                t.scores[eb + sl] = S_[sl];
            }
            if (S_[sl] < lm || (S_[sl] == lm && K_[sl] < lk)) {
                lm = S_[sl];
                lk = K_[sl];
            }
        }
        if (full) {
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t xm = __shfl_xor(lm, o), xk = __shfl_xor(lk, o);
                if (xm < lm || (xm == lm && xk < lk)) {
                    lm = xm;
                    lk = xk;
                }
            }
            if (lane == 0) {
                t.bmin[2 * (size_t)b] = lm;
                t.bmin[2 * (size_t)b + 1] = lk;
            }
        }
        if (lane == 0) t.cnt[b] = 0;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_finish(UpsertWs w, uint64_t n, uint8_t* __restrict__ status, uint32_t dim) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = w.slot_of[i];
    if (status) status[i] = (p == kNoSlot) ? 5 : w.sstat[p];
    if (!w.out || p == kNoSlot) return;
    // find_or_insert: an occurrence returns its representative's row (local dedupe), or its key's
    // last occurrence's (global dedupe, when a key repeated)
    uint32_t src_pos = (uint32_t)i;
    if (w.local) {
        src_pos = p;
    } else if (w.ctr[kCtrDup]) {
        const DedupeEntry de = w.dd[p];
        src_pos = (de.claim > de.last ? de.claim : de.last) - 1;
    }
    if (src_pos != (uint32_t)i) {
        const uint4* src = reinterpret_cast<const uint4*>(w.out + (size_t)src_pos * dim);
        uint4* dst = reinterpret_cast<uint4*>(w.out + i * dim);
        for (uint32_t c = 0; c < (dim >> 2); ++c) dst[c] = src[c];
    }
}

template <int G>
static void launch_route(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys, const float* vals,
                         const uint64_t* scores, hipStream_t s) {
    if (w.local)
        k_route<G, true><<<blocks_for(n * G, 256), 256, 0, s>>>(t, w, n, keys, vals, scores);
    else
        k_route<G, false><<<blocks_for(n * G, 256), 256, 0, s>>>(t, w, n, keys, vals, scores);
}

hipError_t launch_upsert_prep(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                              const uint64_t* scores, const EvictOut& ev, size_t zero_bytes, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipError_t e = launch_fill_zero(w.dd, zero_bytes, s);
    if (e != hipSuccess) return e;
    k_dedupe<<<blocks_for(n, 256), 256, 0, s>>>(t, w, n, keys, scores, ev.count);
    return hipGetLastError();
}

hipError_t launch_upsert_route(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                               const float* vals, const uint64_t* scores, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (group) {
        case 4: launch_route<4>(t, w, n, keys, vals, scores, s); break;
        case 16: launch_route<16>(t, w, n, keys, vals, scores, s); break;
        default: launch_route<8>(t, w, n, keys, vals, scores, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_upsert_apply(const TableView& t, const UpsertWs& w, uint64_t n, const float* vals, const EvictOut& ev,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t visit = w.list_mode ? (n < t.nbuckets ? n : t.nbuckets) : t.nbuckets;
    // the one-thread commit pays off once the touched buckets are many; below that the fast apply
    // finishes plain buckets itself and the call saves a launch
    if (n > kCommitMinKeys) k_apply_commit<<<(unsigned)((visit + 255) / 256), 256, 0, s>>>(t, w);
    k_apply_fast<<<(unsigned)((visit + kApplyGroups - 1) / kApplyGroups), 256, 0, s>>>(t, w, vals, ev);
    uint64_t slow_blocks = n < t.nbuckets ? n : t.nbuckets;
    if (slow_blocks > 2048) slow_blocks = 2048;
    k_apply_slow<<<(unsigned)slow_blocks, 64, 0, s>>>(t, w, vals, ev);
    return hipGetLastError();
}

hipError_t launch_upsert_finish(const UpsertWs& w, uint64_t n, uint8_t* status, uint32_t dim, hipStream_t s) {
    if (n == 0 || (!status && !w.out)) return hipSuccess;
    k_finish<<<blocks_for(n, 256), 256, 0, s>>>(w, n, status, dim);
    return hipGetLastError();
}

hipError_t launch_upsert_rounds(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                                const float* vals, const uint64_t* scores, const EvictOut& ev, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t nblk = (n + 255) / 256;
    k_rank_count<<<(unsigned)nblk, 256, 0, s>>>(w, n);
    k_rank_scan<<<1, 256, 0, s>>>(w, nblk);
    k_rank_write<<<(unsigned)nblk, 256, 0, s>>>(w, n);
    hipError_t e = hipGetLastError();
    UpsertWs wr = w;
    for (int c = 0; c < w.rounds && e == hipSuccess; ++c) {
        wr.round = c;
        if (c > 0) {  // the previous round's overflow lists and slow / touched cursors
            if ((e = launch_fill_zero(w.okey, w.P * 8, s)) != hipSuccess) break;
            if ((e = launch_fill_zero(w.ctr + kCtrSlow, 2 * sizeof(uint32_t), s)) != hipSuccess) break;
        }
        if ((e = launch_upsert_route(t, wr, n, keys, vals, scores, group, s)) != hipSuccess) break;
        e = launch_upsert_apply(t, wr, n, vals, ev, s);
    }
    return e;
}

hipError_t launch_upsert(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys, const float* vals,
                         const uint64_t* scores, uint8_t* status, const EvictOut& ev, size_t zero_bytes, int group,
                         hipStream_t s) {
    hipError_t e;
    if (n == 0) return hipSuccess;
    if (w.rounds > 1) {
        if ((e = launch_upsert_prep(t, w, n, keys, scores, ev, zero_bytes, s)) != hipSuccess) return e;
        if ((e = launch_upsert_rounds(t, w, n, keys, vals, scores, ev, group, s)) != hipSuccess) return e;
        return launch_upsert_finish(w, n, status, t.dim, s);
    }
    // one route round: block-local dedupe, routing of the representatives, apply
    UpsertWs wl = w;
    wl.local = 1;
    uint4* zero = reinterpret_cast<uint4*>(w.dd);  // the dedupe pass clears the scratch (a multiple of 256 bytes)
    const unsigned nblk = (unsigned)((n + kLocalKeys - 1) / kLocalKeys);
    if (t.policy == 2)
        k_local_dedupe<true><<<nblk, kLocalThreads, 0, s>>>(wl, n, keys, scores, ev.count, zero, zero_bytes / 16);
    else
        k_local_dedupe<false><<<nblk, kLocalThreads, 0, s>>>(wl, n, keys, scores, ev.count, zero, zero_bytes / 16);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_upsert_route(t, wl, n, keys, vals, scores, group, s)) != hipSuccess) return e;
    if ((e = launch_upsert_apply(t, wl, n, vals, ev, s)) != hipSuccess) return e;
    return launch_upsert_finish(wl, n, status, t.dim, s);
}

}  // namespace cskv
