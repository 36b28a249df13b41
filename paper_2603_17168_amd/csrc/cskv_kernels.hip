// HIP kernels of the cache-semantic hash table for CDNA4 (gfx950, wave64).
//
// A key is served by a group of G lanes of one wave (G = 4, 8 or 16).  The group loads a
// bucket's 128-byte digest line with one 128/G-byte load per lane, compares the bytes with
// the key's digest using exact SWAR byte equality, and verifies candidates against the key
// line (Alg. 1).  Value rows move as 16-byte chunks spread over the group's lanes.
//
// An upsert batch runs as a fixed kernel sequence on one stream (Alg. 2 inside Alg. 3, under
// the batch order of the header):
//   zero    clear the call's scratch
//   dedupe  one set entry per distinct key: last occurrence (atomicMax), LFU increment sum
//   route   per distinct key, against the table as it was before the call: update slot, or
//           target bucket by phase D1 (occupancy) / D2 (minimum (score, key)); an atomic count
//           per target bucket gives each insert a rank
//   commit  updates in place; inserts into buckets whose incoming count fits their free slots
//           take the rank-th free slot of the pre-call digest line; contended buckets get a
//           region of the contended list and an entry in the contended-bucket list
//   scatter contended inserts into their bucket's region
//   apply   one wave per contended bucket: best-128 incoming by (score desc, key asc), the
//           residents ranked by (score asc, key asc), then every decision in parallel (an
//           incoming key j past the free slots is admitted iff its score beats the j-th
//           smallest resident), victims copied out, keys/digests/scores/rows written
//   finish  per-occurrence statuses; per-bucket counts back to zero
#include <hip/hip_runtime.h>

#include "cskv_internal.h"

namespace cskv {

// ------------------------------------------------------------------------------------------
// hashing (Sec. 3.1/3.2: a Murmur3-derived hash; here MurmurHash3's 64-bit finalizer)
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

struct KeyHash {
    uint32_t b1, b2, dg;
};

__device__ __forceinline__ KeyHash hash_key(const TableView& t, uint64_t k) {
    const uint64_t h = fmix64(k);
    KeyHash r;
    r.b1 = (uint32_t)h & t.bmask;
    r.b2 = t.dual ? ((uint32_t)(h >> 40) & t.bmask) : r.b1;
    uint32_t d = (uint32_t)(h >> 32) & 0xFFu;  // digest: bits 32..39; 0 marks an empty slot
    r.dg = d ? d : 1u;
    return r;
}

__device__ __forceinline__ bool reserved_key(uint64_t k) { return k == 0ull || k == ~0ull; }

// ------------------------------------------------------------------------------------------
// group helpers (G lanes of one wave)
template <int G>
__device__ __forceinline__ int glane() {
    return threadIdx.x & (G - 1);
}

template <int G>
__device__ __forceinline__ int gmax_i(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, G));
    return v;
}

template <int G>
__device__ __forceinline__ int gsum_i(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

template <int G>
__device__ __forceinline__ uint64_t gmin_u64(uint64_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        uint64_t x = __shfl_xor(v, o, G);
        v = x < v ? x : v;
    }
    return v;
}

// byte-equality of a 32-bit word with a broadcast byte: 4 result bits (byte q -> bit q)
__device__ __forceinline__ uint32_t match4(uint32_t w, uint32_t pat) {
    const uint32_t x = w ^ pat;
    const uint32_t nz = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // bit 7 of a byte = (byte != 0)
    const uint32_t z = ~nz & 0x80808080u;
    return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
}

// this lane's 128/G digest bytes of a bucket line, as 32-bit words
template <int G>
struct LineSeg {
    static constexpr int BYTES = 128 / G;
    static constexpr int NW = BYTES / 4;
    uint32_t w[NW];

    __device__ __forceinline__ void load(const uint8_t* line, int lane) {
        const uint8_t* p = line + lane * BYTES;
        if constexpr (NW == 8) {
            const uint4 a = *reinterpret_cast<const uint4*>(p);
            const uint4 b = *reinterpret_cast<const uint4*>(p + 16);
            w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
            w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
        } else if constexpr (NW == 4) {
            const uint4 a = *reinterpret_cast<const uint4*>(p);
            w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
        } else if constexpr (NW == 2) {
            const uint2 a = *reinterpret_cast<const uint2*>(p);
            w[0] = a.x; w[1] = a.y;
        } else {
            w[0] = *reinterpret_cast<const uint32_t*>(p);
        }
    }
    // bit j set <=> byte j of this lane's segment equals `byte`
    __device__ __forceinline__ uint32_t match(uint32_t byte) const {
        const uint32_t pat = byte * 0x01010101u;
        uint32_t m = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) m |= match4(w[q], pat) << (4 * q);
        return m;
    }
    __device__ __forceinline__ uint32_t empty_mask() const { return match(0u); }
};

// slot of key k in bucket b given the lane's candidate mask, or -1 (same value on all G lanes)
template <int G>
__device__ __forceinline__ int verify(const TableView& t, uint32_t b, uint32_t cand, uint64_t k, int lane) {
    int hit = -1;
    const uint64_t* bk = t.keys + (size_t)b * kSlots;
    while (cand) {
        const int j = __builtin_ctz(cand);
        cand &= cand - 1;
        const int slot = lane * LineSeg<G>::BYTES + j;
        if (bk[slot] == k) {
            hit = slot;
            break;
        }
    }
    return gmax_i<G>(hit);
}

// the rank-th free slot of a digest line (rank < number of free slots), on all G lanes
template <int G>
__device__ __forceinline__ int nth_free(uint32_t emask, int rank, int lane) {
    const int c = __popc(emask);
    int incl = c;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int tt = __shfl_up(incl, o, G);
        if (lane >= o) incl += tt;
    }
    const int excl = incl - c;
    int res = -1;
    if (rank >= excl && rank < incl) {
        uint32_t m = emask;
        for (int q = 0; q < rank - excl; ++q) m &= m - 1;
        res = lane * LineSeg<G>::BYTES + __builtin_ctz(m);
    }
    return gmax_i<G>(res);
}

// minimum (score, key) of a full bucket, on all G lanes.  Lane l reads 16-byte chunks
// l, l+G, l+2G, ... of the score line so that each load of the group is one contiguous span.
template <int G>
__device__ __forceinline__ void bucket_min(const TableView& t, uint32_t b, int lane, uint64_t& ms, uint64_t& mk) {
    constexpr int CH = 64 / G;  // 16-byte chunks (2 scores) per lane
    const ulonglong2* sp = reinterpret_cast<const ulonglong2*>(t.scores + (size_t)b * kSlots);
    uint64_t sc[2 * CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const ulonglong2 v = sp[q * G + lane];
        sc[2 * q] = v.x;
        sc[2 * q + 1] = v.y;
    }
    uint64_t m = ~0ull;
#pragma unroll
    for (int q = 0; q < 2 * CH; ++q) m = sc[q] < m ? sc[q] : m;
    m = gmin_u64<G>(m);
    uint64_t km = ~0ull;
    const uint64_t* bk = t.keys + (size_t)b * kSlots;
#pragma unroll
    for (int q = 0; q < 2 * CH; ++q) {
        if (sc[q] == m) {
            const uint64_t kk = bk[2 * ((q >> 1) * G + lane) + (q & 1)];
            km = kk < km ? kk : km;
        }
    }
    ms = m;
    mk = gmin_u64<G>(km);
}

// copy one dim-wide row with the group's lanes (16 bytes per lane per step)
template <int G>
__device__ __forceinline__ void copy_row(float* __restrict__ dst, const float* __restrict__ src, uint32_t dim, int lane) {
    const uint32_t chunks = dim >> 2;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    for (uint32_t c = lane; c < chunks; c += G) d[c] = s[c];
}

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
    const uint64_t s = a + b;
    return s < a ? ~0ull : s;
}

// ------------------------------------------------------------------------------------------
// zero fill (used instead of hipMemsetAsync so that every call can be graph-captured)
__global__ void __launch_bounds__(256) k_fill_zero(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    k_fill_zero<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<uint4*>(p), n16,
                                                  reinterpret_cast<uint8_t*>(p) + n16 * 16, ntail);
    return hipGetLastError();
}

hipError_t launch_clear_table(const TableView& t, hipStream_t s) {
    hipError_t e;
    if ((e = launch_fill_zero(t.dig, t.nbuckets * kSlots, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(t.keys, t.nbuckets * kSlots * 8, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(t.scores, t.nbuckets * kSlots * 8, s)) != hipSuccess) return e;
    return launch_fill_zero(t.cnt, t.nbuckets * 4, s);
}

// ------------------------------------------------------------------------------------------
// find (Alg. 1; dual mode probes b2 after a miss in b1)
template <int G>
__global__ void __launch_bounds__(256) k_find(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
                                              float* __restrict__ out, uint8_t* __restrict__ found,
                                              uint64_t* __restrict__ scores_out) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    const uint64_t k = keys[i];
    int slot = -1;
    uint32_t b = 0;
    if (!reserved_key(k)) {
        const KeyHash h = hash_key(t, k);
        LineSeg<G> seg;
        seg.load(t.dig + (size_t)h.b1 * kSlots, lane);
        b = h.b1;
        slot = verify<G>(t, h.b1, seg.match(h.dg), k, lane);
        if (slot < 0 && h.b2 != h.b1) {
            seg.load(t.dig + (size_t)h.b2 * kSlots, lane);
            b = h.b2;
            slot = verify<G>(t, h.b2, seg.match(h.dg), k, lane);
        }
    }
    if (slot >= 0) {
        const size_t e = (size_t)b * kSlots + slot;
        copy_row<G>(out + i * t.dim, t.vals + e * t.dim, t.dim, lane);
        if (lane == 0) {
            found[i] = 1;
            if (scores_out) scores_out[i] = t.scores[e];
        }
    } else if (lane == 0) {
        found[i] = 0;
    }
}

hipError_t launch_find(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                       uint64_t* scores_out, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t threads = n * (uint64_t)group;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    switch (group) {
        case 4: k_find<4><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
        case 16: k_find<16><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
        default: k_find<8><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// upsert: dedupe (one thread per input key)
__global__ void __launch_bounds__(256) k_dedupe(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                                const uint64_t* __restrict__ scores) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (reserved_key(k)) {
        w.slot_of[i] = kNoSlot;
        return;
    }
    const uint64_t mask = w.P - 1;
    uint64_t p = (fmix64(k) * 0x9E3779B97F4A7C15ull) >> (64 - w.logP);
    for (;;) {
        const uint64_t cur = w.skeys[p];
        if (cur == k) break;
        if (cur == 0) {
            const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(w.skeys + p), 0ull,
                                                     (unsigned long long)k);
            if (old == 0ull || old == k) break;
        }
        p = (p + 1) & mask;
    }
    w.slot_of[i] = (uint32_t)p;
    atomicMax(w.slast + p, (uint32_t)(i + 1));
    if (t.policy == 2) {  // LFU: saturating sum of the increments
        const uint64_t inc = scores ? scores[i] : 1ull;
        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(w.sinc + p),
                                                 (unsigned long long)inc);
        if (old + inc < old) atomicOr(w.ssat + p, 1u);
    }
}

// upsert: route (G lanes per input position; only last occurrences act)
template <int G>
__global__ void __launch_bounds__(256) k_route(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                               const uint64_t* __restrict__ scores, uint64_t clock) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    const uint32_t p = w.slot_of[i];
    if (p == kNoSlot || w.slast[p] != (uint32_t)(i + 1)) {
        if (lane == 0) w.op_kind[i] = kOpNone;
        return;
    }
    const uint64_t k = keys[i];
    const KeyHash h = hash_key(t, k);
    uint64_t inc = 0;
    if (t.policy == 2) inc = w.ssat[p] ? ~0ull : w.sinc[p];

    LineSeg<G> s1, s2;
    s1.load(t.dig + (size_t)h.b1 * kSlots, lane);
    int slot = verify<G>(t, h.b1, s1.match(h.dg), k, lane);
    uint32_t ub = h.b1;
    const bool two = h.b2 != h.b1;
    if (slot < 0 && two) {
        s2.load(t.dig + (size_t)h.b2 * kSlots, lane);
        slot = verify<G>(t, h.b2, s2.match(h.dg), k, lane);
        ub = h.b2;
    }
    if (slot >= 0) {  // UPDATE in place
        if (lane == 0) {
            uint64_t ns;
            if (t.policy == 0) ns = scores[i];
            else if (t.policy == 1) ns = clock;
            else ns = sat_add(t.scores[(size_t)ub * kSlots + slot], inc);
            w.op_kind[i] = kOpUpdate;
            w.op_tgt[i] = ub;
            w.op_aux[i] = (uint32_t)slot;
            w.op_score[i] = ns;
        }
        return;
    }
    // INSERT: choose the target bucket
    const uint32_t e1 = s1.empty_mask();
    const int occ1 = kSlots - gsum_i<G>(__popc(e1));
    uint32_t tgt = h.b1, emask = e1;
    int occ = occ1;
    if (two) {
        const uint32_t e2 = s2.empty_mask();
        const int occ2 = kSlots - gsum_i<G>(__popc(e2));
        if (occ1 < kSlots || occ2 < kSlots) {  // phase D1: less occupied, b1 on a tie
            if (occ2 < occ1) {
                tgt = h.b2; emask = e2; occ = occ2;
            }
        } else {  // phase D2: smaller minimum (score, key)
            uint64_t m1s, m1k, m2s, m2k;
            bucket_min<G>(t, h.b1, lane, m1s, m1k);
            bucket_min<G>(t, h.b2, lane, m2s, m2k);
            if (m2s < m1s || (m2s == m1s && m2k < m1k)) {
                tgt = h.b2; emask = e2; occ = occ2;
            }
        }
    }
    int rank = 0;
    if (lane == 0) rank = (int)atomicAdd(t.cnt + tgt, 1u);
    rank = __shfl(rank, 0, G);
    const int nfree = kSlots - occ;
    int fslot = 0xFF;
    if (rank < nfree) fslot = nth_free<G>(emask, rank, lane);
    if (lane == 0) {
        uint64_t ns;
        if (t.policy == 0) ns = scores[i];
        else if (t.policy == 1) ns = clock;
        else ns = inc;
        w.op_kind[i] = kOpInsert;
        w.op_tgt[i] = tgt;
        w.op_aux[i] = ((uint32_t)rank << 8) | (uint32_t)(fslot & 0xFF);
        w.op_score[i] = ns;
        t.freeb[tgt] = (uint8_t)nfree;  // same value from every key routed here
    }
}

// upsert: commit updates and uncontended inserts; allocate contended regions
template <int G>
__global__ void __launch_bounds__(256) k_commit(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                                const float* __restrict__ vals) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    const uint8_t kind = w.op_kind[i];
    if (kind == kOpNone) return;
    const uint32_t tgt = w.op_tgt[i];
    const uint32_t aux = w.op_aux[i];
    if (kind == kOpUpdate) {
        const size_t e = (size_t)tgt * kSlots + aux;
        copy_row<G>(t.vals + e * t.dim, vals + i * t.dim, t.dim, lane);
        if (lane == 0) {
            t.scores[e] = w.op_score[i];
            w.sstat[w.slot_of[i]] = 1;  // UPDATED
        }
        return;
    }
    const uint32_t m = t.cnt[tgt];
    const uint32_t nfree = t.freeb[tgt];
    if (m <= nfree) {  // every insert of this bucket has its own free slot
        const uint64_t k = keys[i];
        const size_t e = (size_t)tgt * kSlots + (aux & 0xFF);
        copy_row<G>(t.vals + e * t.dim, vals + i * t.dim, t.dim, lane);
        if (lane == 0) {
            t.keys[e] = k;
            t.scores[e] = w.op_score[i];
            t.dig[e] = (uint8_t)hash_key(t, k).dg;
            w.sstat[w.slot_of[i]] = 2;  // INSERTED
        }
        return;
    }
    if (lane == 0 && (aux >> 8) == 0) {  // first insert of a contended bucket allocates its region
        t.cbase[tgt] = atomicAdd(w.ctr + kCtrListFill, m);
        const uint32_t ci = atomicAdd(w.ctr + kCtrContended, 1u);
        w.clist[ci] = tgt;
    }
}

// upsert: scatter contended inserts into their bucket's region
__global__ void __launch_bounds__(256) k_scatter(TableView t, UpsertWs w, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || w.op_kind[i] != kOpInsert) return;
    const uint32_t tgt = w.op_tgt[i];
    if (t.cnt[tgt] <= t.freeb[tgt]) return;
    w.glist[t.cbase[tgt] + (w.op_aux[i] >> 8)] = (uint32_t)i;
}

// upsert: one wave per contended bucket
__global__ void __launch_bounds__(64) k_apply(TableView t, UpsertWs w, const uint64_t* __restrict__ keys,
                                              const float* __restrict__ vals, EvictOut ev) {
    __shared__ uint64_t cs[192], ck[192];  // incoming candidates: score, key
    __shared__ uint32_t cp[192];           // input position
    __shared__ uint64_t ns_[128], nk_[128];
    __shared__ uint32_t np_[128];
    __shared__ uint64_t S_[128], K_[128];  // residents by slot
    __shared__ uint64_t rs[128], rk[128];  // smallest residents in (score, key) order
    __shared__ uint8_t rslot[128];
    __shared__ uint8_t elist[128];         // free slots
    __shared__ uint8_t dslot[128];         // slot taken by admitted item j
    __shared__ unsigned long long ev_base_s;

    const int lane = threadIdx.x;
    const uint32_t ncont = w.ctr[kCtrContended];
    for (uint32_t ci = blockIdx.x; ci < ncont; ci += gridDim.x) {
        const uint32_t b = w.clist[ci];
        const uint32_t m = t.cnt[b];
        const uint32_t base = t.cbase[b];

        // 1. best min(m,128) incoming keys, sorted by (score desc, key asc)
        int nbest = 0;
        for (uint32_t c0 = 0; c0 < m; c0 += 64) {
            const int cn = (int)min(64u, m - c0);
            if (lane < cn) {
                const uint32_t pos = w.glist[base + c0 + lane];
                cp[nbest + lane] = pos;
                ck[nbest + lane] = keys[pos];
                cs[nbest + lane] = w.op_score[pos];
            }
            __syncthreads();
            const int tot = nbest + cn;
            int r[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int j = lane + 64 * q;
                r[q] = -1;
                if (j < tot) {
                    const uint64_t s = cs[j], k = ck[j];
                    int rr = 0;
                    for (int x = 0; x < tot; ++x) {
                        const uint64_t sx = cs[x];
                        rr += (sx > s) || (sx == s && ck[x] < k);
                    }
                    r[q] = rr;
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int j = lane + 64 * q;
                if (j < tot) {
                    if (r[q] < 128) {
                        ns_[r[q]] = cs[j];
                        nk_[r[q]] = ck[j];
                        np_[r[q]] = cp[j];
                    } else {
                        w.sstat[w.slot_of[cp[j]]] = 4;  // REJECTED: 128 better keys target this bucket
                    }
                }
            }
            __syncthreads();
            nbest = min(tot, 128);
            for (int j = lane; j < nbest; j += 64) {
                cs[j] = ns_[j];
                ck[j] = nk_[j];
                cp[j] = np_[j];
            }
            __syncthreads();
        }

        // 2. residents: occupancy, free-slot list, smallest (score, key) entries
        const size_t eb = (size_t)b * kSlots;
        const bool o0 = t.dig[eb + lane] != 0;
        const bool o1 = t.dig[eb + lane + 64] != 0;
        const uint64_t bal0 = __ballot(o0), bal1 = __ballot(o1);
        const int occ = __popcll(bal0) + __popcll(bal1);
        const int nfree = kSlots - occ;
        const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
        if (!o0) elist[__popcll(~bal0 & below)] = (uint8_t)lane;
        if (!o1) elist[__popcll(~bal0) + __popcll(~bal1 & below)] = (uint8_t)(lane + 64);
        const int need = nbest - nfree;  // > 0 for a contended bucket unless it was empty
        if (need > 0) {
            S_[lane] = o0 ? t.scores[eb + lane] : ~0ull;
            K_[lane] = o0 ? t.keys[eb + lane] : ~0ull;
            S_[lane + 64] = o1 ? t.scores[eb + lane + 64] : ~0ull;
            K_[lane + 64] = o1 ? t.keys[eb + lane + 64] : ~0ull;
        }
        __syncthreads();
        if (need > 0) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int sl = lane + 64 * q;
                if (!(q ? o1 : o0)) continue;
                const uint64_t s = S_[sl], k = K_[sl];
                int rr = 0;
                for (int x = 0; x < kSlots; ++x) {
                    const uint64_t sx = S_[x];
                    rr += (sx < s) || (sx == s && K_[x] < k);  // empty slots sort last (~0, ~0)
                }
                if (rr < need) {
                    rs[rr] = s;
                    rk[rr] = k;
                    rslot[rr] = (uint8_t)sl;
                }
            }
        }
        __syncthreads();

        // 3. decisions: item j takes free slot j, or competes with the (j-nfree)-th smallest resident
        bool adm[2];
        uint8_t st[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = lane + 64 * q;
            adm[q] = false;
            st[q] = 0;
            if (j < nbest) {
                if (j < nfree) {
                    adm[q] = true;
                    st[q] = 2;  // INSERTED
                    dslot[j] = elist[j];
                } else {
                    const int v = j - nfree;
                    if (v < occ && cs[j] > rs[v]) {
                        adm[q] = true;
                        st[q] = 3;  // INSERTED_EVICT
                        dslot[j] = rslot[v];
                    } else {
                        st[q] = 4;  // REJECTED
                    }
                }
            }
        }
        const int nadm = __popcll(__ballot(adm[0])) + __popcll(__ballot(adm[1]));
        const int nev = nadm > nfree ? nadm - nfree : 0;
        if (lane == 0) ev_base_s = (ev.count && nev) ? atomicAdd(reinterpret_cast<unsigned long long*>(ev.count),
                                                                 (unsigned long long)nev)
                                                     : 0ull;
        __syncthreads();
        const uint64_t ev_base = ev_base_s;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = lane + 64 * q;
            if (j >= nbest) continue;
            w.sstat[w.slot_of[cp[j]]] = st[q];
            if (!adm[q]) continue;
            const size_t e = eb + dslot[j];
            if (st[q] == 3 && ev.keys) {
                const uint64_t x = ev_base + (uint64_t)(j - nfree);
                ev.keys[x] = rk[j - nfree];
                ev.scores[x] = rs[j - nfree];
            }
            const uint64_t k = ck[j];
            t.keys[e] = k;
            t.scores[e] = cs[j];
            t.dig[e] = (uint8_t)hash_key(t, k).dg;
        }
        // 4. value rows: victims copied out first, then the new rows written
        const uint32_t chunks = t.dim >> 2;
        const uint32_t total = (uint32_t)nadm * chunks;
        for (uint32_t x = lane; x < total; x += 64) {
            const uint32_t j = x / chunks, c = x - j * chunks;
            uint4* row = reinterpret_cast<uint4*>(t.vals + (eb + dslot[j]) * t.dim) + c;
            if ((int)j >= nfree && ev.vals) {
                const uint64_t xe = ev_base + (uint64_t)(j - nfree);
                reinterpret_cast<uint4*>(ev.vals + xe * t.dim)[c] = *row;
            }
            *row = reinterpret_cast<const uint4*>(vals + (size_t)cp[j] * t.dim)[c];
        }
        __syncthreads();
    }
}

// upsert: per-occurrence status, reset of the per-bucket counts
__global__ void __launch_bounds__(256) k_finish(TableView t, UpsertWs w, uint64_t n, uint8_t* __restrict__ status) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = w.slot_of[i];
    if (status) status[i] = (p == kNoSlot) ? 5 : w.sstat[p];
    if (p != kNoSlot && w.op_kind[i] == kOpInsert) t.cnt[w.op_tgt[i]] = 0;
}

static inline unsigned blocks_for(uint64_t threads, unsigned bs) { return (unsigned)((threads + bs - 1) / bs); }

template <int G>
static void launch_route_commit(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                                const float* vals, const uint64_t* scores, uint64_t clock, hipStream_t s) {
    const unsigned nb = blocks_for(n * G, 256);
    k_route<G><<<nb, 256, 0, s>>>(t, w, n, keys, scores, clock);
    k_commit<G><<<nb, 256, 0, s>>>(t, w, n, keys, vals);
}

hipError_t launch_upsert(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                         const float* vals, const uint64_t* scores, uint8_t* status, const EvictOut& ev,
                         uint64_t clock, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipError_t e;
    // scratch: dedupe set keys + last + (LFU sums) and the counters; evicted count
    if ((e = launch_fill_zero(w.skeys, w.P * 8, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(w.slast, w.P * 4, s)) != hipSuccess) return e;
    if (t.policy == 2) {
        if ((e = launch_fill_zero(w.sinc, w.P * 8, s)) != hipSuccess) return e;
        if ((e = launch_fill_zero(w.ssat, w.P * 4, s)) != hipSuccess) return e;
    }
    if ((e = launch_fill_zero(w.ctr, 64 * 4, s)) != hipSuccess) return e;
    if (ev.count && (e = launch_fill_zero(ev.count, 8, s)) != hipSuccess) return e;
    k_dedupe<<<blocks_for(n, 256), 256, 0, s>>>(t, w, n, keys, scores);
    switch (group) {
        case 4: launch_route_commit<4>(t, w, n, keys, vals, scores, clock, s); break;
        case 16: launch_route_commit<16>(t, w, n, keys, vals, scores, clock, s); break;
        default: launch_route_commit<8>(t, w, n, keys, vals, scores, clock, s); break;
    }
    k_scatter<<<blocks_for(n, 256), 256, 0, s>>>(t, w, n);
    uint64_t apply_blocks = n < t.nbuckets ? n : t.nbuckets;
    if (apply_blocks > 16384) apply_blocks = 16384;
    k_apply<<<(unsigned)apply_blocks, 64, 0, s>>>(t, w, keys, vals, ev);
    k_finish<<<blocks_for(n, 256), 256, 0, s>>>(t, w, n, status);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// erase: probe against the pre-call table, then clear (two kernels so that duplicates of a key
// all see it present)
template <int G>
__global__ void __launch_bounds__(256) k_erase_probe(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
                                                     uint8_t* __restrict__ erased, uint32_t* __restrict__ ws_slot) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    const uint64_t k = keys[i];
    int slot = -1;
    uint32_t b = 0;
    if (!reserved_key(k)) {
        const KeyHash h = hash_key(t, k);
        LineSeg<G> seg;
        seg.load(t.dig + (size_t)h.b1 * kSlots, lane);
        b = h.b1;
        slot = verify<G>(t, h.b1, seg.match(h.dg), k, lane);
        if (slot < 0 && h.b2 != h.b1) {
            seg.load(t.dig + (size_t)h.b2 * kSlots, lane);
            b = h.b2;
            slot = verify<G>(t, h.b2, seg.match(h.dg), k, lane);
        }
    }
    if (lane == 0) {
        ws_slot[i] = slot >= 0 ? (uint32_t)(b * kSlots + slot) : kNoSlot;
        if (erased) erased[i] = slot >= 0;
    }
}

__global__ void __launch_bounds__(256) k_erase_clear(TableView t, uint64_t n, const uint32_t* __restrict__ ws_slot) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = ws_slot[i];
    if (e == kNoSlot) return;
    t.dig[e] = 0;
    t.keys[e] = 0;
    t.scores[e] = 0;
}

hipError_t launch_erase(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased, uint32_t* ws_slot,
                        int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned nb = blocks_for(n * group, 256);
    switch (group) {
        case 4: k_erase_probe<4><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
        case 16: k_erase_probe<16><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
        default: k_erase_probe<8><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
    }
    k_erase_clear<<<blocks_for(n, 256), 256, 0, s>>>(t, n, ws_slot);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// size: occupied digests summed per block, one atomic per block
__global__ void __launch_bounds__(256) k_size(TableView t, uint64_t* __restrict__ out) {
    __shared__ unsigned int part[4];
    const uint64_t nwords = t.nbuckets * (kSlots / 16);
    const uint4* d = reinterpret_cast<const uint4*>(t.dig);
    unsigned int c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = d[i];
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) c += 4 - __popc(match4(w4[q], 0u));
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = (unsigned long long)part[0] + part[1] + part[2] + part[3];
        if (tot) atomicAdd(reinterpret_cast<unsigned long long*>(out), tot);
    }
}

hipError_t launch_size(const TableView& t, uint64_t* d_size, hipStream_t s) {
    hipError_t e = launch_fill_zero(d_size, 8, s);
    if (e != hipSuccess) return e;
    uint64_t blocks = (t.nbuckets * 8 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_size<<<(unsigned)blocks, 256, 0, s>>>(t, d_size);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// export: one wave per bucket; output positions from one atomic per bucket
__global__ void __launch_bounds__(64) k_export(TableView t, uint64_t b0, uint64_t b1, uint64_t* __restrict__ keys,
                                               float* __restrict__ vals, uint64_t* __restrict__ scores,
                                               uint64_t* __restrict__ slots, uint64_t* __restrict__ count) {
    __shared__ unsigned long long base_s;
    __shared__ uint8_t sl[128];
    const int lane = threadIdx.x;
    for (uint64_t b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
        const size_t eb = (size_t)b * kSlots;
        const bool o0 = t.dig[eb + lane] != 0, o1 = t.dig[eb + lane + 64] != 0;
        const uint64_t bal0 = __ballot(o0), bal1 = __ballot(o1);
        const int c = __popcll(bal0) + __popcll(bal1);
        const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
        if (o0) sl[__popcll(bal0 & below)] = (uint8_t)lane;
        if (o1) sl[__popcll(bal0) + __popcll(bal1 & below)] = (uint8_t)(lane + 64);
        if (lane == 0) base_s = c ? atomicAdd(reinterpret_cast<unsigned long long*>(count), (unsigned long long)c) : 0ull;
        __syncthreads();
        const uint64_t base = base_s;
        for (int j = lane; j < c; j += 64) {
            const size_t e = eb + sl[j];
            keys[base + j] = t.keys[e];
            if (scores) scores[base + j] = t.scores[e];
            if (slots) slots[base + j] = e;
        }
        if (vals) {
            const uint32_t chunks = t.dim >> 2;
            for (uint32_t x = lane; x < (uint32_t)c * chunks; x += 64) {
                const uint32_t j = x / chunks, cc = x - j * chunks;
                reinterpret_cast<uint4*>(vals + (base + j) * t.dim)[cc] =
                    reinterpret_cast<const uint4*>(t.vals + (eb + sl[j]) * t.dim)[cc];
            }
        }
        __syncthreads();
    }
}

hipError_t launch_export(const TableView& t, uint64_t b0, uint64_t b1, uint64_t* keys, float* vals,
                         uint64_t* scores, uint64_t* slots, uint64_t* count, hipStream_t s) {
    hipError_t e = launch_fill_zero(count, 8, s);
    if (e != hipSuccess || b1 <= b0) return e;
    uint64_t blocks = b1 - b0;
    if (blocks > 65536) blocks = 65536;
    k_export<<<(unsigned)blocks, 64, 0, s>>>(t, b0, b1, keys, vals, scores, slots, count);
    return hipGetLastError();
}

}  // namespace cskv
