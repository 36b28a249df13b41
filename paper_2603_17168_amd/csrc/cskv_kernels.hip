// HIP kernels of the cache-semantic hash table for CDNA4 (gfx950, wave64): find, erase, size,
// export and the zero fill.  The upsert kernels live in cskv_upsert.hip.
//
// A key is served by a group of G lanes of one wave (G = 4, 8 or 16).  The group loads a
// bucket's 128-byte digest line with one 128/G-byte load per lane, compares the bytes with
// the key's digest using exact SWAR byte equality, and verifies candidates against the key
// line (Alg. 1).  Value rows move as 16-byte chunks spread over the group's lanes.
#include <hip/hip_runtime.h>

#include "cskv_device.h"
#include "cskv_internal.h"

namespace cskv {

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
    if ((e = launch_fill_zero(t.bmin, t.nbuckets * 16, s)) != hipSuccess) return e;
    return launch_fill_zero(t.cnt, t.nbuckets * 4, s);
}

// ------------------------------------------------------------------------------------------
// find (Alg. 1; dual mode probes b2 after a miss in b1).  With PRE the b2 line is loaded
// together with the b1 line (one round trip less on b2 hits and misses, 128 B more per b1 hit).
template <int G, bool PRE>
__device__ __forceinline__ void find_one(const TableView& t, uint64_t k, float* __restrict__ out_row,
                                         uint8_t* __restrict__ found, uint64_t* __restrict__ score_out, int lane) {
    int slot = -1;
    uint32_t b = 0;
    if (!reserved_key(k)) {
        const KeyHash h = hash_key(t, k);
        LineSeg<G> s1, s2;
        s1.load(t.dig + (size_t)h.b1 * kSlots, lane);
        if (PRE && h.b2 != h.b1) s2.load(t.dig + (size_t)h.b2 * kSlots, lane);
        b = h.b1;
        slot = verify<G>(t, h.b1, s1.match(h.dg), k, lane);
        if (slot < 0 && h.b2 != h.b1) {
            if (!PRE) s2.load(t.dig + (size_t)h.b2 * kSlots, lane);
            b = h.b2;
            slot = verify<G>(t, h.b2, s2.match(h.dg), k, lane);
        }
    }
    if (slot >= 0) {
        const size_t e = (size_t)b * kSlots + slot;
        copy_row<G>(out_row, t.vals + e * t.dim, t.dim, lane);
        if (lane == 0) {
            *found = 1;
            if (score_out) *score_out = t.scores[e];
        }
    } else if (lane == 0) {
        *found = 0;
    }
}

// Two keys per lane group, their dependent loads interleaved (digest lines, first candidate keys,
// rows), so a wave keeps twice as many independent accesses in flight.  Candidates beyond the
// first digest match of a lane (about 1/256 per occupied slot) are verified one by one.
template <int G>
__device__ __forceinline__ void verify_pair(const TableView& t, uint32_t bA, uint32_t cA, uint64_t kA, uint32_t bB,
                                            uint32_t cB, uint64_t kB, int lane, int& slotA, int& slotB) {
    constexpr int BY = LineSeg<G>::BYTES;
    const int jA = cA ? __builtin_ctz(cA) : -1;
    const int jB = cB ? __builtin_ctz(cB) : -1;
    const uint64_t xA = jA >= 0 ? t.keys[(size_t)bA * kSlots + lane * BY + jA] : 0ull;
    const uint64_t xB = jB >= 0 ? t.keys[(size_t)bB * kSlots + lane * BY + jB] : 0ull;
    int hA = (jA >= 0 && xA == kA) ? lane * BY + jA : -1;
    int hB = (jB >= 0 && xB == kB) ? lane * BY + jB : -1;
    if (hA < 0 && jA >= 0) {
        for (uint32_t c = cA & (cA - 1); c; c &= c - 1) {
            const int j = __builtin_ctz(c);
            if (t.keys[(size_t)bA * kSlots + lane * BY + j] == kA) {
                hA = lane * BY + j;
                break;
            }
        }
    }
    if (hB < 0 && jB >= 0) {
        for (uint32_t c = cB & (cB - 1); c; c &= c - 1) {
            const int j = __builtin_ctz(c);
            if (t.keys[(size_t)bB * kSlots + lane * BY + j] == kB) {
                hB = lane * BY + j;
                break;
            }
        }
    }
    slotA = gmax_i<G>(hA);
    slotB = gmax_i<G>(hB);
}

template <int G, bool PRE>
__device__ __forceinline__ void find_pair(const TableView& t, uint64_t kA, uint64_t kB, bool hasB, float* __restrict__ outA,
                                          float* __restrict__ outB, uint8_t* __restrict__ fA, uint8_t* __restrict__ fB,
                                          uint64_t* __restrict__ sA, uint64_t* __restrict__ sB, int lane) {
    const bool vA = !reserved_key(kA), vB = hasB && !reserved_key(kB);
    const KeyHash hA = hash_key(t, vA ? kA : 1ull), hB = hash_key(t, vB ? kB : 1ull);
    LineSeg<G> a1, b1, a2, b2;
    a1.load(t.dig + (size_t)hA.b1 * kSlots, lane);
    b1.load(t.dig + (size_t)hB.b1 * kSlots, lane);
    if (PRE) {
        a2.load(t.dig + (size_t)hA.b2 * kSlots, lane);
        b2.load(t.dig + (size_t)hB.b2 * kSlots, lane);
    }
    int slA, slB;
    verify_pair<G>(t, hA.b1, vA ? a1.match(hA.dg) : 0u, kA, hB.b1, vB ? b1.match(hB.dg) : 0u, kB, lane, slA, slB);
    uint32_t bkA = hA.b1, bkB = hB.b1;
    const bool missA = vA && slA < 0 && hA.b2 != hA.b1;
    const bool missB = vB && slB < 0 && hB.b2 != hB.b1;
    if (missA || missB) {
        if (!PRE) {
            if (missA) a2.load(t.dig + (size_t)hA.b2 * kSlots, lane);
            if (missB) b2.load(t.dig + (size_t)hB.b2 * kSlots, lane);
        }
        int s2A, s2B;
        verify_pair<G>(t, hA.b2, missA ? a2.match(hA.dg) : 0u, kA, hB.b2, missB ? b2.match(hB.dg) : 0u, kB, lane, s2A,
                       s2B);
        if (missA) {
            slA = s2A;
            bkA = hA.b2;
        }
        if (missB) {
            slB = s2B;
            bkB = hB.b2;
        }
    }
    // rows: both reads issued before the writes
    const uint32_t chunks = t.dim >> 2;
    const uint4* srcA = reinterpret_cast<const uint4*>(t.vals + ((size_t)bkA * kSlots + (slA < 0 ? 0 : slA)) * t.dim);
    const uint4* srcB = reinterpret_cast<const uint4*>(t.vals + ((size_t)bkB * kSlots + (slB < 0 ? 0 : slB)) * t.dim);
    uint4* dA = reinterpret_cast<uint4*>(outA);
    uint4* dB = reinterpret_cast<uint4*>(outB);
    for (uint32_t c = lane; c < chunks; c += G) {
        uint4 xa = make_uint4(0, 0, 0, 0), xb = make_uint4(0, 0, 0, 0);
        if (slA >= 0) xa = srcA[c];
        if (slB >= 0) xb = srcB[c];
        if (slA >= 0) dA[c] = xa;
        if (slB >= 0) dB[c] = xb;
    }
    if (lane == 0) {
        *fA = slA >= 0;
        if (sA && slA >= 0) *sA = t.scores[(size_t)bkA * kSlots + slA];
        if (hasB) {
            *fB = slB >= 0;
            if (sB && slB >= 0) *sB = t.scores[(size_t)bkB * kSlots + slB];
        }
    }
}

template <int G, bool PRE>
__global__ void __launch_bounds__(256) k_find_x2(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
                                                 float* __restrict__ out, uint8_t* __restrict__ found,
                                                 uint64_t* __restrict__ scores_out) {
    const uint64_t i = 2 * (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G);
    if (i >= n) return;
    const bool hasB = i + 1 < n;
    find_pair<G, PRE>(t, keys[i], hasB ? keys[i + 1] : 0ull, hasB, out + i * t.dim, out + (i + 1) * t.dim, found + i,
                      found + i + 1, scores_out ? scores_out + i : nullptr, scores_out ? scores_out + i + 1 : nullptr,
                      glane<G>());
}

template <int G, bool PRE>
__global__ void __launch_bounds__(256) k_find(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
                                              float* __restrict__ out, uint8_t* __restrict__ found,
                                              uint64_t* __restrict__ scores_out) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    find_one<G, PRE>(t, keys[i], out + i * t.dim, found + i, scores_out ? scores_out + i : nullptr, glane<G>());
}

// a merged run of find batches (readers never conflict, Sec. 3.5): a persistent grid strides over
// the concatenated keys; each key finds its batch by binary search over the batch offsets
template <int G, bool PRE>
__global__ void __launch_bounds__(256) k_find_multi(TableView t, const FindDesc* __restrict__ d, uint32_t nd,
                                                    uint64_t total) {
    const uint64_t ngroups = ((uint64_t)gridDim.x * blockDim.x) / G;
    const int lane = glane<G>();
    for (uint64_t gi = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; gi < total; gi += ngroups) {
        uint32_t lo = 0, hi = nd - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (d[mid].begin <= gi) lo = mid;
            else hi = mid - 1;
        }
        const FindDesc& q = d[lo];
        const uint64_t i = gi - q.begin;
        find_one<G, PRE>(t, q.keys[i], q.out + i * t.dim, q.found + i, q.scores ? q.scores + i : nullptr, lane);
    }
}

// a merged run whose descriptors travel as kernel arguments (serving loop)
template <int G, bool PRE>
__global__ void __launch_bounds__(256) k_find_args(TableView t, FindDescArgs a) {
    const uint64_t gi = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (gi >= a.total) return;
    uint32_t lo = 0, hi = a.nd - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (a.d[mid].begin <= gi) lo = mid;
        else hi = mid - 1;
    }
    const FindDesc& q = a.d[lo];
    const uint64_t i = gi - q.begin;
    find_one<G, PRE>(t, q.keys[i], q.out + i * t.dim, q.found + i, q.scores ? q.scores + i : nullptr, glane<G>());
}

hipError_t launch_find_args(const TableView& t, const FindDescArgs& a, int group, int prefetch_b2, hipStream_t s) {
    if (a.total == 0 || a.nd == 0) return hipSuccess;
    const unsigned blocks = blocks_for(a.total * (uint64_t)group, 256);
    const bool pre = prefetch_b2 != 0;
    switch (group) {
        case 4: pre ? k_find_args<4, true><<<blocks, 256, 0, s>>>(t, a) : k_find_args<4, false><<<blocks, 256, 0, s>>>(t, a); break;
        case 16: pre ? k_find_args<16, true><<<blocks, 256, 0, s>>>(t, a) : k_find_args<16, false><<<blocks, 256, 0, s>>>(t, a); break;
        default: pre ? k_find_args<8, true><<<blocks, 256, 0, s>>>(t, a) : k_find_args<8, false><<<blocks, 256, 0, s>>>(t, a); break;
    }
    return hipGetLastError();
}

template <int G>
static void launch_find_multi_g(const TableView& t, const FindDesc* d, uint32_t nd, uint64_t total, bool pre,
                                unsigned blocks, hipStream_t s) {
    if (pre) k_find_multi<G, true><<<blocks, 256, 0, s>>>(t, d, nd, total);
    else k_find_multi<G, false><<<blocks, 256, 0, s>>>(t, d, nd, total);
}

hipError_t launch_find_multi(const TableView& t, const FindDesc* d, uint32_t nd, uint64_t total, int group,
                             int prefetch_b2, unsigned blocks, hipStream_t s) {
    if (total == 0 || nd == 0) return hipSuccess;
    const bool pre = prefetch_b2 != 0;
    if (blocks == 0) blocks = blocks_for(total * (uint64_t)group, 256);
    switch (group) {
        case 4: launch_find_multi_g<4>(t, d, nd, total, pre, blocks, s); break;
        case 16: launch_find_multi_g<16>(t, d, nd, total, pre, blocks, s); break;
        default: launch_find_multi_g<8>(t, d, nd, total, pre, blocks, s); break;
    }
    return hipGetLastError();
}

template <int G>
static void launch_find_g(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                          uint64_t* scores_out, bool pre, bool pairs, hipStream_t s) {
    if (pairs) {
        const unsigned blocks = blocks_for(((n + 1) / 2) * G, 256);
        if (pre) k_find_x2<G, true><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out);
        else k_find_x2<G, false><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out);
        return;
    }
    const unsigned blocks = blocks_for(n * G, 256);
    if (pre) k_find<G, true><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out);
    else k_find<G, false><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out);
}

hipError_t launch_find(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                       uint64_t* scores_out, int group, int prefetch_b2, int pairs, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool pre = prefetch_b2 != 0;
    switch (group) {
        case 4: launch_find_g<4>(t, n, keys, out, found, scores_out, pre, pairs != 0, s); break;
        case 16: launch_find_g<16>(t, n, keys, out, found, scores_out, pre, pairs != 0, s); break;
        default: launch_find_g<8>(t, n, keys, out, found, scores_out, pre, pairs != 0, s); break;
    }
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
    t.bmin[2 * (e / kSlots) + 1] = 0;  // the bucket is no longer full: its cached minimum is void
}

hipError_t launch_erase_probe(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased, uint32_t* ws_slot,
                              int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned nb = blocks_for(n * group, 256);
    switch (group) {
        case 4: k_erase_probe<4><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
        case 16: k_erase_probe<16><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
        default: k_erase_probe<8><<<nb, 256, 0, s>>>(t, n, keys, erased, ws_slot); break;
    }
    return hipGetLastError();
}

hipError_t launch_erase_clear(const TableView& t, uint64_t n, uint32_t* ws_slot, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_erase_clear<<<blocks_for(n, 256), 256, 0, s>>>(t, n, ws_slot);
    return hipGetLastError();
}

hipError_t launch_erase(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased, uint32_t* ws_slot,
                        int group, hipStream_t s) {
    const hipError_t e = launch_erase_probe(t, n, keys, erased, ws_slot, group, s);
    if (e != hipSuccess) return e;
    return launch_erase_clear(t, n, ws_slot, s);
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
