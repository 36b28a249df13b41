// Find kernels of the cache-semantic hash table for CDNA4 (gfx950, wave64) (Alg. 1).
//
// A key is served by a group of G lanes of one wave (G = 4, 8 or 16).  The group loads a
// bucket's 128-byte digest line with one 128/G-byte load per lane, compares the bytes with
// the key's digest using exact SWAR byte equality, and verifies candidates against the key
// line.  Value rows move as 16-byte chunks spread over the group's lanes.  Variants: one key
// per group (k_find), two keys per group with interleaved probes and rows (k_find_x2), merged
// runs of batches over a descriptor table (k_find_multi) or kernel arguments (k_find_args).
#include <hip/hip_runtime.h>

#include "cskv_device.h"
#include "cskv_internal.h"

namespace cskv {

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
        copy_row<G>(out_row, t.row(e), t.dim, lane);
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
    const uint4* srcA = reinterpret_cast<const uint4*>(t.row((size_t)bkA * kSlots + (slA < 0 ? 0 : slA)));
    const uint4* srcB = reinterpret_cast<const uint4*>(t.row((size_t)bkB * kSlots + (slB < 0 ? 0 : slB)));
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

// ------------------------------------------------------------------------------------------
// digest ablation (Exp. 3a): the same lookup with no digest filter.  The group compares the key
// with all 128 stored keys of each candidate bucket (1 KiB); at step j lane l reads slots
// 2(jG + l) and 2(jG + l) + 1, so each load instruction of a group covers one contiguous
// 16G-byte run.  A matching slot still has its digest byte read, because a freed slot keeps its
// stale key.
template <int G>
__device__ __forceinline__ int scan_keys(const TableView& t, uint32_t b, uint64_t k, int lane) {
    constexpr int STEPS = kSlots / (2 * G);
    const size_t eb = (size_t)b * kSlots;
    const ulonglong2* bk = reinterpret_cast<const ulonglong2*>(t.keys + eb);
    ulonglong2 x[STEPS];
#pragma unroll
    for (int j = 0; j < STEPS; ++j) x[j] = bk[j * G + lane];
    int hit = -1;
#pragma unroll
    for (int j = 0; j < STEPS; ++j) {
        const int s0 = 2 * (j * G + lane);
        if (x[j].x == k && hit < 0 && t.dig[eb + s0] != 0) hit = s0;
        if (x[j].y == k && hit < 0 && t.dig[eb + s0 + 1] != 0) hit = s0 + 1;
    }
    return gmax_i<G>(hit);
}

template <int G>
__global__ void __launch_bounds__(256) k_find_nodigest(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
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
        b = h.b1;
        slot = scan_keys<G>(t, h.b1, k, lane);
        if (slot < 0 && h.b2 != h.b1) {
            b = h.b2;
            slot = scan_keys<G>(t, h.b2, k, lane);
        }
    }
    if (slot >= 0) {
        const size_t e = (size_t)b * kSlots + slot;
        copy_row<G>(out + i * t.dim, t.row(e), t.dim, lane);
        if (lane == 0) {
            found[i] = 1;
            if (scores_out) scores_out[i] = t.scores[e];
        }
    } else if (lane == 0) {
        found[i] = 0;
    }
}

hipError_t launch_find_nodigest(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                                uint64_t* scores_out, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = blocks_for(n * (uint64_t)group, 256);
    switch (group) {
        case 4: k_find_nodigest<4><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
        case 16: k_find_nodigest<16><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
        default: k_find_nodigest<8><<<blocks, 256, 0, s>>>(t, n, keys, out, found, scores_out); break;
    }
    return hipGetLastError();
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

}  // namespace cskv
