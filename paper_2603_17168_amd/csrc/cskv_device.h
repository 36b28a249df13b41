// Device helpers of the cache-semantic hash table kernels (CDNA4, wave64): the bucket hash,
// lane-group reductions, SWAR digest matching, probing and row copies.
#pragma once

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

// Exchange inside aligned groups of up to 16 lanes by DPP lane moves (no LDS traffic): step 0
// swaps lanes i and i^1, step 1 swaps i and i^2 (quad permutes), step 2 mirrors each 8-lane half
// of a 16-lane row, step 3 mirrors the row.  In a reduction, after steps 0..s-1 every lane holds
// its block's partial result, so step s pairs each block with the other half of the next larger
// block and the result reaches every lane.  Groups wider than 16 lanes finish with shuffles.
template <int S>
__device__ __forceinline__ int dpp_xchg(int v) {
    constexpr int ctrl = S == 0 ? 0xB1 : S == 1 ? 0x4E : S == 2 ? 0x141 : 0x140;
    return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, false);
}

template <int S>
__device__ __forceinline__ uint64_t dpp_xchg(uint64_t v) {
    const uint32_t lo = (uint32_t)dpp_xchg<S>((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)dpp_xchg<S>((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int G, typename T, typename Op>
__device__ __forceinline__ T group_reduce(T v, Op op) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size");
    if constexpr (G >= 2) v = op(v, dpp_xchg<0>(v));
    if constexpr (G >= 4) v = op(v, dpp_xchg<1>(v));
    if constexpr (G >= 8) v = op(v, dpp_xchg<2>(v));
    if constexpr (G >= 16) v = op(v, dpp_xchg<3>(v));
    if constexpr (G >= 32) v = op(v, (T)__shfl_xor(v, 16, G));
    if constexpr (G >= 64) v = op(v, (T)__shfl_xor(v, 32, G));
    return v;
}

template <int G>
__device__ __forceinline__ int gmax_i(int v) {
    return group_reduce<G>(v, [](int a, int b) { return max(a, b); });
}

template <int G>
__device__ __forceinline__ int gsum_i(int v) {
    return group_reduce<G>(v, [](int a, int b) { return a + b; });
}

template <int G>
__device__ __forceinline__ uint64_t gmin_u64(uint64_t v) {
    return group_reduce<G>(v, [](uint64_t a, uint64_t b) { return b < a ? b : a; });
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

static inline unsigned blocks_for(uint64_t threads, unsigned bs) { return (unsigned)((threads + bs - 1) / bs); }

}  // namespace cskv
