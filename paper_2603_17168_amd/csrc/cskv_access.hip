// Readers and updaters of the cache-semantic hash table beyond find (Sec. 3.5's role list, Sec.
// 4.1) for CDNA4 (gfx950, wave64):
//   contains        reader: found flag per key
//   find_ptr        reader: the device address of the resident row (the position-returning find)
//   assign          updater: row and score of resident keys, never bucket structure
//   assign_scores   updater: score of resident keys
// Each key is served by a group of G lanes that probe the digest lines as find does (Alg. 1).
// The updaters run after the upsert path's dedupe pass (one set entry per distinct key, last
// occurrence wins, LFU increments summed); only a key's last occurrence writes.
#include <hip/hip_runtime.h>

#include "cskv_device.h"
#include "cskv_internal.h"

namespace cskv {

// bucket and slot of key k (slot -1 when absent), on all G lanes
template <int G>
__device__ __forceinline__ int locate_key(const TableView& t, uint64_t k, int lane, uint32_t& b) {
    b = 0;
    if (reserved_key(k)) return -1;
    const KeyHash h = hash_key(t, k);
    LineSeg<G> s1;
    s1.load(t.dig + (size_t)h.b1 * kSlots, lane);
    b = h.b1;
    int slot = verify<G>(t, h.b1, s1.match(h.dg), k, lane);
    if (slot < 0 && h.b2 != h.b1) {
        LineSeg<G> s2;
        s2.load(t.dig + (size_t)h.b2 * kSlots, lane);
        b = h.b2;
        slot = verify<G>(t, h.b2, s2.match(h.dg), k, lane);
    }
    return slot;
}

// PTR = false: contains; PTR = true: find_ptr (address of the row, 0 when absent)
template <int G, bool PTR>
__global__ void __launch_bounds__(256) k_locate(TableView t, uint64_t n, const uint64_t* __restrict__ keys,
                                                uint8_t* __restrict__ found, uint64_t* __restrict__ ptrs,
                                                uint64_t* __restrict__ scores) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    uint32_t b;
    const int slot = locate_key<G>(t, keys[i], lane, b);
    if (lane != 0) return;
    found[i] = slot >= 0;
    if (slot < 0) {
        if (PTR) ptrs[i] = 0;
        return;
    }
    const size_t e = (size_t)b * kSlots + slot;
    if (PTR) ptrs[i] = (uint64_t)(uintptr_t)t.row(e);
    if (scores) scores[i] = t.scores[e];
}

// assign (vals != null) / assign_scores: every occurrence reports residency; the last occurrence
// of a resident key sets its score as an update of insert_or_assign would (custom: its score; LRU:
// this call's clock; LFU: old + summed increments, saturating) and, for assign, its row.  The
// bucket's cached minimum is voided (the score change may move it).
template <int G>
__global__ void __launch_bounds__(256) k_assign(TableView t, UpsertWs w, uint64_t n, const uint64_t* __restrict__ keys,
                                                const float* __restrict__ vals, const uint64_t* __restrict__ scores,
                                                uint8_t* __restrict__ found) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= n) return;
    const int lane = glane<G>();
    uint32_t b;
    const int slot = locate_key<G>(t, keys[i], lane, b);
    if (found && lane == 0) found[i] = slot >= 0;
    if (slot < 0) return;
    const uint32_t p = w.slot_of[i];
    const bool dups = w.ctr[kCtrDup] != 0;  // else every occurrence is its key's only one
    if (dups) {
        const DedupeEntry de = w.dd[p];
        if ((de.claim > de.last ? de.claim : de.last) != (uint32_t)(i + 1)) return;  // not the last occurrence
    }
    const size_t e = (size_t)b * kSlots + slot;
    if (lane == 0) {
        uint64_t ns;
        if (t.policy == 0) ns = scores[i];
        else if (t.policy == 1) ns = *t.clock + 1;  // advanced by k_clock_tick after this kernel
        else ns = sat_add(t.scores[e], dups ? (w.sat[p] ? ~0ull : w.inc[p]) : (scores ? scores[i] : 1ull));
        t.scores[e] = ns;
        t.bmin[2 * (size_t)b + 1] = 0;
    }
    if (vals) copy_row<G>(t.row(e), vals + i * t.dim, t.dim, lane);
}

// an atomic add: updaters may run at the same time on several streams under the role lock
__global__ void k_clock_tick(TableView t) { atomicAdd(reinterpret_cast<unsigned long long*>(t.clock), 1ull); }

template <int G, bool PTR>
static void launch_locate_g(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* found, uint64_t* ptrs,
                            uint64_t* scores, hipStream_t s) {
    k_locate<G, PTR><<<blocks_for(n * G, 256), 256, 0, s>>>(t, n, keys, found, ptrs, scores);
}

hipError_t launch_locate(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* found, uint64_t* ptrs,
                         uint64_t* scores, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool ptr = ptrs != nullptr;
    switch (group) {
        case 4: ptr ? launch_locate_g<4, true>(t, n, keys, found, ptrs, scores, s)
                    : launch_locate_g<4, false>(t, n, keys, found, ptrs, scores, s); break;
        case 16: ptr ? launch_locate_g<16, true>(t, n, keys, found, ptrs, scores, s)
                     : launch_locate_g<16, false>(t, n, keys, found, ptrs, scores, s); break;
        default: ptr ? launch_locate_g<8, true>(t, n, keys, found, ptrs, scores, s)
                     : launch_locate_g<8, false>(t, n, keys, found, ptrs, scores, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_assign(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys, const float* vals,
                         const uint64_t* scores, uint8_t* found, int group, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned nb = blocks_for(n * (uint64_t)group, 256);
    switch (group) {
        case 4: k_assign<4><<<nb, 256, 0, s>>>(t, w, n, keys, vals, scores, found); break;
        case 16: k_assign<16><<<nb, 256, 0, s>>>(t, w, n, keys, vals, scores, found); break;
        default: k_assign<8><<<nb, 256, 0, s>>>(t, w, n, keys, vals, scores, found); break;
    }
    if (t.policy == 1) k_clock_tick<<<1, 1, 0, s>>>(t);
    return hipGetLastError();
}

}  // namespace cskv
