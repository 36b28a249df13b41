// HIP kernels of the cache-semantic hash table for CDNA4 (gfx950, wave64): erase, size, export,
// table clear and the zero fill.  Find kernels live in cskv_find.hip, upsert kernels in
// cskv_upsert.hip.
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
    return launch_fill_zero(t.cnt, t.nbuckets * 8, s);
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
    // a zero digest frees the slot: every reader of a slot's key or score tests its digest first,
    // and a bucket's cached minimum is read only while the bucket is full and rewritten by the
    // apply kernels whenever a call leaves it full, so nothing else needs clearing
    t.dig[e] = 0;
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
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < nwords; i += 4 * stride) {  // four 16-byte loads in flight
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = d[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) c += 4 - __popc(match4(w4[q], 0u));
        }
    }
    for (; i < nwords; i += stride) {
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
    uint64_t blocks = (t.nbuckets * 8 + 1023) / 1024;  // about four 16-byte words per thread
    if (blocks > 8192) blocks = 8192;
    k_size<<<(unsigned)blocks, 256, 0, s>>>(t, d_size);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// export: a block of 4 waves takes 16 consecutive buckets (4 per wave).  Each wave forms the
// occupancy (and predicate) masks of its buckets with ballots; the block adds up the 16 counts
// and takes its output range with ONE atomic; then every wave writes its buckets' entries at
// their offsets (output order is unspecified).
constexpr int kExportWaves = 4;
constexpr int kExportPerWave = 4;
constexpr int kExportBuckets = kExportWaves * kExportPerWave;

__global__ void __launch_bounds__(256) k_export(TableView t, uint64_t b0, uint64_t b1, uint64_t* __restrict__ keys,
                                                float* __restrict__ vals, uint64_t* __restrict__ scores,
                                                uint64_t* __restrict__ slots, uint64_t* __restrict__ count,
                                                uint64_t min_score) {
    __shared__ uint32_t cnt_s[kExportBuckets];
    __shared__ uint32_t off_s[kExportBuckets];
    __shared__ unsigned long long base_s;
    __shared__ uint8_t sl[kExportWaves][128];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (uint64_t tile = b0 + (uint64_t)blockIdx.x * kExportBuckets; tile < b1;
         tile += (uint64_t)gridDim.x * kExportBuckets) {
        uint64_t bal0[kExportPerWave], bal1[kExportPerWave];
#pragma unroll
        for (int q = 0; q < kExportPerWave; ++q) {
            const uint64_t b = tile + (uint64_t)wv * kExportPerWave + q;
            bool o0 = false, o1 = false;
            if (b < b1) {
                const size_t eb = (size_t)b * kSlots;
                o0 = t.dig[eb + lane] != 0;
                o1 = t.dig[eb + lane + 64] != 0;
                if (min_score) {  // export_batch_if: entries whose score is at least min_score
                    o0 = o0 && t.scores[eb + lane] >= min_score;
                    o1 = o1 && t.scores[eb + lane + 64] >= min_score;
                }
            }
            bal0[q] = __ballot(o0);
            bal1[q] = __ballot(o1);
            if (lane == 0) cnt_s[wv * kExportPerWave + q] = (uint32_t)(__popcll(bal0[q]) + __popcll(bal1[q]));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int q = 0; q < kExportBuckets; ++q) {
                off_s[q] = tot;
                tot += cnt_s[q];
            }
            base_s = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(count), (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kExportPerWave; ++q) {
            const uint64_t b = tile + (uint64_t)wv * kExportPerWave + q;
            const int c = (int)cnt_s[wv * kExportPerWave + q];
            if (b >= b1 || c == 0) continue;
            const size_t eb = (size_t)b * kSlots;
            const uint64_t base = base_s + off_s[wv * kExportPerWave + q];
            if ((bal0[q] >> lane) & 1ull) sl[wv][__popcll(bal0[q] & below)] = (uint8_t)lane;
            if ((bal1[q] >> lane) & 1ull) sl[wv][__popcll(bal0[q]) + __popcll(bal1[q] & below)] = (uint8_t)(lane + 64);
            __builtin_amdgcn_wave_barrier();  // one wave: its LDS accesses stay in order
            for (int j = lane; j < c; j += 64) {
                const size_t e = eb + sl[wv][j];
                keys[base + j] = t.keys[e];
                if (scores) scores[base + j] = t.scores[e];
                if (slots) slots[base + j] = e;
            }
            if (vals) {
                const uint32_t chunks = t.dim >> 2;
                for (uint32_t x = lane; x < (uint32_t)c * chunks; x += 64) {
                    const uint32_t j = x / chunks, cc = x - j * chunks;
                    reinterpret_cast<uint4*>(vals + (base + j) * t.dim)[cc] =
                        reinterpret_cast<const uint4*>(t.row(eb + sl[wv][j]))[cc];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

hipError_t launch_export(const TableView& t, uint64_t b0, uint64_t b1, uint64_t* keys, float* vals,
                         uint64_t* scores, uint64_t* slots, uint64_t* count, uint64_t min_score, hipStream_t s) {
    hipError_t e = launch_fill_zero(count, 8, s);
    if (e != hipSuccess || b1 <= b0) return e;
    uint64_t blocks = (b1 - b0 + kExportBuckets - 1) / kExportBuckets;
    if (blocks > 32768) blocks = 32768;
    k_export<<<(unsigned)blocks, 256, 0, s>>>(t, b0, b1, keys, vals, scores, slots, count, min_score);
    return hipGetLastError();
}

}  // namespace cskv

