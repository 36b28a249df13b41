// Memory-system reference kernels (cskv_probe.h): a 16-byte-per-lane copy and random gathers of
// 8..128 bytes per access, for pricing the table's kernels against the device's attainable rates.
#include <hip/hip_runtime.h>

#include "../../include/cskv.h"
#include "../../include/cskv_probe.h"
#include "cskv_internal.h"

namespace cskv {

// one 16-byte element per lane over a grid that covers the whole buffer: on MI355X this form copies
// at 6.1-6.3 TB/s (read + write), where a grid-stride loop over 65536 blocks reached 4.7-5.5
__global__ void __launch_bounds__(256) k_probe_copy(const uint4* __restrict__ s, uint4* __restrict__ d, uint64_t n16) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) d[i] = s[i];
}

// SplitMix64's output function: spreads consecutive access indices over the whole array
__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// W bytes per access: one lane per access up to 16 bytes, W/16 lanes per access above
template <int W>
__global__ void __launch_bounds__(256) k_probe_gather(const uint8_t* __restrict__ src, uint64_t units, uint64_t n,
                                                      uint64_t salt, uint8_t* __restrict__ out) {
    constexpr int L = W > 16 ? W / 16 : 1;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i = t / L;
    if (i >= n) return;
    const uint64_t u = probe_mix(i ^ salt) & (units - 1);
    const uint64_t off = u * W + (t % L) * 16;
    if constexpr (W == 8) {
        *reinterpret_cast<uint64_t*>(out + i * 8) = *reinterpret_cast<const uint64_t*>(src + off);
    } else {
        *reinterpret_cast<uint4*>(out + i * W + (t % L) * 16) = *reinterpret_cast<const uint4*>(src + off);
    }
}

}  // namespace cskv

using namespace cskv;

extern "C" {

int cskv_probe_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
    if (!d_src || !d_dst || bytes % 16 || ((uintptr_t)d_src & 15) || ((uintptr_t)d_dst & 15)) return CSKV_EINVAL;
    if (bytes == 0) return CSKV_OK;
    const uint64_t n16 = bytes / 16;
    const uint64_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return CSKV_EINVAL;  // beyond one launch's grid (over 8 TiB)
    k_probe_copy<<<(unsigned)blocks, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        reinterpret_cast<const uint4*>(d_src), reinterpret_cast<uint4*>(d_dst), n16);
    return hipGetLastError() == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

int cskv_probe_gather(const void* d_src, size_t src_bytes, uint32_t width, uint64_t n, uint64_t salt, void* d_out,
                      void* stream) {
    if (!d_src || !d_out || ((uintptr_t)d_src & 15) || ((uintptr_t)d_out & 15)) return CSKV_EINVAL;
    if (width != 8 && width != 16 && width != 32 && width != 64 && width != 128) return CSKV_EINVAL;
    if (src_bytes < width || (src_bytes & (src_bytes - 1))) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (n >= (1ull << 32)) return CSKV_EINVAL;
    const uint64_t units = src_bytes / width;
    const uint64_t lanes = width > 16 ? width / 16 : 1;
    const unsigned blocks = (unsigned)((n * lanes + 255) / 256);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint8_t* src = reinterpret_cast<const uint8_t*>(d_src);
    uint8_t* out = reinterpret_cast<uint8_t*>(d_out);
    switch (width) {
        case 8: k_probe_gather<8><<<blocks, 256, 0, s>>>(src, units, n, salt, out); break;
        case 16: k_probe_gather<16><<<blocks, 256, 0, s>>>(src, units, n, salt, out); break;
        case 32: k_probe_gather<32><<<blocks, 256, 0, s>>>(src, units, n, salt, out); break;
        case 64: k_probe_gather<64><<<blocks, 256, 0, s>>>(src, units, n, salt, out); break;
        default: k_probe_gather<128><<<blocks, 256, 0, s>>>(src, units, n, salt, out); break;
    }
    return hipGetLastError() == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

}  // extern "C"
