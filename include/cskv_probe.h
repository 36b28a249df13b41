/*
 * cskv_probe.h - memory-system reference kernels that the benchmark prices the table's kernels
 * against (no hash-table arithmetic).
 *
 * The roofline of every kernel of the table is HBM bandwidth: the figures here give the two
 * reference rates on the running device, measured with the same launch machinery as the table:
 *  - a plain copy with 16 bytes per lane per step (the attainable streaming rate of a kernel that
 *    moves data with the table's row-copy width), and
 *  - random gathers of `width` bytes per access, one access per lane group, from a power-of-two
 *    array (the cost of the table's random accesses: digest lines, key verifies, score reads);
 *    comparing the access rates of 8-byte and 128-byte gathers gives the DRAM access granule
 *    that a random 8-byte read costs.
 *
 * Conventions as in cskv.h: device pointers are caller-owned, calls are asynchronous on
 * `stream` (a hipStream_t, NULL = default), argument errors return CSKV_EINVAL synchronously and
 * enqueue nothing, a failed launch returns CSKV_EHIP.
 */
#ifndef CSKV_PROBE_H
#define CSKV_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copies `bytes` (a multiple of 16) from d_src to d_dst (both 16-byte aligned, not overlapping)
 * with one 16-byte load and one 16-byte store per lane, one lane per 16 bytes.  CSKV_EINVAL for
 * misaligned or null pointers, a size that is not a multiple of 16, or more than 2^31 - 1 blocks
 * of 256 lanes (over 8 TiB). */
int cskv_probe_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* n random gathers: access i reads `width` bytes (8, 16, 32, 64 or 128) at the width-aligned
 * offset (h(i, salt) mod (src_bytes / width)) * width of d_src, where h is a 64-bit mixing
 * function of the access index, and writes them to d_out[i * width ...].  src_bytes must be a
 * power of two, at least `width`; d_src and d_out 16-byte aligned; d_out holds n * width bytes. */
int cskv_probe_gather(const void* d_src, size_t src_bytes, uint32_t width, uint64_t n, uint64_t salt, void* d_out,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CSKV_PROBE_H */
