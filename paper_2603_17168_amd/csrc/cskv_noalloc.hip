// insert_or_assign without allocation: its workspace is a fixed device array of this library
// instead of a caller buffer, for callers that cannot allocate device memory.  The kernels are
// the ones cskv_insert_or_assign launches; only the workspace layout differs (the compact one,
// sized by the batch alone, so that a fixed array serves any table).
#include <hip/hip_runtime.h>

#include <mutex>

#include "cskv.h"
#include "cskv_internal.h"

// The workspace: one copy per GPU, allocated when the library's code object loads on that GPU and
// held until the process ends.  Host code never passes this name to a kernel (on the host it
// stands for a shadow variable, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[CSKV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// device address of device dev's copy of the array, looked up once per device with dev current
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return CSKV_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return CSKV_EHIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return CSKV_EHIP;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return CSKV_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return CSKV_OK;
}
}  // namespace

extern "C" {

size_t cskv_noalloc_scratch_bytes(void) { return (size_t)CSKV_NOALLOC_SCRATCH_BYTES; }

int cskv_insert_or_assign_noalloc(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                                  const uint64_t* d_scores, uint8_t* d_status, void* stream) {
    using namespace cskv;
    if (!table || n > CSKV_NOALLOC_MAX_KEYS) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    const size_t need = upsert_layout(n, table->view.nbuckets, table->subrounds, true).total;
    if (need > (size_t)CSKV_NOALLOC_SCRATCH_BYTES) return CSKV_ENOMEM;
    void* ws = nullptr;
    const int rc = scratch_address(table->device, &ws);
    if (rc != CSKV_OK) return rc;
    UpsertArgs a{n, d_keys, d_values, d_scores, d_status, EvictOut{nullptr, nullptr, nullptr, nullptr}};
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RoleScope role(table, kInserter, s);
    if (!role.ok()) return CSKV_EHIP;
    return enqueue_upsert(table, a, ws, (size_t)CSKV_NOALLOC_SCRATCH_BYTES, s, -1, true);
}

}  // extern "C"
