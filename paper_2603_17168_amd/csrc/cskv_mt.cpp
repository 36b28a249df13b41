// Concurrent-caller driver: host threads with their own streams issue batches on one table
// through the C ABI at the same time (the setting of the concurrency ablation, Exp. 3e).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "../../include/cskv.h"
#include "../../include/cskv_mt.h"
#include "cskv_internal.h"

namespace {

int run_thread(cskv_table* t, cskv_mt_thread& a, hipStream_t s) {
    a.failed_call = a.calls;
    for (uint64_t c = 0; c < a.calls; ++c) {
        int rc = CSKV_OK;
        switch (a.op) {
            case CSKV_MT_FIND:
                rc = cskv_find(t, a.n, a.d_keys, a.d_values_out, a.d_flags, nullptr, s);
                break;
            case CSKV_MT_ASSIGN:
                rc = cskv_assign(t, a.n, a.d_keys, a.d_values, a.d_scores, a.d_flags, a.d_ws, a.ws_bytes, s);
                break;
            default:
                rc = (c & 1) ? cskv_erase(t, a.n, a.d_keys, a.d_flags, a.d_ws, a.ws_bytes, s)
                             : cskv_insert_or_assign(t, a.n, a.d_keys, a.d_values, a.d_scores, a.d_flags, a.d_ws,
                                                     a.ws_bytes, s);
                break;
        }
        if (rc != CSKV_OK) {
            a.failed_call = c;
            a.hip_error = (int)hipGetLastError();
            return rc;
        }
    }
    return CSKV_OK;
}

}  // namespace

extern "C" int cskv_mt_run(cskv_table* table, int nthreads, cskv_mt_thread* threads, double* wall_ms) {
    if (!table || nthreads < 1 || nthreads > 64 || !threads || !wall_ms) return CSKV_EINVAL;
    for (int i = 0; i < nthreads; ++i) {
        const cskv_mt_thread& a = threads[i];
        if (a.op < CSKV_MT_FIND || a.op > CSKV_MT_INSERT_ERASE || a.n == 0 || a.n >= (1ull << 31) || !a.d_keys ||
            !a.d_flags)
            return CSKV_EINVAL;
        if (a.op == CSKV_MT_FIND && !a.d_values_out) return CSKV_EINVAL;
        if (a.op != CSKV_MT_FIND && (!a.d_values || !a.d_ws)) return CSKV_EINVAL;
    }
    for (int i = 0; i < nthreads; ++i) {
        threads[i].status = CSKV_OK;
        threads[i].hip_error = 0;
        threads[i].failed_call = threads[i].calls;
    }
    // the streams outlive the threads: the table's lock is reset (its events synchronized and
    // forgotten) before they are destroyed
    int prev_dev = 0;
    if (hipGetDevice(&prev_dev) != hipSuccess || hipSetDevice(table->device) != hipSuccess) return CSKV_EHIP;
    std::vector<hipStream_t> streams(nthreads, nullptr);
    int rc_all = CSKV_OK;
    for (int i = 0; i < nthreads && rc_all == CSKV_OK; ++i)
        if (hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking) != hipSuccess) rc_all = CSKV_EHIP;
    if (rc_all == CSKV_OK) {
        std::vector<int> rc(nthreads, CSKV_OK);
        std::atomic<int> ready{0};
        std::atomic<bool> go{false};
        std::vector<std::thread> th;
        for (int i = 0; i < nthreads; ++i) {
            th.emplace_back([&, i] {
                const bool ok = hipSetDevice(table->device) == hipSuccess;
                ready.fetch_add(1);
                while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
                if (!ok) {
                    rc[i] = threads[i].status = CSKV_EHIP;
                    threads[i].hip_error = (int)hipGetLastError();
                    threads[i].failed_call = 0;
                    return;
                }
                rc[i] = run_thread(table, threads[i], streams[i]);
                const hipError_t se = hipStreamSynchronize(streams[i]);
                if (se != hipSuccess && rc[i] == CSKV_OK) {
                    rc[i] = CSKV_EHIP;
                    threads[i].hip_error = (int)se;
                }
                threads[i].status = rc[i];
            });
        }
        while (ready.load() < nthreads) std::this_thread::yield();
        const auto t0 = std::chrono::steady_clock::now();
        go.store(true, std::memory_order_release);
        for (auto& x : th) x.join();
        *wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int r : rc)
            if (r != CSKV_OK && rc_all == CSKV_OK) rc_all = r;
        if (!table->roles->reset() && rc_all == CSKV_OK) rc_all = CSKV_EHIP;
    }
    for (hipStream_t s : streams)
        if (s) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev_dev);
    return rc_all;
}
