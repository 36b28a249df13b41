// Serving loop: real-time admission of find / insert_and_evict requests under an HBM budget,
// continuous batching of queued finds into merged reader launches, inserts as serialization
// points, completion by polled HIP events.  Single host thread; inserters on the caller's stream,
// reader groups on it too or rotating over reader streams of their own (ordered by events: a
// reader group after the last inserter before it, an inserter after every reader group before
// it), so that reader groups between inserters run concurrently.
#include <hip/hip_runtime.h>

#include <chrono>
#include <deque>
#include <vector>

#include "../../include/cskv.h"
#include "cskv_internal.h"
#include "cskv_ring.h"

using namespace cskv;

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Group {
    hipEvent_t done;
    uint64_t first, last;  // admitted sequence range [first, last)
};

// output bytes a request needs from the arena when it brings no result buffers
size_t arena_bytes(const cskv_request& r, uint32_t dim) {
    if (r.op == CSKV_REQ_FIND) {
        size_t b = 0;
        if (!r.d_values_out) b += align256(r.n * dim * 4);
        if (!r.d_flags) b += align256(r.n);
        return b;
    }
    size_t b = 0;
    if (!r.d_flags) b += align256(r.n);
    if (!r.d_ev_keys) b += align256(r.n * 8) + align256(r.n * dim * 4) + align256(r.n * 8) + 256;
    return b;
}

// bytes a request holds while in flight: its inputs and outputs
uint64_t footprint(const cskv_request& r, uint32_t dim) {
    const uint64_t row = (uint64_t)dim * 4;
    if (r.op == CSKV_REQ_FIND) return r.n * 8 + r.n * row + r.n;
    return r.n * 8 + r.n * row + (r.d_scores ? r.n * 8 : 0) + r.n + r.n * (16 + row) + 8;
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

size_t cskv_serve_workspace_bytes(const cskv_table* table, uint64_t max_request_keys, uint64_t arena_budget_bytes) {
    if (!table) return 0;
    return align256(upsert_layout(max_request_keys, table->view.nbuckets, table->subrounds).total) +
           align256(arena_budget_bytes);
}

int cskv_serve_trace(cskv_table* t, cskv_request* reqs, uint64_t nreq, const cskv_serve_config* cfg, void* d_ws,
                     size_t ws_bytes, void* stream, cskv_serve_stats* stats) {
    if (!t || (!reqs && nreq) || !cfg || !d_ws || ((uintptr_t)d_ws & 255)) return CSKV_EINVAL;
    if (cfg->max_merge == 0 || cfg->max_merge > (uint32_t)kMaxArgDescs || cfg->max_inflight_groups == 0 ||
        cfg->reader_streams > 4)
        return CSKV_EINVAL;
    const uint32_t dim = t->view.dim;
    uint64_t max_n = 1;
    for (uint64_t i = 0; i < nreq; ++i) {
        const cskv_request& r = reqs[i];
        if (r.op != CSKV_REQ_FIND && r.op != CSKV_REQ_INSERT_AND_EVICT) return CSKV_EINVAL;
        if (!r.d_keys || (r.op == CSKV_REQ_INSERT_AND_EVICT && !r.d_values)) return CSKV_EINVAL;
        if (r.op == CSKV_REQ_INSERT_AND_EVICT && t->policy == CSKV_SCORE_CUSTOM && !r.d_scores) return CSKV_EINVAL;
        if (footprint(r, dim) > cfg->arena_budget_bytes || arena_bytes(r, dim) > cfg->arena_budget_bytes)
            return CSKV_EINVAL;
        if (r.n > max_n) max_n = r.n;
    }
    const size_t ups_bytes = align256(upsert_layout(max_n, t->view.nbuckets, t->subrounds).total);
    if (ws_bytes < ups_bytes + align256(cfg->arena_budget_bytes)) return CSKV_ENOMEM;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RoleScope role(t, kInserter, s);  // the whole trace holds the table as one inserter
    if (!role.ok()) return CSKV_EHIP;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_ws);
    cskv::Ring ring;
    uint8_t* const arena = ws + ups_bytes;
    ring.size = align256(cfg->arena_budget_bytes);

    cskv_serve_stats st{};
    std::deque<Group> inflight;
    std::vector<hipEvent_t> event_pool;
    uint64_t next_arrival = 0;   // next request not yet admitted (arrival order == admission order)
    uint64_t next_launch = 0;    // next admitted request not yet launched
    uint64_t next_complete = 0;  // next request not yet completed
    uint64_t inflight_bytes = 0;
    bool deferred_flag = false;
    int rc = CSKV_OK;
    const auto t0 = std::chrono::steady_clock::now();

    auto get_event = [&](hipEvent_t* e) -> bool {
        if (!event_pool.empty()) {
            *e = event_pool.back();
            event_pool.pop_back();
            return true;
        }
        return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    };

    // reader streams (default priority) and the events that order them against the inserters:
    // `writer` is recorded after every inserter (and at the start), `tail[k]` after every reader
    // group on stream k; `waited[k]` is the inserter count stream k last waited for
    const uint32_t K = cfg->reader_streams;
    hipStream_t rs[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t tail[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t writer = nullptr;
    uint64_t writers = 0, waited[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    bool dirty[4] = {false, false, false, false};
    uint32_t next_rs = 0;
    if (K) {
        bool ok = hipEventCreateWithFlags(&writer, hipEventDisableTiming) == hipSuccess &&
                  hipEventRecord(writer, s) == hipSuccess;
        for (uint32_t k = 0; k < K && ok; ++k)
            ok = hipStreamCreateWithFlags(&rs[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&tail[k], hipEventDisableTiming) == hipSuccess;
        if (!ok) rc = CSKV_EHIP;
    }

    while (next_complete < nreq && rc == CSKV_OK) {
        bool progress = false;
        const double now = now_s(t0);
        // 1. admission, in arrival order, while the budget allows
        while (next_arrival < nreq && (!cfg->realtime || reqs[next_arrival].arrival_s <= now)) {
            cskv_request& r = reqs[next_arrival];
            const uint64_t fp = footprint(r, dim);
            size_t off = 0;
            if (inflight_bytes + fp > cfg->arena_budget_bytes || !ring.alloc(arena_bytes(r, dim), &off)) {
                if (!deferred_flag) {
                    ++st.deferred_for_memory;
                    deferred_flag = true;
                }
                break;
            }
            deferred_flag = false;
            uint8_t* a = arena + off;
            if (r.op == CSKV_REQ_FIND) {
                if (!r.d_values_out) {
                    r.d_values_out = reinterpret_cast<float*>(a);
                    a += align256(r.n * dim * 4);
                }
                if (!r.d_flags) r.d_flags = a;
            } else {
                if (!r.d_flags) {
                    r.d_flags = a;
                    a += align256(r.n);
                }
                if (!r.d_ev_keys) {
                    r.d_ev_keys = reinterpret_cast<uint64_t*>(a);
                    a += align256(r.n * 8);
                    r.d_ev_values = reinterpret_cast<float*>(a);
                    a += align256(r.n * dim * 4);
                    r.d_ev_scores = reinterpret_cast<uint64_t*>(a);
                    a += align256(r.n * 8);
                    r.d_n_evicted = reinterpret_cast<uint64_t*>(a);
                }
            }
            inflight_bytes += fp;
            if (inflight_bytes > st.peak_inflight_bytes) st.peak_inflight_bytes = inflight_bytes;
            r.admit_s = now;
            r.seq = next_arrival;
            ++next_arrival;
            progress = true;
        }
        // 2. launch admitted requests as groups
        while (next_launch < next_arrival && inflight.size() < cfg->max_inflight_groups) {
            Group g;
            g.first = next_launch;
            const double tl = now_s(t0);
            hipStream_t q = s;  // the group's stream
            uint32_t qk = 0;    // and, for a reader group on a reader stream, that stream's index
            if (reqs[next_launch].op == CSKV_REQ_FIND) {
                if (K) {  // the next reader stream, after the last inserter before this group
                    const uint32_t k = next_rs;
                    qk = k;
                    next_rs = (next_rs + 1) % K;
                    q = rs[k];
                    if (waited[k] != writers) {
                        if (hipStreamWaitEvent(q, writer, 0) != hipSuccess) rc = CSKV_EHIP;
                        waited[k] = writers;
                    }
                    dirty[k] = true;
                }
                FindDescArgs a{};
                a.nd = 0;
                a.total = 0;
                while (next_launch < next_arrival && reqs[next_launch].op == CSKV_REQ_FIND && a.nd < cfg->max_merge) {
                    cskv_request& r = reqs[next_launch];
                    a.d[a.nd++] = FindDesc{r.d_keys, r.d_values_out, r.d_flags, nullptr, a.total, r.n};
                    a.total += r.n;
                    r.launch_s = tl;
                    r.group = (uint32_t)st.groups;
                    ++next_launch;
                }
                if (rc == CSKV_OK && launch_find_args(t->view, a, t->group, t->prefetch_b2, q) != hipSuccess)
                    rc = CSKV_EHIP;
                if (K && rc == CSKV_OK && hipEventRecord(tail[qk], q) != hipSuccess) rc = CSKV_EHIP;
                ++st.reader_launches;
            } else {
                for (uint32_t k = 0; k < K && rc == CSKV_OK; ++k)  // after every reader group before it
                    if (dirty[k]) {
                        if (hipStreamWaitEvent(s, tail[k], 0) != hipSuccess) rc = CSKV_EHIP;
                        dirty[k] = false;
                    }
                cskv_request& r = reqs[next_launch];
                UpsertArgs ua{r.n, r.d_keys, r.d_values, r.d_scores, r.d_flags,
                              EvictOut{r.d_ev_keys, r.d_ev_values, r.d_ev_scores, r.d_n_evicted}};
                if (rc == CSKV_OK) rc = enqueue_upsert(t, ua, ws, ups_bytes, s);
                if (K && rc == CSKV_OK) {
                    if (hipEventRecord(writer, s) != hipSuccess) rc = CSKV_EHIP;
                    ++writers;
                }
                r.launch_s = tl;
                r.group = (uint32_t)st.groups;
                ++next_launch;
                ++st.inserter_launches;
            }
            g.last = next_launch;
            if (rc == CSKV_OK && (!get_event(&g.done) || hipEventRecord(g.done, q) != hipSuccess)) rc = CSKV_EHIP;
            if (rc != CSKV_OK) break;
            inflight.push_back(g);
            ++st.groups;
            progress = true;
        }
        // 3. completions, in launch order
        while (!inflight.empty() && rc == CSKV_OK) {
            const hipError_t q = hipEventQuery(inflight.front().done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                rc = CSKV_EHIP;
                break;
            }
            const double tc = now_s(t0);
            const Group g = inflight.front();
            inflight.pop_front();
            event_pool.push_back(g.done);
            for (uint64_t i = g.first; i < g.last; ++i) {
                reqs[i].complete_s = tc;
                inflight_bytes -= footprint(reqs[i], dim);
                ring.free_front();
                ++st.completed;
            }
            next_complete = g.last;
            progress = true;
        }
        (void)progress;
    }
    // the caller's stream (and the role lock's release on it) follows every reader group
    for (uint32_t k = 0; k < K; ++k) {
        if (rs[k] && tail[k] && hipEventRecord(tail[k], rs[k]) == hipSuccess) (void)hipStreamWaitEvent(s, tail[k], 0);
    }
    if (rc != CSKV_OK || K) {
        for (uint32_t k = 0; k < K; ++k)
            if (rs[k]) (void)hipStreamSynchronize(rs[k]);
        (void)hipStreamSynchronize(s);
    }
    for (uint32_t k = 0; k < K; ++k) {
        if (tail[k]) (void)hipEventDestroy(tail[k]);
        if (rs[k]) (void)hipStreamDestroy(rs[k]);
    }
    if (writer) (void)hipEventDestroy(writer);
    for (auto& g : inflight) event_pool.push_back(g.done);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    st.wall_s = now_s(t0);
    if (stats) *stats = st;
    return rc;
}

}  // extern "C"
