// Serving loop: real-time admission of find / insert_and_evict requests under an HBM budget,
// continuous batching of queued finds into merged reader launches, inserts as serialization
// points, completion by polled HIP events.  Single host thread, one stream.
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
    if (cfg->max_merge == 0 || cfg->max_merge > (uint32_t)kMaxArgDescs || cfg->max_inflight_groups == 0)
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
            if (reqs[next_launch].op == CSKV_REQ_FIND) {
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
                if (launch_find_args(t->view, a, t->group, t->prefetch_b2, s) != hipSuccess) rc = CSKV_EHIP;
                ++st.reader_launches;
            } else {
                cskv_request& r = reqs[next_launch];
                UpsertArgs ua{r.n, r.d_keys, r.d_values, r.d_scores, r.d_flags,
                              EvictOut{r.d_ev_keys, r.d_ev_values, r.d_ev_scores, r.d_n_evicted}};
                rc = enqueue_upsert(t, ua, ws, ups_bytes, s);
                r.launch_s = tl;
                r.group = (uint32_t)st.groups;
                ++next_launch;
                ++st.inserter_launches;
            }
            g.last = next_launch;
            if (rc == CSKV_OK && (!get_event(&g.done) || hipEventRecord(g.done, s) != hipSuccess)) rc = CSKV_EHIP;
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
    if (rc != CSKV_OK) (void)hipStreamSynchronize(s);
    for (auto& g : inflight) event_pool.push_back(g.done);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    st.wall_s = now_s(t0);
    if (stats) *stats = st;
    return rc;
}

}  // extern "C"
