// Batched programs over one table: consecutive finds merge into one reader run executed by a
// single (optionally persistent) kernel; upserts and erases are serialization points.  The whole
// sequence can be captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "../../include/cskv.h"
#include "cskv_internal.h"

using namespace cskv;

namespace {

enum OpKind { kFind = 0, kUpsert = 1, kUpsertEvict = 2, kErase = 3 };

struct Op {
    int kind;
    uint64_t n;
    const uint64_t* keys;
    const float* vals;
    const uint64_t* scores;
    float* out;
    uint8_t* flags;       // found / status / erased
    uint64_t* scores_out;
    EvictOut ev;
    int group, prefetch, blocks_per_cu;  // tuning snapshot (finds)
};

struct Segment {
    int kind;            // kFind = merged run, else the op kind
    uint32_t first;      // first op
    uint32_t count;      // ops in the run (1 otherwise)
    uint64_t total;      // keys in the run
    uint32_t desc_off;   // index of the run's first descriptor
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace

constexpr int kSlotsScratch = 2;  // scratch regions rotated over the upserts and erases

struct cskv_program {
    cskv_table* table;
    std::vector<Op> ops;
    std::vector<Segment> segs;
    std::vector<FindDesc> descs;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    size_t scratch_off = 0;
    size_t scratch_bytes = 0;  // per slot
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ready = false;
    bool overlap = true;  // order phases by events (readers together, writers after the reads before them)
    hipStream_t rd = nullptr, wr = nullptr, prep[kSlotsScratch] = {nullptr, nullptr};
    std::vector<hipEvent_t> events;
};

static void build_plan(cskv_program* p) {
    p->segs.clear();
    p->descs.clear();
    for (uint32_t i = 0; i < p->ops.size(); ++i) {
        const Op& o = p->ops[i];
        if (o.n == 0) continue;
        if (o.kind == kFind) {
            if (p->segs.empty() || p->segs.back().kind != kFind) {
                p->segs.push_back(Segment{kFind, i, 0, 0, (uint32_t)p->descs.size()});
            }
            Segment& s = p->segs.back();
            p->descs.push_back(FindDesc{o.keys, o.out, o.flags, o.scores_out, s.total, o.n});
            s.count += 1;
            s.total += o.n;
        } else {
            p->segs.push_back(Segment{o.kind, i, 1, o.n, 0});
        }
    }
}

static size_t scratch_need(const cskv_program* p) {
    size_t need = 256;
    for (const Op& o : p->ops) {
        if (o.n == 0) continue;
        size_t b = 0;
        if (o.kind == kUpsert || o.kind == kUpsertEvict) b = upsert_layout(o.n, p->table->view.nbuckets).total;
        else if (o.kind == kErase) b = erase_ws_bytes(o.n);
        if (b > need) need = b;
    }
    return need;
}

extern "C" {

int cskv_program_create(cskv_program** out, cskv_table* table) {
    if (!out || !table) return CSKV_EINVAL;
    cskv_program* p = new (std::nothrow) cskv_program;
    if (!p) return CSKV_ENOMEM;
    p->table = table;
    *out = p;
    return CSKV_OK;
}

int cskv_program_destroy(cskv_program* p) {
    if (!p) return CSKV_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    if (p->rd) (void)hipStreamDestroy(p->rd);
    if (p->wr) (void)hipStreamDestroy(p->wr);
    for (hipStream_t q : p->prep)
        if (q) (void)hipStreamDestroy(q);
    delete p;
    return CSKV_OK;
}

int cskv_program_set_overlap(cskv_program* p, int enabled) {
    if (!p || p->ready) return CSKV_EINVAL;
    p->overlap = enabled != 0;
    return CSKV_OK;
}

static int add_op(cskv_program* p, const Op& o) {
    if (!p || p->ready) return CSKV_EINVAL;
    if (o.n >= (1ull << 31)) return CSKV_EINVAL;
    p->ops.push_back(o);
    return CSKV_OK;
}

int cskv_program_add_find(cskv_program* p, uint64_t n, const uint64_t* d_keys, float* d_values_out, uint8_t* d_found,
                          uint64_t* d_scores_out) {
    if (!p) return CSKV_EINVAL;
    if (n && (!d_keys || !d_values_out || !d_found || !aligned(d_keys, 8) || !aligned(d_values_out, 16) ||
              (d_scores_out && !aligned(d_scores_out, 8))))
        return CSKV_EINVAL;
    Op o{};
    o.kind = kFind;
    o.n = n;
    o.keys = d_keys;
    o.out = d_values_out;
    o.flags = d_found;
    o.scores_out = d_scores_out;
    o.group = p->table->group;
    o.prefetch = p->table->prefetch_b2;
    o.blocks_per_cu = p->table->blocks_per_cu;
    return add_op(p, o);
}

int cskv_program_add_insert_or_assign(cskv_program* p, uint64_t n, const uint64_t* d_keys, const float* d_values,
                                      const uint64_t* d_scores, uint8_t* d_status) {
    if (!p) return CSKV_EINVAL;
    if (n && (!d_keys || !d_values)) return CSKV_EINVAL;
    if (n && p->table->policy == CSKV_SCORE_CUSTOM && !d_scores) return CSKV_EINVAL;
    Op o{};
    o.kind = kUpsert;
    o.n = n;
    o.keys = d_keys;
    o.vals = d_values;
    o.scores = d_scores;
    o.flags = d_status;
    return add_op(p, o);
}

int cskv_program_add_insert_and_evict(cskv_program* p, uint64_t n, const uint64_t* d_keys, const float* d_values,
                                      const uint64_t* d_scores, uint8_t* d_status, uint64_t* d_ev_keys,
                                      float* d_ev_values, uint64_t* d_ev_scores, uint64_t* d_n_evicted) {
    if (!p) return CSKV_EINVAL;
    if (n && (!d_keys || !d_values || !d_status || !d_ev_keys || !d_ev_values || !d_ev_scores || !d_n_evicted))
        return CSKV_EINVAL;
    if (n && p->table->policy == CSKV_SCORE_CUSTOM && !d_scores) return CSKV_EINVAL;
    Op o{};
    o.kind = kUpsertEvict;
    o.n = n;
    o.keys = d_keys;
    o.vals = d_values;
    o.scores = d_scores;
    o.flags = d_status;
    o.ev = EvictOut{d_ev_keys, d_ev_values, d_ev_scores, d_n_evicted};
    return add_op(p, o);
}

int cskv_program_add_erase(cskv_program* p, uint64_t n, const uint64_t* d_keys, uint8_t* d_erased) {
    if (!p) return CSKV_EINVAL;
    if (n && !d_keys) return CSKV_EINVAL;
    Op o{};
    o.kind = kErase;
    o.n = n;
    o.keys = d_keys;
    o.flags = d_erased;
    return add_op(p, o);
}

size_t cskv_program_workspace_bytes(const cskv_program* p) {
    if (!p) return 0;
    size_t nd = 0;
    for (const Op& o : p->ops)
        if (o.kind == kFind && o.n) ++nd;
    return align256(nd * sizeof(FindDesc) + 1) + (p->overlap ? kSlotsScratch : 1) * align256(scratch_need(p));
}

int cskv_program_set_workspace(cskv_program* p, void* d_ws, size_t ws_bytes) {
    if (!p || !d_ws || !aligned(d_ws, 256)) return CSKV_EINVAL;
    if (ws_bytes < cskv_program_workspace_bytes(p)) return CSKV_ENOMEM;
    build_plan(p);
    p->ws = reinterpret_cast<uint8_t*>(d_ws);
    p->ws_bytes = ws_bytes;
    p->scratch_off = align256(p->descs.size() * sizeof(FindDesc) + 1);
    p->scratch_bytes = align256(scratch_need(p));
    if (!p->descs.empty() &&
        hipMemcpy(p->ws, p->descs.data(), p->descs.size() * sizeof(FindDesc), hipMemcpyHostToDevice) != hipSuccess)
        return CSKV_EHIP;
    if (p->overlap) {
        // default-priority streams; one event per ordering point of the plan
        if (hipStreamCreateWithFlags(&p->rd, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&p->wr, hipStreamNonBlocking) != hipSuccess)
            return CSKV_EHIP;
        for (int j = 0; j < kSlotsScratch; ++j)
            if (hipStreamCreateWithFlags(&p->prep[j], hipStreamNonBlocking) != hipSuccess) return CSKV_EHIP;
        const size_t nev = 8 + 4 * p->segs.size();
        p->events.resize(nev, nullptr);
        for (auto& e : p->events)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CSKV_EHIP;
    }
    p->ready = true;
    return CSKV_OK;
}

uint32_t cskv_program_segments(const cskv_program* p) { return p ? (uint32_t)p->segs.size() : 0; }

static int launch_serial(cskv_program* p, hipStream_t s) {
    cskv_table* t = p->table;
    void* scratch = p->ws + p->scratch_off;
    const size_t sbytes = p->scratch_bytes;
    const FindDesc* d = reinterpret_cast<const FindDesc*>(p->ws);
    for (const Segment& g : p->segs) {
        const Op& o = p->ops[g.first];
        int rc = CSKV_OK;
        if (g.kind == kFind) {
            const unsigned blocks = o.blocks_per_cu > 0 ? (unsigned)(o.blocks_per_cu * t->num_cus) : 0u;
            rc = launch_find_multi(t->view, d + g.desc_off, g.count, g.total, o.group, o.prefetch, blocks, s) ==
                         hipSuccess
                     ? CSKV_OK
                     : CSKV_EHIP;
        } else if (g.kind == kErase) {
            rc = enqueue_erase(t, o.n, o.keys, o.flags, scratch, sbytes, s);
        } else {
            UpsertArgs a{o.n, o.keys, o.vals, o.scores, o.flags,
                         g.kind == kUpsertEvict ? o.ev : EvictOut{nullptr, nullptr, nullptr, nullptr}};
            rc = enqueue_upsert(t, a, scratch, sbytes, s);
        }
        if (rc != CSKV_OK) return rc;
    }
    return CSKV_OK;
}

// Phases ordered by events after the reader/writer rule of Sec. 3.5: a reader (find run, upsert
// route, erase probe) waits for the last writer; a writer (upsert apply, erase clear) waits for
// the last writer and every reader since.  Scratch preparation (clear, dedupe) of an upsert
// touches only its scratch slot and waits only for that slot's previous user to finish.
static int launch_overlapped(cskv_program* p, hipStream_t s) {
    cskv_table* t = p->table;
    const FindDesc* d = reinterpret_cast<const FindDesc*>(p->ws);
    size_t next_ev = 0;
    bool ok = true;
    auto ev = [&]() -> hipEvent_t { return p->events[next_ev++]; };
    auto rec = [&](hipStream_t q) -> hipEvent_t {
        hipEvent_t e = ev();
        ok = ok && hipEventRecord(e, q) == hipSuccess;
        return e;
    };
    auto wait = [&](hipStream_t q, hipEvent_t e) {
        if (e) ok = ok && hipStreamWaitEvent(q, e, 0) == hipSuccess;
    };
    auto chk = [&](hipError_t e) { ok = ok && e == hipSuccess; };
    // fork from the caller's stream
    const hipEvent_t start = rec(s);
    wait(p->rd, start);
    wait(p->wr, start);
    for (hipStream_t q : p->prep) wait(q, start);
    hipEvent_t last_writer = nullptr;
    std::vector<hipEvent_t> readers;
    hipEvent_t slot_free[kSlotsScratch] = {nullptr, nullptr};
    int slot = 0;
    for (const Segment& g : p->segs) {
        if (!ok) break;
        const Op& o = p->ops[g.first];
        if (g.kind == kFind) {
            wait(p->rd, last_writer);
            const unsigned blocks = o.blocks_per_cu > 0 ? (unsigned)(o.blocks_per_cu * t->num_cus) : 0u;
            chk(launch_find_multi(t->view, d + g.desc_off, g.count, g.total, o.group, o.prefetch, blocks, p->rd));
            readers.push_back(rec(p->rd));
            continue;
        }
        const int j = slot;
        slot = (slot + 1) % kSlotsScratch;
        void* scratch = p->ws + p->scratch_off + (size_t)j * p->scratch_bytes;
        hipStream_t pj = p->prep[j];
        wait(pj, slot_free[j]);
        if (g.kind == kErase) {
            if (o.n >= (1ull << 31) || p->scratch_bytes < erase_ws_bytes(o.n)) return CSKV_ENOMEM;
            uint32_t* pos = reinterpret_cast<uint32_t*>(scratch);
            wait(pj, last_writer);
            chk(launch_erase_probe(t->view, o.n, o.keys, o.flags, pos, t->group, pj));
            readers.push_back(rec(pj));
            for (hipEvent_t e : readers) wait(p->wr, e);
            readers.clear();
            chk(launch_erase_clear(t->view, o.n, pos, p->wr));
            last_writer = rec(p->wr);
            slot_free[j] = last_writer;
            continue;
        }
        UpsertArgs a{o.n, o.keys, o.vals, o.scores, o.flags,
                     g.kind == kUpsertEvict ? o.ev : EvictOut{nullptr, nullptr, nullptr, nullptr}};
        UpsertWs w;
        size_t zero_bytes = 0;
        const int rc = plan_upsert(t, a, scratch, p->scratch_bytes, &w, &zero_bytes);
        if (rc != CSKV_OK) return rc;
        chk(launch_upsert_prep(t->view, w, a.n, a.keys, a.scores, a.ev, zero_bytes, pj));
        wait(p->wr, rec(pj));
        chk(launch_upsert_route(t->view, w, a.n, a.keys, a.scores, t->route_group, p->wr));
        readers.push_back(rec(p->wr));
        for (hipEvent_t e : readers) wait(p->wr, e);
        readers.clear();
        chk(launch_upsert_apply(t->view, w, a.n, a.vals, a.ev, p->wr));
        last_writer = rec(p->wr);
        wait(pj, last_writer);
        chk(launch_upsert_finish(w, a.n, a.status, pj));
        slot_free[j] = rec(pj);
    }
    // join everything back into the caller's stream
    wait(s, rec(p->rd));
    wait(s, rec(p->wr));
    for (hipStream_t q : p->prep) wait(s, rec(q));
    return ok ? CSKV_OK : CSKV_EHIP;
}

int cskv_program_launch(cskv_program* p, void* stream) {
    if (!p || !p->ready) return CSKV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return p->overlap ? launch_overlapped(p, s) : launch_serial(p, s);
}

int cskv_program_capture(cskv_program* p, void* stream) {
    if (!p || !p->ready || !stream) return CSKV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CSKV_EHIP;
    const int rc = cskv_program_launch(p, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != CSKV_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != CSKV_OK ? rc : CSKV_EHIP;
    }
    p->graph = g;
    if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) return CSKV_EHIP;
    return CSKV_OK;
}

int cskv_program_replay(cskv_program* p, void* stream) {
    if (!p || !p->ready || !p->exec) return CSKV_EINVAL;
    return hipGraphLaunch(p->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

}  // extern "C"
