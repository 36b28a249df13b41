// Batched programs over one table: consecutive finds merge into one reader run executed by a
// single (optionally persistent) kernel; upserts and erases are serialization points.  In the
// overlapped form the program is a dependency graph of phases (reader/writer rule of Sec. 3.5)
// run on several streams ordered by events, or built once into a hipGraph with explicit edges.
#include <hip/hip_runtime.h>

#include <algorithm>
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
    int group, prefetch, blocks_per_cu;  // tuning snapshot: find and erase-probe shapes
    int route_group;                     // tuning snapshot: upsert routing shape
};

struct Segment {
    int kind;            // kFind = merged run, else the op kind
    uint32_t first;      // first op
    uint32_t count;      // ops in the run (1 otherwise)
    uint64_t total;      // keys in the run
    uint32_t desc_off;   // index of the run's first descriptor
    uint32_t last;       // last op of the run
    uint32_t shape;      // the op whose launch shape the run takes: its largest batch
};

// Phases of the overlapped form.  A find run is one phase; an erase is probe (reader) + clear
// (writer); an upsert is prep (scratch clear + dedupe: touches only its scratch slot), route
// (a reader of the table: the only table memory it writes is that of slots free before the call,
// whose zero digests keep every reader away from them), apply (writer) and finish (status gather,
// scratch only).
enum PhaseKind { kPhFind, kPhProbe, kPhClear, kPhPrep, kPhRoute, kPhApply, kPhFinish };
enum Lane { kLaneRead = 0, kLaneWrite = 1, kLanePrep = 2 };  // kLanePrep + scratch slot

struct Phase {
    int kind;
    int lane;
    uint32_t seg;
    int slot;
    std::vector<uint32_t> deps;  // earlier phases that must be complete
    bool signal = false;         // a phase on another lane, or the final join, waits for it
};

// A byte range an op reads or writes.
struct Range {
    uintptr_t b, e;
    uint32_t op;
    bool write;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace

constexpr int kSlotsScratch = 2;  // scratch regions rotated over the upserts and erases
constexpr int kLanes = kLanePrep + kSlotsScratch;

struct cskv_program {
    cskv_table* table;
    std::vector<Op> ops;
    std::vector<Segment> segs;
    std::vector<FindDesc> descs;
    std::vector<std::vector<uint32_t>> hazards;  // per op: earlier ops whose buffers overlap its own
    std::vector<Phase> phases;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    size_t scratch_off = 0;
    size_t scratch_bytes = 0;  // per slot
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraph_t> children;  // per-phase graphs of the overlapped form's graph
    bool ready = false;
    uint32_t subrounds = 1;  // the table's route sub-rounds when the phases were built
    int overlap = 0;  // 0: one stream; 1: phase graph on reader / writer / prep streams; 2: prep ahead
    hipStream_t lane[kLanes] = {};
    std::vector<hipEvent_t> events;  // one per phase, then the fork event
};

// Ranges of every non-empty op: inputs read, outputs written (device addresses as recorded).
static void op_ranges(const cskv_program* p, std::vector<Range>* out) {
    const uint64_t row = (uint64_t)p->table->view.dim * sizeof(float);
    auto add = [&](const void* ptr, uint64_t bytes, uint32_t op, bool write) {
        if (ptr && bytes) out->push_back(Range{(uintptr_t)ptr, (uintptr_t)ptr + bytes, op, write});
    };
    for (uint32_t i = 0; i < p->ops.size(); ++i) {
        const Op& o = p->ops[i];
        if (o.n == 0) continue;
        add(o.keys, o.n * 8, i, false);
        if (o.kind == kFind) {
            add(o.out, o.n * row, i, true);
            add(o.flags, o.n, i, true);
            add(o.scores_out, o.n * 8, i, true);
        } else if (o.kind == kErase) {
            add(o.flags, o.n, i, true);
        } else {
            add(o.vals, o.n * row, i, false);
            add(o.scores, o.n * 8, i, false);
            add(o.flags, o.n, i, true);
            if (o.kind == kUpsertEvict) {
                add(o.ev.keys, o.n * 8, i, true);
                add(o.ev.vals, o.n * row, i, true);
                add(o.ev.scores, o.n * 8, i, true);
                add(o.ev.count, 8, i, true);
            }
        }
    }
}

// hazards[j] = earlier ops i < j such that one of the two writes bytes the other reads or writes.
static void find_hazards(cskv_program* p) {
    std::vector<Range> r;
    op_ranges(p, &r);
    std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.b < b.b; });
    p->hazards.assign(p->ops.size(), {});
    std::vector<const Range*> active;  // ranges that may still overlap the next one in start order
    for (const Range& x : r) {
        size_t keep = 0;
        for (const Range* y : active) {
            if (y->e <= x.b) continue;  // ended before x starts: drop
            active[keep++] = y;
            if (y->op != x.op && (y->write || x.write))
                p->hazards[std::max(x.op, y->op)].push_back(std::min(x.op, y->op));
        }
        active.resize(keep);
        active.push_back(&x);
    }
    for (auto& h : p->hazards) {
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
    }
}

static void build_plan(cskv_program* p) {
    p->segs.clear();
    p->descs.clear();
    for (uint32_t i = 0; i < p->ops.size(); ++i) {
        const Op& o = p->ops[i];
        if (o.n == 0) continue;
        if (o.kind == kFind) {
            // a find joins the open run unless its buffers overlap those of a find already in it
            bool open = !p->segs.empty() && p->segs.back().kind == kFind;
            if (open)
                for (uint32_t h : p->hazards[i])
                    if (h >= p->segs.back().first) open = false;
            if (!open) p->segs.push_back(Segment{kFind, i, 0, 0, (uint32_t)p->descs.size(), i, i});
            Segment& s = p->segs.back();
            p->descs.push_back(FindDesc{o.keys, o.out, o.flags, o.scores_out, s.total, o.n});
            s.count += 1;
            s.total += o.n;
            s.last = i;
            if (o.n > p->ops[s.shape].n) s.shape = i;
        } else {
            p->segs.push_back(Segment{o.kind, i, 1, o.n, 0, i, i});
        }
    }
}

// The phase graph.  Readers (find runs, routes, probes) depend on the last writer; writers
// (applies, clears) on the last writer and every reader since; the first phase of an upsert or
// erase on the previous user of its scratch slot.  A segment whose buffers overlap an earlier
// segment's additionally starts after that segment's last phase.
static void build_phases(cskv_program* p) {
    p->phases.clear();
    std::vector<int> seg_of(p->ops.size(), -1);
    for (uint32_t s = 0; s < p->segs.size(); ++s)
        for (uint32_t i = p->segs[s].first; i <= p->segs[s].last; ++i) seg_of[i] = (int)s;
    std::vector<int> seg_end(p->segs.size(), -1);  // last phase of each segment
    int last_writer = -1;
    std::vector<int> readers;
    int slot_free[kSlotsScratch] = {-1, -1};
    int slot = 0;
    auto add = [&](int kind, int lane, uint32_t seg, int sl, const std::vector<int>& deps) -> int {
        Phase ph;
        ph.kind = kind;
        ph.lane = lane;
        ph.seg = seg;
        ph.slot = sl;
        for (int d : deps)
            if (d >= 0) ph.deps.push_back((uint32_t)d);
        std::sort(ph.deps.begin(), ph.deps.end());
        ph.deps.erase(std::unique(ph.deps.begin(), ph.deps.end()), ph.deps.end());
        p->phases.push_back(std::move(ph));
        return (int)p->phases.size() - 1;
    };
    for (uint32_t s = 0; s < p->segs.size(); ++s) {
        const Segment& g = p->segs[s];
        std::vector<int> entry;  // ends of earlier segments whose buffers overlap this one's
        for (uint32_t i = g.first; i <= g.last; ++i) {
            if (p->ops[i].n == 0) continue;
            for (uint32_t h : p->hazards[i])
                if (seg_of[h] >= 0 && seg_of[h] != (int)s) entry.push_back(seg_end[seg_of[h]]);
        }
        if (g.kind == kFind) {
            entry.push_back(last_writer);
            const int f = add(kPhFind, kLaneRead, s, 0, entry);
            readers.push_back(f);
            seg_end[s] = f;
            continue;
        }
        const int j = slot;
        slot = (slot + 1) % kSlotsScratch;
        entry.push_back(slot_free[j]);
        if (g.kind == kErase) {
            entry.push_back(last_writer);
            const int probe = add(kPhProbe, kLanePrep + j, s, j, entry);
            std::vector<int> w = readers;
            w.push_back(probe);
            w.push_back(last_writer);
            const int clear = add(kPhClear, kLaneWrite, s, j, w);
            readers.clear();
            last_writer = clear;
            slot_free[j] = clear;
            seg_end[s] = clear;
            continue;
        }
        const int prep = add(kPhPrep, kLanePrep + j, s, j, entry);
        std::vector<int> w;
        if (p->table->subrounds == 1) {  // routing reads the table beside the running readers
            const int route = add(kPhRoute, kLaneWrite, s, j, {prep, last_writer});
            readers.push_back(route);
        } else {  // sub-rounds: every round's routing runs inside the apply phase
            w.push_back(prep);
        }
        w.insert(w.end(), readers.begin(), readers.end());
        w.push_back(last_writer);
        const int apply = add(kPhApply, kLaneWrite, s, j, w);
        readers.clear();
        last_writer = apply;
        int end = apply;
        if (p->ops[g.first].flags) end = add(kPhFinish, kLanePrep + j, s, j, {apply});
        slot_free[j] = end;
        seg_end[s] = end;
    }
    // prep ahead: every phase but the scratch preparations runs in program order on one stream
    if (p->overlap == 2) {
        int prev = -1;
        for (uint32_t i = 0; i < p->phases.size(); ++i) {
            Phase& ph = p->phases[i];
            if (ph.kind == kPhPrep) continue;
            ph.lane = kLaneWrite;
            if (prev >= 0 && std::find(ph.deps.begin(), ph.deps.end(), (uint32_t)prev) == ph.deps.end()) {
                ph.deps.push_back((uint32_t)prev);  // explicit in the graph form; stream order in the event form
                std::sort(ph.deps.begin(), ph.deps.end());
            }
            prev = (int)i;
        }
    }
    // a phase signals when a phase on another lane waits for it, or when it is its lane's last
    int lane_last[kLanes];
    std::fill(lane_last, lane_last + kLanes, -1);
    for (uint32_t i = 0; i < p->phases.size(); ++i) {
        const Phase& ph = p->phases[i];
        for (uint32_t d : ph.deps)
            if (p->phases[d].lane != ph.lane) p->phases[d].signal = true;
        lane_last[ph.lane] = (int)i;
    }
    for (int l = 0; l < kLanes; ++l)
        if (lane_last[l] >= 0) p->phases[lane_last[l]].signal = true;
}

static size_t scratch_need(const cskv_program* p) {
    size_t need = 256;
    for (const Op& o : p->ops) {
        if (o.n == 0) continue;
        size_t b = 0;
        if (o.kind == kUpsert || o.kind == kUpsertEvict)
            b = upsert_layout(o.n, p->table->view.nbuckets, p->table->subrounds).total;
        else if (o.kind == kErase) b = erase_ws_bytes(o.n);
        if (b > need) need = b;
    }
    return need;
}

static void drop_graph(cskv_program* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (hipGraph_t g : p->children) (void)hipGraphDestroy(g);
    p->exec = nullptr;
    p->graph = nullptr;
    p->children.clear();
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
    drop_graph(p);
    for (hipEvent_t e : p->events)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : p->lane)
        if (q) (void)hipStreamDestroy(q);
    delete p;
    return CSKV_OK;
}

int cskv_program_set_overlap(cskv_program* p, int mode) {
    if (!p || p->ready || mode < 0 || mode > 2) return CSKV_EINVAL;
    p->overlap = mode;
    return CSKV_OK;
}

// every operation keeps the launch shapes the table had when it was added (results never depend
// on them; a tuner sets them per batch size before each add)
static int add_op(cskv_program* p, Op o) {
    if (!p || p->ready) return CSKV_EINVAL;
    if (o.n >= (1ull << 31)) return CSKV_EINVAL;
    o.group = p->table->group;
    o.prefetch = p->table->prefetch_b2;
    o.blocks_per_cu = p->table->blocks_per_cu;
    o.route_group = p->table->route_group;
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
    if (!p || p->ready || !d_ws || !aligned(d_ws, 256)) return CSKV_EINVAL;
    if (ws_bytes < cskv_program_workspace_bytes(p)) return CSKV_ENOMEM;
    p->subrounds = p->table->subrounds;
    find_hazards(p);
    build_plan(p);
    p->ws = reinterpret_cast<uint8_t*>(d_ws);
    p->ws_bytes = ws_bytes;
    p->scratch_off = align256(p->descs.size() * sizeof(FindDesc) + 1);
    p->scratch_bytes = align256(scratch_need(p));
    if (!p->descs.empty() &&
        hipMemcpy(p->ws, p->descs.data(), p->descs.size() * sizeof(FindDesc), hipMemcpyHostToDevice) != hipSuccess)
        return CSKV_EHIP;
    if (p->overlap) {
        build_phases(p);
        // default-priority streams, one per lane; one event per phase and one for the fork
        for (hipStream_t& q : p->lane)
            if (!q && hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) return CSKV_EHIP;
        p->events.assign(p->phases.size() + 1, nullptr);
        for (auto& e : p->events)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CSKV_EHIP;
    }
    p->ready = true;
    return CSKV_OK;
}

uint32_t cskv_program_segments(const cskv_program* p) { return p ? (uint32_t)p->segs.size() : 0; }

uint32_t cskv_program_phases(const cskv_program* p) { return p ? (uint32_t)p->phases.size() : 0; }

}  // extern "C"

static int run_find_run(cskv_program* p, const Segment& g, hipStream_t s) {
    const cskv_table* t = p->table;
    const Op& o = p->ops[g.shape];  // the largest batch of the run sets the shape
    const FindDesc* d = reinterpret_cast<const FindDesc*>(p->ws);
    const unsigned blocks = o.blocks_per_cu > 0 ? (unsigned)(o.blocks_per_cu * t->num_cus) : 0u;
    return launch_find_multi(t->view, d + g.desc_off, g.count, g.total, o.group, o.prefetch, blocks, s) == hipSuccess
               ? CSKV_OK
               : CSKV_EHIP;
}

static UpsertArgs upsert_args(const Op& o) {
    return UpsertArgs{o.n, o.keys, o.vals, o.scores, o.flags,
                      o.kind == kUpsertEvict ? o.ev : EvictOut{nullptr, nullptr, nullptr, nullptr}};
}

static int launch_serial(cskv_program* p, hipStream_t s) {
    cskv_table* t = p->table;
    void* scratch = p->ws + p->scratch_off;
    const size_t sbytes = p->scratch_bytes;
    for (const Segment& g : p->segs) {
        const Op& o = p->ops[g.first];
        int rc = CSKV_OK;
        if (g.kind == kFind) rc = run_find_run(p, g, s);
        else if (g.kind == kErase) rc = enqueue_erase(t, o.n, o.keys, o.flags, scratch, sbytes, s, o.group);
        else rc = enqueue_upsert(t, upsert_args(o), scratch, sbytes, s, o.route_group);
        if (rc != CSKV_OK) return rc;
    }
    return CSKV_OK;
}

// Enqueue the kernels of one phase on `s`.
static int run_phase(cskv_program* p, const Phase& ph, hipStream_t s) {
    cskv_table* t = p->table;
    const Segment& g = p->segs[ph.seg];
    if (ph.kind == kPhFind) return run_find_run(p, g, s);
    const Op& o = p->ops[g.first];
    void* scratch = p->ws + p->scratch_off + (size_t)ph.slot * p->scratch_bytes;
    hipError_t e = hipSuccess;
    if (ph.kind == kPhProbe || ph.kind == kPhClear) {
        if (p->scratch_bytes < erase_ws_bytes(o.n)) return CSKV_ENOMEM;
        uint32_t* pos = reinterpret_cast<uint32_t*>(scratch);
        e = ph.kind == kPhProbe ? launch_erase_probe(t->view, o.n, o.keys, o.flags, pos, o.group, s)
                                : launch_erase_clear(t->view, o.n, pos, s);
        return e == hipSuccess ? CSKV_OK : CSKV_EHIP;
    }
    const UpsertArgs a = upsert_args(o);
    UpsertWs w;
    size_t zero_bytes = 0;
    const int rc = plan_upsert(t, a, scratch, p->scratch_bytes, &w, &zero_bytes);
    if (rc != CSKV_OK) return rc;
    switch (ph.kind) {
        case kPhPrep: e = launch_upsert_prep(t->view, w, a.n, a.keys, a.scores, a.ev, zero_bytes, s); break;
        // with route sub-rounds every round routes after the previous one applied: all of it runs
        // in the apply phase (on the writer lane, after the concurrent readers)
        case kPhRoute:
            if (w.rounds == 1) e = launch_upsert_route(t->view, w, a.n, a.keys, a.vals, a.scores, o.route_group, s);
            break;
        case kPhApply:
            e = w.rounds == 1 ? launch_upsert_apply(t->view, w, a.n, a.vals, a.ev, s)
                              : launch_upsert_rounds(t->view, w, a.n, a.keys, a.vals, a.scores, a.ev, o.route_group, s);
            break;
        default: e = launch_upsert_finish(w, a.n, a.status, t->view.dim, s); break;
    }
    return e == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

// The phase graph on the lane streams: each phase waits for the events of its dependencies on
// other lanes (same-lane order is stream order) and records its own event when another lane or
// the join waits for it.  The lanes fork from and join back into the caller's stream.
static int launch_overlapped(cskv_program* p, hipStream_t s) {
    hipEvent_t fork = p->events.back();
    bool ok = hipEventRecord(fork, s) == hipSuccess;
    for (hipStream_t q : p->lane) ok = ok && hipStreamWaitEvent(q, fork, 0) == hipSuccess;
    int rc = CSKV_OK;
    int lane_last[kLanes];
    std::fill(lane_last, lane_last + kLanes, -1);
    for (uint32_t i = 0; i < p->phases.size() && ok && rc == CSKV_OK; ++i) {
        const Phase& ph = p->phases[i];
        hipStream_t q = p->lane[ph.lane];
        for (uint32_t d : ph.deps)
            if (p->phases[d].lane != ph.lane) ok = ok && hipStreamWaitEvent(q, p->events[d], 0) == hipSuccess;
        if (!ok) break;
        rc = run_phase(p, ph, q);
        if (rc == CSKV_OK && ph.signal) ok = hipEventRecord(p->events[i], q) == hipSuccess;
        lane_last[ph.lane] = (int)i;
    }
    // join: the caller's stream waits for the last phase of every lane
    for (int l = 0; l < kLanes; ++l)
        if (lane_last[l] >= 0) ok = ok && hipStreamWaitEvent(s, p->events[lane_last[l]], 0) == hipSuccess;
    if (rc != CSKV_OK) return rc;
    return ok ? CSKV_OK : CSKV_EHIP;
}

// The phase graph as a hipGraph: each phase is recorded alone by stream capture on `s` (one
// stream, no events) into a child graph, and the parent graph gets one child node per phase with
// the phase's dependencies as its edges.
static int build_graph_overlapped(cskv_program* p, hipStream_t s) {
    hipGraph_t g = nullptr;
    if (hipGraphCreate(&g, 0) != hipSuccess) return CSKV_EHIP;
    p->graph = g;
    std::vector<hipGraphNode_t> node(p->phases.size(), nullptr);
    std::vector<hipGraphNode_t> deps;
    for (uint32_t i = 0; i < p->phases.size(); ++i) {
        const Phase& ph = p->phases[i];
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CSKV_EHIP;
        const int rc = run_phase(p, ph, s);
        hipGraph_t child = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &child);
        if (child) p->children.push_back(child);
        if (rc != CSKV_OK) return rc;
        if (e != hipSuccess || !child) return CSKV_EHIP;
        deps.clear();
        for (uint32_t d : ph.deps) deps.push_back(node[d]);
        if (hipGraphAddChildGraphNode(&node[i], g, deps.empty() ? nullptr : deps.data(), deps.size(), child) !=
            hipSuccess)
            return CSKV_EHIP;
    }
    return hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

// a program holds its table as one call: an inserter if it changes the table, else a reader
static int program_role(const cskv_program* p) {
    for (const Op& o : p->ops)
        if (o.kind != kFind) return kInserter;
    return kReader;
}

extern "C" {

// the table's route sub-rounds changed since set_workspace: phases and scratch no longer fit
static bool stale(const cskv_program* p) { return p->table->subrounds != p->subrounds; }

int cskv_program_launch(cskv_program* p, void* stream) {
    if (!p || !p->ready || stale(p)) return CSKV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RoleScope role(p->table, program_role(p), s);
    if (!role.ok()) return CSKV_EHIP;
    return p->overlap ? launch_overlapped(p, s) : launch_serial(p, s);
}

int cskv_program_capture(cskv_program* p, void* stream) {
    if (!p || !p->ready || !stream || stale(p)) return CSKV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    drop_graph(p);
    int rc;
    if (p->overlap) {
        rc = build_graph_overlapped(p, s);
    } else {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CSKV_EHIP;
        rc = launch_serial(p, s);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        p->graph = g;
        if (rc == CSKV_OK && (e != hipSuccess || !g)) rc = CSKV_EHIP;
        if (rc == CSKV_OK && hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = CSKV_EHIP;
    }
    if (rc != CSKV_OK) drop_graph(p);
    return rc;
}

int cskv_program_replay(cskv_program* p, void* stream) {
    if (!p || !p->ready || !p->exec || stale(p)) return CSKV_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RoleScope role(p->table, program_role(p), s);
    if (!role.ok()) return CSKV_EHIP;
    return hipGraphLaunch(p->exec, s) == hipSuccess ? CSKV_OK : CSKV_EHIP;
}

}  // extern "C"
