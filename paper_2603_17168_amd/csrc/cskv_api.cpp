// C-ABI of the cache-semantic hash table: argument checks, storage and workspace layout,
// kernel sequencing.  No allocation happens here: storage and workspaces belong to the caller.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/cskv.h"
#include "cskv_internal.h"

namespace cskv {

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

StorageLayout storage_layout(uint64_t nb, uint32_t dim, uint64_t hbm_rows) {
    StorageLayout L;
    size_t o = 0;
    L.off_dig = o;    o = align256(o + nb * kSlots);
    L.off_keys = o;   o = align256(o + nb * kSlots * 8);
    L.off_scores = o; o = align256(o + nb * kSlots * 8);
    L.off_vals = o;   o = align256(o + hbm_rows * (size_t)dim * 4);
    L.off_cnt = o;    o = align256(o + nb * 8);
    L.off_bmin = o;   o = align256(o + nb * 16);
    L.off_clock = o;  o = align256(o + 8);
    L.total = o;
    return L;
}

// per-bucket inline capacity: about mean + 5 sd + 3 operations per bucket (Poisson), 4..16
static uint32_t inline_capacity(uint64_t n, uint64_t nb) {
    const double mu = (double)n / (double)nb;
    const double want = mu + 5.0 * __builtin_sqrt(mu) + 3.0;
    uint32_t c = 4;
    while (c < (uint32_t)kFastMax && (double)c < want) c <<= 1;
    return c;
}

UpsertLayout upsert_layout(uint64_t n, uint64_t nb, uint32_t rounds, bool compact) {
    UpsertLayout L;
    uint64_t P = 64;
    int logP = 6;
    while (P < 2 * n) {
        P <<= 1;
        ++logP;
    }
    L.P = P;
    L.logP = logP;
    L.cap = compact ? 0u : inline_capacity(n, nb);
    const uint64_t nl = nb * L.cap;
    const uint64_t nslow = n < nb ? n : nb;
    size_t o = 0;
    // zeroed on every call: dedupe set, overflow keys, counters (and the LFU sums)
    L.off_dd = o;      o = align256(o + P * sizeof(DedupeEntry));
    L.off_okey = o;    o = align256(o + P * 8);
    L.off_ctr = o;     o = align256(o + 64 * 4);
    L.off_zero_end = o;
    L.off_inc = o;     o = align256(o + P * 8);
    L.off_sat = o;     o = align256(o + P * 4);
    L.off_minc = o;    o = align256(o + P * 8);
    L.off_zero_end_lfu = o;
    L.off_sstat = o;   o = align256(o + P);
    L.off_slot_of = o; o = align256(o + n * 4);
    L.off_rinc = o;    o = align256(o + n * 8);
    L.off_il = o;      o = align256(o + nl * sizeof(OpEntry));
    L.off_ol = o;      o = align256(o + P * sizeof(OpEntry));
    L.off_slow = o;    o = align256(o + nslow * 4);
    L.off_touched = o; o = align256(o + nslow * 4);
    L.off_rank = o;    o = align256(o + (rounds > 1 ? n * 4 : 0));
    L.off_bsum = o;    o = align256(o + (rounds > 1 ? ((n + 255) / 256) * 4 : 0));
    L.list_mode = compact || n * 4 <= nb;  // apply visits only the touched buckets (route lists them)
    L.total = o;
    return L;
}

size_t erase_ws_bytes(uint64_t n) { return align256(n * 4); }

}  // namespace cskv

using namespace cskv;

static inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }
static inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
static inline int hip_rc(hipError_t e) { return e == hipSuccess ? CSKV_OK : CSKV_EHIP; }

static bool valid_geometry(uint64_t capacity, uint32_t bucket_size, uint32_t dim, uint64_t* nb_out) {
    if (bucket_size != (uint32_t)kSlots) return false;
    if (capacity == 0 || capacity % kSlots) return false;
    const uint64_t nb = capacity / kSlots;
    if (nb & (nb - 1)) return false;
    if (nb > (1ull << 24)) return false;
    if (dim < 4 || dim > 1024 || (dim & 3)) return false;
    *nb_out = nb;
    return true;
}

extern "C" {

size_t cskv_table_bytes(uint64_t capacity, uint32_t bucket_size, uint32_t dim) {
    uint64_t nb;
    if (!valid_geometry(capacity, bucket_size, dim, &nb)) return 0;
    return storage_layout(nb, dim, capacity).total;
}

size_t cskv_table_bytes_tiered(uint64_t capacity, uint32_t bucket_size, uint32_t dim, uint64_t hbm_value_rows) {
    uint64_t nb;
    if (!valid_geometry(capacity, bucket_size, dim, &nb) || hbm_value_rows > capacity) return 0;
    return storage_layout(nb, dim, hbm_value_rows).total;
}

size_t cskv_host_value_bytes(uint64_t capacity, uint32_t dim, uint64_t hbm_value_rows) {
    uint64_t nb;
    if (!valid_geometry(capacity, (uint32_t)kSlots, dim, &nb) || hbm_value_rows > capacity) return 0;
    return (size_t)(capacity - hbm_value_rows) * dim * 4;
}

int cskv_create(cskv_table** out, uint64_t capacity, uint32_t bucket_size, uint32_t dim, int mode,
                int score_policy, void* d_storage, size_t storage_bytes, void* stream) {
    return cskv_create_tiered(out, capacity, bucket_size, dim, mode, score_policy, d_storage, storage_bytes,
                              capacity, nullptr, 0, stream);
}

int cskv_create_tiered(cskv_table** out, uint64_t capacity, uint32_t bucket_size, uint32_t dim, int mode,
                       int score_policy, void* d_storage, size_t storage_bytes, uint64_t hbm_value_rows,
                       void* h_values, size_t host_bytes, void* stream) {
    if (!out || !d_storage) return CSKV_EINVAL;
    *out = nullptr;
    if (mode != CSKV_MODE_SINGLE && mode != CSKV_MODE_DUAL) return CSKV_EINVAL;
    if (score_policy != CSKV_SCORE_CUSTOM && score_policy != CSKV_SCORE_LRU && score_policy != CSKV_SCORE_LFU)
        return CSKV_EINVAL;
    if (bucket_size != (uint32_t)kSlots) return CSKV_EUNSUPPORTED;
    uint64_t nb;
    if (!valid_geometry(capacity, bucket_size, dim, &nb)) return CSKV_EINVAL;
    if (!aligned(d_storage, 256) || hbm_value_rows > capacity) return CSKV_EINVAL;
    const StorageLayout L = storage_layout(nb, dim, hbm_value_rows);
    if (storage_bytes < L.total) return CSKV_ENOMEM;
    // the host tier: pinned host memory, addressed by kernels through its device alias
    float* host_rows = nullptr;
    if (hbm_value_rows < capacity) {
        if (!h_values || !aligned(h_values, 16)) return CSKV_EINVAL;
        if (host_bytes < (size_t)(capacity - hbm_value_rows) * dim * 4) return CSKV_ENOMEM;
        void* dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, h_values, 0) != hipSuccess || !dptr) {
            (void)hipGetLastError();
            return CSKV_EINVAL;  // not pinned (hipHostMalloc) host memory
        }
        host_rows = reinterpret_cast<float*>(dptr);
    }
    cskv_table* t = new (std::nothrow) cskv_table;
    if (!t) return CSKV_ENOMEM;
    uint8_t* base = reinterpret_cast<uint8_t*>(d_storage);
    t->view.dig = base + L.off_dig;
    t->view.keys = reinterpret_cast<uint64_t*>(base + L.off_keys);
    t->view.scores = reinterpret_cast<uint64_t*>(base + L.off_scores);
    t->view.vals = reinterpret_cast<float*>(base + L.off_vals);
    t->view.vals_host = host_rows;
    t->view.hbm_rows = hbm_value_rows;
    t->view.cnt = reinterpret_cast<uint64_t*>(base + L.off_cnt);
    t->view.bmin = reinterpret_cast<uint64_t*>(base + L.off_bmin);
    t->view.clock = reinterpret_cast<uint64_t*>(base + L.off_clock);
    t->view.nbuckets = nb;
    t->view.bmask = (uint32_t)(nb - 1);
    t->view.dim = dim;
    t->view.dual = (mode == CSKV_MODE_DUAL);
    t->view.policy = score_policy;
    t->capacity = capacity;
    t->mode = mode;
    t->policy = score_policy;
    t->group = 8;
    t->route_group = 8;
    t->prefetch_b2 = 0;
    t->blocks_per_cu = 0;
    t->find_pairs = 0;
    t->find_digest = 1;
    t->subrounds = 1;
    t->roles = new (std::nothrow) TableLock();
    if (!t->roles) {
        delete t;
        return CSKV_ENOMEM;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete t;
        return CSKV_EHIP;
    }
    t->num_cus = cus;
    t->device = dev;
    int rc = hip_rc(launch_clear_table(t->view, as_stream(stream)));
    if (rc == CSKV_OK) rc = hip_rc(launch_fill_zero(t->view.clock, 8, as_stream(stream)));
    if (rc != CSKV_OK) {
        delete t;
        return rc;
    }
    *out = t;
    return CSKV_OK;
}

int cskv_destroy(cskv_table* table) {
    delete table;
    return CSKV_OK;
}

int cskv_clear(cskv_table* table, void* stream) {
    if (!table) return CSKV_EINVAL;
    RoleScope role(table, kInserter, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_clear_table(table->view, as_stream(stream)));
}

size_t cskv_workspace_bytes(const cskv_table* table, int op, uint64_t n) {
    if (!table) return 0;
    switch (op) {
        case CSKV_OP_FIND: return 0;
        case CSKV_OP_INSERT_OR_ASSIGN:
        case CSKV_OP_INSERT_AND_EVICT:
        case CSKV_OP_ASSIGN:
        case CSKV_OP_FIND_OR_INSERT: return upsert_layout(n, table->view.nbuckets, table->subrounds).total;
        case CSKV_OP_ERASE: return erase_ws_bytes(n);
        default: return 0;
    }
}

static bool n_ok(uint64_t n) { return n < (1ull << 31); }

int cskv_find(cskv_table* table, uint64_t n, const uint64_t* d_keys, float* d_values_out, uint8_t* d_found,
              uint64_t* d_scores_out, void* stream) {
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!d_keys || !d_values_out || !d_found) return CSKV_EINVAL;
    if (!aligned(d_keys, 8) || !aligned(d_values_out, 16) || (d_scores_out && !aligned(d_scores_out, 8)))
        return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    if (!table->find_digest)
        return hip_rc(launch_find_nodigest(table->view, n, d_keys, d_values_out, d_found, d_scores_out, table->group,
                                           as_stream(stream)));
    return hip_rc(launch_find(table->view, n, d_keys, d_values_out, d_found, d_scores_out, table->group,
                              table->prefetch_b2, table->find_pairs, as_stream(stream)));
}

}  // extern "C"

namespace cskv {

int plan_upsert(cskv_table* table, const UpsertArgs& a, void* d_ws, size_t ws_bytes, UpsertWs* out,
                size_t* zero_out, bool need_vals, bool compact) {
    const uint64_t n = a.n;
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!a.keys || (need_vals && !a.vals) || !d_ws) return CSKV_EINVAL;
    if (table->policy == CSKV_SCORE_CUSTOM && !a.scores) return CSKV_EINVAL;
    if (!aligned(a.keys, 8) || (a.vals && !aligned(a.vals, 16)) || !aligned(d_ws, 256) ||
        (a.scores && !aligned(a.scores, 8)) || (a.out && !aligned(a.out, 16)))
        return CSKV_EINVAL;
    const UpsertLayout L = upsert_layout(n, table->view.nbuckets, table->subrounds, compact);
    if (ws_bytes < L.total) return CSKV_ENOMEM;
    uint8_t* b = reinterpret_cast<uint8_t*>(d_ws);
    UpsertWs& w = *out;
    w.dd = reinterpret_cast<DedupeEntry*>(b + L.off_dd);
    w.okey = reinterpret_cast<uint64_t*>(b + L.off_okey);
    w.ctr = reinterpret_cast<uint32_t*>(b + L.off_ctr);
    w.inc = reinterpret_cast<uint64_t*>(b + L.off_inc);
    w.sat = reinterpret_cast<uint32_t*>(b + L.off_sat);
    w.sstat = b + L.off_sstat;
    w.slot_of = reinterpret_cast<uint32_t*>(b + L.off_slot_of);
    w.rinc = reinterpret_cast<uint64_t*>(b + L.off_rinc);
    w.minc = reinterpret_cast<uint64_t*>(b + L.off_minc);
    w.il = reinterpret_cast<OpEntry*>(b + L.off_il);
    w.ol = reinterpret_cast<OpEntry*>(b + L.off_ol);
    w.slow = reinterpret_cast<uint32_t*>(b + L.off_slow);
    w.touched = reinterpret_cast<uint32_t*>(b + L.off_touched);
    w.rank = reinterpret_cast<uint32_t*>(b + L.off_rank);
    w.bsum = reinterpret_cast<uint32_t*>(b + L.off_bsum);
    w.rounds = (int)table->subrounds;
    w.round = 0;
    w.P = L.P;
    w.logP = L.logP;
    w.cap = L.cap;
    w.list_mode = L.list_mode;
    w.out = a.out;
    *zero_out = table->policy == CSKV_SCORE_LFU ? L.off_zero_end_lfu : L.off_zero_end;
    return CSKV_OK;
}

int enqueue_upsert(cskv_table* table, const UpsertArgs& a, void* d_ws, size_t ws_bytes, hipStream_t stream, int group,
                   bool compact) {
    UpsertWs w;
    size_t zero_bytes = 0;
    const int rc = plan_upsert(table, a, d_ws, ws_bytes, &w, &zero_bytes, true, compact);
    if (rc != CSKV_OK || a.n == 0) return rc;
    return hip_rc(launch_upsert(table->view, w, a.n, a.keys, a.vals, a.scores, a.status, a.ev, zero_bytes,
                                group > 0 ? group : table->route_group, stream));
}

int enqueue_erase(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint8_t* d_erased, void* d_ws,
                  size_t ws_bytes, hipStream_t stream, int group) {
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!d_keys || !d_ws || !aligned(d_keys, 8) || !aligned(d_ws, 256)) return CSKV_EINVAL;
    if (ws_bytes < erase_ws_bytes(n)) return CSKV_ENOMEM;
    return hip_rc(launch_erase(table->view, n, d_keys, d_erased, reinterpret_cast<uint32_t*>(d_ws),
                               group > 0 ? group : table->group, stream));
}

}  // namespace cskv

extern "C" {

int cskv_insert_or_assign(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                          const uint64_t* d_scores, uint8_t* d_status, void* d_ws, size_t ws_bytes, void* stream) {
    UpsertArgs a{n, d_keys, d_values, d_scores, d_status, EvictOut{nullptr, nullptr, nullptr, nullptr}};
    RoleScope role(table, kInserter, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return enqueue_upsert(table, a, d_ws, ws_bytes, as_stream(stream));
}

int cskv_insert_and_evict(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                          const uint64_t* d_scores, uint8_t* d_status, uint64_t* d_ev_keys, float* d_ev_values,
                          uint64_t* d_ev_scores, uint64_t* d_n_evicted, void* d_ws, size_t ws_bytes,
                          void* stream) {
    if (!table) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!d_status || !d_ev_keys || !d_ev_values || !d_ev_scores || !d_n_evicted) return CSKV_EINVAL;
    if (!aligned(d_ev_keys, 8) || !aligned(d_ev_values, 16) || !aligned(d_ev_scores, 8) || !aligned(d_n_evicted, 8))
        return CSKV_EINVAL;
    UpsertArgs a{n, d_keys, d_values, d_scores, d_status, EvictOut{d_ev_keys, d_ev_values, d_ev_scores, d_n_evicted}};
    RoleScope role(table, kInserter, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return enqueue_upsert(table, a, d_ws, ws_bytes, as_stream(stream));
}

int cskv_erase(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint8_t* d_erased, void* d_ws, size_t ws_bytes,
               void* stream) {
    if (!table) return CSKV_EINVAL;
    RoleScope role(table, kInserter, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return enqueue_erase(table, n, d_keys, d_erased, d_ws, ws_bytes, as_stream(stream));
}

int cskv_size(cskv_table* table, uint64_t* d_size, void* stream) {
    if (!table || !d_size || !aligned(d_size, 8)) return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_size(table->view, d_size, as_stream(stream)));
}

int cskv_export(cskv_table* table, uint64_t bucket_begin, uint64_t bucket_end, uint64_t* d_keys, float* d_values,
                uint64_t* d_scores, uint64_t* d_slots, uint64_t* d_count, void* stream) {
    if (!table || !d_keys || !d_count) return CSKV_EINVAL;
    if (bucket_begin > bucket_end || bucket_end > table->view.nbuckets) return CSKV_EINVAL;
    if (!aligned(d_keys, 8) || !aligned(d_count, 8) || (d_values && !aligned(d_values, 16)) ||
        (d_scores && !aligned(d_scores, 8)) || (d_slots && !aligned(d_slots, 8)))
        return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_export(table->view, bucket_begin, bucket_end, d_keys, d_values, d_scores, d_slots, d_count,
                                0, as_stream(stream)));
}

int cskv_export_if(cskv_table* table, uint64_t bucket_begin, uint64_t bucket_end, uint64_t min_score,
                   uint64_t* d_keys, float* d_values, uint64_t* d_scores, uint64_t* d_slots, uint64_t* d_count,
                   void* stream) {
    if (!table || !d_keys || !d_count) return CSKV_EINVAL;
    if (bucket_begin > bucket_end || bucket_end > table->view.nbuckets) return CSKV_EINVAL;
    if (!aligned(d_keys, 8) || !aligned(d_count, 8) || (d_values && !aligned(d_values, 16)) ||
        (d_scores && !aligned(d_scores, 8)) || (d_slots && !aligned(d_slots, 8)))
        return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_export(table->view, bucket_begin, bucket_end, d_keys, d_values, d_scores, d_slots, d_count,
                                min_score, as_stream(stream)));
}

int cskv_contains(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint8_t* d_found, void* stream) {
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!d_keys || !d_found || !aligned(d_keys, 8)) return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_locate(table->view, n, d_keys, d_found, nullptr, nullptr, table->group, as_stream(stream)));
}

int cskv_find_ptr(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint64_t* d_ptrs, uint8_t* d_found,
                  uint64_t* d_scores_out, void* stream) {
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    if (!d_keys || !d_ptrs || !d_found || !aligned(d_keys, 8) || !aligned(d_ptrs, 8) ||
        (d_scores_out && !aligned(d_scores_out, 8)))
        return CSKV_EINVAL;
    RoleScope role(table, kReader, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return hip_rc(launch_locate(table->view, n, d_keys, d_found, d_ptrs, d_scores_out, table->group, as_stream(stream)));
}

static int enqueue_assign(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                          const uint64_t* d_scores, uint8_t* d_found, void* d_ws, size_t ws_bytes, void* stream) {
    if (!table || !n_ok(n)) return CSKV_EINVAL;
    if (n == 0) return CSKV_OK;
    UpsertArgs a{n, d_keys, d_values, d_scores, nullptr, EvictOut{nullptr, nullptr, nullptr, nullptr}};
    UpsertWs w;
    size_t zero_bytes = 0;
    const int rc = plan_upsert(table, a, d_ws, ws_bytes, &w, &zero_bytes, false);
    if (rc != CSKV_OK) return rc;
    hipStream_t s = as_stream(stream);
    RoleScope role(table, kUpdater, s);
    if (!role.ok()) return CSKV_EHIP;
    const hipError_t e = launch_upsert_prep(table->view, w, n, d_keys, d_scores, a.ev, zero_bytes, s);
    if (e != hipSuccess) return CSKV_EHIP;
    return hip_rc(launch_assign(table->view, w, n, d_keys, d_values, d_scores, d_found, table->group, s));
}

int cskv_assign(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values, const uint64_t* d_scores,
                uint8_t* d_found, void* d_ws, size_t ws_bytes, void* stream) {
    if (n && !d_values) return CSKV_EINVAL;
    return enqueue_assign(table, n, d_keys, d_values, d_scores, d_found, d_ws, ws_bytes, stream);
}

int cskv_assign_scores(cskv_table* table, uint64_t n, const uint64_t* d_keys, const uint64_t* d_scores,
                       uint8_t* d_found, void* d_ws, size_t ws_bytes, void* stream) {
    return enqueue_assign(table, n, d_keys, nullptr, d_scores, d_found, d_ws, ws_bytes, stream);
}

int cskv_find_or_insert(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_init_values,
                        const uint64_t* d_scores, float* d_values_out, uint8_t* d_status, void* d_ws, size_t ws_bytes,
                        void* stream) {
    if (n && (!d_init_values || !d_values_out)) return CSKV_EINVAL;
    UpsertArgs a{n, d_keys, d_init_values, d_scores, d_status, EvictOut{nullptr, nullptr, nullptr, nullptr}};
    a.out = d_values_out;
    RoleScope role(table, kInserter, as_stream(stream));
    if (!role.ok()) return CSKV_EHIP;
    return enqueue_upsert(table, a, d_ws, ws_bytes, as_stream(stream));
}

int cskv_set_tuning(cskv_table* table, int param, int value) {
    if (!table) return CSKV_EINVAL;
    switch (param) {
        case CSKV_TUNE_FIND_GROUP:
            if (value != 4 && value != 8 && value != 16) return CSKV_EINVAL;
            table->group = value;
            return CSKV_OK;
        case CSKV_TUNE_ROUTE_GROUP:
            if (value != 4 && value != 8 && value != 16) return CSKV_EINVAL;
            table->route_group = value;
            return CSKV_OK;
        case CSKV_TUNE_FIND_PREFETCH_B2:
            if (value != 0 && value != 1) return CSKV_EINVAL;
            table->prefetch_b2 = value;
            return CSKV_OK;
        case CSKV_TUNE_FIND_BLOCKS_PER_CU:
            if (value < 0 || value > 64) return CSKV_EINVAL;
            table->blocks_per_cu = value;
            return CSKV_OK;
        case CSKV_TUNE_FIND_PAIRS:
            if (value != 0 && value != 1) return CSKV_EINVAL;
            table->find_pairs = value;
            return CSKV_OK;
        case CSKV_TUNE_FIND_DIGEST:
            if (value != 0 && value != 1) return CSKV_EINVAL;
            table->find_digest = value;
            return CSKV_OK;
        default: return CSKV_EINVAL;
    }
}

int cskv_get_tuning(const cskv_table* table, int param) {
    if (!table) return -1;
    switch (param) {
        case CSKV_TUNE_FIND_GROUP: return table->group;
        case CSKV_TUNE_ROUTE_GROUP: return table->route_group;
        case CSKV_TUNE_FIND_PREFETCH_B2: return table->prefetch_b2;
        case CSKV_TUNE_FIND_BLOCKS_PER_CU: return table->blocks_per_cu;
        case CSKV_TUNE_FIND_PAIRS: return table->find_pairs;
        case CSKV_TUNE_FIND_DIGEST: return table->find_digest;
        default: return -1;
    }
}

int cskv_set_route_subrounds(cskv_table* table, uint32_t rounds) {
    if (!table || rounds < 1 || rounds > 64) return CSKV_EINVAL;
    table->subrounds = rounds;
    return CSKV_OK;
}

uint32_t cskv_get_route_subrounds(const cskv_table* table) { return table ? table->subrounds : 0; }

int cskv_set_lock_mode(cskv_table* table, int mode) {
    if (!table || (mode != CSKV_LOCK_NONE && mode != CSKV_LOCK_TRIPLE_GROUP && mode != CSKV_LOCK_READER_WRITER))
        return CSKV_EINVAL;
    return table->roles->set_mode(mode) ? CSKV_OK : CSKV_EINVAL;
}

int cskv_get_lock_mode(const cskv_table* table) { return table ? table->roles->mode() : -1; }

uint64_t cskv_clock(const cskv_table* table) {
    if (!table) return 0;
    uint64_t c = 0;
    if (hipDeviceSynchronize() != hipSuccess) return 0;
    if (hipMemcpy(&c, table->view.clock, 8, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    return c;
}

int cskv_set_clock(cskv_table* table, uint64_t clock) {
    if (!table) return CSKV_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return CSKV_EHIP;
    return hip_rc(hipMemcpy(table->view.clock, &clock, 8, hipMemcpyHostToDevice));
}

uint64_t cskv_num_buckets(const cskv_table* table) { return table ? table->view.nbuckets : 0; }
uint64_t cskv_hbm_value_rows(const cskv_table* table) { return table ? table->view.hbm_rows : 0; }

uint64_t cskv_row_address(const cskv_table* table, uint64_t slot) {
    if (!table || slot >= table->capacity) return 0;
    return (uint64_t)(uintptr_t)table->view.row(slot);
}
uint32_t cskv_dim(const cskv_table* table) { return table ? table->view.dim : 0; }
int cskv_mode(const cskv_table* table) { return table ? table->mode : -1; }
int cskv_policy(const cskv_table* table) { return table ? table->policy : -1; }

const char* cskv_strerror(int code) {
    switch (code) {
        case CSKV_OK: return "ok";
        case CSKV_EINVAL: return "invalid argument";
        case CSKV_ENOMEM: return "storage or workspace too small";
        case CSKV_EHIP: return "HIP error";
        case CSKV_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown error";
    }
}

}  // extern "C"
