// Internal declarations shared by the HIP kernels and the C-ABI host code of the cache-semantic
// hash table.  Layouts:
//
//   table storage (one caller buffer, each array 256-byte aligned, B = number of buckets):
//     dig    u8 [B][128]          digest line per bucket (0 = empty slot)
//     keys   u64[B][128]          key line(s) per bucket (0 = empty)
//     scores u64[B][128]          score line(s) per bucket
//     vals   f32[B][128][dim]     value rows, addressed by (bucket, slot)
//     cnt    u64[B]               operations routed to a bucket by the running call: inserts in the
//                                  low 32 bits, updates in the high 32 bits (0 between calls)
//     bmin   u64[B][2]            (score, key) of a full bucket's minimum entry; key 0 = not known
//     clock  u64                  LRU logical clock (device-resident so captured graphs advance it)
//
//   upsert workspace (n keys, P = power of two >= 2n, C = per-bucket inline capacity):
//     zeroed on entry: dd {key u64, last u32, claim u32}[P], okey u64[P], ctr u32[64],
//                      and for LFU inc u64[P], sat u32[P], minc u64[P]
//     sstat u8[P]                      status of each distinct key's operation
//     slot_of u32[n]                   dedupe slot of input i, or (block-local dedupe) the position of
//                                      its block representative (kNoSlot: reserved key)
//     rinc u64[n]                      block-local dedupe, LFU: representatives' increment sums
//     il OpEntry[B*C]                  per-bucket operation lists: key, new score,
//                                      (dedupe slot << 32 | input position), and a meta word (slot,
//                                      digest, kind, free slots of the bucket before the call)
//     ol OpEntry[P]                    list positions >= C, hashed on (bucket, position) via okey
//     slow u32[min(n, B)]              buckets with more operations than the fast path takes
//     touched u32[min(n, B)]           buckets that received an operation (small batches only)
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cskv_roles.h"

namespace cskv {

constexpr int kSlots = 128;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
// kinds of a routed operation: an update of a resident slot; an insert that routing already
// wrote into one of the bucket's free slots (its digest byte is written by the apply pass); an
// insert that found no free slot left and waits in the bucket's list for the apply pass
enum OpKind : uint8_t { kOpUpdate = 0, kOpDirect = 1, kOpListed = 2 };
constexpr int kFastMax = 16;  // operations per bucket handled by the 16-lane fast path

// kCtrDup: the call repeats a key; kCtrDistinct: its number of distinct keys (sub-rounds only)
enum Counter { kCtrSlow = 0, kCtrTouched = 1, kCtrDup = 2, kCtrDistinct = 3 };

struct TableView {
    uint8_t* dig;
    uint64_t* keys;
    uint64_t* scores;
    float* vals;       // value rows [0, hbm_rows), in HBM
    float* vals_host;  // value rows [hbm_rows, nbuckets * 128), pinned host memory (device address)
    uint64_t* cnt;
    uint64_t* bmin;
    uint64_t* clock;
    uint64_t nbuckets;
    uint64_t hbm_rows;  // nbuckets * 128 unless the table has a host value tier
    uint32_t bmask;  // nbuckets - 1
    uint32_t dim;
    int dual;
    int policy;

    // the value row of slot e (= bucket * 128 + slot): position-based, no per-entry pointer
    __host__ __device__ __forceinline__ float* row(size_t e) const {
        return e < hbm_rows ? vals + e * dim : vals_host + (e - hbm_rows) * dim;
    }
};

struct DedupeEntry {
    uint64_t key;
    uint32_t last;   // largest index + 1 among the occurrences that found the key already claimed
    uint32_t claim;  // index + 1 of the occurrence that claimed the entry
};

struct OpEntry {
    uint64_t key;
    uint64_t score;
    uint64_t w;     // dedupe slot << 32 | input position
    uint64_t meta;  // bits 0-7: table slot (update: the resident slot; direct insert: the free slot it
                    // took); 8-15: the key's digest; 16-23: OpKind; 24-31: free slots of the target
                    // bucket before the call (inserts)
};

struct UpsertWs {
    DedupeEntry* dd;
    uint64_t* okey;
    uint32_t* ctr;
    uint64_t* inc;
    uint32_t* sat;
    uint8_t* sstat;
    uint32_t* slot_of;
    OpEntry* il;
    OpEntry* ol;
    uint32_t* slow;
    uint32_t* touched;
    uint32_t* rank;  // sub-rounds: rank of each last occurrence among them, in input order
    uint32_t* bsum;  // sub-rounds: per-block counts of last occurrences, then their offsets
    uint64_t P;
    int logP;
    uint32_t cap;    // inline operations per bucket
    int list_mode;   // apply visits only the touched buckets (small batches)
    float* out;      // find_or_insert: rows returned per occurrence (resident rows are kept); else null
    int rounds;      // route sub-rounds of the call (1: the whole batch routes at once)
    int round;       // the sub-round a route / apply launch serves
    int local = 0;   // block-local dedupe: slot_of[i] is the position of the occurrence that represents
                     // key i in its block of the input (its last occurrence there), statuses are kept per
                     // representative position, and a key repeated across blocks has one list entry
                     // per block, merged by the apply pass
    uint64_t* rinc;  // local dedupe, LFU: a representative's block sum of increments (saturated = ~0)
    uint64_t* minc;  // LFU: per dedupe-set slot, the sum of the merged entries' increments (slow apply)
};

// one batch of a merged run of finds (reader group): keys [begin, begin + n) of the run
struct FindDesc {
    const uint64_t* keys;
    float* out;
    uint8_t* found;
    uint64_t* scores;
    uint64_t begin;
    uint64_t n;
};

// a small merged run passed by value as kernel arguments (no descriptor upload)
constexpr int kMaxArgDescs = 64;
struct FindDescArgs {
    FindDesc d[kMaxArgDescs];
    uint32_t nd;
    uint64_t total;
};

struct EvictOut {
    uint64_t* keys;
    float* vals;
    uint64_t* scores;
    uint64_t* count;
};

struct StorageLayout {
    size_t off_dig, off_keys, off_scores, off_vals, off_cnt, off_bmin, off_clock, total;
};

struct UpsertLayout {
    size_t off_dd, off_okey, off_ctr, off_inc, off_sat, off_minc, off_zero_end, off_zero_end_lfu;
    size_t off_sstat, off_slot_of, off_rinc, off_il, off_ol, off_slow, off_touched, off_rank, off_bsum, total;
    uint64_t P;
    int logP;
    uint32_t cap;
    int list_mode;
};

StorageLayout storage_layout(uint64_t nbuckets, uint32_t dim, uint64_t hbm_rows);
// compact: no per-bucket inline lists (every list position in the hashed overflow table) and the
// apply visits only the touched buckets, so that the size depends on n alone
UpsertLayout upsert_layout(uint64_t n, uint64_t nbuckets, uint32_t rounds = 1, bool compact = false);
size_t erase_ws_bytes(uint64_t n);

// launchers (return hipError_t of the last launch)
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_clear_table(const TableView& t, hipStream_t s);
hipError_t launch_find_nodigest(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                                uint64_t* scores_out, int group, hipStream_t s);
hipError_t launch_find(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                       uint64_t* scores_out, int group, int prefetch_b2, int pairs, hipStream_t s);
hipError_t launch_find_multi(const TableView& t, const FindDesc* d, uint32_t nd, uint64_t total, int group,
                             int prefetch_b2, unsigned blocks, hipStream_t s);
hipError_t launch_find_args(const TableView& t, const FindDescArgs& a, int group, int prefetch_b2, hipStream_t s);
hipError_t launch_upsert(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                         const float* vals, const uint64_t* scores, uint8_t* status, const EvictOut& ev,
                         size_t zero_bytes, int group, hipStream_t s);
hipError_t launch_erase(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased,
                        uint32_t* ws_slot, int group, hipStream_t s);
// the phases of an upsert / erase, for callers that order them with events (batched programs):
// prep (scratch clear, dedupe) reads the table; route reads it and writes only slots that are free
// (zero digest) before the call, which no reader looks at; apply writes it; finish writes the
// statuses; an erase probe reads, its clear writes
hipError_t launch_upsert_prep(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                              const uint64_t* scores, const EvictOut& ev, size_t zero_bytes, hipStream_t s);
hipError_t launch_upsert_route(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                               const float* vals, const uint64_t* scores, int group, hipStream_t s);
hipError_t launch_upsert_apply(const TableView& t, const UpsertWs& w, uint64_t n, const float* vals,
                               const EvictOut& ev, hipStream_t s);
hipError_t launch_upsert_finish(const UpsertWs& w, uint64_t n, uint8_t* status, uint32_t dim, hipStream_t s);
// route + apply of every sub-round (w.rounds > 1), after launch_upsert_prep
hipError_t launch_upsert_rounds(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                                const float* vals, const uint64_t* scores, const EvictOut& ev, int group, hipStream_t s);
hipError_t launch_erase_probe(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased,
                              uint32_t* ws_slot, int group, hipStream_t s);
hipError_t launch_erase_clear(const TableView& t, uint64_t n, uint32_t* ws_slot, hipStream_t s);
hipError_t launch_size(const TableView& t, uint64_t* d_size, hipStream_t s);
hipError_t launch_export(const TableView& t, uint64_t b0, uint64_t b1, uint64_t* keys, float* vals,
                         uint64_t* scores, uint64_t* slots, uint64_t* count, uint64_t min_score, hipStream_t s);
// contains (ptrs null) / find_ptr; assign / assign_scores (vals null) after the dedupe pass
hipError_t launch_locate(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* found, uint64_t* ptrs,
                         uint64_t* scores, int group, hipStream_t s);
hipError_t launch_assign(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys, const float* vals,
                         const uint64_t* scores, uint8_t* found, int group, hipStream_t s);

// enqueue helpers shared by the single-call C ABI and the batched program (return CSKV_* codes)
struct UpsertArgs {
    uint64_t n;
    const uint64_t* keys;
    const float* vals;
    const uint64_t* scores;
    uint8_t* status;
    EvictOut ev;
    float* out = nullptr;  // find_or_insert: returned rows (resident rows are kept, not replaced)
};

}  // namespace cskv

// the C ABI's opaque table object
namespace cskv {
// the role lock's backend: HIP events ordering streams
struct HipEvents {
    using Event = hipEvent_t;
    using Stream = hipStream_t;
    Event make() {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    bool record(Event e, Stream s) { return e && hipEventRecord(e, s) == hipSuccess; }
    bool wait(Stream s, Event e) { return hipStreamWaitEvent(s, e, 0) == hipSuccess; }
    bool done(Event e) { return hipEventQuery(e) == hipSuccess; }
    void destroy(Event e) {
        if (e) (void)hipEventDestroy(e);
    }
};
using TableLock = RoleLock<HipEvents>;
}  // namespace cskv

struct cskv_table {
    cskv::TableView view;
    uint64_t capacity;
    int mode;
    int policy;
    int group;          // lanes per key of the find / erase probe kernels
    int route_group;    // lanes per key of the upsert route kernel
    int prefetch_b2;    // find loads both candidate digest lines at once
    int blocks_per_cu;  // persistent grid of merged find runs: blocks per compute unit (0 = one group per key)
    int find_pairs;     // find: two keys per lane group
    int find_digest;    // find: 1 = digest-filtered probes, 0 = the no-digest ablation
    uint32_t subrounds; // route sub-rounds per upsert call (a semantic setting, 1 by default)
    int num_cus;
    int device;  // HIP device the table lives on
    cskv::TableLock* roles = nullptr;  // role lock across host threads and streams (off in lock mode none)
    ~cskv_table() { delete roles; }
};

namespace cskv {
// holds a table's role for one call when its lock is on: the stream waits for the group before
// on entry; the call's event is recorded on exit
class RoleScope {
  public:
    RoleScope(cskv_table* t, int role, hipStream_t s) : t_(t), s_(s) {
        on_ = t && t->roles && t->roles->mode() != kLockNone;
        if (on_) tk_ = t->roles->acquire(role, s);
    }
    ~RoleScope() {
        if (on_) t_->roles->release(tk_, s_);
    }
    bool ok() const { return !on_ || tk_.ok; }
    RoleScope(const RoleScope&) = delete;
    RoleScope& operator=(const RoleScope&) = delete;

  private:
    cskv_table* t_;
    hipStream_t s_;
    bool on_ = false;
    TableLock::Ticket tk_;
};
}  // namespace cskv

namespace cskv {
// validates an upsert and lays out its workspace (CSKV_* code)
int plan_upsert(cskv_table* t, const UpsertArgs& a, void* ws, size_t ws_bytes, UpsertWs* w, size_t* zero_bytes,
                bool need_vals = true, bool compact = false);
// group: lanes per key of the routing (upsert) or probe (erase) kernel; -1 = the table's setting
// compact: the workspace layout sized by n alone (upsert_layout)
int enqueue_upsert(cskv_table* t, const UpsertArgs& a, void* ws, size_t ws_bytes, hipStream_t s, int group = -1,
                   bool compact = false);
int enqueue_erase(cskv_table* t, uint64_t n, const uint64_t* keys, uint8_t* erased, void* ws, size_t ws_bytes,
                  hipStream_t s, int group = -1);
}  // namespace cskv
