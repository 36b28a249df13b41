// Internal declarations shared by the HIP kernels and the C-ABI host code of the cache-semantic
// hash table.  Layouts:
//
//   table storage (one caller buffer, each array 256-byte aligned, B = number of buckets):
//     dig    u8 [B][128]          digest line per bucket (0 = empty slot)
//     keys   u64[B][128]          key line(s) per bucket (0 = empty)
//     scores u64[B][128]          score line(s) per bucket
//     vals   f32[B][128][dim]     value rows, addressed by (bucket, slot)
//     cnt    u32[B]               inserts routed to a bucket by the running call (0 between calls)
//     cbase  u32[B]               start of a contended bucket's incoming list in the workspace
//     freeb  u8 [B]               free slots of a routed-to bucket when the call started
//
//   upsert workspace (n keys, P = power of two >= 2n, each array 256-byte aligned):
//     skeys u64[P], slast u32[P], sinc u64[P], ssat u32[P], sstat u8[P]   batch dedupe set
//     slot_of u32[n]                                                       set slot of key i
//     op_kind u8[n], op_tgt u32[n], op_aux u32[n], op_score u64[n]         routed operations
//     glist u32[n]                                                         contended ops by bucket
//     clist u32[min(n, B)]                                                 contended buckets
//     ctr u32[64]                                                          counters
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cskv {

constexpr int kSlots = 128;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

enum OpKind : uint8_t { kOpNone = 0, kOpUpdate = 1, kOpInsert = 2 };
enum Counter { kCtrContended = 0, kCtrListFill = 1 };

struct TableView {
    uint8_t* dig;
    uint64_t* keys;
    uint64_t* scores;
    float* vals;
    uint32_t* cnt;
    uint32_t* cbase;
    uint8_t* freeb;
    uint64_t nbuckets;
    uint32_t bmask;  // nbuckets - 1
    uint32_t dim;
    int dual;
    int policy;
};

struct UpsertWs {
    uint64_t* skeys;
    uint32_t* slast;
    uint64_t* sinc;
    uint32_t* ssat;
    uint8_t* sstat;
    uint32_t* slot_of;
    uint8_t* op_kind;
    uint32_t* op_tgt;
    uint32_t* op_aux;
    uint64_t* op_score;
    uint32_t* glist;
    uint32_t* clist;
    uint32_t* ctr;
    uint64_t P;
    int logP;
};

struct EvictOut {
    uint64_t* keys;
    float* vals;
    uint64_t* scores;
    uint64_t* count;
};

struct StorageLayout {
    size_t off_dig, off_keys, off_scores, off_vals, off_cnt, off_cbase, off_freeb, total;
};

struct UpsertLayout {
    size_t off_skeys, off_slast, off_sinc, off_ssat, off_sstat, off_slot_of, off_op_kind, off_op_tgt,
        off_op_aux, off_op_score, off_glist, off_clist, off_ctr, total;
    uint64_t P;
    int logP;
};

StorageLayout storage_layout(uint64_t nbuckets, uint32_t dim);
UpsertLayout upsert_layout(uint64_t n, uint64_t nbuckets);
size_t erase_ws_bytes(uint64_t n);

// launchers (return hipError_t of the last launch)
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_clear_table(const TableView& t, hipStream_t s);
hipError_t launch_find(const TableView& t, uint64_t n, const uint64_t* keys, float* out, uint8_t* found,
                       uint64_t* scores_out, int group, hipStream_t s);
hipError_t launch_upsert(const TableView& t, const UpsertWs& w, uint64_t n, const uint64_t* keys,
                         const float* vals, const uint64_t* scores, uint8_t* status, const EvictOut& ev,
                         uint64_t clock, int group, hipStream_t s);
hipError_t launch_erase(const TableView& t, uint64_t n, const uint64_t* keys, uint8_t* erased,
                        uint32_t* ws_slot, int group, hipStream_t s);
hipError_t launch_size(const TableView& t, uint64_t* d_size, hipStream_t s);
hipError_t launch_export(const TableView& t, uint64_t b0, uint64_t b1, uint64_t* keys, float* vals,
                         uint64_t* scores, uint64_t* slots, uint64_t* count, hipStream_t s);

}  // namespace cskv
