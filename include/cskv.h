/*
 * cskv.h - C interface of an MI355X-native cache-semantic GPU hash table.
 *
 * The table follows arxiv 2603.17168 ("HierarchicalKV"): u64 keys with u64 scores in
 * buckets of 128 slots (Sec. 3.2), each bucket stored as a 128-byte digest line plus key and
 * score lines; value rows of `dim` fp32 stored apart from the keys and addressed by
 * (bucket, slot) (Sec. 3.6, position-based addressing).  A full bucket is resolved in place by
 * evicting its lowest-score entry or by refusing admission (Sec. 3.3, Alg. 2); each key has two
 * candidate buckets chosen by load, then by score (Sec. 3.4, Alg. 3).  The API mirrors the
 * paper's batched STL-style interface (Sec. 4.1): every call processes a batch of keys with a
 * sequence of kernels enqueued on the caller's stream.
 *
 * Conventions that hold for every call:
 *  - Pointers named d_* are device pointers owned by the caller.  The library never allocates,
 *    frees or keeps them after the call returns.  Table storage and workspaces are caller
 *    memory too (e.g. a torch uint8 tensor).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are asynchronous and ordered
 *    on that stream; outputs are valid once the stream has reached the end of the call.  One
 *    table must be used from one stream at a time (or with the caller ordering the streams).
 *  - Argument errors are returned synchronously and nothing is enqueued.  A failed kernel
 *    launch returns CSKV_EHIP.  Problems with single keys (reserved words) are reported as
 *    per-key statuses, not as call errors.
 *  - n = 0 is a valid no-op (no clock tick, no kernel).
 *  - Reserved key words: 0 marks an empty slot and 2^64-1 a locked slot; neither is a valid
 *    user key (status CSKV_ST_INVALID_KEY; find reports not found; erase reports not erased).
 *  - Value rows are float32[dim]; dim must be a multiple of 4 in [4, 1024].  d_values pointers
 *    must be 16-byte aligned; key, score and count pointers 8-byte aligned.
 *  - Output buffers must not alias table storage or one another.
 *
 * Batch semantics of an upsert call (insert_or_assign / insert_and_evict):
 *  1. Scores: CUSTOM takes d_scores[i]; LRU gives every key of the call the table clock,
 *     which advances by one per call; LFU adds d_scores[i] (1 if d_scores is NULL) per
 *     occurrence, saturating at 2^64-1, to the key's score (0 for a new key).
 *  2. Duplicate keys collapse to one operation; the last occurrence provides the value row
 *     (and the CUSTOM score); every occurrence gets that operation's status.
 *  3. Routing reads the table as it was before the call: a key present in one of its
 *     candidates is updated in place; otherwise single mode (or equal candidates) targets b1,
 *     dual mode targets the less occupied candidate while either has a free slot (b1 on a
 *     tie, phase D1) and else the candidate whose minimum (score, key) entry is smaller
 *     (phase D2).
 *  4. Per bucket, updates first; then inserts in (score descending, key ascending) order:
 *     a free slot takes the key; else the minimum (score, key) entry is evicted if the new
 *     score is strictly greater than its score, otherwise the key is rejected.
 * The result (statuses, evicted set, table contents per bucket) is deterministic and equals
 * the sequential CPU definition; slot positions inside a bucket and the order of evicted
 * entries in the output are not part of the result.
 */
#ifndef CSKV_H
#define CSKV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cskv_table cskv_table;

/* return codes */
enum {
    CSKV_OK = 0,
    CSKV_EINVAL = -1,      /* bad argument (null, misaligned, out of range) */
    CSKV_ENOMEM = -2,      /* storage or workspace smaller than required */
    CSKV_EHIP = -3,        /* a HIP call or kernel launch failed */
    CSKV_EUNSUPPORTED = -4 /* valid but unsupported configuration */
};

/* table modes (Sec. 3.2 single-bucket confinement; Sec. 3.4 dual-bucket selection) */
enum { CSKV_MODE_SINGLE = 1, CSKV_MODE_DUAL = 2 };

/* score policies (Sec. 3.3 "scoring policies") */
enum { CSKV_SCORE_CUSTOM = 0, CSKV_SCORE_LRU = 1, CSKV_SCORE_LFU = 2 };

/* per-key statuses of upserts (Alg. 2 outcomes) */
enum {
    CSKV_ST_UPDATED = 1,
    CSKV_ST_INSERTED = 2,
    CSKV_ST_INSERTED_EVICT = 3,
    CSKV_ST_REJECTED = 4,
    CSKV_ST_INVALID_KEY = 5
};

/* operation ids for cskv_workspace_bytes */
enum { CSKV_OP_FIND = 0, CSKV_OP_INSERT_OR_ASSIGN = 1, CSKV_OP_INSERT_AND_EVICT = 2, CSKV_OP_ERASE = 3,
       CSKV_OP_ASSIGN = 4, CSKV_OP_FIND_OR_INSERT = 5 };

/*
 * Bytes of device storage a table needs (Sec. 3.2 bucket layout, Sec. 3.6 value store):
 * per bucket a 128-B digest line, 128 keys, 128 scores, 128 value rows, plus 20 B of per-bucket
 * bookkeeping (an operation counter and the cached minimum entry of a full bucket).
 * capacity must be 128 * B with B a power of two, 1 <= B <= 2^24; bucket_size must be 128.
 * Returns 0 if the arguments are invalid.
 */
size_t cskv_table_bytes(uint64_t capacity, uint32_t bucket_size, uint32_t dim);

/*
 * Creates a table over caller storage d_storage (>= cskv_table_bytes, 256-byte aligned) and
 * enqueues on `stream` the kernel that empties it.  The host object *out is freed by
 * cskv_destroy; the storage stays the caller's.  mode: CSKV_MODE_*; score_policy: CSKV_SCORE_*.
 * Errors: CSKV_EINVAL (null out/storage, bad mode/policy/dim, misaligned storage),
 * CSKV_EUNSUPPORTED (bucket_size != 128), CSKV_ENOMEM (storage too small), CSKV_EHIP.
 */
int cskv_create(cskv_table** out, uint64_t capacity, uint32_t bucket_size, uint32_t dim, int mode,
                int score_policy, void* d_storage, size_t storage_bytes, void* stream);

/*
 * Tiered value storage (Sec. 3.6 key-value separation, Sec. 4.2 HBM watermark): digests, keys,
 * scores and the first hbm_value_rows value rows live in HBM; the remaining
 * capacity - hbm_value_rows rows live in pinned host memory that kernels read and write through
 * its device alias (no CPU thread on the data path).  A value row's address follows from its
 * position: slot e = bucket * 128 + slot holds its row in HBM at e * dim * 4 if e <
 * hbm_value_rows, else in host memory at (e - hbm_value_rows) * dim * 4.
 *   cskv_table_bytes_tiered: device bytes for the table with hbm_value_rows rows in HBM
 *                            (0 on bad arguments or hbm_value_rows > capacity);
 *   cskv_host_value_bytes:   host bytes for the rest;
 *   cskv_create_tiered:      cskv_create with h_values = host memory from hipHostMalloc (or any
 *                            pinned allocation hipHostGetDevicePointer accepts), 16-byte aligned,
 *                            host_bytes >= cskv_host_value_bytes; h_values is ignored when
 *                            hbm_value_rows == capacity.  The host memory stays the caller's and
 *                            must outlive the table.  CSKV_EINVAL if it is not pinned.
 * Every call works unchanged on a tiered table; find_ptr and cskv_row_address may return
 * device aliases of host memory.  cskv_create is cskv_create_tiered with hbm_value_rows =
 * capacity.
 */
size_t cskv_table_bytes_tiered(uint64_t capacity, uint32_t bucket_size, uint32_t dim, uint64_t hbm_value_rows);
size_t cskv_host_value_bytes(uint64_t capacity, uint32_t dim, uint64_t hbm_value_rows);
int cskv_create_tiered(cskv_table** out, uint64_t capacity, uint32_t bucket_size, uint32_t dim, int mode,
                       int score_policy, void* d_storage, size_t storage_bytes, uint64_t hbm_value_rows,
                       void* h_values, size_t host_bytes, void* stream);
uint64_t cskv_hbm_value_rows(const cskv_table* table);
/* device address of the value row of slot e (= bucket * 128 + slot); 0 if e >= capacity */
uint64_t cskv_row_address(const cskv_table* table, uint64_t slot);

/* Frees the host object (never the storage).  NULL is accepted. */
int cskv_destroy(cskv_table* table);

/* Empties the table (all slots free) on `stream`; the LRU clock is kept. */
int cskv_clear(cskv_table* table, void* stream);

/*
 * Bytes of device workspace an operation on n keys needs (CSKV_OP_*); 0 for find.  The
 * workspace is scratch for one call: its contents on entry are ignored.  Must be 256-byte
 * aligned.  Returns 0 for an unknown op.
 */
size_t cskv_workspace_bytes(const cskv_table* table, int op, uint64_t n);

/*
 * find (Alg. 1, digest-accelerated lookup; dual mode probes b2 after a miss in b1).
 * d_keys[n] in; d_values_out[n*dim] gets the row of every found key, rows of missing keys are
 * left untouched; d_found[n] (u8) gets 1/0; d_scores_out[n] (nullable) gets the score of every
 * found key.  No table state changes.
 */
int cskv_find(cskv_table* table, uint64_t n, const uint64_t* d_keys, float* d_values_out,
              uint8_t* d_found, uint64_t* d_scores_out, void* stream);

/*
 * insert_or_assign (Alg. 2 with Alg. 3's bucket choice; batch semantics above).
 * d_keys[n], d_values[n*dim] in.  d_scores[n]: CUSTOM - required, the scores; LRU - ignored
 * (may be NULL); LFU - increments, NULL means 1 each.  d_status[n] (nullable) gets CSKV_ST_*.
 * d_ws: workspace of cskv_workspace_bytes(table, CSKV_OP_INSERT_OR_ASSIGN, n) bytes.
 */
int cskv_insert_or_assign(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                          const uint64_t* d_scores, uint8_t* d_status, void* d_ws, size_t ws_bytes,
                          void* stream);

/*
 * insert_or_assign that allocates nothing, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same inputs,
 * outputs, semantics and kernels as cskv_insert_or_assign; the workspace is instead a fixed
 * device array of the library, CSKV_NOALLOC_SCRATCH_BYTES (12 MiB) per GPU, allocated when the
 * library's code loads on that GPU and held until the process ends.  The call makes no
 * hipMalloc / hipFree and calls no allocating routine.  n is at most CSKV_NOALLOC_MAX_KEYS
 * (65536): a larger n returns CSKV_EINVAL and launches nothing (CSKV_ENOMEM if the workspace
 * would not fit, which this limit rules out).  The array keeps the last call's contents; every
 * call clears what must start at zero, with a fill kernel on its stream.  All calls on one GPU
 * share the array, whatever the table or stream: calls that overlap in time on one GPU (other
 * streams, other host threads) race and give undefined results; order them on one stream or
 * with events.  The first call on a GPU looks up the array's address there (hipGetSymbolAddress,
 * with that GPU current) and keeps it; a failure returns CSKV_EHIP.
 */
#define CSKV_NOALLOC_MAX_KEYS 65536u
#define CSKV_NOALLOC_SCRATCH_BYTES (12u << 20)
int cskv_insert_or_assign_noalloc(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                                  const uint64_t* d_scores, uint8_t* d_status, void* stream);
/* bytes of the fixed array above (CSKV_NOALLOC_SCRATCH_BYTES) */
size_t cskv_noalloc_scratch_bytes(void);

/*
 * insert_and_evict (Sec. 4.1: insert_or_assign that also returns what it evicted).
 * Same inputs as insert_or_assign; d_status is required.  Every entry displaced by the call
 * is written to d_ev_keys[j], d_ev_scores[j] (the score it had, after any update in the same
 * call) and d_ev_values[j*dim..] for j < *d_n_evicted (a device u64 written by the call; at
 * most n).  Output order is unspecified.  Rejected incoming keys are not in the evicted list.
 */
int cskv_insert_and_evict(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values,
                          const uint64_t* d_scores, uint8_t* d_status, uint64_t* d_ev_keys,
                          float* d_ev_values, uint64_t* d_ev_scores, uint64_t* d_n_evicted, void* d_ws,
                          size_t ws_bytes, void* stream);

/*
 * erase (inserter-group call of Sec. 3.5): removes every present key.  d_erased[n] (nullable)
 * gets 1 if key i was present before the call (duplicates all report 1), else 0.
 * d_ws: cskv_workspace_bytes(table, CSKV_OP_ERASE, n) bytes.
 */
int cskv_erase(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint8_t* d_erased, void* d_ws,
               size_t ws_bytes, void* stream);

/* size (reader-group call of Sec. 3.5): number of occupied slots, written to device u64 *d_size. */
int cskv_size(cskv_table* table, uint64_t* d_size, void* stream);

/*
 * export (Sec. 4.1's export for checkpointing, without a predicate): every entry of buckets
 * [bucket_begin, bucket_end) is written to d_keys[j], d_scores[j], d_values[j*dim..] and, if
 * d_slots is not NULL, its slot index bucket*128+slot to d_slots[j], for j < *d_count (device
 * u64).  Output capacity must be (bucket_end - bucket_begin) * 128.  Order unspecified.
 * d_values and d_scores may be NULL.
 */
int cskv_export(cskv_table* table, uint64_t bucket_begin, uint64_t bucket_end, uint64_t* d_keys,
                float* d_values, uint64_t* d_scores, uint64_t* d_slots, uint64_t* d_count, void* stream);

/*
 * export_if (Sec. 4.1's export_batch_if, streaming entries that match a predicate for
 * checkpointing): as cskv_export, restricted to entries whose score is at least min_score
 * (min_score 0 = every entry).  Same buffers, capacity and errors as cskv_export.
 */
int cskv_export_if(cskv_table* table, uint64_t bucket_begin, uint64_t bucket_end, uint64_t min_score,
                   uint64_t* d_keys, float* d_values, uint64_t* d_scores, uint64_t* d_slots, uint64_t* d_count,
                   void* stream);

/*
 * contains (reader-group call of Sec. 3.5): d_found[i] (u8) = 1 when d_keys[i] is resident,
 * else 0 (reserved keys: 0).  No state change; no workspace.  CSKV_EINVAL for n >= 2^31, NULL
 * or misaligned (8-byte keys) buffers.
 */
int cskv_contains(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint8_t* d_found, void* stream);

/*
 * find_ptr (the position-returning find* of Sec. 5, a reader): d_ptrs[i] (u64) = the device
 * address of key i's value row inside the table storage (dim floats), 0 when absent; d_found[i]
 * as contains; d_scores_out[i] (nullable) = its score.  The addresses stay valid until the next
 * call that changes table structure (an insert, an eviction, erase, clear).  Errors as contains.
 */
int cskv_find_ptr(cskv_table* table, uint64_t n, const uint64_t* d_keys, uint64_t* d_ptrs, uint8_t* d_found,
                  uint64_t* d_scores_out, void* stream);

/*
 * assign / assign_scores (updater-group calls of Sec. 3.5: values or scores of existing
 * entries, never bucket structure).  One batch: duplicates collapse to the last occurrence (its
 * row and CUSTOM score), LFU increments (d_scores, or 1 each when NULL) are summed; a resident
 * key's score is set as an UPDATE of insert_or_assign sets it (CUSTOM: the score; LRU: this
 * call's clock, which advances by one per non-empty call; LFU: old + sum, saturating) and
 * assign also replaces its row with d_values (n x dim fp32); absent keys change nothing.
 * d_found (nullable) = residency per occurrence.  d_ws: cskv_workspace_bytes(table,
 * CSKV_OP_ASSIGN, n) bytes.  CSKV_EINVAL as insert_or_assign (d_scores required for CUSTOM).
 */
int cskv_assign(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_values, const uint64_t* d_scores,
                uint8_t* d_found, void* d_ws, size_t ws_bytes, void* stream);
int cskv_assign_scores(cskv_table* table, uint64_t n, const uint64_t* d_keys, const uint64_t* d_scores,
                       uint8_t* d_found, void* d_ws, size_t ws_bytes, void* stream);

/*
 * find_or_insert (inserter-group call of Sec. 3.5; Sec. 4.1's lookup with insertion for cold
 * starts): insert_or_assign in which a resident key keeps its row (its score is updated as an
 * UPDATE), absent keys are inserted with d_init_values under the same routing, admission and
 * eviction rules (evicted entries are dropped).  d_values_out (n x dim fp32) receives, for every
 * occurrence, the key's row from before the call if it was resident, else its last occurrence's
 * init row (inserted or rejected alike; rows of reserved keys are left untouched).  d_status
 * (nullable) as insert_or_assign.  d_ws: cskv_workspace_bytes(table, CSKV_OP_FIND_OR_INSERT, n)
 * bytes.  Output rows must not alias the inputs.  Errors as insert_or_assign.
 */
int cskv_find_or_insert(cskv_table* table, uint64_t n, const uint64_t* d_keys, const float* d_init_values,
                        const uint64_t* d_scores, float* d_values_out, uint8_t* d_status, void* d_ws, size_t ws_bytes,
                        void* stream);

/*
 * Launch-shape tuning (results never depend on it; the autotuner sets these):
 *  CSKV_TUNE_FIND_GROUP        lanes per key of the find and erase probes: 4, 8 (default) or 16
 *  CSKV_TUNE_ROUTE_GROUP       lanes per key of the upsert routing kernel: 4, 8 (default) or 16
 *  CSKV_TUNE_FIND_PREFETCH_B2  1 = find loads both candidates' digest lines at once, 0 = b2 only
 *                              after a miss in b1 (default)
 *  CSKV_TUNE_FIND_BLOCKS_PER_CU  grid of a program's merged find run: 0 (default) = one lane group
 *                              per key; k in 1..64 = a persistent grid of k 256-thread blocks per
 *                              compute unit striding over the run's keys
 *  CSKV_TUNE_FIND_PAIRS        1 = cskv_find serves two keys per lane group with their loads
 *                              interleaved, 0 = one key per group (default)
 *  CSKV_TUNE_FIND_DIGEST       1 = cskv_find filters candidate slots by the digest line (Alg. 1,
 *                              default); 0 = the digest ablation of Exp. 3a: every probe compares
 *                              the key with all 128 stored keys of the bucket (1 KiB instead of
 *                              the 128-byte digest line).  Programs and the server always filter.
 * cskv_set_tuning returns CSKV_EINVAL for an unknown parameter or value; cskv_get_tuning returns
 * the current value, or -1.
 */
enum {
    CSKV_TUNE_FIND_GROUP = 1,
    CSKV_TUNE_ROUTE_GROUP = 2,
    CSKV_TUNE_FIND_PREFETCH_B2 = 3,
    CSKV_TUNE_FIND_BLOCKS_PER_CU = 4,
    CSKV_TUNE_FIND_PAIRS = 5,
    CSKV_TUNE_FIND_DIGEST = 6
};
int cskv_set_tuning(cskv_table* table, int param, int value);
int cskv_get_tuning(const cskv_table* table, int param);

/*
 * Route sub-rounds (a semantic setting of the upsert calls: insert_or_assign, insert_and_evict,
 * find_or_insert; default 1).  Within one call every key routes against the table as it was
 * before the call (Alg. 3's occupancy and minimum tests see no key of the same call), which
 * leaves large batches less evenly spread than the paper's one-key-at-a-time picture.  With r
 * sub-rounds a call's distinct keys, ordered by the index of their last occurrence, are cut into
 * r chunks (rank q of N goes to chunk floor(q * r / N)); chunk after chunk is routed and applied
 * against the table the chunks before it left.  Statuses, scores (one LRU clock per call),
 * dedupe and LFU sums stay per call.  r = 1..64, else CSKV_EINVAL.  The workspace an upsert needs
 * grows with r > 1 (query cskv_workspace_bytes after setting it); a program built before a change
 * refuses to launch (CSKV_EINVAL) until it is rebuilt.
 */
int cskv_set_route_subrounds(cskv_table* table, uint32_t rounds);
uint32_t cskv_get_route_subrounds(const cskv_table* table);

/*
 * Concurrent calls from several host threads and streams (Sec. 3.5, the three operation groups
 * and their compatibility table; Sec. 4.4, the host/device lock).  Roles: readers = find,
 * contains, find_ptr, size, export, export_if and programs without writes; updaters = assign,
 * assign_scores; inserters = insert_or_assign, insert_and_evict, find_or_insert, erase, clear,
 * programs with writes and cskv_serve_trace (one call for the whole trace).
 *
 *   CSKV_LOCK_NONE           (default) no ordering across streams: the caller orders its calls
 *   CSKV_LOCK_TRIPLE_GROUP   readers run together, updaters run together, an inserter runs alone
 *   CSKV_LOCK_READER_WRITER  readers run together, every updater and inserter runs alone (the
 *                            conventional lock the paper's Exp. 3e compares against)
 *
 * With a lock on, calls are admitted in the order they enter the library (host order across
 * threads).  A call whose role cannot join the running group starts a new group: its stream is
 * made to wait (hipStreamWaitEvent) for events recorded after every call of the group before,
 * so calls of different groups execute in admission order on the GPU while calls of one group
 * may overlap.  No call waits on the host for GPU work; a thread blocks only while another
 * thread is still enqueueing a call of the group being closed.  Each call records one event on
 * its stream.  Concurrent updaters that touch the same key race (last writer unspecified, LFU
 * increments may be lost); callers give concurrent updaters disjoint keys.  Workspaces must not
 * be shared by calls that may overlap.  cskv_program_capture takes no role (the replay does).
 * The lock keeps the latest events of the streams it has seen and may query or wait on them in
 * later calls; cskv_set_lock_mode (even to the current mode) forgets all of them.  So: call it only while no call is in flight on the table (CSKV_EINVAL otherwise), and
 * call it after synchronizing, and before destroying, any stream that made calls under a lock.
 * CSKV_EINVAL for another mode.
 */
enum { CSKV_LOCK_NONE = 0, CSKV_LOCK_TRIPLE_GROUP = 1, CSKV_LOCK_READER_WRITER = 2 };
int cskv_set_lock_mode(cskv_table* table, int mode);
int cskv_get_lock_mode(const cskv_table* table);

/*
 * LRU logical clock: the number of non-empty upsert calls of an LRU table so far (plus any value
 * set here).  It lives in table storage so that captured programs advance it on every replay.
 * Both calls synchronize the device before reading or writing it.
 */
uint64_t cskv_clock(const cskv_table* table);
int cskv_set_clock(cskv_table* table, uint64_t clock);

/*
 * Batched programs: many uneven find / insert_or_assign / insert_and_evict / erase batches on one
 * table, enqueued by one call and optionally captured once as a hipGraph and replayed.
 * Semantics are exactly those of issuing the same calls one by one, in order, on one stream:
 *  - consecutive finds form a reader run (readers never conflict, Sec. 3.5 triple-group matrix)
 *    and execute as ONE merged kernel over all their keys (a persistent grid when
 *    CSKV_TUNE_FIND_BLOCKS_PER_CU > 0), with the table's tuning at the time the run's first
 *    find was added; a find whose buffers overlap an output of a find already in the run
 *    starts a new run;
 *  - every upsert or erase is a serialization point (inserter group) run as its usual kernels,
 *    in the launch shapes (route and probe lanes) the table had when it was added.
 * All pointers are recorded at add time and must stay valid (and unchanged in size) while the
 * program is launched or replayed.  The program needs a device workspace of
 * cskv_program_workspace_bytes bytes (256-byte aligned), given once with
 * cskv_program_set_workspace, which also uploads the merged runs' descriptors (synchronously).
 * cskv_program_capture records the program on `stream` (which must not be the NULL stream) into
 * a graph and instantiates it; cskv_program_replay launches that graph.  Launch, capture and
 * replay return CSKV_EINVAL before set_workspace; add after set_workspace returns CSKV_EINVAL.
 */
typedef struct cskv_program cskv_program;
int cskv_program_create(cskv_program** out, cskv_table* table);
int cskv_program_destroy(cskv_program* prog);
int cskv_program_add_find(cskv_program* prog, uint64_t n, const uint64_t* d_keys, float* d_values_out,
                          uint8_t* d_found, uint64_t* d_scores_out);
int cskv_program_add_insert_or_assign(cskv_program* prog, uint64_t n, const uint64_t* d_keys,
                                      const float* d_values, const uint64_t* d_scores, uint8_t* d_status);
int cskv_program_add_insert_and_evict(cskv_program* prog, uint64_t n, const uint64_t* d_keys,
                                      const float* d_values, const uint64_t* d_scores, uint8_t* d_status,
                                      uint64_t* d_ev_keys, float* d_ev_values, uint64_t* d_ev_scores,
                                      uint64_t* d_n_evicted);
int cskv_program_add_erase(cskv_program* prog, uint64_t n, const uint64_t* d_keys, uint8_t* d_erased);
/*
 * 1: the program is a graph of phases instead of one kernel sequence.  Phases: a find
 * run; the probe and the clear of an erase; the scratch preparation (clear, dedupe), routing,
 * apply and status gather of an upsert.  Readers (find runs, routings, probes) wait only for the
 * last writer; writers (applies, clears) wait for the last writer and every reader since (the
 * reader/writer rule of Sec. 3.5); the first phase of an upsert or erase waits only for the
 * previous user of its scratch slot (two slots rotate).  An op whose buffers (keys, values,
 * scores, outputs) overlap a buffer of an earlier op that one of the two writes starts after that
 * op is complete, and such a find is not merged into the earlier find's run, so results equal
 * those of the calls issued one by one whatever the aliasing.  cskv_program_launch runs the
 * phases on the program's own default-priority streams ordered by events, forked from and joined
 * back into the launch stream; cskv_program_capture builds a hipGraph with one child node per
 * phase (each recorded alone on `stream`) and the dependencies as edges.  Independent phases of
 * different batches then overlap on the device, at the price of cross-stream event waits.
 * 2: prep ahead: the same graph with every phase but the scratch preparations chained in program
 * order on one stream, so that only each upsert's clear and dedupe run ahead, beside earlier
 * batches (two cross-stream waits per upsert).
 * 0 (default): every phase in program order on the launch stream (the captured graph is that one
 * sequence).  Set before cskv_program_set_workspace; CSKV_EINVAL for another mode.
 */
int cskv_program_set_overlap(cskv_program* prog, int mode);
size_t cskv_program_workspace_bytes(const cskv_program* prog);
int cskv_program_set_workspace(cskv_program* prog, void* d_ws, size_t ws_bytes);
/* number of kernel-sequence segments: merged find runs + upserts + erases */
uint32_t cskv_program_segments(const cskv_program* prog);
/* number of phases of the overlapped form (0 when overlap is off or before set_workspace) */
uint32_t cskv_program_phases(const cskv_program* prog);
int cskv_program_launch(cskv_program* prog, void* stream);
int cskv_program_capture(cskv_program* prog, void* stream);
int cskv_program_replay(cskv_program* prog, void* stream);

/* number of buckets, value dim, mode and policy of a table (0 / -1 for NULL) */
uint64_t cskv_num_buckets(const cskv_table* table);
uint32_t cskv_dim(const cskv_table* table);
int cskv_mode(const cskv_table* table);
int cskv_policy(const cskv_table* table);

/* static text for a return code */
const char* cskv_strerror(int code);

/*
 * Serving loop (continuous batching).  cskv_serve_trace runs a trace of requests against one
 * table, in real time when cfg->realtime is 1 (a request exists only from its arrival time on)
 * or with every request present at time 0 otherwise, and returns when all have completed.
 *  - Admission: requests are admitted in arrival order while their footprint (input and output
 *    bytes) fits into cfg->arena_budget_bytes together with every admitted, unfinished request;
 *    a request that does not fit waits (it is deferred, never failed); a request larger than
 *    the whole budget is refused with CSKV_EINVAL before anything runs.
 *  - Execution: admitted requests are launched in admission order whenever fewer than
 *    cfg->max_inflight_groups groups are on the GPU.  Consecutive admitted finds merge into one
 *    reader launch of at most cfg->max_merge (<= 64) requests; each insert_and_evict is a
 *    serialization point (inserter group, Sec. 3.5).  With cfg->reader_streams = 0 every group
 *    runs on `stream`, in order, and new groups are enqueued while earlier ones run.  With 1..4
 *    reader streams (created for the call at default priority, destroyed before it returns),
 *    inserters run on `stream` and reader groups rotate over the reader streams: a reader group
 *    waits only for the last inserter before it and an inserter for every reader group before
 *    it (events), so reader groups between two inserters execute concurrently (Sec. 3.5: readers
 *    are compatible with readers).  Either way the result of every request is exactly that of
 *    issuing the requests alone, one by one, in admission order.
 *  - Outputs go to the request's d_* result pointers; when those are NULL they go to a ring
 *    arena in the workspace (of arena_budget_bytes) and are recycled after completion.
 *  - Times (seconds from the start of the trace, host clock): admit_s, launch_s, complete_s
 *    (the host saw the group's completion event); seq is the admission order.
 * Workspace: cskv_serve_workspace_bytes(table, max_request_keys, arena_budget_bytes), 256-byte
 * aligned; max_request_keys bounds every request's n.
 */
enum { CSKV_REQ_FIND = 0, CSKV_REQ_INSERT_AND_EVICT = 1 };

typedef struct cskv_request {
    int op;              /* CSKV_REQ_* */
    uint64_t n;
    const uint64_t* d_keys;
    const float* d_values;      /* insert_and_evict: n*dim rows */
    const uint64_t* d_scores;   /* as for cskv_insert_and_evict */
    float* d_values_out;        /* find rows (nullable: arena) */
    uint8_t* d_flags;           /* find: found; insert: status (nullable: arena) */
    uint64_t* d_ev_keys;        /* insert results (nullable together: arena) */
    float* d_ev_values;
    uint64_t* d_ev_scores;
    uint64_t* d_n_evicted;
    double arrival_s;
    /* written by the server */
    double admit_s, launch_s, complete_s;
    uint64_t seq;
    uint32_t group;
} cskv_request;

typedef struct cskv_serve_config {
    uint64_t arena_budget_bytes;
    uint32_t max_inflight_groups;
    uint32_t max_merge;
    int realtime;
    uint32_t reader_streams;  /* 0: every group on `stream`; 1..4: reader groups rotate over that many
                                 streams of their own, so that consecutive reader groups run
                                 concurrently on the device */
} cskv_serve_config;

typedef struct cskv_serve_stats {
    uint64_t completed, groups, reader_launches, inserter_launches, deferred_for_memory, peak_inflight_bytes;
    double wall_s;
} cskv_serve_stats;

size_t cskv_serve_workspace_bytes(const cskv_table* table, uint64_t max_request_keys, uint64_t arena_budget_bytes);
int cskv_serve_trace(cskv_table* table, cskv_request* reqs, uint64_t nreq, const cskv_serve_config* cfg,
                     void* d_ws, size_t ws_bytes, void* stream, cskv_serve_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* CSKV_H */
