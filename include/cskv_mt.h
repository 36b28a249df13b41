/*
 * Concurrent-caller driver of the cache-semantic hash table (the setting of the paper's
 * concurrency ablation, Sec. 5.4 Exp. 3e): several host threads, each with its own HIP stream,
 * issue fixed batches on one table at the same time through the cskv.h calls, under whatever
 * lock mode the table has (cskv_set_lock_mode).
 *
 * Ownership: every pointer is the caller's device memory and must stay valid until the call
 * returns; the driver allocates only the threads' streams (created before the start barrier,
 * destroyed after) and returns after every thread's stream has drained.  Before destroying the
 * streams it resets the table's lock (cskv_set_lock_mode to the current mode), so no other
 * caller may use the table during the run.
 */
#ifndef CSKV_MT_H
#define CSKV_MT_H

#include <stddef.h>
#include <stdint.h>

#include "cskv.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CSKV_MT_FIND = 0,          /* reader: find of d_keys into d_values_out / d_flags */
    CSKV_MT_ASSIGN = 1,        /* updater: assign d_values (and d_scores) to d_keys */
    CSKV_MT_INSERT_ERASE = 2   /* inserter: insert_or_assign d_keys, then erase them, alternately */
};

typedef struct cskv_mt_thread {
    int op;                    /* CSKV_MT_* */
    uint64_t n;                /* keys per call (1 .. 2^31-1) */
    uint64_t calls;            /* calls this thread makes */
    const uint64_t* d_keys;    /* n keys, the same on every call */
    const float* d_values;     /* n x dim rows for ASSIGN / INSERT_ERASE */
    const uint64_t* d_scores;  /* n scores (CUSTOM policy; else may be NULL) */
    float* d_values_out;       /* n x dim rows for FIND */
    uint8_t* d_flags;          /* n bytes: found / status / erased flags of the latest call */
    void* d_ws;                /* this thread's workspace (not shared with another thread) */
    size_t ws_bytes;
    /* outputs */
    int status;                /* CSKV_* result of this thread */
    int hip_error;             /* hipGetLastError() after the failing call (0 if none failed) */
    uint64_t failed_call;      /* index of the failing call (calls if none failed) */
} cskv_mt_thread;

/*
 * Runs nthreads (1..64) threads at once from a common start; *wall_ms = host wall time from the
 * start until the last thread's stream has drained.  Returns the first error any call returned
 * (CSKV_* code; each thread's status, HIP error and failing call are written to its entry),
 * CSKV_EINVAL for bad arguments (checked before any thread starts).
 */
int cskv_mt_run(cskv_table* table, int nthreads, cskv_mt_thread* threads, double* wall_ms);

#ifdef __cplusplus
}
#endif

#endif /* CSKV_MT_H */
