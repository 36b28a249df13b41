/*
 * Sequential CPU oracle for the cache-semantic GPU hash table of arxiv 2603.17168
 * ("HierarchicalKV").  TEST INFRASTRUCTURE ONLY: it is linked by the test suite, by the
 * GPU smoke check and by the benchmark's CPU-baseline leg, never by the product path.
 * It shares no code, header or table with the HIP library.
 *
 * What it computes, one batch call at a time, with no parallelism and no blocking:
 *
 *   State.  B buckets (B a power of two), each an unordered set of at most S entries
 *   (key, score, value-id).  Slot positions are not modelled: they are not observable.
 *   Value rows are opaque and only ever copied, so the oracle stores a 64-bit value-id per
 *   entry instead of the row; the caller maps ids back to rows.
 *
 *   Hash (Sec. 3.1/3.2: a Murmur3-derived hash picks the bucket).  h = fmix64(key), the
 *   64-bit finalizer of Appleby's MurmurHash3.  Candidate buckets: b1 = h mod B and, in
 *   dual mode (Sec. 3.4, Alg. 3), b2 = (h >> 40) mod B.  The 8-bit digest only filters
 *   probes (Alg. 1) and cannot change any result, so the oracle has none.
 *
 *   Reserved words: 0 (empty slot) and 2^64-1 (slot lock) are not user keys; a batch
 *   entry carrying one gets status INVALID_KEY (find: not found; erase: not erased).
 *
 *   find (Alg. 1): look in b1, then b2; a hit returns the value-id and score; a miss
 *   leaves the outputs untouched.  No state change.
 *
 *   insert_or_assign / insert_and_evict (Alg. 2 inside Alg. 3), one batch:
 *     1. Scores.  LRU: the table clock advances by one per call and every key of the
 *        call gets that clock value.  CUSTOM: the caller's score.  LFU: the caller's
 *        increment (1 if none given), summed over a key's occurrences, saturating.
 *     2. Duplicates in the batch collapse to one operation per key; the last occurrence
 *        provides the value (and the CUSTOM score); every occurrence reports that
 *        operation's status.
 *     3. Route, against the table as it was before the batch: a key already present in
 *        b1 or b2 is an UPDATE there (Alg. 2 steps for a found key).  Otherwise it is an
 *        INSERT into: b1 in single mode or when b1 == b2; else phase D1 when either
 *        candidate has a free slot - the less occupied one, b1 on a tie; else phase D2 -
 *        the candidate whose minimum entry, ordered by (score, key), is smaller.
 *     4. Apply, bucket by bucket: first every UPDATE (score: CUSTOM the new score, LRU
 *        the clock, LFU old + sum, saturating; value-id replaced).  Then the INSERTs in
 *        order of descending score, ascending key: a free slot takes the key; in a full
 *        bucket the minimum entry by (score, key) is evicted when the new score is
 *        strictly greater than its score (admission control, Sec. 3.3), else the key is
 *        rejected.  Evicted entries are reported with the score and value they had.
 *     Sub-rounds (a semantic setting, 1 by default; the paper's batches are r = 1): with r
 *        sub-rounds the call's N distinct operations, ordered by the index of their key's
 *        last occurrence, are cut into r chunks - operation of rank q goes to chunk
 *        floor(q * r / N) - and steps 3 and 4 run chunk after chunk, each routing against
 *        the table the chunks before it left.  Steps 1, 2 and the statuses are per call.
 *
 *   erase: every present key is removed; erased[i] tells whether key[i] was present
 *   before the call.  size: number of entries.  export: all entries of a bucket range.
 *
 *   The rest of the API named by Sec. 3.5's role list and Sec. 4.1:
 *   contains (reader): found[i] tells whether key[i] is resident.
 *   locate (reader): found[i] and the bucket of a resident key (the oracle models no slots;
 *     the GPU's position-returning find is checked against this bucket).
 *   assign / assign_scores (updaters: values or scores of existing entries, never bucket
 *     structure): LRU clock +1 per call; duplicates collapse to the last occurrence (value
 *     and CUSTOM score), LFU increments summed; a resident key's score is set as an UPDATE of
 *     insert_or_assign sets it and (assign only) its value-id replaced; absent keys change
 *     nothing; found[i] tells whether key[i] is resident.
 *   find_or_insert (inserter): insert_or_assign in which a resident key keeps its value-id
 *     (only its score is updated); out_vids[i] is key[i]'s value-id if it was resident before
 *     the call, else its last occurrence's value-id (inserted or rejected alike; a resident
 *     key that the same call then evicts still returns the value it had).
 *   export_if: the entries of a bucket range whose score is at least a threshold.
 *
 * Readings where the paper is silent or inconsistent (the batch order above, strict
 * admission, (score, key) victim order, digest bits, second hash, reserved words) are the
 * ones listed with the design notes of this repository.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_EMPTY 0ULL
#define ORA_LOCKED 0xFFFFFFFFFFFFFFFFULL

enum { ORA_SINGLE = 1, ORA_DUAL = 2 };
enum { ORA_CUSTOM = 0, ORA_LRU = 1, ORA_LFU = 2 };
enum { ST_UPDATED = 1, ST_INSERTED = 2, ST_INSERTED_EVICT = 3, ST_REJECTED = 4, ST_INVALID = 5 };

typedef struct {
    uint64_t key, score, vid;
} ora_entry;

typedef struct {
    uint64_t B;
    uint32_t S;
    int mode, policy;
    uint64_t clock;
    uint32_t subrounds; /* route sub-rounds per upsert call (1 = the whole batch at once) */
    ora_entry* e;  /* bucket b holds e[b*S .. b*S + cnt[b]) */
    uint32_t* cnt;
    /* path counters of the last calls (used for byte accounting) */
    uint64_t st_find_hit1, st_find_hit2, st_find_miss;
    uint64_t st_upd, st_ins, st_evict, st_rej, st_invalid, st_d2_routes;
} ora_table;

/* MurmurHash3 64-bit finalizer (Appleby, public domain). */
uint64_t ora_fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

uint64_t ora_b1(const ora_table* t, uint64_t key) { return ora_fmix64(key) & (t->B - 1); }

uint64_t ora_b2(const ora_table* t, uint64_t key) {
    if (t->mode != ORA_DUAL) return ora_b1(t, key);
    return (ora_fmix64(key) >> 40) & (t->B - 1);
}

static int is_reserved(uint64_t k) { return k == ORA_EMPTY || k == ORA_LOCKED; }

static uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? ~0ULL : s;
}

ora_table* ora_create(uint64_t B, uint32_t S, int mode, int policy) {
    if (B == 0 || (B & (B - 1)) != 0 || S == 0) return NULL;
    if (mode != ORA_SINGLE && mode != ORA_DUAL) return NULL;
    if (policy != ORA_CUSTOM && policy != ORA_LRU && policy != ORA_LFU) return NULL;
    ora_table* t = (ora_table*)calloc(1, sizeof(ora_table));
    t->B = B;
    t->S = S;
    t->mode = mode;
    t->policy = policy;
    t->subrounds = 1;
    t->e = (ora_entry*)calloc(B * S, sizeof(ora_entry));
    t->cnt = (uint32_t*)calloc(B, sizeof(uint32_t));
    if (!t->e || !t->cnt) {
        free(t->e);
        free(t->cnt);
        free(t);
        return NULL;
    }
    return t;
}

/* an independent copy of a table's whole state (entries, counts, clock, settings) */
ora_table* ora_clone(const ora_table* src) {
    if (!src) return NULL;
    ora_table* t = ora_create(src->B, src->S, src->mode, src->policy);
    if (!t) return NULL;
    memcpy(t->e, src->e, (size_t)src->B * src->S * sizeof(ora_entry));
    memcpy(t->cnt, src->cnt, (size_t)src->B * sizeof(uint32_t));
    t->clock = src->clock;
    t->subrounds = src->subrounds;
    return t;
}

void ora_destroy(ora_table* t) {
    if (!t) return;
    free(t->e);
    free(t->cnt);
    free(t);
}

uint64_t ora_clock(const ora_table* t) { return t->clock; }

uint64_t ora_size(const ora_table* t) {
    uint64_t s = 0;
    for (uint64_t b = 0; b < t->B; ++b) s += t->cnt[b];
    return s;
}

uint32_t ora_bucket_count(const ora_table* t, uint64_t b) { return t->cnt[b]; }

/* index of key within bucket b, or -1 */
static long find_in(const ora_table* t, uint64_t b, uint64_t key) {
    const ora_entry* e = t->e + b * t->S;
    for (uint32_t j = 0; j < t->cnt[b]; ++j)
        if (e[j].key == key) return (long)j;
    return -1;
}

/* (score, key) lexicographic order: is entry a smaller than entry b? */
static int entry_less(const ora_entry* a, const ora_entry* b) {
    if (a->score != b->score) return a->score < b->score;
    return a->key < b->key;
}

/* index of the minimum entry of a non-empty bucket under (score, key) */
static uint32_t min_in(const ora_table* t, uint64_t b) {
    const ora_entry* e = t->e + b * t->S;
    uint32_t m = 0;
    for (uint32_t j = 1; j < t->cnt[b]; ++j)
        if (entry_less(&e[j], &e[m])) m = j;
    return m;
}

void ora_find(ora_table* t, uint64_t n, const uint64_t* keys, uint8_t* found, uint64_t* vids,
              uint64_t* scores) {
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        found[i] = 0;
        if (is_reserved(k)) {
            t->st_invalid++;
            continue;
        }
        uint64_t b1 = ora_b1(t, k), b2 = ora_b2(t, k);
        long j = find_in(t, b1, k);
        uint64_t b = b1;
        if (j < 0 && b2 != b1) {
            j = find_in(t, b2, k);
            b = b2;
            if (j >= 0) t->st_find_hit2++;
        } else if (j >= 0) {
            t->st_find_hit1++;
        }
        if (j < 0) {
            t->st_find_miss++;
            continue;
        }
        const ora_entry* e = t->e + b * t->S + j;
        found[i] = 1;
        if (vids) vids[i] = e->vid;
        if (scores) scores[i] = e->score;
    }
}

/* ---- batch dedupe map: open addressing on the key, linear probing ---- */
typedef struct {
    uint64_t key;   /* 0 = unused (reserved keys never enter the map) */
    uint64_t last;  /* index of the last occurrence */
    uint64_t inc;   /* LFU: saturating sum of increments */
    long op;        /* index into the op array */
} dd_slot;

typedef struct {
    uint64_t key, bucket, s_new, vid;
    uint64_t last; /* index of the key's last occurrence in the batch */
    long slot;  /* UPDATE: index in bucket at routing time */
    int kind;   /* 1 = UPDATE, 2 = INSERT */
    uint64_t inc;
    int status;
    uint64_t out_vid; /* find_or_insert: the resident value-id, else the batch's */
} ora_op;

static uint64_t dd_find(dd_slot* m, uint64_t mask, uint64_t key) {
    uint64_t p = ora_fmix64(key ^ 0x5bd1e995ULL) & mask;
    while (m[p].key != 0 && m[p].key != key) p = (p + 1) & mask;
    return p;
}

static int cmp_last(const void* pa, const void* pb) {
    const ora_op* a = *(ora_op* const*)pa;
    const ora_op* b = *(ora_op* const*)pb;
    return a->last < b->last ? -1 : (a->last > b->last ? 1 : 0);
}

static int cmp_insert(const void* pa, const void* pb) {
    const ora_op* a = *(ora_op* const*)pa;
    const ora_op* b = *(ora_op* const*)pb;
    if (a->bucket != b->bucket) return a->bucket < b->bucket ? -1 : 1;
    if (a->s_new != b->s_new) return a->s_new > b->s_new ? -1 : 1; /* score descending */
    if (a->key != b->key) return a->key < b->key ? -1 : 1;          /* key ascending */
    return 0;
}

/*
 * One insert_or_assign / insert_and_evict call.  scores may be NULL (LRU always ignores
 * it; LFU then uses increment 1; CUSTOM requires it).  status, ev_* may be NULL.
 * Returns the number of evicted entries, or -1 on bad arguments / allocation failure.
 */
static long upsert_core(ora_table* t, uint64_t n, const uint64_t* keys, const uint64_t* vids,
                        const uint64_t* scores, uint8_t* status, uint64_t* ev_keys, uint64_t* ev_vids,
                        uint64_t* ev_scores, int keep_found, uint64_t* out_vids) {
    if (n == 0) return 0;
    if (t->policy == ORA_CUSTOM && !scores) return -1;
    /* 1. clock */
    if (t->policy == ORA_LRU) t->clock += 1;
    /* 2. dedupe, last writer wins */
    uint64_t cap = 1;
    while (cap < 2 * n) cap <<= 1;
    dd_slot* m = (dd_slot*)calloc(cap, sizeof(dd_slot));
    ora_op* ops = (ora_op*)calloc(n, sizeof(ora_op));
    if (!m || !ops) {
        free(m);
        free(ops);
        return -1;
    }
    long nops = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        if (is_reserved(k)) continue;
        uint64_t p = dd_find(m, cap - 1, k);
        if (m[p].key == 0) {
            m[p].key = k;
            m[p].op = nops++;
            m[p].inc = 0;
        }
        m[p].last = i;
        if (t->policy == ORA_LFU) m[p].inc = sat_add(m[p].inc, scores ? scores[i] : 1);
    }
    for (uint64_t p = 0; p < cap; ++p) {
        if (m[p].key == 0) continue;
        ora_op* o = &ops[m[p].op];
        o->key = m[p].key;
        o->last = m[p].last;
        o->vid = vids[m[p].last];
        o->inc = m[p].inc;
        if (t->policy == ORA_CUSTOM) o->s_new = scores[m[p].last];
        else if (t->policy == ORA_LRU) o->s_new = t->clock;
        else o->s_new = m[p].inc;
    }
    /* operations in order of their key's last occurrence; chunk of rank q: q * r / N */
    ora_op** ord = (ora_op**)malloc((size_t)(nops ? nops : 1) * sizeof(ora_op*));
    ora_op** ins = (ora_op**)malloc((size_t)(nops ? nops : 1) * sizeof(ora_op*));
    ora_op** sel = (ora_op**)malloc((size_t)(nops ? nops : 1) * sizeof(ora_op*));
    if (!ord || !ins || !sel) {
        free(ord); free(ins); free(sel); free(m); free(ops);
        return -1;
    }
    for (long q = 0; q < nops; ++q) ord[q] = &ops[q];
    qsort(ord, (size_t)nops, sizeof(ora_op*), cmp_last);
    const uint64_t r = t->subrounds ? t->subrounds : 1;
    long nev = 0;
    for (uint64_t c = 0; c < r; ++c) {
        long nsel = 0;
        for (long q = 0; q < nops; ++q)
            if ((uint64_t)q * r / (uint64_t)nops == c) sel[nsel++] = ord[q];
        /* 3. route against the table before this chunk (routing writes nothing) */
        for (long q = 0; q < nsel; ++q) {
            ora_op* o = sel[q];
            uint64_t b1 = ora_b1(t, o->key), b2 = ora_b2(t, o->key);
            long j = find_in(t, b1, o->key);
            if (j >= 0) {
                o->kind = 1; o->bucket = b1; o->slot = j;
                continue;
            }
            if (b2 != b1 && (j = find_in(t, b2, o->key)) >= 0) {
                o->kind = 1; o->bucket = b2; o->slot = j;
                continue;
            }
            o->kind = 2;
            if (b1 == b2) {
                o->bucket = b1;
            } else if (t->cnt[b1] < t->S || t->cnt[b2] < t->S) { /* phase D1 */
                o->bucket = (t->cnt[b1] <= t->cnt[b2]) ? b1 : b2;
            } else { /* phase D2 */
                const ora_entry* m1 = t->e + b1 * t->S + min_in(t, b1);
                const ora_entry* m2 = t->e + b2 * t->S + min_in(t, b2);
                o->bucket = entry_less(m2, m1) ? b2 : b1;
                t->st_d2_routes++;
            }
        }
        /* 4a. updates */
        for (long q = 0; q < nsel; ++q) {
            ora_op* o = sel[q];
            if (o->kind != 1) continue;
            ora_entry* e = t->e + o->bucket * t->S + o->slot;
            if (t->policy == ORA_LFU) e->score = sat_add(e->score, o->inc);
            else e->score = o->s_new;
            if (!keep_found) e->vid = o->vid;
            o->out_vid = e->vid;
            o->status = ST_UPDATED;
            t->st_upd++;
        }
        /* 4b. inserts, per bucket, by (score desc, key asc) */
        long nins = 0;
        for (long q = 0; q < nsel; ++q)
            if (sel[q]->kind == 2) ins[nins++] = sel[q];
        qsort(ins, (size_t)nins, sizeof(ora_op*), cmp_insert);
        for (long q = 0; q < nins; ++q) {
            ora_op* o = ins[q];
            uint64_t b = o->bucket;
            o->out_vid = o->vid; /* inserted, or rejected: the key's own value-id */
            ora_entry* be = t->e + b * t->S;
            if (t->cnt[b] < t->S) {
                ora_entry* e = be + t->cnt[b]++;
                e->key = o->key; e->score = o->s_new; e->vid = o->vid;
                o->status = ST_INSERTED;
                t->st_ins++;
                continue;
            }
            uint32_t mi = min_in(t, b);
            if (o->s_new > be[mi].score) {
                if (ev_keys) ev_keys[nev] = be[mi].key;
                if (ev_vids) ev_vids[nev] = be[mi].vid;
                if (ev_scores) ev_scores[nev] = be[mi].score;
                nev++;
                be[mi].key = o->key; be[mi].score = o->s_new; be[mi].vid = o->vid;
                o->status = ST_INSERTED_EVICT;
                t->st_evict++;
            } else {
                o->status = ST_REJECTED;
                t->st_rej++;
            }
        }
    }
    /* 5. per-occurrence status */
    if (status) {
        for (uint64_t i = 0; i < n; ++i) {
            if (is_reserved(keys[i])) {
                status[i] = ST_INVALID;
                continue;
            }
            status[i] = (uint8_t)ops[m[dd_find(m, cap - 1, keys[i])].op].status;
        }
    }
    if (out_vids) {
        for (uint64_t i = 0; i < n; ++i)
            if (!is_reserved(keys[i])) out_vids[i] = ops[m[dd_find(m, cap - 1, keys[i])].op].out_vid;
    }
    for (uint64_t i = 0; i < n; ++i)
        if (is_reserved(keys[i])) t->st_invalid++;
    free(ord);
    free(ins);
    free(sel);
    free(ops);
    free(m);
    return nev;
}

int ora_set_subrounds(ora_table* t, uint32_t r) {
    if (!t || r < 1 || r > 64) return -1;
    t->subrounds = r;
    return 0;
}

long ora_upsert(ora_table* t, uint64_t n, const uint64_t* keys, const uint64_t* vids,
                const uint64_t* scores, uint8_t* status, uint64_t* ev_keys, uint64_t* ev_vids,
                uint64_t* ev_scores) {
    return upsert_core(t, n, keys, vids, scores, status, ev_keys, ev_vids, ev_scores, 0, NULL);
}

/* find_or_insert; out_vids[i] untouched for reserved keys.  Returns 0, or -1 on bad arguments. */
long ora_find_or_insert(ora_table* t, uint64_t n, const uint64_t* keys, const uint64_t* vids,
                        const uint64_t* scores, uint8_t* status, uint64_t* out_vids) {
    long r = upsert_core(t, n, keys, vids, scores, status, NULL, NULL, NULL, 1, out_vids);
    return r < 0 ? -1 : 0;
}

/* bucket holding key k, or -1 */
static long bucket_of(const ora_table* t, uint64_t k) {
    uint64_t b1 = ora_b1(t, k), b2 = ora_b2(t, k);
    if (find_in(t, b1, k) >= 0) return (long)b1;
    if (b2 != b1 && find_in(t, b2, k) >= 0) return (long)b2;
    return -1;
}

void ora_contains(const ora_table* t, uint64_t n, const uint64_t* keys, uint8_t* found) {
    for (uint64_t i = 0; i < n; ++i) found[i] = !is_reserved(keys[i]) && bucket_of(t, keys[i]) >= 0;
}

void ora_locate(const ora_table* t, uint64_t n, const uint64_t* keys, uint8_t* found, uint64_t* buckets) {
    for (uint64_t i = 0; i < n; ++i) {
        long b = is_reserved(keys[i]) ? -1 : bucket_of(t, keys[i]);
        found[i] = b >= 0;
        if (b >= 0) buckets[i] = (uint64_t)b;
    }
}

/*
 * assign (vids != NULL) or assign_scores (vids == NULL).  scores as for ora_upsert.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
long ora_assign(ora_table* t, uint64_t n, const uint64_t* keys, const uint64_t* vids,
                const uint64_t* scores, uint8_t* found) {
    if (n == 0) return 0;
    if (t->policy == ORA_CUSTOM && !scores) return -1;
    if (t->policy == ORA_LRU) t->clock += 1;
    uint64_t cap = 1;
    while (cap < 2 * n) cap <<= 1;
    dd_slot* m = (dd_slot*)calloc(cap, sizeof(dd_slot));
    if (!m) return -1;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        if (is_reserved(k)) continue;
        uint64_t p = dd_find(m, cap - 1, k);
        m[p].key = k;
        m[p].last = i;
        if (t->policy == ORA_LFU) m[p].inc = sat_add(m[p].inc, scores ? scores[i] : 1);
    }
    for (uint64_t p = 0; p < cap; ++p) {
        if (m[p].key == 0) continue;
        long b = bucket_of(t, m[p].key);
        if (b < 0) continue;
        ora_entry* e = t->e + (uint64_t)b * t->S + find_in(t, (uint64_t)b, m[p].key);
        if (t->policy == ORA_CUSTOM) e->score = scores[m[p].last];
        else if (t->policy == ORA_LRU) e->score = t->clock;
        else e->score = sat_add(e->score, m[p].inc);
        if (vids) e->vid = vids[m[p].last];
    }
    for (uint64_t i = 0; i < n; ++i) found[i] = !is_reserved(keys[i]) && bucket_of(t, keys[i]) >= 0;
    free(m);
    return 0;
}

void ora_erase(ora_table* t, uint64_t n, const uint64_t* keys, uint8_t* erased) {
    /* presence is decided against the table before the call */
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        uint8_t f = 0;
        if (!is_reserved(k)) {
            uint64_t b1 = ora_b1(t, k), b2 = ora_b2(t, k);
            f = find_in(t, b1, k) >= 0 || (b2 != b1 && find_in(t, b2, k) >= 0);
        }
        if (erased) erased[i] = f;
    }
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        if (is_reserved(k)) continue;
        uint64_t bs[2] = {ora_b1(t, k), ora_b2(t, k)};
        for (int c = 0; c < 2; ++c) {
            long j = find_in(t, bs[c], k);
            if (j < 0) continue;
            ora_entry* be = t->e + bs[c] * t->S;
            be[j] = be[--t->cnt[bs[c]]];
            break;
        }
    }
}

/* entries of buckets [b0, b1) into the output arrays; returns the count */
uint64_t ora_export(const ora_table* t, uint64_t b0, uint64_t b1, uint64_t* keys, uint64_t* vids,
                    uint64_t* scores, uint64_t* buckets) {
    uint64_t c = 0;
    if (b1 > t->B) b1 = t->B;
    for (uint64_t b = b0; b < b1; ++b) {
        const ora_entry* be = t->e + b * t->S;
        for (uint32_t j = 0; j < t->cnt[b]; ++j, ++c) {
            if (keys) keys[c] = be[j].key;
            if (vids) vids[c] = be[j].vid;
            if (scores) scores[c] = be[j].score;
            if (buckets) buckets[c] = b;
        }
    }
    return c;
}

/* entries of buckets [b0, b1) with score >= min_score; returns the count */
uint64_t ora_export_if(const ora_table* t, uint64_t b0, uint64_t b1, uint64_t min_score, uint64_t* keys,
                       uint64_t* vids, uint64_t* scores, uint64_t* buckets) {
    uint64_t c = 0;
    if (b1 > t->B) b1 = t->B;
    for (uint64_t b = b0; b < b1; ++b) {
        const ora_entry* be = t->e + b * t->S;
        for (uint32_t j = 0; j < t->cnt[b]; ++j) {
            if (be[j].score < min_score) continue;
            if (keys) keys[c] = be[j].key;
            if (vids) vids[c] = be[j].vid;
            if (scores) scores[c] = be[j].score;
            if (buckets) buckets[c] = b;
            ++c;
        }
    }
    return c;
}

/* path counters: [hit1, hit2, miss, upd, ins, evict, rej, invalid, d2_routes] */
void ora_stats(const ora_table* t, uint64_t* out9) {
    out9[0] = t->st_find_hit1; out9[1] = t->st_find_hit2; out9[2] = t->st_find_miss;
    out9[3] = t->st_upd; out9[4] = t->st_ins; out9[5] = t->st_evict; out9[6] = t->st_rej;
    out9[7] = t->st_invalid; out9[8] = t->st_d2_routes;
}

void ora_reset_stats(ora_table* t) {
    t->st_find_hit1 = t->st_find_hit2 = t->st_find_miss = 0;
    t->st_upd = t->st_ins = t->st_evict = t->st_rej = t->st_invalid = t->st_d2_routes = 0;
}
