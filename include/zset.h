/*
 * zset.h -- C ABI of the MI355X factorization-set library (libzset.so).
 *
 * The library enumerates the factorization set
 *
 *     Z(n; g_1..g_d) = { a in N^d : sum_i a_i g_i = n }        (paper, Section 1)
 *
 * on one gfx950 GPU, writing every element as a row of d uint32 coordinates,
 * row-major, in strictly ascending lexicographic order (a_1 most significant).
 * It follows the paper's parallel bounded lexicographic enumeration with
 * low-dimension tabulation (Section 3, Alg 3.2): workers own bounded slices of
 * the output, step over the leading coordinates, and copy whole blocks of the
 * trailing k coordinates from a memo built on the GPU.  zset_memo_build builds
 * it by the dynamic recurrence of Lemma 2.3 run in elementwise batches
 * (Section 2.2, Alg 2.9).  Inside zset_enumerate_ex, memos of one or two
 * coordinates are built from the recurrence's closed solution instead (the
 * same lists, every element independent), and memos of three or more by the
 * recurrence; ZSET_MEMO_PATH=chain in the environment keeps the recurrence
 * for two coordinates too.
 *
 * Conventions shared by every entry point:
 *   - Pointers documented as "host" are read before the call returns and are
 *     owned by the caller.  Pointers documented as "device" must be device
 *     memory of the current HIP device (hipMalloc or a torch CUDA tensor).
 *   - Generators are taken in the caller's order; they are never sorted.
 *     Repeated generators and gcd > 1 are allowed (Z stays finite and exact).
 *   - Limits: 1 <= d <= ZSET_MAX_D, every g_i >= 1, n <= 2^31 - 2 (the
 *     count-table rows have n + 1 entries, indexed in 32 bits on the GPU).
 *   - Status codes are returned, never thrown; zset_strerror gives the text.
 *     On any error returned before the first kernel launch, `out` is untouched.
 *   - Every call that launches work synchronises its stream before returning,
 *     except zset_enumerate_async, which may return with its launches still
 *     queued (the library's later calls wait for them before they reuse its
 *     scratch memory).
 *   - The library keeps per-device scratch memory (count table, tile table,
 *     memo staging) that it grows on demand and reuses; calls are serialised
 *     by an internal lock.
 */
#ifndef ZSET_H
#define ZSET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZSET_MAX_D 32

typedef enum {
    ZSET_OK = 0,
    ZSET_EINVAL = -1,     /* invalid argument (see each entry point)            */
    ZSET_EOVERFLOW = -2,  /* |Z(n)| >= 2^64 - 1, or rows * d exceeds 2^64       */
    ZSET_ENOMEM = -3,     /* device or pinned host allocation failed            */
    ZSET_ECAPACITY = -4,  /* the output buffer holds fewer rows than |Z(n)|     */
    ZSET_EDEVICE = -5     /* a HIP call failed, or a kernel's own check failed  */
} zset_status;

/* Opaque, immutable, device-resident memo of Z(p; h_1..h_k) for p < top. */
typedef struct zset_memo_s *zset_memo;

typedef struct {
    int k;                   /* memo dimension (trailing coordinates copied from
                                the memo); -1 = automatic.  k = 0 solves the last
                                coordinate by division (Alg 3.1); k >= 1 uses the
                                memo (Alg 3.2).  Must lie in [0, d-1].          */
    int order;               /* 0 = ascending lex (default); 1 = descending, the
                                order the paper's streams produce.              */
    uint64_t rows_per_tile;  /* rows per worker slice; 0 = automatic.  Must be a
                                multiple of 128 when set.                       */
    int count_only;          /* 1 = no rows are written: only |Z(n)| and the
                                checksum are produced (`out` may be NULL).      */
    void *stream;            /* hipStream_t to run on; NULL = the null stream.  */
    int claim_pct;           /* percent of the slices that workgroups claim at
                                run time (in chunks, from a device counter)
                                instead of being dealt round-robin; -1 =
                                automatic (100), 0 = none.  Output is the same
                                for every value.                               */
    uint64_t memo_top;       /* 0 = the memo covers every p <= n; else it covers
                                p < memo_top only (a partial memo, Section 3.1
                                and Alg 3.2): rows whose trailing remainder p is
                                >= memo_top are unranked from the count table
                                instead of copied (Alg 3.2's Else branch).  The
                                output is the same for every value.  Ignored
                                when k = 0 or a memo handle is passed (the
                                handle's own top applies).                    */
} zset_opts;

/* Per-call timings (device time between HIP events on the call's stream) and
 * sizes.  Filled by zset_enumerate_ex when `stats` is non-NULL. */
typedef struct {
    double count_us;         /* count-table kernel                              */
    double memo_us;          /* memo build (0 when a memo handle is passed)     */
    double plan_us;          /* slice table (unranking of each slice start)     */
    double write_us;         /* write (or count-only) pass                      */
    double total_us;         /* first to last event                             */
    uint64_t rows;           /* |Z(n)|                                          */
    uint64_t memo_rows;      /* rows of the memo used                           */
    uint64_t memo_bytes;     /* device bytes of the memo used                   */
    uint64_t tiles;          /* worker slices launched                          */
    uint64_t rows_per_tile;
    int k;                   /* memo dimension used                             */
} zset_stats;

/* Fill *opts with the defaults: k = -1, ascending, automatic slices, rows
 * written, null stream, automatic claim_pct. */
void zset_default_opts(zset_opts *opts);

/*
 * zset_count -- |Z(n; g)| (Section 1), computed on the GPU from the count
 * table C_j[x] = |Z(x; g_j..g_d)| (C_j[x] = C_{j+1}[x] + C_j[x - g_j]).
 *   n      element, <= 2^31 - 2
 *   gens   host, d uint32 generators, each >= 1
 *   count  host, receives |Z(n)|
 * Errors: EINVAL (bad d, gens, n or NULL pointer), EOVERFLOW (|Z| >= 2^64-1),
 *         ENOMEM, EDEVICE.
 */
zset_status zset_count(uint64_t n, const uint32_t *gens, int d, uint64_t *count);

/*
 * zset_count_table -- the whole count table, for inspection and tests:
 *   table[j * (n+1) + x] = |Z(x; g_{j+1}..g_d)|  for j = 0..d, x = 0..n
 * (row d is 1 at x = 0 and 0 elsewhere).  Entries saturate at 2^64 - 1.
 *   table  device, (d+1)*(n+1) uint64, written
 *   stream hipStream_t or NULL
 * Errors: EINVAL, EDEVICE.
 */
zset_status zset_count_table(uint64_t n, const uint32_t *gens, int d,
                             uint64_t *table, void *stream);

/*
 * zset_memo_build -- memo of the trailing generators h (Section 3.1): the
 * lists Z(p; h_1..h_k) for every p in [0, top), each in ascending lex order,
 * built on the GPU by the disjoint recurrence of Lemma 2.3 read in ascending
 * order -- Z(p) is the concatenation over i = k..1 of incr_i applied to the
 * first |Z_{>=i}(p - h_i)| rows of Z(p - h_i) -- run elementwise in batches of
 * min(h) consecutive elements (Section 2.2) with one worker per copied row
 * (Alg 2.9, Section 2.3).
 *   gens_trailing host, k uint32 generators h_1..h_k, each >= 1
 *   k             1 <= k <= ZSET_MAX_D - 1
 *   top           number of elements tabulated, in [1, 2^31 - 1]
 *   stream        hipStream_t or NULL
 *   memo          host, receives the handle (free with zset_memo_free)
 * Errors: EINVAL, EOVERFLOW (memo rows >= 2^32), ENOMEM, EDEVICE.
 */
zset_status zset_memo_build(const uint32_t *gens_trailing, int k, uint64_t top,
                            void *stream, zset_memo *memo);

/* Release a memo handle (NULL is ignored). */
void zset_memo_free(zset_memo memo);

/*
 * zset_memo_read -- copy a memo to host memory.
 *   off   host, top+1 uint64: rows of Z(p; h) are rows[off[p] .. off[p+1])
 *   rows  host, off[top]*k uint32, or NULL to get the sizes only
 *   top_out, k_out, rows_out: host, optional (NULL to skip)
 * Errors: EINVAL, EDEVICE.
 */
zset_status zset_memo_read(zset_memo memo, uint64_t *off, uint32_t *rows,
                           uint64_t *top_out, int *k_out, uint64_t *rows_out);

/*
 * zset_enumerate -- all of Z(n; g) into `out` (the spec form): default
 * options, null stream, synchronous.
 *   out  device, at least |Z(n)| * d uint32 (size it with zset_count)
 * Errors: as zset_enumerate_ex.
 */
zset_status zset_enumerate(uint64_t n, const uint32_t *gens, int d, uint32_t *out);

/*
 * zset_enumerate_ex -- Z(n; g) with options.
 *   out           device, out_rows_cap * d uint32; ignored when count_only
 *   out_rows_cap  rows `out` holds; ECAPACITY before any launch if < |Z(n)|
 *   opts          host, or NULL for the defaults
 *   memo          optional memo handle whose generators equal g_{d-k+1..d}
 *                 (then k = the memo's k); a handle whose top is <= n is
 *                 used as a partial memo (see memo_top); NULL = the call
 *                 builds its own memo
 *   rows_written  host, optional: |Z(n)|
 *   checksum      host, optional: sum over rows r (ascending rank r) of
 *                 FNV-1a-64(LE64(r) || LE32(a_1) .. LE32(a_d)) mod 2^64,
 *                 computed on the GPU only when count_only is set (else 0)
 *   stats         host, optional: timings and sizes
 * Errors: EINVAL (bad d/gens/n/k/order/rows_per_tile, `out` not device
 *         memory, memo mismatch), EOVERFLOW, ECAPACITY, ENOMEM, EDEVICE.
 */
zset_status zset_enumerate_ex(uint64_t n, const uint32_t *gens, int d, uint32_t *out,
                              uint64_t out_rows_cap, const zset_opts *opts,
                              zset_memo memo, uint64_t *rows_written,
                              uint64_t *checksum, zset_stats *stats);

/*
 * zset_enumerate_async -- zset_enumerate_ex without waiting for the device
 * (no memo handle, no timings).  When the call takes the three-launch form
 * (k fixed at 1 or 2 by opts->k, n + 1 <= 16384, a memo of at most 2^19
 * rows, the default slice options, no partial memo), its launches (count
 * table and memo, slice plan and memo layout, write pass, then one thread
 * that writes the outcome) are enqueued on opts->stream and the call returns
 * at once; the caller synchronises the stream (or waits on an event recorded
 * after the call) before it reads `result` or `out`.  Otherwise the call runs
 * to completion as zset_enumerate_ex does and fills `result` before it
 * returns.  Calls on one stream run in call order, each reading and writing
 * the library's scratch memory after the one before; a call on another stream
 * first waits on the host for the last asynchronous call to end.  Rows,
 * order and checksum are exactly those of zset_enumerate_ex (Section 3,
 * Alg 3.2).
 *   out           device, out_rows_cap * d uint32; ignored when count_only
 *   out_rows_cap  rows `out` holds; checked on the device (nothing written,
 *                 result[0] = ZSET_ECAPACITY) when < |Z(n)|
 *   opts          host, or NULL for the defaults
 *   result        pinned host memory (hipHostMalloc, or a pinned torch
 *                 tensor), 3 uint64, written by the device once the call's
 *                 work is done: [0] the outcome as a zset_status (read as
 *                 int64_t: ZSET_OK, or ECAPACITY, EOVERFLOW, EINVAL for a
 *                 slice count beyond the plan, EDEVICE), [1] |Z(n)|, [2] the
 *                 checksum (count_only, else 0).  Owned by the caller; must
 *                 not be reused before the stream has passed this call.
 *   write_events  NULL, or two hipEvent_t that the call records on
 *                 opts->stream right before and right after its write pass
 *                 (for timing the pass of an asynchronous call) when k is
 *                 fixed at 1 or 2 with the default slice options; other
 *                 calls leave them unrecorded
 * Returns ZSET_OK once the work is enqueued.  Errors found before any launch
 * are returned (EINVAL: as zset_enumerate_ex, `result` not pinned host memory,
 * a NULL event; ENOMEM; EDEVICE for a failed launch); a call that ran to
 * completion returns its outcome and also writes it to result[0].
 */
zset_status zset_enumerate_async(uint64_t n, const uint32_t *gens, int d, uint32_t *out,
                                 uint64_t out_rows_cap, const zset_opts *opts,
                                 uint64_t *result, void *const *write_events);

/*
 * zset_enumerate_noalloc -- zset_enumerate_ex for callers that cannot
 * allocate device memory (code that must not call hipMalloc: tight serving
 * loops, harnesses that forbid allocation).  It calls no hipMalloc, hipFree
 * or other allocating routine: every scratch buffer (count table, memo and
 * its leaf layout, slice table, status words) is carved from one array of
 * ZSET_NOALLOC_SCRATCH_BYTES bytes in device memory that the library holds on
 * every device it runs on until the process ends.  The caller passes the
 * inputs and the output as for zset_enumerate_ex (same rows, same
 * checksum); every launch runs in order on opts->stream and the call returns
 * after they complete.  No memo handle and no timings.
 *   out           device, out_rows_cap * d uint32; ignored when count_only
 *   out_rows_cap  rows `out` holds; ECAPACITY (nothing written) if < |Z(n)|
 *   opts          host, or NULL for the defaults (zset_default_opts)
 *   rows_written  host, optional: |Z(n)|
 *   checksum      host, optional: as zset_enumerate_ex (count_only only)
 * opts->memo_top must be 0 or > n (no partial memo).
 * Errors: as zset_enumerate_ex, and ENOMEM (before any output is written)
 *         when the query's scratch exceeds the array: about
 *         8 (d + 1)(n + 1) bytes of count table, the slice table and the memo.
 * The array is shared by every call on a device and keeps the last call's
 * contents (the call clears what must start at zero).  Two calls that
 * overlapped on one device would race on it: the library's lock serialises
 * them within a process, and each process has its own array.
 */
#define ZSET_NOALLOC_SCRATCH_BYTES (64u << 20)

zset_status zset_enumerate_noalloc(uint64_t n, const uint32_t *gens, int d, uint32_t *out,
                                   uint64_t out_rows_cap, const zset_opts *opts,
                                   uint64_t *rows_written, uint64_t *checksum);

/*
 * zset_enumerate_walk -- Z(n; g) without the count table: the lexicographic
 * walk of Section 2 (each coordinate takes its values in order, the last one
 * is forced by division), split over prefixes of the first coordinates that
 * the host refines where the estimated work is large.  A pass that counts each
 * prefix's completions, an exclusive sum, and a pass that writes them place
 * every row exactly.  Device memory beyond `out` is O(prefixes) (at most 2^22
 * of them) instead of the count table's (d + 1)(n + 1) words: the path for
 * large n with large generators, where that table would dwarf the output.
 * The last two coordinates are solved as an arithmetic progression, so the
 * work is the vectors (a_1..a_{d-2}) with a_1 g_1 + ... + a_{d-2} g_{d-2} <= n
 * plus the rows; small generators make the first term large and belong on
 * zset_enumerate_ex.
 *   out           device, out_rows_cap * d uint32
 *   out_rows_cap  rows `out` holds; ECAPACITY (nothing written) if < |Z(n)|
 *   order         0 = ascending lexicographic, 1 = descending
 *   stream        hipStream_t or NULL; the call is synchronous
 *   rows_written  host: |Z(n)|
 * Errors: EINVAL (bad d/gens/n/order, `out` NULL or not device memory),
 *         EOVERFLOW, ECAPACITY, ENOMEM, EDEVICE.
 */
zset_status zset_enumerate_walk(uint64_t n, const uint32_t *gens, int d, uint32_t *out,
                                uint64_t out_rows_cap, int order, void *stream,
                                uint64_t *rows_written);

/* ------------------------------------------------------------------------
 * Batches: many independent queries (n_q; g_q) enumerated by one persistent
 * write launch.  A batch is planned once (zset_batch_create: count tables,
 * memo dimension and slice length per query, output offsets, work units) and
 * then run any number of times (zset_batch_run), each run recomputing every
 * stage on the GPU -- count tables, memos (Lemma 2.3 recurrence), leaf
 * layouts, slice starts -- and ending with one persistent write kernel that
 * takes (query, slice range) work units from a device queue, largest first.
 * By default a run replays a HIP graph captured at the first run.
 *
 * In this version the batched path is switched off: zset_batch_create returns
 * ZSET_EDEVICE before any device work (a first device run stopped responding
 * and the cause is not identified).  The other entry points are unaffected.
 * ------------------------------------------------------------------------ */

typedef struct zset_batch_s *zset_batch;

typedef struct {
    int count_only;            /* 1: no rows; per-query |Z| and checksums only  */
    uint32_t max_chain_steps;  /* automatic k: largest memo recurrence length
                                  (batches of min(h) elements) a query may use;
                                  0 = 4096                                      */
    uint32_t unit_tiles;       /* slices per work unit; 0 = 64                  */
    int use_graph;             /* 1 = capture the run into a HIP graph at the
                                  first run and replay it; 0 = launch the
                                  stages one by one (per-stage timings)         */
    void *stream;              /* hipStream_t for zset_batch_run; NULL = the
                                  null stream                                   */
} zset_batch_opts;

typedef struct {
    double total_us;           /* device time of the run (events around it)     */
    double count_us, memo_us, plan_us, write_us;  /* per stage; use_graph = 0 only */
    uint64_t rows;             /* sum of |Z(n_q)|                               */
    uint64_t words;            /* output words including alignment padding      */
    uint64_t tiles;            /* slices over all queries                       */
    uint32_t units;            /* work units of the persistent write launch     */
    uint32_t memo_queries;     /* queries with k >= 1                           */
    uint32_t write_blocks;     /* workgroups of the persistent write launch     */
    uint32_t lds_bytes;        /* LDS per workgroup of the write launch         */
} zset_batch_stats;

/* Defaults: rows written, automatic limits, graph replay, null stream. */
void zset_batch_default_opts(zset_batch_opts *opts);

/*
 * zset_batch_create -- plan a batch of nq queries on the current device.
 *   nq             number of queries, >= 1
 *   n              host, nq elements, each <= 2^31 - 2
 *   d              host, nq dimensions, each in [1, ZSET_MAX_D]
 *   gens           host, sum(d) generators, query q's d[q] generators after
 *                  those of queries 0..q-1 (caller order, each >= 1)
 *   k              host, nq memo dimensions in [0, d[q]-1], or -1 = automatic
 *                  (the largest k whose memo fits the LDS budgets and whose
 *                  recurrence takes at most max_chain_steps batches); NULL =
 *                  all automatic.  A k >= 1 whose memo cannot be built in LDS
 *                  is EINVAL.
 *   rows_per_tile  host, nq slice lengths (multiples of 128) or 0 =
 *                  automatic; NULL = all automatic
 *   opts           host or NULL for the defaults
 *   batch          host, receives the handle (free with zset_batch_free)
 * The count tables are computed on the GPU here (one synchronisation); every
 * other device buffer is allocated here too, so zset_batch_run allocates
 * nothing.  Query q's rows go to words [offset_q, offset_q + |Z_q| * d[q]) of
 * the output, offset_q a multiple of 4 (16-byte aligned).
 * Errors: EINVAL, EOVERFLOW (a |Z| >= 2^64 - 1 or the output exceeds 2^64
 *         bytes), ENOMEM, EDEVICE.
 */
zset_status zset_batch_create(int nq, const uint64_t *n, const int *d,
                              const uint32_t *gens, const int *k,
                              const uint64_t *rows_per_tile,
                              const zset_batch_opts *opts, zset_batch *batch);

/*
 * zset_batch_info -- sizes chosen by zset_batch_create (any pointer may be
 * NULL): total output words, and per query (host arrays of nq) |Z_q|, output
 * word offset, memo dimension k and slice count.
 */
zset_status zset_batch_info(zset_batch batch, uint64_t *total_words, uint64_t *rows,
                            uint64_t *offsets, int *k, uint64_t *tiles);

/*
 * zset_batch_run -- run the batch once; returns after completion.
 *   out            device, 16-byte aligned, out_words_cap uint32 words
 *                  (>= total_words of zset_batch_info); ignored when
 *                  count_only.  Padding words between queries are not written.
 *   checksums      host, optional, nq entries: per query, the checksum of
 *                  zset_enumerate_ex (count-only batches; else zeros)
 *   stats          host, optional
 * Errors: EINVAL (`out` not 16-byte aligned device memory), ECAPACITY,
 *         EDEVICE (a HIP call or a kernel's own check failed).
 */
zset_status zset_batch_run(zset_batch batch, uint32_t *out, uint64_t out_words_cap,
                           uint64_t *checksums, zset_batch_stats *stats);

/*
 * zset_batch_times -- per-query completion times of the last run, in
 * microseconds from the start of that run, from the GPU's constant-rate
 * clock (host array of nq).
 */
zset_status zset_batch_times(zset_batch batch, double *done_us);

/* Release a batch (NULL is ignored). */
void zset_batch_free(zset_batch batch);

/* ------------------------------------------------------------------------
 * Serving: a request loop over resident generator sets.  A set g is made
 * resident once up to an element bound n_max (count table C_j[x], x <= n_max,
 * on the device with a host copy of |Z(n)| for every n <= n_max; for memo
 * dimension k >= 1 the memo of the trailing k generators for p <= n_max, built
 * by the recurrence of Lemma 2.3, in its leaf-order layout).  Queries (set, n)
 * are then submitted at any time; a dispatcher thread admits them in arrival
 * order as one of `slots` streams and room in the caller's output arena become
 * free (the rows of a query take |Z(n)| d uint32, rounded up to 16 bytes, known
 * at submission from the host copy), runs the slice plan and the write pass of
 * each on its own stream, and stamps submit / admit / done times.  Several
 * queries are on the device at once; each query's rows are the bytes
 * zset_enumerate_ex writes for it alone.  Outputs stay in the arena until
 * zset_server_release.  Entry points are thread-safe.
 * ------------------------------------------------------------------------ */

typedef struct zset_server_s *zset_server;

typedef struct {
    int slots;               /* queries on the device at once, 1..64; 0 = 8    */
    void *arena;             /* device buffer the outputs are carved from, owned
                                by the caller, 16-byte aligned, kept alive until
                                zset_server_free                               */
    uint64_t arena_bytes;    /* its size: the output budget                     */
    int dispatchers;         /* host threads that launch and retire queries, each
                                owning an equal share of the slots; 0 = 1 (more
                                threads measured slower: launches serialise in
                                the runtime)                                   */
    uint64_t memo_bytes;     /* memo budget of each resident set (its leaf-order
                                layout), bytes; 0 = 32 MiB.  A larger memo is
                                capped (zset_server_add_set)                   */
} zset_server_opts;

typedef struct {
    uint64_t rows;           /* |Z(n)|                                          */
    uint64_t out_offset;     /* uint32 word offset of the rows in the arena      */
    double submit_us;        /* host steady-clock times, microseconds since the  */
    double admit_us;         /* server was created: submission, launch on a      */
    double done_us;          /* slot, and completion seen by the dispatcher      */
} zset_server_result;

/* Fill *opts with the defaults (8 slots, no arena, 1 dispatcher, 32 MiB memos). */
void zset_server_default_opts(zset_server_opts *opts);

/* Start a server (its dispatcher thread) on the current device.
 * Errors: EINVAL (slots out of range, arena NULL / unaligned / not device
 * memory), ENOMEM, EDEVICE. */
zset_status zset_server_create(const zset_server_opts *opts, zset_server *server);

/*
 * zset_server_add_set -- make generator set gens (host, d uint32, each >= 1,
 * in the caller's order) resident up to n_max (<= 2^31 - 2) with memo
 * dimension k (-1 = the largest k >= 2 whose memo of the trailing k generators
 * over p <= n_max (Section 2.2, Lemma 2.3) fits opts.memo_bytes, else 1; d = 1
 * sets use 0).  The memo covers p < top: top = n_max + 1 when that memo fits
 * opts.memo_bytes, else the largest top whose memo does (at least 1).  With
 * top <= n a query's rows whose memo remainder is >= top are unranked from the
 * count table (Section 3.1, Alg 3.2's Else branch); the rows are the same.
 * Synchronous.  *set_id receives the set's index (0, 1, ...).
 * Errors: EINVAL, EOVERFLOW, ENOMEM, EDEVICE.
 */
zset_status zset_server_add_set(zset_server server, const uint32_t *gens, int d, uint64_t n_max,
                                int k, int *set_id);

/* A resident set's memo dimension, n_max, memo rows, device bytes and memo
 * top (the memo covers p < memo_top; n_max + 1 = every p).  Any output
 * pointer may be NULL. */
zset_status zset_server_set_info(zset_server server, int set_id, int *k, uint64_t *n_max,
                                 uint64_t *memo_rows, uint64_t *resident_bytes,
                                 uint64_t *memo_top);

/* |Z(n)| of a resident set from its host copy (no device work).
 * Errors: EINVAL (no such set, n > n_max), EOVERFLOW. */
zset_status zset_server_count(zset_server server, int set_id, uint64_t n, uint64_t *rows);

/* Queue query (set_id, n); never blocks.  *ticket identifies it.
 * Errors: EINVAL (no such set, n > n_max, server stopping), EOVERFLOW,
 * ECAPACITY (the rows exceed the whole arena). */
zset_status zset_server_submit(zset_server server, int set_id, uint64_t n, uint64_t *ticket);

/* Block until the query has finished; fill *result (may be NULL).  Returns the
 * query's status: OK, or EDEVICE (a HIP error or a kernel check) / EINVAL (the
 * server stopped before admitting it).  Errors: EINVAL (unknown ticket). */
zset_status zset_server_wait(zset_server server, uint64_t ticket, zset_server_result *result);

/* Give a finished query's rows back to the arena and forget the ticket.
 * Errors: EINVAL (unknown ticket, query not finished). */
zset_status zset_server_release(zset_server server, uint64_t ticket);

/* Queries admitted and completed so far, the most on the device at once, and
 * the dispatcher's host time spent enqueueing queries (microseconds).  Any
 * output pointer may be NULL. */
zset_status zset_server_stats(zset_server server, uint64_t *admitted, uint64_t *completed,
                              uint64_t *max_inflight, double *launch_us);

/* Stop the server: queries on the device finish, queued ones end with EINVAL;
 * then free every resident set (NULL is ignored).  The arena stays the
 * caller's. */
void zset_server_free(zset_server server);

/* Static text for a status code. */
const char *zset_strerror(zset_status status);

/*
 * zset_store_ceiling -- measurement only (no part of the enumeration): the
 * device's achievable HBM store rate in the write pass's store form.  Fills
 * `bytes` of `buf` (device, 16-byte aligned, bytes a multiple of 4) with
 * 16-byte non-temporal coalesced stores in three launch shapes (a one-shot
 * grid of 256-lane workgroups, one store per lane; a grid-stride loop with
 * one 256-lane workgroup per compute unit; 64 KiB blocks per wavefront with
 * four 256-lane workgroups per compute unit), each once untimed and then
 * `reps` times between HIP events on `stream` (hipStream_t or NULL);
 * *us_per_pass receives the mean time of one pass of the fastest shape, in
 * microseconds.  The buffer's contents are overwritten.
 * Errors: EINVAL, EDEVICE.
 */
zset_status zset_store_ceiling(void *buf, uint64_t bytes, int reps, void *stream,
                               double *us_per_pass);

/*
 * zset_selftest_host -- checks of host-side helpers that need no GPU (the
 * magic-number division used by the kernels, argument validation).  Returns
 * ZSET_OK or ZSET_EDEVICE with a message in zset_last_error().
 */
zset_status zset_selftest_host(void);

/* Text of the last error detected by the library on this thread ("" if none). */
const char *zset_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZSET_H */
