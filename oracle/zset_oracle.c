/*
 * zset_oracle.c -- CPU oracle for the factorization-set enumeration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes (Barron, "Two parallel dynamic lexicographic algorithms for
 * factorization sets in numerical semigroups", Section 1):
 *
 *     Z(n; g_1..g_d) = { a in N^d : sum_i a_i g_i = n }
 *
 * written as rows of d uint32 coordinates, row-major, strictly ascending in
 * lexicographic order with a_1 most significant.  Z is a set and lex order is
 * total, so this byte string is unique: the paper's parallel method (Alg 3.2
 * with its memo, Lemma 2.3 disjointness) reaches exactly this set, and the
 * oracle is the plain definition written out, not a transcription of the
 * method.  The paper enumerates in descending order; ascending is its exact
 * reversal.
 *
 * Every routine here is deliberately simple: nested loops and recursion, no
 * blocking, no reuse of one routine's arithmetic inside another beyond what
 * the definition states.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_EOVERFLOW -2
#define ORACLE_ENOMEM -3
#define ORACLE_ECAPACITY -4

/* ------------------------------------------------------------------------ */
/* Counting by the generating function prod_i 1/(1 - x^{g_i}) (Section 1).   */
/* ------------------------------------------------------------------------ */

static uint64_t sat_add(uint64_t a, uint64_t b)
{
    uint64_t s = a + b;
    return (s < a) ? UINT64_MAX : s;
}

/*
 * oracle_count: |Z(n; g)| as the coefficient of x^n in prod_i 1/(1-x^{g_i}),
 * extracted by the classical coin-change recurrence: multiply the series by
 * 1/(1-x^g) one generator at a time (ways[x] += ways[x-g] for x ascending).
 * Saturates at UINT64_MAX and then reports ORACLE_EOVERFLOW.
 */
int oracle_count(uint64_t n, const uint32_t *g, int d, uint64_t *count)
{
    if (d < 1 || !g || !count) return ORACLE_EINVAL;
    for (int i = 0; i < d; ++i) if (g[i] == 0) return ORACLE_EINVAL;
    uint64_t *ways = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!ways) return ORACLE_ENOMEM;
    ways[0] = 1;
    for (int i = 0; i < d; ++i)
        for (uint64_t x = g[i]; x <= n; ++x)
            ways[x] = sat_add(ways[x], ways[x - g[i]]);
    *count = ways[n];
    free(ways);
    return (*count == UINT64_MAX) ? ORACLE_EOVERFLOW : ORACLE_OK;
}

/*
 * oracle_count_table: table[j*(n+1) + x] = |Z(x; g_{j+1}..g_d)| for
 * j = 0..d (row d is the empty product: 1 at x = 0, else 0), x = 0..n.
 * Each row is its own coin-change series over its suffix of generators,
 * computed from scratch (no row is derived from another).  Entries saturate
 * at UINT64_MAX.
 */
int oracle_count_table(uint64_t n, const uint32_t *g, int d, uint64_t *table)
{
    if (d < 1 || !g || !table) return ORACLE_EINVAL;
    for (int i = 0; i < d; ++i) if (g[i] == 0) return ORACLE_EINVAL;
    for (int j = 0; j <= d; ++j) {
        uint64_t *ways = table + (size_t)j * (size_t)(n + 1);
        memset(ways, 0, (size_t)(n + 1) * sizeof(uint64_t));
        ways[0] = 1;
        for (int i = j; i < d; ++i)
            for (uint64_t x = g[i]; x <= n; ++x)
                ways[x] = sat_add(ways[x], ways[x - g[i]]);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Enumeration in ascending lexicographic order (Section 1 definition).      */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint32_t *g;
    int d;
    uint32_t *out;       /* rows, d uint32 each */
    uint64_t cap;        /* capacity in rows */
    uint64_t rows;       /* rows produced (may exceed cap: then not stored) */
    uint32_t prefix[64];
} enum_ctx;

/*
 * Fix coordinate j to 0, 1, 2, ... in ascending order while a_j g_j <= rem,
 * recursing on the rest; the last coordinate is forced: it exists iff g_d
 * divides what is left.  Ascending choices at every level give ascending
 * lexicographic order of the emitted rows.
 */
static void enum_rec(enum_ctx *c, int j, uint64_t rem)
{
    if (j == c->d - 1) {
        if (rem % c->g[j] != 0) return;
        uint64_t last = rem / c->g[j];
        if (c->rows < c->cap) {
            uint32_t *row = c->out + (size_t)c->rows * (size_t)c->d;
            for (int i = 0; i < j; ++i) row[i] = c->prefix[i];
            row[j] = (uint32_t)last;
        }
        c->rows++;
        return;
    }
    for (uint64_t a = 0; a * c->g[j] <= rem; ++a) {
        c->prefix[j] = (uint32_t)a;
        enum_rec(c, j + 1, rem - a * c->g[j]);
    }
}

/*
 * oracle_enumerate_a1: the rows of Z(n; g) whose first coordinate lies in
 * [a1_lo, a1_hi), ascending.  Writes at most cap rows to out; *rows gets the
 * number of rows in the range (ORACLE_ECAPACITY if that exceeds cap).
 */
int oracle_enumerate_a1(uint64_t n, const uint32_t *g, int d, uint64_t a1_lo,
                        uint64_t a1_hi, uint32_t *out, uint64_t cap,
                        uint64_t *rows)
{
    if (d < 1 || d > 64 || !g || !rows || (cap && !out)) return ORACLE_EINVAL;
    if (n > UINT32_MAX) return ORACLE_EINVAL;
    for (int i = 0; i < d; ++i) if (g[i] == 0) return ORACLE_EINVAL;
    enum_ctx c;
    memset(&c, 0, sizeof c);
    c.g = g; c.d = d; c.out = out; c.cap = cap;
    if (d == 1) {
        /* A single coordinate is forced: a_1 = n / g_1 when g_1 divides n. */
        if (n % g[0] == 0 && n / g[0] >= a1_lo && n / g[0] < a1_hi) {
            if (cap >= 1) out[0] = (uint32_t)(n / g[0]);
            c.rows = 1;
        }
    } else {
        for (uint64_t a = a1_lo; a < a1_hi && a * g[0] <= n; ++a) {
            c.prefix[0] = (uint32_t)a;
            enum_rec(&c, 1, n - a * g[0]);
        }
    }
    *rows = c.rows;
    return (c.rows > cap) ? ORACLE_ECAPACITY : ORACLE_OK;
}

/* oracle_enumerate: all of Z(n; g), ascending lexicographic order. */
int oracle_enumerate(uint64_t n, const uint32_t *g, int d, uint32_t *out,
                     uint64_t cap, uint64_t *rows)
{
    return oracle_enumerate_a1(n, g, d, 0, UINT64_MAX, out, cap, rows);
}

/*
 * oracle_unrank: the row of Z(n; g) at ascending rank r, found by walking the
 * coordinates left to right and, for each value a = 0, 1, ... of the current
 * coordinate, skipping the whole block of rows that share the prefix when r
 * lies past it.  Block sizes come from oracle_count_table's rows (passed in
 * as `table`, (d+1) x (n+1)).  ORACLE_EINVAL if r >= |Z(n)|.
 */
int oracle_unrank(uint64_t n, const uint32_t *g, int d, const uint64_t *table,
                  uint64_t r, uint32_t *row)
{
    if (d < 1 || !g || !table || !row) return ORACLE_EINVAL;
    if (r >= table[n]) return ORACLE_EINVAL;
    uint64_t rem = n;
    for (int j = 0; j < d; ++j) {
        const uint64_t *next = table + (size_t)(j + 1) * (size_t)(n + 1);
        uint64_t a = 0;
        for (;; ++a) {
            if (a * g[j] > rem) return ORACLE_EINVAL; /* unreachable */
            uint64_t block = next[rem - a * g[j]];
            if (r < block) break;
            r -= block;
        }
        row[j] = (uint32_t)a;
        rem -= a * g[j];
    }
    return (rem == 0) ? ORACLE_OK : ORACLE_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Memo of the trailing generators (Section 3.1): Z(p; h) for p < top.       */
/* ------------------------------------------------------------------------ */

/*
 * oracle_memo: for every p in [0, top) the list Z(p; h_1..h_k) in ascending
 * order, concatenated.  off[p] is the first row of Z(p; h) and off[top] the
 * total.  Built by running the plain enumerator once per p: it does not use
 * the dynamic recurrence that the GPU memo build follows, so it checks it.
 * Call with rows == NULL to size the table (off still filled).
 */
int oracle_memo(const uint32_t *h, int k, uint64_t top, uint64_t *off,
                uint32_t *rows, uint64_t cap)
{
    if (k < 1 || !h || !off) return ORACLE_EINVAL;
    uint64_t total = 0;
    for (uint64_t p = 0; p < top; ++p) {
        uint64_t cnt = 0;
        uint64_t room = (rows && total < cap) ? cap - total : 0;
        int st = oracle_enumerate(p, h, k, rows ? rows + (size_t)total * k : NULL,
                                  room, &cnt);
        if (st != ORACLE_OK && st != ORACLE_ECAPACITY) return st;
        off[p] = total;
        total += cnt;
    }
    off[top] = total;
    return (rows && total > cap) ? ORACLE_ECAPACITY : ORACLE_OK;
}

/*
 * oracle_memo_dynamic: the same lists built serially by the paper's dynamic
 * recurrence (Lemma 2.3; lists up to an element as in Alg 2.8; saved
 * cardinalities and block copies as in Section 2.3), read in ascending order.
 * The rows of Z(p) whose first nonzero coordinate is i are incr_i of the rows
 * of Z(p - h_i) that are zero left of i; in an ascending list those rows come
 * first, and there are ge[p - h_i][i] of them, where ge[m][i] = |Z_{>=i}(m)|
 * counts the rows of Z(m) that are zero left of i.  So Z(p) is the
 * concatenation over i = k, k-1, .., 1 of incr_i applied to the first
 * ge[p - h_i][i] rows of Z(p - h_i), and ge[p][i] is the number of rows in
 * the blocks i' >= i.  Z(0) = [0], ge[0][i] = 1.  One element at a time, on
 * one CPU thread: this is the CPU memo population the paper times against
 * its GPU one (Section 4.1, Table 1), used as that baseline.  It is checked
 * against oracle_memo, which does not use the recurrence.  Call with rows ==
 * NULL to size the table (off still filled).
 */
int oracle_memo_dynamic(const uint32_t *h, int k, uint64_t top, uint64_t *off,
                        uint32_t *rows, uint64_t cap)
{
    if (k < 1 || !h || !off || top < 1) return ORACLE_EINVAL;
    uint64_t *ge = (uint64_t *)malloc((size_t)top * k * sizeof(uint64_t));
    if (!ge) return ORACLE_ENOMEM;
    for (int i = 0; i < k; ++i) ge[i] = 1;
    off[0] = 0;
    if (rows && cap >= 1)
        for (int c = 0; c < k; ++c) rows[c] = 0;
    uint64_t total = 1;
    int st = ORACLE_OK;
    for (uint64_t p = 1; p < top; ++p) {
        off[p] = total;
        uint64_t acc = 0;
        for (int i = k - 1; i >= 0; --i) {
            uint64_t len = 0;
            if (p >= h[i]) {
                const uint64_t src = p - h[i];
                len = ge[src * k + i];
                if (rows) {
                    for (uint64_t t = 0; t < len; ++t) {
                        const uint64_t from = off[src] + t, to = total + t;
                        if (to >= cap) { st = ORACLE_ECAPACITY; break; }
                        for (int c = 0; c < k; ++c)
                            rows[to * k + c] = rows[from * k + c] + (c == i ? 1u : 0u);
                    }
                }
            }
            total += len;
            acc += len;
            ge[p * k + i] = acc;
        }
    }
    off[top] = total;
    free(ge);
    return (rows && total > cap) ? ORACLE_ECAPACITY : st;
}

/* ------------------------------------------------------------------------ */
/* Checksum of a row list.                                                   */
/* ------------------------------------------------------------------------ */

/*
 * FNV-1a, 64-bit, from the public FNV specification (Fowler, Noll, Vo):
 * start at the offset basis 14695981039346656037, and for each byte xor it
 * in and multiply by the prime 1099511628211, modulo 2^64.
 */
uint64_t oracle_fnv1a64(const uint8_t *bytes, uint64_t len)
{
    uint64_t h = 14695981039346656037ULL;
    for (uint64_t i = 0; i < len; ++i) {
        h ^= bytes[i];
        h *= 1099511628211ULL;
    }
    return h;
}

/*
 * oracle_checksum: S = sum over rows r of FNV1a64(LE64(rank0 + r) ||
 * LE32(row_r[0]) || ... || LE32(row_r[d-1])) modulo 2^64, where rank0 is the
 * ascending rank of the first row passed.  The rank makes S depend on order;
 * the sum makes it reducible in any grouping.
 */
uint64_t oracle_checksum(const uint32_t *rows, uint64_t nrows, int d,
                         uint64_t rank0)
{
    uint8_t buf[8 + 4 * 64];
    uint64_t s = 0;
    for (uint64_t r = 0; r < nrows; ++r) {
        uint64_t rank = rank0 + r;
        for (int b = 0; b < 8; ++b) buf[b] = (uint8_t)(rank >> (8 * b));
        for (int i = 0; i < d; ++i) {
            uint32_t v = rows[(size_t)r * d + i];
            for (int b = 0; b < 4; ++b)
                buf[8 + 4 * i + b] = (uint8_t)(v >> (8 * b));
        }
        s += oracle_fnv1a64(buf, 8 + 4 * (uint64_t)d);
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Multi-threaded form used only as the timed CPU baseline.                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t n;
    const uint32_t *g;
    int d;
    uint64_t a1_lo, a1_hi;
    uint32_t *out;
    uint64_t cap;
    uint64_t rows;
    int status;
} thread_job;

static void *thread_main(void *arg)
{
    thread_job *j = (thread_job *)arg;
    j->status = oracle_enumerate_a1(j->n, j->g, j->d, j->a1_lo, j->a1_hi,
                                    j->out, j->cap, &j->rows);
    return NULL;
}

/*
 * oracle_enumerate_a1_threads: same output as oracle_enumerate_a1, with the
 * a_1 values of [a1_lo, a1_hi) dealt out in contiguous runs to nthreads POSIX
 * threads.  Each thread's output offset is the number of rows before its run,
 * taken from the suffix count |Z(n - a_1 g_1; g_2..g_d)| per a_1 value (from
 * oracle_count_table's row 1, passed in as `row1`, length n+1).
 */
int oracle_enumerate_a1_threads(uint64_t n, const uint32_t *g, int d,
                                uint64_t a1_lo, uint64_t a1_hi,
                                const uint64_t *row1, uint32_t *out,
                                uint64_t cap, int nthreads, uint64_t *rows)
{
    if (d < 2 || nthreads < 1 || nthreads > 1024 || !row1 || !rows)
        return ORACLE_EINVAL;
    uint64_t a1_max = n / g[0];
    if (a1_hi > a1_max + 1) a1_hi = a1_max + 1;
    if (a1_lo > a1_hi) a1_lo = a1_hi;
    thread_job *jobs = (thread_job *)calloc((size_t)nthreads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof *tid);
    if (!jobs || !tid) { free(jobs); free(tid); return ORACLE_ENOMEM; }
    /* Thread t gets a contiguous run of a_1 values chosen so that the runs
       hold roughly equal row counts; the last thread takes what is left. */
    uint64_t total = 0;
    for (uint64_t a = a1_lo; a < a1_hi; ++a) total += row1[n - a * g[0]];
    if (total > cap) { free(jobs); free(tid); *rows = total; return ORACLE_ECAPACITY; }
    uint64_t a = a1_lo, before = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t target = (total * (uint64_t)(t + 1)) / (uint64_t)nthreads;
        uint64_t start = a, acc = before;
        while (a < a1_hi && (acc < target || t == nthreads - 1)) {
            acc += row1[n - a * g[0]];
            ++a;
        }
        jobs[t].n = n; jobs[t].g = g; jobs[t].d = d;
        jobs[t].a1_lo = start; jobs[t].a1_hi = a;
        jobs[t].out = out + (size_t)before * (size_t)d;
        jobs[t].cap = acc - before;
        before = acc;
    }
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&tid[t], NULL, thread_main, &jobs[t]) != 0) break;
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    int st = (started == nthreads) ? ORACLE_OK : ORACLE_ENOMEM;
    uint64_t got = 0;
    for (int t = 0; t < started; ++t) {
        if (jobs[t].status != ORACLE_OK) st = jobs[t].status;
        got += jobs[t].rows;
    }
    *rows = got;
    free(jobs); free(tid);
    return st;
}
