// zset_internal.h -- declarations shared by the kernel files and the host
// library of libzset.so.  Not part of the public ABI (include/zset.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "zset_common.h"

namespace zset {

// Everything the slice planner and the write pass read.
struct EnumParams {
  Gens g;                   // generators g_0..g_{d-1}, caller order
  uint32_t n;               // element
  int d;                    // dimension
  int U;                    // coordinates fixed by a slice start
  int k;                    // memo dimension (0: last coordinate by division)
  uint64_t total;           // |Z(n)|
  uint64_t rows_per_tile;   // rows per slice (multiple of 128)
  uint64_t ntiles;          // slices
  const uint64_t* table;    // count table, (d+1) rows of table_stride entries (x = 0..n used)
  uint64_t table_stride;    // entries per count-table row: n + 1, or more for a resident table
  const uint64_t* endc;     // residue-class ends of the leaf-order memo (k >= 1)
  const uint32_t* leaf;     // leaf-order memo rows, k+1 uint32 each (k >= 1)
  uint64_t leaf_rows;       // rows in `leaf`
  uint32_t* tiles;          // slice starts, U+2 uint32 each
  uint32_t* out;            // rows, d uint32 each
  uint64_t* checksum;       // count-only: wrapping sum of row hashes
  int* err;                 // device status word
  DivMod32 dG;              // division by g_U
  DivMod32 dG1;             // division by g_{U-1} (pair lanes)
  uint32_t memo_top;        // the memo covers p < memo_top; 0 or > n: every p <= n (a
                            // partial memo's other rows are unranked from the count table)
  int desc;                 // 1: rows stored in descending lexicographic order (rank r at
                            // row total - 1 - r)
  int pair;                 // 1: the write pass's lanes range over (a_{U-2}, a_{U-1}) pairs
                            // (MODE 1, U >= 2), 0: over a_{U-1}
  uint32_t ring;            // rows in each wavefront's LDS staging ring (power of two)
  uint32_t flush;           // rows per coalesced flush (ring / 2)
  int pack;                 // memo row format: 0 plain words in global, 1 / 2 packed
                            // 32- / 64-bit words copied into LDS
  uint64_t memo_words;      // uint32 words of packed memo copied into LDS (0 if pack == 0)
  uint32_t fshift[kMaxD + 1];  // packed field c (0 = floor(p / G), c >= 1 = m_c): bit offset
  uint32_t fmask[kMaxD + 1];   // and mask
  int lds_cnt;              // 1: segment counts C[U][x] and class ends copied to LDS as uint32
  uint32_t nclass;          // residue classes of the leaf layout: min(G, n + 1)
  uint32_t max_tiles;       // slices one workgroup may own (their starts are held in LDS)
  uint32_t write_blocks;    // workgroups of the write pass; slice t < static_tiles goes to
                            // workgroup t mod NB
  uint64_t static_tiles;    // slices dealt round-robin; the rest are claimed in chunks
  uint32_t chunk;           // slices per claimed chunk (0: every slice is dealt)
  uint32_t* pool;           // chunk counter, zeroed by the slice planner
  int reset_status;         // 1: the slice planner also clears *err, *checksum, *blocks_done
  uint32_t* blocks_done;    // write workgroups finished (with done_flag)
  uint64_t* done_flag;      // non-NULL: the last write workgroup stores *err to done_flag[1]
  uint64_t done_seq;        // and then done_seq to done_flag[0] (pinned host words)
  // When total_dev is non-NULL, |Z(n)| is read there (dyn_size below): the
  // slice planner sizes the slices as slice_rows(|Z(n)|, want_tiles), and the
  // write pass, given no host-side |Z(n)| (total, rows_per_tile and ntiles
  // unset, every slice claimed), takes its slices the same way.
  const uint64_t* total_dev;
  uint64_t want_tiles;
  uint64_t out_rows_cap;    // with total_dev: rows the output holds (0: no check)
  int dyn;                  // write pass: 1 = total, slice length and count from dyn_size
};

// Rows per slice when `want` slices are asked for |Z| = total rows: a
// multiple of 128, at least 128 and at most 2^30.
__host__ __device__ inline uint64_t slice_rows(uint64_t total, uint64_t want) {
  uint64_t T = (total + want - 1) / want;
  T = (T + 127) / 128 * 128;
  if (T < 128) T = 128;
  if (T > (uint64_t(1) << 30)) T = uint64_t(1) << 30;
  return T;
}

// |Z(n)| read on the device (P.total_dev), with the slice length and count
// the planner uses for it, and the error that refuses the query: its bytes
// overflow 64 bits, it exceeds P.out_rows_cap rows, or its slices (at most
// 2^30 rows each) outnumber the want_tiles planned for.  A refused query gets
// no slices, so nothing is written.
struct DynSize {
  uint64_t total, T, ntiles;
  int err;
};
__device__ inline DynSize dyn_size(const EnumParams& P) {
  DynSize z;
  z.total = *P.total_dev;
  z.err = 0;
  if (z.total == ~uint64_t(0) || z.total > ~uint64_t(0) / (4 * uint64_t(P.d)))
    z.err = kErrOverflow;
  else if (P.out_rows_cap && z.total > P.out_rows_cap)
    z.err = kErrCapacity;
  z.T = slice_rows(z.err ? 0 : z.total, P.want_tiles);
  z.ntiles = z.err ? 0 : (z.total + z.T - 1) / z.T;
  if (z.ntiles > P.want_tiles) {
    z.err = kErrSlices;
    z.ntiles = 0;
  }
  return z;
}

// One query's share of a batched launch.
struct CountJob {
  uint64_t* table;          // (d+1) x N
  uint64_t* sums;           // d+1 row sums
  uint64_t* total;          // C[0][n]
  uint32_t N;               // n + 1
  int d;
  uint32_t g[kMaxD];
};

struct MemoJob {
  uint32_t h[kMaxD];        // memo generators
  int k;
  uint32_t top, step, W, R; // elements, batch width, ring size, rows
  uint32_t* nat;            // R x k natural-order rows
  uint64_t* off;            // top + 1 offsets
  uint32_t block0;          // batched k = 1 pass: first workgroup of this job
};

struct LeafJob {
  int k;
  uint32_t n;
  DivMod32 dG;              // division by g_U
  const uint64_t* off;
  const uint32_t* nat;
  const uint64_t* cu;       // count-table row U
  const uint64_t* endc;
  uint32_t* leaf;
  uint64_t leaf_rows;
  int pack;
  uint32_t block0;          // batched: first workgroup of this job
  uint32_t fshift[kMaxD + 1];
  int exact;                // 1: leaf_rows is the memo's row count; 0: a bound (partial
                            // memo), the rows being off[n + 1]
  const uint32_t* rowp;     // non-NULL: rowp[t] = the element p of natural-order row t
                            // (written with the memo), else found by bisection of off
};

// One memo row of the leaf-order layout: thread t takes natural-order row t;
// its element p is the last one with off[p] <= t (bisection of the offsets),
// and its place in the leaf layout is end[p mod G] - C_U[p] + (t - off[p]).
// Rows of one element are adjacent in both layouts, so neighbouring threads
// read and write neighbouring rows, and a long list costs no more than many
// short ones.  Row 0 also checks the memo's row count against leaf_rows.
__device__ inline void memo_leaf_row(const LeafJob& J, uint64_t t, int* __restrict__ err) {
  const uint64_t rows = J.off[uint64_t(J.n) + 1];
  if (J.exact ? (t == 0 && rows != J.leaf_rows) : (t == 0 && rows > J.leaf_rows))
    set_error(err, kErrMemoTotal);
  if (t >= rows || t >= J.leaf_rows) return;
  uint32_t p;
  if (J.rowp) {
    p = J.rowp[t];
  } else {
    uint32_t lo = 0, hi = J.n;
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      if (J.off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    p = lo;
  }
  const int k = J.k;
  const uint32_t q = J.dG.div(p);
  const uint32_t rho = J.dG.mod(p, q);
  const uint64_t pos = J.endc[rho] - J.cu[p] + (t - J.off[p]);
  if (pos >= J.leaf_rows) {
    set_error(err, kErrMemoTotal);
    return;
  }
  const uint32_t* src = J.nat + t * k;
  if (J.pack == 0) {
    uint32_t* dst = J.leaf + pos * (k + 1);
    dst[0] = q;
    for (int c = 0; c < k; ++c) dst[1 + c] = src[c];
  } else {
    uint64_t w = uint64_t(q) << J.fshift[0];
    for (int c = 0; c < k; ++c) w |= uint64_t(src[c]) << J.fshift[1 + c];
    if (J.pack == 1) J.leaf[pos] = uint32_t(w);
    else reinterpret_cast<uint64_t*>(J.leaf)[pos] = w;
  }
}

// k = 2 memo lists Z(p; h_1, h_2) in closed form.  With c = gcd(h_1, h_2), p
// has rows only when c divides p; then m_1 runs over the progression
// m_1 = m0 (mod h_2 / c), m0 = (p / c) (h_1 / c)^{-1} mod (h_2 / c), from m0
// to (p / c) / (h_1 / c), and m_2 = (p - m_1 h_1) / h_2.  Every element is
// independent: counts per element, an exclusive sum (the natural offsets) and
// a fill give the recurrence's lists (Lemma 2.3) in the same ascending order
// without its top / min(h) dependent batches.
struct Memo2 {
  uint32_t h1, h2, c, h1c, h2c, inv;  // inv = (h1 / c)^{-1} mod (h2 / c)
};
Memo2 make_memo2(uint32_t h1, uint32_t h2);  // host

__device__ inline bool memo2_first(const Memo2& M, uint32_t p, uint32_t* m0, uint32_t* rows) {
  if (p % M.c != 0) return false;
  const uint32_t q = p / M.c;
  const uint32_t mmax = q / M.h1c;
  const uint32_t a = uint32_t((uint64_t(q % M.h2c) * M.inv) % M.h2c);
  if (a > mmax) return false;
  *m0 = a;
  *rows = (mmax - a) / M.h2c + 1;
  return true;
}

// The last two rows of a count table in closed form (d >= 2): C[d-1][x] =
// [g_{d-1} divides x], and C[d-2][x] = |Z(x; g_{d-2}, g_{d-1})|, the number of
// rows of Memo2 for (h_1, h_2) = (g_{d-2}, g_{d-1}) at p = x, with every
// division by an invariant divisor.  `on` is 0 when the table must be scanned
// from row d instead (d = 1, or h_2 / gcd >= 2^16, where the product below
// could leave 32 bits).
struct LastRows {
  int on;
  uint32_t inv;             // (h_1 / c)^{-1} mod (h_2 / c), c = gcd(h_1, h_2)
  DivMod32 dg;              // g_{d-1}
  DivMod32 dc, dh1c, dh2c;  // c, h_1 / c, h_2 / c
};
LastRows make_last_rows(const uint32_t* gens, int d);  // host

__host__ __device__ inline uint32_t last_row_divides(const LastRows& L, uint32_t x) {
  return x == L.dg.div(x) * L.dg.d ? 1u : 0u;
}

__host__ __device__ inline uint32_t last_row_pair(const LastRows& L, uint32_t x) {
  const uint32_t q = L.dc.div(x);
  if (x != q * L.dc.d) return 0;
  const uint32_t mmax = L.dh1c.div(q);
  const uint32_t qm = q - L.dh2c.div(q) * L.dh2c.d;
  const uint32_t prod = qm * L.inv;  // < (h_2 / c)^2 < 2^32
  const uint32_t a = prod - L.dh2c.div(prod) * L.dh2c.d;
  return a > mmax ? 0u : L.dh2c.div(mmax - a) + 1u;
}

// The first launch of a call with the memo dimension fixed at 1 or 2 and a
// count table that fits LDS (count_table.hip): workgroup 0 clears the two
// status words, computes the rows of the count table that the slice plan, the
// leaf layout and the write pass read (rows 1..U; row 0 only on the residue
// class of n mod g_0 when U >= 1) and |Z(n)| into sums[d + 1], and then the
// residue-class ends of row U;
// workgroup 1 builds the memo in natural order (off: top + 1 offsets, nat: R
// rows; k = 1 or 2 in closed form) and stamps its start and end on the
// device's constant-rate clock into stamps[0..1].
struct SetupJob {
  uint64_t* table;          // (d+1) x N
  uint64_t* sums;           // 2d + 3 words; [d + 1] receives |Z(n)|
  uint64_t* status;         // 2 words cleared first
  Gens g;
  uint32_t N;               // n + 1 (<= count_table_lds_max())
  int d;
  uint32_t walk;            // count-table column walk bound
  int U;
  uint32_t nclass;          // min(g_U, N)
  DivMod32 dG;              // division by g_U
  uint64_t* endc;
  int k;                    // 1 or 2
  Memo2 M;                  // k = 2
  uint32_t h1;              // k = 1: the memo generator
  uint32_t R;               // memo rows
  uint32_t* nat;
  uint64_t* off;
  uint64_t* stamps;
  LastRows last;            // the table's rows d-1 and d-2 in closed form (when on)
  uint32_t* rowp;           // R words: the element p of each natural-order memo row
};

struct ClassJob {
  const uint64_t* cu;       // count-table row U
  uint64_t* endc;
  uint32_t n;
  uint32_t nclass;
  DivMod32 dG;
};

// A batched write-pass work unit: slices [tile_lo, tile_hi) of query q.
struct BatchUnit {
  uint32_t q, tile_lo, tile_hi, pad;
};

// LDS layout (uint32 words) of the batched write pass.
struct BatchLds {
  uint32_t desc, memo, cnt, endc, states, waves;  // region offsets
  uint32_t wave_words;      // per wavefront: staging ring + 64 marks
  uint32_t ring_words;      // staging ring words (ring rows x largest d)
  uint32_t total_words;
};

// count_table.hip
// Count table (d+1) x (n+1); when sums is non-NULL (2d+3 entries) also
// sums[j] = sum_x C[j][x] for j = 0..d, sums[d+1] = C[0][n] = |Z(n)| and
// sums[d+2+j] = max_x C[j][x] (all saturating).
hipError_t launch_count_table(uint64_t* table, uint64_t n, const uint32_t* gens, int d,
                              uint64_t* sums, hipStream_t s);
// ZSET_COUNT_LAST=0 scans every row from row d (tests); else rows d-1 and d-2
// come from their closed forms when make_last_rows allows.
bool count_last_rows_enabled();
uint32_t count_table_lds_max();
hipError_t prepare_count_table_batch(uint32_t max_lds_n);
hipError_t launch_setup_fixed(const SetupJob& J, hipStream_t s);
hipError_t launch_count_table_batch(const CountJob* jobs, uint32_t njobs, uint32_t max_lds_n,
                                    bool lds, hipStream_t s);

// scan.hip
hipError_t launch_exclusive_scan(const uint64_t* in, uint64_t count, uint64_t* out,
                                 hipStream_t s);
hipError_t launch_class_ends(const uint64_t* count_row_u, uint64_t n, uint32_t G,
                             uint64_t* endc, uint32_t* nclass_out, hipStream_t s);
hipError_t launch_class_ends_batch(const ClassJob* jobs, uint32_t njobs, hipStream_t s);

// memo.hip
// Words of the one-wavefront recurrence's cardinality rings (GE and OFF) and
// its 64 row marks, rounded up so that the memo rows after them start 16-byte
// aligned.
__host__ __device__ inline uint32_t memo_ring_words(int k, uint32_t W) {
  return ((W * uint32_t(k + 1) + 3u) & ~3u) + 64u;
}
size_t memo_wave_lds_bytes(int k, uint64_t R, uint32_t W);
// Rows of memo that fit beside the rings in lds_bytes of LDS.
uint64_t memo_wave_capacity(int k, uint32_t W, size_t lds_bytes);
// Rcap: rows the LDS holds; Rexp: expected rows (0 = not known yet).
hipError_t launch_memo_chain_wave(const uint32_t* h, int k, uint64_t top, uint32_t step,
                                  uint32_t W, uint64_t Rcap, uint64_t Rexp, uint32_t* nat,
                                  uint64_t* off_out, int* err, hipStream_t s);
// The recurrence for memos larger than LDS: a ring of cap_rows rows (a power
// of two, >= (max(h) + step) x the longest list) and rows streamed to nat.
hipError_t launch_memo_chain_window(const uint32_t* h, int k, uint64_t top, uint32_t step,
                                    uint32_t W, uint32_t hmax, uint32_t cap_rows, uint64_t Rexp,
                                    uint32_t* nat, uint64_t* off_out, int* err, hipStream_t s);
hipError_t launch_memo_global(const uint32_t* h, int k, uint64_t top, uint32_t b,
                              const uint64_t* off, const uint64_t* ge, uint64_t ge_stride,
                              uint64_t* srcw, uint32_t* nat, int* err, hipStream_t s,
                              uint64_t rows);
LeafJob make_leaf_job(int k, uint64_t n, uint32_t G, const uint64_t* off, const uint32_t* nat,
                      const uint64_t* cu, const uint64_t* endc, uint32_t* leaf,
                      uint64_t leaf_rows, const EnumParams& P);
hipError_t launch_memo_leaf(const LeafJob& J, int* err, hipStream_t s);
hipError_t launch_memo_leaf_batch(const LeafJob* jobs, uint32_t njobs, uint32_t blocks,
                                  int* err, hipStream_t s);
// k = 2 in closed form: counts per element into cnt (top + 1 words), their
// exclusive sum into off (top + 1 words: off[top] = rows over p < top) and
// the rows into nat (at most cap rows written).
hipError_t launch_memo_k2(uint32_t h1, uint32_t h2, uint64_t top, uint64_t cap, uint32_t* nat,
                          uint64_t* off, uint64_t* cnt, hipStream_t s);
// k = 1: the closed solution of the recurrence, one parallel pass.
uint32_t memo_k1_blocks(uint64_t top);
hipError_t launch_memo_k1(uint32_t h, uint64_t top, uint64_t R, uint32_t* nat, uint64_t* off,
                          hipStream_t s);
hipError_t launch_memo_k1_batch(const MemoJob* jobs, uint32_t njobs, uint32_t blocks,
                                hipStream_t s);
// prepare = true only sets the launch attributes (before graph capture).
hipError_t launch_memo_chain_batch(const MemoJob* jobs, uint32_t njobs, int kmax_class,
                                   size_t lds_bytes, int* err, hipStream_t s, bool prepare);

// enumerate.hip
size_t write_lds_bytes(const EnumParams& P);
int write_waves_per_block();
hipError_t write_occupancy(const EnumParams& P, bool count_only, bool align16, int* per_cu);
hipError_t launch_plan(const EnumParams& P, hipStream_t s);
// The same planner sized on the device (P.total_dev, P.want_tiles): a grid for
// want_tiles slices, of which the first ceil(|Z| / slice_rows) are planned.
hipError_t launch_plan_device_sized(const EnumParams& P, hipStream_t s);
// The device-sized planner and the memo's leaf layout (memo_leaf_row over
// J.leaf_rows rows) in one grid: the planner's workgroups first.
hipError_t launch_plan_leaf(const EnumParams& P, const LeafJob& J, hipStream_t s);
hipError_t launch_write(const EnumParams& P, bool count_only, bool align16, hipStream_t s);
hipError_t launch_single(uint64_t n, uint32_t g, uint32_t* out, bool count_only,
                         uint64_t* checksum, hipStream_t s);

// Batched forms (batch.hip drives them).  qp: one EnumParams per query;
// qout: each query's first output word.
int write_batch_waves();
hipError_t launch_batch_reset(uint32_t* queue, int* err, uint32_t* done_tiles,
                              uint64_t* checksums, uint64_t* t_done, uint64_t* t_start,
                              uint32_t nq, hipStream_t s);
hipError_t launch_plan_batch(const EnumParams* qp, const uint64_t* tile_base,
                             const uint32_t* plan_q, uint32_t nplan, uint64_t total_tiles,
                             hipStream_t s);
hipError_t prepare_write_batch(const BatchLds& L, bool count_only);
hipError_t write_batch_occupancy(const BatchLds& L, bool count_only, int* per_cu);
hipError_t launch_write_batch(const EnumParams* qp, const uint64_t* qout, const BatchUnit* units,
                              uint32_t nunits, uint32_t* queue, uint32_t* done_tiles,
                              uint64_t* t_done, uint32_t* out, const BatchLds& L,
                              uint32_t blocks, bool count_only, hipStream_t s);
hipError_t launch_single_batch(const EnumParams* qp, const uint64_t* qout, const uint32_t* idx,
                               uint32_t count, uint32_t* out, bool count_only, uint64_t* t_done,
                               hipStream_t s);

}  // namespace zset
