// enumerate.hip -- slice planning and the write pass.
//
// The output Z(n; g) in ascending lexicographic order is cut into slices of
// `rows_per_tile` consecutive rows (the paper's lexicographically bounded
// worker slices, Section 3).  Because every row count is known from the count
// table, the bounds are exact ranks and the slices need no re-splitting: a
// slice starting at rank r0 writes rows [r0, r0 + T) of `out`.
//
// k_plan unranks each slice start into its first U coordinates plus an offset
// t0 inside the block of rows sharing them: with the count table C, the rows
// whose coordinate j is below A (the coordinates before j fixed, remainder x)
// number C[j][x] - C[j][x - A g_j], a nondecreasing function of A that is
// bisected.
//
// k_write runs a persistent grid: slice t belongs to workgroup t mod NB.  In a
// prologue each workgroup copies the packed leaf-order memo (memo.hip), the
// segment counts and class ends (when they fit) and the start states of its
// slices into LDS; its wavefronts then take the slices one at a time from an
// LDS counter, so the load balances within the workgroup while no global load
// is issued after the prologue -- only LDS traffic and the coalesced stores
// of the output.  Within a slice the first U-1
// coordinates are the outer prefix, kept lane-distributed (lane j holds a_j)
// and advanced by an odometer in ascending lex order (Alg 3.1's successor,
// mirrored).  Coordinate U-1 is spread across the 64 lanes.  Then:
//  * k = 0 (MODE 0, Alg 3.1): the last coordinate is solved by division; each
//    lane is a candidate giving 0 or 1 row; a ballot plus mbcnt gives each
//    valid lane its output row.
//  * k >= 1 (MODE 1, Alg 3.2): each lane owns the segment of rows sharing its
//    prefix, one contiguous run of the leaf-order memo of length C[U][x].  A
//    wave prefix sum of the segment lengths gives row offsets; rows are then
//    produced 64 at a time: segment starts are marked in LDS and a wave
//    prefix-max gives every row lane its segment, and each lane copies one
//    memo row.
// Rows are staged in a per-wave LDS ring and written to HBM `flush` rows at a
// time with 16-byte stores, so the global stores are fully coalesced for any
// d.  Loads and stores share one wait counter on this GPU, so a global load
// issued after stores waits for all of them to reach memory; keeping every
// load in the prologue is what lets the stores stream.
// In count-only mode no row is stored: each row's FNV-1a-64 (rank, row) hash is
// summed instead.
#include <map>
#include <mutex>

#include "zset_internal.h"

namespace zset {

namespace {

constexpr int kWriteWaves = 16;  // wavefronts per workgroup of the write pass

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return int(threadIdx.x & (kWave - 1)); }

__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }

__device__ inline uint32_t mbcnt64(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ inline uint32_t readlane_u32(uint32_t v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}

// DPP move with lanes outside the pattern reading `identity`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline uint32_t dpp_u32(uint32_t v, uint32_t identity) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(identity), int(v), CTRL, ROW_MASK, 0xf, false));
}

// Inclusive prefix max over the wave: row_shr 1/2/4/8 inside each 16-lane
// row, then row_bcast 15 and 31 across rows.
__device__ inline uint32_t wave_incl_max(uint32_t v) {
  v = max(v, dpp_u32<0x111>(v, 0u));
  v = max(v, dpp_u32<0x112>(v, 0u));
  v = max(v, dpp_u32<0x114>(v, 0u));
  v = max(v, dpp_u32<0x118>(v, 0u));
  v = max(v, dpp_u32<0x142, 0xa>(v, 0u));
  v = max(v, dpp_u32<0x143, 0xc>(v, 0u));
  return v;
}

// Inclusive prefix sum over the wave, saturated at cap (cap < 2^31).
__device__ inline uint32_t wave_incl_sum_sat(uint32_t v, uint32_t cap) {
  v = min(v + dpp_u32<0x111>(v, 0u), cap);
  v = min(v + dpp_u32<0x112>(v, 0u), cap);
  v = min(v + dpp_u32<0x114>(v, 0u), cap);
  v = min(v + dpp_u32<0x118>(v, 0u), cap);
  v = min(v + dpp_u32<0x142, 0xa>(v, 0u), cap);
  v = min(v + dpp_u32<0x143, 0xc>(v, 0u), cap);
  return v;
}

// Slice start: first U coordinates and the offset t0 inside their block.
__device__ inline void plan_tile(const EnumParams& P, uint64_t tile, uint64_t T) {
  const uint64_t N = P.table_stride;
  uint64_t r = tile * T;
  uint32_t x = P.n;
  uint32_t* st = P.tiles + tile * uint64_t(P.U + 2);
  for (int j = 0; j < P.U; ++j) {
    const uint64_t* Cj = P.table + uint64_t(j) * N;
    const uint32_t g = P.g.g[j];
    const uint64_t all = Cj[x];
    uint32_t lo = 0, hi = x / g;
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      const uint64_t before = all - Cj[x - uint64_t(mid) * g];
      if (before <= r) lo = mid; else hi = mid - 1;
    }
    r -= all - Cj[x - uint64_t(lo) * g];
    x -= lo * g;
    st[j] = lo;
  }
  st[P.U] = uint32_t(r);
  st[P.U + 1] = uint32_t(r >> 32);
  if (r >= P.table[uint64_t(P.U) * N + x]) set_error(P.err, kErrUnrank);
}

// The same slice start computed by one wavefront: per coordinate a_j, the
// 64 lanes test 64 evenly spaced candidates at once (rows before a_j = a is
// nondecreasing in a, so the lanes that pass form a prefix) and narrow the
// interval 64-fold per round: ceil(log64(x / g_j + 1)) dependent loads per
// coordinate instead of log2.  Lane 0 writes the U + 2 words to st.
__device__ inline void plan_tile_wave(const EnumParams& P, uint64_t tile, uint32_t* st,
                                      int lane) {
  const uint64_t N = P.table_stride;
  const int U = P.U;
  uint64_t r = tile * P.rows_per_tile;
  uint32_t x = P.n;
  for (int j = 0; j < U; ++j) {
    const uint64_t* Cj = P.table + uint64_t(j) * N;
    const uint32_t g = P.g.g[j];
    const uint64_t all = Cj[x];
    uint32_t lo = 0, hi = x / g;  // the answer lies in [lo, hi]; lo passes
    while (lo < hi) {
      const uint32_t step = (hi - lo + 63) / 64;
      const uint64_t a = uint64_t(lo) + uint64_t(lane + 1) * step;
      const bool pass = a <= hi && all - Cj[x - a * g] <= r;
      const uint32_t t = uint32_t(__popcll(ballot64(pass)));
      const uint64_t fail_a = uint64_t(lo) + uint64_t(t + 1) * step;
      hi = fail_a <= hi ? uint32_t(fail_a - 1) : hi;
      lo += t * step;
    }
    r -= all - Cj[x - uint64_t(lo) * g];
    x -= lo * g;
    if (lane == 0) st[j] = lo;
  }
  if (lane == 0) {
    st[U] = uint32_t(r);
    st[U + 1] = uint32_t(r >> 32);
    if (r >= P.table[uint64_t(U) * N + x]) set_error(P.err, kErrUnrank);
  }
}

__device__ inline void plan_slice(const EnumParams& P, uint64_t tile) {
  if (tile == 0) {
    if (P.pool) *P.pool = 0;  // the write pass's chunk counter
    if (P.reset_status) {     // a query of its own: status words start clear
      *P.err = 0;
      *P.checksum = 0;
      if (P.blocks_done) *P.blocks_done = 0;
    }
  }
  uint64_t T = P.rows_per_tile, ntiles = P.ntiles;
  if (P.total_dev) {  // sized on the device from |Z(n)|
    const DynSize z = dyn_size(P);
    T = z.T;
    ntiles = z.ntiles;
    if (tile == 0 && z.err) set_error(P.err, z.err);
  }
  if (tile >= ntiles) return;
  plan_tile(P, tile, T);
}

__global__ __launch_bounds__(256) void k_plan(EnumParams P) {
  plan_slice(P, uint64_t(blockIdx.x) * 256 + threadIdx.x);
}

// The device-sized planner (workgroups below plan_blocks) and the memo's leaf
// layout (the others) in one grid: both read only the count table, the class
// ends and the natural-order memo, and neither waits for the other.
__global__ __launch_bounds__(256) void k_plan_leaf(EnumParams P, LeafJob J,
                                                   uint32_t plan_blocks) {
  if (blockIdx.x < plan_blocks) {
    plan_slice(P, uint64_t(blockIdx.x) * 256 + threadIdx.x);
    return;
  }
  memo_leaf_row(J, uint64_t(blockIdx.x - plan_blocks) * 256 + threadIdx.x, P.err);
}

// Batched: global slice index -> (query, slice) by bisection of the slice
// bases of the queries that have slices (tile_base[i] = slices of the queries
// plan_q[0..i-1], strictly increasing).
__global__ __launch_bounds__(256) void k_plan_batch(const EnumParams* __restrict__ qp,
                                                    const uint64_t* __restrict__ tile_base,
                                                    const uint32_t* __restrict__ plan_q,
                                                    uint32_t nplan, uint64_t total_tiles) {
  const uint64_t t = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= total_tiles) return;
  uint32_t lo = 0, hi = nplan - 1;  // last entry whose base <= t
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (tile_base[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const EnumParams& Q = qp[plan_q[lo]];
  plan_tile(Q, t - tile_base[lo], Q.rows_per_tile);
}

// Output rows are written once and never read back by the kernel: the stores
// are non-temporal (streaming), which measured 2.5% faster on the write pass.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <bool ALIGN16>
__device__ inline void flush_rows(const uint32_t* ring, uint32_t slot0, uint32_t rows, int d,
                                  uint32_t* out_rows) {
  const uint32_t nd = rows * uint32_t(d);
  const uint32_t* src = ring + slot0 * uint32_t(d);
  const int lane = lane_id();
  if (ALIGN16) {
    const uint32_t nd4 = nd & ~3u;
    for (uint32_t v = uint32_t(lane) * 4; v < nd4; v += kWave * 4) {
      const u32x4 val = *reinterpret_cast<const u32x4*>(src + v);
      __builtin_nontemporal_store(val, reinterpret_cast<u32x4*>(out_rows + v));
    }
    for (uint32_t v = nd4 + lane; v < nd; v += kWave) __builtin_nontemporal_store(src[v], out_rows + v);
  } else {
    for (uint32_t v = lane; v < nd; v += kWave) __builtin_nontemporal_store(src[v], out_rows + v);
  }
}

// Descending output: `rows` staged rows (ascending) written as one block in
// reverse row order, one word per lane per store (coalesced; the block's
// start need not be 16-byte aligned).  Row of word v: v / d by a multiply and
// shift, exact for v < 2^12 (at most 128 rows of at most 32 words).
__device__ inline void flush_rows_rev(const uint32_t* ring, uint32_t slot0, uint32_t rows, int d,
                                      uint32_t* out_rows) {
  const uint32_t nd = rows * uint32_t(d);
  const uint32_t* src = ring + slot0 * uint32_t(d);
  const uint32_t m = (1u << 20) / uint32_t(d) + 1u;
  for (uint32_t v = uint32_t(lane_id()); v < nd; v += kWave) {
    const uint32_t row = (v * m) >> 20;
    const uint32_t col = v - row * uint32_t(d);
    __builtin_nontemporal_store(src[(rows - 1 - row) * uint32_t(d) + col], out_rows + v);
  }
}

// Memo row access: PACK 1 = one packed 32-bit word in LDS, PACK 2 = one packed
// 64-bit word in LDS, PACK 0 = k+1 plain words in global memory.  Field c is
// (word >> shift_c) & mask_c; shifts and masks live in lanes 0..k of fsh/fmk.
template <int PACK>
struct MemoRow {
  uint64_t w;
  const uint32_t* g;
  __device__ inline void load(const uint32_t* lds_memo, const uint32_t* leaf, uint64_t row,
                              int k) {
    if (PACK == 1) {
      w = lds_memo[row];
    } else if (PACK == 2) {
      w = reinterpret_cast<const uint64_t*>(lds_memo)[row];
    } else {
      g = leaf + row * uint64_t(k + 1);
    }
  }
  __device__ inline uint32_t field(uint32_t fsh, uint32_t fmk, int c) const {
    if (PACK == 0) return g[c];
    return uint32_t(w >> readlane_u32(fsh, c)) & readlane_u32(fmk, c);
  }
};

__host__ __device__ inline uint64_t align4(uint64_t words) { return (words + 3) & ~uint64_t(3); }

// LDS words of one workgroup of the write pass: packed memo, segment counts and
// class ends (LDSCNT), the start states of the workgroup's slices, then per
// wavefront its staging ring and 64 marks.
__host__ __device__ inline uint64_t write_wave_words(const EnumParams& P) {
  return uint64_t(P.ring) * P.d + kWave + (P.chunk ? align4(uint64_t(P.U) + 2) : 0);
}
// Claimed chunks pass through a ring of kChunkSlots LDS slots: per slot a
// flag, the global chunk index and a count of wavefronts done reading it, then
// the start states of the chunk's slices.
constexpr uint32_t kChunkSlots = 4;
__host__ __device__ inline uint64_t claim_words(const EnumParams& P) {
  if (P.chunk == 0) return 0;
  return 4 * kChunkSlots + align4(uint64_t(kChunkSlots) * P.chunk * (P.U + 2));
}
__host__ __device__ inline uint64_t write_shared_words(const EnumParams& P) {
  uint64_t w = align4(P.memo_words);
  if (P.lds_cnt) w += align4(uint64_t(P.n) + 1) + align4(P.nclass);
  w += align4(uint64_t(P.max_tiles) * (P.U + 2));
  w += claim_words(P);
  return w;
}

// The per-query scalars one slice needs, held in scalar registers: the
// single-query kernel fills them from its kernel arguments, the batched kernel
// from the query's descriptor.
struct TileArgs {
  uint32_t n, d, U, k;
  uint32_t gseg;               // g_{U-1} (U >= 1): step of the lane coordinate
  uint32_t gpre;               // g_{U-2} (pair lanes)
  int pair;                    // 1: lanes range over (a_{U-2}, a_{U-1}) pairs
  int desc;                    // 1: rows stored in descending order
  uint32_t top;                // memo covers p < top; top <= n: partial memo (Else branch)
  uint32_t nclass;             // residue classes of the leaf layout (with rows below top)
  const uint64_t* table;       // count table (rows U.. unrank the head rows of a partial memo)
  uint64_t table_stride;
  uint32_t ring, flush;        // staging ring rows (power of two), rows per flush
  uint64_t total;              // |Z(n)|
  uint64_t rows_per_tile;      // slice length
  const uint64_t* cnt_row;     // count-table row U: C[U][x]
  const uint64_t* endc;        // residue-class ends of the leaf-order memo
  const uint32_t* leaf;        // leaf-order memo rows
  uint64_t leaf_rows;
  uint32_t* out;               // first row of this query
  int* err;
  DivMod32 dG;                 // division by g_U
  DivMod32 dG1;                // division by g_{U-1} (pair lanes)
};

__device__ inline TileArgs tile_args(const EnumParams& P) {
  TileArgs A;
  A.n = P.n;
  A.d = uint32_t(P.d);
  A.U = uint32_t(P.U);
  A.k = uint32_t(P.k);
  A.gseg = P.U >= 1 ? P.g.g[P.U - 1] : 0;
  A.gpre = P.U >= 2 ? P.g.g[P.U - 2] : 0;
  A.pair = P.pair;
  A.desc = P.desc;
  A.top = P.memo_top ? P.memo_top : P.n + 1;
  A.nclass = P.nclass;
  A.table = P.table;
  A.table_stride = P.table_stride;
  A.dG1 = P.dG1;
  A.ring = P.ring;
  A.flush = P.flush;
  A.total = P.total;
  A.rows_per_tile = P.rows_per_tile;
  A.cnt_row = P.table + uint64_t(P.U) * P.table_stride;
  A.endc = P.endc;
  A.leaf = P.leaf;
  A.leaf_rows = P.leaf_rows;
  A.out = P.out;
  A.err = P.err;
  A.dG = P.dG;
  return A;
}

// Row t (ascending) of Z(x; g_U, .., g_{d-1}), for a row that the memo does
// not hold (a partial memo, the Else branch of Alg 3.2): coordinates U..d-2
// by bisection of the count table's rows (the rows before a_j = a number
// C_j[x] - C_j[x - a g_j]), the last one by division.  put(j, a_j) is called
// in coordinate order.  Lane j of gj holds g_j.
template <class F>
__device__ inline void unrank_suffix(const TileArgs& P, uint32_t gj, int U, int d, uint32_t x,
                                     uint64_t t, F&& put) {
  for (int j = U; j < d - 1; ++j) {
    const uint32_t g = readlane_u32(gj, j);
    const uint64_t* Cj = P.table + uint64_t(j) * P.table_stride;
    const uint64_t all = Cj[x];
    uint32_t lo = 0, hi = x / g;
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      if (all - Cj[x - mid * g] <= t) lo = mid; else hi = mid - 1;
    }
    t -= all - Cj[x - lo * g];
    x -= lo * g;
    put(j, lo);
  }
  put(d - 1, x / readlane_u32(gj, d - 1));
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  const uint32_t lo = __shfl(uint32_t(v), src, kWave), hi = __shfl(uint32_t(v >> 32), src, kWave);
  return (uint64_t(hi) << 32) | lo;
}

// One slice: rows [tile * T, tile * T + target) of the query, starting from
// the slice start `st` (first U coordinates and t0).  Shared by the
// single-query and the batched write kernels.  NO >= 0 and KF >= 1 fix the
// outer-prefix length (U - 1) and k at compile time, so that a row is
// assembled with no loop and with the prefix and field shifts held in scalar
// registers; -1 leaves them to run time, and kNoPartial (generic row
// assembly too) also serves a partial memo, whose head rows are unranked from
// the count table: a separate instantiation, so that the others carry none of
// its registers.
constexpr int kNoPartial = -2;
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO = -1, int KF = -1>
__device__ inline void write_tile(const TileArgs& P, uint64_t tile, const uint32_t* st,
                                  uint32_t* ring, uint32_t* marks, const uint32_t* lds_memo,
                                  const uint32_t* lds_cnt, const uint32_t* lds_endc, uint32_t gj,
                                  uint32_t fsh, uint32_t fmk, uint64_t& csum) {
  const int lane = lane_id();
  const int d = int(P.d), U = int(P.U), k = int(P.k);
  const uint32_t ring_mask = P.ring - 1;
  const uint32_t flush_rows_n = P.flush;
  // A batch or chunk yields up to 64 rows; with flush + 64 <= ring they are
  // staged at once, else in two halves with a flush check between them.
  const uint32_t nphase = (P.flush + uint32_t(kWave) <= P.ring) ? 1u : 2u;
  const uint32_t phase_rows = uint32_t(kWave) / nphase;
  // Pair lanes (MODE 1, U >= 2): the lanes range over the pairs (a_{U-2},
  // a_{U-1}) of the current outer prefix in lex order, 64 pairs per step, so
  // that a step covers 64 segments even when a_{U-1} alone takes few values.
  const bool pair = MODE == 1 && NO < 0 && P.pair && U >= 2;  // generic row assembly only
  // Partial memo (generic row assembly only): the memo covers p < top <= n.
  const bool partial = MODE == 1 && NO == kNoPartial && P.top <= P.n;
  // Coordinates 0..nouter-1 form the outer prefix.
  const int nouter = pair ? U - 2 : (U >= 1 ? U - 1 : 0);
  const uint32_t gseg = P.gseg;
  const uint32_t gpre = P.gpre;
  const uint64_t* cnt_row = P.cnt_row;
  const uint64_t r0 = tile * P.rows_per_tile;
  const uint64_t left = P.total - r0;
  const uint32_t target = uint32_t(left < P.rows_per_tile ? left : P.rows_per_tile);

  // Slice start, lane-distributed: lane j < U holds a_j and the remainder
  // after coordinate j.
  uint32_t aj = lane < U ? st[lane] : 0;
  const uint64_t t0 = uint64_t(st[U]) | (uint64_t(st[U + 1]) << 32);
  uint32_t remj;
  {
    uint32_t ps = lane < U ? aj * gj : 0;  // every partial sum is <= n
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(ps, off, kWave);
      if (lane >= off) ps += y;
    }
    remj = P.n - ps;
  }
  // Remainder after the outer prefix; first lane-coordinate value (or pair).
  uint32_t xouter = nouter >= 1 ? readlane_u32(remj, nouter - 1) : P.n;
  uint32_t aseg = (U >= 1) ? readlane_u32(aj, U - 1) : 0;
  uint32_t tc = pair ? readlane_u32(aj, U - 2) : 0;  // pair of the step's first lane

  constexpr bool kSpec = NO >= 0 && KF >= 1;
  uint32_t hsh[kSpec ? KF + 1 : 1], hmk[kSpec ? KF + 1 : 1];
  if constexpr (kSpec) {
#pragma unroll
    for (int c2 = 0; c2 <= KF; ++c2) {
      hsh[c2] = readlane_u32(fsh, c2);
      hmk[c2] = readlane_u32(fmk, c2);
    }
  }
  uint32_t produced = 0, flushed = 0;
  bool first = true;
  bool single_done = false;
  uint32_t* out_tile = P.out + r0 * uint64_t(d);
  // Staged rows [f, f + rows) of the slice go to ranks r0 + f ..; in
  // descending order the rank r is stored at row total - 1 - r, so the block
  // starts at row total - r0 - f - rows and is written in reverse.
  auto emit = [&](uint32_t slot0, uint32_t rows, uint32_t f) {
    if (P.desc)
      flush_rows_rev(ring, slot0, rows, d, P.out + (P.total - r0 - f - rows) * uint64_t(d));
    else
      flush_rows<ALIGN16>(ring, slot0, rows, d, out_tile + uint64_t(f) * d);
  };

  while (produced < target) {
    const uint32_t remaining = target - produced;
    uint32_t hpre[kSpec && NO > 0 ? NO : 1];
    if constexpr (kSpec) {
#pragma unroll
      for (int j = 0; j < NO; ++j) hpre[j] = readlane_u32(aj, j);
    }
    const uint32_t A = aseg + uint32_t(lane);
    bool ok;
    uint32_t xs;
    uint32_t pt = 0, pa = 0, npairs = 0;  // pair lanes: this lane's (a_{U-2}, a_{U-1})
    if (pair) {
      // Row j of the pair space holds a_{U-2} = tc + j and a_{U-1} in
      // [0, (xouter - a_{U-2} g_{U-2}) / g_{U-1}] (row 0 from aseg on); the
      // rows' first lanes are marked and a wave prefix max gives each lane
      // its row.
      const uint32_t tj = tc + uint32_t(lane);
      const uint64_t tg = uint64_t(tj) * gpre;
      uint32_t cnt = tg <= xouter ? P.dG1.div(xouter - uint32_t(tg)) + 1 : 0;
      if (lane == 0) cnt -= aseg;  // aseg <= the row's last value (a valid pair)
      cnt = cnt < uint32_t(kWave) ? cnt : uint32_t(kWave);
      const uint32_t cincl = wave_incl_sum_sat(cnt, 1u << 30);
      const uint32_t cst = cincl - cnt;
      const uint32_t call = readlane_u32(cincl, kWave - 1);
      npairs = call < uint32_t(kWave) ? call : uint32_t(kWave);
      marks[lane] = 0;
      wave_sync();
      if (cnt != 0 && cst < uint32_t(kWave)) marks[cst] = lane + 1;
      wave_sync();
      const int r = int(wave_incl_max(marks[lane])) - 1;  // row 0 starts at lane 0
      const uint32_t o_cst = __shfl(cst, r, kWave);
      pt = tc + uint32_t(r);
      pa = uint32_t(lane) - o_cst + (r == 0 ? aseg : 0u);
      ok = uint32_t(lane) < npairs;
      xs = ok ? xouter - pt * gpre - pa * gseg : 0;
      wave_sync();
    } else if (U >= 1) {
      const uint64_t ag = uint64_t(A) * gseg;
      ok = ag <= xouter;
      xs = ok ? xouter - uint32_t(ag) : 0;
    } else {
      ok = (lane == 0) && !single_done;
      xs = P.n;
    }
    const uint32_t qx = P.dG.div(xs);
    uint32_t tot;

    if (MODE == 0) {
      const bool valid = ok && (P.dG.mod(xs, qx) == 0);
      const uint64_t mask = ballot64(valid);
      const uint32_t pos = mbcnt64(mask);
      const uint32_t cnt = uint32_t(__popcll((unsigned long long)mask));
      tot = cnt < remaining ? cnt : remaining;
      if (COUNT_ONLY) {
        if (valid && pos < tot) {
          uint64_t h = fnv1a_u64(kFnvOffset, r0 + produced + pos);
          for (int j = 0; j < nouter; ++j) h = fnv1a_u32(h, readlane_u32(aj, j));
          h = fnv1a_u32(h, A);
          h = fnv1a_u32(h, qx);
          csum += h;
        }
      } else {
        // Staged in `nphase` parts so that the ring never holds more than
        // flush + 64 / nphase unflushed rows.
        for (uint32_t ph = 0; ph < nphase; ++ph) {
          const uint32_t plo = ph * phase_rows, phi = plo + phase_rows;
          if (valid && pos < tot && pos >= plo && pos < phi) {
            uint32_t* row = ring + ((produced + pos) & ring_mask) * uint32_t(d);
            for (int j = 0; j < nouter; ++j) row[j] = readlane_u32(aj, j);
            row[U - 1] = A;
            row[U] = qx;
          }
          wave_sync();
          const uint32_t written = produced + (tot < phi ? tot : phi);
          while (written - flushed >= flush_rows_n) {
            emit(flushed & ring_mask, flush_rows_n, flushed);
            flushed += flush_rows_n;
          }
          wave_sync();
        }
      }
    } else {
      const uint32_t rx = P.dG.mod(xs, qx);
      uint64_t c, start;
      // Class ends of rx and rx - 1 (a partial memo has classes only below top).
      const bool inc = ok && rx < P.nclass;
      uint64_t ec = 0, ep = 0;
      if (LDSCNT) {
        const uint32_t c32v = ok ? lds_cnt[xs] : 0;
        c = c32v;
        ec = inc ? lds_endc[rx] : 0;
        if (partial && inc && rx) ep = lds_endc[rx - 1];
      } else {
        c = ok ? cnt_row[xs] : 0;
        ec = inc ? P.endc[rx] : 0;
        if (partial && inc && rx) ep = P.endc[rx - 1];
      }
      start = ok ? ec - c : 0;
      // Partial memo: a segment with x >= top begins with the rows whose memo
      // remainder x - a_U G is >= top (the smallest a_U), which the memo does
      // not hold; the rest of it is the whole memo class of x mod G.  hcnt =
      // the head's rows; tb + rho = a batch row's index in its segment.
      const uint64_t hcnt = (partial && ok && xs >= P.top) ? c - (inc ? ec - ep : 0) : 0;
      uint64_t t_adj = 0;
      if (first && lane == 0) {
        if (t0 >= c) {  // the plan guarantees t0 < c; refuse to read past the segment
          set_error(P.err, kErrUnrank);
          c = 0;
        } else {
          start += t0;
          c -= t0;
          t_adj = t0;
        }
      }
      const uint32_t c32 = uint32_t(c < remaining ? c : remaining);
      const uint32_t incl = wave_incl_sum_sat(c32, remaining);
      const uint32_t up = __shfl_up(incl, 1, kWave);
      const uint32_t excl = lane ? up : 0;
      tot = readlane_u32(incl, kWave - 1);
      // Memo row of batch row rho is segbase[owner] + rho (wrapping arithmetic).
      const uint64_t segbase = start - excl;
      const uint64_t tb = t_adj - excl;
      const uint32_t seg_lo = uint32_t(segbase), seg_hi = uint32_t(segbase >> 32);
      uint32_t carry = 0;  // 1 + segment lane of the row just before this chunk
      for (uint32_t beta = 0; beta < tot; beta += kWave) {
        const uint32_t rho = beta + uint32_t(lane);
        const bool act = rho < tot;
        marks[lane] = 0;
        wave_sync();
        if (c32 != 0 && excl >= beta && excl - beta < uint32_t(kWave)) marks[excl - beta] = lane + 1;
        wave_sync();
        uint32_t m = wave_incl_max(marks[lane]);
        m = max(m, carry);
        carry = readlane_u32(m, kWave - 1);
        const int owner = int(m) - 1;  // >= 0: row 0 of a batch always starts a segment
        const uint32_t o_lo = __shfl(seg_lo, owner, kWave);
        const uint32_t o_qx = __shfl(qx, owner, kWave);
        uint64_t mrow;
        if (PACK == 0) {
          const uint32_t o_hi = __shfl(seg_hi, owner, kWave);
          mrow = ((uint64_t(o_hi) << 32) | o_lo) + rho;
        } else {
          mrow = uint32_t(o_lo + rho);
        }
        const uint32_t o_A = pair ? __shfl(pa, owner, kWave) : aseg + uint32_t(owner);
        const uint32_t o_T = pair ? __shfl(pt, owner, kWave) : 0u;
        bool head = false;  // partial memo: a row before its segment's memo class
        uint64_t t_seg = 0;
        uint32_t o_xs = 0;
        if (partial) {
          t_seg = shfl_u64(tb, owner) + rho;
          o_xs = __shfl(xs, owner, kWave);
          // Every lane reads the owner's head count (outside the `act` test):
          // a cross-lane read from an inactive lane returns 0, and the owner
          // of an active row can be a lane past the chunk's last row.
          const uint64_t o_hcnt = shfl_u64(hcnt, owner);
          head = act && t_seg < o_hcnt;
        }
        const bool bad = act && !head && mrow >= P.leaf_rows;
        if (bad) set_error(P.err, kErrTileRows);
        const bool live = act && !bad && !head;
        MemoRow<PACK> mr;
        uint32_t aU = 0;
        if (live) {
          mr.load(lds_memo, P.leaf, mrow, k);
          uint32_t f0;
          if constexpr (kSpec) f0 = uint32_t(mr.w >> hsh[0]) & hmk[0];
          else f0 = mr.field(fsh, fmk, 0);
          aU = o_qx - f0;
        }
        if (COUNT_ONLY) {
          if (live) {
            uint64_t h = fnv1a_u64(kFnvOffset, r0 + produced + rho);
            for (int j = 0; j < nouter; ++j) h = fnv1a_u32(h, readlane_u32(aj, j));
            if (pair) h = fnv1a_u32(h, o_T);
            if (U >= 1) h = fnv1a_u32(h, o_A);
            h = fnv1a_u32(h, aU);
            for (int c2 = 1; c2 <= k; ++c2) h = fnv1a_u32(h, mr.field(fsh, fmk, c2));
            csum += h;
          }
          if (head) {
            uint64_t h = fnv1a_u64(kFnvOffset, r0 + produced + rho);
            for (int j = 0; j < nouter; ++j) h = fnv1a_u32(h, readlane_u32(aj, j));
            if (pair) h = fnv1a_u32(h, o_T);
            if (U >= 1) h = fnv1a_u32(h, o_A);
            unrank_suffix(P, gj, U, d, o_xs, t_seg, [&](int, uint32_t v) { h = fnv1a_u32(h, v); });
            csum += h;
          }
          wave_sync();
        } else {
          const uint32_t nrows = (tot - beta) < uint32_t(kWave) ? (tot - beta) : uint32_t(kWave);
          for (uint32_t ph = 0; ph < nphase; ++ph) {
            const uint32_t plo = ph * phase_rows, phi = plo + phase_rows;
            if (live && uint32_t(lane) >= plo && uint32_t(lane) < phi) {
              if constexpr (kSpec) {
                constexpr uint32_t kD = uint32_t(NO + 2 + KF);
                uint32_t* row = ring + ((produced + rho) & ring_mask) * kD;
#pragma unroll
                for (int j = 0; j < NO; ++j) row[j] = hpre[j];
                row[NO] = o_A;
                row[NO + 1] = aU;
#pragma unroll
                for (int c2 = 1; c2 <= KF; ++c2)
                  row[NO + 1 + c2] = uint32_t(mr.w >> hsh[c2]) & hmk[c2];
              } else {
                uint32_t* row = ring + ((produced + rho) & ring_mask) * uint32_t(d);
                for (int j = 0; j < nouter; ++j) row[j] = readlane_u32(aj, j);
                if (pair) row[U - 2] = o_T;
                if (U >= 1) row[U - 1] = o_A;
                row[U] = aU;
                for (int c2 = 1; c2 <= k; ++c2) row[U + c2] = mr.field(fsh, fmk, c2);
              }
            }
            if (head && uint32_t(lane) >= plo && uint32_t(lane) < phi) {
              uint32_t* row = ring + ((produced + rho) & ring_mask) * uint32_t(d);
              for (int j = 0; j < nouter; ++j) row[j] = readlane_u32(aj, j);
              if (pair) row[U - 2] = o_T;
              if (U >= 1) row[U - 1] = o_A;
              unrank_suffix(P, gj, U, d, o_xs, t_seg, [&](int j, uint32_t v) { row[j] = v; });
            }
            wave_sync();
            const uint32_t written = produced + beta + (nrows < phi ? nrows : phi);
            while (written - flushed >= flush_rows_n) {
              emit(flushed & ring_mask, flush_rows_n, flushed);
              flushed += flush_rows_n;
            }
            wave_sync();
          }
        }
      }
    }

    produced += tot;
    if (produced >= target) break;
    first = false;
    if (U == 0) {
      if (single_done) break;
      single_done = true;
      continue;
    }
    if (pair) {
      if (npairs == uint32_t(kWave)) {  // step past lane 63's pair
        const uint32_t t63 = readlane_u32(pt, kWave - 1), a63 = readlane_u32(pa, kWave - 1);
        if (a63 < P.dG1.div(xouter - t63 * gpre)) {
          tc = t63;
          aseg = a63 + 1;
          continue;
        }
        if (uint64_t(t63 + 1) * gpre <= xouter) {
          tc = t63 + 1;
          aseg = 0;
          continue;
        }
      }
    } else if (uint64_t(aseg + kWave) * gseg <= xouter) {
      aseg += kWave;
      continue;
    }
    // Odometer: the rightmost outer coordinate that can still grow.
    const bool can = lane < nouter && remj >= gj;
    const uint64_t mask = ballot64(can);
    if (mask == 0) {
      if (lane == 0) set_error(P.err, kErrOdometer);
      break;
    }
    const int js = 63 - __clzll((unsigned long long)mask);
    if (lane == js) {
      aj += 1;
      remj -= gj;
    }
    const uint32_t nrem = readlane_u32(remj, js);
    if (lane > js && lane < nouter) {
      aj = 0;
      remj = nrem;
    }
    xouter = nrem;
    aseg = 0;
    tc = 0;
  }

  if (!COUNT_ONLY && produced > flushed) {
    emit(flushed & ring_mask, produced - flushed, flushed);
  }
  wave_sync();
  if (lane == 0 && produced != target) set_error(P.err, kErrTileRows);
}

// LDS words of the chunk ring: wait until a word holds v; publish a word after
// every LDS write of the wavefront before it.
__device__ inline void wait_word(uint32_t* f, uint32_t v) {
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != v)
    __builtin_amdgcn_s_sleep(2);
}
__device__ inline void publish_flag(uint32_t* f, uint32_t v, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  wave_sync();
  if (lane == 0) __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Memo rows read from global memory (PACK 0, generic row assembly): such a
// load waits for every store the wavefront has issued before it (one counter
// for both), so these kernels are held to 64 VGPRs for 8 wavefronts per SIMD:
// two workgroups per compute unit when LDS allows, twice the wavefronts to
// cover the waits.
template <int MODE, int PACK, int NO>
constexpr int write_waves_per_simd() { return (PACK == 0 && NO == -1) ? 8 : 1; }

template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
__global__ __launch_bounds__(kWriteWaves * kWave, (write_waves_per_simd<MODE, PACK, NO>()))
void k_write(EnumParams P) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int lane = lane_id();
  const int wave = int(threadIdx.x / kWave);
  const int d = P.d, U = P.U, k = P.k;
  const uint64_t N = uint64_t(P.n) + 1;
  const uint32_t ring_rows = P.ring;
  const uint32_t S = uint32_t(U + 2);  // words of one slice start

  // ---- Prologue: every global load of the kernel happens here, before the
  // first store (a load issued after stores would wait for all of them).
  const uint32_t* lds_memo = lds;
  uint32_t* lds_cnt = lds + align4(P.memo_words);
  uint32_t* lds_endc = lds_cnt + align4(N);
  if (MODE == 1 && PACK > 0) {
    const uint64_t nvec = P.memo_words / 4;
    const uint4* src = reinterpret_cast<const uint4*>(P.leaf);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    const uint64_t stride = blockDim.x;
    uint64_t i = threadIdx.x;
    for (; i + 3 * stride < nvec; i += 4 * stride) {
      const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], e = src[i + 3 * stride];
      dst[i] = a;
      dst[i + stride] = b;
      dst[i + 2 * stride] = c;
      dst[i + 3 * stride] = e;
    }
    for (; i < nvec; i += stride) dst[i] = src[i];
    for (uint64_t w = nvec * 4 + threadIdx.x; w < P.memo_words; w += stride) lds[w] = P.leaf[w];
  }
  if (MODE == 1 && LDSCNT) {
    // Values fit 32 bits (checked by the host).
    const uint64_t* cu = P.table + uint64_t(U) * P.table_stride;
    for (uint64_t x = threadIdx.x; x < N; x += blockDim.x) lds_cnt[x] = uint32_t(cu[x]);
    for (uint32_t r = threadIdx.x; r < P.nclass; r += blockDim.x) lds_endc[r] = uint32_t(P.endc[r]);
  }
  // Slices of this workgroup: blockIdx.x, + gridDim.x, + 2 gridDim.x, ...  Their
  // start states go to LDS; the wavefronts take them in turn from an LDS counter.
  uint32_t* tstates =
      lds + align4(P.memo_words) + (P.lds_cnt ? align4(N) + align4(P.nclass) : 0);
  uint32_t* wbase = lds + write_shared_words(P) + size_t(wave) * write_wave_words(P);
  uint32_t* ring = wbase;  // 16-byte aligned: every region above is a multiple of 4 words
  uint32_t* marks = ring + ring_rows * d;
  __shared__ uint32_t next_slot, first_chunk;
  const uint64_t B = blockIdx.x, NB = gridDim.x;
  const uint64_t nstatic = P.static_tiles;
  // Slices sized on the device (P.dyn): |Z(n)|, the slice length and count
  // as the planner took them; every slice is claimed (nstatic = 0).
  uint64_t ntiles = P.ntiles, dyn_total = P.total, dyn_T = P.rows_per_tile;
  if (P.dyn) {
    const DynSize z = dyn_size(P);
    ntiles = z.ntiles;
    dyn_total = z.total;
    dyn_T = z.T;
  }
  uint32_t my_tiles = B < nstatic ? uint32_t((nstatic - B + NB - 1) / NB) : 0;
  if (my_tiles > P.max_tiles) {  // the host sizes the grid so that this cannot happen
    if (threadIdx.x == 0) set_error(P.err, kErrTileRows);
    my_tiles = 0;
  }
  if (P.tiles) {
    for (uint32_t i = threadIdx.x; i < my_tiles * S; i += blockDim.x) {
      const uint32_t t = i / S, w = i - t * S;
      tstates[i] = P.tiles[(B + uint64_t(t) * NB) * S + w];
    }
  } else {
    // No slice table: the wavefronts compute the starts of the workgroup's
    // slices themselves (every slice is dealt; the host sets chunk = 0).
    const uint32_t nw = blockDim.x / kWave;
    for (uint32_t t = uint32_t(wave); t < my_tiles; t += nw)
      plan_tile_wave(P, B + uint64_t(t) * NB, tstates + t * S, lane);
  }
  // Claimed slices (nstatic.. ntiles-1, in chunks of CH consecutive slices
  // taken from a global counter, from the end of the order backwards: the last
  // slices, whose outer prefixes hold few rows each and so cost the most per
  // row, start first and the pass ends on cheap ones; chunk g holds slices
  // [hi - cnt, hi) with hi = ntiles - g CH, its e-th taker gets slice
  // hi - 1 - e).  The workgroup's c-th chunk goes through
  // ring slot c mod R: cflag = c + 1 once published, cgid = global chunk
  // index (nchunks when the counter is exhausted), cdone = wavefronts that
  // have copied their slice start out of the slot (CH when the slot is free).
  // The first chunk is claimed here, before any store; chunk c + 1 by the
  // wavefront that takes the first slice of chunk c, so a claim (whose wait
  // covers that wavefront's pending stores) is paid once per CH slices and
  // lands about CH slices ahead of use.
  const uint32_t CH = P.chunk;
  constexpr uint32_t R = kChunkSlots;
  const uint32_t nchunks = CH ? uint32_t((ntiles - nstatic + CH - 1) / CH) : 0;
  uint32_t* cflag = tstates + align4(uint64_t(P.max_tiles) * S);
  uint32_t* cgid = cflag + R;
  uint32_t* cdone = cgid + R;
  uint32_t* cstate = cdone + 2 * R;
  uint32_t* mystate = marks + kWave;
  if (CH) {
    if (threadIdx.x == 0) first_chunk = atomicAdd(P.pool, 1u);
    __syncthreads();
    const uint32_t gc = min(first_chunk, nchunks);
    if (gc < nchunks) {
      const uint64_t hi = ntiles - uint64_t(gc) * CH;
      const uint32_t cnt = uint32_t(min<uint64_t>(CH, hi - nstatic));
      const uint64_t t0 = hi - cnt;
      for (uint32_t i = threadIdx.x; i < cnt * S; i += blockDim.x) cstate[i] = P.tiles[t0 * S + i];
    }
    if (threadIdx.x < R) {
      cflag[threadIdx.x] = threadIdx.x == 0 ? 1 : 0;
      cgid[threadIdx.x] = threadIdx.x == 0 ? gc : 0;
      cdone[threadIdx.x] = threadIdx.x == 0 ? 0 : CH;
    }
  }
  if (threadIdx.x == 0) next_slot = 0;
  const uint32_t gj = lane < d ? P.g.g[lane] : 0;
  const uint32_t fsh = lane <= k ? P.fshift[lane] : 0;
  const uint32_t fmk = lane <= k ? P.fmask[lane] : 0;
  TileArgs A = tile_args(P);
  A.total = dyn_total;
  A.rows_per_tile = dyn_T;
  __syncthreads();

  uint64_t csum = 0;

  for (;;) {
    uint32_t slot_l = 0;
    if (lane == 0) slot_l = atomicAdd(&next_slot, 1u);
    const uint32_t ti = __builtin_amdgcn_readfirstlane(slot_l);
    if (ti < my_tiles) {
      const uint64_t tile = B + uint64_t(ti) * NB;
      write_tile<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(A, tile, tstates + ti * S, ring,
                                                                  marks, lds_memo, lds_cnt,
                                                                  lds_endc, gj, fsh, fmk, csum);
      continue;
    }
    if (CH == 0) break;
    const uint32_t dj = ti - my_tiles, c = dj / CH, e = dj - c * CH, r = c % R;
    // Chunk c is published by the taker of the first slice of chunk c - 1 (or
    // the prologue), taken earlier; that taker waits only on readers of chunk
    // c - R, taken earlier still, who wait on nothing after their copy: every
    // wait ends.
    wait_word(cflag + r, c + 1);
    const uint32_t gc = cgid[r];
    const uint64_t hi = gc < nchunks ? ntiles - uint64_t(gc) * CH : nstatic;
    const uint32_t cnt = uint32_t(min<uint64_t>(CH, hi - nstatic));
    const bool live = e < cnt;  // the chunk claimed last may be short
    const uint64_t tile = hi - 1 - e;
    if (live && lane < int(S)) mystate[lane] = cstate[(r * CH + (cnt - 1 - e)) * S + lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    wave_sync();
    if (lane == 0) __hip_atomic_fetch_add(cdone + r, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (e == 0) {
      // Claim chunk c + 1 into slot c + 1 mod R once the readers of the chunk
      // it held (c + 1 - R, all of whose slices were taken before this one)
      // have copied their starts.
      const uint32_t rn = (c + 1) % R;
      wait_word(cdone + rn, CH);
      uint32_t gn = nchunks;  // an exhausted counter passes exhaustion on
      if (gc < nchunks) {
        uint32_t g_l = 0;
        if (lane == 0) g_l = atomicAdd(P.pool, 1u);
        gn = min(__builtin_amdgcn_readfirstlane(g_l), nchunks);
      }
      if (gn < nchunks) {
        const uint64_t hn = ntiles - uint64_t(gn) * CH;
        const uint32_t cn = uint32_t(min<uint64_t>(CH, hn - nstatic));
        const uint64_t t0 = hn - cn;
        uint32_t* dst = cstate + rn * CH * S;
        for (uint32_t i = lane; i < cn * S; i += kWave) dst[i] = P.tiles[t0 * S + i];
      }
      if (lane == 0) {
        cdone[rn] = 0;
        cgid[rn] = gn;
      }
      publish_flag(cflag + rn, c + 2, lane);
    }
    if (gc >= nchunks) break;
    if (!live) continue;
    write_tile<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(A, tile, mystate, ring, marks,
                                                                lds_memo, lds_cnt, lds_endc, gj,
                                                                fsh, fmk, csum);
  }

  if (COUNT_ONLY) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) csum += __shfl_xor(csum, off, kWave);
    if (lane == 0 && csum != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(P.checksum),
                static_cast<unsigned long long>(csum));
  }
  if (P.done_flag) {
    // Completion for a host that polls pinned memory: every workgroup counts
    // itself after its stores and error word (device-scope release); the
    // last one copies the status word out and then publishes the sequence
    // number at system scope.
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const uint32_t prev = atomicAdd(P.blocks_done, 1u);
      if (prev == gridDim.x - 1) {
        __threadfence();
        reinterpret_cast<volatile int*>(P.done_flag + 1)[0] =
            __hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Every workgroup has counted itself: leave the status word and the
        // counter clear for the stream's next query.
        __hip_atomic_store(P.err, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(P.blocks_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(P.done_flag, P.done_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Batched write pass: one persistent launch over the work units of many
// queries.  A workgroup takes units (slices [tile_lo, tile_hi) of one query)
// from a global counter, the largest units first; for each it copies the
// query's descriptor into LDS, runs the same prologue as k_write (packed memo,
// segment counts and class ends, slice starts), lets its wavefronts take the
// slices from an LDS counter, and records the query's completion time when
// its last slice is done.
constexpr uint32_t kDescWords = uint32_t(sizeof(EnumParams) / 4);

__device__ inline uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t rfl64(uint64_t v) {
  return (uint64_t(rfl(uint32_t(v >> 32))) << 32) | rfl(uint32_t(v));
}
template <class T>
__device__ inline T* rflp(T* p) {
  return reinterpret_cast<T*>(rfl64(reinterpret_cast<uint64_t>(p)));
}

// The descriptor fields read from LDS, made wave-uniform (scalar registers).
__device__ inline TileArgs uniform_args(const TileArgs& a) {
  TileArgs A;
  A.n = rfl(a.n);
  A.d = rfl(a.d);
  A.U = rfl(a.U);
  A.k = rfl(a.k);
  A.gseg = rfl(a.gseg);
  A.gpre = rfl(a.gpre);
  A.pair = int(rfl(uint32_t(a.pair)));
  A.desc = int(rfl(uint32_t(a.desc)));
  A.top = rfl(a.top);
  A.nclass = rfl(a.nclass);
  A.table = rflp(a.table);
  A.table_stride = rfl64(a.table_stride);
  A.dG1.d = rfl(a.dG1.d);
  A.dG1.m = rfl(a.dG1.m);
  A.dG1.sh1 = rfl(a.dG1.sh1);
  A.dG1.sh2 = rfl(a.dG1.sh2);
  A.ring = rfl(a.ring);
  A.flush = rfl(a.flush);
  A.total = rfl64(a.total);
  A.rows_per_tile = rfl64(a.rows_per_tile);
  A.cnt_row = rflp(a.cnt_row);
  A.endc = rflp(a.endc);
  A.leaf = rflp(a.leaf);
  A.leaf_rows = rfl64(a.leaf_rows);
  A.out = rflp(a.out);
  A.err = rflp(a.err);
  A.dG.d = rfl(a.dG.d);
  A.dG.m = rfl(a.dG.m);
  A.dG.sh1 = rfl(a.dG.sh1);
  A.dG.sh2 = rfl(a.dG.sh2);
  return A;
}

template <bool COUNT_ONLY>
__global__ __launch_bounds__(kWriteWaves * kWave) void k_write_batch(
    const EnumParams* __restrict__ qp, const uint64_t* __restrict__ qout,
    const BatchUnit* __restrict__ units, uint32_t nunits, uint32_t* __restrict__ queue,
    uint32_t* __restrict__ done_tiles, uint64_t* __restrict__ t_done, uint32_t* out, BatchLds L) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t s_unit, next_slot;
  const int lane = lane_id();
  const int wave = int(threadIdx.x / kWave);
  uint32_t* ring = lds + L.waves + uint32_t(wave) * L.wave_words;
  uint32_t* marks = ring + L.ring_words;
  const uint32_t* lds_memo = lds + L.memo;
  uint32_t* lds_cnt = lds + L.cnt;
  uint32_t* lds_endc = lds + L.endc;
  uint32_t* tstates = lds + L.states;
  const EnumParams& P = *reinterpret_cast<const EnumParams*>(lds + L.desc);

  for (;;) {
    if (threadIdx.x == 0) s_unit = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t u = s_unit;
    if (u >= nunits) break;
    const uint32_t q = rfl(units[u].q);
    const uint32_t tlo = rfl(units[u].tile_lo), thi = rfl(units[u].tile_hi);
    const uint64_t obase = rfl64(qout[q]);
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(qp + q);
      for (uint32_t i = threadIdx.x; i < kDescWords; i += blockDim.x) lds[L.desc + i] = src[i];
    }
    __syncthreads();
    const int U = int(rfl(uint32_t(P.U))), k = int(rfl(uint32_t(P.k))), d = int(rfl(uint32_t(P.d)));
    const int pack = int(rfl(uint32_t(P.pack))), ldscnt = int(rfl(uint32_t(P.lds_cnt)));
    const uint32_t S = uint32_t(U + 2);
    const uint32_t ntl = thi - tlo;
    // Prologue: every global load for this unit, before its first store.
    if (k >= 1 && pack > 0) {
      const uint32_t* leaf = rflp(P.leaf);
      const uint64_t words = rfl64(P.memo_words);
      const uint64_t nvec = words / 4;
      const uint4* src = reinterpret_cast<const uint4*>(leaf);
      uint4* dst = reinterpret_cast<uint4*>(lds + L.memo);
      for (uint64_t i = threadIdx.x; i < nvec; i += blockDim.x) dst[i] = src[i];
      for (uint64_t w = nvec * 4 + threadIdx.x; w < words; w += blockDim.x)
        lds[L.memo + w] = leaf[w];
    }
    if (k >= 1 && ldscnt) {
      const uint64_t N = uint64_t(rfl(P.n)) + 1;
      const uint64_t* cu = rflp(P.table) + uint64_t(U) * rfl64(P.table_stride);
      const uint64_t* endc = rflp(P.endc);
      const uint32_t nclass = rfl(P.nclass);
      for (uint64_t x = threadIdx.x; x < N; x += blockDim.x) lds_cnt[x] = uint32_t(cu[x]);
      for (uint32_t r = threadIdx.x; r < nclass; r += blockDim.x) lds_endc[r] = uint32_t(endc[r]);
    }
    {
      const uint32_t* st = rflp(P.tiles) + uint64_t(tlo) * S;
      for (uint32_t i = threadIdx.x; i < ntl * S; i += blockDim.x) tstates[i] = st[i];
    }
    if (threadIdx.x == 0) next_slot = 0;
    const uint32_t gj = lane < d ? P.g.g[lane] : 0;
    const uint32_t fsh = lane <= k ? P.fshift[lane] : 0;
    const uint32_t fmk = lane <= k ? P.fmask[lane] : 0;
    TileArgs A = uniform_args(tile_args(P));
    A.out = out + obase;
    __syncthreads();

    uint64_t csum = 0;
    for (;;) {
      uint32_t slot_l = 0;
      if (lane == 0) slot_l = atomicAdd(&next_slot, 1u);
      const uint32_t ti = rfl(slot_l);
      if (ti >= ntl) break;
      const uint64_t tile = tlo + ti;
      const uint32_t* st = tstates + ti * S;
#define ZSET_TILE(MODE, PACK, LDSCNT)                                                         \
  write_tile<MODE, COUNT_ONLY, true, PACK, LDSCNT>(A, tile, st, ring, marks, lds_memo, lds_cnt, \
                                                    lds_endc, gj, fsh, fmk, csum)
      if (k == 0) {
        ZSET_TILE(0, 0, false);
      } else if (pack == 1) {
        if (ldscnt) ZSET_TILE(1, 1, true); else ZSET_TILE(1, 1, false);
      } else if (pack == 2) {
        if (ldscnt) ZSET_TILE(1, 2, true); else ZSET_TILE(1, 2, false);
      } else {
        if (ldscnt) ZSET_TILE(1, 0, true); else ZSET_TILE(1, 0, false);
      }
#undef ZSET_TILE
    }
    if (COUNT_ONLY) {
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) csum += __shfl_xor(csum, off, kWave);
      if (lane == 0 && csum != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(rflp(P.checksum)),
                  static_cast<unsigned long long>(csum));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t before = atomicAdd(done_tiles + q, ntl);
      if (uint64_t(before) + ntl == rfl64(P.ntiles)) t_done[q] = wall_clock64();
    }
  }
}

// Clears the per-run state of a batch (a kernel, not a memset node, so that
// it can sit in a captured graph) and stamps the start time.
__global__ __launch_bounds__(256) void k_batch_reset(uint32_t* queue, int* err,
                                                     uint32_t* done_tiles, uint64_t* checksums,
                                                     uint64_t* t_done, uint64_t* t_start,
                                                     uint32_t nq) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {
    *queue = 0;
    *err = 0;
    *t_start = wall_clock64();
  }
  if (i < nq) {
    done_tiles[i] = 0;
    checksums[i] = 0;
    t_done[i] = 0;
  }
}

// d = 1 queries of a batch: at most one row each.
__global__ __launch_bounds__(256) void k_single_batch(const EnumParams* __restrict__ qp,
                                                      const uint64_t* __restrict__ qout,
                                                      const uint32_t* __restrict__ idx,
                                                      uint32_t count, uint32_t* out,
                                                      int count_only, uint64_t* t_done) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const uint32_t q = idx[i];
  const EnumParams& P = qp[q];
  const uint32_t g = P.g.g[0];
  if (P.n % g == 0) {
    if (count_only) {
      uint64_t h = fnv1a_u64(kFnvOffset, 0);
      h = fnv1a_u32(h, P.n / g);
      *P.checksum += h;
    } else {
      out[qout[q]] = P.n / g;
    }
  }
  t_done[q] = wall_clock64();
}

// d = 1: Z(n; g_1) is {n / g_1} when g_1 divides n.
__global__ void k_single(uint32_t n, uint32_t g, uint32_t* out, int count_only,
                         uint64_t* checksum) {
  if (threadIdx.x != 0 || n % g != 0) return;
  if (count_only) {
    uint64_t h = fnv1a_u64(kFnvOffset, 0);
    h = fnv1a_u32(h, n / g);
    *checksum += h;
  } else {
    out[0] = n / g;
  }
}

// Per instantiation of the write kernel: the largest dynamic LDS its function
// attribute has been raised to, and the occupancy found for each LDS size
// (both fixed for a kernel and a size, and costly to ask for per call).
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
struct WriteKernelCache {
  static std::mutex mu;
  static size_t attr_lds;
  static std::map<size_t, int> occupancy;
};
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
std::mutex WriteKernelCache<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>::mu;
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
size_t WriteKernelCache<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>::attr_lds = 0;
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
std::map<size_t, int> WriteKernelCache<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>::occupancy;

template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
hipError_t raise_lds_attr(size_t lds) {
  using C = WriteKernelCache<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>;
  auto kern = k_write<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>;
  std::lock_guard<std::mutex> lock(C::mu);
  if (lds <= C::attr_lds) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e == hipSuccess) C::attr_lds = lds;
  return e;
}

template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
hipError_t launch_write_t(const EnumParams& P, hipStream_t s) {
  auto kern = k_write<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>;
  const size_t lds = write_lds_bytes(P);
  hipError_t e = raise_lds_attr<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(P.write_blocks), dim3(kWriteWaves * kWave), lds, s, P);
  return hipGetLastError();
}

template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
hipError_t occupancy_t(const EnumParams& P, int* per_cu) {
  using C = WriteKernelCache<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>;
  auto kern = k_write<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>;
  const size_t lds = write_lds_bytes(P);
  {
    std::lock_guard<std::mutex> lock(C::mu);
    auto it = C::occupancy.find(lds);
    if (it != C::occupancy.end()) {
      *per_cu = it->second;
      return hipSuccess;
    }
  }
  hipError_t e = raise_lds_attr<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(lds);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, kWriteWaves * kWave, lds);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(C::mu);
  C::occupancy[lds] = *per_cu;
  return hipSuccess;
}

// Outer-prefix length and k compiled in for the common materialising shapes
// (memo packed and segment counts in LDS, 16-byte-aligned output).
constexpr int kSpecMaxOuter = 3, kSpecMaxK = 3;

template <template <int, bool, bool, int, bool, int, int> class F, int PK, class... A>
hipError_t dispatch_spec(const EnumParams& P, A... args) {
  const int no = P.U - 1, kf = P.k;
#define ZSET_SPEC(NO_, KF_) \
  if (no == NO_ && kf == KF_) return F<1, false, true, PK, true, NO_, KF_>::run(P, args...);
  ZSET_SPEC(0, 1) ZSET_SPEC(0, 2) ZSET_SPEC(0, 3)
  ZSET_SPEC(1, 1) ZSET_SPEC(1, 2) ZSET_SPEC(1, 3)
  ZSET_SPEC(2, 1) ZSET_SPEC(2, 2) ZSET_SPEC(2, 3)
  ZSET_SPEC(3, 1) ZSET_SPEC(3, 2) ZSET_SPEC(3, 3)
#undef ZSET_SPEC
  return F<1, false, true, PK, true, -1, -1>::run(P, args...);
}

// Partial memos: the kNoPartial instantiations.
template <template <int, bool, bool, int, bool, int, int> class F, int PK, class... A>
hipError_t dispatch_partial(const EnumParams& P, bool count_only, bool align16, A... args) {
  constexpr int X = kNoPartial;
  if (P.lds_cnt) {
    if (count_only) return F<1, true, false, PK, true, X, -1>::run(P, args...);
    return align16 ? F<1, false, true, PK, true, X, -1>::run(P, args...)
                   : F<1, false, false, PK, true, X, -1>::run(P, args...);
  }
  if (count_only) return F<1, true, false, PK, false, X, -1>::run(P, args...);
  return align16 ? F<1, false, true, PK, false, X, -1>::run(P, args...)
                 : F<1, false, false, PK, false, X, -1>::run(P, args...);
}

// Dispatch on the run-time choices to the matching instantiation.
template <template <int, bool, bool, int, bool, int, int> class F, class... A>
hipError_t dispatch(const EnumParams& P, bool count_only, bool align16, A... args) {
  if (P.k == 0) {
    if (count_only) return F<0, true, false, 0, false, -1, -1>::run(P, args...);
    return align16 ? F<0, false, true, 0, false, -1, -1>::run(P, args...)
                   : F<0, false, false, 0, false, -1, -1>::run(P, args...);
  }
  if (P.memo_top && P.memo_top <= P.n) {  // a partial memo
    switch (P.pack) {
      case 1: return dispatch_partial<F, 1>(P, count_only, align16, args...);
      case 2: return dispatch_partial<F, 2>(P, count_only, align16, args...);
      default: return dispatch_partial<F, 0>(P, count_only, align16, args...);
    }
  }
  const bool spec = !P.pair && !count_only && align16 &&
                    P.lds_cnt && P.U >= 1 &&
                    P.U - 1 <= kSpecMaxOuter && P.k <= kSpecMaxK;
  if (spec && P.pack == 1) return dispatch_spec<F, 1>(P, args...);
  if (spec && P.pack == 2) return dispatch_spec<F, 2>(P, args...);
#define ZSET_PACK_CASES(PK)                                                              \
  if (P.lds_cnt) {                                                                       \
    if (count_only) return F<1, true, false, PK, true, -1, -1>::run(P, args...);         \
    return align16 ? F<1, false, true, PK, true, -1, -1>::run(P, args...)                \
                   : F<1, false, false, PK, true, -1, -1>::run(P, args...);              \
  }                                                                                      \
  if (count_only) return F<1, true, false, PK, false, -1, -1>::run(P, args...);          \
  return align16 ? F<1, false, true, PK, false, -1, -1>::run(P, args...)                 \
                 : F<1, false, false, PK, false, -1, -1>::run(P, args...);
  switch (P.pack) {
    case 1: { ZSET_PACK_CASES(1) }
    case 2: { ZSET_PACK_CASES(2) }
    default: { ZSET_PACK_CASES(0) }
  }
#undef ZSET_PACK_CASES
}

template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
struct LaunchF {
  static hipError_t run(const EnumParams& P, hipStream_t s) {
    return launch_write_t<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(P, s);
  }
};
template <int MODE, bool COUNT_ONLY, bool ALIGN16, int PACK, bool LDSCNT, int NO, int KF>
struct OccF {
  static hipError_t run(const EnumParams& P, int* per_cu) {
    return occupancy_t<MODE, COUNT_ONLY, ALIGN16, PACK, LDSCNT, NO, KF>(P, per_cu);
  }
};

}  // namespace

size_t write_lds_bytes(const EnumParams& P) {
  return size_t(write_shared_words(P) + kWriteWaves * write_wave_words(P)) * sizeof(uint32_t);
}

int write_waves_per_block() { return kWriteWaves; }

hipError_t write_occupancy(const EnumParams& P, bool count_only, bool align16, int* per_cu) {
  return dispatch<OccF>(P, count_only, align16, per_cu);
}

hipError_t launch_plan(const EnumParams& P, hipStream_t s) {
  const uint64_t blocks = (P.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_plan, dim3(uint32_t(blocks)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_plan_device_sized(const EnumParams& P, hipStream_t s) {
  if (!P.total_dev || P.want_tiles == 0) return hipErrorInvalidValue;
  const uint64_t blocks = (P.want_tiles + 255) / 256;
  hipLaunchKernelGGL(k_plan, dim3(uint32_t(blocks)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_plan_leaf(const EnumParams& P, const LeafJob& J, hipStream_t s) {
  if (!P.total_dev || P.want_tiles == 0) return hipErrorInvalidValue;
  const uint64_t pb = (P.want_tiles + 255) / 256;
  const uint64_t lb = std::max<uint64_t>(1, (J.leaf_rows + 255) / 256);
  if (pb + lb > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plan_leaf, dim3(uint32_t(pb + lb)), dim3(256), 0, s, P, J, uint32_t(pb));
  return hipGetLastError();
}

hipError_t launch_write(const EnumParams& P, bool count_only, bool align16, hipStream_t s) {
  // Without a slice table the kernel plans its dealt slices itself; claimed
  // chunks need the table.
  if (!P.tiles && (P.chunk != 0 || P.static_tiles != P.ntiles)) return hipErrorInvalidValue;
  return dispatch<LaunchF>(P, count_only, align16, s);
}

int write_batch_waves() { return kWriteWaves; }

hipError_t launch_batch_reset(uint32_t* queue, int* err, uint32_t* done_tiles,
                              uint64_t* checksums, uint64_t* t_done, uint64_t* t_start,
                              uint32_t nq, hipStream_t s) {
  const uint32_t blocks = (nq + 255) / 256 + 1;
  hipLaunchKernelGGL(k_batch_reset, dim3(blocks), dim3(256), 0, s, queue, err, done_tiles,
                     checksums, t_done, t_start, nq);
  return hipGetLastError();
}

hipError_t launch_plan_batch(const EnumParams* qp, const uint64_t* tile_base,
                             const uint32_t* plan_q, uint32_t nplan, uint64_t total_tiles,
                             hipStream_t s) {
  if (total_tiles == 0 || nplan == 0) return hipSuccess;
  const uint64_t blocks = (total_tiles + 255) / 256;
  hipLaunchKernelGGL(k_plan_batch, dim3(uint32_t(blocks)), dim3(256), 0, s, qp, tile_base, plan_q,
                     nplan, total_tiles);
  return hipGetLastError();
}

template <bool CO>
hipError_t prepare_write_batch_t(const BatchLds& L) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_write_batch<CO>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(size_t(L.total_words) * 4));
}

hipError_t prepare_write_batch(const BatchLds& L, bool count_only) {
  return count_only ? prepare_write_batch_t<true>(L) : prepare_write_batch_t<false>(L);
}

hipError_t write_batch_occupancy(const BatchLds& L, bool count_only, int* per_cu) {
  hipError_t e = prepare_write_batch(L, count_only);
  if (e != hipSuccess) return e;
  const size_t lds = size_t(L.total_words) * 4;
  if (count_only)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_write_batch<true>,
                                                        kWriteWaves * kWave, lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_write_batch<false>,
                                                      kWriteWaves * kWave, lds);
}

hipError_t launch_write_batch(const EnumParams* qp, const uint64_t* qout, const BatchUnit* units,
                              uint32_t nunits, uint32_t* queue, uint32_t* done_tiles,
                              uint64_t* t_done, uint32_t* out, const BatchLds& L,
                              uint32_t blocks, bool count_only, hipStream_t s) {
  if (nunits == 0) return hipSuccess;
  const size_t lds = size_t(L.total_words) * 4;
  if (count_only)
    hipLaunchKernelGGL(k_write_batch<true>, dim3(blocks), dim3(kWriteWaves * kWave), lds, s, qp,
                       qout, units, nunits, queue, done_tiles, t_done, out, L);
  else
    hipLaunchKernelGGL(k_write_batch<false>, dim3(blocks), dim3(kWriteWaves * kWave), lds, s, qp,
                       qout, units, nunits, queue, done_tiles, t_done, out, L);
  return hipGetLastError();
}

hipError_t launch_single_batch(const EnumParams* qp, const uint64_t* qout, const uint32_t* idx,
                               uint32_t count, uint32_t* out, bool count_only, uint64_t* t_done,
                               hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_single_batch, dim3((count + 255) / 256), dim3(256), 0, s, qp, qout, idx,
                     count, out, int(count_only), t_done);
  return hipGetLastError();
}

hipError_t launch_single(uint64_t n, uint32_t g, uint32_t* out, bool count_only,
                         uint64_t* checksum, hipStream_t s) {
  hipLaunchKernelGGL(k_single, dim3(1), dim3(64), 0, s, uint32_t(n), g, out, int(count_only),
                     checksum);
  return hipGetLastError();
}

}  // namespace zset
