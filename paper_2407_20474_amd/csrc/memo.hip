// memo.hip -- the memo of the trailing generators (paper, Section 3.1) and
// its leaf-order layout.
//
// Memo[p] = Z(p; h_1..h_k) for p in [0, top), every list ascending.  It is
// built by the disjoint recurrence of Lemma 2.3 read in ascending order
// (Lemma 2.6 mirrored): Z_{>=i}(m) is a prefix of the ascending list Z(m), so
//
//   Memo[p] = incr_k(first |Z_{>=k}(p-h_k)| rows of Memo[p-h_k])
//           ++ ... ++
//             incr_1(first |Z_{>=1}(p-h_1)| rows of Memo[p-h_1])
//
// with |Z_{>=i}(m)| = sum_{i' >= i} |Z_{=i'}(m)| and |Z_{=i}(m)| =
// |Z_{>=i}(m - h_i)| (Section 2.3).  Elements are processed in batches of
// b = min(h) consecutive values, which never depend on each other (Section
// 2.2, elementwise parallelism); inside a batch every copied row is its own
// work item (factorizationwise parallelism, Alg 2.9).
//
// For k = 1 the recurrence's solution is closed (k_memo_k1).  For k >= 2 two
// schedules compute the same natural-order memo:
//  * k_memo_chain_wave: one wavefront keeps the whole memo in LDS and saves
//    the cardinalities |Z_{>=i}(p)| as it goes (Section 2.3), in a ring of the
//    last W elements, so a batch costs a few LDS round trips and no barrier.
//  * k_memo_src + k_memo_batch: for memos larger than LDS, every destination
//    row's source is precomputed in parallel from the count table, then one
//    multi-workgroup launch per batch copies rows in global memory.
//
// k_memo_leaf rewrites the natural-order memo into the leaf order used by the
// write pass (see enumerate.hip): for a generator G just left of the memo
// coordinates, the elements p <= n are grouped by residue class rho = p mod G,
// each class by descending p.  Then for any x <= n the rows of
// Z(x; G, h) = {(a, m) : m in Memo[x - a G]} are one contiguous run that
// starts at end[x mod G] - |Z(x; G, h)|, in ascending lex order, and each
// memo row carries floor(p / G) so that a = floor(x / G) - floor(p / G).
#include <algorithm>
#include <cstring>

#include <map>
#include <mutex>

#include "zset_internal.h"

namespace zset {

namespace {

// Inclusive prefix sum over the 64 lanes with DPP (row_shr within 16-lane
// rows, then row_bcast 15 / 31 across rows): no LDS round trip.
__device__ inline uint32_t wave_incl_sum_u32(uint32_t v) {
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xf, 0xf, false));
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xf, 0xf, false));
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xf, 0xf, false));
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xf, 0xf, false));
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xa, 0xf, false));
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xc, 0xf, false));
  return v;
}

// Inclusive prefix max over the wave (same DPP pattern as the sum above).
__device__ inline uint32_t wave_incl_max_u32(uint32_t v) {
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xf, 0xf, false)));
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xf, 0xf, false)));
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xf, 0xf, false)));
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xf, 0xf, false)));
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xa, 0xf, false)));
  v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xc, 0xf, false)));
  return v;
}

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront, no barriers.  Steps take `step` = min(64, min(h)) consecutive
// elements, one per lane; a step never reads an element of its own (p - h_i <
// x0), so steps are the paper's elementwise batches cut to the wave width.
// Per step:
//  * every lane reads, for each i, |Z_{>=i}(p - h_i)| and where the list
//    Z(p - h_i) starts, from rings GE and OFF of the last W elements (the
//    cardinalities saved as they are computed, Section 2.3);
//  * |Z_{=i}(p)| = |Z_{>=i}(p - h_i)|, so |Z_{>=i}(p)| is a suffix sum over i,
//    saved for later steps, and |Z(p)| = |Z_{>=1}(p)|; a wave prefix sum of the
//    sizes places every list;
//  * the copy-and-increment: when the step's longest list is at most
//    kLaneCopyRows rows per 64 rows of the step, each lane copies its own
//    element's blocks (in the order i = k..1); otherwise it runs one lane per
//    copied row
//    (factorizationwise parallelism, Alg 2.9), 64 rows at a time: the first
//    row of each element is marked in LDS and a wave prefix max gives every
//    row its element, whose saved cardinalities then give the row's block i
//    and its source row.
// Dynamic LDS layout (uint32): GE[W*k] | OFF[W] | marks[64] | M rows, W a power
// of two >= max(h) + step and M 16-byte aligned (memo_ring_words).
//  * WINDOW = false: M holds the whole memo (Rcap rows); a memo that would
//    outgrow it stops and marks off_out[top] = ~0 (the caller then takes
//    another schedule); the rows are copied to `nat` at the end.
//  * WINDOW = true: M is a ring of Mmask + 1 rows holding the lists of the last
//    max(h) + step elements (the only ones a step reads), and every row is also
//    stored to `nat` as it is made; a step that would overrun the ring stops
//    the build with an error (the caller sizes the ring from the longest list).
// Rexp, when non-zero, is the row count the count table predicts.
// A step copies one element per lane while its longest list has at most this
// many rows per 64 rows of the step (else one lane per row).
constexpr uint32_t kLaneCopyRows = 3;

template <int KMAX, bool WINDOW>
__device__ inline void memo_chain(const uint32_t (&hg)[KMAX], int k, uint32_t top, uint32_t step,
                                  uint32_t W, uint32_t hmax, uint32_t Mmask, uint32_t Rcap,
                                  uint32_t Rexp, uint32_t* __restrict__ nat,
                                  uint64_t* __restrict__ off_out, int* __restrict__ err,
                                  uint32_t* lds) {
  uint32_t* GE = lds;
  uint32_t* OFF = GE + size_t(W) * k;
  uint32_t* marks = lds + memo_ring_words(k, W) - kWave;
  uint32_t* M = lds + memo_ring_words(k, W);
  const uint32_t lane = threadIdx.x;
  const uint32_t Wm = W - 1;
  auto mrow = [&](uint32_t row) { return WINDOW ? (row & Mmask) : row; };

  // Z(0) = [0]: one all-zero row, and |Z_{>=i}(0)| = 1 for every i.
  if (lane < uint32_t(k)) {
    M[lane] = 0;
    GE[lane] = 1;
    if (WINDOW) nat[lane] = 0;
  }
  if (lane == 0) {
    OFF[0] = 0;
    off_out[0] = 0;
  }
  uint32_t running = 1;
  wave_sync_lds();

  for (uint32_t x0 = 1; x0 < top; x0 += step) {
    const uint32_t p = x0 + lane;
    const bool valid = lane < step && p < top;
    uint32_t s[KMAX], so[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      s[i] = 0;
      so[i] = 0;
      if (i < k && valid && p >= hg[i]) {
        const uint32_t slot = (p - hg[i]) & Wm;
        s[i] = GE[slot * k + i];
        so[i] = OFF[slot];
      }
    }
    // ge[i] = |Z_{>=i}(p)| = sum over i' >= i of |Z_{=i'}(p)|.
    uint32_t ge[KMAX];
    uint32_t acc = 0;
#pragma unroll
    for (int i = KMAX - 1; i >= 0; --i) {
      if (i < k) {
        acc += s[i];
        if (valid) GE[(p & Wm) * k + i] = acc;
      }
      ge[i] = acc;
    }
    const uint32_t size = valid ? acc : 0;
    const uint32_t incl = wave_incl_sum_u32(size);
    const uint32_t tot = __builtin_amdgcn_readlane(incl, kWave - 1);
    bool over;
    if (WINDOW) {
      const uint32_t oldest = x0 > hmax ? OFF[(x0 - hmax) & Wm] : 0;
      over = uint64_t(running) + tot - oldest > uint64_t(Mmask) + 1;
    } else {
      over = uint64_t(running) + tot > Rcap;
    }
    if (over) {
      if (lane == 0) {
        off_out[top] = ~uint64_t(0);
        if (WINDOW) set_error(err, kErrMemoTotal);
      }
      return;
    }
    const uint32_t first = incl - size;  // this element's first row in the step
    if (valid) {
      OFF[p & Wm] = running + first;
      off_out[p] = running + first;
    }
    // Copy-and-increment.  Each lane copying its own element's blocks costs
    // about one LDS round trip per row of the longest list of the step; one
    // lane per row of the step costs a few round trips per 64 rows.  The step takes the cheaper: lanes per element
    // when its lists are of similar length, lanes per row when a few long
    // lists would leave most lanes idle.
    const uint32_t smax = __builtin_amdgcn_readlane(wave_incl_max_u32(size), kWave - 1);
    if (smax <= kLaneCopyRows * ((tot + kWave - 1) / kWave)) {
      uint32_t dst = running + first;
#pragma unroll
      for (int i = KMAX - 1; i >= 0; --i) {
        if (i < k) {
          for (uint32_t r = 0; r < s[i]; ++r) {
            uint32_t v[KMAX];
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
              if (c < k) v[c] = M[mrow(so[i] + r) * k + c];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
              if (c < k) {
                const uint32_t w = v[c] + (c == i ? 1u : 0u);
                M[mrow(dst + r) * k + c] = w;
                if (WINDOW) nat[uint64_t(dst + r) * k + c] = w;
              }
            }
          }
          dst += s[i];
        }
      }
      wave_sync_lds();
      running += tot;
      continue;
    }
    uint32_t carry = 0;
    for (uint32_t beta = 0; beta < tot; beta += kWave) {
      marks[lane] = 0;
      wave_sync_lds();
      if (size != 0 && first >= beta && first - beta < uint32_t(kWave)) marks[first - beta] = lane + 1;
      wave_sync_lds();
      uint32_t m = wave_incl_max_u32(marks[lane]);
      m = max(m, carry);
      carry = __builtin_amdgcn_readlane(m, kWave - 1);
      const int owner = int(m) - 1;  // row 0 of a step always starts an element
      const uint32_t rho = beta + lane;
      const uint32_t t = rho - uint32_t(__shfl(int(first), owner, kWave));
      // Block i holds the rows t in [ge[i + 1], ge[i]) of the element.
      uint32_t src = 0, inc = 0, hi_prev = 0;
#pragma unroll
      for (int i = KMAX - 1; i >= 0; --i) {
        if (i < k) {
          const uint32_t hi = uint32_t(__shfl(int(ge[i]), owner, kWave));
          const uint32_t o = uint32_t(__shfl(int(so[i]), owner, kWave));
          if (t >= hi_prev && t < hi) {
            src = o + (t - hi_prev);
            inc = uint32_t(i);
          }
          hi_prev = hi;
        }
      }
      if (rho < tot) {
        uint32_t v[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
          if (c < k) v[c] = M[mrow(src) * k + c];
        const uint32_t dst = running + rho;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
          if (c < k) {
            const uint32_t w = v[c] + (uint32_t(c) == inc ? 1u : 0u);
            M[mrow(dst) * k + c] = w;
            if (WINDOW) nat[uint64_t(dst) * k + c] = w;
          }
        }
      }
      wave_sync_lds();
    }
    running += tot;
  }
  if (lane == 0) {
    off_out[top] = running;
    if (Rexp != 0 && running != Rexp) set_error(err, kErrMemoTotal);
  }
  if (!WINDOW) {
    const uint32_t words = running * uint32_t(k);
    const uint32_t nvec = words / 4;
    const uint4* src = reinterpret_cast<const uint4*>(M);
    uint4* dstv = reinterpret_cast<uint4*>(nat);
    for (uint32_t v = lane; v < nvec; v += kWave) dstv[v] = src[v];
    for (uint32_t w = nvec * 4 + lane; w < words; w += kWave) nat[w] = M[w];
  }
}

template <int KMAX>
__global__ __launch_bounds__(kWave) void k_memo_chain_wave(Gens h, int k, uint32_t top,
                                                            uint32_t step, uint32_t W,
                                                            uint32_t Rcap, uint32_t Rexp,
                                                            uint32_t* __restrict__ nat,
                                                            uint64_t* __restrict__ off_out,
                                                            int* __restrict__ err) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t hg[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) hg[i] = h.g[i];
  memo_chain<KMAX, false>(hg, k, top, step, W, 0, 0, Rcap, Rexp, nat, off_out, err, lds);
}

template <int KMAX>
__global__ __launch_bounds__(kWave) void k_memo_chain_window(Gens h, int k, uint32_t top,
                                                              uint32_t step, uint32_t W,
                                                              uint32_t hmax, uint32_t Mmask,
                                                              uint32_t Rexp,
                                                              uint32_t* __restrict__ nat,
                                                              uint64_t* __restrict__ off_out,
                                                              int* __restrict__ err) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t hg[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) hg[i] = h.g[i];
  memo_chain<KMAX, true>(hg, k, top, step, W, hmax, Mmask, 0, Rexp, nat, off_out, err, lds);
}

// Batched: workgroup b (one wavefront) builds the memo of jobs[b].
template <int KMAX>
__global__ __launch_bounds__(kWave) void k_memo_chain_batch(const MemoJob* __restrict__ jobs,
                                                             int* __restrict__ err) {
  extern __shared__ __align__(16) uint32_t lds[];
  const MemoJob& J = jobs[blockIdx.x];
  uint32_t hg[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) hg[i] = __builtin_amdgcn_readfirstlane(J.h[i]);
  const int k = __builtin_amdgcn_readfirstlane(J.k);
  const uint32_t top = __builtin_amdgcn_readfirstlane(J.top);
  const uint32_t step = __builtin_amdgcn_readfirstlane(J.step);
  const uint32_t W = __builtin_amdgcn_readfirstlane(J.W);
  const uint32_t R = __builtin_amdgcn_readfirstlane(J.R);
  memo_chain<KMAX, false>(hg, k, top, step, W, 0, 0, R, R, J.nat, J.off, err, lds);
}

// k = 1: the recurrence Memo[p] = incr_1(Memo[p - h]) from Memo[0] = {()}
// has the solution Memo[p] = {(p / h)} when h divides p and {} otherwise
// (induction on p), so every element is independent: row j (the element
// p = j h) holds j and off[p] = ceil(p / h).  One pass, no batches.
__device__ inline void memo_k1_item(uint32_t h, uint32_t top, uint32_t R, uint64_t i,
                                    uint32_t* __restrict__ nat, uint64_t* __restrict__ off) {
  if (i <= top) off[i] = (i + h - 1) / h;
  if (i < R) nat[i] = uint32_t(i);
}

__global__ __launch_bounds__(256) void k_memo_k1(uint32_t h, uint32_t top, uint32_t R,
                                                 uint32_t* __restrict__ nat,
                                                 uint64_t* __restrict__ off) {
  memo_k1_item(h, top, R, uint64_t(blockIdx.x) * 256 + threadIdx.x, nat, off);
}

// k = 2: Z(p; h_1, h_2) in closed form (Memo2, memo2_first: zset_internal.h).
__global__ __launch_bounds__(256) void k_memo2_count(Memo2 M, uint32_t top,
                                                     uint64_t* __restrict__ cnt) {
  const uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p > top) return;
  uint32_t m0 = 0, rows = 0;
  cnt[p] = (p < top && memo2_first(M, uint32_t(p), &m0, &rows)) ? rows : 0;  // cnt[top] = 0
}

// Rows beyond cap (the buffer's capacity) are not written; the caller
// compares the total with cap.
__global__ __launch_bounds__(256) void k_memo2_fill(Memo2 M, uint32_t top, uint64_t cap,
                                                    const uint64_t* __restrict__ off,
                                                    uint32_t* __restrict__ nat) {
  const uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= top) return;
  uint32_t m0 = 0, rows = 0;
  if (!memo2_first(M, uint32_t(p), &m0, &rows)) return;
  const uint64_t o = off[p];
  for (uint32_t t = 0; t < rows && o + t < cap; ++t) {
    const uint32_t m1 = m0 + t * M.h2c;
    nat[(o + t) * 2] = m1;
    nat[(o + t) * 2 + 1] = (uint32_t(p) - m1 * M.h1) / M.h2;
  }
}

// Batched: the workgroups of job j are [jobs[j].block0, jobs[j + 1].block0).
__global__ __launch_bounds__(256) void k_memo_k1_batch(const MemoJob* __restrict__ jobs,
                                                       uint32_t njobs) {
  uint32_t lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (jobs[mid].block0 <= blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const MemoJob& J = jobs[lo];
  memo_k1_item(J.h[0], J.top, J.R, uint64_t(blockIdx.x - J.block0) * 256 + threadIdx.x, J.nat,
               J.off);
}

// Sources of every destination row, from the count table.  Row j of Memo[p]
// (p >= 1) in block i at position t is incr_i of row off[p - h_i] + t.
// srcw[j] = (source row << 5) | i.  ge_i(m) = |Z(m; h_i..h_k)| = ge[i * ge_stride + m].
__global__ __launch_bounds__(256) void k_memo_src(Gens h, int k, uint32_t top,
                                                  const uint64_t* __restrict__ off,
                                                  const uint64_t* __restrict__ ge,
                                                  uint64_t ge_stride,
                                                  uint64_t* __restrict__ srcw,
                                                  uint32_t* __restrict__ nat,
                                                  int* __restrict__ err) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= top) return;
  if (p == 0) {
    for (int c = 0; c < k; ++c) nat[c] = 0;
    srcw[0] = ~uint64_t(0);
    return;
  }
  uint64_t o = off[p];
  for (int i = k - 1; i >= 0; --i) {
    if (p < h.g[i]) continue;
    const uint32_t src = p - h.g[i];
    const uint64_t s = ge[uint64_t(i) * ge_stride + src];
    const uint64_t so = off[src];
    const uint64_t end = off[p + 1];
    if (o + s > end) {  // counts disagree: never write past this element's rows
      set_error(err, kErrMemoTotal);
      return;
    }
    for (uint64_t t = 0; t < s; ++t) srcw[o++] = ((so + t) << 5) | uint64_t(i);
  }
  if (o != off[p + 1]) set_error(err, kErrMemoTotal);
}

// One batch of copies: rows [off[x0], off[x1]).
__global__ __launch_bounds__(256) void k_memo_batch(int k, const uint64_t* __restrict__ off,
                                                    uint32_t x0, uint32_t x1,
                                                    const uint64_t* __restrict__ srcw,
                                                    uint32_t* __restrict__ nat) {
  const uint64_t lo = off[x0], hi = off[x1];
  for (uint64_t j = lo + uint64_t(blockIdx.x) * 256 + threadIdx.x; j < hi;
       j += uint64_t(gridDim.x) * 256) {
    const uint64_t w = srcw[j];
    const uint64_t src = w >> 5;
    const int i = int(w & 31);
    if (src >= j) continue;  // sources always precede their copies
    for (int c = 0; c < k; ++c)
      nat[j * k + c] = nat[src * k + c] + (c == i ? 1u : 0u);
  }
}

// Every batch in one workgroup: batch [x0, x0 + b) copies rows
// [off[x0], off[x0 + b)) and a workgroup barrier separates it from the next,
// whose sources it may hold.  For memos whose batches hold few rows, where a
// launch per batch would cost more than its copies.
__global__ __launch_bounds__(1024) void k_memo_batches_wg(int k, const uint64_t* __restrict__ off,
                                                          uint32_t top, uint32_t b,
                                                          const uint64_t* __restrict__ srcw,
                                                          uint32_t* __restrict__ nat) {
  for (uint32_t x0 = 1; x0 < top; x0 += b) {
    const uint32_t x1 = top - x0 > b ? x0 + b : top;
    const uint64_t lo = off[x0], hi = off[x1];
    for (uint64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
      const uint64_t w = srcw[j];
      const uint64_t src = w >> 5;
      const int i = int(w & 31);
      if (src >= j) continue;  // sources always precede their copies
      for (int c = 0; c < k; ++c) nat[j * k + c] = nat[src * k + c] + (c == i ? 1u : 0u);
    }
    __syncthreads();
  }
}

// Natural order -> leaf order for p in [0, n]: row t of Memo[p] goes to
// pos(p) + t with pos(p) = end[p mod G] - cu[p]; it is stored as the fields
// (floor(p / G), m_1..m_k): k+1 plain words (pack 0), or packed into one 32-
// or 64-bit word at the bit offsets of the write pass (pack 1, 2).
__device__ inline void memo_leaf_element(const LeafJob& J, uint32_t p, int* __restrict__ err) {
  const int k = J.k;
  const uint32_t q = J.dG.div(p);
  const uint32_t rho = J.dG.mod(p, q);
  const uint64_t pos = J.endc[rho] - J.cu[p];
  const uint64_t o = J.off[p];
  const uint64_t cnt = J.off[p + 1] - o;
  if (pos > J.leaf_rows || cnt > J.leaf_rows - pos) {
    set_error(err, kErrMemoTotal);
    return;
  }
  for (uint64_t t = 0; t < cnt; ++t) {
    const uint32_t* src = J.nat + (o + t) * k;
    if (J.pack == 0) {
      uint32_t* dst = J.leaf + (pos + t) * (k + 1);
      dst[0] = q;
      for (int c = 0; c < k; ++c) dst[1 + c] = src[c];
    } else {
      uint64_t w = uint64_t(q) << J.fshift[0];
      for (int c = 0; c < k; ++c) w |= uint64_t(src[c]) << J.fshift[1 + c];
      if (J.pack == 1) J.leaf[pos + t] = uint32_t(w);
      else reinterpret_cast<uint64_t*>(J.leaf)[pos + t] = w;
    }
  }
}

// One thread per memo row t, in natural order: its element p is the last one
// with off[p] <= t (bisection of the offsets), and its place in the leaf
// layout is end[p mod G] - C_U[p] + (t - off[p]).  Rows of one element are
// adjacent in both layouts, so neighbouring threads read and write
// neighbouring rows, and a long list costs no more than many short ones.
__global__ __launch_bounds__(256) void k_memo_leaf(LeafJob J, int* __restrict__ err) {
  memo_leaf_row(J, uint64_t(blockIdx.x) * 256 + threadIdx.x, err);
}

// Batched: the workgroups of job j are [jobs[j].block0, jobs[j + 1].block0).
__global__ __launch_bounds__(256) void k_memo_leaf_batch(const LeafJob* __restrict__ jobs,
                                                         uint32_t njobs, int* __restrict__ err) {
  uint32_t lo = 0, hi = njobs - 1;  // last job whose block0 <= blockIdx.x
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (jobs[mid].block0 <= blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const LeafJob& J = jobs[lo];
  const uint64_t p64 = uint64_t(blockIdx.x - J.block0) * 256 + threadIdx.x;
  if (p64 > J.n) return;
  memo_leaf_element(J, uint32_t(p64), err);
}

}  // namespace

size_t memo_wave_lds_bytes(int k, uint64_t R, uint32_t W) {
  return (size_t(R) * k + memo_ring_words(k, W)) * sizeof(uint32_t);
}

uint64_t memo_wave_capacity(int k, uint32_t W, size_t lds_bytes) {
  const size_t words = lds_bytes / sizeof(uint32_t);
  const size_t ring = memo_ring_words(k, W);
  return words > ring ? (words - ring) / size_t(k) : 0;
}

hipError_t launch_memo_chain_wave(const uint32_t* h, int k, uint64_t top, uint32_t step,
                                  uint32_t W, uint64_t Rcap, uint64_t Rexp, uint32_t* nat,
                                  uint64_t* off_out, int* err, hipStream_t s) {
  Gens hg{};
  for (int i = 0; i < k; ++i) hg.g[i] = h[i];
  const size_t lds = memo_wave_lds_bytes(k, Rcap, W);
  // The LDS attribute of each instantiation is raised once to the largest size
  // asked for so far (setting it costs as much as a launch).
  static std::mutex attr_mu;
  static std::map<const void*, size_t> attr_lds;
  auto go = [&](auto kern) {
    const void* f = reinterpret_cast<const void*>(kern);
    {
      std::lock_guard<std::mutex> lock(attr_mu);
      size_t& have = attr_lds[f];
      if (lds > have) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        have = lds;
      }
    }
    hipLaunchKernelGGL(kern, dim3(1), dim3(kWave), lds, s, hg, k, uint32_t(top), step, W,
                       uint32_t(Rcap), uint32_t(Rexp), nat, off_out, err);
    return hipGetLastError();
  };
  if (k <= 2) return go(k_memo_chain_wave<2>);
  if (k <= 4) return go(k_memo_chain_wave<4>);
  if (k <= 8) return go(k_memo_chain_wave<8>);
  return go(k_memo_chain_wave<kMaxD>);
}

hipError_t launch_memo_chain_window(const uint32_t* h, int k, uint64_t top, uint32_t step,
                                    uint32_t W, uint32_t hmax, uint32_t cap_rows, uint64_t Rexp,
                                    uint32_t* nat, uint64_t* off_out, int* err, hipStream_t s) {
  Gens hg{};
  for (int i = 0; i < k; ++i) hg.g[i] = h[i];
  const size_t lds = memo_wave_lds_bytes(k, cap_rows, W);
  static std::mutex attr_mu;
  static std::map<const void*, size_t> attr_lds;
  auto go = [&](auto kern) {
    const void* f = reinterpret_cast<const void*>(kern);
    {
      std::lock_guard<std::mutex> lock(attr_mu);
      size_t& have = attr_lds[f];
      if (lds > have) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        have = lds;
      }
    }
    hipLaunchKernelGGL(kern, dim3(1), dim3(kWave), lds, s, hg, k, uint32_t(top), step, W, hmax,
                       cap_rows - 1, uint32_t(Rexp), nat, off_out, err);
    return hipGetLastError();
  };
  if (k <= 2) return go(k_memo_chain_window<2>);
  if (k <= 4) return go(k_memo_chain_window<4>);
  if (k <= 8) return go(k_memo_chain_window<8>);
  return go(k_memo_chain_window<kMaxD>);
}

uint32_t memo_k1_blocks(uint64_t top) { return uint32_t((top + 1 + 255) / 256); }

Memo2 make_memo2(uint32_t h1, uint32_t h2) {
  auto gcd = [](uint32_t a, uint32_t b) {
    while (b) {
      const uint32_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  Memo2 M;
  M.h1 = h1;
  M.h2 = h2;
  M.c = gcd(h1, h2);
  M.h1c = h1 / M.c;
  M.h2c = h2 / M.c;
  // (h1 / c)^{-1} mod (h2 / c) by the extended Euclidean algorithm.
  int64_t t0 = 0, t1 = 1, r0 = M.h2c, r1 = M.h1c % M.h2c;
  while (r1 != 0) {
    const int64_t q = r0 / r1;
    int64_t x = t0 - q * t1;
    t0 = t1;
    t1 = x;
    x = r0 - q * r1;
    r0 = r1;
    r1 = x;
  }
  M.inv = M.h2c == 1 ? 0 : uint32_t(t0 < 0 ? t0 + M.h2c : t0);
  return M;
}

hipError_t launch_memo_k2(uint32_t h1, uint32_t h2, uint64_t top, uint64_t cap, uint32_t* nat,
                          uint64_t* off, uint64_t* cnt, hipStream_t s) {
  if (top == 0 || top >= 0xffffffffull) return hipErrorInvalidValue;
  const Memo2 M = make_memo2(h1, h2);
  const uint32_t blocks = uint32_t((top + 1 + 255) / 256);
  hipLaunchKernelGGL(k_memo2_count, dim3(blocks), dim3(256), 0, s, M, uint32_t(top), cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan(cnt, top + 1, off, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_memo2_fill, dim3(blocks), dim3(256), 0, s, M, uint32_t(top), cap, off, nat);
  return hipGetLastError();
}

hipError_t launch_memo_k1(uint32_t h, uint64_t top, uint64_t R, uint32_t* nat, uint64_t* off,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_memo_k1, dim3(memo_k1_blocks(top)), dim3(256), 0, s, h, uint32_t(top),
                     uint32_t(R), nat, off);
  return hipGetLastError();
}

hipError_t launch_memo_k1_batch(const MemoJob* jobs, uint32_t njobs, uint32_t blocks,
                                hipStream_t s) {
  if (njobs == 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_memo_k1_batch, dim3(blocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

// Average rows per batch up to which every batch runs in one workgroup.
constexpr uint64_t kMemoRowsPerLaunch = 16384;

hipError_t launch_memo_global(const uint32_t* h, int k, uint64_t top, uint32_t b,
                              const uint64_t* off, const uint64_t* ge, uint64_t ge_stride,
                              uint64_t* srcw, uint32_t* nat, int* err, hipStream_t s,
                              uint64_t rows) {
  Gens hg{};
  for (int i = 0; i < k; ++i) hg.g[i] = h[i];
  const uint32_t blocks = uint32_t((top + 255) / 256);
  hipLaunchKernelGGL(k_memo_src, dim3(blocks), dim3(256), 0, s, hg, k, uint32_t(top), off, ge,
                     ge_stride, srcw, nat, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Few rows per batch on average: every batch in one workgroup (a barrier
  // per batch); else one launch per batch over the whole device.
  const uint64_t nbatch = top > 1 ? (top - 2) / b + 1 : 0;
  if (nbatch && rows / nbatch <= kMemoRowsPerLaunch) {
    hipLaunchKernelGGL(k_memo_batches_wg, dim3(1), dim3(1024), 0, s, k, off, uint32_t(top), b,
                       srcw, nat);
    return hipGetLastError();
  }
  for (uint64_t x0 = 1; x0 < top; x0 += b) {
    const uint64_t x1 = (x0 + b < top) ? x0 + b : top;
    hipLaunchKernelGGL(k_memo_batch, dim3(1024), dim3(256), 0, s, k, off, uint32_t(x0),
                       uint32_t(x1), srcw, nat);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

LeafJob make_leaf_job(int k, uint64_t n, uint32_t G, const uint64_t* off, const uint32_t* nat,
                      const uint64_t* cu, const uint64_t* endc, uint32_t* leaf,
                      uint64_t leaf_rows, const EnumParams& P) {
  LeafJob J;
  std::memset(&J, 0, sizeof J);
  J.k = k;
  J.n = uint32_t(n);
  J.dG = DivMod32::make(G);
  J.off = off;
  J.nat = nat;
  J.cu = cu;
  J.endc = endc;
  J.leaf = leaf;
  J.leaf_rows = leaf_rows;
  J.pack = P.pack;
  for (int c = 0; c <= k; ++c) J.fshift[c] = P.fshift[c];
  J.exact = 1;
  return J;
}

hipError_t launch_memo_leaf(const LeafJob& J, int* err, hipStream_t s) {
  const uint64_t blocks = std::max<uint64_t>(1, (J.leaf_rows + 255) / 256);
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_memo_leaf, dim3(uint32_t(blocks)), dim3(256), 0, s, J, err);
  return hipGetLastError();
}

hipError_t launch_memo_leaf_batch(const LeafJob* jobs, uint32_t njobs, uint32_t blocks,
                                  int* err, hipStream_t s) {
  if (njobs == 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_memo_leaf_batch, dim3(blocks), dim3(256), 0, s, jobs, njobs, err);
  return hipGetLastError();
}

template <int KMAX>
hipError_t chain_batch_t(const MemoJob* jobs, uint32_t njobs, size_t lds, int* err,
                         hipStream_t s, bool prepare) {
  auto kern = k_memo_chain_batch<KMAX>;
  if (prepare)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(kern, dim3(njobs), dim3(kWave), lds, s, jobs, err);
  return hipGetLastError();
}

// kmax_class: 8 for k <= 8, 32 otherwise.
hipError_t launch_memo_chain_batch(const MemoJob* jobs, uint32_t njobs, int kmax_class,
                                   size_t lds_bytes, int* err, hipStream_t s, bool prepare) {
  if (njobs == 0) return hipSuccess;
  if (kmax_class <= 8) return chain_batch_t<8>(jobs, njobs, lds_bytes, err, s, prepare);
  return chain_batch_t<kMaxD>(jobs, njobs, lds_bytes, err, s, prepare);
}

}  // namespace zset
