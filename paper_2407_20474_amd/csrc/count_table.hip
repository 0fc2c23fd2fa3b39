// count_table.hip -- the counting pass.
//
// Table rows j = 0..d (0-based generators g_0..g_{d-1}):
//   C[d][x] = [x == 0]
//   C[j][x] = C[j+1][x] + C[j][x - g_j]          (x >= g_j)
// so C[j][x] = |Z(x; g_j..g_{d-1})|, the coefficient of t^x in
// prod_{i >= j} 1/(1 - t^{g_i}) (paper, Section 1).  C[0][n] is |Z(n)|; the
// other rows give every slice's row count, the unranking of slice starts and
// the memo sizes.  Entries saturate at 2^64 - 1, which makes every entry equal
// to min(true value, 2^64 - 1).
//
// Row j is a column-wise inclusive prefix sum of row j+1 viewed as a matrix
// with g_j columns (x = t * g_j + rho): column rho is the residue class
// rho mod g_j.  Tables of at most 16384 entries per row: one workgroup
// computes all rows in LDS with a three-phase blocked scan per row (chunk
// sums, carries per column, rescan), the row sums reduced on the way.  Larger
// tables: one launch per row over all workgroups, every residue class scanned
// at once.  In a batch, each workgroup computes the table of one query.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "zset_internal.h"

namespace zset {

namespace {

constexpr int kCtThreads = 1024;
constexpr int kCtPart = 2048;  // chunk partial sums held in LDS

__device__ inline uint64_t block_max_u64(uint64_t v, uint64_t* red) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    const uint64_t y = __shfl_xor(v, off, kWave);
    v = y > v ? y : v;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kCtThreads / kWave; ++w) t = red[w] > t ? red[w] : t;
  __syncthreads();
  return t;
}

__device__ inline uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v = sat_add_u64(v, __shfl_xor(v, off, kWave));
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kCtThreads / kWave; ++w) t = sat_add_u64(t, red[w]);
  __syncthreads();
  return t;
}

// The whole table by one workgroup in global memory (any N; the batched form
// for tables beyond LDS), with the row sums sums[j] = sum_x C[j][x]
// (saturating) when sums is non-NULL.  `gs` is
// a copy of the generators in LDS.
__device__ void count_table_global(uint64_t* __restrict__ T, uint32_t N, const uint32_t* gs,
                                   int d, uint64_t* __restrict__ sums,
                                   uint64_t* __restrict__ maxes) {
  __shared__ uint64_t part[kCtPart];
  __shared__ uint64_t red[kCtThreads / kWave];
  const int tid = threadIdx.x;
  uint64_t* last = T + size_t(d) * N;
  for (uint64_t x = tid; x < N; x += kCtThreads) last[x] = (x == 0) ? 1 : 0;
  if (tid == 0 && sums) sums[d] = 1;
  if (tid == 0 && maxes) maxes[d] = 1;
  __syncthreads();

  for (int j = d - 1; j >= 0; --j) {
    const uint64_t* __restrict__ U = T + size_t(j + 1) * N;
    uint64_t* __restrict__ V = T + size_t(j) * N;
    const uint32_t G = gs[j];
    uint64_t acc = 0, mx = 0;
    if (G >= N) {  // no x - g_j >= 0: the row is a copy
      for (uint64_t x = tid; x < N; x += kCtThreads) {
        const uint64_t v = U[x];
        V[x] = v;
        acc = sat_add_u64(acc, v);
        mx = v > mx ? v : mx;
      }
    } else {
      const uint32_t rows = uint32_t((uint64_t(N) + G - 1) / G);
      for (uint32_t c0 = 0; c0 < G; c0 += kCtThreads) {
        const uint32_t CG = (G - c0) < uint32_t(kCtThreads) ? (G - c0) : uint32_t(kCtThreads);
        uint32_t B = kCtPart / CG;
        if (B > rows) B = rows;
        if (B < 1) B = 1;
        const uint32_t RB = (rows + B - 1) / B;
        const uint32_t items = B * CG;
        // Phase 1: sum of each (chunk, column).
        for (uint32_t it = tid; it < items; it += kCtThreads) {
          const uint32_t b = it / CG, rho = c0 + it % CG;
          const uint32_t t0 = b * RB;
          const uint32_t t1 = (t0 + RB < rows) ? t0 + RB : rows;
          uint64_t s = 0;
          for (uint32_t t = t0; t < t1; ++t) {
            const uint64_t x = uint64_t(t) * G + rho;
            if (x < N) s = sat_add_u64(s, U[x]);
          }
          part[it] = s;
        }
        __syncthreads();
        // Phase 2: exclusive scan of the chunk sums down each column.
        for (uint32_t col = tid; col < CG; col += kCtThreads) {
          uint64_t run = 0;
          for (uint32_t b = 0; b < B; ++b) {
            const uint64_t v = part[b * CG + col];
            part[b * CG + col] = run;
            run = sat_add_u64(run, v);
          }
        }
        __syncthreads();
        // Phase 3: rescan each chunk from its carry.
        for (uint32_t it = tid; it < items; it += kCtThreads) {
          const uint32_t b = it / CG, rho = c0 + it % CG;
          const uint32_t t0 = b * RB;
          const uint32_t t1 = (t0 + RB < rows) ? t0 + RB : rows;
          uint64_t run = part[it];
          for (uint32_t t = t0; t < t1; ++t) {
            const uint64_t x = uint64_t(t) * G + rho;
            if (x < N) {
              run = sat_add_u64(run, U[x]);
              V[x] = run;
              acc = sat_add_u64(acc, run);
              mx = run > mx ? run : mx;
            }
          }
        }
        __syncthreads();
      }
    }
    const uint64_t total = block_sum_u64(acc, red);
    if (tid == 0 && sums) sums[j] = total;
    const uint64_t top = block_max_u64(mx, red);
    if (tid == 0 && maxes) maxes[j] = top;
    __syncthreads();
  }
}

// The same table with the working row held in LDS (`buf`, N entries).  Row j
// is row j+1 scanned down each residue class mod g_j in place: a class x =
// r, r + g_j, r + 2 g_j, ... is one column of the row viewed as a matrix with
// g_j columns.  Columns of at most kColWalk entries are walked by one thread
// each (neighbouring threads take neighbouring columns).  Longer columns go
// to a segment of 16, 32 or 64 lanes each (2 to 4 short columns share a
// wavefront): lane l takes a run of E consecutive entries of its column,
// scans it in registers, and a segmented inclusive scan of the run totals
// (DPP, no LDS round trip) gives each run its carry; E is odd so that the
// lanes' runs fall in different LDS banks, and a column longer than the
// segment's reach takes several passes with a running carry.  Between rows the workgroup
// synchronises on LDS only: the row's global copy-out need not complete before
// the next row starts.  Row sums and maxima are reduced per wavefront as the
// row is copied and combined once at the end (skipped when neither is asked
// for).  A caller that reads only rows 0..top_row, and row 0 only at its
// entries x = n mod g_0 (mod g_0), passes top_row and row0_class: rows above
// top_row stay in LDS, and row 0 is scanned and stored on that one class.
constexpr uint32_t kCtLdsMax = 16384;
constexpr uint32_t kColWalk = 64;
constexpr uint32_t kColRun = 15;  // longest run per lane (odd)

__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One DPP step on a 64-bit value (lanes outside the pattern read 0).
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = uint32_t(
      __builtin_amdgcn_update_dpp(0, int(uint32_t(v)), CTRL, ROW_MASK, 0xf, false));
  const uint32_t hi = uint32_t(
      __builtin_amdgcn_update_dpp(0, int(uint32_t(v >> 32)), CTRL, ROW_MASK, 0xf, false));
  return (uint64_t(hi) << 32) | lo;
}

// Saturating inclusive prefix sums over segments of `seg` = 16, 32 or 64
// lanes: row_shr 1/2/4/8 inside each 16-lane row, then row_bcast 15 (rows 1
// and 3 add the last lane of rows 0 and 2: 32-lane segments) and row_bcast 31
// (rows 2 and 3 add lane 31: the whole wave).
__device__ inline uint64_t wave_incl_scan_sat_u64(uint64_t v, uint32_t seg) {
  v = sat_add_u64(v, dpp_u64<0x111>(v));
  v = sat_add_u64(v, dpp_u64<0x112>(v));
  v = sat_add_u64(v, dpp_u64<0x114>(v));
  v = sat_add_u64(v, dpp_u64<0x118>(v));
  if (seg >= 32) v = sat_add_u64(v, dpp_u64<0x142, 0xa>(v));
  if (seg >= 64) v = sat_add_u64(v, dpp_u64<0x143, 0xc>(v));
  return v;
}

__device__ __forceinline__ void count_table_lds(uint64_t* __restrict__ T, uint32_t N,
                                                const uint32_t* gs, int d,
                                uint64_t* __restrict__ sums, uint64_t* __restrict__ maxes,
                                uint64_t* buf, uint32_t walk_max = kColWalk,
                                const LastRows* lr = nullptr, int top_row = kMaxD,
                                bool row0_class = false) {
  constexpr int kWaves = kCtThreads / kWave;
  __shared__ uint64_t wsum[kMaxD][kWaves];
  __shared__ uint64_t wmax[kMaxD][kWaves];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const bool closed = lr && lr->on && d >= 2;
  const bool stats = sums || maxes;
  for (uint32_t x = tid; x < N; x += kCtThreads) {
    if (!closed) buf[x] = (x == 0) ? 1 : 0;
    if (d <= top_row) T[size_t(d) * N + x] = (x == 0) ? 1 : 0;
  }
  if (tid == 0 && sums) sums[d] = 1;
  if (tid == 0 && maxes) maxes[d] = 1;
  int jtop = d - 1;
  if (closed) {
    // Rows d-1 and d-2 from their closed forms (LastRows); the scans start
    // at row d-3 from row d-2 in buf.
    uint64_t acc = 0, mx = 0;
    for (uint32_t x = tid; x < N; x += kCtThreads) {
      if (d - 1 <= top_row) T[size_t(d - 1) * N + x] = last_row_divides(*lr, x);
      const uint64_t v = last_row_pair(*lr, x);
      buf[x] = v;
      if (d - 2 <= top_row) T[size_t(d - 2) * N + x] = v;
      acc += v;
      mx = v > mx ? v : mx;
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
      acc += __shfl_xor(acc, off, kWave);
      const uint64_t y = __shfl_xor(mx, off, kWave);
      mx = y > mx ? y : mx;
    }
    if (lane == 0) {
      wsum[d - 2][wave] = acc;
      wmax[d - 2][wave] = mx;
      wsum[d - 1][wave] = wave == 0 ? uint64_t(lr->dg.div(N - 1)) + 1 : 0;
      wmax[d - 1][wave] = wave == 0 ? 1 : 0;
    }
    jtop = d - 3;
  }
  lds_barrier();

  for (int j = jtop; j >= 0; --j) {
    const uint32_t G = gs[j];
    // Row 0 on one class only: the class of n, scanned as the single column
    // of a one-column view (columns r0 + c, c < ncol).
    const bool one = row0_class && j == 0 && G < N;
    const uint32_t r0 = one ? (N - 1) % G : 0u, ncol = one ? 1u : G;
    if (G < N) {  // else no x - g_j >= 0: row j equals row j + 1
      const uint32_t L = (N + G - 1) / G;  // entries of the longest column
      if (L <= walk_max) {
        for (uint32_t rc = tid; rc < ncol; rc += kCtThreads) {
          const uint32_t r = r0 + rc;
          uint64_t run = 0;
          for (uint32_t t0 = 0; t0 < L; t0 += 8) {
            uint64_t v[8];
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q) {
              const uint32_t x = r + (t0 + q) * G;
              v[q] = (t0 + q < L && x < N) ? buf[x] : 0;
            }
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q) {
              const uint32_t x = r + (t0 + q) * G;
              if (t0 + q < L && x < N) {
                run = sat_add_u64(run, v[q]);
                buf[x] = run;
              }
            }
          }
        }
      } else {
        // Segments of `seg` lanes (16, 32 or 64), one column each: the
        // smallest segment whose runs of at most kColRun entries cover the
        // column, so that short columns share a wavefront pass.
        uint32_t seg = 16;
        while (seg < uint32_t(kWave) && seg * kColRun < L) seg *= 2;
        uint32_t E = (L + seg - 1) / seg;
        E = (E < kColRun ? E : kColRun) | 1u;
        const uint32_t span = E * seg;
        const uint32_t passes = (L + span - 1) / span;
        const uint32_t per_wave = uint32_t(kWave) / seg;  // columns per wavefront pass
        const uint32_t sl = uint32_t(lane) % seg, sb = uint32_t(lane) - sl;
        for (uint32_t c0 = uint32_t(wave) * per_wave; c0 < ncol; c0 += kWaves * per_wave) {
          const uint32_t rc = c0 + uint32_t(lane) / seg;
          const uint32_t r = r0 + rc;
          const bool col = rc < ncol;
          uint64_t carry = 0;
          for (uint32_t ps = 0; ps < passes; ++ps) {
            const uint32_t t0 = ps * span + sl * E;
            uint64_t v[kColRun];
#pragma unroll
            for (uint32_t q = 0; q < kColRun; ++q) {
              const uint32_t x = (t0 + q) * G + r;
              v[q] = (col && q < E && x < N) ? buf[x] : 0;
            }
            uint64_t run = 0;
#pragma unroll
            for (uint32_t q = 0; q < kColRun; ++q) {
              run = sat_add_u64(run, v[q]);
              v[q] = run;
            }
            const uint64_t incl = wave_incl_scan_sat_u64(run, seg);
            const uint64_t up = __shfl_up(incl, 1, kWave);
            const uint64_t base = sat_add_u64(carry, sl ? up : 0);
#pragma unroll
            for (uint32_t q = 0; q < kColRun; ++q) {
              const uint32_t x = (t0 + q) * G + r;
              if (col && q < E && x < N) buf[x] = sat_add_u64(base, v[q]);
            }
            carry = sat_add_u64(carry, __shfl(incl, int(sb + seg - 1), kWave));
          }
        }
      }
    }
    lds_barrier();
    if (one) {  // row 0 on the class of n only (no statistics); the last row
      for (uint32_t x = r0 + tid * G; x < N; x += kCtThreads * G) T[x] = buf[x];
      continue;
    }
    uint64_t acc = 0, mx = 0;
    for (uint32_t x = tid; x < N; x += kCtThreads) {
      const uint64_t v = buf[x];
      if (j <= top_row) T[size_t(j) * N + x] = v;
      acc = sat_add_u64(acc, v);
      mx = v > mx ? v : mx;
    }
    if (stats) {
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) {
        acc = sat_add_u64(acc, __shfl_xor(acc, off, kWave));
        const uint64_t y = __shfl_xor(mx, off, kWave);
        mx = y > mx ? y : mx;
      }
      if (lane == 0) {
        wsum[j][wave] = acc;
        wmax[j][wave] = mx;
      }
    }
    lds_barrier();
  }
  if (stats && tid < d) {
    uint64_t s = 0, m = 0;
    for (int w = 0; w < kWaves; ++w) {
      s = sat_add_u64(s, wsum[tid][w]);
      m = wmax[tid][w] > m ? wmax[tid][w] : m;
    }
    if (sums) sums[tid] = s;
    if (maxes) maxes[tid] = m;
  }
}

__global__ __launch_bounds__(kCtThreads) void k_count_table_lds(uint64_t* __restrict__ T,
                                                                uint32_t N, Gens gs, int d,
                                                                uint64_t* __restrict__ sums,
                                                                uint32_t walk_max, LastRows lr) {
  __shared__ uint64_t buf[kCtLdsMax];
  __shared__ uint32_t g[kMaxD];
  if (threadIdx.x < uint32_t(kMaxD)) g[threadIdx.x] = gs.g[threadIdx.x];
  __syncthreads();
  count_table_lds(T, N, g, d, sums, sums ? sums + d + 2 : nullptr, buf, walk_max, &lr);
  if (threadIdx.x == 0 && sums) sums[d + 1] = buf[N - 1];  // |Z(n)| = C[0][n] (row 0 in LDS)
}

// Inclusive prefix sums (saturating) of load(0..count-1) into out, by the
// whole 1024-thread workgroup: rounds of 4096 entries, 4 consecutive entries
// per thread, a DPP scan per wavefront and the wavefront totals in wtot.
template <class Load>
__device__ inline void block_scan_incl_u64(uint32_t count, Load load, uint64_t* __restrict__ out,
                                           uint64_t* wtot) {
  constexpr int kWaves = kCtThreads / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < count; base += kCtThreads * 4) {
    const uint32_t first = base + uint32_t(tid) * 4;
    uint64_t v[4];
    uint64_t run = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      run = sat_add_u64(run, first + q < count ? load(first + q) : 0);
      v[q] = run;
    }
    const uint64_t incl = wave_incl_scan_sat_u64(run, kWave);
    if (lane == kWave - 1) wtot[wave] = incl;
    lds_barrier();
    uint64_t before = carry, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (w < wave) before = sat_add_u64(before, wtot[w]);
      tot = sat_add_u64(tot, wtot[w]);
    }
    const uint64_t up = __shfl_up(incl, 1, kWave);
    before = sat_add_u64(before, lane ? up : 0);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
      if (first + q < count) out[first + q] = sat_add_u64(before, v[q]);
    carry = sat_add_u64(carry, tot);
    lds_barrier();
  }
}

// The first launch of a fixed-k call (SetupJob, zset_internal.h).  Workgroup
// 0: status words, count table, |Z(n)|, then the class ends of the leaf
// layout, end[r] = sum over r' <= r of C_U[pmax(r')] with pmax(r) = r +
// floor((n - r) / G) G the largest element <= n in class r.  Workgroup 1: the
// memo in natural order, off[p] = rows of the elements below p (p = 0..top),
// rows in ascending order of p and, within p, the closed form's order.
__global__ __launch_bounds__(kCtThreads) void k_setup_fixed(SetupJob J) {
  __shared__ uint64_t buf[kCtLdsMax];
  __shared__ uint32_t g[kMaxD];
  __shared__ uint64_t wtot[kCtThreads / kWave];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0) {
    if (tid == 0) {
      J.status[0] = 0;
      J.status[1] = 0;
    }
    if (tid < kMaxD) g[tid] = J.g.g[tid];
    __syncthreads();
    // The rest of the call reads rows 1..U of the table, and row 0 only on
    // the class of n (the slice plan's first coordinate): rows above U stay
    // in LDS, row 0 is scanned on that class, and no row statistics are kept.
    count_table_lds(J.table, J.N, g, J.d, nullptr, nullptr, buf, J.walk, &J.last, J.U,
                    J.U >= 1);
    if (tid == 0) J.sums[J.d + 1] = buf[J.N - 1];
    __syncthreads();  // the table's global rows are visible to the workgroup
    const uint64_t* CU = J.table + uint64_t(J.U) * J.N;
    const uint32_t n = J.N - 1;
    const DivMod32 dG = J.dG;
    block_scan_incl_u64(
        J.nclass,
        [&](uint32_t r) { return CU[uint64_t(r) + uint64_t(dG.div(n - r)) * dG.d]; }, J.endc,
        wtot);
    return;
  }
  if (tid == 0) J.stamps[0] = wall_clock64();
  const uint32_t top = J.N;
  if (J.k == 1) {
    // Memo[p] = {(p / h)} when h divides p (the recurrence's closed solution).
    const uint64_t h = J.h1;
    for (uint32_t i = tid; i <= top; i += kCtThreads) {
      J.off[i] = (uint64_t(i) + h - 1) / h;
      if (i < J.R) {
        J.nat[i] = i;
        J.rowp[i] = uint32_t(i * h);  // row i lists p = i h (i h < top)
      }
    }
  } else {
    uint64_t carry = 0;
    for (uint32_t base = 0; base <= top; base += kCtThreads * 4) {
      const uint32_t first = base + uint32_t(tid) * 4;
      uint32_t m0[4], rows[4];
      uint64_t ex[4];
      uint64_t run = 0;
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t p = first + q;
        rows[q] = 0;
        m0[q] = 0;
        if (p < top) (void)memo2_first(J.M, p, &m0[q], &rows[q]);  // element top: no rows
        ex[q] = run;
        run += rows[q];
      }
      constexpr int kWaves = kCtThreads / kWave;
      const int lane = tid & (kWave - 1), wave = tid / kWave;
      const uint64_t incl = wave_incl_scan_sat_u64(run, kWave);
      if (lane == kWave - 1) wtot[wave] = incl;
      lds_barrier();
      uint64_t before = carry, tot = 0;
      for (int w = 0; w < kWaves; ++w) {
        if (w < wave) before += wtot[w];
        tot += wtot[w];
      }
      const uint64_t up = __shfl_up(incl, 1, kWave);
      before += lane ? up : 0;
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t p = first + q;
        if (p > top) break;
        const uint64_t o = before + ex[q];
        J.off[p] = o;
        for (uint32_t t = 0; t < rows[q] && o + t < J.R; ++t) {
          const uint32_t m1 = m0[q] + t * J.M.h2c;
          J.nat[(o + t) * 2] = m1;
          J.nat[(o + t) * 2 + 1] = (p - m1 * J.M.h1) / J.M.h2;
          J.rowp[o + t] = p;
        }
      }
      carry += tot;
      lds_barrier();
    }
  }
  __syncthreads();
  if (tid == 0) J.stamps[1] = wall_clock64();
}

// ---------------------------------------------------------------------------
// Tables beyond LDS (n + 1 > kCtLdsMax): one launch per row, all workgroups.
// Row j's residue classes mod g_j are independent prefix sums of row j+1, so
// a launch scans every class at once: classes of at most kShortClass entries
// one per thread, longer ones one per workgroup (a blocked scan in tiles of
// 1024 entries).  Row sums and maxima follow in one launch, a workgroup per
// chunk of 32768 entries of each row.
constexpr int kRowThreads = 256;
constexpr uint32_t kShortClass = 64;

// Row d = [x == 0]; the sums and maxima start clear (the stats launch adds
// into them).
__global__ __launch_bounds__(kRowThreads) void k_count_init(uint64_t* __restrict__ T, uint32_t N,
                                                            int d, uint64_t* __restrict__ sums,
                                                            LastRows lr) {
  const uint64_t i = uint64_t(blockIdx.x) * kRowThreads + threadIdx.x;
  uint64_t* last = T + uint64_t(d) * N;
  const bool closed = lr.on && d >= 2;
  for (uint64_t x = i; x < N; x += uint64_t(gridDim.x) * kRowThreads) {
    last[x] = (x == 0) ? 1 : 0;
    if (closed) {  // rows d-1 and d-2 in closed form (LastRows)
      T[uint64_t(d - 1) * N + x] = last_row_divides(lr, uint32_t(x));
      T[uint64_t(d - 2) * N + x] = last_row_pair(lr, uint32_t(x));
    }
  }
  if (sums && i < uint64_t(2 * d + 3)) sums[i] = 0;
}

__device__ inline void sat_atomic_add(uint64_t* p, uint64_t v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const unsigned long long seen = atomicCAS(q, old, sat_add_u64(old, v));
    if (seen == old) break;
    old = seen;
  }
}

// Row sums and maxima: workgroup (c, j) reduces chunk c of row j and adds its
// result into sums[j] and sums[d + 2 + j] (a saturating compare-and-swap and
// an atomic maximum, a few dozen per word); also |Z(n)| = C[0][n].
constexpr uint32_t kStatsChunk = 1 << 15;
__global__ __launch_bounds__(kCtThreads) void k_count_stats(const uint64_t* __restrict__ T,
                                                            uint32_t N, int d,
                                                            uint64_t* __restrict__ sums) {
  __shared__ uint64_t red[kCtThreads / kWave];
  const int j = blockIdx.y;
  const uint64_t* V = T + uint64_t(j) * N;
  const uint64_t lo = uint64_t(blockIdx.x) * kStatsChunk;
  const uint64_t hi = std::min<uint64_t>(N, lo + kStatsChunk);
  uint64_t acc = 0, mx = 0;
  for (uint64_t x = lo + threadIdx.x; x < hi; x += kCtThreads) {
    const uint64_t v = V[x];
    acc = sat_add_u64(acc, v);
    mx = v > mx ? v : mx;
  }
  const uint64_t total = block_sum_u64(acc, red);
  const uint64_t top = block_max_u64(mx, red);
  if (threadIdx.x == 0) {
    sat_atomic_add(sums + j, total);
    atomicMax(reinterpret_cast<unsigned long long*>(sums + d + 2 + j),
              static_cast<unsigned long long>(top));
    if (j == 0 && hi == N) sums[d + 1] = V[N - 1];
  }
}

// Row j from row j + 1, one thread per residue class (classes of at most
// kShortClass entries, or g_j >= N: a copy).
__global__ __launch_bounds__(kRowThreads) void k_count_row_short(uint64_t* __restrict__ T,
                                                                 uint32_t N, uint32_t G, int j) {
  const uint64_t rho = uint64_t(blockIdx.x) * kRowThreads + threadIdx.x;
  const uint64_t* U = T + uint64_t(j + 1) * N;
  uint64_t* V = T + uint64_t(j) * N;
  if (rho < G && rho < N) {
    uint64_t run = 0;
    for (uint64_t x = rho; x < N; x += G) {
      run = sat_add_u64(run, U[x]);
      V[x] = run;
    }
  }
}

// Row j from row j + 1, one workgroup per residue class (longer classes).
__global__ __launch_bounds__(kRowThreads) void k_count_row_long(uint64_t* __restrict__ T,
                                                                uint32_t N, uint32_t G, int j) {
  __shared__ uint64_t wsum[kRowThreads / kWave];
  const uint32_t rho = blockIdx.x;
  const uint64_t L = (uint64_t(N) - rho + G - 1) / G;  // entries of the class
  const uint64_t* U = T + uint64_t(j + 1) * N;
  uint64_t* V = T + uint64_t(j) * N;
  constexpr uint32_t kItems = 4;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < L; base += uint64_t(kRowThreads) * kItems) {
    const uint64_t t0 = base + uint64_t(threadIdx.x) * kItems;
    uint64_t v[kItems];
    uint64_t local = 0;
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
      v[q] = (t0 + q < L) ? U[rho + (t0 + q) * G] : 0;
      local = sat_add_u64(local, v[q]);
    }
    // Exclusive scan of the threads' sums: in the wavefront, then across.
    uint64_t incl = local;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint64_t y = __shfl_up(incl, off, kWave);
      if (lane >= off) incl = sat_add_u64(incl, y);
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    uint64_t before = carry, total = carry;
    for (int w = 0; w < kRowThreads / kWave; ++w) {
      if (w < wave) before = sat_add_u64(before, wsum[w]);
      total = sat_add_u64(total, wsum[w]);
    }
    __syncthreads();
    const uint64_t prev = __shfl_up(incl, 1, kWave);  // the previous lane's inclusive sum
    uint64_t run = sat_add_u64(before, lane ? prev : 0);
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
      if (t0 + q < L) {
        run = sat_add_u64(run, v[q]);
        V[rho + (t0 + q) * G] = run;
      }
    }
    carry = total;
  }
}

// Batched forms: workgroup b computes the table of jobs[first + b], and
// writes |Z(n)| = C[0][n] to its `total`.
__device__ inline void load_job(const CountJob* __restrict__ jobs, uint32_t* g, uint64_t** T,
                                uint32_t* N, int* d, uint64_t** sums, uint64_t** total) {
  const CountJob& J = jobs[blockIdx.x];
  if (threadIdx.x < uint32_t(kMaxD)) g[threadIdx.x] = J.g[threadIdx.x];
  *T = J.table;
  *N = J.N;
  *d = J.d;
  *sums = J.sums;
  *total = J.total;
  __syncthreads();
}

__global__ __launch_bounds__(kCtThreads) void k_count_table_batch_lds(
    const CountJob* __restrict__ jobs) {
  extern __shared__ __align__(16) uint64_t dyn_buf[];
  __shared__ uint32_t g[kMaxD];
  uint64_t *T, *sums, *total;
  uint32_t N;
  int d;
  load_job(jobs, g, &T, &N, &d, &sums, &total);
  count_table_lds(T, N, g, d, sums, nullptr, dyn_buf);
  if (threadIdx.x == 0) *total = dyn_buf[N - 1];  // row 0 in LDS
}

__global__ __launch_bounds__(kCtThreads) void k_count_table_batch_global(
    const CountJob* __restrict__ jobs) {
  __shared__ uint32_t g[kMaxD];
  uint64_t *T, *sums, *total;
  uint32_t N;
  int d;
  load_job(jobs, g, &T, &N, &d, &sums, &total);
  count_table_global(T, N, g, d, sums, nullptr);
  __syncthreads();
  if (threadIdx.x == 0) *total = T[N - 1];
}

}  // namespace

hipError_t launch_count_table(uint64_t* table, uint64_t n, const uint32_t* gens, int d,
                              uint64_t* sums, hipStream_t s) {
  Gens gs{};
  for (int i = 0; i < d; ++i) gs.g[i] = gens[i];
  const uint32_t N = uint32_t(n + 1);
  // ZSET_COUNT_PATH=rows takes the one-launch-per-row form at any size (tests).
  const char* path = std::getenv("ZSET_COUNT_PATH");
  const bool rows_form = path && std::strcmp(path, "rows") == 0;
  LastRows lr{};
  if (count_last_rows_enabled()) lr = make_last_rows(gens, d);
  if (N <= kCtLdsMax && !rows_form) {
    const char* we = std::getenv("ZSET_COUNT_WALK");
    const uint32_t walk = we ? uint32_t(std::atoi(we)) : kColWalk;
    hipLaunchKernelGGL(k_count_table_lds, dim3(1), dim3(kCtThreads), 0, s, table, N, gs, d, sums,
                       walk, lr);
  } else {
    const uint32_t ib = uint32_t(std::min<uint64_t>((uint64_t(N) + kRowThreads - 1) / kRowThreads,
                                                    4096));
    hipLaunchKernelGGL(k_count_init, dim3(ib), dim3(kRowThreads), 0, s, table, N, d, sums, lr);
    for (int j = lr.on ? d - 3 : d - 1; j >= 0; --j) {
      const uint32_t G = gs.g[j];
      const uint64_t classes = std::min<uint64_t>(G, N);
      const uint64_t len = (uint64_t(N) + G - 1) / G;
      if (len <= kShortClass) {
        hipLaunchKernelGGL(k_count_row_short, dim3(uint32_t((classes + kRowThreads - 1) / kRowThreads)),
                           dim3(kRowThreads), 0, s, table, N, G, j);
      } else {
        hipLaunchKernelGGL(k_count_row_long, dim3(uint32_t(classes)), dim3(kRowThreads), 0, s,
                           table, N, G, j);
      }
    }
    if (sums) {
      const uint32_t chunks = uint32_t((uint64_t(N) + kStatsChunk - 1) / kStatsChunk);
      hipLaunchKernelGGL(k_count_stats, dim3(chunks, uint32_t(d + 1)), dim3(kCtThreads), 0, s,
                         table, N, d, sums);
    }
  }
  return hipGetLastError();
}

uint32_t count_table_lds_max() { return kCtLdsMax; }

bool count_last_rows_enabled() {
  const char* e = std::getenv("ZSET_COUNT_LAST");
  return !(e && std::strcmp(e, "0") == 0);
}

LastRows make_last_rows(const uint32_t* gens, int d) {
  LastRows L;
  std::memset(&L, 0, sizeof L);
  if (d < 2) return L;
  const Memo2 M = make_memo2(gens[d - 2], gens[d - 1]);
  if (M.h2c >= (1u << 16)) return L;
  L.on = 1;
  L.inv = M.inv;
  L.dg = DivMod32::make(gens[d - 1]);
  L.dc = DivMod32::make(M.c);
  L.dh1c = DivMod32::make(M.h1c);
  L.dh2c = DivMod32::make(M.h2c);
  return L;
}

hipError_t launch_setup_fixed(const SetupJob& J, hipStream_t s) {
  if (J.N == 0 || J.N > kCtLdsMax || (J.k != 1 && J.k != 2) || J.d < 2 || J.U < 0 ||
      J.U >= J.d || J.nclass == 0 || J.nclass > J.N || !J.rowp || !J.nat || !J.off)
    return hipErrorInvalidValue;
  SetupJob j = J;
  if (j.walk == 0) {
    const char* we = std::getenv("ZSET_COUNT_WALK");
    j.walk = we ? uint32_t(std::atoi(we)) : kColWalk;
  }
  hipLaunchKernelGGL(k_setup_fixed, dim3(2), dim3(kCtThreads), 0, s, j);
  return hipGetLastError();
}

hipError_t prepare_count_table_batch(uint32_t max_lds_n) {
  const size_t bytes = size_t(max_lds_n) * sizeof(uint64_t);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_count_table_batch_lds),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

hipError_t launch_count_table_batch(const CountJob* jobs, uint32_t njobs, uint32_t max_lds_n,
                                    bool lds, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  if (lds) {
    const size_t bytes = size_t(max_lds_n) * sizeof(uint64_t);
    hipLaunchKernelGGL(k_count_table_batch_lds, dim3(njobs), dim3(kCtThreads), bytes, s, jobs);
  } else {
    hipLaunchKernelGGL(k_count_table_batch_global, dim3(njobs), dim3(kCtThreads), 0, s, jobs);
  }
  return hipGetLastError();
}

}  // namespace zset
