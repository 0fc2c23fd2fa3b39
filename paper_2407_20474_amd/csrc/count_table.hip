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
// rho mod g_j.  One workgroup computes all rows with a three-phase blocked scan
// per row (chunk sums, carries per column, rescan), which keeps every load
// coalesced across adjacent residues.
#include "zset_internal.h"

namespace zset {

namespace {

constexpr int kCtThreads = 1024;
constexpr int kCtPart = 2048;  // chunk partial sums held in LDS

__global__ __launch_bounds__(kCtThreads) void k_count_table(uint64_t* __restrict__ T,
                                                            uint32_t N, Gens gs, int d) {
  __shared__ uint64_t part[kCtPart];
  const int tid = threadIdx.x;
  uint64_t* last = T + size_t(d) * N;
  for (uint64_t x = tid; x < N; x += kCtThreads) last[x] = (x == 0) ? 1 : 0;
  __syncthreads();

  for (int j = d - 1; j >= 0; --j) {
    const uint64_t* __restrict__ U = T + size_t(j + 1) * N;
    uint64_t* __restrict__ V = T + size_t(j) * N;
    const uint32_t G = gs.g[j];
    if (G >= N) {  // no x - g_j >= 0: the row is a copy
      for (uint64_t x = tid; x < N; x += kCtThreads) V[x] = U[x];
      __syncthreads();
      continue;
    }
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
          }
        }
      }
      __syncthreads();
    }
  }
}

// The same table with the working row held in LDS (n + 1 <= kCtLdsMax): each
// row is transformed in place from row j+1 into row j by the three-phase
// column scan, copied out with coalesced stores, and summed on the way
// (sums[j] = sum_x C[j][x], saturating).
constexpr uint32_t kCtLdsMax = 16384;

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

__global__ __launch_bounds__(kCtThreads) void k_count_table_lds(uint64_t* __restrict__ T,
                                                                uint32_t N, Gens gs, int d,
                                                                uint64_t* __restrict__ sums) {
  __shared__ uint64_t buf[kCtLdsMax];
  __shared__ uint64_t part[kCtPart];
  __shared__ uint64_t red[kCtThreads / kWave];
  const int tid = threadIdx.x;
  for (uint32_t x = tid; x < N; x += kCtThreads) {
    buf[x] = (x == 0) ? 1 : 0;
    T[size_t(d) * N + x] = (x == 0) ? 1 : 0;
  }
  if (tid == 0 && sums) sums[d] = 1;
  __syncthreads();

  for (int j = d - 1; j >= 0; --j) {
    const uint32_t G = gs.g[j];
    if (G < N) {
      const uint32_t rows = (N + G - 1) / G;
      for (uint32_t c0 = 0; c0 < G; c0 += kCtThreads) {
        const uint32_t CG = (G - c0) < uint32_t(kCtThreads) ? (G - c0) : uint32_t(kCtThreads);
        // At most 64 chunks per column, so that one wavefront scans a column's
        // chunk sums in one pass.
        uint32_t B = kCtPart / CG;
        if (B > uint32_t(kWave)) B = kWave;
        if (B > rows) B = rows;
        if (B < 1) B = 1;
        const uint32_t RB = (rows + B - 1) / B;
        const uint32_t items = B * CG;
        for (uint32_t it = tid; it < items; it += kCtThreads) {
          const uint32_t b = it / CG, rho = c0 + it % CG;
          const uint32_t t0 = b * RB;
          const uint32_t t1 = (t0 + RB < rows) ? t0 + RB : rows;
          uint64_t acc = 0;
#pragma unroll 8
          for (uint32_t t = t0; t < t1; ++t) {
            const uint32_t x = t * G + rho;
            if (x < N) acc = sat_add_u64(acc, buf[x]);
          }
          part[it] = acc;
        }
        __syncthreads();
        {
          const int wave = tid / kWave, lane = tid & (kWave - 1);
          for (uint32_t col = wave; col < CG; col += kCtThreads / kWave) {
            const uint64_t v = uint32_t(lane) < B ? part[lane * CG + col] : 0;
            uint64_t incl = v;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
              const uint64_t y = __shfl_up(incl, off, kWave);
              if (lane >= off) incl = sat_add_u64(incl, y);
            }
            const uint64_t up = __shfl_up(incl, 1, kWave);
            if (uint32_t(lane) < B) part[lane * CG + col] = lane ? up : 0;
          }
        }
        __syncthreads();
        for (uint32_t it = tid; it < items; it += kCtThreads) {
          const uint32_t b = it / CG, rho = c0 + it % CG;
          const uint32_t t0 = b * RB;
          const uint32_t t1 = (t0 + RB < rows) ? t0 + RB : rows;
          uint64_t run = part[it];
          // Read a group of the chunk's entries before writing any back.
          constexpr uint32_t kGroup = 8;
          for (uint32_t t = t0; t < t1; t += kGroup) {
            uint64_t v[kGroup];
#pragma unroll
            for (uint32_t q = 0; q < kGroup; ++q) {
              const uint32_t x = (t + q) * G + rho;
              v[q] = (t + q < t1 && x < N) ? buf[x] : 0;
            }
#pragma unroll
            for (uint32_t q = 0; q < kGroup; ++q) {
              const uint32_t x = (t + q) * G + rho;
              if (t + q < t1 && x < N) {
                run = sat_add_u64(run, v[q]);
                buf[x] = run;
              }
            }
          }
        }
        __syncthreads();
      }
    }
    uint64_t acc = 0;
    for (uint32_t x = tid; x < N; x += kCtThreads) {
      const uint64_t v = buf[x];
      T[size_t(j) * N + x] = v;
      acc = sat_add_u64(acc, v);
    }
    const uint64_t total = block_sum_u64(acc, red);
    if (tid == 0 && sums) sums[j] = total;
  }
}

// Saturating sum of each table row: sums[j] = sum_x C[j][x].
__global__ __launch_bounds__(256) void k_row_sums(const uint64_t* __restrict__ T, uint32_t N,
                                                  uint64_t* __restrict__ sums) {
  __shared__ uint64_t red[256];
  const uint64_t* row = T + size_t(blockIdx.x) * N;
  uint64_t s = 0;
  for (uint64_t x = threadIdx.x; x < N; x += 256) s = sat_add_u64(s, row[x]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = sat_add_u64(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

}  // namespace

hipError_t launch_count_table(uint64_t* table, uint64_t n, const uint32_t* gens, int d,
                              uint64_t* sums, hipStream_t s) {
  Gens gs{};
  for (int i = 0; i < d; ++i) gs.g[i] = gens[i];
  const uint32_t N = uint32_t(n + 1);
  if (N <= kCtLdsMax) {
    hipLaunchKernelGGL(k_count_table_lds, dim3(1), dim3(kCtThreads), 0, s, table, N, gs, d, sums);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_count_table, dim3(1), dim3(kCtThreads), 0, s, table, N, gs, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sums) return e;
  hipLaunchKernelGGL(k_row_sums, dim3(d + 1), dim3(256), 0, s, table, N, sums);
  return hipGetLastError();
}

}  // namespace zset
