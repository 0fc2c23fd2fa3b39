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
// k_write: one wavefront per slice.  The first U-1 coordinates are the outer
// prefix, kept lane-distributed (lane j holds a_j) and advanced by an odometer
// in ascending lex order (Alg 3.1's successor, mirrored).  Coordinate U-1 is
// spread across the 64 lanes.  Then:
//  * k = 0 (MODE 0, Alg 3.1): the last coordinate is solved by division; each
//    lane is a candidate giving 0 or 1 row; a ballot plus mbcnt gives each
//    valid lane its output row.
//  * k >= 1 (MODE 1, Alg 3.2): each lane owns the segment of rows sharing its
//    prefix, which is one contiguous run of the leaf-order memo (memo.hip) of
//    length C[U][x].  A wave prefix sum of the segment lengths gives row
//    offsets; rows are then produced 64 at a time, each lane finding its
//    segment by bisection over the prefix sums and copying one memo row.
// Rows are staged in a per-wave LDS ring and written to HBM 128 rows at a time
// with 16-byte stores, so the global stores are fully coalesced for any d.
// In count-only mode no row is stored: each row's FNV-1a-64 (rank, row) hash is
// summed instead.
#include "zset_internal.h"

namespace zset {

namespace {

constexpr uint32_t kRingRows = 256;   // rows per wave in the LDS ring
constexpr uint32_t kFlushRows = 128;  // rows per coalesced flush

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

// Slice start: first U coordinates and the offset t0 inside their block.
__global__ __launch_bounds__(256) void k_plan(EnumParams P) {
  const uint64_t tile = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (tile >= P.ntiles) return;
  const uint64_t N = uint64_t(P.n) + 1;
  uint64_t r = tile * P.rows_per_tile;
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

template <bool ALIGN16>
__device__ inline void flush_rows(const uint32_t* stage, uint32_t slot0, uint32_t rows, int d,
                                  uint32_t* out_rows) {
  const uint32_t nd = rows * uint32_t(d);
  const uint32_t* src = stage + slot0 * uint32_t(d);
  const int lane = lane_id();
  if (ALIGN16) {
    const uint32_t nd4 = nd & ~3u;
    for (uint32_t v = uint32_t(lane) * 4; v < nd4; v += kWave * 4) {
      const uint4 val = *reinterpret_cast<const uint4*>(src + v);
      *reinterpret_cast<uint4*>(out_rows + v) = val;
    }
    for (uint32_t v = nd4 + lane; v < nd; v += kWave) out_rows[v] = src[v];
  } else {
    for (uint32_t v = lane; v < nd; v += kWave) out_rows[v] = src[v];
  }
}

template <int MODE, bool COUNT_ONLY, bool ALIGN16>
__global__ __launch_bounds__(256) void k_write(EnumParams P) {
  extern __shared__ uint32_t stage_all[];
  const int lane = lane_id();
  const int wave = int(threadIdx.x / kWave);
  const int waves = int(blockDim.x / kWave);
  const uint64_t tile = uint64_t(blockIdx.x) * waves + wave;
  if (tile >= P.ntiles) return;

  const int d = P.d, U = P.U, k = P.k;
  const uint64_t N = uint64_t(P.n) + 1;
  uint32_t* stage = stage_all + size_t(wave) * kRingRows * d;
  const uint64_t r0 = tile * P.rows_per_tile;
  const uint64_t left = P.total - r0;
  const uint32_t target = uint32_t(left < P.rows_per_tile ? left : P.rows_per_tile);

  // Slice start, lane-distributed: lane j < U holds a_j and the remainder
  // after coordinate j.
  const uint32_t* st = P.tiles + tile * uint64_t(U + 2);
  uint32_t aj = lane < U ? st[lane] : 0;
  const uint32_t gj = lane < d ? P.g.g[lane] : 0;
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
  const int nouter = U >= 1 ? U - 1 : 0;  // coordinates 0..U-2 form the outer prefix
  uint32_t xouter = (U >= 2) ? readlane_u32(remj, U - 2) : P.n;
  uint32_t aseg = (U >= 1) ? readlane_u32(aj, U - 1) : 0;
  const uint32_t gseg = (U >= 1) ? P.g.g[U - 1] : 0;
  const uint64_t* cnt_row = P.table + uint64_t(U) * N;

  uint32_t produced = 0, flushed = 0;
  uint64_t csum = 0;
  bool first = true;
  bool single_done = false;
  uint32_t* out_tile = P.out + r0 * uint64_t(d);

  while (produced < target) {
    const uint32_t remaining = target - produced;
    const uint32_t A = aseg + uint32_t(lane);
    bool ok;
    uint32_t xs;
    if (U >= 1) {
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
      if (valid && pos < tot) {
        if (COUNT_ONLY) {
          uint64_t h = fnv1a_u64(kFnvOffset, r0 + produced + pos);
          for (int j = 0; j < nouter; ++j) h = fnv1a_u32(h, readlane_u32(aj, j));
          h = fnv1a_u32(h, A);
          h = fnv1a_u32(h, qx);
          csum += h;
        } else {
          uint32_t* row = stage + ((produced + pos) & (kRingRows - 1)) * uint32_t(d);
          for (int j = 0; j < nouter; ++j) row[j] = readlane_u32(aj, j);
          row[U - 1] = A;
          row[U] = qx;
        }
      }
      if (!COUNT_ONLY) {
        wave_sync();
        uint32_t written = produced + tot;
        while (written - flushed >= kFlushRows) {
          flush_rows<ALIGN16>(stage, flushed & (kRingRows - 1), kFlushRows, d,
                              out_tile + uint64_t(flushed) * d);
          flushed += kFlushRows;
        }
        wave_sync();
      }
    } else {
      uint64_t c = ok ? cnt_row[xs] : 0;
      const uint32_t rx = P.dG.mod(xs, qx);
      uint64_t start = ok ? P.endc[rx] - c : 0;
      if (first && lane == 0) {
        if (t0 >= c) {  // the plan guarantees t0 < c; refuse to read past the segment
          set_error(P.err, kErrUnrank);
          c = 0;
        } else {
          start += t0;
          c -= t0;
        }
      }
      const uint32_t c32 = uint32_t(c < remaining ? c : remaining);
      // Inclusive prefix sum saturated at `remaining`.
      uint32_t incl = c32;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, kWave);
        if (lane >= off) {
          const uint32_t s = incl + y;
          incl = s < remaining ? s : remaining;
        }
      }
      const uint32_t up = __shfl_up(incl, 1, kWave);
      const uint32_t excl = lane ? up : 0;
      tot = readlane_u32(incl, kWave - 1);
      const int ms = k + 1;
      for (uint32_t beta = 0; beta < tot; beta += kWave) {
        const uint32_t rho = beta + uint32_t(lane);
        const bool act = rho < tot;
        // Segment of this row: the number of lanes whose inclusive sum is <= rho.
        int owner = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const uint32_t v = __shfl(incl, owner + step - 1, kWave);
          if (v <= rho) owner += step;
        }
        owner = owner < kWave ? owner : kWave - 1;
        const uint32_t o_excl = __shfl(excl, owner, kWave);
        const uint64_t o_start = __shfl(start, owner, kWave);
        const uint32_t o_qx = __shfl(qx, owner, kWave);
        const uint32_t o_A = aseg + uint32_t(owner);
        const uint64_t mrow = o_start + (rho - o_excl);
        if (act && mrow >= P.leaf_rows) {
          set_error(P.err, kErrTileRows);
        } else if (act) {
          const uint32_t* mr = P.leaf + mrow * ms;
          const uint32_t aU = o_qx - mr[0];
          if (COUNT_ONLY) {
            uint64_t h = fnv1a_u64(kFnvOffset, r0 + produced + rho);
            for (int j = 0; j < nouter; ++j) h = fnv1a_u32(h, readlane_u32(aj, j));
            if (U >= 1) h = fnv1a_u32(h, o_A);
            h = fnv1a_u32(h, aU);
            for (int c2 = 0; c2 < k; ++c2) h = fnv1a_u32(h, mr[1 + c2]);
            csum += h;
          } else {
            uint32_t* row = stage + ((produced + rho) & (kRingRows - 1)) * uint32_t(d);
            for (int j = 0; j < nouter; ++j) row[j] = readlane_u32(aj, j);
            if (U >= 1) row[U - 1] = o_A;
            row[U] = aU;
            for (int c2 = 0; c2 < k; ++c2) row[U + 1 + c2] = mr[1 + c2];
          }
        }
        if (!COUNT_ONLY) {
          wave_sync();
          const uint32_t nrows = (tot - beta) < uint32_t(kWave) ? (tot - beta) : uint32_t(kWave);
          const uint32_t written = produced + beta + nrows;
          while (written - flushed >= kFlushRows) {
            flush_rows<ALIGN16>(stage, flushed & (kRingRows - 1), kFlushRows, d,
                                out_tile + uint64_t(flushed) * d);
            flushed += kFlushRows;
          }
          wave_sync();
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
    if (uint64_t(aseg + kWave) * gseg <= xouter) {
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
  }

  if (!COUNT_ONLY) {
    if (produced > flushed) {
      flush_rows<ALIGN16>(stage, flushed & (kRingRows - 1), produced - flushed, d,
                          out_tile + uint64_t(flushed) * d);
    }
  } else {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) csum += __shfl_xor(csum, off, kWave);
    if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(P.checksum),
                             static_cast<unsigned long long>(csum));
  }
  if (lane == 0 && produced != target) set_error(P.err, kErrTileRows);
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

// Reverse the order of `rows` rows of d dwords in place (descending output).
__global__ __launch_bounds__(256) void k_reverse_rows(uint32_t* out, uint64_t rows, int d) {
  const uint64_t half = rows / 2;
  const uint64_t total = half * uint64_t(d);
  for (uint64_t w = uint64_t(blockIdx.x) * 256 + threadIdx.x; w < total;
       w += uint64_t(gridDim.x) * 256) {
    const uint64_t r = w / d, c = w % d;
    uint32_t* a = out + r * d + c;
    uint32_t* b = out + (rows - 1 - r) * d + c;
    const uint32_t t = *a;
    *a = *b;
    *b = t;
  }
}

template <int MODE, bool COUNT_ONLY, bool ALIGN16>
hipError_t launch_write_t(const EnumParams& P, int waves, hipStream_t s) {
  const uint64_t blocks = (P.ntiles + waves - 1) / waves;
  const size_t lds = COUNT_ONLY ? 0 : size_t(waves) * kRingRows * P.d * sizeof(uint32_t);
  hipLaunchKernelGGL((k_write<MODE, COUNT_ONLY, ALIGN16>), dim3(uint32_t(blocks)),
                     dim3(waves * kWave), lds, s, P);
  return hipGetLastError();
}

}  // namespace

uint32_t write_ring_rows() { return kRingRows; }
uint32_t write_flush_rows() { return kFlushRows; }

hipError_t launch_plan(const EnumParams& P, hipStream_t s) {
  const uint64_t blocks = (P.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_plan, dim3(uint32_t(blocks)), dim3(256), 0, s, P);
  return hipGetLastError();
}

int write_waves_per_block(int d) { return d <= 12 ? 4 : 2; }

hipError_t launch_write(const EnumParams& P, bool count_only, bool align16, hipStream_t s) {
  const int waves = write_waves_per_block(P.d);
  if (P.k == 0) {
    if (count_only) return launch_write_t<0, true, false>(P, waves, s);
    return align16 ? launch_write_t<0, false, true>(P, waves, s)
                   : launch_write_t<0, false, false>(P, waves, s);
  }
  if (count_only) return launch_write_t<1, true, false>(P, waves, s);
  return align16 ? launch_write_t<1, false, true>(P, waves, s)
                 : launch_write_t<1, false, false>(P, waves, s);
}

hipError_t launch_single(uint64_t n, uint32_t g, uint32_t* out, bool count_only,
                         uint64_t* checksum, hipStream_t s) {
  hipLaunchKernelGGL(k_single, dim3(1), dim3(64), 0, s, uint32_t(n), g, out, int(count_only),
                     checksum);
  return hipGetLastError();
}

hipError_t launch_reverse(uint32_t* out, uint64_t rows, int d, hipStream_t s) {
  uint64_t blocks = (rows / 2 * uint64_t(d) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reverse_rows, dim3(uint32_t(blocks)), dim3(256), 0, s, out, rows, d);
  return hipGetLastError();
}

}  // namespace zset
