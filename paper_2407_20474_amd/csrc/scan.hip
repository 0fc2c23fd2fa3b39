// scan.hip -- single-workgroup prefix sums used to lay out the memo.
//
//  * k_exclusive_scan: natural memo offsets, off[p] = sum_{p' < p} |Z(p'; h)|
//    (the "pre-assigned output locations" of Section 2.3).
//  * k_class_ends: ends of the residue classes of the leaf-order memo layout
//    (see memo.hip): end[rho] = sum_{r <= rho} C_U[pmax(r)], with
//    pmax(r) = r + floor((n - r) / G) * G the largest element <= n in class r.
// Sums saturate at 2^64 - 1 (values used downstream are all below |Z(n)|).
#include "zset_internal.h"

namespace zset {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;

__device__ inline uint64_t wave_inclusive_scan_u64(uint64_t v, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t y = __shfl_up(v, off, kWave);
    if (lane >= off) v = sat_add_u64(v, y);
  }
  return v;
}

// Exclusive scan of one value per thread over a 1024-thread block.
__device__ inline uint64_t block_exclusive_scan_u64(uint64_t v, uint64_t* wsum, uint64_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const uint64_t incl = wave_inclusive_scan_u64(v, lane);
  const uint64_t prev = __shfl_up(incl, 1, kWave);
  const uint64_t excl = lane ? prev : 0;
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int nw = kScanThreads / kWave;
    uint64_t w = lane < nw ? wsum[lane] : 0;
    w = wave_inclusive_scan_u64(w, lane);
    if (lane < nw) wsum[lane] = w;
  }
  __syncthreads();
  const uint64_t before = wave ? wsum[wave - 1] : 0;
  *total = wsum[kScanThreads / kWave - 1];
  __syncthreads();
  return sat_add_u64(before, excl);
}

template <class Load>
__device__ void scan_chunks(uint64_t count, uint64_t* out, bool inclusive, Load load) {
  __shared__ uint64_t wsum[kScanThreads / kWave];
  uint64_t carry = 0;
  const uint64_t per_chunk = uint64_t(kScanThreads) * kScanItems;
  for (uint64_t base = 0; base < count; base += per_chunk) {
    const uint64_t first = base + uint64_t(threadIdx.x) * kScanItems;
    uint64_t v[kScanItems];
    uint64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (first + i < count) ? load(first + i) : 0;
      local = sat_add_u64(local, v[i]);
    }
    uint64_t total = 0;
    uint64_t run = sat_add_u64(carry, block_exclusive_scan_u64(local, wsum, &total));
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (first + i < count) {
        if (inclusive) {
          run = sat_add_u64(run, v[i]);
          out[first + i] = run;
        } else {
          out[first + i] = run;
          run = sat_add_u64(run, v[i]);
        }
      }
    }
    carry = sat_add_u64(carry, total);
  }
  if (!inclusive && threadIdx.x == 0) out[count] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_exclusive_scan(const uint64_t* __restrict__ in,
                                                                 uint64_t count,
                                                                 uint64_t* __restrict__ out) {
  scan_chunks(count, out, false, [&](uint64_t i) { return in[i]; });
}

__global__ __launch_bounds__(kScanThreads) void k_class_ends(const uint64_t* __restrict__ CU,
                                                             uint32_t n, DivMod32 dG,
                                                             uint32_t nclass,
                                                             uint64_t* __restrict__ endc) {
  scan_chunks(nclass, endc, true, [&](uint64_t r) {
    const uint32_t rr = uint32_t(r);
    const uint32_t q = dG.div(n - rr);
    return CU[uint64_t(rr) + uint64_t(q) * dG.d];
  });
}

// Batched: workgroup b lays out the class ends of jobs[b].
__global__ __launch_bounds__(kScanThreads) void k_class_ends_batch(
    const ClassJob* __restrict__ jobs) {
  const ClassJob& J = jobs[blockIdx.x];
  const uint64_t* CU = J.cu;
  const uint32_t n = J.n;
  const DivMod32 dG = J.dG;
  scan_chunks(J.nclass, J.endc, true, [&](uint64_t r) {
    const uint32_t rr = uint32_t(r);
    const uint32_t q = dG.div(n - rr);
    return CU[uint64_t(rr) + uint64_t(q) * dG.d];
  });
}

}  // namespace

hipError_t launch_class_ends_batch(const ClassJob* jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_ends_batch, dim3(njobs), dim3(kScanThreads), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const uint64_t* in, uint64_t count, uint64_t* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(kScanThreads), 0, s, in, count, out);
  return hipGetLastError();
}

hipError_t launch_class_ends(const uint64_t* count_row_u, uint64_t n, uint32_t G,
                             uint64_t* endc, uint32_t* nclass_out, hipStream_t s) {
  const uint32_t nclass = uint32_t(G < n + 1 ? G : n + 1);
  *nclass_out = nclass;
  hipLaunchKernelGGL(k_class_ends, dim3(1), dim3(kScanThreads), 0, s, count_row_u, uint32_t(n),
                     DivMod32::make(G), nclass, endc);
  return hipGetLastError();
}

}  // namespace zset
