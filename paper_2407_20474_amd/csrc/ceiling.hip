// ceiling.hip -- the achievable HBM store rate of this device, for the write
// pass's roofline: store-only kernels with the write pass's store form
// (16-byte non-temporal stores, coalesced, every byte written once) over a
// caller's buffer, in four launch shapes, of which the fastest is reported.
// Measurement only; no part of the enumeration.
#include <stdint.h>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte store per lane, one workgroup per 256 x 16 bytes: the
// dispatcher hands out workgroups in address order, so the stores in flight
// stay within a few megabytes of each other.
__global__ __launch_bounds__(256) void k_store_oneshot(u32x4* __restrict__ dst, uint64_t nvec,
                                                       uint32_t value) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const u32x4 v = {value, value, value, value};
  if (i < nvec) __builtin_nontemporal_store(v, dst + i);
}

// Grid-stride: every step of the loop, the whole grid writes one contiguous
// region (grid x block x 16 bytes).
__global__ __launch_bounds__(1024) void k_store_stride(u32x4* __restrict__ dst, uint64_t nvec,
                                                       uint32_t value) {
  const u32x4 v = {value, value, value, value};
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec; i += stride)
    __builtin_nontemporal_store(v, dst + i);
}

// Each wavefront writes contiguous blocks of `vpb` 16-byte words, taken in
// turn over the grid's wavefronts.
__global__ __launch_bounds__(1024) void k_store_blocks(u32x4* __restrict__ dst, uint64_t nvec,
                                                       uint64_t vpb, uint32_t value) {
  const u32x4 v = {value, value, value, value};
  const uint64_t wpb = blockDim.x / 64;
  const uint64_t waves = uint64_t(gridDim.x) * wpb;
  const uint64_t wave = uint64_t(blockIdx.x) * wpb + threadIdx.x / 64;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nblocks = (nvec + vpb - 1) / vpb;
  for (uint64_t b = wave; b < nblocks; b += waves) {
    const uint64_t lo = b * vpb;
    const uint64_t hi = lo + vpb < nvec ? lo + vpb : nvec;
    for (uint64_t i = lo + lane; i < hi; i += 64) __builtin_nontemporal_store(v, dst + i);
  }
}

// The tail (bytes % 16) in 4-byte words.
__global__ void k_store_tail(uint32_t* __restrict__ buf, uint64_t first, uint64_t words,
                             uint32_t value) {
  const uint64_t w = first + threadIdx.x;
  if (w < words) __builtin_nontemporal_store(value, buf + w);
}

}  // namespace
}  // namespace zset

using namespace zset;

extern "C" zset_status zset_store_ceiling(void* buf, uint64_t bytes, int reps, void* stream,
                                          double* us_per_pass) {
  g_last_error.clear();
  if (!buf || !us_per_pass || reps < 1) return fail(ZSET_EINVAL, "buf, us_per_pass and reps >= 1");
  if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0 || bytes % 4 != 0)
    return fail(ZSET_EINVAL, "buf must be 16-byte aligned and bytes a multiple of 4");
  if (!is_device_pointer(buf)) return fail(ZSET_EINVAL, "buf is not device memory");
  const uint64_t nvec = bytes / 16, words = bytes / 4;
  if ((nvec + 255) / 256 > 0x7fffffffull) return fail(ZSET_EINVAL, "buffer too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  ZSET_HIP(hipGetDevice(&dev));
  ZSET_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ZSET_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(hipGetLastError(), "hipEventCreate");
  }
  u32x4* dst = static_cast<u32x4*>(buf);
  uint32_t* w32 = static_cast<uint32_t*>(buf);
  // Launch shapes (measured on a 4.8 GB buffer: the one-shot grid fastest,
  // then the grid-stride loop with one 256-lane workgroup per compute unit
  // and 64 KiB blocks per wavefront with four such workgroups).
  auto pass = [&](int form, uint32_t value) {
    switch (form) {
      case 0:
        hipLaunchKernelGGL(k_store_oneshot, dim3(uint32_t((nvec + 255) / 256)), dim3(256), 0, s,
                           dst, nvec, value);
        break;
      case 1:
        hipLaunchKernelGGL(k_store_stride, dim3(uint32_t(cus)), dim3(256), 0, s, dst, nvec, value);
        break;
      default:
        hipLaunchKernelGGL(k_store_blocks, dim3(uint32_t(cus) * 4), dim3(256), 0, s, dst, nvec,
                           uint64_t(4096), value);
        break;
    }
    if (words > nvec * 4)
      hipLaunchKernelGGL(k_store_tail, dim3(1), dim3(64), 0, s, w32, nvec * 4, words, value);
    return hipGetLastError();
  };
  double best = 0;
  hipError_t e = hipSuccess;
  for (int form = 0; form < 3 && e == hipSuccess; ++form) {
    // One untimed pass first (page mapping, clocks), then `reps` timed ones.
    e = pass(form, 0u);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = pass(form, uint32_t(r + 1));
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double us = double(ms) * 1000.0 / reps;
    if (e == hipSuccess && (best == 0 || us < best)) best = us;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "store ceiling");
  *us_per_pass = best;
  return ZSET_OK;
}
