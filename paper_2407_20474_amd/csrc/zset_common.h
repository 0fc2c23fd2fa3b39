// zset_common.h -- types and small device helpers shared by the HIP kernels
// and the host side of libzset.so.  gfx950 only (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zset {

constexpr int kWave = 64;
constexpr int kMaxD = 32;

// Kernel-side error codes written to the device status word (first writer wins).
enum DeviceError : int {
  kErrNone = 0,
  kErrOdometer = 1,      // a slice ran out of prefixes before its rows were written
  kErrTileRows = 2,      // a slice wrote a different number of rows than planned
  kErrMemoTotal = 3,     // memo chain produced a different row total than counted
  kErrUnrank = 4,        // a slice start could not be unranked
  kErrCapacity = 5,      // |Z(n)| exceeds the output's rows (nothing written)
  kErrOverflow = 6,      // |Z(n)| or its bytes overflow 64 bits (nothing written)
  kErrSlices = 7,        // |Z(n)| needs more slices than were planned for (nothing written)
};

// Generators passed by value in kernel arguments.
struct Gens {
  uint32_t g[kMaxD];
};

// Unsigned 32-bit division by an invariant divisor with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Figure 4.1): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, sh1 = min(l, 1), sh2 = max(l - 1, 0),
// q = (t + ((x - t) >> sh1)) >> sh2 where t = mulhi(m, x).  Exact for every
// 32-bit x and 1 <= d < 2^32.
struct DivMod32 {
  uint32_t d;
  uint32_t m;
  uint32_t sh1;
  uint32_t sh2;

  __host__ __device__ static DivMod32 make(uint32_t div) {
    DivMod32 r;
    r.d = div;
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < uint64_t(div)) ++l;
    r.m = uint32_t((((uint64_t(1) << l) - div) << 32) / div + 1);
    r.sh1 = l < 1 ? l : 1;
    r.sh2 = l > 1 ? l - 1 : 0;
    return r;
  }
  __host__ __device__ inline uint32_t div(uint32_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(m, x);
#else
    uint32_t t = uint32_t((uint64_t(m) * x) >> 32);
#endif
    return (t + ((x - t) >> sh1)) >> sh2;
  }
  __host__ __device__ inline uint32_t mod(uint32_t x, uint32_t q) const { return x - q * d; }
};

__host__ __device__ inline uint64_t sat_add_u64(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  return s < a ? ~uint64_t(0) : s;
}

// FNV-1a 64 over the four little-endian bytes of v (public FNV parameters).
__device__ inline uint64_t fnv1a_u32(uint64_t h, uint32_t v) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    h ^= (v >> (8 * b)) & 0xffu;
    h *= 1099511628211ull;
  }
  return h;
}

__device__ inline uint64_t fnv1a_u64(uint64_t h, uint64_t v) {
  h = fnv1a_u32(h, uint32_t(v));
  return fnv1a_u32(h, uint32_t(v >> 32));
}

constexpr uint64_t kFnvOffset = 14695981039346656037ull;

// Record the first device-side error.
__device__ inline void set_error(int* err, int code) {
  atomicCAS(err, 0, code);
}

}  // namespace zset
