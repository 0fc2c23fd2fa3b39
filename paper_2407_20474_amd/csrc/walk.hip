// walk.hip -- Z(n; g) without the count table (zset_enumerate_walk).
//
// The count-table path keeps (d + 1)(n + 1) counts on the device.  When n is
// large and the generators are large too, that table dwarfs the output: at
// n = 2e9 and d = 6 it would take 112 GB for perhaps a million rows.  This
// path keeps O(prefixes) instead.  It is the lexicographic walk of Section 2
// (each coordinate takes its values in order, the last one is forced by
// division), split over the prefixes (a_1..a_m) of the first m coordinates:
//
//   host:   the prefixes with a_1 g_1 + ... + a_m g_m <= n, in lexicographic
//           order, m grown until there are enough of them to fill the device
//           (or m = d - 1); each is stored with its remainder.
//   pass 1: one thread per prefix walks the rest of the coordinates and
//           counts the rows that complete it;
//   scan:   exclusive sum of the counts = each prefix's first output row;
//   pass 2: the same walk again, writing every row at its place.
//
// Prefixes in ascending order and each walk ascending give the rows in
// ascending lexicographic order; both reversed give descending order, the
// order of the paper's streams.  Every row is found twice (count, then
// write), the price of exact placement without counts.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {
namespace {

constexpr int kWalkThreads = 256;
constexpr uint64_t kWantPrefixes = 1 << 16;   // enough threads for the device
constexpr uint64_t kMaxPrefixes = 1 << 22;    // host enumeration bound

struct WalkArgs {
  Gens g;
  int d, m;                  // dimension, coordinates fixed by a prefix
  int desc;                  // 1: descending order
  uint64_t nprefix;
  const uint32_t* pre;       // nprefix x (m + 1): remainder, a_1..a_m
  uint64_t* cnt;             // pass 1 output
  const uint64_t* off;       // pass 2 input (exclusive sums of cnt)
  uint32_t* out;             // rows, d uint32 each
};

// The walk below one prefix: free coordinates m..d-2 take their values in
// order (ascending, or descending when desc), coordinate d-1 is forced.
// WRITE = false counts the rows, WRITE = true stores them from row `first`.
template <bool WRITE>
__device__ uint64_t walk_prefix(const WalkArgs& A, uint64_t i, uint64_t first) {
  const int d = A.d, m = A.m;
  const uint32_t* p = A.pre + i * uint64_t(m + 1);
  uint32_t a[kMaxD], r[kMaxD];
  r[m] = p[0];
  uint64_t rows = 0;
  auto emit = [&](uint32_t last) {
    if (WRITE) {
      uint32_t* row = A.out + (first + rows) * uint64_t(d);
      for (int j = 0; j < m; ++j) row[j] = p[1 + j];
      for (int j = m; j < d - 1; ++j) row[j] = a[j];
      row[d - 1] = last;
    }
    ++rows;
  };
  const uint32_t gl = A.g.g[d - 1];
  if (m == d - 1) {
    if (r[m] % gl == 0) emit(r[m] / gl);
    return rows;
  }
  int j = m;
  a[j] = A.desc ? r[j] / A.g.g[j] : 0;
  for (;;) {
    // Descend to the forced coordinate with the first value at each level.
    while (j < d - 2) {
      r[j + 1] = r[j] - a[j] * A.g.g[j];
      ++j;
      a[j] = A.desc ? r[j] / A.g.g[j] : 0;
    }
    const uint32_t rest = r[j] - a[j] * A.g.g[j];
    if (rest % gl == 0) emit(rest / gl);
    // Next value at the deepest level that has one.
    while (j >= m && (A.desc ? a[j] == 0 : a[j] == r[j] / A.g.g[j])) --j;
    if (j < m) break;
    a[j] = A.desc ? a[j] - 1 : a[j] + 1;
  }
  return rows;
}

__global__ __launch_bounds__(kWalkThreads) void k_walk_count(WalkArgs A) {
  for (uint64_t i = uint64_t(blockIdx.x) * kWalkThreads + threadIdx.x; i < A.nprefix;
       i += uint64_t(gridDim.x) * kWalkThreads)
    A.cnt[i] = walk_prefix<false>(A, i, 0);
}

__global__ __launch_bounds__(kWalkThreads) void k_walk_write(WalkArgs A) {
  for (uint64_t i = uint64_t(blockIdx.x) * kWalkThreads + threadIdx.x; i < A.nprefix;
       i += uint64_t(gridDim.x) * kWalkThreads)
    (void)walk_prefix<true>(A, i, A.off[i]);
}

// Prefixes (remainder, a_1..a_m) of the first m coordinates in ascending
// lexicographic order, m grown while the next level stays within
// kMaxPrefixes and the current one has fewer than kWantPrefixes.
void make_prefixes(uint64_t n, const uint32_t* g, int d, std::vector<uint32_t>* pre, int* m_out) {
  // Level m = 1 (the caller has checked that n / g_1 + 1 <= kMaxPrefixes).
  std::vector<uint32_t> cur;
  cur.reserve(2 * (n / g[0] + 1));
  int m = 1;
  for (uint64_t a = 0; a * g[0] <= n; ++a) {
    cur.push_back(uint32_t(n - a * g[0]));
    cur.push_back(uint32_t(a));
  }
  while (m < d - 1 && cur.size() / (m + 1) < kWantPrefixes) {
    std::vector<uint32_t> next;
    bool over = false;
    const uint64_t np = cur.size() / (m + 1);
    for (uint64_t i = 0; i < np && !over; ++i) {
      const uint32_t* p = &cur[i * (m + 1)];
      for (uint64_t a = 0; uint64_t(a) * g[m] <= p[0]; ++a) {
        if (next.size() / (m + 2) >= kMaxPrefixes) {
          over = true;
          break;
        }
        next.push_back(uint32_t(p[0] - a * g[m]));
        for (int j = 0; j < m; ++j) next.push_back(p[1 + j]);
        next.push_back(uint32_t(a));
      }
    }
    if (over) break;
    cur.swap(next);
    ++m;
  }
  pre->swap(cur);
  *m_out = m;
}

struct WalkCtx {
  DevBuf pre, cnt, off;
  uint64_t* pinned = nullptr;
};
WalkCtx g_walk[64];

}  // namespace
}  // namespace zset

using namespace zset;

extern "C" zset_status zset_enumerate_walk(uint64_t n, const uint32_t* gens, int d, uint32_t* out,
                                           uint64_t out_rows_cap, int order, void* stream,
                                           uint64_t* rows_written) {
  g_last_error.clear();
  zset_status st = check_query(n, gens, d);
  if (st != ZSET_OK) return st;
  if (order != 0 && order != 1) return fail(ZSET_EINVAL, "order must be 0 or 1");
  if (!rows_written) return fail(ZSET_EINVAL, "rows_written is NULL");
  if (!out) return fail(ZSET_EINVAL, "out is NULL");
  if (!is_device_pointer(out)) return fail(ZSET_EINVAL, "out is not device memory");
  *rows_written = 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  ZSET_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(ZSET_EDEVICE, "device index out of range");
  WalkCtx& c = g_walk[dev];
  if (!c.pinned) {
    if (hipHostMalloc(reinterpret_cast<void**>(&c.pinned), 2 * sizeof(uint64_t),
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c.pinned = nullptr;
      return fail(ZSET_ENOMEM, "pinned readback word");
    }
  }

  if (d == 1) {  // the only coordinate is forced
    if (n % gens[0] != 0) return ZSET_OK;
    if (out_rows_cap < 1) return fail(ZSET_ECAPACITY, "out holds 0 rows, |Z(n)| = 1");
    const uint32_t v = uint32_t(n / gens[0]);
    ZSET_HIP(hipMemcpyAsync(out, &v, sizeof v, hipMemcpyHostToDevice, s));
    ZSET_HIP(hipStreamSynchronize(s));
    *rows_written = 1;
    return ZSET_OK;
  }

  if (n / gens[0] + 1 > kMaxPrefixes)
    return fail(ZSET_EINVAL, "n / g_1 + 1 exceeds 2^22 first-coordinate values: use "
                             "zset_enumerate_ex");
  std::vector<uint32_t> pre;
  int m = 1;
  make_prefixes(n, gens, d, &pre, &m);
  const uint64_t np = pre.size() / uint64_t(m + 1);
  if (order == 1) {  // descending: prefixes in reverse order
    for (uint64_t i = 0, j = np - 1; i < j; ++i, --j)
      for (int w = 0; w <= m; ++w) std::swap(pre[i * (m + 1) + w], pre[j * (m + 1) + w]);
  }
  if ((st = ensure(c.pre, pre.size() * sizeof(uint32_t))) != ZSET_OK) return st;
  if ((st = ensure(c.cnt, (np + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  if ((st = ensure(c.off, (np + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  ZSET_HIP(hipMemcpyAsync(c.pre.p, pre.data(), pre.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s));

  WalkArgs A;
  std::memset(&A, 0, sizeof A);
  for (int i = 0; i < d; ++i) A.g.g[i] = gens[i];
  A.d = d;
  A.m = m;
  A.desc = order;
  A.nprefix = np;
  A.pre = reinterpret_cast<const uint32_t*>(c.pre.p);
  A.cnt = reinterpret_cast<uint64_t*>(c.cnt.p);
  A.off = reinterpret_cast<const uint64_t*>(c.off.p);
  A.out = out;
  const uint64_t blocks = std::min<uint64_t>((np + kWalkThreads - 1) / kWalkThreads, 65535);
  hipLaunchKernelGGL(k_walk_count, dim3(uint32_t(blocks)), dim3(kWalkThreads), 0, s, A);
  ZSET_HIP(hipGetLastError());
  // off[i] = rows of prefixes before i; off[np] = |Z(n)| (cnt[np] is zero).
  ZSET_HIP(hipMemsetAsync(A.cnt + np, 0, sizeof(uint64_t), s));
  ZSET_HIP(launch_exclusive_scan(A.cnt, np + 1, reinterpret_cast<uint64_t*>(c.off.p), s));
  ZSET_HIP(hipMemcpyAsync(c.pinned, reinterpret_cast<uint64_t*>(c.off.p) + np, sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
  ZSET_HIP(hipStreamSynchronize(s));
  const uint64_t total = c.pinned[0];
  if (total == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
  if (total > out_rows_cap)
    return fail(ZSET_ECAPACITY, "out holds " + std::to_string(out_rows_cap) + " rows, |Z(n)| = " +
                                    std::to_string(total));
  if (total > 0) {
    hipLaunchKernelGGL(k_walk_write, dim3(uint32_t(blocks)), dim3(kWalkThreads), 0, s, A);
    ZSET_HIP(hipGetLastError());
    ZSET_HIP(hipStreamSynchronize(s));
  }
  *rows_written = total;
  return ZSET_OK;
}
