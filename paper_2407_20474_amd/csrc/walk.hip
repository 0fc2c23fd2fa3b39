// walk.hip -- Z(n; g) without the count table (zset_enumerate_walk).
//
// The count-table path keeps (d + 1)(n + 1) counts on the device.  When n is
// large and the generators are large too, that table dwarfs the output: at
// n = 1.6e9 and d = 6 it would take 90 GB for 6e7 rows.  This path keeps
// O(prefixes) instead.  It is the lexicographic walk of Section 2 (each
// coordinate takes its values in order, the last one is forced by division),
// split over prefixes (a_1..a_m):
//
//   host:   prefixes in lexicographic order, refined where the work below
//           them is large: a prefix whose estimated work exceeds its share is
//           replaced by its children (the prefixes one coordinate longer), in
//           order, until the work is spread over enough prefixes (the static
//           counterpart of re-splitting the heaviest remaining range);
//   pass 1: one thread per prefix walks the rest and counts the rows;
//   scan:   exclusive sum of the counts = each prefix's first output row;
//   pass 2: the same walk again, writing every row at its place.
//
// The walk below a prefix takes coordinates m..d-3 one value at a time.  For
// the last free coordinate a_{d-1} only values that leave a remainder divisible
// by g_d can complete a row: with h = gcd(g_{d-1}, g_d) they are the
// progression a = a0 (mod g_d / h), a0 = (R / h) (g_{d-1} / h)^{-1} mod (g_d / h),
// when h divides the remainder R.  So the walk's cost is its nodes above the
// last two coordinates plus its rows, not the (g_d times larger) number of
// vectors (a_1..a_{d-1}).
//
// Prefixes in ascending order and each walk ascending give the rows in
// ascending lexicographic order; both reversed give descending order, the
// order of the paper's streams.  Every row is found twice (count, then
// write), the price of exact placement without counts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {
namespace {

constexpr int kWalkThreads = 256;
constexpr uint64_t kWantPrefixes = 1 << 17;   // lanes the work is spread over
constexpr uint64_t kMaxPrefixes = 1 << 22;    // host refinement bound
constexpr int kSplitThreads = 8;              // host threads that refine records

struct WalkArgs {
  Gens g;
  int d;
  int desc;                  // 1: descending order
  uint32_t h, step, inv;     // gcd(g_{d-1}, g_d), g_d / h, (g_{d-1} / h)^{-1} mod step
  uint64_t nprefix;
  const uint32_t* pre;       // nprefix x (d + 3): m, remainder, lo, hi, a_1..a_m
  uint64_t* cnt;             // pass 1 output
  const uint64_t* off;       // pass 2 input (exclusive sums of cnt)
  uint32_t* out;             // rows, d uint32 each
};

// The walk below one prefix record: a_1..a_m fixed, a_{m+1} in [lo, hi],
// later coordinates free.  WRITE = false counts the rows, WRITE = true stores
// them from row `first`.
template <bool WRITE>
__device__ uint64_t walk_prefix(const WalkArgs& A, uint64_t i, uint64_t first) {
  const int d = A.d;
  const uint32_t* p = A.pre + i * uint64_t(d + 3);
  const int m = int(p[0]);
  const uint32_t lo = p[2], hi = p[3];
  uint32_t a[kMaxD], r[kMaxD];
  uint64_t rows = 0;
  auto emit = [&](uint32_t al, uint32_t last) {  // al = a_{d-1}
    if (WRITE) {
      uint32_t* row = A.out + (first + rows) * uint64_t(d);
      for (int j = 0; j < m; ++j) row[j] = p[4 + j];
      for (int j = m; j < d - 2; ++j) row[j] = a[j];
      row[d - 2] = al;
      row[d - 1] = last;
    }
    ++rows;
  };
  const uint32_t g2 = A.g.g[d - 2], g1 = A.g.g[d - 1];
  // Rows of the last two coordinates for remainder R with a_{d-1} in
  // [vlo, vhi], in order: a_{d-1} runs over a progression of difference step.
  auto progression = [&](uint32_t R, uint32_t vlo, uint32_t vhi) {
    if (R % A.h != 0) return;
    const uint64_t amax = min(uint64_t(R / g2), uint64_t(vhi));
    const uint64_t a0 = (uint64_t((R / A.h) % A.step) * A.inv) % A.step;
    const uint64_t v0 = vlo > a0 ? a0 + (uint64_t(vlo) - a0 + A.step - 1) / A.step * A.step : a0;
    if (v0 > amax) return;
    const uint64_t nv = (amax - v0) / A.step + 1;
    for (uint64_t t = 0; t < nv; ++t) {
      const uint32_t v = uint32_t(A.desc ? v0 + (nv - 1 - t) * A.step : v0 + t * A.step);
      emit(v, (R - v * g2) / g1);
    }
  };
  if (m == d - 1) {  // only the last coordinate is left: forced
    if (p[1] % g1 == 0) {
      if (WRITE) {
        uint32_t* row = A.out + first * uint64_t(d);
        for (int j = 0; j < d - 1; ++j) row[j] = p[4 + j];
        row[d - 1] = p[1] / g1;
      }
      ++rows;
    }
    return rows;
  }
  if (m == d - 2) {
    progression(p[1], lo, hi);
    return rows;
  }
  int j = m;
  r[j] = p[1];
  a[j] = A.desc ? hi : lo;
  for (;;) {
    // Descend to coordinate d - 3 with the first value at each level.
    while (j < d - 3) {
      r[j + 1] = r[j] - a[j] * A.g.g[j];
      ++j;
      a[j] = A.desc ? r[j] / A.g.g[j] : 0;
    }
    progression(r[j] - a[j] * A.g.g[j], 0, 0xffffffffu);
    // Next value at the deepest level that has one (level m keeps to [lo, hi]).
    for (; j >= m; --j) {
      const uint32_t end = A.desc ? (j == m ? lo : 0u) : (j == m ? hi : r[j] / A.g.g[j]);
      if (a[j] != end) break;
    }
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

// Host side: prefix records and their estimated work.
struct Prefix {
  int m;
  uint64_t x, lo, hi;        // remainder before a_{m+1}; a_{m+1} in [lo, hi]
  uint32_t a[kMaxD];         // a_1..a_m
};

// Progressions run below coordinate m with remainder y when a_{m+1} takes
// every value: the simplex volume of (a_{m+1}..a_{d-2}), sum a_j g_j <= y.
double walk_volume(double y, int m, const uint32_t* g, int d) {
  if (y < 0) return 0;
  double e = 1.0;
  for (int j = m, t = 1; j < d - 2; ++j, ++t) e *= y / double(g[j]) / double(t);
  return e;
}

// Estimated work of a record: its progressions (the volume between the
// remainders left by lo and by hi + 1), each with the rows of an average
// progression; at the progression level, its rows.
double walk_estimate(const Prefix& p, const uint32_t* g, int d, uint32_t step) {
  if (p.m >= d - 1) return 0;
  if (p.m == d - 2) return double(p.hi - p.lo + 1) / double(step);
  const double y0 = double(p.x) - double(p.lo) * g[p.m];
  const double y1 = double(p.x) - double(p.hi + 1) * g[p.m];
  const double vol = walk_volume(y0, p.m, g, d) - walk_volume(y1, p.m, g, d);
  const double prog = double(p.x) / double(d - 1 - p.m) / double(g[d - 2]) / double(step);
  return vol * (1.0 + prog);
}

// The record of a_1..a_m = a[0..m) with a_{m+1} over all its values.
Prefix full_prefix(int m, uint64_t x, const uint32_t* a, const uint32_t* g, int d) {
  Prefix p;
  p.m = m;
  p.x = x;
  std::memcpy(p.a, a, sizeof(uint32_t) * size_t(m));
  p.lo = 0;
  p.hi = m < d - 1 ? x / g[m] : 0;
  return p;
}

// One split: a range into two halves of about equal estimated work (the
// volume is a power of the remainder), a single value into the next
// coordinate's range.  Pushes the parts in reverse order onto `stack`.
void split_record(Prefix p, const uint32_t* g, int d, std::vector<Prefix>* stack) {
  if (p.hi > p.lo) {
    uint64_t mid = p.lo + (p.hi - p.lo) / 2;
    if (p.m < d - 2) {
      const double k = double(d - 2 - p.m);
      const double y0 = double(p.x) - double(p.lo) * g[p.m];
      const double y1 = std::max(0.0, double(p.x) - double(p.hi + 1) * g[p.m]);
      const double ym = std::pow(0.5 * (std::pow(y0, k) + std::pow(y1, k)), 1.0 / k);
      const double cut = (double(p.x) - ym) / double(g[p.m]);
      if (cut >= double(p.lo) && cut < double(p.hi)) mid = uint64_t(cut);
    }
    Prefix l = p;
    l.hi = mid;
    p.lo = mid + 1;
    stack->push_back(std::move(p));  // the upper half is taken after the lower
    stack->push_back(std::move(l));
  } else {
    p.a[p.m] = uint32_t(p.lo);
    stack->push_back(full_prefix(p.m + 1, p.x - p.lo * g[p.m], p.a, g, d));
  }
}

// The records below one seed, depth first, in order, at most `cap` of them.
void split_below(Prefix seed, const uint32_t* g, int d, uint32_t step, double share,
                 uint64_t cap, std::vector<Prefix>* out) {
  std::vector<Prefix> stack;
  stack.push_back(std::move(seed));
  while (!stack.empty()) {
    Prefix p = std::move(stack.back());
    stack.pop_back();
    if (p.m >= d - 1 || out->size() + stack.size() + 2 > cap ||
        walk_estimate(p, g, d, step) <= share) {
      out->push_back(std::move(p));
      continue;
    }
    split_record(std::move(p), g, d, &stack);
  }
}

// Prefix records in lexicographic order: from the whole range, every record
// whose estimate exceeds twice the share of one of kWantPrefixes lanes (and
// one unit) is split -- a range of a_{m+1} in two halves of about equal work,
// a single value into the next coordinate's range -- until the list holds
// kMaxPrefixes.  This is the static counterpart of re-splitting the heaviest
// remaining lexicographic range.  Depth first with an explicit stack, so the
// records come out in order in one pass per seed.
// The first splits, heaviest record first, make up to kSplitThreads seeds in
// order; each is refined below by its own host thread and the lists are
// concatenated in seed order.
std::vector<Prefix> make_prefixes(uint64_t n, const uint32_t* g, int d, uint32_t step) {
  Prefix root = full_prefix(0, n, nullptr, g, d);
  const double share =
      std::max(1.0, 2.0 * walk_estimate(root, g, d, step) / double(kWantPrefixes));
  std::vector<Prefix> seeds{std::move(root)};
  while (seeds.size() < size_t(kSplitThreads)) {
    size_t heavy = 0;
    double most = -1;
    for (size_t i = 0; i < seeds.size(); ++i) {
      const double e = seeds[i].m >= d - 1 ? -1 : walk_estimate(seeds[i], g, d, step);
      if (e > most) {
        most = e;
        heavy = i;
      }
    }
    if (most <= share) break;
    std::vector<Prefix> parts;
    split_record(seeds[heavy], g, d, &parts);
    std::reverse(parts.begin(), parts.end());
    seeds.erase(seeds.begin() + long(heavy));
    seeds.insert(seeds.begin() + long(heavy), parts.begin(), parts.end());
  }
  std::vector<std::vector<Prefix>> lists(seeds.size());
  const uint64_t cap = kMaxPrefixes / seeds.size();
  std::vector<std::thread> pool;
  for (size_t i = 0; i < seeds.size(); ++i)
    pool.emplace_back(split_below, seeds[i], g, d, step, share, cap, &lists[i]);
  for (auto& t : pool) t.join();
  std::vector<Prefix> out;
  size_t total = 0;
  for (const auto& l : lists) total += l.size();
  out.reserve(total);
  for (auto& l : lists) out.insert(out.end(), std::make_move_iterator(l.begin()),
                                   std::make_move_iterator(l.end()));
  return out;
}

uint32_t gcd32(uint32_t a, uint32_t b) {
  while (b) {
    const uint32_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// x^{-1} mod m for gcd(x, m) = 1 (0 when m = 1), by the extended Euclidean
// algorithm.
uint32_t inverse_mod(uint32_t x, uint32_t m) {
  if (m == 1) return 0;
  int64_t t = 0, nt = 1, r = m, nr = x % m;
  while (nr != 0) {
    const int64_t q = r / nr;
    int64_t tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  if (t < 0) t += m;
  return uint32_t(t);
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

  const uint32_t h = gcd32(gens[d - 2], gens[d - 1]);
  std::vector<Prefix> list = make_prefixes(n, gens, d, gens[d - 1] / h);
  if (order == 1) std::reverse(list.begin(), list.end());  // descending: reverse order
  const uint64_t W = uint64_t(d + 3);
  const uint64_t np = list.size();
  std::vector<uint32_t> pre(np * W, 0);
  for (uint64_t i = 0; i < np; ++i) {
    const Prefix& p = list[i];
    uint32_t* r = &pre[i * W];
    r[0] = uint32_t(p.m);
    r[1] = uint32_t(p.x);
    r[2] = uint32_t(p.lo);
    r[3] = uint32_t(p.hi);
    for (int j = 0; j < p.m; ++j) r[4 + j] = p.a[j];
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
  A.desc = order;
  A.h = h;
  A.step = gens[d - 1] / A.h;
  A.inv = inverse_mod((gens[d - 2] / A.h) % A.step, A.step);
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
