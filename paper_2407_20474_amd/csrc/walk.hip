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
//   pass 1: one thread per prefix walks the rest and counts the rows (a
//           progression of the last two coordinates at a time);
//   scan:   exclusive sum of the counts = each prefix's first output row;
//   pass 2: the same walk again, 64 consecutive prefixes per wavefront (their
//           rows are one contiguous range): each lane stages a few rows of its
//           own in LDS, and the wavefront writes the staged words with
//           consecutive lanes on consecutive words of the output.
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
// Lanes the work is spread over: one per kWorkPerRecord units of estimated
// work (walk_estimate), between kMinPrefixes and kWantPrefixes.  Small walks
// then take few records (the host's splitting is most of their time), large
// ones enough wavefronts to hide the walk's dependent LDS and division chains.
constexpr uint64_t kWantPrefixes = 1 << 18;
constexpr uint64_t kMinPrefixes = 1 << 12;
constexpr double kWorkPerRecord = 256.0;
constexpr uint64_t kMaxPrefixes = 1 << 22;    // host refinement bound
constexpr int kSplitThreads = 16;             // host threads that refine records, at most

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
  DivMod32 dg[kMaxD];        // division by g_j
  DivMod32 dh, dstep;        // division by h and by step
  uint32_t stage_rows;       // pass 2: rows each lane stages in LDS per round
};

// The walk below one prefix record (a_1..a_m fixed, a_{m+1} in [lo, hi],
// later coordinates free) as a resumable generator: a[0..m) the record's
// coordinates, a[m..d-3] and r[m..d-3] the current node's coordinates and
// remainders, and the progression of the last two coordinates below it (pn
// rows left, pv the next value of a_{d-1}, pR the remainder the two share).
// next_prog moves to the next node in the walk's order; rows are taken from
// the progression one at a time.  a[] and r[] live in LDS, one column per
// thread (entry j at j * kWalkThreads), as do the generators and their
// divisions: indexed per lane, registers would spill to scratch and kernel
// arguments would be read from memory, and either load would wait for the
// wavefront's earlier stores.
struct WalkState {
  int m, j;
  bool done;
  uint32_t lo, hi;
  uint32_t* a;  // this thread's columns
  uint32_t* r;
  uint32_t pR, pv, pn;
};
#define WA(j) S.a[(j) * kWalkThreads]
#define WR(j) S.r[(j) * kWalkThreads]

struct WalkLds {
  uint32_t g[kMaxD];
  DivMod32 dg[kMaxD];
};

// Rows of the last two coordinates for remainder R with a_{d-1} in
// [vlo, vhi]: a_{d-1} runs over the progression a0 (mod step), a0 =
// (R / h) (g_{d-1} / h)^{-1} mod step, when h divides R, up to R / g_{d-1}.
__device__ inline void prog_setup(const WalkArgs& A, const WalkLds& W, WalkState& S, uint32_t R,
                                  uint32_t vlo, uint32_t vhi) {
  const int d = A.d;
  S.pn = 0;
  S.pR = R;
  const uint32_t qh = A.dh.div(R);
  if (A.dh.mod(R, qh) != 0) return;
  const uint32_t rh = A.dstep.mod(qh, A.dstep.div(qh));
  uint32_t a0;
  if (A.step <= 65536u) {
    const uint32_t t = rh * A.inv;  // both below step: no overflow
    a0 = A.dstep.mod(t, A.dstep.div(t));
  } else {
    a0 = uint32_t((uint64_t(rh) * A.inv) % A.step);
  }
  const uint32_t qmax = W.dg[d - 2].div(R);  // (an explicit compare: min() of two uint32_t
  const uint32_t amax = qmax < vhi ? qmax : vhi;  // can resolve to the int overload)
  uint64_t v0 = a0;
  if (vlo > a0) v0 = a0 + (uint64_t(vlo) - a0 + A.step - 1) / A.step * A.step;
  if (v0 > amax) return;
  S.pn = A.dstep.div(amax - uint32_t(v0)) + 1;
  S.pv = A.desc ? uint32_t(v0) + (S.pn - 1) * A.step : uint32_t(v0);
}

// Descend from level j to level d - 3, each coordinate at its first value
// (the last, in descending order), and set up that node's progression.
__device__ inline void descend(const WalkArgs& A, const WalkLds& W, WalkState& S) {
  const int d = A.d;
  int j = S.j;
  while (j < d - 3) {
    WR(j + 1) = WR(j) - WA(j) * W.g[j];
    ++j;
    WA(j) = A.desc ? W.dg[j].div(WR(j)) : 0;
  }
  S.j = j;
  prog_setup(A, W, S, WR(j) - WA(j) * W.g[j], 0, 0xffffffffu);
}

__device__ inline void walk_init(const WalkArgs& A, const WalkLds& W, WalkState& S,
                                 const uint32_t* p) {
  const int d = A.d;
  S.m = int(p[0]);
  S.lo = p[2];
  S.hi = p[3];
  S.done = false;
  S.pn = 0;
  for (int j = 0; j < S.m && j < d - 2; ++j) WA(j) = p[4 + j];
  if (S.m == d - 1) {  // a_1..a_{d-1} fixed: the last coordinate is forced
    S.done = true;     // a progression of one row (a_{d-1} = p[4 + d - 2]) or none
    const uint32_t x = p[1];
    const uint32_t q = W.dg[d - 1].div(x);
    if (W.dg[d - 1].mod(x, q) == 0) {
      S.pn = 1;
      S.pv = p[4 + d - 2];
      S.pR = x + S.pv * W.g[d - 2];  // so that (pR - pv g_{d-1}) / g_d = x / g_d
    }
    return;
  }
  if (S.m == d - 2) {  // one progression over a_{d-1} in [lo, hi]
    S.done = true;
    prog_setup(A, W, S, p[1], S.lo, S.hi);
    return;
  }
  S.j = S.m;
  WR(S.m) = p[1];
  WA(S.m) = A.desc ? S.hi : S.lo;
  descend(A, W, S);
}

// The next node at level d - 3 in the walk's order (its progression set
// up), or done: the deepest level below m whose coordinate can still move,
// else level m within [lo, hi].
__device__ inline void next_prog(const WalkArgs& A, const WalkLds& W, WalkState& S) {
  int j = S.j;
  while (j > S.m) {
    const uint32_t last = A.desc ? 0u : W.dg[j].div(WR(j));
    if (WA(j) != last) break;
    --j;
  }
  if (j == S.m && WA(j) == (A.desc ? S.lo : S.hi)) {
    S.done = true;
    return;
  }
  WA(j) = A.desc ? WA(j) - 1 : WA(j) + 1;
  S.j = j;
  descend(A, W, S);
}

__device__ inline void walk_lds_init(const WalkArgs& A, WalkLds& W) {
  if (threadIdx.x < uint32_t(kMaxD)) {
    W.g[threadIdx.x] = A.g.g[threadIdx.x];
    W.dg[threadIdx.x] = A.dg[threadIdx.x];
  }
  __syncthreads();
}

// Pass 1: one thread per record counts its rows (a progression at a time).
__global__ __launch_bounds__(kWalkThreads) void k_walk_count(WalkArgs A) {
  __shared__ WalkLds W;
  extern __shared__ uint32_t cols[];  // a[] then r[]: (d - 2) columns each
  walk_lds_init(A, W);
  const uint32_t levels = uint32_t(A.d > 2 ? A.d - 2 : 1);
  for (uint64_t i = uint64_t(blockIdx.x) * kWalkThreads + threadIdx.x; i < A.nprefix;
       i += uint64_t(gridDim.x) * kWalkThreads) {
    WalkState S;
    S.a = cols + threadIdx.x;
    S.r = cols + levels * kWalkThreads + threadIdx.x;
    walk_init(A, W, S, A.pre + i * uint64_t(A.d + 3));
    uint64_t rows = S.pn;
    while (!S.done) {
      next_prog(A, W, S);
      if (!S.done) rows += S.pn;
    }
    A.cnt[i] = rows;
  }
}

__device__ inline void wave_sync_walk() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass 2: a wavefront takes 64 consecutive records, one per lane.  In
// rounds, every lane stages up to stage_rows rows of its record in LDS (each
// lane's rows are contiguous in the output); then the wavefront writes the
// staged words two lanes' rows at a time, consecutive lanes on consecutive
// words: a store instruction covers two contiguous runs instead of 64
// scattered words.
constexpr uint32_t kWalkLaneWords = 32;  // LDS words staged per lane per round
// Each lane's staging area starts kWalkLaneWords + 1 words after the previous
// lane's: with an odd stride the lanes' stores of one staged word fall in
// different LDS banks (a stride of 32 words puts every lane in one bank).
constexpr uint32_t kWalkLaneStride = kWalkLaneWords + 1;
// The flush covers a lane's staged words with 32 lanes, and a row of up to
// kMaxD words must fit.
static_assert(kWalkLaneWords <= 32 && kWalkLaneWords >= uint32_t(kMaxD), "walk staging size");
__global__ __launch_bounds__(kWalkThreads) void k_walk_write(WalkArgs A) {
  __shared__ WalkLds W;
  __shared__ uint32_t stage[kWalkThreads * kWalkLaneStride];
  extern __shared__ uint32_t cols[];  // a[] then r[]: (d - 2) columns each
  walk_lds_init(A, W);
  const uint32_t levels = uint32_t(A.d > 2 ? A.d - 2 : 1);
  const int lane = int(threadIdx.x & 63);
  const int wave = int(threadIdx.x >> 6);
  uint32_t* buf = stage + uint32_t(threadIdx.x) * kWalkLaneStride;
  const uint32_t* wstage = stage + uint32_t(wave) * 64 * kWalkLaneStride;
  const int d = A.d;
  const uint32_t g2 = W.g[d - 2];
  const DivMod32 dlast = W.dg[d - 1];
  const uint64_t waves = uint64_t(gridDim.x) * (kWalkThreads / 64);
  for (uint64_t w = uint64_t(blockIdx.x) * (kWalkThreads / 64) + uint64_t(wave);
       w * 64 < A.nprefix; w += waves) {
    const uint64_t i = w * 64 + uint64_t(lane);
    const bool has = i < A.nprefix;
    WalkState S;
    S.a = cols + threadIdx.x;
    S.r = cols + levels * kWalkThreads + threadIdx.x;
    uint64_t pos = 0;
    S.done = true;
    S.pn = 0;
    if (has) {
      walk_init(A, W, S, A.pre + i * uint64_t(d + 3));
      pos = A.off[i];
    }
    for (;;) {
      // Stage up to stage_rows rows (divergent: each lane in its own walk).
      uint32_t nb = 0;
      while (nb < A.stage_rows) {
        if (S.pn == 0) {
          if (S.done) break;
          next_prog(A, W, S);
          continue;
        }
        uint32_t* row = buf + nb * uint32_t(d);
        for (int j = 0; j < d - 2; ++j) row[j] = WA(j);
        row[d - 2] = S.pv;
        row[d - 1] = dlast.div(S.pR - S.pv * g2);
        ++nb;
        --S.pn;
        if (S.pn) S.pv = A.desc ? S.pv - A.step : S.pv + A.step;
      }
      const bool more = !(S.done && S.pn == 0);
      // Flush: two lanes' staged rows per step, lanes 0-31 on the first
      // one's words and lanes 32-63 on the second's (at most 32 words each),
      // so that every store instruction covers two contiguous runs.
      const uint32_t wl = nb * uint32_t(d);
      const uint64_t gw = pos * uint64_t(d);  // this lane's first output word
      const uint32_t gw_lo = uint32_t(gw), gw_hi = uint32_t(gw >> 32);
      wave_sync_walk();  // the staged rows are visible to the wavefront
      const bool upper = lane >= 32;
      const uint32_t t = uint32_t(lane) & 31u;
      for (int s2 = 0; s2 < 64; s2 += 2) {
        const uint32_t wa = __builtin_amdgcn_readlane(wl, s2);
        const uint32_t wb = __builtin_amdgcn_readlane(wl, s2 + 1);
        if ((wa | wb) == 0) continue;
        const uint32_t w = upper ? wb : wa;
        const uint32_t lo = upper ? __builtin_amdgcn_readlane(gw_lo, s2 + 1)
                                  : __builtin_amdgcn_readlane(gw_lo, s2);
        const uint32_t hi = upper ? __builtin_amdgcn_readlane(gw_hi, s2 + 1)
                                  : __builtin_amdgcn_readlane(gw_hi, s2);
        if (t < w) {
          const uint32_t src = uint32_t(s2) + (upper ? 1u : 0u);
          const uint32_t v = wstage[src * kWalkLaneStride + t];
          __builtin_nontemporal_store(v, A.out + ((uint64_t(hi) << 32) | lo) + t);
        }
      }
      wave_sync_walk();  // every lane has read the staged rows
      pos += nb;
      if (__ballot(more) == 0) break;
    }
  }
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
      const int k = d - 2 - p.m;
      const double y0 = double(p.x) - double(p.lo) * g[p.m];
      const double y1 = std::max(0.0, double(p.x) - double(p.hi + 1) * g[p.m]);
      // The cut where the volumes (powers k of the remainders) halve: y0 times
      // the k-th root of (1 + (y1 / y0)^k) / 2.
      double q = 1.0, rk = y0 > 0 ? y1 / y0 : 0.0;
      for (int t = 0; t < k; ++t) q *= rk;
      const double ym = k == 1 ? 0.5 * (y0 + y1) : y0 * std::pow(0.5 * (1.0 + q), 1.0 / k);
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

// A record as the kernels read it: d + 3 words, m, the remainder, lo, hi,
// then a_1..a_m (zero-padded).
void pack_record(const Prefix& p, int d, std::vector<uint32_t>* out) {
  const size_t at = out->size();
  out->resize(at + size_t(d + 3), 0u);
  uint32_t* r = out->data() + at;
  r[0] = uint32_t(p.m);
  r[1] = uint32_t(p.x);
  r[2] = uint32_t(p.lo);
  r[3] = uint32_t(p.hi);
  for (int j = 0; j < p.m; ++j) r[4 + j] = p.a[j];
}

// The records below one seed, depth first, in order, at most `cap` of them,
// packed into `out`.
void split_below(Prefix seed, const uint32_t* g, int d, uint32_t step, double share,
                 uint64_t cap, std::vector<uint32_t>* out) {
  std::vector<Prefix> stack;
  stack.push_back(std::move(seed));
  uint64_t count = 0;
  while (!stack.empty()) {
    Prefix p = std::move(stack.back());
    stack.pop_back();
    if (p.m >= d - 1 || count + stack.size() + 2 > cap ||
        walk_estimate(p, g, d, step) <= share) {
      pack_record(p, d, out);
      ++count;
      continue;
    }
    split_record(std::move(p), g, d, &stack);
  }
}

// Prefix records in lexicographic order: from the whole range, every record
// whose estimate exceeds twice the share of one of the lanes above (and
// one unit) is split -- a range of a_{m+1} in two halves of about equal work,
// a single value into the next coordinate's range -- until the list holds
// kMaxPrefixes.  This is the static counterpart of re-splitting the heaviest
// remaining lexicographic range.  Depth first with an explicit stack, so the
// records come out in order in one pass per seed.
// The first splits, heaviest record first, make up to kSplitThreads seeds (no
// more than the host's hardware threads) in
// order; each is refined below by its own host thread into its own list of
// packed records (the lists, in seed order, are the records in order).
std::vector<std::vector<uint32_t>> make_prefixes(uint64_t n, const uint32_t* g, int d,
                                                 uint32_t step) {
  Prefix root = full_prefix(0, n, nullptr, g, d);
  const double work = walk_estimate(root, g, d, step);
  const double want = std::min(double(kWantPrefixes),
                               std::max(double(kMinPrefixes), work / kWorkPerRecord));
  const double share = std::max(1.0, 2.0 * work / want);
  std::vector<Prefix> seeds{std::move(root)};
  const unsigned hw = std::thread::hardware_concurrency();
  const size_t nseeds = size_t(std::max(1, std::min(kSplitThreads, hw ? int(hw) : 1)));
  while (seeds.size() < nseeds) {
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
  std::vector<std::vector<uint32_t>> lists(seeds.size());
  const uint64_t cap = kMaxPrefixes / seeds.size();
  std::vector<std::thread> pool;
  for (size_t i = 0; i < seeds.size(); ++i)
    pool.emplace_back(split_below, seeds[i], g, d, step, share, cap, &lists[i]);
  for (auto& t : pool) t.join();
  return lists;
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
  uint32_t* hpre = nullptr;  // pinned host staging of the records, hpre_words long
  size_t hpre_words = 0;
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
  const std::vector<std::vector<uint32_t>> lists = make_prefixes(n, gens, d, gens[d - 1] / h);
  const uint64_t W = uint64_t(d + 3);
  size_t words = 0;
  for (const auto& l : lists) words += l.size();
  const uint64_t np = words / W;
  // The records in pinned host memory (grown on demand, kept for later
  // calls), in order, or in reverse order for the descending walk.
  if (words > c.hpre_words) {
    if (c.hpre) (void)hipHostFree(c.hpre);
    c.hpre = nullptr;
    c.hpre_words = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&c.hpre), words * sizeof(uint32_t),
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c.hpre = nullptr;
      return fail(ZSET_ENOMEM, "pinned staging of the walk's records");
    }
    c.hpre_words = words;
  }
  if (order == 0) {
    size_t at = 0;
    for (const auto& l : lists) {
      std::memcpy(c.hpre + at, l.data(), l.size() * sizeof(uint32_t));
      at += l.size();
    }
  } else {  // descending: the records in reverse order
    size_t at = 0;
    for (auto l = lists.rbegin(); l != lists.rend(); ++l)
      for (size_t r = l->size(); r >= W; r -= W, at += W)
        std::memcpy(c.hpre + at, l->data() + (r - W), W * sizeof(uint32_t));
  }
  if ((st = ensure(c.pre, words * sizeof(uint32_t))) != ZSET_OK) return st;
  if ((st = ensure(c.cnt, (np + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  if ((st = ensure(c.off, (np + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  ZSET_HIP(hipMemcpyAsync(c.pre.p, c.hpre, words * sizeof(uint32_t), hipMemcpyHostToDevice, s));

  WalkArgs A;
  std::memset(&A, 0, sizeof A);
  for (int i = 0; i < d; ++i) A.g.g[i] = gens[i];
  A.d = d;
  A.desc = order;
  A.h = h;
  A.step = gens[d - 1] / A.h;
  A.inv = inverse_mod((gens[d - 2] / A.h) % A.step, A.step);
  for (int i = 0; i < d; ++i) A.dg[i] = DivMod32::make(gens[i]);
  A.dh = DivMod32::make(A.h);
  A.dstep = DivMod32::make(A.step);
  A.stage_rows = std::max<uint32_t>(1, kWalkLaneWords / uint32_t(d));
  A.nprefix = np;
  A.pre = reinterpret_cast<const uint32_t*>(c.pre.p);
  A.cnt = reinterpret_cast<uint64_t*>(c.cnt.p);
  A.off = reinterpret_cast<const uint64_t*>(c.off.p);
  A.out = out;
  const uint64_t blocks = std::min<uint64_t>((np + kWalkThreads - 1) / kWalkThreads, 65535);
  const size_t cols_bytes = size_t(2) * std::max(d - 2, 1) * kWalkThreads * sizeof(uint32_t);
  hipLaunchKernelGGL(k_walk_count, dim3(uint32_t(blocks)), dim3(kWalkThreads), cols_bytes, s, A);
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
    hipLaunchKernelGGL(k_walk_write, dim3(uint32_t(blocks)), dim3(kWalkThreads), cols_bytes, s,
                       A);
    ZSET_HIP(hipGetLastError());
    ZSET_HIP(hipStreamSynchronize(s));
  }
  *rows_written = total;
  return ZSET_OK;
}
