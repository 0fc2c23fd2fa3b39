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
//   pass 1: one wavefront per prefix walks the rest and counts the rows: an
//           odometer over the coordinates above the last three, 64 values
//           of coordinate d-3 at a time across the lanes, each with the
//           progression of the last two coordinates below it (closed form);
//   scan:   exclusive sum of the counts = each prefix's first output row;
//   pass 2: the same walk again, the rows placed by a wave prefix sum of the
//           progressions' lengths, staged in LDS and written 64 rows at a time
//           with consecutive lanes on consecutive words of the output.
//
// The walk below a prefix takes the coordinates above the last three as an
// odometer and coordinate d-3 in 64-value steps.  For
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
constexpr uint64_t kWantPrefixes = 1 << 16;
constexpr uint64_t kMinPrefixes = 1 << 10;
constexpr double kWorkPerRecord = 1024.0;
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
  DivMod32 dd;               // division by d (descending flush)
};

// The walk below one record, by one wavefront.  A record fixes coordinates
// 0..m-1 (0-based), lets coordinate m run over [lo, hi] with remainder x
// before it, and leaves the later ones free.  With l = d - 3, the last
// coordinate above the progression of coordinates d-2 and d-1:
//   - coordinates m..l-1 ("outer") step as an odometer, lane j holding a_j and
//     the remainder after it (lanes below m hold the record's coordinates);
//   - the 64 lanes take 64 consecutive values v of coordinate l at a time;
//     lane v's remainder R = y - v g_l (y: the remainder before l) completes
//     pn(R) rows, the progression of coordinate d-2 below R (closed form);
//   - a wave prefix sum of the pn places the rows.  They are produced 64 at a
//     time, each lane finding the lane whose first row is the last one at or
//     before its own (LDS marks and a wave prefix max), staged in the
//     wavefront's LDS ring and written out 64 rows at a time, consecutive
//     lanes on consecutive words.
// m = d-2 is one progression (coordinate d-2 in [lo, hi]); m = d-1 at most one
// row.  Rows come out in ascending order within the record; in descending
// output, the record's row of ascending rank t goes to its last place - t.
constexpr int kWalkWaves = kWalkThreads / 64;  // wavefronts per workgroup
constexpr uint32_t kWalkRing = 128;            // rows in a wavefront's LDS ring
constexpr uint32_t kWalkFlush = 64;            // rows per flush

__device__ inline void wave_sync_walk() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t readlane_u64(uint64_t v, int l) {
  return (uint64_t(__builtin_amdgcn_readlane(uint32_t(v >> 32), l)) << 32) |
         __builtin_amdgcn_readlane(uint32_t(v), l);
}

__device__ inline uint64_t wave_incl_sum_u64(uint64_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  return v;
}

__device__ inline uint32_t wave_incl_max_u32(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(v, off, 64);
    if (lane >= off && y > v) v = y;
  }
  return v;
}

// Rows of the last two coordinates for remainder R with coordinate d-2 in
// [vlo, vhi]: its values run over the progression a0 (mod step), a0 =
// (R / h) (g_{d-2} / h)^{-1} mod step, when h divides R, up to R / g_{d-2}.
// Returns their number; *v0 = the first.
__device__ inline uint32_t prog_count(const WalkArgs& A, const DivMod32& dg2, uint32_t R,
                                      uint32_t vlo, uint32_t vhi, uint32_t* v0) {
  *v0 = 0;
  const uint32_t qh = A.dh.div(R);
  if (A.dh.mod(R, qh) != 0) return 0;
  const uint32_t rh = A.dstep.mod(qh, A.dstep.div(qh));
  uint32_t a0;
  if (A.step <= 65536u) {
    const uint32_t t = rh * A.inv;  // both below step: no overflow
    a0 = A.dstep.mod(t, A.dstep.div(t));
  } else {
    a0 = uint32_t((uint64_t(rh) * A.inv) % A.step);
  }
  const uint32_t qmax = dg2.div(R);
  const uint32_t amax = qmax < vhi ? qmax : vhi;
  uint64_t first = a0;
  if (vlo > a0) first = a0 + (uint64_t(vlo) - a0 + A.step - 1) / A.step * A.step;
  if (first > amax) return 0;
  *v0 = uint32_t(first);
  return A.dstep.div(amax - uint32_t(first)) + 1;
}

// Rows [first, first + nrows) of a record from the ring (first a multiple of
// kWalkFlush, so the rows are contiguous there) to the output: in place, or
// reversed for descending order (the record's rows are base .. base + cnt - 1).
__device__ inline void walk_flush(const WalkArgs& A, const uint32_t* ring, uint64_t base,
                                  uint64_t cnt, uint64_t first, uint32_t nrows, int lane) {
  if (first + nrows > cnt) return;  // never: the count pass walked the same rows
  const uint32_t d = uint32_t(A.d);
  const uint32_t nw = nrows * d;
  const uint32_t* src = ring + (uint32_t(first) & (kWalkRing - 1)) * d;
  if (!A.desc) {
    uint32_t* dst = A.out + (base + first) * d;
    for (uint32_t w = uint32_t(lane); w < nw; w += 64) __builtin_nontemporal_store(src[w], dst + w);
  } else {
    uint32_t* dst = A.out + (base + cnt - first - nrows) * d;
    for (uint32_t w = uint32_t(lane); w < nw; w += 64) {
      const uint32_t r = A.dd.div(w), c = w - r * d;
      __builtin_nontemporal_store(src[(nrows - 1 - r) * d + c], dst + w);
    }
  }
}

// The rows of one record (kind 0: values of coordinate l per lane; 1: one
// progression; 2: a single row), counted, or staged and written (WRITE).
struct RecordOut {
  uint32_t* ring;
  uint32_t* marks;
  uint64_t base, cnt, produced, flushed;
};

// One chunk: lane i has pn rows (0 if idle); they follow in lane order.
// Counting, it returns pn (the record sums its lanes once at its end).
// Writing, every row is staged (its words from the owning lane's v, v0 and
// R, and the prefix in lanes 0..npre-1 of aj) and full blocks are written out.
template <bool WRITE>
__device__ inline uint64_t walk_chunk(const WalkArgs& A, RecordOut& O, int lane, uint32_t pn,
                                      uint32_t aj, int npre, int kind, uint32_t v, uint32_t v0,
                                      uint32_t R, const DivMod32& dg2, const DivMod32& dlast) {
  if (!WRITE) return pn;
  const uint64_t some = __ballot(pn != 0);
  if (some == 0) return 0;
  const int d = A.d;
  if (__ballot(pn > 1) == 0) {
    // At most one row per lane (the usual case for large generators): the
    // rows' places come from a ballot, and each lane stages its own row.
    const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
        uint32_t(some >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(some), 0u));
    const uint32_t nrows = uint32_t(__popcll((unsigned long long)some));
    if (pn != 0) {
      uint32_t* row = O.ring + (uint32_t(O.produced + pos) & (kWalkRing - 1)) * uint32_t(d);
      for (int j = 0; j < npre; ++j) row[j] = __builtin_amdgcn_readlane(aj, j);
      if (kind == 2) {
        row[d - 1] = v;
      } else {
        if (kind == 0) row[d - 3] = v;
        row[d - 2] = v0;
        row[d - 1] = dlast.div(R - v0 * dg2.d);
      }
    }
    wave_sync_walk();
    const uint64_t written = O.produced + nrows;
    while (written - O.flushed >= kWalkFlush) {
      walk_flush(A, O.ring, O.base, O.cnt, O.flushed, kWalkFlush, lane);
      O.flushed += kWalkFlush;
    }
    wave_sync_walk();
    O.produced = written;
    return nrows;
  }
  const uint64_t incl = wave_incl_sum_u64(pn, lane);
  const uint64_t tot = readlane_u64(incl, 63);
  const uint64_t excl = incl - pn;
  uint32_t carry = 0;
  for (uint64_t beta = 0; beta < tot; beta += 64) {
    const uint64_t rho = beta + uint64_t(lane);
    O.marks[lane] = 0;
    wave_sync_walk();
    if (pn != 0 && excl >= beta && excl - beta < 64) O.marks[excl - beta] = uint32_t(lane) + 1;
    wave_sync_walk();
    uint32_t mk = wave_incl_max_u32(O.marks[lane], lane);
    mk = mk > carry ? mk : carry;
    carry = __builtin_amdgcn_readlane(mk, 63);
    const int owner = int(mk) - 1;  // row beta's owner: a first row at or before it
    // Every lane reads the owner's values (a cross-lane read runs in all lanes).
    const uint32_t o_lo = __shfl(uint32_t(excl), owner, 64);
    const uint32_t o_hi = __shfl(uint32_t(excl >> 32), owner, 64);
    const uint32_t o_v = __shfl(v, owner, 64);
    const uint32_t o_v0 = __shfl(v0, owner, 64);
    const uint32_t o_R = __shfl(R, owner, 64);
    if (rho < tot) {
      const uint64_t t = rho - ((uint64_t(o_hi) << 32) | o_lo);
      uint32_t* row = O.ring + (uint32_t(O.produced + rho) & (kWalkRing - 1)) * uint32_t(d);
      for (int j = 0; j < npre; ++j) row[j] = __builtin_amdgcn_readlane(aj, j);
      if (kind == 2) {
        row[d - 1] = o_v;  // the forced last coordinate
      } else {
        if (kind == 0) row[d - 3] = o_v;
        const uint32_t pv = o_v0 + uint32_t(t) * A.step;
        row[d - 2] = pv;
        row[d - 1] = dlast.div(o_R - pv * dg2.d);
      }
    }
    wave_sync_walk();
    const uint64_t left = tot - beta;
    const uint64_t written = O.produced + beta + (left < 64 ? left : 64);
    while (written - O.flushed >= kWalkFlush) {
      walk_flush(A, O.ring, O.base, O.cnt, O.flushed, kWalkFlush, lane);
      O.flushed += kWalkFlush;
    }
    wave_sync_walk();
  }
  O.produced += tot;
  return tot;
}

// The record's rows: counted (returned, in every lane), or written to their
// place (WRITE; the return value is then unused).
template <bool WRITE>
__device__ uint64_t walk_record(const WalkArgs& A, uint64_t rec, RecordOut& O, int lane,
                                uint32_t gj) {
  const int d = A.d;
  const uint32_t* p = A.pre + rec * uint64_t(d + 3);
  const int m = int(p[0]);
  const uint32_t x = p[1], lo = p[2], hi = p[3];
  uint32_t aj = lane < m && lane < d - 1 ? p[4 + lane] : 0;
  const DivMod32 dg2 = A.dg[d - 2 >= 0 ? d - 2 : 0];
  const DivMod32 dlast = A.dg[d - 1];
  if (m >= d - 1) {  // coordinates 0..d-2 fixed: the last is forced, or no row
    const uint32_t q = dlast.div(x);
    const uint32_t pn = dlast.mod(x, q) == 0 ? 1u : 0u;
    walk_chunk<WRITE>(A, O, lane, lane == 0 ? pn : 0u, aj, d - 1, 2, q, 0, 0, dg2, dlast);
    return pn;
  }
  if (m == d - 2) {  // one progression of coordinate d-2 over [lo, hi]
    uint32_t v0 = 0;
    const uint32_t c = prog_count(A, dg2, x, lo, hi, &v0);
    walk_chunk<WRITE>(A, O, lane, lane == 0 ? c : 0u, aj, d - 2, 1, 0, v0, x, dg2, dlast);
    return c;
  }
  const int l = d - 3;
  const DivMod32 dgl = A.dg[l];
  uint32_t rj = 0;  // lanes m..l-1: the remainder after coordinate j
  uint32_t y = x;   // the remainder before coordinate l
  if (m < l) {
    const uint32_t rm = x - lo * gj;  // lane m's value of gj is g_m
    const uint32_t r0 = __builtin_amdgcn_readlane(rm, m);
    if (lane == m) aj = lo;
    if (lane >= m && lane < l) rj = r0;
    y = r0;
  }
  uint64_t rows = 0;
  for (;;) {
    const uint32_t vlo = m == l ? lo : 0u;
    uint32_t vhi = dgl.div(y);
    if (m == l && hi < vhi) vhi = hi;
    for (uint64_t vb = vlo; vb <= vhi; vb += 64) {
      const uint64_t v64 = vb + uint64_t(lane);
      const bool act = v64 <= vhi;
      const uint32_t v = uint32_t(v64);
      const uint32_t R = act ? y - v * dgl.d : 0u;
      uint32_t v0 = 0;
      const uint32_t c = act ? prog_count(A, dg2, R, 0, 0xffffffffu, &v0) : 0u;
      rows += walk_chunk<WRITE>(A, O, lane, c, aj, l, 0, v, v0, R, dg2, dlast);
    }
    if (m >= l) break;
    // Odometer over coordinates m..l-1: the deepest one that can still grow.
    const bool can = lane >= m && lane < l && rj >= gj && (lane != m || aj < hi);
    const uint64_t mask = __ballot(can);
    if (mask == 0) break;
    const int js = 63 - __clzll((unsigned long long)mask);
    if (lane == js) {
      aj += 1;
      rj -= gj;
    }
    const uint32_t nrem = __builtin_amdgcn_readlane(rj, js);
    if (lane > js && lane < l) {
      aj = 0;
      rj = nrem;
    }
    y = __builtin_amdgcn_readlane(rj, l - 1);
  }
  if (!WRITE) {  // this lane's rows summed over the wavefront
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rows += __shfl_xor(rows, off, 64);
  }
  return rows;
}

// Pass 1 (WRITE = false): each wavefront counts records w, w + W, ... into
// cnt.  Pass 2 (WRITE = true): the same walks write each record's rows at
// off[record].
template <bool WRITE>
__global__ __launch_bounds__(kWalkThreads) void k_walk(WalkArgs A) {
  extern __shared__ uint32_t lds[];  // per wavefront: ring (kWalkRing x d words), 64 marks
  const int lane = int(threadIdx.x & 63);
  const int wave = int(threadIdx.x >> 6);
  const uint32_t wave_words = kWalkRing * uint32_t(A.d) + 64;
  RecordOut O;
  O.ring = lds + uint32_t(wave) * wave_words;
  O.marks = O.ring + kWalkRing * uint32_t(A.d);
  const uint32_t gj = lane < A.d ? A.g.g[lane] : 0u;
  const uint64_t waves = uint64_t(gridDim.x) * kWalkWaves;
  for (uint64_t rec = uint64_t(blockIdx.x) * kWalkWaves + uint64_t(wave); rec < A.nprefix;
       rec += waves) {
    O.produced = 0;
    O.flushed = 0;
    if (WRITE) {
      O.base = A.off[rec];
      O.cnt = A.off[rec + 1] - O.base;
      if (O.cnt == 0) continue;
    }
    const uint64_t rows = walk_record<WRITE>(A, rec, O, lane, gj);
    if (!WRITE) {
      if (lane == 0) A.cnt[rec] = rows;
    } else if (O.produced > O.flushed) {
      walk_flush(A, O.ring, O.base, O.cnt, O.flushed, uint32_t(O.produced - O.flushed), lane);
      wave_sync_walk();
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
  A.dd = DivMod32::make(uint32_t(d));
  A.nprefix = np;
  A.pre = reinterpret_cast<const uint32_t*>(c.pre.p);
  A.cnt = reinterpret_cast<uint64_t*>(c.cnt.p);
  A.off = reinterpret_cast<const uint64_t*>(c.off.p);
  A.out = out;
  // One wavefront per record (records w, w + W, ... beyond the grid).
  const uint64_t blocks = std::min<uint64_t>((np + kWalkWaves - 1) / kWalkWaves, 65535);
  const size_t ring_bytes = size_t(kWalkWaves) * (kWalkRing * uint32_t(d) + 64) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_walk<false>, dim3(uint32_t(blocks)), dim3(kWalkThreads), 0, s, A);
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
    hipLaunchKernelGGL(k_walk<true>, dim3(uint32_t(blocks)), dim3(kWalkThreads), ring_bytes, s,
                       A);
    ZSET_HIP(hipGetLastError());
    ZSET_HIP(hipStreamSynchronize(s));
  }
  *rows_written = total;
  return ZSET_OK;
}
