// batch.hip -- the batched C ABI (zset_batch_*): many independent queries
// planned once and enumerated by one persistent write launch per run.
//
// Create: the count tables of every query are computed on the GPU (one
// workgroup per query) and their totals and row sums read back once.  From
// them the host picks, per query, the memo dimension k (the largest k >= 2
// whose memo fits the LDS budgets of the memo recurrence and of the write pass
// and whose recurrence is at most max_chain_steps elementwise batches long,
// else k = 1, whose memo is the recurrence's closed solution), the slice
// length, the output offset, and cuts the slices into work units of at most
// unit_tiles slices, sorted largest first.  Every device buffer is allocated
// here.
//
// Run: reset -> count tables -> memo recurrences (one wavefront per query,
// Lemma 2.3 in batches of min(h)) -> class ends and leaf layouts -> slice
// starts -> one persistent write launch over the unit queue -> d = 1
// queries.  The sequence is captured into a HIP graph at the first run and
// replayed afterwards (re-captured when the output pointer changes).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {
namespace {

// zset_batch_create refuses every batch while this is set (see zset_batch_create).
constexpr bool kBatchSwitchedOff = true;

constexpr uint32_t kCountLdsSmall = 4096;   // N bound of the small-table launch
constexpr uint32_t kDefaultChainSteps = 4096;
constexpr uint32_t kDefaultUnitTiles = 64;
constexpr uint64_t kMaxTileRows = 2048;

struct QueryPlan {
  uint64_t n = 0;
  int d = 0;
  uint32_t g[kMaxD] = {};
  uint64_t total = 0;
  uint64_t sums[kMaxD + 1] = {};
  int k = 0, U = 0, L = 0;
  uint64_t T = 0, ntiles = 0;
  uint64_t out_off = 0;
  uint64_t table_off = 0;   // uint64 elements
  uint64_t Rn = 0;          // memo rows over p <= n
  uint64_t off_off = 0;     // uint64 elements (N + 1 per memo query)
  uint64_t nat_off = 0;     // uint32 words
  uint64_t leaf_off = 0;    // uint32 words (16-byte aligned)
  uint64_t leaf_words = 0;
  uint64_t endc_off = 0;    // uint64 elements
  uint64_t state_off = 0;   // uint32 words
  uint32_t chain_lds = 0;   // bytes of the memo recurrence workgroup
  EnumParams P{};
};

inline uint64_t align4(uint64_t words) { return (words + 3) & ~uint64_t(3); }

// LDS of one memo-recurrence workgroup under automatic k (a larger one would
// lower the occupancy of every recurrence in the launch).
constexpr size_t kAutoChainLds = 64 * 1024;

template <class T>
T* at(DevBuf& b, uint64_t elems) {
  return reinterpret_cast<T*>(b.p) + elems;
}

zset_status upload(DevBuf& b, const void* host, size_t bytes) {
  zset_status st = ensure(b, bytes);
  if (st != ZSET_OK) return st;
  if (bytes) ZSET_HIP(hipMemcpy(b.p, host, bytes, hipMemcpyHostToDevice));
  return ZSET_OK;
}

// Bits of the packed leaf-order memo row (floor(p/G), m_1..m_k) for p <= n.
int pack_fields(const QueryPlan& q, uint32_t* fshift, uint32_t* fmask) {
  uint32_t shift = 0;
  for (int c = 0; c <= q.k; ++c) {
    const uint32_t vmax = uint32_t(q.n / q.g[q.U + c]);
    uint32_t bits = 0;
    while (bits < 32 && (uint64_t(vmax) >> bits) != 0) ++bits;
    fshift[c] = shift;
    fmask[c] = bits >= 32 ? ~0u : ((1u << bits) - 1u);
    shift += bits;
  }
  return shift <= 32 ? 1 : (shift <= 64 ? 2 : 0);
}

}  // namespace
}  // namespace zset

using namespace zset;

struct zset_batch_s {
  int device = -1;
  int nq = 0;
  zset_batch_opts opts{};
  std::vector<QueryPlan> q;
  uint64_t total_words = 0, total_rows = 0, total_tiles = 0;
  uint32_t nunits = 0, write_blocks = 0, memo_queries = 0;
  uint32_t count_small_max = 0, count_mid_max = 0;
  uint32_t n_count_small = 0, n_count_mid = 0, n_count_big = 0;
  uint32_t n_chain8 = 0, n_chain32 = 0, n_k1 = 0, k1_blocks = 0;
  size_t chain8_lds = 0, chain32_lds = 0;
  uint32_t n_leaf = 0, leaf_blocks = 0, n_single = 0, n_plan = 0;
  BatchLds L{};
  // device memory
  DevBuf table, sums, totals, qp, qout, tile_base, plan_q, units;
  DevBuf count_jobs, memo_jobs, class_jobs, leaf_jobs, single_idx;
  DevBuf off, nat, leaf, endc, tiles;
  DevBuf done_tiles, checksums, t_done, misc;  // misc: [0] queue, [1] err, [2] t_start
  hipEvent_t ev[6] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t* graph_out = nullptr;
  int wall_khz = 0;
};

namespace {

void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

void destroy(zset_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  for (DevBuf* p : {&b->table, &b->sums, &b->totals, &b->qp, &b->qout, &b->tile_base,
                    &b->plan_q, &b->units, &b->count_jobs, &b->memo_jobs, &b->class_jobs,
                    &b->leaf_jobs, &b->single_idx, &b->off, &b->nat, &b->leaf, &b->endc,
                    &b->tiles, &b->done_tiles, &b->checksums, &b->t_done, &b->misc})
    free_buf(*p);
  delete b;
}

uint32_t* misc_queue(zset_batch b) { return at<uint32_t>(b->misc, 0); }
int* misc_err(zset_batch b) { return reinterpret_cast<int*>(at<uint32_t>(b->misc, 2)); }
uint64_t* misc_t_start(zset_batch b) { return at<uint64_t>(b->misc, 2); }

const CountJob* count_jobs_at(zset_batch b, uint32_t first) {
  return at<CountJob>(b->count_jobs, first);
}

// The count-table launches: small tables (LDS), mid tables (LDS), large ones
// (global memory).
zset_status launch_counts(zset_batch b, hipStream_t s) {
  ZSET_HIP(launch_count_table_batch(count_jobs_at(b, 0), b->n_count_small, b->count_small_max,
                                    true, s));
  ZSET_HIP(launch_count_table_batch(count_jobs_at(b, b->n_count_small), b->n_count_mid,
                                    b->count_mid_max, true, s));
  ZSET_HIP(launch_count_table_batch(count_jobs_at(b, b->n_count_small + b->n_count_mid),
                                    b->n_count_big, 0, false, s));
  return ZSET_OK;
}

zset_status launch_stages(zset_batch b, uint32_t* out, hipStream_t s, bool timed) {
  const bool co = b->opts.count_only != 0;
  int* err = misc_err(b);
  if (timed) ZSET_HIP(hipEventRecord(b->ev[0], s));
  ZSET_HIP(launch_batch_reset(misc_queue(b), err, at<uint32_t>(b->done_tiles, 0),
                              at<uint64_t>(b->checksums, 0), at<uint64_t>(b->t_done, 0),
                              misc_t_start(b), uint32_t(b->nq), s));
  zset_status st = launch_counts(b, s);
  if (st != ZSET_OK) return st;
  if (timed) ZSET_HIP(hipEventRecord(b->ev[1], s));
  const MemoJob* mj = at<MemoJob>(b->memo_jobs, 0);
  ZSET_HIP(launch_memo_chain_batch(mj, b->n_chain8, 8, b->chain8_lds, err, s, false));
  ZSET_HIP(launch_memo_chain_batch(mj + b->n_chain8, b->n_chain32, kMaxD, b->chain32_lds, err, s,
                                   false));
  ZSET_HIP(launch_memo_k1_batch(mj + b->n_chain8 + b->n_chain32, b->n_k1, b->k1_blocks, s));
  ZSET_HIP(launch_class_ends_batch(at<ClassJob>(b->class_jobs, 0), b->n_leaf, s));
  ZSET_HIP(launch_memo_leaf_batch(at<LeafJob>(b->leaf_jobs, 0), b->n_leaf, b->leaf_blocks, err, s));
  if (timed) ZSET_HIP(hipEventRecord(b->ev[2], s));
  ZSET_HIP(launch_plan_batch(at<EnumParams>(b->qp, 0), at<uint64_t>(b->tile_base, 0),
                             at<uint32_t>(b->plan_q, 0), b->n_plan, b->total_tiles, s));
  if (timed) ZSET_HIP(hipEventRecord(b->ev[3], s));
  ZSET_HIP(launch_write_batch(at<EnumParams>(b->qp, 0), at<uint64_t>(b->qout, 0),
                              at<BatchUnit>(b->units, 0), b->nunits, misc_queue(b),
                              at<uint32_t>(b->done_tiles, 0), at<uint64_t>(b->t_done, 0), out,
                              b->L, b->write_blocks, co, s));
  ZSET_HIP(launch_single_batch(at<EnumParams>(b->qp, 0), at<uint64_t>(b->qout, 0),
                               at<uint32_t>(b->single_idx, 0), b->n_single, out, co,
                               at<uint64_t>(b->t_done, 0), s));
  if (timed) ZSET_HIP(hipEventRecord(b->ev[4], s));
  return ZSET_OK;
}

zset_status plan_queries(zset_batch b, const int* kreq, const uint64_t* treq, int cus) {
  const uint32_t max_steps = b->opts.max_chain_steps ? b->opts.max_chain_steps : kDefaultChainSteps;
  const uint32_t unit_tiles = b->opts.unit_tiles ? b->opts.unit_tiles : kDefaultUnitTiles;
  const uint32_t lds_words = uint32_t(write_lds_budget(b->device) / 4);
  const bool co = b->opts.count_only != 0;

  int dmax = 1;
  for (auto& q : b->q) dmax = std::max(dmax, q.d);
  const uint32_t ring = dmax <= 16 ? 128 : 64;
  const uint32_t wave_words = uint32_t(align4(uint64_t(ring) * dmax) + kWave);
  const uint32_t desc_words = uint32_t(align4(sizeof(EnumParams) / 4));
  const uint32_t waves = uint32_t(write_batch_waves());
  // Slice starts of one unit: unit_tiles x (U + 2) <= unit_tiles x (dmax + 1).
  const uint32_t state_words = uint32_t(align4(uint64_t(unit_tiles) * (dmax + 1)));
  const uint64_t fixed = uint64_t(desc_words) + state_words + uint64_t(waves) * wave_words;
  if (fixed + 64 > lds_words)
    return fail(ZSET_EINVAL, "unit_tiles too large for the write pass's LDS");
  const uint64_t spare = lds_words - fixed;
  const uint64_t memo_cap = spare / 2;                // packed memo words in LDS
  const uint64_t cnt_cap = spare - memo_cap;          // segment counts + class ends
  const size_t lds_max_bytes = size_t(device_max_lds_bytes(b->device));

  for (int i = 0; i < b->nq; ++i) {
    QueryPlan& q = b->q[i];
    const uint64_t N = q.n + 1;
    auto memo_ok = [&](int kk, size_t cap, std::string* why) -> bool {
      const int L = q.d - kk;
      const uint64_t R = q.sums[L];
      uint32_t hmin = q.g[L], hmax = q.g[L];
      for (int j = L; j < q.d; ++j) {
        hmin = std::min(hmin, q.g[j]);
        hmax = std::max(hmax, q.g[j]);
      }
      const uint32_t step = std::min<uint32_t>(hmin, kWave);
      const uint64_t Wl = uint64_t(hmax) + step;
      if (R >= (uint64_t(1) << 30) || Wl >= (uint64_t(1) << 30)) {
        if (why) *why = "memo too large";
        return false;
      }
      const uint32_t W = next_pow2(uint32_t(Wl));
      if (memo_wave_lds_bytes(kk, R, W) > cap) {
        if (why) *why = "memo recurrence does not fit in LDS";
        return false;
      }
      return true;
    };
    if (q.d == 1 || q.total == 0) {
      q.k = 0;
    } else if (kreq && kreq[i] >= 0) {
      if (kreq[i] > q.d - 1) return fail(ZSET_EINVAL, "query " + std::to_string(i) + ": k > d-1");
      q.k = kreq[i];
      std::string why;
      if (q.k >= 2 && !memo_ok(q.k, lds_max_bytes, &why))
        return fail(ZSET_EINVAL, "query " + std::to_string(i) + ": " + why);
    } else {
      // Largest k >= 2 whose recurrence is short enough and whose memo fits
      // the LDS budgets (recurrence and write pass); else k = 1, whose memo
      // is the recurrence's closed solution (any size; copied from global
      // memory when it does not fit LDS).
      q.k = 1;
      for (int kk = q.d - 1; kk >= 2; --kk) {
        const int L = q.d - kk;
        const uint64_t R = q.sums[L];
        uint32_t hmin = q.g[L];
        for (int j = L; j < q.d; ++j) hmin = std::min(hmin, q.g[j]);
        const uint32_t step = std::min<uint32_t>(hmin, kWave);
        const uint64_t steps = (N + step - 1) / step;
        if (R == ~uint64_t(0) || R > std::max<uint64_t>(4096, q.total / 16)) continue;
        if (steps > max_steps || !memo_ok(kk, std::min(kAutoChainLds, lds_max_bytes), nullptr))
          continue;
        QueryPlan t = q;
        t.k = kk;
        t.L = q.d - kk;
        t.U = t.L - 1;
        uint32_t fs[kMaxD + 1], fm[kMaxD + 1];
        const int pk = pack_fields(t, fs, fm);
        if (pk == 0 || R * uint64_t(pk) > memo_cap) continue;
        q.k = kk;
        break;
      }
    }
    q.L = q.d - std::max(q.k, 1);
    q.U = (q.k == 0) ? q.d - 1 : q.L - 1;
    if (treq && treq[i]) {
      if (treq[i] % 128 != 0 || treq[i] > (uint64_t(1) << 30))
        return fail(ZSET_EINVAL, "rows_per_tile must be a multiple of 128 and at most 2^30");
      q.T = treq[i];
    } else {
      uint64_t T = (q.total + 255) / 256;
      T = (T + 127) / 128 * 128;
      q.T = std::min(std::max<uint64_t>(T, 128), kMaxTileRows);
    }
    q.ntiles = (q.d >= 2 && q.total > 0) ? (q.total + q.T - 1) / q.T : 0;
  }

  // Offsets of every per-query region.
  uint64_t tab = 0, outw = 0, offe = 0, natw = 0, leafw = 0, endce = 0, statew = 0, tiles = 0;
  uint64_t memo_max_words = 0, cnt_max_words = 0, endc_max_words = 0;
  std::vector<uint64_t> tile_base;
  std::vector<uint32_t> plan_q;
  std::vector<MemoJob> chain8, chain32, k1;
  uint32_t k1_blocks = 0;
  std::vector<ClassJob> cjobs;
  std::vector<LeafJob> ljobs;
  std::vector<uint32_t> single;
  uint32_t leaf_blocks = 0;
  b->memo_queries = 0;
  for (int i = 0; i < b->nq; ++i) {
    QueryPlan& q = b->q[i];
    const uint64_t N = q.n + 1;
    q.table_off = tab;
    tab += uint64_t(q.d + 1) * N;
    q.out_off = outw;
    if (!co) {
      if (q.total > (~uint64_t(0) - outw) / uint64_t(q.d) - 4)
        return fail(ZSET_EOVERFLOW, "batch output exceeds 2^64 words");
      outw += align4(q.total * uint64_t(q.d));
    }
    EnumParams& P = q.P;
    std::memset(&P, 0, sizeof P);
    for (int j = 0; j < q.d; ++j) P.g.g[j] = q.g[j];
    P.n = uint32_t(q.n);
    P.d = q.d;
    P.U = q.U;
    P.k = q.k;
    P.total = q.total;
    P.rows_per_tile = q.T;
    P.ntiles = q.ntiles;
    P.ring = ring;
    P.flush = ring / 2;
    P.dG = DivMod32::make(q.g[q.U]);
    if (q.d == 1) {
      single.push_back(uint32_t(i));
      continue;
    }
    if (q.ntiles == 0) continue;
    q.state_off = statew;
    statew += q.ntiles * uint64_t(q.U + 2);
    tile_base.push_back(tiles);
    plan_q.push_back(uint32_t(i));
    tiles += q.ntiles;
    if (q.k >= 1) {
      ++b->memo_queries;
      q.Rn = q.sums[q.L];
      P.pack = pack_fields(q, P.fshift, P.fmask);
      if (P.pack != 0 && q.Rn * uint64_t(P.pack) > memo_cap) P.pack = 0;
      P.memo_words = P.pack ? q.Rn * uint64_t(P.pack) : 0;
      P.nclass = uint32_t(std::min<uint64_t>(q.g[q.U], N));
      if (q.sums[q.U] < (uint64_t(1) << 32) && q.Rn < (uint64_t(1) << 32) &&
          align4(N) + align4(P.nclass) <= cnt_cap)
        P.lds_cnt = 1;
      if (P.pack) memo_max_words = std::max(memo_max_words, align4(P.memo_words));
      if (P.lds_cnt) {
        cnt_max_words = std::max(cnt_max_words, align4(N));
        endc_max_words = std::max(endc_max_words, align4(P.nclass));
      }
      q.leaf_words = P.pack ? q.Rn * uint64_t(P.pack) : q.Rn * uint64_t(q.k + 1);
      q.off_off = offe;
      offe += N + 1;
      q.nat_off = natw;
      natw += q.Rn * uint64_t(q.k);
      q.leaf_off = leafw;
      leafw += align4(q.leaf_words);
      q.endc_off = endce;
      endce += P.nclass;
      P.leaf_rows = q.Rn;

      MemoJob J;
      std::memset(&J, 0, sizeof J);
      uint32_t hmin = q.g[q.L], hmax = q.g[q.L];
      for (int j = 0; j < q.k; ++j) {
        J.h[j] = q.g[q.L + j];
        hmin = std::min(hmin, J.h[j]);
        hmax = std::max(hmax, J.h[j]);
      }
      J.k = q.k;
      J.top = uint32_t(N);
      J.step = std::min<uint32_t>(hmin, kWave);
      J.W = next_pow2(hmax + J.step);
      J.R = uint32_t(q.Rn);
      if (q.Rn >= (uint64_t(1) << 32)) return fail(ZSET_EOVERFLOW, "a memo has 2^32 rows or more");
      if (q.k == 1) {
        if (q.Rn != q.n / q.g[q.L] + 1) return fail(ZSET_EDEVICE, "internal: k = 1 memo rows");
        J.block0 = k1_blocks;
        const uint64_t nb = memo_k1_blocks(N);
        if (uint64_t(k1_blocks) + nb > 0x7fffffffull)
          return fail(ZSET_EINVAL, "batch too large for the k = 1 memo launch");
        k1_blocks += uint32_t(nb);
        k1.push_back(J);
        continue;
      }
      const size_t lds = memo_wave_lds_bytes(q.k, q.Rn, J.W);
      q.chain_lds = uint32_t(lds);
      if (q.k <= 8) {
        chain8.push_back(J);
        b->chain8_lds = std::max(b->chain8_lds, lds);
      } else {
        chain32.push_back(J);
        b->chain32_lds = std::max(b->chain32_lds, lds);
      }
    }
  }
  b->total_words = outw;
  b->total_tiles = tiles;
  b->n_plan = uint32_t(plan_q.size());
  b->n_single = uint32_t(single.size());
  b->n_chain8 = uint32_t(chain8.size());
  b->n_chain32 = uint32_t(chain32.size());
  b->n_k1 = uint32_t(k1.size());
  b->k1_blocks = k1_blocks;

  // LDS layout of the persistent write launch.
  BatchLds& L = b->L;
  L.desc = 0;
  L.memo = desc_words;
  L.cnt = uint32_t(L.memo + memo_max_words);
  L.endc = uint32_t(L.cnt + cnt_max_words);
  L.states = uint32_t(L.endc + endc_max_words);
  L.waves = L.states + state_words;
  L.ring_words = uint32_t(align4(uint64_t(ring) * dmax));
  L.wave_words = wave_words;
  L.total_words = L.waves + waves * wave_words;
  if (L.total_words > lds_words) return fail(ZSET_EINVAL, "batch LDS layout exceeds the device");

  // Allocations.
  zset_status st;
  const uint64_t nq = uint64_t(b->nq);
  if ((st = ensure(b->off, std::max<uint64_t>(offe, 1) * 8)) != ZSET_OK) return st;
  if ((st = ensure(b->nat, std::max<uint64_t>(natw, 1) * 4)) != ZSET_OK) return st;
  if ((st = ensure(b->leaf, std::max<uint64_t>(leafw, 4) * 4)) != ZSET_OK) return st;
  if ((st = ensure(b->endc, std::max<uint64_t>(endce, 1) * 8)) != ZSET_OK) return st;
  if ((st = ensure(b->tiles, std::max<uint64_t>(statew, 1) * 4)) != ZSET_OK) return st;
  if ((st = ensure(b->done_tiles, nq * 4)) != ZSET_OK) return st;
  if ((st = ensure(b->checksums, nq * 8)) != ZSET_OK) return st;
  if ((st = ensure(b->t_done, nq * 8)) != ZSET_OK) return st;

  // Device pointers in the descriptors and jobs.
  std::vector<EnumParams> qp(b->nq);
  std::vector<uint64_t> qout(b->nq);
  uint64_t* table0 = at<uint64_t>(b->table, 0);
  int* err = misc_err(b);
  size_t c8 = 0, c32 = 0, ck1 = 0;
  for (int i = 0; i < b->nq; ++i) {
    QueryPlan& q = b->q[i];
    const uint64_t N = q.n + 1;
    EnumParams& P = q.P;
    P.table = table0 + q.table_off;
    P.table_stride = q.n + 1;
    P.err = err;
    P.checksum = at<uint64_t>(b->checksums, uint64_t(i));
    P.out = nullptr;
    if (q.ntiles > 0) P.tiles = at<uint32_t>(b->tiles, q.state_off);
    if (q.k >= 1 && q.ntiles > 0) {
      uint64_t* off = at<uint64_t>(b->off, q.off_off);
      uint32_t* nat = at<uint32_t>(b->nat, q.nat_off);
      uint32_t* leaf = at<uint32_t>(b->leaf, q.leaf_off);
      uint64_t* endc = at<uint64_t>(b->endc, q.endc_off);
      MemoJob& J = q.k == 1 ? k1[ck1++] : (q.k <= 8 ? chain8[c8++] : chain32[c32++]);
      J.nat = nat;
      J.off = off;
      P.leaf = leaf;
      P.endc = endc;
      const uint64_t* cu = P.table + uint64_t(q.U) * N;
      ClassJob C;
      std::memset(&C, 0, sizeof C);
      C.cu = cu;
      C.endc = endc;
      C.n = uint32_t(q.n);
      C.nclass = P.nclass;
      C.dG = DivMod32::make(q.g[q.U]);
      cjobs.push_back(C);
      LeafJob LJ = make_leaf_job(q.k, q.n, q.g[q.U], off, nat, cu, endc, leaf, q.Rn, P);
      LJ.block0 = leaf_blocks;
      const uint64_t nb = (N + 255) / 256;
      if (uint64_t(leaf_blocks) + nb > 0x7fffffffull)
        return fail(ZSET_EINVAL, "batch too large for the leaf-layout launch");
      leaf_blocks += uint32_t(nb);
      ljobs.push_back(LJ);
    }
    qp[i] = P;
    qout[i] = q.out_off;
  }
  b->n_leaf = uint32_t(ljobs.size());
  b->leaf_blocks = leaf_blocks;
  std::vector<MemoJob> mj;
  mj.reserve(chain8.size() + chain32.size() + k1.size());
  mj.insert(mj.end(), chain8.begin(), chain8.end());
  mj.insert(mj.end(), chain32.begin(), chain32.end());
  mj.insert(mj.end(), k1.begin(), k1.end());

  // Work units, largest first.
  std::vector<BatchUnit> units;
  std::vector<uint64_t> unit_rows;
  for (int i = 0; i < b->nq; ++i) {
    const QueryPlan& q = b->q[i];
    for (uint64_t lo = 0; lo < q.ntiles; lo += unit_tiles) {
      const uint64_t hi = std::min<uint64_t>(q.ntiles, lo + unit_tiles);
      if (hi > 0xffffffffull) return fail(ZSET_EINVAL, "a query has more than 2^32 slices");
      units.push_back(BatchUnit{uint32_t(i), uint32_t(lo), uint32_t(hi), 0});
      unit_rows.push_back(std::min(q.total, hi * q.T) - lo * q.T);
    }
  }
  std::vector<uint32_t> order(units.size());
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t c) { return unit_rows[a] > unit_rows[c]; });
  std::vector<BatchUnit> sorted(units.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = units[order[i]];
  b->nunits = uint32_t(sorted.size());

  if ((st = upload(b->qp, qp.data(), qp.size() * sizeof(EnumParams))) != ZSET_OK) return st;
  if ((st = upload(b->qout, qout.data(), qout.size() * 8)) != ZSET_OK) return st;
  if ((st = upload(b->tile_base, tile_base.data(), tile_base.size() * 8)) != ZSET_OK) return st;
  if ((st = upload(b->plan_q, plan_q.data(), plan_q.size() * 4)) != ZSET_OK) return st;
  if ((st = upload(b->units, sorted.data(), sorted.size() * sizeof(BatchUnit))) != ZSET_OK)
    return st;
  if ((st = upload(b->memo_jobs, mj.data(), mj.size() * sizeof(MemoJob))) != ZSET_OK) return st;
  if ((st = upload(b->class_jobs, cjobs.data(), cjobs.size() * sizeof(ClassJob))) != ZSET_OK)
    return st;
  if ((st = upload(b->leaf_jobs, ljobs.data(), ljobs.size() * sizeof(LeafJob))) != ZSET_OK)
    return st;
  if ((st = upload(b->single_idx, single.data(), single.size() * 4)) != ZSET_OK) return st;

  // Launch attributes (set before any graph capture) and the persistent grid.
  ZSET_HIP(launch_memo_chain_batch(nullptr, b->n_chain8 ? 1 : 0, 8, b->chain8_lds, nullptr,
                                   nullptr, true));
  ZSET_HIP(launch_memo_chain_batch(nullptr, b->n_chain32 ? 1 : 0, kMaxD, b->chain32_lds, nullptr,
                                   nullptr, true));
  int per_cu = 0;
  ZSET_HIP(write_batch_occupancy(L, co, &per_cu));
  if (per_cu < 1) return fail(ZSET_EDEVICE, "the batched write pass does not fit on a compute unit");
  b->write_blocks = uint32_t(std::max<uint64_t>(
      1, std::min<uint64_t>(uint64_t(cus) * per_cu, std::max<uint32_t>(b->nunits, 1))));
  return ZSET_OK;
}

}  // namespace

extern "C" {

void zset_batch_default_opts(zset_batch_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->use_graph = 1;
}

zset_status zset_batch_create(int nq, const uint64_t* n, const int* d, const uint32_t* gens,
                              const int* k, const uint64_t* rows_per_tile,
                              const zset_batch_opts* opts, zset_batch* out_batch) {
  g_last_error.clear();
  if (!out_batch) return fail(ZSET_EINVAL, "batch is NULL");
  *out_batch = nullptr;
  // Switched off: the first device run of a batch stopped responding and the
  // cause is not identified yet, so no batch work reaches the device.
  if (kBatchSwitchedOff)
    return fail(ZSET_EDEVICE, "batched enumeration is switched off in this version");
  if (nq < 1) return fail(ZSET_EINVAL, "nq must be >= 1");
  if (!n || !d || !gens) return fail(ZSET_EINVAL, "n, d and gens must be non-NULL");
  zset_batch_opts o;
  if (opts) o = *opts; else zset_batch_default_opts(&o);
  if (o.unit_tiles > 4096) return fail(ZSET_EINVAL, "unit_tiles must be at most 4096");

  zset_batch b = new zset_batch_s();
  b->nq = nq;
  b->opts = o;
  b->q.resize(nq);
  auto bail = [&](zset_status st) {
    destroy(b);
    return st;
  };
  uint64_t goff = 0;
  for (int i = 0; i < nq; ++i) {
    QueryPlan& q = b->q[i];
    zset_status st = check_query(n[i], gens + goff, d[i]);
    if (st != ZSET_OK)
      return bail(fail(st, "query " + std::to_string(i) + ": " + g_last_error));
    q.n = n[i];
    q.d = d[i];
    for (int j = 0; j < q.d; ++j) q.g[j] = gens[goff + j];
    goff += uint64_t(d[i]);
  }

  std::lock_guard<std::mutex> lock(g_mu);
  if (hipGetDevice(&b->device) != hipSuccess) return bail(hip_fail(hipGetLastError(), "hipGetDevice"));
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
    return bail(hip_fail(hipGetLastError(), "hipDeviceGetAttribute"));
  if (hipDeviceGetAttribute(&b->wall_khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess) {
    (void)hipGetLastError();
    b->wall_khz = 0;
  }
  for (auto& e : b->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(hip_fail(hipGetLastError(), "hipEventCreate"));

  // Count tables: small and mid tables in LDS, large ones in global memory.
  uint64_t tab = 0;
  std::vector<uint32_t> idx(nq);
  std::iota(idx.begin(), idx.end(), 0u);
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t c) {
    auto cls = [&](uint32_t i) {
      const uint64_t N = b->q[i].n + 1;
      return N <= kCountLdsSmall ? 0 : (N <= count_table_lds_max() ? 1 : 2);
    };
    return cls(a) < cls(c);
  });
  std::vector<uint64_t> table_off(nq);
  for (int i = 0; i < nq; ++i) {
    table_off[i] = tab;
    tab += uint64_t(b->q[i].d + 1) * (b->q[i].n + 1);
  }
  zset_status st;
  if ((st = ensure(b->table, tab * 8)) != ZSET_OK) return bail(st);
  if ((st = ensure(b->sums, uint64_t(nq) * (kMaxD + 1) * 8)) != ZSET_OK) return bail(st);
  if ((st = ensure(b->totals, uint64_t(nq) * 8)) != ZSET_OK) return bail(st);
  if ((st = ensure(b->misc, 64)) != ZSET_OK) return bail(st);
  std::vector<CountJob> cj(nq);
  for (int r = 0; r < nq; ++r) {
    const uint32_t i = idx[r];
    const QueryPlan& q = b->q[i];
    CountJob& J = cj[r];
    std::memset(&J, 0, sizeof J);
    J.table = at<uint64_t>(b->table, table_off[i]);
    J.sums = at<uint64_t>(b->sums, uint64_t(i) * (kMaxD + 1));
    J.total = at<uint64_t>(b->totals, i);
    J.N = uint32_t(q.n + 1);
    J.d = q.d;
    for (int j = 0; j < q.d; ++j) J.g[j] = q.g[j];
    if (J.N <= kCountLdsSmall) {
      ++b->n_count_small;
      b->count_small_max = std::max(b->count_small_max, J.N);
    } else if (J.N <= count_table_lds_max()) {
      ++b->n_count_mid;
      b->count_mid_max = std::max(b->count_mid_max, J.N);
    } else {
      ++b->n_count_big;
    }
  }
  if ((st = upload(b->count_jobs, cj.data(), cj.size() * sizeof(CountJob))) != ZSET_OK)
    return bail(st);
  if (hipError_t e = prepare_count_table_batch(count_table_lds_max()); e != hipSuccess)
    return bail(hip_fail(e, "prepare_count_table_batch"));
  if ((st = launch_counts(b, nullptr)) != ZSET_OK) return bail(st);
  if (hipError_t e = hipDeviceSynchronize(); e != hipSuccess)
    return bail(hip_fail(e, "batch count tables"));
  std::vector<uint64_t> sums(uint64_t(nq) * (kMaxD + 1)), totals(nq);
  if (hipMemcpy(sums.data(), b->sums.p, sums.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(totals.data(), b->totals.p, totals.size() * 8, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return bail(hip_fail(hipGetLastError(), "batch count readback"));
  for (int i = 0; i < nq; ++i) {
    QueryPlan& q = b->q[i];
    q.total = totals[i];
    for (int j = 0; j <= q.d; ++j) q.sums[j] = sums[uint64_t(i) * (kMaxD + 1) + j];
    if (q.total == ~uint64_t(0))
      return bail(fail(ZSET_EOVERFLOW, "query " + std::to_string(i) + ": |Z(n)| >= 2^64 - 1"));
    if (q.total > (~uint64_t(0)) / (4 * uint64_t(q.d)))
      return bail(fail(ZSET_EOVERFLOW, "query " + std::to_string(i) + ": rows * d overflows"));
    b->total_rows += q.total;
  }
  if ((st = plan_queries(b, k, rows_per_tile, cus)) != ZSET_OK) return bail(st);
  // The tables were laid out in query order above; plan_queries recomputes the
  // same offsets.
  for (int i = 0; i < nq; ++i)
    if (b->q[i].table_off != table_off[i])
      return bail(fail(ZSET_EDEVICE, "internal: table layout mismatch"));
  *out_batch = b;
  return ZSET_OK;
}

zset_status zset_batch_info(zset_batch b, uint64_t* total_words, uint64_t* rows,
                            uint64_t* offsets, int* k, uint64_t* tiles) {
  g_last_error.clear();
  if (!b) return fail(ZSET_EINVAL, "batch is NULL");
  if (total_words) *total_words = b->total_words;
  for (int i = 0; i < b->nq; ++i) {
    if (rows) rows[i] = b->q[i].total;
    if (offsets) offsets[i] = b->q[i].out_off;
    if (k) k[i] = b->q[i].k;
    if (tiles) tiles[i] = b->q[i].ntiles;
  }
  return ZSET_OK;
}

zset_status zset_batch_run(zset_batch b, uint32_t* out, uint64_t out_words_cap,
                           uint64_t* checksums, zset_batch_stats* stats) {
  g_last_error.clear();
  if (!b) return fail(ZSET_EINVAL, "batch is NULL");
  const bool co = b->opts.count_only != 0;
  if (!co) {
    if (!out && b->total_words > 0) return fail(ZSET_EINVAL, "out is NULL");
    if (out && (reinterpret_cast<uintptr_t>(out) & 15) != 0)
      return fail(ZSET_EINVAL, "out must be 16-byte aligned");
    if (out && !is_device_pointer(out)) return fail(ZSET_EINVAL, "out is not device memory");
    if (out_words_cap < b->total_words)
      return fail(ZSET_ECAPACITY, "out holds " + std::to_string(out_words_cap) +
                                      " words, the batch needs " +
                                      std::to_string(b->total_words));
  } else {
    out = nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  ZSET_HIP(hipGetDevice(&dev));
  if (dev != b->device) return fail(ZSET_EINVAL, "batch lives on another device");
  hipStream_t s = reinterpret_cast<hipStream_t>(b->opts.stream);
  ZSET_HIP(prepare_write_batch(b->L, co));
  if (b->opts.use_graph) {
    if (!b->exec || b->graph_out != out) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
      hipStream_t cs = nullptr;
      ZSET_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      zset_status st = ZSET_OK;
      if (e == hipSuccess) {
        st = launch_stages(b, out, cs, false);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (st == ZSET_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
        b->graph = g;
      } else {
        st = hip_fail(e, "hipStreamBeginCapture");
      }
      (void)hipStreamDestroy(cs);
      if (st != ZSET_OK) return st;
      ZSET_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_out = out;
    }
    ZSET_HIP(hipEventRecord(b->ev[0], s));
    ZSET_HIP(hipGraphLaunch(b->exec, s));
    ZSET_HIP(hipEventRecord(b->ev[4], s));
  } else {
    zset_status st = launch_stages(b, out, s, true);
    if (st != ZSET_OK) return st;
  }
  ZSET_HIP(hipStreamSynchronize(s));
  int code = 0;
  ZSET_HIP(hipMemcpy(&code, misc_err(b), sizeof(int), hipMemcpyDeviceToHost));
  if (code != 0) return fail(ZSET_EDEVICE, device_error_text(code));
  if (checksums) {
    if (co) {
      ZSET_HIP(hipMemcpy(checksums, b->checksums.p, uint64_t(b->nq) * 8, hipMemcpyDeviceToHost));
    } else {
      for (int i = 0; i < b->nq; ++i) checksums[i] = 0;
    }
  }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->total_us = elapsed_us(b->ev[0], b->ev[4]);
    if (!b->opts.use_graph) {
      stats->count_us = elapsed_us(b->ev[0], b->ev[1]);
      stats->memo_us = elapsed_us(b->ev[1], b->ev[2]);
      stats->plan_us = elapsed_us(b->ev[2], b->ev[3]);
      stats->write_us = elapsed_us(b->ev[3], b->ev[4]);
    }
    stats->rows = b->total_rows;
    stats->words = b->total_words;
    stats->tiles = b->total_tiles;
    stats->units = b->nunits;
    stats->memo_queries = b->memo_queries;
    stats->write_blocks = b->write_blocks;
    stats->lds_bytes = b->L.total_words * 4;
  }
  return ZSET_OK;
}

zset_status zset_batch_times(zset_batch b, double* done_us) {
  g_last_error.clear();
  if (!b || !done_us) return fail(ZSET_EINVAL, "batch and done_us must be non-NULL");
  if (b->wall_khz <= 0) return fail(ZSET_EDEVICE, "the device reports no wall-clock rate");
  std::vector<uint64_t> t(b->nq);
  uint64_t t0 = 0;
  ZSET_HIP(hipMemcpy(t.data(), b->t_done.p, t.size() * 8, hipMemcpyDeviceToHost));
  ZSET_HIP(hipMemcpy(&t0, misc_t_start(b), 8, hipMemcpyDeviceToHost));
  const double us_per_tick = 1000.0 / double(b->wall_khz);
  for (int i = 0; i < b->nq; ++i)
    done_us[i] = t[i] >= t0 && t[i] != 0 ? double(t[i] - t0) * us_per_tick : 0.0;
  return ZSET_OK;
}

void zset_batch_free(zset_batch b) { destroy(b); }

}  // extern "C"
