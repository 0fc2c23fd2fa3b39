// serve.hip -- a request loop over resident generator sets (zset_server_*).
//
// A generator set g is made resident once, up to an element bound n_max:
//   * its count table C[j][x] = |Z(x; g_j..g_d)| for x <= n_max, on the device,
//     with a host copy of row 0 (|Z(n)| for every n <= n_max), which prices a
//     query's output bytes (|Z(n)| d 4) without touching the device;
//   * for memo dimension k >= 1, the memo Z(p; h) of the trailing k generators
//     for p < top, built by the dynamic recurrence (zset_memo_build), and its
//     leaf-order layout with the residue-class ends.  top = n_max + 1 when
//     that memo fits the server's memo budget, else the largest top whose
//     memo does (a partial memo: the rows of a query with n >= top whose memo
//     remainder is >= top are unranked from the count table, Alg 3.2's Else
//     branch).  A segment Z(x; G, h) starts at end[x mod G] - C_U[x] whatever
//     the query's n, so one layout serves every n <= n_max.
// A query (set, n) then needs only the slice plan and the write pass, with no
// host synchronisation.  Queries run on `slots` streams at once (continuous
// batching): a dispatcher thread admits waiting queries in arrival order as a
// slot and room in the output arena become free, launches them, watches their
// completion flags (pinned host words that the last kernel of a query writes)
// and stamps submit / admit / done times on the host's steady clock.  The rows of a query are the bytes zset_enumerate_ex writes
// for it alone: the kernels and their arguments are the same, only the memo
// covers more elements.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {
namespace {

constexpr int kMaxSlots = 64;
constexpr int kDefaultSlots = 8;
// Slices of one query at most: size_write_pass picks about 128 per resident
// wavefront (and rows_per_tile >= 128 rows below that), so this bounds every
// query's slice table once the device's resident wavefronts are known.
constexpr uint64_t kSlicesPerWave = 128;
// Default memo budget of a resident set (its leaf-order layout): the
// automatic memo dimension is the largest k whose memo over p <= n_max fits
// it, and a larger memo is capped to it.
constexpr uint64_t kResidentMemoBytes = uint64_t(32) << 20;
// Slices per wavefront up to which the write pass plans its own slices.
constexpr uint64_t kFusedSlicesPerWave = 4;

double now_us(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

struct ResidentSet {
  int d = 0, k = 0, L = 0, U = 0;
  uint32_t g[kMaxD] = {};
  uint64_t n_max = 0;
  std::vector<uint64_t> c0;  // |Z(n)| for n <= n_max
  DevBuf table, endc, leaf;
  uint64_t memo_rows = 0;
  uint64_t memo_top = 0;     // the memo covers p < memo_top (n_max + 1: every p)
  uint64_t sum_u = 0;        // sum over x <= n_max of C_U[x]
  EnumParams tmpl;           // per-set fields of the write pass
};

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Request {
  int set = 0;
  uint64_t n = 0, rows = 0, words = 0, out_off = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = kQueued;
  int slot = -1;
  int waiters = 0;  // threads in zset_server_wait on this query
  zset_status status = ZSET_OK;
  std::string msg;
};

struct Slot {
  hipStream_t s = nullptr;
  DevBuf tiles, misc;  // misc: [0] status word, [1] checksum, [2] chunk counter,
                       // [3] write workgroups done
  // Pinned host words written by the device when a query ends: [0] the
  // query's sequence number, [1] its status word.
  uint64_t* flag = nullptr;      // host address
  uint64_t* flag_dev = nullptr;  // device address of the same words
  uint64_t seq = 0;
  double t_launch = 0;
  uint64_t ticket = 0;
  bool busy = false;
};

// End of one served query on its slot's stream: the status word, then the
// sequence number (released at system scope) to pinned host memory, which the
// dispatcher reads with plain loads.
__global__ void k_query_done(const int* __restrict__ err, uint64_t* flag, uint64_t seq) {
  if (threadIdx.x == 0) {
    reinterpret_cast<volatile int*>(flag + 1)[0] = *err;
    __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace
}  // namespace zset

struct zset_server_s {
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::vector<zset::ResidentSet*> sets;
  std::vector<zset::Slot> slots;
  uint32_t* arena = nullptr;
  uint64_t arena_words = 0;
  std::map<uint64_t, uint64_t> free_list;  // word offset -> words, coalesced
  uint64_t slice_cap = 0;                  // slices one slot's table holds
  uint64_t memo_bytes = 0;                 // memo budget of each resident set
  std::mutex mu;
  std::condition_variable cv;       // dispatchers: submissions, arena room, stop
  std::condition_variable cv_done;  // zset_server_wait: a waited-for query ended
  std::deque<uint64_t> queue;
  std::map<uint64_t, zset::Request> reqs;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t admitted = 0, completed = 0, max_inflight = 0;
  double launch_us = 0;  // dispatcher host time spent enqueueing queries
};

namespace zset {
namespace {

uint64_t words_of(uint64_t rows, int d) { return (rows * uint64_t(d) + 3) / 4 * 4; }

// First fit in the arena (16-byte granules); false when no hole is large enough.
bool arena_alloc(zset_server_s* S, uint64_t words, uint64_t* off) {
  for (auto it = S->free_list.begin(); it != S->free_list.end(); ++it) {
    if (it->second >= words) {
      *off = it->first;
      const uint64_t rest = it->second - words, at = it->first + words;
      S->free_list.erase(it);
      if (rest) S->free_list[at] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(zset_server_s* S, uint64_t off, uint64_t words) {
  if (words == 0) return;
  auto it = S->free_list.emplace(off, words).first;
  auto next = std::next(it);
  if (next != S->free_list.end() && it->first + it->second == next->first) {
    it->second += next->second;
    S->free_list.erase(next);
  }
  if (it != S->free_list.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      S->free_list.erase(it);
    }
  }
}

// Enqueues one admitted query on its slot's stream.  Called by a dispatcher
// without the server lock (the resident set is immutable once added; the
// slot belongs to this dispatcher); every call is asynchronous.
// share: queries on the device or waiting when this one is admitted (at most
// the slot count); the write pass gets that share of the device.
zset_status launch_query(zset_server_s* S, const ResidentSet& R, uint64_t n, uint64_t rows,
                         uint64_t out_off, Slot& sl, int share) {
  int* err = reinterpret_cast<int*>(sl.misc.p);
  uint64_t* misc = reinterpret_cast<uint64_t*>(sl.misc.p);
  uint32_t* out = S->arena + out_off;
  if (R.d == 1) {
    ZSET_HIP(hipMemsetAsync(sl.misc.p, 0, 3 * sizeof(uint64_t), sl.s));
    ZSET_HIP(launch_single(n, R.g[0], out, false, misc + 1, sl.s));
  } else {
    EnumParams P = R.tmpl;
    P.n = uint32_t(n);
    P.total = rows;
    P.out = out;
    P.err = err;
    P.checksum = misc + 1;
    P.pool = reinterpret_cast<uint32_t*>(misc + 2);
    P.reset_status = 1;  // the slice planner clears err and checksum
    P.lds_cnt = 0;
    const size_t lds_max = size_t(write_lds_budget(S->device));
    if (R.k >= 1 && R.sum_u < (uint64_t(1) << 32) && R.memo_rows < (uint64_t(1) << 32)) {
      P.lds_cnt = 1;
      if (write_lds_bytes(P) > lds_max) P.lds_cnt = 0;
    }
    // Every slice dealt: when that leaves each wavefront at most
    // kFusedSlicesPerWave slices, the write pass computes the slice starts
    // itself (one launch, no slice table); otherwise the slice planner runs
    // first and the write pass claims slices at run time.
    EnumParams D = P;
    zset_status st = size_write_pass(D, 0, 0, S->device, false, true, share);
    if (st != ZSET_OK) return st;
    const bool fused = D.ntiles <= uint64_t(D.write_blocks) *
                                       uint64_t(write_waves_per_block()) * kFusedSlicesPerWave;
    if (fused) {
      P = D;
      P.tiles = nullptr;
    } else {
      st = size_write_pass(P, 0, -1, S->device, false, true, share);
      if (st != ZSET_OK) return st;
      if (P.ntiles > S->slice_cap) return fail(ZSET_EDEVICE, "internal: slice table too small");
      P.tiles = reinterpret_cast<uint32_t*>(sl.tiles.p);
    }
    // The write pass's last workgroup posts the completion.
    P.blocks_done = reinterpret_cast<uint32_t*>(misc + 3);
    P.done_flag = sl.flag_dev;
    P.done_seq = sl.seq + 1;
    if (!fused) ZSET_HIP(launch_plan(P, sl.s));
    ZSET_HIP(launch_write(P, false, true, sl.s));
    ++sl.seq;
    return ZSET_OK;
  }
  ++sl.seq;
  hipLaunchKernelGGL(k_query_done, dim3(1), dim3(64), 0, sl.s, err, sl.flag_dev, sl.seq);
  ZSET_HIP(hipGetLastError());
  return ZSET_OK;
}

// Dispatcher `id` of `nth` serves the slots id, id + nth, ...: it notes their
// completions and admits queued queries into them.
void dispatcher(zset_server_s* S, int id, int nth) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lock(S->mu);
  const int nslots = int(S->slots.size());
  for (;;) {
    bool busy = false;
    // Completions: the slot's flag words in pinned host memory.  A slot
    // whose flag has not come after 2 s asks the runtime whether its stream
    // failed (a query that ends normally always sets the flag).
    for (int si = id; si < nslots; si += nth) {
      Slot& sl = S->slots[si];
      if (!sl.busy) continue;
      const uint64_t got = __atomic_load_n(sl.flag, __ATOMIC_ACQUIRE);
      hipError_t q = hipSuccess;
      if (got != sl.seq) {
        if (now_us(S->t0) - sl.t_launch < 2e6) {
          busy = true;
          continue;
        }
        q = hipStreamQuery(sl.s);
        if (q == hipErrorNotReady) {
          busy = true;
          continue;
        }
        // The stream is done: the flag was written before it drained unless
        // the query failed, so it is read again now that the stream is idle
        // (it may have landed between the first read and the query).
        if (q == hipSuccess && __atomic_load_n(sl.flag, __ATOMIC_ACQUIRE) != sl.seq)
          q = hipErrorUnknown;  // stream done, flag never written
      }
      Request& r = S->reqs[sl.ticket];
      r.t_done = now_us(S->t0);
      const int code = reinterpret_cast<volatile int*>(sl.flag + 1)[0];
      if (q != hipSuccess) {
        (void)hipGetLastError();
        r.state = kFailed;
        r.status = ZSET_EDEVICE;
        r.msg = std::string("query on the device: ") + hipGetErrorString(q);
      } else if (code != 0) {
        r.state = kFailed;
        r.status = ZSET_EDEVICE;
        r.msg = device_error_text(code);
      } else {
        r.state = kDone;
      }
      sl.busy = false;
      ++S->completed;
      if (r.waiters) S->cv_done.notify_all();
    }
    // Admissions, in arrival order: the head waits for a slot and for room in
    // the arena.
    while (!S->queue.empty()) {
      Slot* free_slot = nullptr;
      for (int si = id; si < nslots; si += nth)
        if (!S->slots[si].busy) {
          free_slot = &S->slots[si];
          break;
        }
      if (!free_slot) break;
      const uint64_t t = S->queue.front();
      Request& r = S->reqs[t];
      if (r.rows == 0) {  // nothing to write: done without the device
        S->queue.pop_front();
        r.t_admit = r.t_done = now_us(S->t0);
        r.state = kDone;
        ++S->admitted;
        ++S->completed;
        if (r.waiters) S->cv_done.notify_all();
        continue;
      }
      if (r.words > 0 && !arena_alloc(S, r.words, &r.out_off)) break;
      S->queue.pop_front();
      r.t_admit = now_us(S->t0);
      r.state = kRunning;
      free_slot->busy = true;  // this dispatcher's slot: no other thread touches it
      const ResidentSet* R = S->sets[r.set];
      const uint64_t qn = r.n, qrows = r.rows, qoff = r.out_off;
      uint64_t share = S->queue.size() + 1;
      for (const Slot& o : S->slots) share += o.busy && &o != free_slot ? 1 : 0;
      share = std::min<uint64_t>(share, uint64_t(nslots));
      lock.unlock();
      zset_status st = launch_query(S, *R, qn, qrows, qoff, *free_slot, int(share));
      std::string msg = st != ZSET_OK ? g_last_error : std::string();
      lock.lock();
      S->launch_us += now_us(S->t0) - r.t_admit;
      if (st != ZSET_OK) {
        free_slot->busy = false;
        r.state = kFailed;
        r.status = st;
        r.msg = msg;
        r.t_done = now_us(S->t0);
        if (r.waiters) S->cv_done.notify_all();
        continue;
      }
      free_slot->t_launch = r.t_admit;
      r.slot = int(free_slot - S->slots.data());
      free_slot->ticket = t;
      busy = true;
      ++S->admitted;
    }
    if (S->stop) {  // queries never admitted end here, with an error
      for (const uint64_t t : S->queue) {
        Request& r = S->reqs[t];
        r.state = kFailed;
        r.status = ZSET_EINVAL;
        r.msg = "the server stopped before the query was admitted";
      }
      S->queue.clear();
      S->cv.notify_all();
      S->cv_done.notify_all();
    }
    uint64_t inflight = 0;
    for (const Slot& sl : S->slots) inflight += sl.busy ? 1 : 0;
    S->max_inflight = std::max(S->max_inflight, inflight);
    if (S->stop && !busy && S->queue.empty()) break;
    if (!busy) {
      // Nothing on the device: sleep until a submission, a release (room in
      // the arena) or the end.
      S->cv.wait(lock);
    } else {
      // Queries on the device: poll again at once (a timed sleep lasts tens
      // of microseconds, longer than many queries).
      lock.unlock();
      std::this_thread::yield();
      lock.lock();
    }
  }
}

}  // namespace
}  // namespace zset

using namespace zset;

void zset_server_default_opts(zset_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->slots = kDefaultSlots;
}

zset_status zset_server_create(const zset_server_opts* opts, zset_server* out) {
  g_last_error.clear();
  if (!opts || !out) return fail(ZSET_EINVAL, "opts or server is NULL");
  *out = nullptr;
  const int slots = opts->slots ? opts->slots : kDefaultSlots;
  if (slots < 1 || slots > kMaxSlots) return fail(ZSET_EINVAL, "slots must lie in [1, 64]");
  if (!opts->arena || opts->arena_bytes < 16)
    return fail(ZSET_EINVAL, "the output arena is missing or smaller than 16 bytes");
  if ((reinterpret_cast<uintptr_t>(opts->arena) & 15) != 0)
    return fail(ZSET_EINVAL, "the output arena must be 16-byte aligned");
  if (!is_device_pointer(opts->arena)) return fail(ZSET_EINVAL, "the arena is not device memory");
  zset_server_s* S = new zset_server_s();
  S->t0 = std::chrono::steady_clock::now();
  auto bail = [&](zset_status st) {
    zset_server_free(S);
    return st;
  };
  int cus = 0;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) !=
          hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(ZSET_EDEVICE, "device query failed"));
  }
  S->memo_bytes = opts->memo_bytes ? opts->memo_bytes : kResidentMemoBytes;
  S->arena = reinterpret_cast<uint32_t*>(opts->arena);
  S->arena_words = opts->arena_bytes / 16 * 4;
  S->free_list[0] = S->arena_words;
  // At most 2 write workgroups per compute unit fit beside the smallest memo.
  S->slice_cap = uint64_t(cus) * 2 * write_waves_per_block() * kSlicesPerWave + 1;
  S->slots.resize(slots);
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(ZSET_EDEVICE, "stream creation failed"));
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.flag), 16, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.flag_dev), sl.flag, 0) !=
            hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(ZSET_ENOMEM, "pinned completion words"));
    }
    sl.flag[0] = 0;
    sl.flag[1] = 0;
    zset_status st = ensure(sl.misc, 4 * sizeof(uint64_t));
    // Status word and workgroup counter start clear; the write pass's last
    // workgroup leaves them clear after every query.
    if (st == ZSET_OK && hipMemset(sl.misc.p, 0, 4 * sizeof(uint64_t)) != hipSuccess) {
      (void)hipGetLastError();
      st = fail(ZSET_EDEVICE, "clearing the slot's status words");
    }
    if (st == ZSET_OK)
      st = ensure(sl.tiles, size_t(S->slice_cap) * (kMaxD + 2) * sizeof(uint32_t));
    if (st != ZSET_OK) return bail(st);
  }
  const int nth = std::max(1, std::min(opts->dispatchers ? opts->dispatchers : 1, slots));
  for (int i = 0; i < nth; ++i) S->workers.emplace_back(dispatcher, S, i, nth);
  *out = S;
  return ZSET_OK;
}

zset_status zset_server_add_set(zset_server S, const uint32_t* gens, int d, uint64_t n_max, int k,
                                int* set_id) {
  g_last_error.clear();
  if (!S || !set_id) return fail(ZSET_EINVAL, "server or set_id is NULL");
  zset_status st = check_query(n_max, gens, d);
  if (st != ZSET_OK) return st;
  if (k < -1 || k > d - 1) return fail(ZSET_EINVAL, "k must be -1 or lie in [0, d-1]");
  ResidentSet* R = new ResidentSet();
  auto bail = [&](zset_status e) {
    for (DevBuf* b : {&R->table, &R->endc, &R->leaf})
      if (b->p) (void)hipFree(b->p);
    delete R;
    return e;
  };
  R->d = d;
  R->n_max = n_max;
  for (int i = 0; i < d; ++i) R->g[i] = gens[i];
  const uint64_t N = n_max + 1;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(ZSET_EDEVICE, "hipStreamCreate failed"));
  }
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{s};
  DevBuf scratch;  // row sums, status word
  struct ScratchGuard {
    DevBuf& b;
    ~ScratchGuard() {
      if (b.p) (void)hipFree(b.p);
    }
  } sguard{scratch};
  if ((st = ensure(R->table, size_t(d + 1) * N * sizeof(uint64_t))) != ZSET_OK) return bail(st);
  if ((st = ensure(scratch, (2 * kMaxD + 4) * sizeof(uint64_t))) != ZSET_OK) return bail(st);
  uint64_t* T = reinterpret_cast<uint64_t*>(R->table.p);
  uint64_t* sums_dev = reinterpret_cast<uint64_t*>(scratch.p);
  int* err = reinterpret_cast<int*>(sums_dev + 2 * kMaxD + 3);  // after sums, |Z|, maxima
  if (hipMemsetAsync(scratch.p, 0, (2 * kMaxD + 4) * sizeof(uint64_t), s) != hipSuccess ||
      launch_count_table(T, n_max, gens, d, sums_dev, s) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(ZSET_EDEVICE, "count table launch failed"));
  }
  uint64_t sums[kMaxD + 1];
  R->c0.resize(N);
  if (hipMemcpyAsync(sums, sums_dev, (d + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(R->c0.data(), T, N * sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(ZSET_EDEVICE, "count table readback failed"));
  }
  const size_t lds_max = size_t(write_lds_budget(S->device));

  // Memo dimension: the requested one, else the largest k whose memo over
  // p <= n_max takes at most the server's memo budget.  The memo is built once per
  // set, so only the write pass counts: a larger k leaves fewer outer
  // coordinates and longer segments per outer prefix, and that gain outweighs
  // reading the memo from global memory instead of LDS up to memos of tens of
  // megabytes.
  auto tmpl_for = [&](int kk, EnumParams& P) {
    std::memset(&P, 0, sizeof P);
    const int L = d - std::max(kk, 1);
    const int U = (kk == 0) ? d - 1 : L - 1;
    for (int i = 0; i < d; ++i) P.g.g[i] = gens[i];
    P.n = uint32_t(n_max);
    P.d = d;
    P.U = U;
    P.k = kk;
    P.table = T;
    P.table_stride = N;
    P.dG = DivMod32::make(gens[U]);
    P.ring = d <= 16 ? 128 : 64;
    P.flush = P.ring / 2;
    P.max_tiles = 16;
    P.chunk = uint32_t(write_waves_per_block());
    if (kk >= 1) {
      leaf_format(P, n_max, gens, U, kk);
      const uint64_t Rn = sums[L];
      if (Rn >= (uint64_t(1) << 32)) P.pack = 0;
      P.memo_words = P.pack ? Rn * uint64_t(P.pack) : 0;
      P.nclass = uint32_t(std::min<uint64_t>(gens[U], N));
      P.leaf_rows = Rn;
    }
  };
  int kk = k;
  if (d == 1) {
    kk = 0;
  } else if (kk < 0) {
    kk = 1;
    for (int c = d - 1; c >= 2; --c) {
      const uint64_t Rc = sums[d - c];
      if (Rc == ~uint64_t(0) || Rc >= (uint64_t(1) << 32)) continue;
      EnumParams P;
      tmpl_for(c, P);
      // The memo as the write pass will hold it: packed when the packed memo
      // fits the write pass's LDS, else k + 1 plain words per row.
      const bool packed =
          P.pack != 0 && write_lds_bytes(P) <= lds_max;
      const uint64_t words = packed ? Rc * uint64_t(P.pack) : Rc * uint64_t(c + 1);
      if (words * 4 <= S->memo_bytes) {
        kk = c;
        break;
      }
    }
  }
  R->k = kk;
  R->L = d - std::max(kk, 1);
  R->U = (kk == 0) ? d - 1 : R->L - 1;
  tmpl_for(kk, R->tmpl);
  R->sum_u = sums[R->U];
  R->memo_top = N;
  if (kk >= 1 && d >= 2) {
    EnumParams& P = R->tmpl;
    uint64_t Rn = sums[R->L];
    const int pack0 = P.pack;
    if (P.pack != 0 && write_lds_bytes(P) > lds_max) {
      P.pack = 0;
      P.memo_words = 0;
    }
    const uint64_t wpr = P.pack ? uint64_t(P.pack) : uint64_t(kk + 1);  // words per memo row
    uint64_t top = N;
    if (Rn == ~uint64_t(0) || Rn > S->memo_bytes / (4 * wpr)) {
      // A partial memo: the largest top whose rows (|Z(p; h)| summed over
      // p < top, row L of the count table) fit the budget, packed when the
      // capped memo fits the write pass's LDS.  The memo of p = 0 (one row)
      // is always kept.
      std::vector<uint64_t> cl(N);
      if (hipMemcpyAsync(cl.data(), T + uint64_t(R->L) * N, N * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(ZSET_EDEVICE, "count table readback failed"));
      }
      auto cap_top = [&](uint64_t words_per_row, uint64_t* rows) {
        const uint64_t max_rows = std::max<uint64_t>(S->memo_bytes / (4 * words_per_row), 1);
        uint64_t acc = 0, t = 0;
        while (t < N && cl[t] <= max_rows - acc) acc += cl[t++];
        if (t == 0) acc = cl[t++];  // |Z(0; h)| = 1
        *rows = acc;
        return t;
      };
      P.pack = pack0;
      if (P.pack != 0) {
        top = cap_top(uint64_t(P.pack), &Rn);
        P.memo_words = Rn * uint64_t(P.pack);
        if (write_lds_bytes(P) > lds_max) P.pack = 0;
      }
      if (P.pack == 0) {
        top = cap_top(uint64_t(kk + 1), &Rn);
        P.memo_words = 0;
      }
      P.memo_top = uint32_t(top);
      P.nclass = uint32_t(std::min<uint64_t>(gens[R->U], top));
      P.leaf_rows = Rn;
    }
    R->memo_rows = Rn;
    R->memo_top = top;
    zset_memo m = nullptr;
    if ((st = zset_memo_build(gens + R->L, kk, top, s, &m)) != ZSET_OK) return bail(st);
    struct MemoGuard {
      zset_memo m;
      ~MemoGuard() { zset_memo_free(m); }
    } mguard{m};
    if (m->rows != Rn) return bail(fail(ZSET_EDEVICE, "internal: resident memo size"));
    const uint32_t G = gens[R->U];
    const uint64_t leaf_words = P.pack ? Rn * uint64_t(P.pack) : Rn * uint64_t(kk + 1);
    if ((st = ensure(R->endc, size_t(P.nclass) * sizeof(uint64_t))) != ZSET_OK) return bail(st);
    if ((st = ensure(R->leaf, size_t(leaf_words) * sizeof(uint32_t))) != ZSET_OK) return bail(st);
    uint64_t* endc = reinterpret_cast<uint64_t*>(R->endc.p);
    uint32_t* leaf = reinterpret_cast<uint32_t*>(R->leaf.p);
    uint32_t nclass = 0;
    const uint64_t* cu = T + uint64_t(R->U) * N;
    if (launch_class_ends(cu, top - 1, G, endc, &nclass, s) != hipSuccess ||
        launch_memo_leaf(make_leaf_job(kk, top - 1, G, m->off, m->nat, cu, endc, leaf, Rn, P),
                         err, s) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(ZSET_EDEVICE, "leaf layout launch failed"));
    }
    int code = 0;
    if (hipMemcpyAsync(&code, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(ZSET_EDEVICE, "leaf layout failed"));
    }
    if (code != 0) return bail(fail(ZSET_EDEVICE, device_error_text(code)));
    P.endc = endc;
    P.leaf = leaf;
    P.nclass = nclass;
  }
  std::lock_guard<std::mutex> lock(S->mu);
  S->sets.push_back(R);
  *set_id = int(S->sets.size() - 1);
  return ZSET_OK;
}

zset_status zset_server_set_info(zset_server S, int set_id, int* k, uint64_t* n_max,
                                 uint64_t* memo_rows, uint64_t* resident_bytes,
                                 uint64_t* memo_top) {
  g_last_error.clear();
  if (!S) return fail(ZSET_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  if (set_id < 0 || set_id >= int(S->sets.size())) return fail(ZSET_EINVAL, "no such set");
  const ResidentSet& R = *S->sets[set_id];
  if (k) *k = R.k;
  if (n_max) *n_max = R.n_max;
  if (memo_rows) *memo_rows = R.memo_rows;
  if (resident_bytes) *resident_bytes = R.table.bytes + R.endc.bytes + R.leaf.bytes;
  if (memo_top) *memo_top = R.memo_top;
  return ZSET_OK;
}

zset_status zset_server_count(zset_server S, int set_id, uint64_t n, uint64_t* rows) {
  g_last_error.clear();
  if (!S || !rows) return fail(ZSET_EINVAL, "server or rows is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  if (set_id < 0 || set_id >= int(S->sets.size())) return fail(ZSET_EINVAL, "no such set");
  const ResidentSet& R = *S->sets[set_id];
  if (n > R.n_max) return fail(ZSET_EINVAL, "n exceeds the set's n_max");
  *rows = R.c0[n];
  if (*rows == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
  return ZSET_OK;
}

zset_status zset_server_submit(zset_server S, int set_id, uint64_t n, uint64_t* ticket) {
  g_last_error.clear();
  if (!S || !ticket) return fail(ZSET_EINVAL, "server or ticket is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  if (S->stop) return fail(ZSET_EINVAL, "the server is stopping");
  if (set_id < 0 || set_id >= int(S->sets.size())) return fail(ZSET_EINVAL, "no such set");
  const ResidentSet& R = *S->sets[set_id];
  if (n > R.n_max) return fail(ZSET_EINVAL, "n exceeds the set's n_max");
  const uint64_t rows = R.c0[n];
  if (rows == ~uint64_t(0) || rows > (~uint64_t(0)) / (4 * uint64_t(R.d)))
    return fail(ZSET_EOVERFLOW, "|Z(n)| * d * 4 bytes overflows 64 bits");
  const uint64_t words = words_of(rows, R.d);
  if (words > S->arena_words)
    return fail(ZSET_ECAPACITY, "the query's rows exceed the whole output arena");
  const uint64_t t = S->next_ticket++;
  Request& r = S->reqs[t];
  r.set = set_id;
  r.n = n;
  r.rows = rows;
  r.words = words;
  r.t_submit = now_us(S->t0);
  S->queue.push_back(t);
  *ticket = t;
  S->cv.notify_all();
  return ZSET_OK;
}

zset_status zset_server_wait(zset_server S, uint64_t ticket, zset_server_result* res) {
  g_last_error.clear();
  if (!S) return fail(ZSET_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(ZSET_EINVAL, "unknown ticket");
  ++it->second.waiters;
  S->cv_done.wait(lock, [&] { return it->second.state >= kDone; });
  --it->second.waiters;
  const Request& r = it->second;
  if (res) {
    res->rows = r.rows;
    res->out_offset = r.out_off;
    res->submit_us = r.t_submit;
    res->admit_us = r.t_admit;
    res->done_us = r.t_done;
  }
  if (r.state == kFailed) return fail(r.status, r.msg);
  return ZSET_OK;
}

zset_status zset_server_release(zset_server S, uint64_t ticket) {
  g_last_error.clear();
  if (!S) return fail(ZSET_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(ZSET_EINVAL, "unknown ticket");
  if (it->second.state < kDone) return fail(ZSET_EINVAL, "the query has not finished");
  if (it->second.waiters > 0) return fail(ZSET_EINVAL, "another thread is waiting on the query");
  if (it->second.t_admit > 0 && it->second.words > 0)
    arena_free(S, it->second.out_off, it->second.words);
  S->reqs.erase(it);
  S->cv.notify_all();
  return ZSET_OK;
}

zset_status zset_server_stats(zset_server S, uint64_t* admitted, uint64_t* completed,
                              uint64_t* max_inflight, double* launch_us) {
  g_last_error.clear();
  if (!S) return fail(ZSET_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  if (admitted) *admitted = S->admitted;
  if (completed) *completed = S->completed;
  if (max_inflight) *max_inflight = S->max_inflight;
  if (launch_us) *launch_us = S->launch_us;
  return ZSET_OK;
}

void zset_server_free(zset_server S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->stop = true;
    S->cv.notify_all();
    S->cv_done.notify_all();
  }
  for (std::thread& w : S->workers)
    if (w.joinable()) w.join();
  for (Slot& sl : S->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    if (sl.flag) (void)hipHostFree(sl.flag);
    for (DevBuf* b : {&sl.tiles, &sl.misc})
      if (b->p) (void)hipFree(b->p);
  }
  for (ResidentSet* R : S->sets) {
    for (DevBuf* b : {&R->table, &R->endc, &R->leaf})
      if (b->p) (void)hipFree(b->p);
    delete R;
  }
  delete S;
}
