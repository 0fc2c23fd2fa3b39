// api.hip -- the C ABI of libzset.so (include/zset.h): argument checks,
// per-device scratch memory, the order of launches, status codes and timings.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>

#include "zset.h"
#include "zset_host.h"
#include "zset_internal.h"

namespace zset {

thread_local std::string g_last_error;
std::mutex g_mu;

zset_status fail(zset_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

zset_status hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(ZSET_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool fault_injected(const char* what) {
  const char* f = std::getenv("ZSET_FAULT");
  return f && std::strcmp(f, what) == 0;
}

zset_status ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return ZSET_OK;
  if (fault_injected("alloc")) return fail(ZSET_ENOMEM, "allocation refused (ZSET_FAULT=alloc)");
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(ZSET_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    want = bytes;
  }
  b.bytes = want;
  return ZSET_OK;
}

namespace {

// Per-device scratch, reused across calls.
struct Ctx {
  int device = -1;
  DevBuf table, off, nat, srcw, endc, leaf, tiles, misc, hcount, cnt2, rowp;
  uint64_t* pinned = nullptr;  // host readback area
  hipEvent_t ev[7] = {};
  // Side stream for a memo recurrence that runs beside the count table, with
  // its fork event and start / end events.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, memo0 = nullptr, memo1 = nullptr;
  // Stream of the class ends and slice plan when they run before the host's
  // readback (k fixed by the caller), with the count table's end and their
  // own end.
  hipStream_t plan = nullptr;
  hipEvent_t counted = nullptr, planned = nullptr;
  int wall_khz = 0;  // the device's constant-rate clock (kernel time stamps)
  // Asynchronous calls: the sequence number of the last one enqueued, its
  // stream, and whether it may still be running.  Its last launch stores the
  // sequence number to pinned[kDoneWord] (through done_dev, the device's
  // address of that word), after its result words.
  uint64_t seq = 0;
  hipStream_t busy_stream = nullptr;
  bool inflight = false;
  uint64_t* done_dev = nullptr;
};

std::map<int, Ctx*> g_ctx;

// Pair lanes in the write pass when n / g_{U-1} is below this (init_params).
constexpr uint64_t kPairBelow = 200;
// Slice start states each write workgroup keeps in LDS, at least.
constexpr uint32_t kMinTileStates = 16;
// Slices per wavefront above which a query sharing the device gets more
// workgroups than its share.
constexpr uint64_t kSharedSlicesPerWave = 8;

// misc layout (uint64 words): [0] status word (int), [1] checksum, [2..] the
// count table's row sums, |Z(n)| and row maxima (2 kMaxD + 3 words), then the
// write pass's chunk counter and two kernel time stamps.
constexpr int kMiscErr = 0, kMiscSum = 1, kMiscRowSums = 2,
              kMiscPool = kMiscRowSums + 2 * kMaxD + 3, kMiscStamp = kMiscPool + 1;
constexpr size_t kMiscWords = kMiscStamp + 2;
constexpr int kDefaultClaimPct = 100;  // percent of slices claimed at run time
constexpr size_t kPinnedWords = 128;
constexpr size_t kDoneWord = kPinnedWords - 1;  // pinned word of the asynchronous calls
static_assert(kMiscWords < kDoneWord && 2 * kMaxD + 3 < kDoneWord, "pinned readback layout");

zset_status get_ctx(Ctx** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) {
    *out = it->second;
    return ZSET_OK;
  }
  Ctx* c = new Ctx();
  c->device = dev;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->pinned), kPinnedWords * sizeof(uint64_t),
                    hipHostMallocDefault) != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail(ZSET_ENOMEM, "hipHostMalloc of the readback area failed");
  }
  for (auto& ev : c->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ZSET_EDEVICE, "hipEventCreate failed");
    }
  }
  if (hipEventCreate(&c->fork) != hipSuccess ||
      hipEventCreate(&c->memo0) != hipSuccess || hipEventCreate(&c->memo1) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->counted, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->planned, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->plan, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ZSET_EDEVICE, "side stream or event creation failed");
  }
  c->pinned[kDoneWord] = 0;
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&c->done_dev), c->pinned + kDoneWord, 0) !=
      hipSuccess) {
    (void)hipGetLastError();
    return fail(ZSET_EDEVICE, "hipHostGetDevicePointer of the readback area failed");
  }
  if (hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
    (void)hipGetLastError();
    c->wall_khz = 0;
  }
  zset_status st = ensure(c->misc, kMiscWords * sizeof(uint64_t));
  if (st != ZSET_OK) return st;
  g_ctx[dev] = c;
  *out = c;
  return ZSET_OK;
}

// Waits for the last asynchronous call's launches, which read and write the
// context's buffers, before anything else may reuse or free them.
// No event is recorded per call (each event marker between kernels leaves
// the device idle for microseconds): the host watches the pinned word that
// the call's last launch stores, and after 30 s falls back to a device-wide
// wait.
zset_status settle(Ctx* c) {
  if (!c->inflight) return ZSET_OK;
  const volatile uint64_t* done = c->pinned + kDoneWord;
  const auto t0 = std::chrono::steady_clock::now();
  while (*done < c->seq) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(30)) {
      const hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      if (*done < c->seq) return fail(ZSET_EDEVICE, "an asynchronous call did not finish");
      break;
    }
    std::this_thread::yield();
  }
  c->inflight = false;
  return ZSET_OK;
}

// ensure() for a context buffer that an asynchronous call may still be using:
// a buffer that must grow is freed only after that call is done.
zset_status grow(Ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes < std::max<size_t>(bytes, 16)) {
    const zset_status st = settle(c);
    if (st != ZSET_OK) return st;
  }
  return ensure(b, bytes);
}

}  // namespace

// Slice length, claimed chunks, slice-state capacity and grid of the write
// pass for P (P.total, P.U, P.d, P.k and the memo fields set; P.pool set by the
// caller).  Slices 0..static_tiles-1 are dealt round-robin; the last claim_pct
// percent (all, by default) are claimed at run time in chunks of one slice per
// wavefront by the workgroups that have capacity: compute units do not all
// drain HBM at one rate, so a fixed share per workgroup ends with the slowest.
// About 128 slices per resident wavefront by default (short slices keep the
// concurrent write streams of a compute unit close together in memory and the
// end of the pass even).
zset_status size_write_pass(EnumParams& P, uint64_t rows_per_tile, int claim_pct, int device,
                            bool count_only, bool align16, int share, uint64_t want_tiles) {
  const int pct = claim_pct < 0 ? kDefaultClaimPct : claim_pct;
  const size_t lds_max = size_t(write_lds_budget(device));
  P.max_tiles = kMinTileStates;
  P.chunk = pct > 0 ? uint32_t(write_waves_per_block()) : 0;
  if (P.chunk && write_lds_bytes(P) > lds_max) P.chunk = 0;
  static std::atomic<int> cus_of[64];  // compute units per device, asked for once
  int cus = (device >= 0 && device < 64) ? cus_of[device].load() : 0, per_cu = 0;
  if (cus == 0) {
    ZSET_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    if (device >= 0 && device < 64) cus_of[device].store(cus);
  }
  ZSET_HIP(write_occupancy(P, count_only, align16, &per_cu));
  if (per_cu < 1) return fail(ZSET_EDEVICE, "the write pass does not fit on a compute unit");
  const uint64_t wpb = uint64_t(write_waves_per_block());
  const uint64_t resident_waves = uint64_t(cus) * per_cu * wpb;
  uint64_t T_rows = rows_per_tile;
  if (T_rows == 0) T_rows = slice_rows(P.total, want_tiles ? want_tiles : resident_waves * 128);
  const uint64_t ntiles = (P.total + T_rows - 1) / T_rows;
  if (ntiles > 0x7fffffffull) return fail(ZSET_EINVAL, "too many slices: raise rows_per_tile");
  // A query that shares the device with share - 1 others gets that share of
  // the resident workgroups, or more when its wavefronts would otherwise take
  // over kSharedSlicesPerWave slices each: small queries pay fewer workgroup
  // prologues per row, large ones keep the whole device (a share fixed at
  // admission would leave them slow once the others end).  The slice length
  // above stays that of the whole device.
  const uint64_t resident_all = uint64_t(cus) * per_cu;
  uint64_t resident = resident_all;
  if (share > 1) {
    const uint64_t by_share = (resident_all + uint64_t(share) - 1) / uint64_t(share);
    const uint64_t by_work = (ntiles + wpb * kSharedSlicesPerWave - 1) / (wpb * kSharedSlicesPerWave);
    resident = std::min(resident_all, std::max<uint64_t>({by_share, by_work, 1}));
  }
  P.static_tiles = P.chunk ? ntiles - (ntiles * uint64_t(pct) + 99) / 100 : ntiles;
  // Give each resident workgroup room for the start states of all of its
  // dealt slices when the LDS left over at this occupancy allows, so that the
  // grid stays one resident round.
  const uint64_t need = (P.static_tiles + resident - 1) / resident;
  const size_t budget = lds_max / size_t(per_cu);
  const size_t base = write_lds_bytes(P);  // with kMinTileStates states
  const uint64_t per_state = uint64_t(P.U + 2) * sizeof(uint32_t);
  uint64_t fit = P.max_tiles;
  if (budget > base + 16) fit += (budget - base - 16) / per_state;
  P.max_tiles = uint32_t(std::min<uint64_t>(std::max<uint64_t>(need, kMinTileStates),
                                            std::min<uint64_t>(fit, 1u << 20)));
  uint64_t blocks = resident;
  const uint64_t min_blocks = (P.static_tiles + P.max_tiles - 1) / P.max_tiles;
  const uint64_t max_blocks = (ntiles + wpb - 1) / wpb;
  blocks = std::max(blocks, min_blocks);
  blocks = std::min(blocks, max_blocks);
  if (blocks > 0x7fffffffull) return fail(ZSET_EINVAL, "too many slices: raise rows_per_tile");
  P.write_blocks = uint32_t(std::max<uint64_t>(blocks, 1));
  P.rows_per_tile = T_rows;
  P.ntiles = ntiles;
  return ZSET_OK;
}

uint64_t plan_want_tiles(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    cus = 1;
  }
  return uint64_t(cus) * uint64_t(write_waves_per_block()) * 128;
}

// Leaf-order row format for elements p <= n: fields floor(p / G) <= n / G and
// m_c <= n / h_c, packed into one 32- or 64-bit word when they fit.
void leaf_format(EnumParams& P, uint64_t n, const uint32_t* gens, int U, int k) {
  uint32_t shift = 0;
  for (int c2 = 0; c2 <= k; ++c2) {
    const uint32_t vmax = uint32_t(n / gens[U + c2]);
    uint32_t bits = 0;
    while (bits < 32 && (uint64_t(vmax) >> bits) != 0) ++bits;
    P.fshift[c2] = shift;
    P.fmask[c2] = bits >= 32 ? ~0u : ((1u << bits) - 1u);
    shift += bits;
  }
  P.pack = shift <= 32 ? 1 : (shift <= 64 ? 2 : 0);
}

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
         attr.type == hipMemoryTypeUnified;
}

zset_status check_gens(const uint32_t* gens, int d, const char* what) {
  if (!gens) return fail(ZSET_EINVAL, std::string(what) + " is NULL");
  if (d < 1 || d > kMaxD) return fail(ZSET_EINVAL, "d must lie in [1, 32]");
  for (int i = 0; i < d; ++i)
    if (gens[i] == 0) return fail(ZSET_EINVAL, "every generator must be >= 1");
  return ZSET_OK;
}

zset_status check_query(uint64_t n, const uint32_t* gens, int d) {
  zset_status st = check_gens(gens, d, "gens");
  if (st != ZSET_OK) return st;
  if (n > kMaxN) return fail(ZSET_EINVAL, "n exceeds 2^31 - 2");
  return ZSET_OK;
}


int write_lds_budget(int device) { return device_max_lds_bytes(device) - 256; }

int device_max_lds_bytes(int device) {
  static std::atomic<int> lds_of[64];  // asked for once per device
  if (device >= 0 && device < 64) {
    const int v = lds_of[device].load();
    if (v != 0) return v;
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  if (device >= 0 && device < 64) lds_of[device].store(v);
  return v;
}

uint32_t next_pow2(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

float elapsed_us(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms * 1000.f;
}

const char* device_error_text(int code) {
  switch (code) {
    case kErrOdometer: return "a slice ran out of prefixes before its rows were written";
    case kErrTileRows: return "a slice wrote a different number of rows than planned";
    case kErrMemoTotal: return "the memo build produced a different row total than counted";
    case kErrUnrank: return "a slice start could not be unranked";
    case kErrCapacity: return "|Z(n)| exceeds the output's rows";
    case kErrOverflow: return "|Z(n)| or its bytes overflow 64 bits";
    case kErrSlices: return "|Z(n)| needs more slices of at most 2^30 rows than were planned";
    default: return "unknown kernel check";
  }
}

namespace {

int max_lds_bytes(Ctx* c) { return device_max_lds_bytes(c->device); }

// Builds Memo[p] = Z(p; h) for p < top into nat (natural order) and the
// natural offsets off[0..top].  `ge` holds |Z(m; h_i..h_k)| for i = 0..k-1
// (row stride ge_stride) and `sizes` = ge row 0; R = the total row count and
// rowmax the longest list.  Memos that fit in LDS are built by one wavefront
// (k_memo_chain_wave), which also writes the offsets; larger ones by one
// wavefront with a ring of the last lists in LDS (k_memo_chain_window) when
// that ring fits, else by the global schedule after a scan.
// ZSET_MEMO_PATH=global / window forces those paths (tests); =chain (and
// either of those) keeps the recurrence for k = 2 memos, which the single path
// otherwise builds in closed form.
// `srcw_for(bytes, &ptr)` provides the global schedule's source table.
// R is the memo's row count when `exact`, else an upper bound (a partial
// memo sized from the row sums over every p <= n).
zset_status build_memo_rows(const uint32_t* h, int k, uint64_t top, uint64_t* off,
                            const uint64_t* ge, uint64_t ge_stride, uint64_t R, uint64_t rowmax,
                            uint32_t* nat, int* err, size_t lds,
                            const std::function<zset_status(size_t, uint64_t**)>& srcw_for,
                            hipStream_t s, bool exact = true) {
  if (k == 1) {
    const uint64_t R1 = (top - 1) / h[0] + 1;
    if (exact ? R != R1 : R < R1) return fail(ZSET_EDEVICE, "memo row count disagrees (k = 1)");
    ZSET_HIP(launch_memo_k1(h[0], top, R1, nat, off, s));
    return ZSET_OK;
  }
  const uint64_t Rexp = exact ? R : 0;
  uint32_t b = h[0], hmax = h[0];
  for (int i = 1; i < k; ++i) {
    b = std::min(b, h[i]);
    hmax = std::max(hmax, h[i]);
  }
  const char* path = std::getenv("ZSET_MEMO_PATH");
  const bool force_global = path && std::strcmp(path, "global") == 0;
  const bool force_window = path && std::strcmp(path, "window") == 0;
  const uint32_t step = std::min<uint32_t>(b, kWave);
  const uint64_t Wl = uint64_t(hmax) + step;
  const uint32_t W = Wl < (uint64_t(1) << 30) ? next_pow2(uint32_t(Wl)) : 0;
  if (!force_global && !force_window && W != 0 && R < (uint64_t(1) << 30) &&
      memo_wave_lds_bytes(k, R, W) <= lds) {
    ZSET_HIP(launch_memo_chain_wave(h, k, top, step, W, R, Rexp, nat, off, err, s));
    return ZSET_OK;
  }
  if (!force_global && W != 0 && R < (uint64_t(1) << 32) && rowmax < (uint64_t(1) << 24)) {
    const uint64_t need = (uint64_t(hmax) + step) * std::max<uint64_t>(rowmax, 1);
    if (need < (uint64_t(1) << 30)) {
      const uint32_t cap = next_pow2(uint32_t(need));
      if (memo_wave_lds_bytes(k, cap, W) <= lds) {
        ZSET_HIP(launch_memo_chain_window(h, k, top, step, W, hmax, cap, Rexp, nat, off, err, s));
        return ZSET_OK;
      }
    }
  }
  ZSET_HIP(launch_exclusive_scan(ge, top, off, s));
  uint64_t* srcw = nullptr;
  zset_status st = srcw_for(size_t(R) * sizeof(uint64_t), &srcw);
  if (st != ZSET_OK) return st;
  ZSET_HIP(launch_memo_global(h, k, top, b, off, ge, ge_stride, srcw, nat, err, s, R));
  return ZSET_OK;
}

// Two-coordinate memos in closed form, unless ZSET_MEMO_PATH asks for one of
// the recurrence's schedules.
bool memo2_closed_form() {
  const char* path = std::getenv("ZSET_MEMO_PATH");
  return !(path && (std::strcmp(path, "chain") == 0 || std::strcmp(path, "global") == 0 ||
                    std::strcmp(path, "window") == 0));
}

// The global schedule's source table from the context's grow-only buffer.
std::function<zset_status(size_t, uint64_t**)> ctx_srcw(Ctx* c) {
  return [c](size_t bytes, uint64_t** p) {
    zset_status st = ensure(c->srcw, bytes);
    *p = reinterpret_cast<uint64_t*>(c->srcw.p);
    return st;
  };
}

// Automatic memo dimension: the largest k whose memo stays small beside the
// output (at most 1/16 of the rows and 512 MiB); k = 1 always qualifies in
// practice.  sums[j] = rows of the count table's row j over x <= n.
int auto_memo_dim(const uint64_t* sums, int d, uint64_t total) {
  for (int kk = d - 1; kk >= 1; --kk) {
    const uint64_t R = sums[d - kk];
    if (R != ~uint64_t(0) && R <= std::max<uint64_t>(uint64_t(1) << 16, total / 16) &&
        R * (kk + 1) * 4 <= (uint64_t(512) << 20))
      return kk;
  }
  return 1;
}

// The write pass's descriptor for memo dimension k: generators, coordinates
// fixed by a slice start (U), the division by g_U and the staging ring; for
// k >= 1 also the leaf-order row format and what the write pass keeps in LDS
// (packed memo rows, segment counts and class ends), decided from the row
// sums alone.  Returns the leaf layout's uint32 words.
uint64_t init_params(EnumParams& P, uint64_t n, const uint32_t* gens, int d, int k,
                     uint64_t total, const uint64_t* sums, const uint64_t* T, int* err,
                     uint64_t* checksum, uint32_t* out, size_t lds_max) {
  const uint64_t N = n + 1;
  const int L = d - std::max(k, 1);
  const int U = (k == 0) ? d - 1 : L - 1;
  const uint32_t G = gens[U];
  std::memset(&P, 0, sizeof P);
  for (int i = 0; i < d; ++i) P.g.g[i] = gens[i];
  P.n = uint32_t(n);
  P.d = d;
  P.U = U;
  P.k = k;
  P.total = total;
  P.table = T;
  P.table_stride = N;
  P.err = err;
  P.checksum = checksum;
  P.out = out;
  P.dG = DivMod32::make(G);
  P.ring = d <= 16 ? 128 : 64;
  P.flush = P.ring / 2;
  P.max_tiles = kMinTileStates;  // grown by size_write_pass to what LDS leaves
  if (k < 1) return 0;
  // Pair lanes when the lane coordinate a_{U-1} takes few values: at most
  // n / g_{U-1} < kPairBelow (its range after the outer prefix is smaller
  // still), so that most steps would leave lanes idle; each step then takes
  // 64 (a_{U-2}, a_{U-1}) pairs.  The threshold is measured: pairs win on the
  // sweep workloads at d = 7 (n / g_{U-1} = 170 and 194) and 9 (57, 59) and
  // lose on the large workload (273, whose row assembly is compiled per shape).
  // ZSET_PAIR=0 / 1 forces the choice (tests).
  if (U >= 2) {
    P.dG1 = DivMod32::make(gens[U - 1]);
    const char* pe = std::getenv("ZSET_PAIR");
    if (pe && (pe[0] == '0' || pe[0] == '1')) P.pair = pe[0] == '1';
    else P.pair = n / gens[U - 1] < kPairBelow;
  }
  const uint64_t Rn = sums[L];  // rows of Memo[p] over p <= n
  leaf_format(P, n, gens, U, k);
  P.nclass = uint32_t(std::min<uint64_t>(G, N));
  const char* lds_env = std::getenv("ZSET_MEMO_LDS");
  const bool lds_off = lds_env && std::strcmp(lds_env, "0") == 0;
  if (lds_off || Rn >= (uint64_t(1) << 32)) P.pack = 0;
  if (P.pack != 0) {
    P.memo_words = Rn * uint64_t(P.pack);
    if (write_lds_bytes(P) > lds_max) P.pack = 0;
  }
  if (P.pack == 0) P.memo_words = 0;
  // Segment counts and class ends in LDS too when every value fits 32 bits
  // (their sum over x <= n bounds each) and the space is there.
  if (!lds_off && sums[U] < (uint64_t(1) << 32) && Rn < (uint64_t(1) << 32)) {
    P.lds_cnt = 1;
    if (write_lds_bytes(P) > lds_max) P.lds_cnt = 0;
  }
  P.leaf_rows = Rn;
  return P.pack ? Rn * uint64_t(P.pack) : Rn * uint64_t(k + 1);
}

// Status words and scratch of zset_enumerate_noalloc carved in order from the
// device's scratch array (256-byte aligned pieces).
struct Carve {
  unsigned char* base;
  size_t cap;
  size_t used;
  template <class Tp>
  Tp* take(size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    if (bytes > cap || off > cap - bytes) return nullptr;
    used = off + (bytes ? bytes : 1);
    return reinterpret_cast<Tp*>(base + off);
  }
};

__global__ void k_clear_words(uint64_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// The outcome of an asynchronous call, for a host that reads pinned memory
// once the stream is done: result[0] = zset_status (as a signed 64-bit value;
// the kernels' status word mapped as the synchronous call maps it), [1] =
// |Z(n)|, [2] = the checksum (count-only calls, else 0).  One thread.
__global__ void k_publish_result(const uint64_t* misc, uint32_t total_word, int count_only,
                                 uint64_t* result, uint64_t* done, uint64_t seq) {
  if (threadIdx.x != 0) return;
  const int code = reinterpret_cast<const volatile int*>(misc)[0];
  int64_t st = ZSET_OK;
  if (code == kErrOverflow) st = ZSET_EOVERFLOW;
  else if (code == kErrCapacity) st = ZSET_ECAPACITY;
  else if (code == kErrSlices) st = ZSET_EINVAL;
  else if (code != 0) st = ZSET_EDEVICE;
  result[1] = misc[total_word];
  result[2] = count_only ? misc[1] : 0;
  __threadfence_system();
  result[0] = uint64_t(st);
  __threadfence_system();
  *reinterpret_cast<volatile uint64_t*>(done) = seq;
}

}  // namespace
}  // namespace zset

// Device scratch of zset_enumerate_noalloc: one copy on every device the
// library runs on, held until the process ends.  Host code never passes this
// name to a kernel or a copy (on the host it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress gives for the current
// device, kept per device in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[ZSET_NOALLOC_SCRATCH_BYTES];

namespace zset {
namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};  // guarded by g_mu

// The scratch array's address on device `dev` (current), looked up on the
// first call on that device.
zset_status noalloc_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ZSET_EDEVICE, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(ZSET_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return ZSET_OK;
}

zset_status scratch_full(const char* what, size_t bytes) {
  return fail(ZSET_ENOMEM, std::string("zset_enumerate_noalloc: the ") + what + " (" +
                               std::to_string(bytes) + " bytes) does not fit in what is left of "
                               "the " + std::to_string(size_t(ZSET_NOALLOC_SCRATCH_BYTES)) +
                               "-byte scratch array; use zset_enumerate_ex");
}

}  // namespace
}  // namespace zset


using namespace zset;

extern "C" {

void zset_default_opts(zset_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->k = -1;
  o->claim_pct = -1;
}

const char* zset_strerror(zset_status s) {
  // A caller may pass any int (the C ABI): read the bits as an int, since a
  // value outside the enumerators' range is not a valid zset_status in C++.
  int v = 0;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case ZSET_OK: return "success";
    case ZSET_EINVAL: return "invalid argument";
    case ZSET_EOVERFLOW: return "count overflows 64 bits";
    case ZSET_ENOMEM: return "out of memory";
    case ZSET_ECAPACITY: return "output buffer too small";
    case ZSET_EDEVICE: return "device error";
  }
  return "unknown status";
}

const char* zset_last_error(void) { return g_last_error.c_str(); }

zset_status zset_count(uint64_t n, const uint32_t* gens, int d, uint64_t* count) {
  g_last_error.clear();
  zset_status st = check_query(n, gens, d);
  if (st != ZSET_OK) return st;
  if (!count) return fail(ZSET_EINVAL, "count is NULL");
  std::lock_guard<std::mutex> lock(g_mu);
  Ctx* c = nullptr;
  if ((st = get_ctx(&c)) != ZSET_OK) return st;
  if ((st = settle(c)) != ZSET_OK) return st;
  const uint64_t N = n + 1;
  if ((st = ensure(c->table, size_t(d + 1) * N * sizeof(uint64_t))) != ZSET_OK) return st;
  uint64_t* T = reinterpret_cast<uint64_t*>(c->table.p);
  ZSET_HIP(launch_count_table(T, n, gens, d, nullptr, nullptr));
  ZSET_HIP(hipMemcpyAsync(c->pinned, T + n, sizeof(uint64_t), hipMemcpyDeviceToHost, nullptr));
  ZSET_HIP(hipStreamSynchronize(nullptr));
  *count = c->pinned[0];
  if (*count == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
  return ZSET_OK;
}

zset_status zset_count_table(uint64_t n, const uint32_t* gens, int d, uint64_t* table,
                             void* stream) {
  g_last_error.clear();
  zset_status st = check_query(n, gens, d);
  if (st != ZSET_OK) return st;
  if (!table) return fail(ZSET_EINVAL, "table is NULL");
  if (!is_device_pointer(table)) return fail(ZSET_EINVAL, "table is not device memory");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ZSET_HIP(launch_count_table(table, n, gens, d, nullptr, s));
  ZSET_HIP(hipStreamSynchronize(s));
  return ZSET_OK;
}

zset_status zset_memo_build(const uint32_t* gens_trailing, int k, uint64_t top, void* stream,
                            zset_memo* memo) {
  g_last_error.clear();
  if (!memo) return fail(ZSET_EINVAL, "memo is NULL");
  *memo = nullptr;
  if (k < 1 || k > kMaxD - 1) return fail(ZSET_EINVAL, "k must lie in [1, 31]");
  zset_status st = check_gens(gens_trailing, k, "gens_trailing");
  if (st != ZSET_OK) return st;
  if (top < 1 || top - 1 > kMaxN) return fail(ZSET_EINVAL, "top must lie in [1, 2^31 - 1]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  Ctx* c = nullptr;
  if ((st = get_ctx(&c)) != ZSET_OK) return st;
  if ((st = settle(c)) != ZSET_OK) return st;
  // Count table of the memo's own generators up to top - 1: row i holds
  // |Z(m; h_i..h_k)| = |Z_{>=i}(m; h)|, and row 0 gives the list sizes.
  const uint64_t nm = top - 1;
  if ((st = ensure(c->hcount, size_t(k + 1) * top * sizeof(uint64_t))) != ZSET_OK) return st;
  uint64_t* CT = reinterpret_cast<uint64_t*>(c->hcount.p);
  uint64_t* msums = reinterpret_cast<uint64_t*>(c->misc.p) + kMiscRowSums;
  ZSET_HIP(launch_count_table(CT, nm, gens_trailing, k, msums, s));
  zset_memo m = new zset_memo_s();
  std::memset(m, 0, sizeof *m);
  m->k = k;
  m->top = top;
  m->device = c->device;
  for (int i = 0; i < k; ++i) m->h[i] = gens_trailing[i];
  auto cleanup = [&](zset_status r) {
    if (m->off) (void)hipFree(m->off);
    if (m->nat) (void)hipFree(m->nat);
    delete m;
    return r;
  };
  if (fault_injected("alloc")) return cleanup(fail(ZSET_ENOMEM, "allocation refused (ZSET_FAULT=alloc)"));
  if (hipMalloc(&m->off, (top + 1) * sizeof(uint64_t)) != hipSuccess) {
    (void)hipGetLastError();
    m->off = nullptr;
    return cleanup(fail(ZSET_ENOMEM, "hipMalloc of memo offsets failed"));
  }
  hipError_t e = launch_exclusive_scan(CT, top, m->off, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->pinned, m->off + top, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)  // the longest list: the count table's row-0 maximum
    e = hipMemcpyAsync(c->pinned + 1, msums + k + 2, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "memo offsets"));
  const uint64_t R = c->pinned[0];
  const uint64_t rowmax = c->pinned[1];
  if (R == ~uint64_t(0)) return cleanup(fail(ZSET_EOVERFLOW, "memo rows overflow 64 bits"));
  m->rows = R;
  if (hipMalloc(&m->nat, std::max<size_t>(16, size_t(R) * k * sizeof(uint32_t))) != hipSuccess) {
    (void)hipGetLastError();
    m->nat = nullptr;
    return cleanup(fail(ZSET_ENOMEM, "hipMalloc of memo rows failed"));
  }
  int* err = reinterpret_cast<int*>(c->misc.p);
  e = hipMemsetAsync(err, 0, sizeof(int), s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemsetAsync"));
  st = build_memo_rows(m->h, k, top, m->off, CT, top, R, rowmax, m->nat, err,
                       size_t(max_lds_bytes(c)), ctx_srcw(c), s);
  if (st != ZSET_OK) return cleanup(st);
  e = hipMemcpyAsync(c->pinned, err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "memo build"));
  const int code = *reinterpret_cast<int*>(c->pinned);
  if (code != 0) return cleanup(fail(ZSET_EDEVICE, device_error_text(code)));
  *memo = m;
  return ZSET_OK;
}

void zset_memo_free(zset_memo memo) {
  if (!memo) return;
  if (memo->off) (void)hipFree(memo->off);
  if (memo->nat) (void)hipFree(memo->nat);
  delete memo;
}

zset_status zset_memo_read(zset_memo memo, uint64_t* off, uint32_t* rows, uint64_t* top_out,
                           int* k_out, uint64_t* rows_out) {
  g_last_error.clear();
  if (!memo) return fail(ZSET_EINVAL, "memo is NULL");
  if (top_out) *top_out = memo->top;
  if (k_out) *k_out = memo->k;
  if (rows_out) *rows_out = memo->rows;
  if (off) ZSET_HIP(hipMemcpy(off, memo->off, (memo->top + 1) * sizeof(uint64_t),
                              hipMemcpyDeviceToHost));
  if (rows && memo->rows)
    ZSET_HIP(hipMemcpy(rows, memo->nat, memo->rows * memo->k * sizeof(uint32_t),
                       hipMemcpyDeviceToHost));
  return ZSET_OK;
}

zset_status zset_enumerate(uint64_t n, const uint32_t* gens, int d, uint32_t* out) {
  return zset_enumerate_ex(n, gens, d, out, ~uint64_t(0), nullptr, nullptr, nullptr, nullptr,
                           nullptr);
}

namespace zset {
namespace {

// Rows of the memo Z(p; h) over p <= n for k = 1 and k = 2 trailing
// generators, counted on the host: the number of m >= 0 with
// m_1 h_1 (+ m_2 h_2) <= n.  For k = 2 the sum runs over multiples of the
// larger generator.  Returns false when that takes more than kHostCountSteps
// steps.
constexpr uint64_t kHostCountSteps = 1 << 16;
// Memo rows the setup launch's one memo workgroup builds, at most (larger
// memos take the element-parallel launches).
constexpr uint64_t kSetupMemoRows = uint64_t(1) << 19;
bool host_memo_rows(uint64_t n, const uint32_t* h, int k, uint64_t* rows) {
  if (k == 1) {
    *rows = n / h[0] + 1;
    return true;
  }
  const uint64_t big = std::max(h[0], h[1]), small = std::min(h[0], h[1]);
  if (n / big + 1 > kHostCountSteps) return false;
  uint64_t r = 0;
  for (uint64_t x = 0; x <= n; x += big) r += (n - x) / small + 1;
  *rows = r;
  return true;
}

// zset_enumerate_ex with the memo dimension fixed at 1 or 2 by the caller:
// every launch is enqueued at once, with no readback of |Z(n)| in the middle.
// The memo's size comes from host_memo_rows; the slice planner and the write
// pass read |Z(n)| from device memory (EnumParams::total_dev) and size the
// slices from it, and a query that overflows or exceeds out_rows_cap is
// refused on the device (no slices: nothing written) and reported at the end.
// *taken = false (and nothing enqueued) when the call needs the general path.
// The three-launch path of a call whose memo dimension is 1 or 2, when the
// call qualifies (*taken).  With async_result the launches are only enqueued:
// the outcome goes to async_result (pinned host words, k_publish_result) and
// wev, if given, are recorded around the write pass.
zset_status enumerate_fixed_k(Ctx* c, uint64_t n, const uint32_t* gens, int d, uint32_t* out,
                              uint64_t out_rows_cap, const zset_opts& opts,
                              uint64_t* rows_written, uint64_t* checksum, zset_stats* stats,
                              hipStream_t s, bool* taken, uint64_t* async_result = nullptr,
                              const hipEvent_t* wev = nullptr) {
  *taken = false;
  const int k = opts.k;
  const bool count_only = opts.count_only != 0;
  if (k < 1 || k > 2 || d < 2 || k > d - 1 || opts.rows_per_tile != 0 ||
      (opts.claim_pct != -1 && opts.claim_pct != 100) ||
      (opts.memo_top != 0 && opts.memo_top <= n) || std::getenv("ZSET_MEMO_PATH") ||
      std::getenv("ZSET_FIXED_K_READBACK"))
    return ZSET_OK;
  const uint64_t N = n + 1;
  const int L = d - k, U = L - 1;
  const uint32_t G = gens[U];
  uint64_t Rn = 0;
  if (!host_memo_rows(n, gens + L, k, &Rn) || Rn >= (uint64_t(1) << 32)) return ZSET_OK;
  // The row sums the write pass's format needs: the memo's rows, and a bound
  // on the sum of C_U[x] over x <= n (each x contributes at most
  // (x / G + 1) memo lists), which decides whether segment counts and class
  // ends fit 32 bits.
  uint64_t sums[kMaxD + 1] = {};
  sums[L] = Rn;
  const uint64_t qmax = n / G + 1;
  sums[U] = Rn > ~uint64_t(0) / qmax ? ~uint64_t(0) : Rn * qmax;
  uint64_t* misc = reinterpret_cast<uint64_t*>(c->misc.p);
  int* err = reinterpret_cast<int*>(misc + kMiscErr);
  zset_status st;
  if ((st = grow(c, c->table, size_t(d + 1) * N * sizeof(uint64_t))) != ZSET_OK) return st;
  uint64_t* T = reinterpret_cast<uint64_t*>(c->table.p);
  EnumParams P;
  const uint64_t leaf_words = init_params(P, n, gens, d, k, 0, sums, T, err, misc + kMiscSum, out,
                                          size_t(write_lds_budget(c->device)));
  P.desc = opts.order == 1 && !count_only;
  const uint64_t want = plan_want_tiles(c->device);
  const bool align16 = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  P.pool = reinterpret_cast<uint32_t*>(misc + kMiscPool);
  // Grid and slice-state room as for want_tiles slices of 128 rows (every
  // slice claimed): the write pass then takes the real slices from the plan.
  P.total = want * 128;
  if ((st = size_write_pass(P, 0, 100, c->device, count_only, align16, 1, want)) != ZSET_OK)
    return st;
  if (P.chunk == 0 || P.static_tiles != 0) return ZSET_OK;  // claims do not fit: general path
  P.total = 0;
  P.rows_per_tile = 0;
  P.ntiles = 0;
  P.total_dev = misc + kMiscRowSums + d + 1;
  P.want_tiles = want;
  P.out_rows_cap = count_only ? 0 : out_rows_cap;
  P.dyn = 1;
  *taken = true;

  if ((st = grow(c, c->off, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  if ((st = grow(c, c->nat, size_t(Rn) * k * sizeof(uint32_t))) != ZSET_OK) return st;
  if ((st = grow(c, c->endc, size_t(std::min<uint64_t>(G, N)) * sizeof(uint64_t))) != ZSET_OK)
    return st;
  if ((st = grow(c, c->leaf, size_t(leaf_words) * sizeof(uint32_t))) != ZSET_OK) return st;
  if ((st = grow(c, c->tiles, size_t(want) * (U + 2) * sizeof(uint32_t))) != ZSET_OK) return st;
  if (k == 2 && (st = grow(c, c->cnt2, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
  P.endc = reinterpret_cast<uint64_t*>(c->endc.p);
  P.leaf = reinterpret_cast<uint32_t*>(c->leaf.p);
  P.tiles = reinterpret_cast<uint32_t*>(c->tiles.p);
  uint64_t* off = reinterpret_cast<uint64_t*>(c->off.p);
  uint32_t* nat = reinterpret_cast<uint32_t*>(c->nat.p);

  const bool fused = N <= count_table_lds_max() && Rn <= kSetupMemoRows &&
                     !std::getenv("ZSET_COUNT_PATH") && !std::getenv("ZSET_FIXED_K_SPLIT");
  if (fused) {
    // Three launches: setup (count table and class ends in one workgroup,
    // the memo in another; status words cleared), slice plan and leaf layout
    // in one grid, write pass.  Fewer launches is less host enqueue time
    // ahead of the write pass.
    SetupJob J;
    std::memset(&J, 0, sizeof J);
    J.table = T;
    J.sums = misc + kMiscRowSums;
    J.status = misc;
    for (int i = 0; i < d; ++i) J.g.g[i] = gens[i];
    J.N = uint32_t(N);
    J.d = d;
    J.U = U;
    J.nclass = P.nclass;
    J.dG = DivMod32::make(G);
    J.endc = const_cast<uint64_t*>(P.endc);
    J.k = k;
    if (k == 2) J.M = make_memo2(gens[L], gens[L + 1]);
    J.h1 = gens[L];
    J.R = uint32_t(Rn);
    J.nat = nat;
    J.off = off;
    J.stamps = misc + kMiscStamp;
    if (count_last_rows_enabled()) J.last = make_last_rows(gens, d);
    if ((st = grow(c, c->rowp, size_t(Rn) * sizeof(uint32_t))) != ZSET_OK) return st;
    J.rowp = reinterpret_cast<uint32_t*>(c->rowp.p);
    LeafJob LJ = make_leaf_job(k, n, G, off, nat, T + uint64_t(U) * N, P.endc,
                               const_cast<uint32_t*>(P.leaf), Rn, P);
    LJ.rowp = J.rowp;
    const bool timed = stats != nullptr;  // no timing events without stats
    if (timed) ZSET_HIP(hipEventRecord(c->ev[0], s));
    ZSET_HIP(launch_setup_fixed(J, s));
    if (timed) ZSET_HIP(hipEventRecord(c->ev[1], s));
    ZSET_HIP(launch_plan_leaf(P, LJ, s));
    if (timed) ZSET_HIP(hipEventRecord(c->ev[4], s));
    if (wev) ZSET_HIP(hipEventRecord(wev[0], s));
    ZSET_HIP(launch_write(P, count_only, align16, s));
    if (wev) ZSET_HIP(hipEventRecord(wev[1], s));
    if (timed) ZSET_HIP(hipEventRecord(c->ev[5], s));
    if (async_result) {
      const uint64_t seq = c->seq + 1;
      hipLaunchKernelGGL(k_publish_result, dim3(1), dim3(64), 0, s, misc,
                         uint32_t(kMiscRowSums + d + 1), count_only ? 1 : 0, async_result,
                         c->done_dev, seq);
      ZSET_HIP(hipGetLastError());
      c->seq = seq;
      c->busy_stream = s;
      c->inflight = true;
      return ZSET_OK;
    }
    ZSET_HIP(hipMemcpyAsync(c->pinned, misc, kMiscWords * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, s));
    ZSET_HIP(hipStreamSynchronize(s));
  } else {
    // Enqueued in the order of the critical path: status words clear, count
    // table, class ends and slice plan on the call's stream; then the memo
    // (closed form) on the side stream, which needs only the status reset and
    // runs beside them; then the leaf layout (after the memo) and the write
    // pass.  The host's enqueue time would otherwise delay the count table.
    ZSET_HIP(hipEventRecord(c->ev[0], s));
    ZSET_HIP(hipMemsetAsync(misc, 0, 2 * sizeof(uint64_t), s));
    ZSET_HIP(hipEventRecord(c->fork, s));
    ZSET_HIP(launch_count_table(T, n, gens, d, misc + kMiscRowSums, s));
    ZSET_HIP(hipEventRecord(c->ev[1], s));
    uint32_t nclass = 0;
    ZSET_HIP(launch_class_ends(T + uint64_t(U) * N, n, G, const_cast<uint64_t*>(P.endc), &nclass,
                               s));
    ZSET_HIP(launch_plan_device_sized(P, s));
    ZSET_HIP(hipEventRecord(c->ev[3], s));
    struct SideJoin {
      Ctx* c = nullptr;
      ~SideJoin() {
        if (c) (void)hipStreamSynchronize(c->side);
      }
    } side_join;
    ZSET_HIP(hipStreamWaitEvent(c->side, c->fork, 0));
    side_join.c = c;
    ZSET_HIP(hipEventRecord(c->memo0, c->side));
    if (k == 2)
      ZSET_HIP(launch_memo_k2(gens[L], gens[L + 1], N, Rn, nat, off,
                              reinterpret_cast<uint64_t*>(c->cnt2.p), c->side));
    else
      ZSET_HIP(launch_memo_k1(gens[L], N, Rn, nat, off, c->side));
    ZSET_HIP(hipEventRecord(c->memo1, c->side));
    ZSET_HIP(hipStreamWaitEvent(s, c->memo1, 0));
    ZSET_HIP(launch_memo_leaf(make_leaf_job(k, n, G, off, nat, T + uint64_t(U) * N, P.endc,
                                            const_cast<uint32_t*>(P.leaf), Rn, P),
                              err, s));
    ZSET_HIP(hipEventRecord(c->ev[4], s));
    if (wev) ZSET_HIP(hipEventRecord(wev[0], s));
    ZSET_HIP(launch_write(P, count_only, align16, s));
    if (wev) ZSET_HIP(hipEventRecord(wev[1], s));
    ZSET_HIP(hipEventRecord(c->ev[5], s));
    // Status, checksum and |Z(n)| in one readback.
    static_assert(kMiscErr == 0 && kMiscSum == 1 && kMiscRowSums == 2, "misc layout");
    ZSET_HIP(hipMemcpyAsync(c->pinned, misc, (kMiscRowSums + d + 2) * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, s));
    ZSET_HIP(hipStreamSynchronize(s));
    side_join.c = nullptr;  // the call's stream waited for the side stream
  }
  const int code = *reinterpret_cast<int*>(c->pinned);
  const uint64_t total = c->pinned[kMiscRowSums + d + 1];
  if (async_result) {
    // An asynchronous call that took the separate launches ran to the end
    // here: its outcome is written from the host.
    int64_t rs = ZSET_OK;
    if (code == kErrOverflow) rs = ZSET_EOVERFLOW;
    else if (code == kErrCapacity) rs = ZSET_ECAPACITY;
    else if (code == kErrSlices) rs = ZSET_EINVAL;
    else if (code != 0) rs = ZSET_EDEVICE;
    async_result[1] = total;
    async_result[2] = count_only ? c->pinned[kMiscSum] : 0;
    async_result[0] = uint64_t(rs);
  }
  if (code == kErrOverflow) {
    if (total == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
    return fail(ZSET_EOVERFLOW, "|Z(n)| * d * 4 bytes overflows 64 bits");
  }
  if (code == kErrCapacity)
    return fail(ZSET_ECAPACITY, "out holds " + std::to_string(out_rows_cap) + " rows, |Z(n)| = " +
                                    std::to_string(total));
  if (code == kErrSlices) return fail(ZSET_EINVAL, "too many slices: raise rows_per_tile");
  if (code != 0) return fail(ZSET_EDEVICE, device_error_text(code));
  if (rows_written) *rows_written = total;
  if (checksum) *checksum = count_only ? c->pinned[kMiscSum] : 0;
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    const uint64_t T_rows = slice_rows(total, want);
    // count: the status reset and the count table; plan: class ends and
    // slice plan; memo: the closed form on the side stream and the leaf
    // layout (from the plan's end).
    if (fused) {
      // count: the setup launch (count table and class ends, the memo beside
      // them); memo: the memo workgroup's own time (device clock); plan: the
      // slice plan and leaf layout launch.
      stats->count_us = elapsed_us(c->ev[0], c->ev[1]);
      const uint64_t t0 = c->pinned[kMiscStamp], t1 = c->pinned[kMiscStamp + 1];
      stats->memo_us = c->wall_khz > 0 && t1 >= t0 ? double(t1 - t0) * 1000.0 / c->wall_khz : 0.0;
      stats->plan_us = elapsed_us(c->ev[1], c->ev[4]);
    } else {
      stats->count_us = elapsed_us(c->ev[0], c->ev[1]);
      stats->plan_us = elapsed_us(c->ev[1], c->ev[3]);
      stats->memo_us = elapsed_us(c->memo0, c->memo1) + elapsed_us(c->ev[3], c->ev[4]);
    }
    stats->write_us = elapsed_us(c->ev[4], c->ev[5]);
    stats->total_us = elapsed_us(c->ev[0], c->ev[5]);
    stats->rows = total;
    stats->memo_rows = Rn;
    stats->memo_bytes = leaf_words * 4;
    stats->tiles = (total + T_rows - 1) / T_rows;
    stats->rows_per_tile = T_rows;
    stats->k = k;
  }
  return ZSET_OK;
}

}  // namespace
}  // namespace zset

namespace zset {
namespace {

// The checks zset_enumerate_ex and zset_enumerate_async share: the query,
// the options (opts = *opts_in or the defaults) and the output pointer's
// presence.
zset_status check_enumerate(uint64_t n, const uint32_t* gens, int d, const uint32_t* out,
                            const zset_opts* opts_in, zset_opts& opts) {
  zset_status st = check_query(n, gens, d);
  if (st != ZSET_OK) return st;
  if (opts_in) opts = *opts_in; else zset_default_opts(&opts);
  if (opts.k < -1 || opts.k > d - 1) return fail(ZSET_EINVAL, "k must be -1 or lie in [0, d-1]");
  if (opts.order != 0 && opts.order != 1) return fail(ZSET_EINVAL, "order must be 0 or 1");
  if (opts.claim_pct < -1 || opts.claim_pct > 100)
    return fail(ZSET_EINVAL, "claim_pct must be -1 or lie in [0, 100]");
  if (opts.rows_per_tile % 128 != 0 || opts.rows_per_tile > (uint64_t(1) << 30))
    return fail(ZSET_EINVAL, "rows_per_tile must be a multiple of 128 and at most 2^30");
  if (opts.count_only == 0 && !out) return fail(ZSET_EINVAL, "out is NULL");
  return ZSET_OK;
}

}  // namespace
}  // namespace zset

zset_status zset_enumerate_ex(uint64_t n, const uint32_t* gens, int d, uint32_t* out,
                              uint64_t out_rows_cap, const zset_opts* opts_in, zset_memo memo,
                              uint64_t* rows_written, uint64_t* checksum, zset_stats* stats) {
  g_last_error.clear();
  zset_opts opts;
  zset_status st = check_enumerate(n, gens, d, out, opts_in, opts);
  if (st != ZSET_OK) return st;
  const bool count_only = opts.count_only != 0;
  if (memo) {
    if (opts.k != -1 && opts.k != memo->k)
      return fail(ZSET_EINVAL, "opts.k differs from the memo's k");
    if (memo->k > d - 1) return fail(ZSET_EINVAL, "memo has more coordinates than d - 1");
    for (int i = 0; i < memo->k; ++i)
      if (memo->h[i] != gens[d - memo->k + i])
        return fail(ZSET_EINVAL, "memo generators differ from the trailing generators");
    // A memo whose top is <= n is partial: rows with memo remainder >= top
    // come from the count table (Alg 3.2's Else branch).
  }
  if (!count_only && !is_device_pointer(out)) return fail(ZSET_EINVAL, "out is not device memory");

  hipStream_t s = reinterpret_cast<hipStream_t>(opts.stream);
  std::lock_guard<std::mutex> lock(g_mu);
  Ctx* c = nullptr;
  if ((st = get_ctx(&c)) != ZSET_OK) return st;
  if ((st = settle(c)) != ZSET_OK) return st;
  if (memo && memo->device != c->device)
    return fail(ZSET_EINVAL, "memo lives on another device");
  if (!memo) {
    bool taken = false;
    st = enumerate_fixed_k(c, n, gens, d, out, out_rows_cap, opts, rows_written, checksum, stats,
                           s, &taken);
    if (taken || st != ZSET_OK) return st;
  }

  const uint64_t N = n + 1;
  uint64_t* misc = reinterpret_cast<uint64_t*>(c->misc.p);
  int* err = reinterpret_cast<int*>(misc + kMiscErr);
  if ((st = ensure(c->table, size_t(d + 1) * N * sizeof(uint64_t))) != ZSET_OK) return st;
  uint64_t* T = reinterpret_cast<uint64_t*>(c->table.p);
  // Memo coverage: every p <= n, or p < top (a partial memo: a memo handle's
  // top, or opts.memo_top).  Rows whose memo remainder is >= top are then
  // unranked from the count table by the write pass (Alg 3.2's Else branch).
  uint64_t top = N;
  if (memo) top = std::min<uint64_t>(memo->top, N);
  else if (opts.memo_top) top = std::min<uint64_t>(opts.memo_top, N);
  const bool partial = top < N;

  // 1. Count table, row sums (memo sizes), total.  When k >= 1 is fixed by the
  // caller, the memo recurrence needs nothing from the count table: it starts
  // at once on the side stream, beside the count table and the readback below,
  // with room for as many memo rows as LDS holds.  If the memo turns out larger
  // (known once the row sums are back), it is rebuilt below.
  ZSET_HIP(hipEventRecord(c->ev[0], s));
  ZSET_HIP(hipMemsetAsync(misc, 0, 2 * sizeof(uint64_t), s));
  struct SideJoin {  // every return after an early launch waits for the side stream
    Ctx* c = nullptr;
    ~SideJoin() {
      if (c) (void)hipStreamSynchronize(c->side);
    }
  } side_join;
  bool early = false;
  uint64_t early_cap = 0;
  // The memo build (closed form for k = 2, else the recurrence) is enqueued
  // first: the rest of the call waits for it.  The fork event orders it after
  // the status reset.
  ZSET_HIP(hipEventRecord(c->fork, s));
  {
    const char* path = std::getenv("ZSET_MEMO_PATH");
    const bool force_global = path && std::strcmp(path, "global") == 0;
    const bool force_chain = path && std::strcmp(path, "chain") == 0;
    if (!memo && opts.k >= 1 && d >= 2 && !force_global && !partial) {
      const int kk = opts.k, L0 = d - kk;
      uint32_t b = gens[L0], hmax = gens[L0];
      for (int i = L0; i < d; ++i) {
        b = std::min(b, gens[i]);
        hmax = std::max(hmax, gens[i]);
      }
      const uint32_t step = std::min<uint32_t>(b, kWave);
      const uint64_t Wl = uint64_t(hmax) + step;
      if (Wl < (uint64_t(1) << 30) && kk >= 2) {
        const uint32_t W = next_pow2(uint32_t(Wl));
        early_cap = std::min<uint64_t>(memo_wave_capacity(kk, W, size_t(max_lds_bytes(c))),
                                       (uint64_t(1) << 30) - 1);
        if (early_cap > 0) {
          if ((st = ensure(c->off, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
          if ((st = ensure(c->nat, size_t(early_cap) * kk * sizeof(uint32_t))) != ZSET_OK)
            return st;
          ZSET_HIP(hipStreamWaitEvent(c->side, c->fork, 0));
          side_join.c = c;
          ZSET_HIP(hipEventRecord(c->memo0, c->side));
          if (kk == 2 && !force_chain) {
            // Two coordinates: the closed form, element-parallel.
            if ((st = ensure(c->cnt2, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
            ZSET_HIP(launch_memo_k2(gens[L0], gens[L0 + 1], N, early_cap,
                                    reinterpret_cast<uint32_t*>(c->nat.p),
                                    reinterpret_cast<uint64_t*>(c->off.p),
                                    reinterpret_cast<uint64_t*>(c->cnt2.p), c->side));
          } else {
            ZSET_HIP(launch_memo_chain_wave(gens + L0, kk, N, step, W, early_cap, 0,
                                            reinterpret_cast<uint32_t*>(c->nat.p),
                                            reinterpret_cast<uint64_t*>(c->off.p), err, c->side));
          }
          ZSET_HIP(hipEventRecord(c->memo1, c->side));
          early = true;
        }
      }
    }
  }
  // Count table, then one readback of the row sums and |Z(n)|.
  ZSET_HIP(launch_count_table(T, n, gens, d, misc + kMiscRowSums, s));
  ZSET_HIP(hipEventRecord(c->ev[1], s));
  // When the caller fixes k (or passes a memo), the class ends and the slice
  // plan need only the count table: they run on the plan stream while the
  // host waits for the readback, the planner reading |Z(n)| on the device
  // and sizing the slices for plan_want_tiles slices (the host repeats the
  // same sizing below).
  const int k_fixed = memo ? memo->k : opts.k;
  const bool early_plan = k_fixed >= 1 && d >= 2 && opts.rows_per_tile == 0;
  const uint64_t want_early = early_plan ? plan_want_tiles(c->device) : 0;
  struct PlanJoin {  // every return after the early plan waits for its stream
    Ctx* c = nullptr;
    ~PlanJoin() {
      if (c) (void)hipStreamSynchronize(c->plan);
    }
  } plan_join;
  if (early_plan) {
    const int Ue = d - k_fixed - 1;
    const uint32_t Ge = gens[Ue];
    if ((st = ensure(c->endc, size_t(std::min<uint64_t>(Ge, top)) * sizeof(uint64_t))) != ZSET_OK)
      return st;
    if ((st = ensure(c->tiles, size_t(want_early) * (Ue + 2) * sizeof(uint32_t))) != ZSET_OK)
      return st;
    EnumParams Pe;
    std::memset(&Pe, 0, sizeof Pe);
    for (int i = 0; i < d; ++i) Pe.g.g[i] = gens[i];
    Pe.n = uint32_t(n);
    Pe.d = d;
    Pe.U = Ue;
    Pe.k = k_fixed;
    Pe.table = T;
    Pe.table_stride = N;
    Pe.err = err;
    Pe.tiles = reinterpret_cast<uint32_t*>(c->tiles.p);
    Pe.pool = reinterpret_cast<uint32_t*>(misc + kMiscPool);
    Pe.total_dev = misc + kMiscRowSums + d + 1;
    Pe.want_tiles = want_early;
    ZSET_HIP(hipEventRecord(c->counted, s));
    ZSET_HIP(hipStreamWaitEvent(c->plan, c->counted, 0));
    plan_join.c = c;
    ZSET_HIP(hipEventRecord(c->ev[2], c->plan));
    uint32_t nclass = 0;
    ZSET_HIP(launch_class_ends(T + uint64_t(Ue) * N, top - 1, Ge,
                               reinterpret_cast<uint64_t*>(c->endc.p), &nclass, c->plan));
    ZSET_HIP(launch_plan_device_sized(Pe, c->plan));
    ZSET_HIP(hipEventRecord(c->ev[3], c->plan));
    ZSET_HIP(hipEventRecord(c->planned, c->plan));
  }
  ZSET_HIP(hipMemcpyAsync(c->pinned, misc + kMiscRowSums, (2 * d + 3) * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
  ZSET_HIP(hipStreamSynchronize(s));
  uint64_t sums[kMaxD + 1], rowmax[kMaxD + 1];
  for (int j = 0; j <= d; ++j) {
    sums[j] = c->pinned[j];
    rowmax[j] = c->pinned[d + 2 + j];
  }
  const uint64_t total = c->pinned[d + 1];
  if (total == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
  if (total > (~uint64_t(0)) / (4 * uint64_t(d)))
    return fail(ZSET_EOVERFLOW, "|Z(n)| * d * 4 bytes overflows 64 bits");
  if (!count_only && total > out_rows_cap)
    return fail(ZSET_ECAPACITY, "out holds " + std::to_string(out_rows_cap) + " rows, |Z(n)| = " +
                                    std::to_string(total));

  // 2. Memo dimension.
  int k = memo ? memo->k : opts.k;
  if (d == 1) {
    k = 0;
  } else if (k < 0) {
    k = auto_memo_dim(sums, d, total);
  }

  double memo_us = 0, plan_us = 0, write_us = 0;
  uint64_t memo_rows = 0, memo_bytes = 0, ntiles = 0, T_rows = 0;

  if (total > 0 && d == 1) {
    ZSET_HIP(hipEventRecord(c->ev[2], s));
    ZSET_HIP(hipEventRecord(c->ev[3], s));
    ZSET_HIP(hipEventRecord(c->ev[6], s));
    ZSET_HIP(launch_single(n, gens[0], out, count_only, misc + kMiscSum, s));
    ZSET_HIP(hipEventRecord(c->ev[4], s));
  } else if (total > 0) {
    const int L = d - std::max(k, 1);
    const int U = (k == 0) ? d - 1 : L - 1;
    const uint32_t G = gens[U];
    EnumParams P;
    // 3. Leaf-order row format and what the write pass keeps in LDS (from the
    // row sums alone), slices, class ends and the slice plan.  None of these
    // needs the memo's rows, so while the recurrence runs on the side stream
    // they run beside it.
    const uint64_t leaf_words = init_params(P, n, gens, d, k, total, sums, T, err,
                                            misc + kMiscSum, out,
                                            size_t(write_lds_budget(c->device)));
    P.desc = opts.order == 1 && !count_only;
    // Rows of Memo[p] over p <= n: the memo's rows, or a bound on them for a
    // partial memo (p < top).
    const uint64_t Rn = k >= 1 ? sums[L] : 0;
    if (k >= 1 && partial) {
      P.memo_top = uint32_t(top);
      P.nclass = uint32_t(std::min<uint64_t>(G, top));
    }
    if (k >= 1) {
      memo_rows = Rn;
      const uint64_t nclass_max = std::min<uint64_t>(G, top);
      if ((st = ensure(c->endc, size_t(nclass_max) * sizeof(uint64_t))) != ZSET_OK) return st;
      if ((st = ensure(c->leaf, size_t(leaf_words) * sizeof(uint32_t))) != ZSET_OK) return st;
      P.endc = reinterpret_cast<uint64_t*>(c->endc.p);
      P.leaf = reinterpret_cast<uint32_t*>(c->leaf.p);
      memo_bytes = leaf_words * 4;
    }
    // Slices: exact rank ranges, starts unranked on the device; about 128
    // slices per resident wavefront by default (short slices keep the
    // concurrent write streams of a compute unit close together in memory and
    // the end of the pass even).
    const bool align16 = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    P.pool = reinterpret_cast<uint32_t*>(misc + kMiscPool);
    if ((st = size_write_pass(P, opts.rows_per_tile, opts.claim_pct, c->device, count_only, align16,
                              1, want_early)) != ZSET_OK)
      return st;
    T_rows = P.rows_per_tile;
    ntiles = P.ntiles;
    if (early_plan) {
      // Planned above on the plan stream, for the same slices.
      if (ntiles > want_early || U != d - k_fixed - 1)
        return fail(ZSET_EDEVICE, "internal: early slice plan disagrees with the write pass");
      P.tiles = reinterpret_cast<uint32_t*>(c->tiles.p);
      ZSET_HIP(hipStreamWaitEvent(s, c->planned, 0));
    } else {
      if ((st = ensure(c->tiles, size_t(ntiles) * (U + 2) * sizeof(uint32_t))) != ZSET_OK) return st;
      P.tiles = reinterpret_cast<uint32_t*>(c->tiles.p);
      ZSET_HIP(hipEventRecord(c->ev[2], s));
      if (k >= 1) {
        uint32_t nclass = 0;
        ZSET_HIP(launch_class_ends(T + uint64_t(U) * N, top - 1, G, const_cast<uint64_t*>(P.endc),
                                   &nclass, s));
      }
      ZSET_HIP(launch_plan(P, s));
      ZSET_HIP(hipEventRecord(c->ev[3], s));
    }

    // 4. Memo rows (k >= 1) -- a memo handle's, the side-stream recurrence's,
    // or built here -- then the leaf-order layout.
    if (k >= 1) {
      const uint64_t* off = nullptr;
      const uint32_t* nat = nullptr;
      if (memo) {
        off = memo->off;
        nat = memo->nat;
      } else if (early && Rn <= early_cap) {
        // The side-stream recurrence holds the whole memo.
        ZSET_HIP(hipStreamWaitEvent(s, c->memo1, 0));
        off = reinterpret_cast<const uint64_t*>(c->off.p);
        nat = reinterpret_cast<const uint32_t*>(c->nat.p);
      } else {
        if (early) ZSET_HIP(hipEventSynchronize(c->memo1));  // before any buffer is regrown
        if ((st = ensure(c->off, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
        if ((st = ensure(c->nat, size_t(Rn) * k * sizeof(uint32_t))) != ZSET_OK) return st;
        uint64_t* o = reinterpret_cast<uint64_t*>(c->off.p);
        const bool closed2 = k == 2 && memo2_closed_form();
        if (closed2) {  // two coordinates: the closed form, element-parallel
          if ((st = ensure(c->cnt2, size_t(N + 1) * sizeof(uint64_t))) != ZSET_OK) return st;
          ZSET_HIP(launch_memo_k2(gens[L], gens[L + 1], top, Rn,
                                  reinterpret_cast<uint32_t*>(c->nat.p), o,
                                  reinterpret_cast<uint64_t*>(c->cnt2.p), s));
        } else {
          st = build_memo_rows(gens + L, k, top, o, T + uint64_t(L) * N, N, Rn, rowmax[L],
                               reinterpret_cast<uint32_t*>(c->nat.p), err,
                               size_t(max_lds_bytes(c)), ctx_srcw(c), s, !partial);
          if (st != ZSET_OK) return st;
        }
        off = o;
        nat = reinterpret_cast<const uint32_t*>(c->nat.p);
      }
      ZSET_HIP(hipEventRecord(c->ev[6], s));
      LeafJob J = make_leaf_job(k, top - 1, G, off, nat, T + uint64_t(U) * N, P.endc,
                                const_cast<uint32_t*>(P.leaf), Rn, P);
      J.exact = !partial;  // else Rn bounds the rows; off[top] on the device counts them
      ZSET_HIP(launch_memo_leaf(J, err, s));
    } else {
      ZSET_HIP(hipEventRecord(c->ev[6], s));
    }
    ZSET_HIP(hipEventRecord(c->ev[4], s));

    // 5. Write (or count-only) pass.
    ZSET_HIP(launch_write(P, count_only, align16, s));
  } else {
    ZSET_HIP(hipEventRecord(c->ev[2], s));
    ZSET_HIP(hipEventRecord(c->ev[3], s));
    ZSET_HIP(hipEventRecord(c->ev[6], s));
    ZSET_HIP(hipEventRecord(c->ev[4], s));
  }
  ZSET_HIP(hipEventRecord(c->ev[5], s));
  if (early) ZSET_HIP(hipStreamWaitEvent(s, c->memo1, 0));

  if (early_plan && !(total > 0 && d > 1)) ZSET_HIP(hipStreamWaitEvent(s, c->planned, 0));
  ZSET_HIP(hipMemcpyAsync(c->pinned, misc, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  ZSET_HIP(hipStreamSynchronize(s));
  plan_join.c = nullptr;  // the call's stream waited for the plan stream
  const int code = *reinterpret_cast<int*>(c->pinned);
  if (code != 0) return fail(ZSET_EDEVICE, device_error_text(code));
  if (rows_written) *rows_written = total;
  if (checksum) *checksum = count_only ? c->pinned[1] : 0;
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->count_us = elapsed_us(c->ev[0], c->ev[1]);
    // plan: class ends + slice plan; memo: the recurrence (on the side stream
    // when it ran there, else on the call's stream up to ev[6]) and the leaf
    // layout; write: the write pass.
    plan_us = elapsed_us(c->ev[2], c->ev[3]);
    memo_us = elapsed_us(c->ev[6], c->ev[4]);
    if (early && k >= 1 && total > 0 && d > 1 && memo_rows <= early_cap)
      memo_us += elapsed_us(c->memo0, c->memo1);
    else
      memo_us += elapsed_us(c->ev[3], c->ev[6]);
    write_us = elapsed_us(c->ev[4], c->ev[5]);
    stats->memo_us = memo ? 0.0 : memo_us;
    stats->plan_us = plan_us;
    stats->write_us = write_us;
    stats->total_us = elapsed_us(c->ev[0], c->ev[5]);
    stats->rows = total;
    stats->memo_rows = memo_rows;
    stats->memo_bytes = memo_bytes;
    stats->tiles = ntiles;
    stats->rows_per_tile = T_rows;
    stats->k = k;
  }
  return ZSET_OK;
}

zset_status zset_enumerate_async(uint64_t n, const uint32_t* gens, int d, uint32_t* out,
                                 uint64_t out_rows_cap, const zset_opts* opts_in,
                                 uint64_t* result, void* const* write_events) {
  g_last_error.clear();
  zset_opts opts;
  zset_status st = check_enumerate(n, gens, d, out, opts_in, opts);
  if (st != ZSET_OK) return st;
  if (!result) return fail(ZSET_EINVAL, "result is NULL");
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  if (hipPointerGetAttributes(&attr, result) != hipSuccess || attr.type != hipMemoryTypeHost ||
      !attr.devicePointer) {
    (void)hipGetLastError();
    return fail(ZSET_EINVAL, "result is not pinned host memory (hipHostMalloc)");
  }
  if (opts.count_only == 0 && !is_device_pointer(out))
    return fail(ZSET_EINVAL, "out is not device memory");
  hipEvent_t wev[2] = {};
  if (write_events) {
    wev[0] = reinterpret_cast<hipEvent_t>(write_events[0]);
    wev[1] = reinterpret_cast<hipEvent_t>(write_events[1]);
    if (!wev[0] || !wev[1]) return fail(ZSET_EINVAL, "write_events holds a NULL event");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(opts.stream);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    Ctx* c = nullptr;
    if ((st = get_ctx(&c)) != ZSET_OK) return st;
    // A previous asynchronous call on another stream may still read the
    // context's buffers; one on this stream runs before this call anyway.
    if (c->inflight && c->busy_stream != s && (st = settle(c)) != ZSET_OK) return st;
    bool taken = false;
    st = enumerate_fixed_k(c, n, gens, d, out, out_rows_cap, opts, nullptr, nullptr, nullptr, s,
                           &taken, static_cast<uint64_t*>(attr.devicePointer),
                           write_events ? wev : nullptr);
    if (taken || st != ZSET_OK) return st;
  }
  // Not the three-launch form: the call runs to completion here.
  uint64_t rows = 0, sum = 0;
  st = zset_enumerate_ex(n, gens, d, out, out_rows_cap, &opts, nullptr, &rows, &sum, nullptr);
  result[1] = rows;
  result[2] = sum;
  result[0] = uint64_t(int64_t(st));
  return st;
}

zset_status zset_enumerate_noalloc(uint64_t n, const uint32_t* gens, int d, uint32_t* out,
                                   uint64_t out_rows_cap, const zset_opts* opts_in,
                                   uint64_t* rows_written, uint64_t* checksum) {
  g_last_error.clear();
  zset_status st = check_query(n, gens, d);
  if (st != ZSET_OK) return st;
  zset_opts opts;
  if (opts_in) opts = *opts_in; else zset_default_opts(&opts);
  if (opts.k < -1 || opts.k > d - 1) return fail(ZSET_EINVAL, "k must be -1 or lie in [0, d-1]");
  if (opts.order != 0 && opts.order != 1) return fail(ZSET_EINVAL, "order must be 0 or 1");
  if (opts.claim_pct < -1 || opts.claim_pct > 100)
    return fail(ZSET_EINVAL, "claim_pct must be -1 or lie in [0, 100]");
  if (opts.rows_per_tile % 128 != 0 || opts.rows_per_tile > (uint64_t(1) << 30))
    return fail(ZSET_EINVAL, "rows_per_tile must be a multiple of 128 and at most 2^30");
  if (opts.memo_top != 0 && opts.memo_top <= n)
    return fail(ZSET_EINVAL, "zset_enumerate_noalloc takes no partial memo (memo_top <= n)");
  const bool count_only = opts.count_only != 0;
  if (!count_only && !out) return fail(ZSET_EINVAL, "out is NULL");
  if (!count_only && !is_device_pointer(out)) return fail(ZSET_EINVAL, "out is not device memory");
  hipStream_t s = reinterpret_cast<hipStream_t>(opts.stream);

  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  ZSET_HIP(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  if ((st = noalloc_scratch(dev, &base)) != ZSET_OK) return st;
  Carve cv{base, size_t(ZSET_NOALLOC_SCRATCH_BYTES), 0};
  const uint64_t N = n + 1;
  uint64_t* misc = cv.take<uint64_t>(kMiscWords * sizeof(uint64_t));
  const size_t table_bytes = size_t(d + 1) * N * sizeof(uint64_t);
  uint64_t* T = cv.take<uint64_t>(table_bytes);
  if (!misc || !T) return scratch_full("count table", table_bytes);
  int* err = reinterpret_cast<int*>(misc + kMiscErr);

  // 1. Status words cleared (a kernel: the array keeps the last call's
  // contents), count table, one readback of the row sums and |Z(n)|.
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(256), 0, s, misc, uint32_t(kMiscWords));
  ZSET_HIP(hipGetLastError());
  ZSET_HIP(launch_count_table(T, n, gens, d, misc + kMiscRowSums, s));
  uint64_t host[2 * kMaxD + 3];
  ZSET_HIP(hipMemcpyAsync(host, misc + kMiscRowSums, (2 * d + 3) * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
  ZSET_HIP(hipStreamSynchronize(s));
  uint64_t sums[kMaxD + 1], rowmax[kMaxD + 1];
  for (int j = 0; j <= d; ++j) {
    sums[j] = host[j];
    rowmax[j] = host[d + 2 + j];
  }
  const uint64_t total = host[d + 1];
  if (total == ~uint64_t(0)) return fail(ZSET_EOVERFLOW, "|Z(n)| >= 2^64 - 1");
  if (total > (~uint64_t(0)) / (4 * uint64_t(d)))
    return fail(ZSET_EOVERFLOW, "|Z(n)| * d * 4 bytes overflows 64 bits");
  if (!count_only && total > out_rows_cap)
    return fail(ZSET_ECAPACITY, "out holds " + std::to_string(out_rows_cap) + " rows, |Z(n)| = " +
                                    std::to_string(total));

  // 2. Memo dimension, descriptor, scratch pieces, then the same launches as
  // zset_enumerate_ex in one stream order.
  int k = opts.k;
  if (d == 1) k = 0;
  else if (k < 0) k = auto_memo_dim(sums, d, total);
  if (total > 0 && d == 1) {
    ZSET_HIP(launch_single(n, gens[0], out, count_only, misc + kMiscSum, s));
  } else if (total > 0) {
    const int L = d - std::max(k, 1);
    const int U = (k == 0) ? d - 1 : L - 1;
    const uint32_t G = gens[U];
    EnumParams P;
    const uint64_t leaf_words = init_params(P, n, gens, d, k, total, sums, T, err,
                                            misc + kMiscSum, out, size_t(write_lds_budget(dev)));
    P.desc = opts.order == 1 && !count_only;
    const uint64_t Rn = k >= 1 ? sums[L] : 0;
    if (k >= 1) {
      const size_t eb = size_t(std::min<uint64_t>(G, N)) * sizeof(uint64_t);
      P.endc = cv.take<uint64_t>(eb);
      if (!P.endc) return scratch_full("class ends", eb);
      const size_t lb = size_t(leaf_words) * sizeof(uint32_t);
      P.leaf = cv.take<uint32_t>(lb);
      if (!P.leaf) return scratch_full("leaf-order memo", lb);
    }
    const bool align16 = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    P.pool = reinterpret_cast<uint32_t*>(misc + kMiscPool);
    if ((st = size_write_pass(P, opts.rows_per_tile, opts.claim_pct, dev, count_only, align16)) !=
        ZSET_OK)
      return st;
    const size_t tb = size_t(P.ntiles) * (U + 2) * sizeof(uint32_t);
    P.tiles = cv.take<uint32_t>(tb);
    if (!P.tiles) return scratch_full("slice table", tb);
    if (k >= 1) {
      uint32_t nclass = 0;
      ZSET_HIP(launch_class_ends(T + uint64_t(U) * N, n, G, const_cast<uint64_t*>(P.endc),
                                 &nclass, s));
    }
    ZSET_HIP(launch_plan(P, s));
    if (k >= 1) {
      const size_t ob = size_t(N + 1) * sizeof(uint64_t);
      uint64_t* off = cv.take<uint64_t>(ob);
      if (!off) return scratch_full("memo offsets", ob);
      const size_t nb = size_t(Rn) * k * sizeof(uint32_t);
      uint32_t* nat = cv.take<uint32_t>(nb);
      if (!nat) return scratch_full("memo rows", nb);
      if (k == 2 && memo2_closed_form()) {
        uint64_t* cnt = cv.take<uint64_t>(ob);
        if (!cnt) return scratch_full("memo counts", ob);
        ZSET_HIP(launch_memo_k2(gens[L], gens[L + 1], N, Rn, nat, off, cnt, s));
      } else {
        auto srcw_for = [&cv](size_t bytes, uint64_t** p) {
          *p = cv.take<uint64_t>(bytes);
          return *p ? ZSET_OK : scratch_full("memo source table", bytes);
        };
        st = build_memo_rows(gens + L, k, N, off, T + uint64_t(L) * N, N, Rn, rowmax[L], nat, err,
                             size_t(device_max_lds_bytes(dev)), srcw_for, s);
        if (st != ZSET_OK) return st;
      }
      ZSET_HIP(launch_memo_leaf(make_leaf_job(k, n, G, off, nat, T + uint64_t(U) * N, P.endc,
                                              const_cast<uint32_t*>(P.leaf), Rn, P),
                                err, s));
    }
    ZSET_HIP(launch_write(P, count_only, align16, s));
  }

  uint64_t fin[2] = {0, 0};
  ZSET_HIP(hipMemcpyAsync(fin, misc, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  ZSET_HIP(hipStreamSynchronize(s));
  const int code = int(uint32_t(fin[0]));
  if (code != 0) return fail(ZSET_EDEVICE, device_error_text(code));
  if (rows_written) *rows_written = total;
  if (checksum) *checksum = count_only ? fin[1] : 0;
  return ZSET_OK;
}

zset_status zset_selftest_host(void) {
  g_last_error.clear();
  // Division by invariant divisors: spot values around powers of two and
  // a deterministic pseudo-random sweep.
  uint64_t state = 0x9e3779b97f4a7c15ull;
  auto next = [&]() {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
  };
  uint32_t divisors[64];
  int nd = 0;
  for (uint32_t v : {1u, 2u, 3u, 5u, 7u, 10u, 13u, 37u, 64u, 100u, 641u, 65535u, 65536u,
                     65537u, 2147483647u, 2147483648u, 4294967295u})
    divisors[nd++] = v;
  while (nd < 64) divisors[nd++] = uint32_t(next() >> (next() % 32)) | 1u;
  for (int i = 0; i < nd; ++i) {
    const DivMod32 dm = DivMod32::make(divisors[i]);
    for (int t = 0; t < 20000; ++t) {
      uint32_t x;
      switch (t % 4) {
        case 0: x = uint32_t(next()); break;
        case 1: x = uint32_t(next() % 100000); break;
        case 2: x = 4294967295u - uint32_t(next() % 1000); break;
        default: x = divisors[i] * uint32_t(next() % 1000) + uint32_t(t % 3); break;
      }
      const uint32_t q = dm.div(x);
      if (q != x / divisors[i] || dm.mod(x, q) != x % divisors[i]) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "DivMod32 wrong for %u / %u: got %u", x, divisors[i], q);
        return fail(ZSET_EDEVICE, buf);
      }
    }
  }
  // The count table's closed-form last rows against direct counts:
  // [h_2 divides x] and |Z(x; h_1, h_2)| = #{m_1 : m_1 h_1 <= x, h_2 divides x - m_1 h_1}.
  const uint32_t pairs[][2] = {{1, 1},   {1, 3},    {3, 1},      {6, 4},     {4, 6},
                               {7, 7},   {13, 83},  {65, 83},    {10, 15},   {12, 18},
                               {2, 70000}, {600, 7}, {65535, 2}, {1, 65535}, {30, 65536}};
  for (const auto& hp : pairs) {
    const uint32_t g2[2] = {hp[0], hp[1]};
    const LastRows L = make_last_rows(g2, 2);
    if (!L.on) return fail(ZSET_EDEVICE, "closed-form rows refused a pair below the bound");
    for (uint32_t x = 0; x < 3000; x += (x < 600 ? 1 : 7)) {
      uint32_t want = 0;
      for (uint64_t m1 = 0; m1 * hp[0] <= x; ++m1) want += ((x - m1 * hp[0]) % hp[1] == 0);
      if (last_row_pair(L, x) != want || last_row_divides(L, x) != (x % hp[1] == 0 ? 1u : 0u)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "closed-form count rows wrong for x = %u, g = (%u, %u)", x,
                      hp[0], hp[1]);
        return fail(ZSET_EDEVICE, buf);
      }
    }
  }
  const uint32_t big[2] = {3, 70001};  // h_2 / gcd >= 2^16: scanned instead
  if (make_last_rows(big, 2).on) return fail(ZSET_EDEVICE, "closed-form rows beyond their bound");
  return ZSET_OK;
}

}  // extern "C"
