// zset_host.h -- host-side helpers shared by the C ABI entry points of
// libzset.so (api.hip: single queries and memos; batch.hip: batches).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "zset.h"

namespace zset {

// Element bound: count-table rows have n + 1 entries indexed in 32 bits on
// the device.
constexpr uint64_t kMaxN = (uint64_t(1) << 31) - 2;

extern thread_local std::string g_last_error;
extern std::mutex g_mu;  // serialises the entry points that share scratch memory

zset_status fail(zset_status st, const std::string& msg);
zset_status hip_fail(hipError_t e, const char* what);
bool fault_injected(const char* what);  // ZSET_FAULT=<what> in the environment

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
zset_status ensure(DevBuf& b, size_t bytes);

zset_status check_gens(const uint32_t* gens, int d, const char* what);
zset_status check_query(uint64_t n, const uint32_t* gens, int d);
bool is_device_pointer(const void* p);
const char* device_error_text(int code);
int device_max_lds_bytes(int device);
// Dynamic LDS the write-pass kernels may request: the device's LDS per
// workgroup less a reserve for their static shared variables (a request that
// fills the device's LDS exactly would not leave room for them).
int write_lds_budget(int device);

struct EnumParams;
// Write-pass sizing (slice length, claimed chunks, slice-state capacity, grid)
// and the leaf-order row format; shared by the single-query path and the server.
// share: queries expected on the device at once (the grid gets 1/share of the
// resident workgroups; 1 = the whole device).
// want_tiles: the slice count the slice length is taken for (0: about 128
// slices per resident wavefront of this write pass).
zset_status size_write_pass(EnumParams& P, uint64_t rows_per_tile, int claim_pct, int device,
                            bool count_only, bool align16, int share = 1,
                            uint64_t want_tiles = 0);
// Slices asked for when the planner sizes them on the device before the
// write pass's occupancy is known: 128 per wavefront of one write workgroup
// on every compute unit.
uint64_t plan_want_tiles(int device);
void leaf_format(EnumParams& P, uint64_t n, const uint32_t* gens, int U, int k);
uint32_t next_pow2(uint32_t v);
float elapsed_us(hipEvent_t a, hipEvent_t b);

}  // namespace zset

#define ZSET_HIP(call)                                     \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::zset::hip_fail(e_, #call); \
  } while (0)

// Memo handle (zset_memo): natural-order lists on the device.
struct zset_memo_s {
  int device;
  int k;
  uint64_t top;
  uint64_t rows;
  uint32_t h[ZSET_MAX_D];
  uint64_t* off;  // device, top + 1
  uint32_t* nat;  // device, rows * k
};

