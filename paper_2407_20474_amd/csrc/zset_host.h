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
uint32_t next_pow2(uint32_t v);
float elapsed_us(hipEvent_t a, hipEvent_t b);

}  // namespace zset

#define ZSET_HIP(call)                                     \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::zset::hip_fail(e_, #call); \
  } while (0)
