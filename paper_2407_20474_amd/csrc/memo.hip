// memo.hip -- the memo of the trailing generators (paper, Section 3.1) and
// its leaf-order layout.
//
// Memo[p] = Z(p; h_1..h_k) for p in [0, top), every list ascending.  It is
// built by the disjoint recurrence of Lemma 2.3 read in ascending order
// (Lemma 2.6 mirrored): Z_{>=i}(m) is a prefix of the ascending list Z(m), so
//
//   Memo[p] = incr_k(first |Z_{>=k}(p-h_k)| rows of Memo[p-h_k])
//           ++ ... ++
//             incr_1(first |Z_{>=1}(p-h_1)| rows of Memo[p-h_1])
//
// with |Z_{>=i}(m)| = sum_{i' >= i} |Z_{=i'}(m)| and |Z_{=i}(m)| =
// |Z_{>=i}(m - h_i)| (Section 2.3).  Elements are processed in batches of
// b = min(h) consecutive values, which never depend on each other (Section
// 2.2, elementwise parallelism); inside a batch every copied row is its own
// work item (factorizationwise parallelism, Alg 2.9).
//
// Two schedules compute the same natural-order memo:
//  * k_memo_chain_lds: one workgroup keeps the whole memo in LDS and saves the
//    cardinalities |Z_{>=i}(p)| as it goes (Section 2.3), in a ring of the
//    last W elements, so a batch costs a few LDS round trips.
//  * k_memo_src + k_memo_batch: for memos larger than LDS, every destination
//    row's source is precomputed in parallel from the count table, then one
//    multi-workgroup launch per batch copies rows in global memory.
//
// k_memo_leaf rewrites the natural-order memo into the leaf order used by the
// write pass (see enumerate.hip): for a generator G just left of the memo
// coordinates, the elements p <= n are grouped by residue class rho = p mod G,
// each class by descending p.  Then for any x <= n the rows of
// Z(x; G, h) = {(a, m) : m in Memo[x - a G]} are one contiguous run that
// starts at end[x mod G] - |Z(x; G, h)|, in ascending lex order, and each
// memo row carries floor(p / G) so that a = floor(x / G) - floor(p / G).
#include "zset_internal.h"

namespace zset {

namespace {

constexpr int kChainThreads = 1024;

__device__ inline uint32_t block_exclusive_scan_u32(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += y;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int nw = kChainThreads / kWave;
    uint32_t w = lane < nw ? wsum[lane] : 0;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(w, off, kWave);
      if (lane >= off) w += y;
    }
    if (lane < nw) wsum[lane] = w;
  }
  __syncthreads();
  const uint32_t before = wave ? wsum[wave - 1] : 0;
  *total = wsum[kChainThreads / kWave - 1];
  __syncthreads();
  return before + incl - v;
}

// Whole memo in LDS.  Dynamic LDS layout (uint32): M[R*k] | GE[W*k] | OFF[W] | S[b*k].
// Requires b <= kChainThreads, W a power of two >= max(h) + b, and
// R*k + W*(k+1) + b*k words of LDS.
__global__ __launch_bounds__(kChainThreads) void k_memo_chain_lds(Gens h, int k, uint32_t top,
                                                                  uint32_t b, uint32_t W,
                                                                  uint32_t R,
                                                                  uint32_t* __restrict__ nat,
                                                                  int* __restrict__ err) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t wsum[kChainThreads / kWave];
  uint32_t* M = lds;
  uint32_t* GE = M + size_t(R) * k;
  uint32_t* OFF = GE + size_t(W) * k;
  uint32_t* S = OFF + W;
  const int tid = threadIdx.x;

  // Z(0) = [0]: one all-zero row, and |Z_{>=i}(0)| = 1 for every i.
  if (tid < k) {
    M[tid] = 0;
    GE[tid] = 1;
  }
  if (tid == 0) OFF[0] = 0;
  uint32_t running = 1;
  __syncthreads();

  for (uint32_t x0 = 1; x0 < top; x0 += b) {
    const uint32_t nb = (top - x0 < b) ? top - x0 : b;
    // Phase A: block sizes |Z_{=i}(p)| = |Z_{>=i}(p - h_i)| and the saved
    // cardinalities |Z_{>=i}(p)| (suffix sums over i).
    uint32_t size = 0;
    uint32_t p = x0 + tid;
    if (uint32_t(tid) < nb) {
      uint32_t acc = 0;
      for (int i = k - 1; i >= 0; --i) {
        const uint32_t s = (p >= h.g[i]) ? GE[((p - h.g[i]) & (W - 1)) * k + i] : 0;
        S[tid * k + i] = s;
        acc += s;
        GE[(p & (W - 1)) * k + i] = acc;
      }
      size = acc;
    }
    uint32_t total = 0;
    const uint32_t excl = block_exclusive_scan_u32(size, wsum, &total);
    if (uint32_t(tid) < nb) OFF[p & (W - 1)] = running + excl;
    __syncthreads();
    // Phase B: one work item per (element, block); copy-and-increment.
    for (uint32_t pair = tid; pair < nb * uint32_t(k); pair += kChainThreads) {
      const uint32_t t = pair / k;
      const int i = int(pair % k);
      const uint32_t s = S[t * k + i];
      if (s == 0) continue;
      const uint32_t pp = x0 + t;
      const uint32_t src = OFF[(pp - h.g[i]) & (W - 1)];
      uint32_t dst = OFF[pp & (W - 1)];
      for (int i2 = k - 1; i2 > i; --i2) dst += S[t * k + i2];
      for (uint32_t r = 0; r < s; ++r) {
        for (int c = 0; c < k; ++c)
          M[(dst + r) * k + c] = M[(src + r) * k + c] + (c == i ? 1u : 0u);
      }
    }
    running += total;
    __syncthreads();
  }
  if (tid == 0 && running != R) set_error(err, kErrMemoTotal);
  for (uint32_t w = tid; w < R * uint32_t(k); w += kChainThreads) nat[w] = M[w];
}

// Sources of every destination row, from the count table.  Row j of Memo[p]
// (p >= 1) in block i at position t is incr_i of row off[p - h_i] + t.
// srcw[j] = (source row << 5) | i.  ge_i(m) = |Z(m; h_i..h_k)| = ge[i * ge_stride + m].
__global__ __launch_bounds__(256) void k_memo_src(Gens h, int k, uint32_t top,
                                                  const uint64_t* __restrict__ off,
                                                  const uint64_t* __restrict__ ge,
                                                  uint64_t ge_stride,
                                                  uint64_t* __restrict__ srcw,
                                                  uint32_t* __restrict__ nat,
                                                  int* __restrict__ err) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= top) return;
  if (p == 0) {
    for (int c = 0; c < k; ++c) nat[c] = 0;
    srcw[0] = ~uint64_t(0);
    return;
  }
  uint64_t o = off[p];
  for (int i = k - 1; i >= 0; --i) {
    if (p < h.g[i]) continue;
    const uint32_t src = p - h.g[i];
    const uint64_t s = ge[uint64_t(i) * ge_stride + src];
    const uint64_t so = off[src];
    const uint64_t end = off[p + 1];
    if (o + s > end) {  // counts disagree: never write past this element's rows
      set_error(err, kErrMemoTotal);
      return;
    }
    for (uint64_t t = 0; t < s; ++t) srcw[o++] = ((so + t) << 5) | uint64_t(i);
  }
  if (o != off[p + 1]) set_error(err, kErrMemoTotal);
}

// One batch of copies: rows [off[x0], off[x1]).
__global__ __launch_bounds__(256) void k_memo_batch(int k, const uint64_t* __restrict__ off,
                                                    uint32_t x0, uint32_t x1,
                                                    const uint64_t* __restrict__ srcw,
                                                    uint32_t* __restrict__ nat) {
  const uint64_t lo = off[x0], hi = off[x1];
  for (uint64_t j = lo + uint64_t(blockIdx.x) * 256 + threadIdx.x; j < hi;
       j += uint64_t(gridDim.x) * 256) {
    const uint64_t w = srcw[j];
    const uint64_t src = w >> 5;
    const int i = int(w & 31);
    if (src >= j) continue;  // sources always precede their copies
    for (int c = 0; c < k; ++c)
      nat[j * k + c] = nat[src * k + c] + (c == i ? 1u : 0u);
  }
}

// Natural order -> leaf order for p in [0, n]: row t of Memo[p] goes to
// pos(p) + t with pos(p) = end[p mod G] - cu[p]; it is stored as the fields
// (floor(p / G), m_1..m_k): k+1 plain words (pack 0), or packed into one 32-
// or 64-bit word at the bit offsets of the write pass (pack 1, 2).
__global__ __launch_bounds__(256) void k_memo_leaf(int k, uint32_t n, DivMod32 dG,
                                                   const uint64_t* __restrict__ off,
                                                   const uint32_t* __restrict__ nat,
                                                   const uint64_t* __restrict__ cu,
                                                   const uint64_t* __restrict__ endc,
                                                   uint32_t* __restrict__ leaf,
                                                   uint64_t leaf_rows, EnumParams P,
                                                   int* __restrict__ err) {
  const uint64_t p64 = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p64 > n) return;
  const uint32_t p = uint32_t(p64);
  const uint32_t q = dG.div(p);
  const uint32_t rho = dG.mod(p, q);
  const uint64_t pos = endc[rho] - cu[p];
  const uint64_t o = off[p];
  const uint64_t cnt = off[p + 1] - o;
  if (pos > leaf_rows || cnt > leaf_rows - pos) {
    set_error(err, kErrMemoTotal);
    return;
  }
  for (uint64_t t = 0; t < cnt; ++t) {
    const uint32_t* src = nat + (o + t) * k;
    if (P.pack == 0) {
      uint32_t* dst = leaf + (pos + t) * (k + 1);
      dst[0] = q;
      for (int c = 0; c < k; ++c) dst[1 + c] = src[c];
    } else {
      uint64_t w = uint64_t(q) << P.fshift[0];
      for (int c = 0; c < k; ++c) w |= uint64_t(src[c]) << P.fshift[1 + c];
      if (P.pack == 1) leaf[pos + t] = uint32_t(w);
      else reinterpret_cast<uint64_t*>(leaf)[pos + t] = w;
    }
  }
}

}  // namespace

size_t memo_chain_lds_bytes(int k, uint64_t R, uint32_t W, uint32_t b) {
  return (size_t(R) * k + size_t(W) * (k + 1) + size_t(b) * k) * sizeof(uint32_t);
}

hipError_t launch_memo_chain_lds(const uint32_t* h, int k, uint64_t top, uint32_t b, uint32_t W,
                                 uint64_t R, uint32_t* nat, int* err, hipStream_t s) {
  Gens hg{};
  for (int i = 0; i < k; ++i) hg.g[i] = h[i];
  const size_t lds = memo_chain_lds_bytes(k, R, W, b);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_memo_chain_lds),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_memo_chain_lds, dim3(1), dim3(kChainThreads), lds, s, hg, k,
                     uint32_t(top), b, W, uint32_t(R), nat, err);
  return hipGetLastError();
}

hipError_t launch_memo_global(const uint32_t* h, int k, uint64_t top, uint32_t b,
                              const uint64_t* off, const uint64_t* ge, uint64_t ge_stride,
                              uint64_t* srcw, uint32_t* nat, int* err, hipStream_t s) {
  Gens hg{};
  for (int i = 0; i < k; ++i) hg.g[i] = h[i];
  const uint32_t blocks = uint32_t((top + 255) / 256);
  hipLaunchKernelGGL(k_memo_src, dim3(blocks), dim3(256), 0, s, hg, k, uint32_t(top), off, ge,
                     ge_stride, srcw, nat, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (uint64_t x0 = 1; x0 < top; x0 += b) {
    const uint64_t x1 = (x0 + b < top) ? x0 + b : top;
    hipLaunchKernelGGL(k_memo_batch, dim3(1024), dim3(256), 0, s, k, off, uint32_t(x0),
                       uint32_t(x1), srcw, nat);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_memo_leaf(int k, uint64_t n, uint32_t G, const uint64_t* off,
                            const uint32_t* nat, const uint64_t* cu, const uint64_t* endc,
                            uint32_t* leaf, uint64_t leaf_rows, const EnumParams& P, int* err,
                            hipStream_t s) {
  const uint32_t blocks = uint32_t((n + 1 + 255) / 256);
  hipLaunchKernelGGL(k_memo_leaf, dim3(blocks), dim3(256), 0, s, k, uint32_t(n),
                     DivMod32::make(G), off, nat, cu, endc, leaf, leaf_rows, P, err);
  return hipGetLastError();
}

}  // namespace zset
