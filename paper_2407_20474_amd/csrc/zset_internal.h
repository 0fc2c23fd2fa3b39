// zset_internal.h -- declarations shared by the kernel files and the host
// library of libzset.so.  Not part of the public ABI (include/zset.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "zset_common.h"

namespace zset {

// Everything the slice planner and the write pass read.
struct EnumParams {
  Gens g;                   // generators g_0..g_{d-1}, caller order
  uint32_t n;               // element
  int d;                    // dimension
  int U;                    // coordinates fixed by a slice start
  int k;                    // memo dimension (0: last coordinate by division)
  uint64_t total;           // |Z(n)|
  uint64_t rows_per_tile;   // rows per slice (multiple of 128)
  uint64_t ntiles;          // slices
  const uint64_t* table;    // count table, (d+1) x (n+1)
  const uint64_t* endc;     // residue-class ends of the leaf-order memo (k >= 1)
  const uint32_t* leaf;     // leaf-order memo rows, k+1 uint32 each (k >= 1)
  uint64_t leaf_rows;       // rows in `leaf`
  uint32_t* tiles;          // slice starts, U+2 uint32 each
  uint32_t* out;            // rows, d uint32 each
  uint64_t* checksum;       // count-only: wrapping sum of row hashes
  int* err;                 // device status word
  DivMod32 dG;              // division by g_U
  uint32_t ring;            // rows in each wavefront's LDS staging ring (power of two)
  uint32_t flush;           // rows per coalesced flush (ring / 2)
  int pack;                 // memo row format: 0 plain words in global, 1 / 2 packed
                            // 32- / 64-bit words copied into LDS
  uint64_t memo_words;      // uint32 words of packed memo copied into LDS (0 if pack == 0)
  uint32_t fshift[kMaxD + 1];  // packed field c (0 = floor(p / G), c >= 1 = m_c): bit offset
  uint32_t fmask[kMaxD + 1];   // and mask
  int lds_cnt;              // 1: segment counts C[U][x] and class ends copied to LDS as uint32
  uint32_t nclass;          // residue classes of the leaf layout: min(G, n + 1)
  uint32_t max_tiles;       // slices one workgroup may own (their starts are held in LDS)
  uint32_t write_blocks;    // workgroups of the write pass; slice t goes to workgroup t mod NB
};

// count_table.hip
// Count table (d+1) x (n+1); when sums is non-NULL also sums[j] = sum_x C[j][x].
hipError_t launch_count_table(uint64_t* table, uint64_t n, const uint32_t* gens, int d,
                              uint64_t* sums, hipStream_t s);

// scan.hip
hipError_t launch_exclusive_scan(const uint64_t* in, uint64_t count, uint64_t* out,
                                 hipStream_t s);
hipError_t launch_class_ends(const uint64_t* count_row_u, uint64_t n, uint32_t G,
                             uint64_t* endc, uint32_t* nclass_out, hipStream_t s);

// memo.hip
size_t memo_wave_lds_bytes(int k, uint64_t R, uint32_t W);
hipError_t launch_memo_chain_wave(const uint32_t* h, int k, uint64_t top, uint32_t step,
                                  uint32_t W, uint64_t R, uint32_t* nat, uint64_t* off_out,
                                  int* err, hipStream_t s);
hipError_t launch_memo_global(const uint32_t* h, int k, uint64_t top, uint32_t b,
                              const uint64_t* off, const uint64_t* ge, uint64_t ge_stride,
                              uint64_t* srcw, uint32_t* nat, int* err, hipStream_t s);
hipError_t launch_memo_leaf(int k, uint64_t n, uint32_t G, const uint64_t* off,
                            const uint32_t* nat, const uint64_t* cu, const uint64_t* endc,
                            uint32_t* leaf, uint64_t leaf_rows, const EnumParams& P, int* err,
                            hipStream_t s);

// enumerate.hip
size_t write_lds_bytes(const EnumParams& P);
int write_waves_per_block();
hipError_t write_occupancy(const EnumParams& P, bool count_only, bool align16, int* per_cu);
hipError_t launch_plan(const EnumParams& P, hipStream_t s);
hipError_t launch_write(const EnumParams& P, bool count_only, bool align16, hipStream_t s);
hipError_t launch_single(uint64_t n, uint32_t g, uint32_t* out, bool count_only,
                         uint64_t* checksum, hipStream_t s);
hipError_t launch_reverse(uint32_t* out, uint64_t rows, int d, hipStream_t s);

}  // namespace zset
