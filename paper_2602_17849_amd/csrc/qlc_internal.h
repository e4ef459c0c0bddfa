// Internal layout shared by the libqlc host code and kernels (not installed).
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "qlc.h"

namespace qlc {

// ---- launch geometry ------------------------------------------------------
constexpr int kHistThreads = 512;     // histogram workgroup
constexpr int kHistCopies = 32;       // LDS sub-histograms (one per lane mod 32)
constexpr int kTableThreads = 512;    // table-building workgroup
constexpr int kEncThreads = 256;      // encode workgroup
constexpr int kEncSymsPerThread = 32; // two 16-byte loads per thread
constexpr int kEncTile = kEncThreads * kEncSymsPerThread;  // symbols per tile
#ifndef QLC_DEC_THREADS_LOG2
#define QLC_DEC_THREADS_LOG2 8
#endif
#ifndef QLC_DEC_STAGE_GROUPS
#define QLC_DEC_STAGE_GROUPS 16
#endif
constexpr int kDecThreadsLog2 = QLC_DEC_THREADS_LOG2;
constexpr int kDecThreads = 1 << kDecThreadsLog2;  // decode workgroup: one lane per chunk
constexpr int kStageGroups = QLC_DEC_STAGE_GROUPS;  // decoded groups staged per lane (8 or 16)
static_assert(kStageGroups == 8 || kStageGroups == 16, "stage depth");
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies
// Layout modes: 0..3, SEARCH_DISTINCT_k = 16 + k for k = 1..8, SEARCH_AREAS4 = 32,
// and the small alphabets 48..51 (16 or 64 symbols).
inline bool valid_layout_mode(uint32_t m) {
  return m <= 3u || (m >= 17u && m <= 24u) || m == 32u || (m >= 48u && m <= 51u);
}
// Bits per symbol of the alphabet a layout mode codes: 4 (16 symbols),
// 6 (64 symbols) or 8 (256 symbols).
__host__ __device__ inline uint32_t mode_symbol_bits(uint32_t m) {
  return (m == 48u || m == 49u) ? 4u : (m == 50u || m == 51u) ? 6u : 8u;
}
// Areas of a layout mode (the area code has log2 of that many bits).
__host__ __device__ inline uint32_t mode_areas(uint32_t m) {
  return m == 48u ? 2u : (m == 32u || m == 49u || m == 50u) ? 4u : 8u;
}
inline bool valid_symbol_bits(uint32_t b) { return b == 4u || b == 6u || b == 8u; }
// Bytes holding n symbols of `bits` bits each, packed.
inline uint64_t packed_bytes(uint64_t n, uint32_t bits) { return (n * bits + 7) / 8; }

// ---- histogram kernel outputs ----------------------------------------------
constexpr uint32_t kHistSegment = 1;     // write each segment's histogram
constexpr uint32_t kHistGlobal = 2;      // fold the whole input's histogram
constexpr uint32_t kHistBuildTable = 4;  // ... and build the table from it
constexpr uint32_t kHistAccumulate = 8;  // add the whole input's histogram to hist_out

// ---- epoch-tagged cross-workgroup words -----------------------------------
// [63] valid, [61:40] launch epoch (22 bits), [39:0] value
constexpr uint32_t kEpochMask = (1u << 22) - 1;
constexpr uint64_t kValueMask = (1ull << 40) - 1;

// ---- workspace layout -----------------------------------------------------
struct WsHeader {
  uint32_t hist_done;   // workgroups finished in the histogram kernel
  uint32_t reserved0;   // (unused)
  uint32_t enc_done;    // segments finished in the encode kernel
  uint32_t enc_epoch;   // epoch tag of this encode launch's published words
  uint32_t enc_err;     // first data error of the encode launch
  uint32_t dec_done;    // workgroups finished in the decode kernel
  uint32_t dec_err;     // first data error of the decode launch
  uint32_t pad[57];
};
static_assert(sizeof(WsHeader) == 256, "header size");

constexpr size_t kWsHistOffset = 256;                              // u64[8][256]
constexpr size_t kWsHistBytes = sizeof(uint64_t) * kNumXcd * 256;
constexpr size_t kWsSegOffset = kWsHistOffset + kWsHistBytes;     // u32[nseg][256], u64[nseg]

// Segments: the unit of the histogram and encode grids, a power of two of
// at least one encode tile.  Each encode workgroup sums the bit counts of
// all segments before it, so their number is a trade between that
// quadratic term and filling the device: about sqrt(n) / 16 segments
// (2^(floor(log2 n / 2) + 4) symbols each), at most about 1024.  Measured
// on MI355X (compress of Laplace e4m3, C = 2048): 9 Mi symbols 48 -> 41 us
// against 1024-segment sizing, 16 Mi 66 -> 47 us, 64 Mi 83 -> 80 us;
// 256 Mi unchanged (1024 segments of 2^18).
inline uint32_t seg_log2(uint64_t n) {
  uint32_t l = 13;                                   // 8192 symbols (one tile)
  while (l < 20 && (n >> l) > 1024) ++l;             // ... up to 1 Mi symbols
  uint32_t lg = 0;
  while (lg < 63 && (n >> (lg + 1)) != 0) ++lg;      // floor(log2 n)
  const uint32_t root = lg / 2 + 4;
  if (root > l) l = root < 20 ? root : 20;
  while ((n >> l) > (1ull << 24)) ++l;               // keep the grid bounded
  return l;
}

inline uint64_t seg_count(uint64_t n) {
  const uint32_t l = seg_log2(n);
  const uint64_t s = (n + (1ull << l) - 1) >> l;
  return s ? s : 1;
}

inline size_t ws_bytes_for(uint64_t n) {
  const uint64_t s = seg_count(n);
  const size_t b = kWsSegOffset + s * 256 * sizeof(uint32_t) + s * sizeof(uint64_t);
  return (b + 255) & ~size_t(255);
}

// ---- batched workspace -----------------------------------------------------
// [BatchHeader][BatchJobState x jobs][uint64 hist[256] x jobs][per-unit arrays]
// Units are encode segments (seg_hist u32[256], seg_word u64, seg_job u32
// each) or decode chunk groups (grp_job u32 each).
struct BatchHeader {
  uint32_t ticket;    // next work item of the persistent launch
  uint32_t units;     // segments (encode) or chunk groups (decode) of all jobs
  uint32_t lag;       // encode: histogram items handed out ahead of encode items
  uint32_t abort;     // the plan found the workspace too small
  uint32_t log2_seg;  // encode: segment size the plan chose (or was given)
  uint32_t pad[59];
};
static_assert(sizeof(BatchHeader) == 256, "batch header size");

struct BatchJobState {
  uint32_t base;         // first unit of the job
  uint32_t count;        // units of the job (0: job skipped)
  union {
    uint32_t hist_done;  // encode: histogram items finished
    uint32_t split;      // decode: 1 = split units of 2^14 symbols
  };
  uint32_t table_ready;  // encode: all histograms in (and the table built)
};

constexpr uint32_t kBatchMinLog2Seg = 13;
constexpr uint32_t kBatchMaxLog2Seg = 24;
constexpr uint32_t kBatchAutoMaxLog2Seg = 19;

// Automatic work split of a batched call (tuning field 0), decided by the
// plan kernel from T, the symbols of the call's valid jobs together.
//
// Encode: segments of 2^l symbols, l = floor(log2 T) / 2 + 4 clamped to
// 13..19, i.e. about sqrt(T) / 16 segments.  An encode work item is one
// workgroup streaming its segment tile after tile, so large segments leave
// a small batch to a few workgroups (a 1 Mi-symbol job in 2^18-symbol
// segments: four items, 106 us), and small ones multiply the predecessor
// sums and table waits of a large batch; measured optima on MI355X: 2^13-14
// up to 1 Mi symbols, 2^15 at 4 Mi, 2^16 at 16 Mi, 2^17 at 64 Mi.
__host__ __device__ inline uint32_t batch_auto_log2_seg(uint64_t T) {
  if (T == 0) return kBatchMinLog2Seg;
  const uint32_t lg = 63u - (uint32_t)__builtin_clzll(T);
  const uint32_t l = lg / 2 + 4;
  return l < kBatchMinLog2Seg ? kBatchMinLog2Seg : l > kBatchAutoMaxLog2Seg ? kBatchAutoMaxLog2Seg : l;
}

// Decode (QLC_DECODER_AUTO): every job in split units when a time model of
// the two decoders, fitted to batched decodes on MI355X, favours the split
// one for T symbols at chunk size C = 2^log2c (C <= 16384): split about
// 26 us + 2.5 ps per symbol (two workgroups of 256 lanes per CU on 2^14-
// symbol units), one lane per chunk at least 19.4 us + 44 ns per code of a
// chunk (a lane walks its chunk alone) and 0.46 ps per symbol once the
// device is full.  Otherwise only jobs of fewer chunks than a lane group
// holds are split.
__host__ __device__ inline bool batch_split_all(uint64_t T, uint32_t log2c) {
  if (log2c > 14 || T > (1ull << 40)) return false;
  const uint64_t split_ns = 26000 + T * 25 / 10000;
  const uint64_t lane_fill = 19400 + (44ull << log2c), lane_rate = T * 46 / 100000;
  return split_ns < (lane_fill > lane_rate ? lane_fill : lane_rate);
}

// Segments a call of at most T symbols over n_jobs jobs can need under the
// automatic encode split: sum_j ceil(n_j / 2^l) <= T' / 2^l(T') + n_jobs
// for the T' <= T the plan sees, and T' / 2^l(T') is at most sqrt(T') / 8
// (2^l >= 8 sqrt(T')), at most T' / 2^13, or T' / 2^19 where the cap holds.
inline uint64_t batch_auto_seg_bound(uint64_t T, uint32_t n_jobs) {
  if (T > (1ull << 62)) T = 1ull << 62;
  uint64_t r = (uint64_t)sqrt((double)T);  // floor(sqrt(T)), corrected for rounding
  while (r * r > T) --r;
  while ((r + 1) * (r + 1) <= T) ++r;
  const uint64_t by_root = r / 8 + 1, by_min = (T >> kBatchMinLog2Seg) + 1;
  const uint64_t lo = by_root < by_min ? by_root : by_min;
  const uint64_t by_cap = (T >> kBatchAutoMaxLog2Seg) + 1;
  return (lo > by_cap ? lo : by_cap) + n_jobs;
}
constexpr size_t kBatchSegBytes = 256 * sizeof(uint32_t) + sizeof(uint64_t) + sizeof(uint32_t);
constexpr size_t kBatchGroupBytes = sizeof(uint32_t);

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
inline size_t batch_js_offset() { return sizeof(BatchHeader); }
inline size_t batch_hist_offset(uint32_t jobs) {
  return batch_js_offset() + round256((size_t)jobs * sizeof(BatchJobState));
}
inline size_t batch_units_offset(uint32_t jobs) {
  return batch_hist_offset(jobs) + (size_t)jobs * 256 * sizeof(uint64_t);
}

}  // namespace qlc
