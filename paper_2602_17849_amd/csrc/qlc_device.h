// Device-side building blocks of libqlc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "qlc_internal.h"

namespace qlc {

// ---------------------------------------------------------------------------
// Candidate width tuples of the layout search (compile-time table).
// Non-decreasing 8-tuples over 0..8 whose greedy fill leaves every area
// non-empty (the first seven areas hold fewer than 256 ranks) and covers all
// 256 ranks.  Entries with at most four distinct widths come first (the
// quad search reads only those), each part in lexicographic order; `lex` is
// the tuple's position in the full lexicographic order (the tie-break) in
// its low 16 bits and the number of distinct widths above them.
// Widths are packed as 4-bit nibbles; `ends` holds the greedy fill's end
// rank of areas 0..6, one byte each (area 7 ends at 256).
// ---------------------------------------------------------------------------
constexpr int kNumCandidates = 3639;
constexpr int kNumQuadCandidates = 1308;

struct Candidate {
  uint32_t packed;
  uint32_t lex;
  uint64_t ends;
  uint64_t steps;  // the width increases (make_steps)
};

// The width increases of a candidate, for its layout cost in the form
//   (area-code bits + last width) * N - sum_j d_j * P[e_j]
// (Abel summation of sum_a w_a * count_a: widths never decrease, P[r] is
// the count of the ranks below r, e_j the end rank of the area before the
// j-th increase and d_j its size).  Up to three increases, in bits
// 13j..13j+12 (e_j: 9 bits, d_j: 4 bits); bit 63 when there are more (the
// cost is then summed area by area).
constexpr uint64_t make_steps(const int* w, int na, uint64_t ends) {
  uint64_t st = 0;
  int k = 0;
  for (int a = 0; a + 1 < na; ++a) {
    const int d = w[a + 1] - w[a];
    if (d <= 0) continue;
    if (k == 3) return 1ull << 63;
    const uint64_t e = (ends >> (8 * a)) & 0xFFu;
    st |= (e | (uint64_t(d) << 9)) << (13 * k);
    ++k;
  }
  return st;
}

struct CandidateTable {
  Candidate c[kNumCandidates];
  int count, quad;
};

constexpr CandidateTable make_candidate_table() {
  CandidateTable t{};
  int w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int n = 0, nq = 0;
  // two passes over the lexicographic order: quad tuples, then the others
  for (int pass = 0; pass < 2; ++pass) {
    for (int a = 0; a < 8; ++a) w[a] = 0;
    int lex = 0;
    while (true) {
      uint32_t head = 0;
      for (int a = 0; a < 7; ++a) head += 1u << w[a];
      if (head < 256 && head + (1u << w[7]) >= 256) {
        uint32_t pk = 0;
        uint64_t ends = 0;
        uint32_t f = 0;
        int d = 1;
        for (int a = 0; a < 8; ++a) {
          pk |= uint32_t(w[a]) << (4 * a);
          if (a > 0 && w[a] != w[a - 1]) ++d;
          f += 1u << w[a];
          if (a < 7) ends |= uint64_t(f) << (8 * a);
        }
        if ((d <= 4) == (pass == 0)) {
          if (n < kNumCandidates)
            t.c[n] = Candidate{pk, uint32_t(lex) | (uint32_t(d) << 16), ends, make_steps(w, 8, ends)};
          ++n;
          if (pass == 0) ++nq;
        }
        ++lex;
      }
      int pos = 7;
      while (pos >= 0 && w[pos] == 8) --pos;
      if (pos < 0) break;
      ++w[pos];
      for (int a = pos + 1; a < 8; ++a) w[a] = w[pos];
    }
  }
  t.count = n;
  t.quad = nq;
  return t;
}

// Candidates of the 4-area layout (2-bit area code): non-decreasing
// 4-tuples over 0..8 whose greedy fill leaves every area non-empty and
// covers 256 ranks, in lexicographic order; widths in nibbles 0..3 (the
// others 0xF), `ends` holds the end rank of areas 0..2.
constexpr int kNumCandidates4 = 147;

struct CandidateTable4 {
  Candidate c[kNumCandidates4];
  int count;
};

constexpr CandidateTable4 make_candidate_table4() {
  CandidateTable4 t{};
  int w[4] = {0, 0, 0, 0};
  int n = 0;
  while (true) {
    uint32_t head = 0;
    for (int a = 0; a < 3; ++a) head += 1u << w[a];
    if (head < 256 && head + (1u << w[3]) >= 256) {
      uint32_t pk = 0xFFFF0000u, f = 0;
      uint64_t ends = 0;
      for (int a = 0; a < 4; ++a) {
        pk |= uint32_t(w[a]) << (4 * a);
        f += 1u << w[a];
        if (a < 3) ends |= uint64_t(f) << (8 * a);
      }
      if (n < kNumCandidates4) t.c[n] = Candidate{pk, uint32_t(n), ends, make_steps(w, 4, ends)};
      ++n;
    }
    int pos = 3;
    while (pos >= 0 && w[pos] == 8) --pos;
    if (pos < 0) break;
    ++w[pos];
    for (int a = pos + 1; a < 4; ++a) w[a] = w[pos];
  }
  t.count = n;
  return t;
}

// Candidates of the small-alphabet layouts: M symbols (16 or 64), A areas
// (2, 4 or 8), non-decreasing A-tuples over 0..log2(M) whose greedy fill
// leaves every area non-empty and covers the M ranks, in lexicographic
// order (the index is the tie-break); widths in nibbles 0..A-1 (the others
// 0xF), `ends` holds the end rank of areas 0..A-2.
template <int kMax>
struct SmallCandidateTable {
  Candidate c[kMax];
  int count;
};

template <int kM, int kA, int kMax>
constexpr SmallCandidateTable<kMax> make_small_candidates() {
  SmallCandidateTable<kMax> t{};
  int maxw = 0;
  while ((1 << maxw) < kM) ++maxw;
  int w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int n = 0;
  while (true) {
    uint32_t head = 0;
    for (int a = 0; a < kA - 1; ++a) head += 1u << w[a];
    if (head < (uint32_t)kM && head + (1u << w[kA - 1]) >= (uint32_t)kM) {
      uint32_t pk = 0xFFFFFFFFu, f = 0;
      uint64_t ends = 0;
      for (int a = 0; a < kA; ++a) {
        pk = (pk & ~(0xFu << (4 * a))) | (uint32_t(w[a]) << (4 * a));
        f += 1u << w[a];
        if (a < kA - 1) ends |= uint64_t(f) << (8 * a);
      }
      if (n < kMax) t.c[n] = Candidate{pk, uint32_t(n), ends, make_steps(w, kA, ends)};
      ++n;
    }
    int pos = kA - 1;
    while (pos >= 0 && w[pos] == maxw) --pos;
    if (pos < 0) break;
    ++w[pos];
    for (int a = pos + 1; a < kA; ++a) w[a] = w[pos];
  }
  t.count = n;
  return t;
}

// Widths of the two printed schemes (Table 1 and Table 2, "#Symbol bits").
constexpr uint32_t kPaperT1Packed = 0x85433333u;  // 3,3,3,3,3,4,5,8
constexpr uint32_t kPaperT2Packed = 0x85533331u;  // 1,3,3,3,3,5,5,8

// ---------------------------------------------------------------------------
// Wave64 helpers
// ---------------------------------------------------------------------------
// 64-bit wave operations with DPP (the two halves moved by the same DPP
// pattern): no LDS round trips, unlike lane shuffles (ds_bpermute).  Lanes
// with no source lane in a step take `old` (0 for sums, their own value for
// minima); row_bcast steps write only the rows their mask names.
#define QLC_DPP_U64(OLD, V, CTRL, ROWS)                                                   \
  ((uint64_t)(uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(OLD),                  \
                                                   (int)(uint32_t)(V), CTRL, ROWS, 0xf,     \
                                                   false) |                                 \
   ((uint64_t)(uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)((OLD) >> 32),         \
                                                    (int)(uint32_t)((V) >> 32), CTRL, ROWS, \
                                                    0xf, false)                             \
    << 32))

// Inclusive wave64 scan: Hillis-Steele inside each 16-lane row (row_shr 1,
// 2, 4, 8), then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then rows 0-1's total into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint64_t wave_inclusive_scan_u64(uint64_t v) {
  v += QLC_DPP_U64(0ull, v, 0x111, 0xf);  // row_shr:1
  v += QLC_DPP_U64(0ull, v, 0x112, 0xf);  // row_shr:2
  v += QLC_DPP_U64(0ull, v, 0x114, 0xf);  // row_shr:4
  v += QLC_DPP_U64(0ull, v, 0x118, 0xf);  // row_shr:8
  v += QLC_DPP_U64(0ull, v, 0x142, 0xa);  // row_bcast:15
  v += QLC_DPP_U64(0ull, v, 0x143, 0xc);  // row_bcast:31
  return v;
}

// Inclusive wave64 scan with DPP: a Hillis-Steele scan inside each 16-lane
// row (row_shr 1, 2, 4, 8; lanes shifted in from outside the row add 0),
// then row 0's total into row 1 and row 2's into row 3 (row_bcast:15), then
// rows 0-1's total into rows 2 and 3 (row_bcast:31).  No LDS round trips.
__device__ __forceinline__ uint32_t wave_inclusive_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Lane 63's value, in every lane.
__device__ __forceinline__ uint64_t lane63_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Sum over the wave, in every lane (the scan's lane 63).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  return lane63_u64(wave_inclusive_scan_u64(v));
}

// Minimum over the wave, in every lane (a prefix-minimum scan's lane 63).
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  uint64_t t;
  t = QLC_DPP_U64(v, v, 0x111, 0xf);
  v = t < v ? t : v;
  t = QLC_DPP_U64(v, v, 0x112, 0xf);
  v = t < v ? t : v;
  t = QLC_DPP_U64(v, v, 0x114, 0xf);
  v = t < v ? t : v;
  t = QLC_DPP_U64(v, v, 0x118, 0xf);
  v = t < v ? t : v;
  t = QLC_DPP_U64(v, v, 0x142, 0xa);
  v = t < v ? t : v;
  t = QLC_DPP_U64(v, v, 0x143, 0xc);
  v = t < v ? t : v;
  return lane63_u64(v);
}

// ---------------------------------------------------------------------------
// Device-scope atomics on the workspace (visible across the 8 XCD L2s).
// ---------------------------------------------------------------------------
// Only relaxed (monotonic) device-scope atomics are used across
// workgroups: on gfx950 they are coherent loads/stores (sc1) and RMWs,
// whereas acquire/release fences at device scope write back and invalidate
// the whole L2 of the XCD.  Cross-workgroup messages therefore carry their
// own validity tag (a launch epoch) instead of relying on release ordering.
__device__ __forceinline__ void store_relaxed_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_add_u32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_relaxed_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_relaxed_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// First error wins.  Returns after the CAS has been performed.
__device__ __forceinline__ void set_error(uint32_t* slot, uint32_t code) {
  uint32_t expected = 0;
  __hip_atomic_compare_exchange_strong(slot, &expected, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);
}

// set_error for a wave: one atomic from the first lane with `bad` set, and
// none once the slot already holds an error (keeps a corrupt input from
// serialising every lane on one address).
__device__ __forceinline__ void set_error_wave(uint32_t* slot, uint32_t code, bool bad) {
  const uint64_t m = __ballot(bad);
  if (m == 0) return;
  if ((threadIdx.x & 63) == (uint32_t)__builtin_ctzll(m) && load_relaxed_u32(slot) == 0)
    set_error(slot, code);
}

// 32 bits of the concatenation hi:lo starting r bits below the top of hi.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t r) {
  return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (32 - r));
}

}  // namespace qlc
