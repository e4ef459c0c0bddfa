// libqlc kernels: histogram, table, encode, decode (gfx950, wave64).
//
// Paper: Quad Length Codes for Lossless Compression of e4m3 (arXiv
// 2602.17849).  Section references are to that paper.
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include "qlc_device.h"
#include "qlc_kernels.h"

namespace qlc {

// Device global memory.  The hot loads and stores of the job buffers go
// through pointers qualified with it: a batched kernel reads a job's
// pointers from the job array, and through such generic pointers the
// compiler would emit flat accesses, which also count against the LDS wait
// counter (every wait for LDS results would then wait for them too).
#define QLC_GLOBAL __attribute__((address_space(1)))
typedef unsigned int GVec4 __attribute__((ext_vector_type(4)));
typedef unsigned int GVec2 __attribute__((ext_vector_type(2)));

// 16-byte element i of a global array, as a uint4.
__device__ __forceinline__ uint4 gload_u4(const QLC_GLOBAL GVec4* p, uint64_t i) {
  const GVec4 v = p[i];
  return make_uint4(v.x, v.y, v.z, v.w);
}

// 8 bytes at an 8-byte aligned global address.
__device__ __forceinline__ void gstore_u2(QLC_GLOBAL uint8_t* p, uint2 v) {
  GVec2 w;
  w.x = v.x;
  w.y = v.y;
  *(QLC_GLOBAL GVec2*)p = w;
}

// ---------------------------------------------------------------------------
// Symbol access by alphabet: 8-bit symbols are bytes; 4-bit symbols are
// packed two per byte (symbol 2k in the low nibble of byte k); 6-bit
// symbols four per three bytes (symbol i in bits 6i .. 6i + 5 of the
// buffer read as a little-endian bit string).  fetch16 returns the 16
// symbols starting at symbol i (a multiple of 16), one per byte.
// ---------------------------------------------------------------------------
template <int kBits>
struct Sym;

template <>
struct Sym<8> {
  static constexpr uint32_t kM = 256;
  typedef uint4 Raw;  // the bytes of 16 symbols as loaded
  __device__ static __forceinline__ Raw load16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return gload_u4((const QLC_GLOBAL GVec4*)in, i >> 4);
  }
  __device__ static __forceinline__ uint4 expand(const Raw& r) { return r; }
  __device__ static __forceinline__ uint4 fetch16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return load16(in, i);
  }
  __device__ static __forceinline__ uint32_t at(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return in[i];
  }
};

// the eight nibbles of w, in order, one per byte of two words
__device__ __forceinline__ uint2 nibbles_to_bytes(uint32_t w) {
  const uint32_t lo = w & 0x0F0F0F0Fu, hi = (w >> 4) & 0x0F0F0F0Fu;
  return make_uint2(__builtin_amdgcn_perm(hi, lo, 0x05010400u),
                    __builtin_amdgcn_perm(hi, lo, 0x07030602u));
}

template <>
struct Sym<4> {
  static constexpr uint32_t kM = 16;
  typedef uint2 Raw;
  __device__ static __forceinline__ Raw load16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    const GVec2 v = *(const QLC_GLOBAL GVec2*)(in + (i >> 1));
    return make_uint2(v.x, v.y);
  }
  __device__ static __forceinline__ uint4 expand(const Raw& r) {
    const uint2 a = nibbles_to_bytes(r.x), b = nibbles_to_bytes(r.y);
    return make_uint4(a.x, a.y, b.x, b.y);
  }
  __device__ static __forceinline__ uint4 fetch16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return expand(load16(in, i));
  }
  __device__ static __forceinline__ uint32_t at(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return (in[i >> 1] >> ((uint32_t)(i & 1) * 4u)) & 15u;
  }
};

// four 6-bit fields of the low 24 bits of x, one per byte
__device__ __forceinline__ uint32_t sixes_to_bytes(uint32_t x) {
  return (x & 0x3Fu) | ((x << 2) & 0x3F00u) | ((x << 4) & 0x3F0000u) | ((x << 6) & 0x3F000000u);
}

template <>
struct Sym<6> {
  static constexpr uint32_t kM = 64;
  typedef uint4 Raw;  // three words used
  __device__ static __forceinline__ Raw load16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    const QLC_GLOBAL uint32_t* p = (const QLC_GLOBAL uint32_t*)(in + (i >> 2) * 3);
    return make_uint4(p[0], p[1], p[2], 0u);
  }
  __device__ static __forceinline__ uint4 expand(const Raw& r) {
    return make_uint4(sixes_to_bytes(r.x), sixes_to_bytes(__builtin_amdgcn_alignbit(r.y, r.x, 24)),
                      sixes_to_bytes(__builtin_amdgcn_alignbit(r.z, r.y, 16)),
                      sixes_to_bytes(r.z >> 8));
  }
  __device__ static __forceinline__ uint4 fetch16(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    return expand(load16(in, i));
  }
  __device__ static __forceinline__ uint32_t at(const QLC_GLOBAL uint8_t* in, uint64_t i) {
    const uint64_t bit = i * 6;
    const uint32_t sh = (uint32_t)(bit & 7);
    uint32_t v = (uint32_t)in[bit >> 3] >> sh;
    if (sh > 2) v |= (uint32_t)in[(bit >> 3) + 1] << (8 - sh);
    return v & 63u;
  }
};

__constant__ CandidateTable g_candidates = make_candidate_table();
static_assert(make_candidate_table().count == kNumCandidates, "candidate count");
static_assert(make_candidate_table().quad == kNumQuadCandidates, "quad candidate count");
__constant__ CandidateTable4 g_candidates4 = make_candidate_table4();
static_assert(make_candidate_table4().count == kNumCandidates4, "4-area candidate count");
// small alphabets: 16 symbols in 2 or 4 areas, 64 symbols in 4 or 8 areas
constexpr int kNumCandM16A2 = 5, kNumCandM16A4 = 25, kNumCandM64A4 = 70, kNumCandM64A8 = 693;
__constant__ SmallCandidateTable<kNumCandM16A2> g_cand_m16a2 =
    make_small_candidates<16, 2, kNumCandM16A2>();
__constant__ SmallCandidateTable<kNumCandM16A4> g_cand_m16a4 =
    make_small_candidates<16, 4, kNumCandM16A4>();
__constant__ SmallCandidateTable<kNumCandM64A4> g_cand_m64a4 =
    make_small_candidates<64, 4, kNumCandM64A4>();
__constant__ SmallCandidateTable<kNumCandM64A8> g_cand_m64a8 =
    make_small_candidates<64, 8, kNumCandM64A8>();
static_assert(make_small_candidates<16, 2, kNumCandM16A2>().count == kNumCandM16A2, "count");
static_assert(make_small_candidates<16, 4, kNumCandM16A4>().count == kNumCandM16A4, "count");
static_assert(make_small_candidates<64, 4, kNumCandM64A4>().count == kNumCandM64A4, "count");
static_assert(make_small_candidates<64, 8, kNumCandM64A8>().count == kNumCandM64A8, "count");


// ===========================================================================
// Table construction (Implementation section, Tables 1-4).  Run by one
// workgroup of any size that is a multiple of 64.
// ===========================================================================
struct TableSmem {
  uint64_t h[256];
  uint64_t key[256];        // count << 8 | (255 - symbol): unique sort keys
  __attribute__((aligned(16))) uint32_t key32[256];  // the same while counts < 2^23
  uint64_t P[257];          // P[r] = sum of the counts of ranks < r
  uint64_t wave_min[16];
  uint32_t wave_pk[16];     // layout of each wave's cheapest candidate
  uint32_t rank[256];       // symbol -> rank
  uint32_t rpart[4 * 256];  // partial ranks, one row per quarter of the keys
  uint32_t r2s[256];        // rank -> symbol
  uint32_t width[8], first[8], count[8], offset[8];
  uint64_t cost;
  uint32_t flagw[16];       // per wave: 1 = a count too large, 2 = a count needing 64-bit keys
  qlc_table stage;          // the table is assembled here, then copied out
};

// kCoherent: copy the table out with device-coherent stores, for readers
// in other workgroups of the same launch (the batched encoder).
template <bool kCoherent>
__device__ __forceinline__ void build_table_block(const uint64_t* h_in, uint32_t mode,
                                  qlc_table* out_g, TableSmem& S) {
  qlc_table* out = &S.stage;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  // the alphabet: M symbols of sbits bits; symbols M..255 take no part
  // (their counts must be zero) and keep ranks M..255 in symbol order
  const uint32_t sbits = mode_symbol_bits(mode);
  const uint32_t M = 1u << sbits;
  int big = 0;   // a count of 2^48 or more, or a count of a symbol outside the alphabet
  int wide = 0;  // a count of 2^23 or more: the keys need 64 bits
  for (int s = tid; s < 256; s += nt) {
    uint64_t c = h_in[s];
    big |= ((c >> 48) != 0 || ((uint32_t)s >= M && c != 0)) ? 1 : 0;
    if ((uint32_t)s >= M) c = 0;
    wide |= (c >> 23) != 0 ? 1 : 0;
    S.h[s] = c;
    S.key[s] = (c << 8) | (uint64_t)(255 - s);
    S.key32[s] = (uint32_t)(c << 8) | (uint32_t)(255 - s);
  }
  // the two flags over the workgroup: a ballot per wave, one word per wave
  // in LDS, one barrier
  {
    const uint64_t bb = __ballot(big != 0), bw = __ballot(wide != 0);
    if ((tid & 63) == 0) S.flagw[tid >> 6] = (bb ? 1u : 0u) | (bw ? 2u : 0u);
    __syncthreads();
    uint32_t f = 0;
    for (int w = 0; w < nt / 64; ++w) f |= S.flagw[w];
    big = (int)(f & 1u);
    wide = (int)(f >> 1);
  }

  // Rank = number of symbols that sort before s: larger count, or equal
  // count and smaller symbol value, i.e. the number of larger keys (counts
  // are below 2^48, so count << 8 loses nothing).  Each (symbol, part) pair
  // counts the larger keys in its part of the 256 keys, read as LDS
  // broadcasts (two or three VALU ops per key, no cross-lane traffic); a
  // workgroup of 256 * parts threads covers all pairs in one pass.
  {
    const int parts = nt >= 1024 ? 4 : (nt >= 512 ? 2 : 1);
    const int span = 256 / parts;
    for (int i = tid; i < 256 * parts; i += nt) {
      const int s = i & 255, p = i >> 8;
      uint32_t r = 0;
      if (!wide) {  // counts below 2^23: 31-bit keys, four per LDS read
        // v > ks exactly when ks - v borrows, i.e. sets bit 31 (both keys
        // below 2^31): no compare-to-mask and its wait states
        const uint32_t ks = S.key32[s];
        const uint4* kk = reinterpret_cast<const uint4*>(&S.key32[p * span]);
#pragma unroll 8
        for (int u = 0; u < span / 4; ++u) {
          const uint4 v = kk[u];
          r += ((ks - v.x) >> 31) + ((ks - v.y) >> 31) + ((ks - v.z) >> 31) +
               ((ks - v.w) >> 31);
        }
      } else {
        const uint64_t ks = S.key[s];
#pragma unroll 16
        for (int u = p * span; u < (p + 1) * span; ++u) r += S.key[u] > ks ? 1u : 0u;
      }
      S.rpart[i] = r;
    }
    __syncthreads();
    for (int s = tid; s < 256; s += nt) {
      uint32_t r = 0;
      for (int p = 0; p < parts; ++p) r += S.rpart[p * 256 + s];
      S.rank[s] = r;
      S.r2s[r] = s;
    }
  }
  __syncthreads();

  // Prefix sums of the counts in rank order (wave 0, 4 ranks per lane).
  if (tid < 64) {
    const uint64_t v0 = S.h[S.r2s[4 * tid + 0]];
    const uint64_t v1 = S.h[S.r2s[4 * tid + 1]];
    const uint64_t v2 = S.h[S.r2s[4 * tid + 2]];
    const uint64_t v3 = S.h[S.r2s[4 * tid + 3]];
    const uint64_t local = v0 + v1 + v2 + v3;
    const uint64_t incl = wave_inclusive_scan_u64(local);
    const uint64_t excl = incl - local;
    S.P[4 * tid + 0] = excl;
    S.P[4 * tid + 1] = excl + v0;
    S.P[4 * tid + 2] = excl + v0 + v1;
    S.P[4 * tid + 3] = excl + v0 + v1 + v2;
    if (tid == 63) S.P[256] = incl;
  }
  __syncthreads();

  // Layout: fixed printed widths, or the cheapest candidate (ties to the
  // smallest index = lexicographically smallest tuple).
  // area code bits: 3 (8 areas), 2 (4 areas) or 1 (2 areas)
  const uint32_t na = mode_areas(mode);
  const uint32_t pbits = na == 8 ? 3u : na == 4 ? 2u : 1u;
  uint32_t packed;
  if (mode == QLC_LAYOUT_PAPER_T1) {
    packed = kPaperT1Packed;
  } else if (mode == QLC_LAYOUT_PAPER_T2) {
    packed = kPaperT2Packed;
  } else {
    // cost = 3 * N + sum_a width_a * (ranks' counts in area a), from the
    // width increases the candidate carries (make_steps: three prefix-sum
    // reads) or, for candidates with more, from its area ends (one read per
    // area); the reads of a candidate are independent.
    const uint32_t max_distinct = mode == QLC_LAYOUT_SEARCH_QUAD ? 4u
                                  : (mode >= 17u && mode <= 24u) ? mode - 16u : 8u;
    const Candidate* ct;
    int ncand;
    if (mode == QLC_LAYOUT_M16_AREAS2) {
      ct = g_cand_m16a2.c;
      ncand = kNumCandM16A2;
    } else if (mode == QLC_LAYOUT_M16_AREAS4) {
      ct = g_cand_m16a4.c;
      ncand = kNumCandM16A4;
    } else if (mode == QLC_LAYOUT_M64_AREAS4) {
      ct = g_cand_m64a4.c;
      ncand = kNumCandM64A4;
    } else if (mode == QLC_LAYOUT_M64_AREAS8) {
      ct = g_cand_m64a8.c;
      ncand = kNumCandM64A8;
    } else if (na == 4) {
      ct = g_candidates4.c;
      ncand = kNumCandidates4;
    } else {
      ct = g_candidates.c;
      ncand = max_distinct <= 4u ? kNumQuadCandidates : kNumCandidates;
    }
    const uint64_t pN = S.P[256];
    uint64_t best = ~0ull;
    uint32_t best_pk = 0;
    // Four candidates per thread and step, all four loaded before any is
    // costed, so the constant-table loads overlap.
    constexpr int kCandStep = 4;
    for (int i0 = tid; i0 < ncand; i0 += kCandStep * nt) {
      Candidate cds[kCandStep];
#pragma unroll
      for (int u = 0; u < kCandStep; ++u) {
        const int i = i0 + u * nt;
        cds[u] = ct[i < ncand ? i : 0];
      }
#pragma unroll
      for (int u = 0; u < kCandStep; ++u) {
        const Candidate& cd = cds[u];
        if (i0 + u * nt >= ncand || (cd.lex >> 16) > max_distinct) continue;
        uint64_t cost;
        if (!(cd.steps >> 63)) {
          // at most three width increases: three prefix-sum reads
          const uint32_t wl = (cd.packed >> (4 * (na - 1))) & 15u;
          cost = (uint64_t)(pbits + wl) * pN;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const uint32_t sj = (uint32_t)(cd.steps >> (13 * j));
            cost -= (uint64_t)((sj >> 9) & 15u) * S.P[sj & 0x1FFu];
          }
        } else {
          cost = pbits * pN;
          uint64_t prev = 0;
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            if ((uint32_t)a >= na) break;
            const uint32_t e = (uint32_t)a < na - 1 ? (uint32_t)(cd.ends >> (8 * a)) & 0xFFu : M;
            const uint64_t pe = S.P[e];
            cost += (uint64_t)((cd.packed >> (4 * a)) & 15u) * (pe - prev);
            prev = pe;
          }
        }
        const uint64_t key = (cost << 12) | (uint64_t)(cd.lex & 0xFFFFu);
        if (key < best) {
          best = key;
          best_pk = cd.packed;
        }
      }
    }
    // keys are unique (lex differs), so exactly one lane of a wave holds
    // the wave's minimum and records its layout; every thread then picks
    // the smallest of the wave minima (a wave without candidates reports
    // ~0, which never wins: every mode has at least one candidate)
    const uint64_t wmin = wave_min_u64(best);
    if ((tid & 63) == 0) S.wave_min[tid >> 6] = wmin;
    if (best == wmin && best != ~0ull) S.wave_pk[tid >> 6] = best_pk;
    __syncthreads();
    uint64_t m = S.wave_min[0];
    int wb = 0;
    for (int w = 1; w < nt / 64; ++w) {
      if (S.wave_min[w] < m) {
        m = S.wave_min[w];
        wb = w;
      }
    }
    packed = S.wave_pk[wb];
  }

  // Greedy fill, offsets (an area whose width is the symbol width carries
  // the raw rank), cost; the areas a table with fewer than 8 areas does not
  // use get width 0xFF and no ranks.  Lane a of wave 0 fills area a: its
  // first rank is the capacity of the areas before it, capped at M.
  if (tid < 64) {
    const uint32_t a = (uint32_t)tid & 7u;
    uint32_t f = 0;
    for (uint32_t k = 0; k < a && k < na; ++k) {
      const uint32_t c = f + (1u << ((packed >> (4 * k)) & 15u));
      f = c < M ? c : M;
    }
    uint64_t term = 0;
    uint32_t w = 0xFFu, first = 256u, cnt = 0u, off = 0u;
    if (a < na) {
      const uint32_t b = (packed >> (4 * a)) & 15u;
      const uint32_t cap = 1u << b;
      cnt = cap < M - f ? cap : M - f;
      w = b;
      first = f;
      off = (b == sbits) ? 0u : f;
      term = (uint64_t)(pbits + b) * (S.P[f + cnt] - S.P[f]);
    }
    // sum of the eight lanes' terms: the 64 lanes hold each of them eight
    // times (lane a + 8i repeats lane a)
    term = wave_sum_u64(term) >> 3;
    if (tid < 8) {
      S.width[a] = w;
      S.first[a] = first;
      S.count[a] = cnt;
      S.offset[a] = off;
    }
    if (tid == 0) S.cost = term;
  }
  __syncthreads();

  // Counts must sum below 2^48 (so that the rank keys and the search keys
  // are exact); a larger histogram yields a table marked unusable: every
  // code length 0 and every width 0xFF, which the encoders reject.
  const bool unusable = big != 0 || (S.P[256] >> 48) != 0;

  // Encoder LUT (Table 3), indexed by input symbol (no code for symbols
  // outside the alphabet).
  for (int s = tid; s < 256; s += nt) {
    const uint32_t r = S.rank[s];
    uint32_t a = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) a = (r >= S.first[k]) ? (uint32_t)k : a;
    const uint32_t b = S.width[a];
    const uint32_t code = (a << b) | (r - S.offset[a]);
    out->enc[s] = (unusable || (uint32_t)s >= M) ? (uint16_t)0
                                                 : (uint16_t)(((pbits + b) << 11) | code);
    out->rank_to_sym[s] = (uint8_t)S.r2s[s];
    out->sym_to_rank[s] = (uint8_t)r;
  }
  if (tid < 8) {
    out->width[tid] = unusable ? (uint8_t)0xFFu : (uint8_t)S.width[tid];
    out->offset[tid] = unusable ? (uint8_t)0u : (uint8_t)S.offset[tid];
    out->first[tid] = unusable ? (uint16_t)256u : (uint16_t)S.first[tid];
    out->count[tid] = unusable ? (uint16_t)0u : (uint16_t)S.count[tid];
  }
  if (tid == 0) {
    out->cost_bits = unusable ? ~0ull : S.cost;
    out->mode = mode;
    out->version = QLC_ABI_VERSION;
  }
  __syncthreads();
  static_assert(sizeof(qlc_table) % 4 == 0, "table words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&S.stage);
  uint32_t* dst = reinterpret_cast<uint32_t*>(out_g);
  for (int w = tid; w < (int)(sizeof(qlc_table) / 4); w += nt) {
    if (kCoherent) store_relaxed_u32(&dst[w], src[w]);
    else dst[w] = src[w];
  }
}

__global__ __launch_bounds__(kTableThreads) void k_table_from_hist(
    const uint64_t* __restrict__ hist, uint32_t mode, qlc_table* __restrict__ out) {
  __shared__ TableSmem S;
  build_table_block<false>(hist, mode, out, S);
}

// ===========================================================================
// Histogram (Observations section: the PMF of the 256 byte symbols).
//
// One workgroup per segment of 2^log2_seg symbols.  The workgroup keeps 32
// LDS copies of the histogram, one per lane mod 32, so the lanes of a wave
// never collide on a bin even under extreme skew.  Outputs, each optional:
//   - the segment's own histogram (uint32[256]), which the encoder turns
//     into the segment's bit count once the table is known;
//   - the whole input's histogram, accumulated with device-scope atomics
//     into per-XCD uint64 partials and folded by the last workgroup, which
//     can then build the table in place.
// ===========================================================================
union HistSmem {
  uint32_t sub[256 * kHistCopies];
  TableSmem table;
};

__device__ __forceinline__ void hist_add_word(uint32_t* sub, uint32_t w, uint32_t copy) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t b = (w >> (8 * k)) & 0xFFu;
    atomicAdd(&sub[(b << 5) | copy], 1u);
  }
}

__device__ __forceinline__ void hist_add_vec(uint32_t* sub, uint4 v, uint32_t copy) {
  hist_add_word(sub, v.x, copy);
  hist_add_word(sub, v.y, copy);
  hist_add_word(sub, v.z, copy);
  hist_add_word(sub, v.w, copy);
}

// Count symbols [seg0, seg1) of `in` into the 32 LDS copies (zeroed by the
// caller); seg0 is a multiple of 16.  Whole groups of 16 symbols are read
// as one vector each (16, 8 or 12 bytes by the alphabet).
template <int kBits>
__device__ __forceinline__ void hist_segment(const uint8_t* __restrict__ in_p, uint64_t seg0,
                                             uint64_t seg1, uint32_t* sub, uint32_t tid) {
  using SI = Sym<kBits>;
  const QLC_GLOBAL uint8_t* in = (const QLC_GLOBAL uint8_t*)in_p;
  const uint32_t nt = blockDim.x;
  const uint32_t copy = tid & (kHistCopies - 1);
  const uint64_t v0 = seg0 >> 4, v1 = seg1 >> 4;  // whole 16-symbol groups of the segment
  uint64_t i = v0 + tid;
  if (i + 3 * nt < v1) {
    // the next four groups are loaded before the current four are counted
    uint4 a = SI::fetch16(in, i << 4), b = SI::fetch16(in, (i + nt) << 4);
    uint4 c = SI::fetch16(in, (i + 2 * nt) << 4), d = SI::fetch16(in, (i + 3 * nt) << 4);
    for (;;) {
      const uint64_t nx = i + 4 * nt;
      const bool more = nx + 3 * nt < v1;
      uint4 na = a, nb = b, nc = c, nd = d;
      if (more) {
        na = SI::fetch16(in, nx << 4);
        nb = SI::fetch16(in, (nx + nt) << 4);
        nc = SI::fetch16(in, (nx + 2 * nt) << 4);
        nd = SI::fetch16(in, (nx + 3 * nt) << 4);
      }
      hist_add_vec(sub, a, copy);
      hist_add_vec(sub, b, copy);
      hist_add_vec(sub, c, copy);
      hist_add_vec(sub, d, copy);
      i = nx;
      if (!more) break;
      a = na;
      b = nb;
      c = nc;
      d = nd;
    }
  }
  for (; i < v1; i += nt) hist_add_vec(sub, SI::fetch16(in, i << 4), copy);
  for (uint64_t j = (v1 << 4) + tid; j < seg1; j += nt)  // ragged tail of the input
    atomicAdd(&sub[(SI::at(in, j) << 5) | copy], 1u);
}

// Per-bin total of the 32 copies (thread t < 256 sums bin t).
__device__ __forceinline__ uint32_t hist_bin_total(const uint32_t* sub, uint32_t t) {
  uint32_t s = 0;
#pragma unroll 8
  for (uint32_t c = 0; c < kHistCopies; ++c) s += sub[(t << 5) | ((c + t) & 31)];
  return s;
}

template <int kBits>
__global__ __launch_bounds__(kHistThreads) void k_histogram(
    const uint8_t* __restrict__ in, uint64_t n, uint32_t log2_seg, WsHeader* __restrict__ hdr,
    uint64_t* __restrict__ xcd_part, uint32_t* __restrict__ seg_hist,
    uint64_t* __restrict__ hist_out, uint32_t flags, uint32_t mode,
    qlc_table* __restrict__ table_out) {
  __shared__ HistSmem S;
  __shared__ uint32_t is_last;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < 256 * kHistCopies; i += kHistThreads) S.sub[i] = 0;
  __syncthreads();

  const uint64_t seg0 = (uint64_t)blockIdx.x << log2_seg;
  const uint64_t seg1 = (seg0 + (1ull << log2_seg)) < n ? seg0 + (1ull << log2_seg) : n;
  hist_segment<kBits>(in, seg0, seg1, S.sub, tid);
  __syncthreads();

  if (tid < 256) {
    const uint32_t s = hist_bin_total(S.sub, tid);
    if (flags & kHistSegment) seg_hist[(uint64_t)blockIdx.x * 256 + tid] = s;
    if ((flags & kHistGlobal) && s)
      atomicAdd((unsigned long long*)&xcd_part[(blockIdx.x % kNumXcd) * 256 + tid],
                (unsigned long long)s);
  }
  if (!(flags & kHistGlobal)) return;
  // Every partial must be performed before this workgroup counts as done:
  // wait for the atomics to be acknowledged (device-scope atomics are
  // coherent across XCDs, so no cache flush is needed).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) is_last = (atomic_add_u32(&hdr->hist_done, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;

  uint64_t* hsum = S.table.h;  // reuse LDS (sub is no longer needed)
  if (tid < 256) {
    uint64_t s = 0;
#pragma unroll
    for (int x = 0; x < kNumXcd; ++x) s += load_relaxed_u64(&xcd_part[x * 256 + tid]);
    if (hist_out) hist_out[tid] = (flags & kHistAccumulate) ? hist_out[tid] + s : s;
    hsum[tid] = s;
#pragma unroll
    for (int x = 0; x < kNumXcd; ++x) store_relaxed_u64(&xcd_part[x * 256 + tid], 0);
  }
  if (tid == 0) store_relaxed_u32(&hdr->hist_done, 0);
  __syncthreads();
  if (flags & kHistBuildTable) build_table_block<false>(hsum, mode, table_out, S.table);
}

// ===========================================================================
// Encode (Implementation section: look up each code, concatenate).
//
// One workgroup per segment (the histogram kernel's segments), segments
// numbered by an atomic ticket.  A segment's bit count is the dot product
// of its histogram with the code lengths, so every workgroup publishes its
// count at once and sums its predecessors' counts (all published within a
// few microseconds: no serial look-back chain).  The workgroup then walks
// its segment in tiles of kEncTile (8192) symbols: LUT gather from LDS,
// block scan of the code lengths, bit packing into LDS at the running
// global alignment, coalesced stores of the whole words; the partial last
// word is carried into the next tile.  A segment's first word also holds
// the last bits of the previous segment, which the workgroup recomputes
// from the 32 symbols before its segment (at least 32 bits, since every
// code has at least one); its own partial last word is left to the next
// segment (the last segment pads and stores it).
// ===========================================================================
struct EncSmem {
  uint32_t lut[256];        // code | length << 16 (halves feed SDWA operands)
  __attribute__((aligned(16))) uint32_t words[2][kEncTile * QLC_MAX_CODE_BITS / 32 + 4];
  uint64_t red[kEncThreads / 64];
  uint32_t wave_sum[kEncThreads / 64];
  uint32_t epoch, cap_hit, bad_table, is_last;
};

// Encoder LUT entry of a table's (len << 11) | code word: code | len << 16.
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t enc_entry(uint32_t e) {
  return (e & 0x7FFu) | ((e >> 11) << 16);
}

// Whether symbol s's encoder entry e ((len << 11) | code) is usable for an
// alphabet of kBits-bit symbols: symbols of the alphabet need a length in
// 1..11; the others are never read.
template <int kBits>
__device__ __forceinline__ bool enc_entry_ok(uint32_t e, uint32_t s) {
  return s >= Sym<kBits>::kM || ((e >> 11) >= 1 && (e >> 11) <= QLC_MAX_CODE_BITS);
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
  v = wave_sum_u64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int w = 0; w < kEncThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Append code `c` of `l` bits to the thread's run in the LDS word buffer
// (64-bit accumulator, a whole word is OR-ed out whenever 32 bits are due;
// the caller guarantees nacc + l <= 63).
struct Packer {
  uint64_t acc;
  uint32_t nacc, widx;
  __device__ __forceinline__ void put(uint32_t* words, uint32_t c, uint32_t l) {
    acc = (acc << l) | c;
    nacc += l;
    if (nacc >= 32) {
      nacc -= 32;
      atomicOr(&words[widx], (uint32_t)(acc >> nacc));
      ++widx;
    }
  }
  __device__ __forceinline__ void finish(uint32_t* words) {
    if (nacc) atomicOr(&words[widx], (uint32_t)(acc << (32 - nacc)));
  }
};

// Code pair of two encoder LUT entries (code | length << 16): code0 << len1
// | code1, and its length.  Written with SDWA word selects (one operation
// each) because the compiler otherwise extracts the halves separately.
__device__ __forceinline__ uint32_t pair_code(uint32_t e0, uint32_t e1) {
  uint32_t t, r;
  asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:WORD_0"
      : "=v"(t) : "v"(e1), "v"(e0));
  asm("v_or_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
      : "=v"(r) : "v"(t), "v"(e1));
  return r;
}
__device__ __forceinline__ uint32_t pair_len(uint32_t e0, uint32_t e1) {
  uint32_t r;
  asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:WORD_1"
      : "=v"(r) : "v"(e0), "v"(e1));
  return r;
}

// State of a segment's encode carried from tile to tile.
template <int kBits>
struct EncSeg {
  const QLC_GLOBAL uint8_t* in;
  uint64_t seg1;
  uint64_t R;                        // global bit offset of the current tile
  uint64_t seg_w0;                   // the segment's first stream word
  uint64_t cap_words;
  uint64_t cmask;                    // chunk_symbols - 1
  uint32_t log2_chunk;
  bool last_seg;
  __amdgpu_buffer_rsrc_t out_rsrc;   // stream words from seg_w0 on, clipped at cap_words
  QLC_GLOBAL uint64_t* index_out;
  typename Sym<kBits>::Raw nx0, nx1;  // the next full tile's input (prefetched, as loaded)
  uint32_t buf;                      // word buffer of the current tile
};

// One tile of 8192 symbols at t0 (kFull: a whole tile; else the input's
// ragged last tile [t0, seg1)).  Thread tid owns two runs of the tile:
// symbols 16*tid.. (first half) and 4096+16*tid.. (second half), so that
// its loads are coalesced; every first-half run precedes every second-half
// run in the stream, and one block scan of the packed pair of run lengths
// (b0 | b1 << 16) places both (run bits <= 176, block totals < 2^16).
// Returns true in a thread one of whose stores would have passed cap_words.
template <int kBits, bool kFull>
__device__ __forceinline__ bool encode_tile(EncSeg<kBits>& E, uint64_t t0, EncSmem& S,
                                            uint32_t tid) {
  using SI = Sym<kBits>;
  const uint32_t lane = tid & 63, wave = tid >> 6;
  bool cap = false;
  uint32_t* const Wd = S.words[E.buf];
  uint32_t pc[16], pl[16];  // code pairs of the thread's 32 symbols
  uint32_t b0 = 0, b1 = 0;  // bits of the thread's two runs
  if (kFull) {
    const typename SI::Raw r0 = E.nx0, r1 = E.nx1;
    {  // prefetch the next tile (this one again when no whole tile follows)
      const uint64_t nt = (t0 + 2 * kEncTile <= E.seg1) ? t0 + kEncTile : t0;
      E.nx0 = SI::load16(E.in, nt + (uint64_t)tid * 16);
      E.nx1 = SI::load16(E.in, nt + kEncTile / 2 + (uint64_t)tid * 16);
    }
    const uint4 v0 = SI::expand(r0), v1 = SI::expand(r1);
    const uint32_t sw[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t w = sw[k >> 1];
      const uint32_t e0 = S.lut[(w >> (16 * (k & 1))) & 0xFFu];
      const uint32_t e1 = S.lut[(w >> (16 * (k & 1) + 8)) & 0xFFu];
      pc[k] = pair_code(e0, e1);
      pl[k] = pair_len(e0, e1);
      if (k < 8) b0 += pl[k];
      else b1 += pl[k];
    }
  } else {
    // The input's ragged last tile: each of the thread's 32 symbols loaded
    // on its own, all loads issued before the first is used (a symbol past
    // seg1 reads as 256, whose entry is 0: no code, no length); then the
    // same code pairs as a whole tile.
    uint32_t sy[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const uint64_t i = t0 + (uint64_t)(k >> 4) * (kEncTile / 2) + (uint64_t)tid * 16 + (k & 15);
      sy[k] = i < E.seg1 ? SI::at(E.in, i) : 256u;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t e0 = sy[2 * k] < 256u ? S.lut[sy[2 * k]] : 0u;
      const uint32_t e1 = sy[2 * k + 1] < 256u ? S.lut[sy[2 * k + 1]] : 0u;
      pc[k] = pair_code(e0, e1);
      pl[k] = pair_len(e0, e1);
      if (k < 8) b0 += pl[k];
      else b1 += pl[k];
    }
  }
  const uint32_t packed = b0 | (b1 << 16);
  const uint32_t incl = wave_inclusive_scan_u32(packed);
  if (lane == 63) S.wave_sum[wave] = incl;
  __syncthreads();
  uint32_t o = 0, h = 0;
#pragma unroll
  for (int w = 0; w < kEncThreads / 64; ++w) {
    const uint32_t ws = S.wave_sum[w];
    o += (w < (int)wave) ? ws : 0u;
    h += ws;
  }
  const uint32_t h0 = h & 0xFFFFu, h1 = h >> 16;
  const uint32_t tile_bits = h0 + h1;
  const uint32_t g = (uint32_t)(E.R & 31);
  const uint32_t off0 = (o & 0xFFFFu) + (incl & 0xFFFFu) - b0;
  const uint32_t off1 = h0 + (o >> 16) + (incl >> 16) - b1;
  {
    Packer P0{0, (g + off0) & 31u, (g + off0) >> 5};
    Packer P1{0, (g + off1) & 31u, (g + off1) >> 5};
#pragma unroll
    for (int k = 0; k < 8; ++k) P0.put(Wd, pc[k], pl[k]);
#pragma unroll
    for (int k = 8; k < 16; ++k) P1.put(Wd, pc[k], pl[k]);
    P0.finish(Wd);
    P1.finish(Wd);
    // chunk index entries: a run's first symbol may start a chunk
    const uint64_t i0s = t0 + (uint64_t)tid * 16;
    const uint64_t i1s = i0s + kEncTile / 2;
    if (i0s < E.seg1 && (i0s & E.cmask) == 0) E.index_out[i0s >> E.log2_chunk] = E.R + off0;
    if (i1s < E.seg1 && (i1s & E.cmask) == 0) E.index_out[i1s >> E.log2_chunk] = E.R + off1;
  }
  __syncthreads();
  // store the whole words (and, at the very end, the padded last word),
  // clearing them for the next tile
  const uint32_t endb = g + tile_bits;
  const bool final_tile = E.last_seg && (t0 + kEncTile >= E.seg1);
  const uint32_t nw = final_tile ? (endb + 31) >> 5 : endb >> 5;
  const uint32_t wr = (uint32_t)((E.R >> 5) - E.seg_w0);  // tile's first word, segment-relative
  if (tid == 0 && (E.R >> 5) + nw > E.cap_words) cap = true;
  // four words per thread per store; the buffer resource drops anything
  // past the capacity
  for (uint32_t i = 4 * tid; i < nw; i += 4 * kEncThreads) {
    uint4* src = reinterpret_cast<uint4*>(&Wd[i]);
    if (i + 4 <= nw) {
      const uint4 v = *src;
      *src = make_uint4(0, 0, 0, 0);
      const v4u32 ov = {__builtin_bswap32(v.x), __builtin_bswap32(v.y), __builtin_bswap32(v.z),
                        __builtin_bswap32(v.w)};
      __builtin_amdgcn_raw_buffer_store_b128(ov, E.out_rsrc, (wr + i) * 4, 0, 0);
    } else {
      for (uint32_t k = i; k < nw; ++k) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bswap32(Wd[k]), E.out_rsrc,
                                              (wr + k) * 4, 0, 0);
        Wd[k] = 0;
      }
    }
  }
  if (tid == 0 && !final_tile) {
    // the partial last word (no store above touches it) becomes word 0 of
    // the other buffer, which the next tile packs into; this buffer is not
    // packed again before every thread has passed the next tile's barriers
    const uint32_t carry = Wd[endb >> 5];
    Wd[endb >> 5] = 0;
    S.words[E.buf ^ 1][0] = carry;
  }
  E.buf ^= 1;
  E.R += tile_bits;
  return cap;
}

// Encode symbols [seg0, seg1) of `in`, whose first code starts at stream
// bit G (kEncThreads threads, tid = threadIdx.x).  On entry S.lut holds the encoder LUT and
// both word buffers are zero except word 0 of buffer 0 (written here).  Tiles
// alternate between the two buffers, so a tile's stores and the next
// tile's packing need no barrier between them.  Every
// whole stream word of the segment is stored; its partial first word also
// carries the previous segment's last bits (recomputed from the 32 symbols
// before seg0, which hold at least 32 bits since every code has at least
// one); its partial last word is left to the next segment, unless
// `last_seg` (padded and stored).  Returns true in a thread one of whose
// stores would have passed cap_words (that store is dropped).  Whole tiles
// run in a loop of their own, the ragged last tile (if any) after it.
template <int kBits>
__device__ __forceinline__ bool encode_segment(const uint8_t* __restrict__ in, uint64_t seg0, uint64_t seg1,
                               uint64_t G, bool last_seg, uint32_t log2_chunk,
                               uint32_t* __restrict__ bits_out, uint64_t cap_words,
                               uint64_t* __restrict__ index_out, EncSmem& S, uint32_t tid) {
  using SI = Sym<kBits>;
  bool cap = false;
  // ---- last bits of the previous segment (recomputed from its input) ----
  if (tid == 0) {
    uint32_t w0 = 0;
    if ((G & 31) != 0) {
      uint64_t acc = 0;
      for (int k = 32; k >= 1; --k) {
        const uint32_t e = S.lut[SI::at((const QLC_GLOBAL uint8_t*)in, seg0 - k)];
        acc = (acc << (e >> 16)) | (e & 0xFFFFu);
      }
      w0 = ((uint32_t)acc) << (32 - (uint32_t)(G & 31));
    }
    S.words[0][0] = w0;
  }
  EncSeg<kBits> E;
  E.in = (const QLC_GLOBAL uint8_t*)in;
  E.seg1 = seg1;
  E.R = G;
  E.cap_words = cap_words;
  E.cmask = (1ull << log2_chunk) - 1;
  E.log2_chunk = log2_chunk;
  E.last_seg = last_seg;
  E.index_out = (QLC_GLOBAL uint64_t*)index_out;
  // Output through a buffer resource based at the segment's first word
  // (segment-relative offsets stay far below 2^32): stores at or past
  // cap_words are dropped by the hardware.
  E.seg_w0 = G >> 5;
  const uint64_t room = cap_words > E.seg_w0 ? (cap_words - E.seg_w0) * 4 : 0;
  E.out_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      bits_out + (cap_words > E.seg_w0 ? E.seg_w0 : 0), (short)0,
      (int)(uint32_t)(room < 0xFFFFFFF0ull ? room : 0xFFFFFFF0ull), 0x00020000);
  E.buf = 0;
  E.nx0 = typename SI::Raw{};
  E.nx1 = E.nx0;
  if (seg0 + kEncTile <= seg1) {
    E.nx0 = SI::load16(E.in, seg0 + (uint64_t)tid * 16);
    E.nx1 = SI::load16(E.in, seg0 + kEncTile / 2 + (uint64_t)tid * 16);
  }
  uint64_t t0 = seg0;
  for (; t0 + kEncTile <= seg1; t0 += kEncTile) cap |= encode_tile<kBits, true>(E, t0, S, tid);
  if (t0 < seg1 || seg0 == seg1) cap |= encode_tile<kBits, false>(E, t0, S, tid);
  return cap;
}

// Bit count of every segment under a given table (the pre-pass of an encode
// with a fixed table): the segment's code lengths summed through an LDS
// copy of the length column, no atomics.
template <int kBits>
__global__ __launch_bounds__(kHistThreads) void k_segment_bits(
    const uint8_t* __restrict__ in_p, uint64_t n, uint32_t log2_seg,
    const qlc_table* __restrict__ table, uint64_t* __restrict__ seg_bits) {
  using SI = Sym<kBits>;
  const QLC_GLOBAL uint8_t* in = (const QLC_GLOBAL uint8_t*)in_p;
  __shared__ uint32_t len[256];
  __shared__ uint64_t red[kHistThreads / 64];
  const uint32_t tid = threadIdx.x;
  if (tid < 256) len[tid] = table->enc[tid] >> 11;
  __syncthreads();
  const uint64_t seg0 = (uint64_t)blockIdx.x << log2_seg;
  const uint64_t seg1 = (seg0 + (1ull << log2_seg)) < n ? seg0 + (1ull << log2_seg) : n;
  const uint64_t v0 = seg0 >> 4, v1 = seg1 >> 4;  // whole 16-symbol groups
  uint32_t s = 0;
  uint64_t i = v0 + tid;
  for (; i + 3 * kHistThreads < v1; i += 4 * kHistThreads) {
    const uint4 a = SI::fetch16(in, i << 4), b = SI::fetch16(in, (i + kHistThreads) << 4);
    const uint4 c = SI::fetch16(in, (i + 2 * kHistThreads) << 4);
    const uint4 d = SI::fetch16(in, (i + 3 * kHistThreads) << 4);
    const uint32_t w[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w,
                            c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
#pragma unroll
    for (int k = 0; k < 16; ++k)
      s += len[w[k] & 0xFFu] + len[(w[k] >> 8) & 0xFFu] + len[(w[k] >> 16) & 0xFFu] +
           len[w[k] >> 24];
  }
  for (; i < v1; i += kHistThreads) {
    const uint4 a = SI::fetch16(in, i << 4);
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      s += len[w[k] & 0xFFu] + len[(w[k] >> 8) & 0xFFu] + len[(w[k] >> 16) & 0xFFu] +
           len[w[k] >> 24];
  }
  for (uint64_t j = (v1 << 4) + tid; j < seg1; j += kHistThreads) s += len[SI::at(in, j)];
  const uint64_t t = wave_sum_u64(s);
  if ((tid & 63) == 0) red[tid >> 6] = t;
  __syncthreads();
  if (tid == 0) {
    uint64_t sum = 0;
#pragma unroll
    for (int w = 0; w < kHistThreads / 64; ++w) sum += red[w];
    seg_bits[blockIdx.x] = sum;
  }
}

// Bit count of segment k from its histogram and the code lengths in the
// encoder LUT (a predecessor's count that was not published in time).
__device__ __forceinline__ uint64_t segment_bits_from_hist(const uint32_t* __restrict__ h,
                                                           const uint32_t* lut) {
  uint64_t b = 0;
#pragma unroll 8
  for (int s = 0; s < 256; ++s) b += (uint64_t)h[s] * (lut[s] >> 16);
  return b;
}

template <int kBits>
__global__ __launch_bounds__(kEncThreads) void k_encode(
    const uint8_t* __restrict__ in, uint64_t n, uint32_t log2_seg,
    const qlc_table* __restrict__ table, const uint32_t* __restrict__ seg_hist,
    const uint64_t* __restrict__ seg_bits, uint32_t log2_chunk, uint32_t* __restrict__ bits_out,
    uint64_t cap_words, uint64_t* __restrict__ index_out, uint64_t* __restrict__ total_out,
    uint32_t* __restrict__ err_out, WsHeader* __restrict__ hdr, uint64_t* __restrict__ seg_word,
    uint32_t nseg, uint32_t spin_polls) {
  __shared__ EncSmem S;
  const uint32_t tid = threadIdx.x;
  // The workgroup's segment is its block index: no shared ticket counter,
  // whose one atomic per workgroup (all issued at once) cost ~15 us per
  // launch of 1024 workgroups.
  const uint32_t seg = blockIdx.x;
  if (tid == 0) {
    S.epoch = load_relaxed_u32(&hdr->enc_epoch) & kEpochMask;
    S.cap_hit = 0;
    S.bad_table = 0;
  }
  const uint32_t e_t = table->enc[tid];
  // the segment's histogram bin, loaded beside the table entry
  const uint32_t h_t = seg_bits ? 0u : seg_hist[(uint64_t)seg * 256 + tid];
  S.lut[tid] = enc_entry(e_t);
  for (uint32_t w = tid; w < sizeof(S.words) / 4; w += kEncThreads) (&S.words[0][0])[w] = 0;
  __syncthreads();
  // A table whose code lengths leave 1..11 for a symbol of the alphabet, or
  // that codes another alphabet, is rejected: 11 keeps every LDS index of
  // the packer in bounds without per-symbol clamps.
  if (!enc_entry_ok<kBits>(e_t, tid) || (tid == 0 && mode_symbol_bits(table->mode) != kBits))
    S.bad_table = 1;
  const uint32_t epoch = S.epoch;
  const uint64_t tag = (uint64_t)(0x800000u | epoch) << 40;

  // ---- this segment's bit count, published; the predecessors' summed ----
  // Given bit counts (a fixed table: k_segment_bits ran before) are summed
  // directly.  Otherwise each workgroup publishes its count as soon as it
  // starts and sums its predecessors' published counts; a count still
  // missing after spin_polls polls (its workgroup not yet running) is
  // computed here from that segment's histogram, so the wait assumes
  // nothing about the order or residency of the workgroups.
  uint64_t my_bits, pre = 0;
  if (seg_bits) {
    my_bits = seg_bits[seg];
    for (uint32_t k = tid; k < seg; k += kEncThreads) pre += seg_bits[k];
  } else {
    my_bits = block_sum_u64((uint64_t)h_t * (e_t >> 11), S.red);
    if (tid == 0) store_relaxed_u64(&seg_word[seg], tag | (my_bits & kValueMask));
    for (uint32_t k = tid; k < seg; k += kEncThreads) {
      uint64_t w = load_relaxed_u64(&seg_word[k]);
      for (uint32_t p = 0; (w & ~kValueMask) != tag && p < spin_polls; ++p) {
        __builtin_amdgcn_s_sleep(1);
        w = load_relaxed_u64(&seg_word[k]);
      }
      pre += (w & ~kValueMask) == tag ? (w & kValueMask)
                                      : segment_bits_from_hist(seg_hist + (uint64_t)k * 256, S.lut);
    }
  }
  const uint64_t G = block_sum_u64(pre, S.red);
  // read after the block sum's barriers, so every thread's length check is in
  const bool bad_table = S.bad_table != 0;
  if (seg == nseg - 1 && tid == 0) *total_out = G + my_bits;

  const uint64_t seg0 = (uint64_t)seg << log2_seg;
  const uint64_t seg1 = (seg0 + (1ull << log2_seg)) < n ? seg0 + (1ull << log2_seg) : n;
  bool cap = false;
  if (!bad_table) {
    cap = encode_segment<kBits>(in, seg0, seg1, G, seg == nseg - 1, log2_chunk, bits_out,
                                cap_words, index_out, S, tid);
  } else if (tid == 0) {
    set_error(&hdr->enc_err, QLC_ERR_INVALID_ARGUMENT);
  }
  if (cap) S.cap_hit = 1;
  __syncthreads();

  // ---- last workgroup to finish publishes the error and resets the state ----
  if (tid == 0) {
    if (S.cap_hit) set_error(&hdr->enc_err, QLC_ERR_CAPACITY);
    S.is_last = atomic_add_u32(&hdr->enc_done, 1u) == nseg - 1;
  }
  __syncthreads();
  if (!S.is_last) return;
  // Every workgroup has finished reading its predecessors' words, so the
  // words this launch published are cleared: a later launch never sees a
  // word tagged by an earlier one, however far the 22-bit epoch has wrapped
  // (words of other sizes' layouts never carry bit 63: those bytes hold
  // segment counts below 2^21 or bit counts below 2^40).
  for (uint32_t k = tid; k < nseg; k += kEncThreads) store_relaxed_u64(&seg_word[k], 0);
  if (tid == 0) {
    *err_out = load_relaxed_u32(&hdr->enc_err);
    store_relaxed_u32(&hdr->enc_err, 0);
    store_relaxed_u32(&hdr->enc_done, 0);
    store_relaxed_u32(&hdr->enc_epoch, (epoch + 1) & kEpochMask);
  }
}

// ===========================================================================
// Decode (Implementation section: 3 bits give the area and thus the suffix
// width; suffix + offset = rank; rank -> symbol via the decoder LUT).
//
// One lane per chunk, kDecThreads (256) chunks per workgroup.  The decoder
// LUT is re-indexed by the whole code word: because widths never decrease,
// the codes of area a occupy the integer range [a << w_a, (a + 1) << w_a)
// and these ranges are disjoint, so a 2048-entry LDS table maps code ->
// symbol (bit 15 flags an invalid suffix; 32-bit entries, so gathered values
// need no zero extension before packing).  The per-symbol chain is pure
// VALU: the 3-bit area code selects the shift 29 - w_a from an 8-byte
// register table (v_perm), the code is the window shifted right by it, and
// three funnel shifts advance a 96-bit window by 3 + w_a bits.
//
// Memory: each lane streams its chunk in 32-byte superblocks (two 16-byte
// bounds-checked buffer loads) into a private 4-superblock LDS ring (plus a
// mirror of the first words, so a 4-word window never wraps), stored
// word-major so that window reads never conflict on LDS banks.  A
// superblock is requested three superblocks ahead of the window, at most
// one per 8-symbol group; whole waves keep four register sets in rotation,
// so a superblock is written to the ring four groups after its load was
// issued (at least six groups before the window can reach it) and every
// wave waits at fixed program points for loads that old.  Lanes that need
// no superblock issue the loads with an out-of-range offset (zeros
// returned, no memory touched).  Decoded bytes are staged per lane in LDS
// and, every kStageGroups (16) groups, the wave stores its 64 lanes'
// 128-byte output runs with coalesced stores (16 lanes per run, whole
// 128-byte lines).
// ===========================================================================
constexpr int kDecLanes = kDecThreads;     // chunks per workgroup
constexpr int kRingWords = 36;             // 4 x 8 ring words + 4 mirror words
constexpr uint32_t kSbLog2Bits = 8;         // superblock: 256 bits = 32 bytes
constexpr uint32_t kLookaheadBits = 768;   // request a superblock three ahead
constexpr uint32_t kOobOffset = 0xFFFFFFC0u;
constexpr uint32_t kAreaSel = 0x01818180u;  // alignbit(kAreaSel, A, 29) = (A >> 29) | 0x0C0C0C00

struct DecSmem {
  uint32_t lut[2048];
  uint32_t ring[kDecLanes * kRingWords];
  uint2 stage[kDecLanes * kStageGroups];    // kStageGroups groups x 8 bytes per lane
};

// Staging slot of group g of lane t: rotated by the lane so that the 8-byte
// writes of a wave, and the reads of the coalesced flush, hit distinct LDS
// banks.
__device__ __forceinline__ uint32_t stage_slot(uint32_t g, uint32_t t) {
  return kStageGroups == 8 ? ((g ^ (t >> 2)) & 7u) : ((g ^ (t >> 1)) & 15u);
}

struct Superblock {
  uint4 q0, q1;
};

__device__ __forceinline__ uint4 bufload16(__amdgpu_buffer_rsrc_t rsrc, uint32_t off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0);
  return make_uint4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ Superblock load_sb(__amdgpu_buffer_rsrc_t rsrc, uint32_t off) {
  Superblock s;
  s.q0 = bufload16(rsrc, off);
  s.q1 = bufload16(rsrc, off + 16);
  return s;
}

// Superblock `sb` (absolute number) into ring slot sb & 3 (words 8*(sb&3)),
// in memory byte order (the window reads swap to most-significant-first);
// slot 0's first four words are mirrored to words 32..35 so that a 4-word
// window never wraps.
// The ring is stored word-major ("transposed"): word w of lane l sits at
// ring[w * kDecLanes + l], so every lane only ever touches LDS bank l mod 64
// and the window reads of a wave are free of bank conflicts whatever the
// lanes' positions.
__device__ __forceinline__ void ring_put(uint32_t* ring, uint32_t sb, const Superblock& s) {
  uint32_t* r = ring + (sb & 3u) * 8u * kDecLanes;
  const uint32_t v[8] = {s.q0.x, s.q0.y, s.q0.z, s.q0.w, s.q1.x, s.q1.y, s.q1.z, s.q1.w};
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i * kDecLanes] = v[i];
  if ((sb & 3u) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ring[(32 + i) * kDecLanes] = v[i];
  }
}

struct DecLane {
  uint32_t* ring;
  uint64_t pm1;        // bit position of the next symbol, minus one
  uint32_t sh_lo, sh_hi;
  uint32_t errbits;
};

struct Window {
  uint32_t w0, w1, w2, w3;
};

// The four ring words holding bits pm1 + 1 .. pm1 + 96 (q = pm1, in the
// ring's coordinates), as stored (memory byte order).
__device__ __forceinline__ Window window_read(const uint32_t* ring, uint32_t q) {
  const uint32_t* rr = ring + ((q >> 5) & 31u) * kDecLanes;
  Window w;
  w.w0 = rr[0];
  w.w1 = rr[kDecLanes];
  w.w2 = rr[2 * kDecLanes];
  w.w3 = rr[3 * kDecLanes];
  return w;
}

// The 8-symbol chain on a window read at q = pm1: e[k] receives the LUT
// entries (gathers issued, not waited for); returns the bits consumed.
__device__ __forceinline__ uint32_t decode_chain(const Window& W, uint32_t q, uint32_t sh_lo,
                                                 uint32_t sh_hi, const uint32_t* __restrict__ lut,
                                                 uint32_t (&e)[8]) {
  const uint32_t w0 = __builtin_bswap32(W.w0), w1 = __builtin_bswap32(W.w1);
  const uint32_t w2 = __builtin_bswap32(W.w2), w3 = __builtin_bswap32(W.w3);
  const uint32_t sh0 = ~q;  // alignbit uses the low 5 bits: 32 - (pos & 31), or 0
  uint32_t A = __builtin_amdgcn_alignbit(w0, w1, sh0);
  uint32_t B = __builtin_amdgcn_alignbit(w1, w2, sh0);
  uint32_t Cw = __builtin_amdgcn_alignbit(w2, w3, sh0);
  uint32_t ssum = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t sel = __builtin_amdgcn_alignbit(kAreaSel, A, 29);
    const uint32_t sft = __builtin_amdgcn_perm(sh_hi, sh_lo, sel);  // 29 - width
    e[k] = lut[A >> sft];
    A = __builtin_amdgcn_alignbit(A, B, sft);
    B = __builtin_amdgcn_alignbit(B, Cw, sft);
    Cw = __builtin_amdgcn_alignbit(Cw, 0u, sft);
    ssum += sft;
  }
  return 256u - ssum;
}

// The 8 decoded bytes packed little-endian; the entries' invalid flags are
// accumulated in errbits.
__device__ __forceinline__ uint2 pack_group(const uint32_t (&e)[8], uint32_t& errbits) {
  uint2 r;
  r.x = __builtin_amdgcn_perm(e[1], e[0], 0x0C0C0400u) | __builtin_amdgcn_perm(e[3], e[2], 0x04000C0Cu);
  r.y = __builtin_amdgcn_perm(e[5], e[4], 0x0C0C0400u) | __builtin_amdgcn_perm(e[7], e[6], 0x04000C0Cu);
  errbits |= e[0] | e[1] | e[2] | e[3] | e[4] | e[5] | e[6] | e[7];
  return r;
}

// Eight decoded symbols (one per byte of r, in order) in the output format
// of the alphabet: bytes (8-bit symbols), four bytes of nibbles (symbol 2k
// in the low nibble of byte k), or six bytes of 6-bit fields in
// little-endian bit order (low word, then the low 16 bits of the high one).
__device__ __forceinline__ uint32_t six_pack(uint32_t x) {
  return (x & 0x3Fu) | ((x >> 2) & 0xFC0u) | ((x >> 4) & 0x3F000u) | ((x >> 6) & 0xFC0000u);
}
template <int kBits>
__device__ __forceinline__ uint2 pack_out(uint2 r) {
  if (kBits == 8) return r;
  if (kBits == 4) {
    const uint32_t t0 = r.x | (r.x >> 4), t1 = r.y | (r.y >> 4);
    return make_uint2(__builtin_amdgcn_perm(t1, t0, 0x06040200u), 0u);
  }
  const uint32_t lo = six_pack(r.x), hi = six_pack(r.y);
  return make_uint2(lo | (hi << 24), hi >> 8);
}

// Store one group's kBits output bytes (from pack_out) at byte address p
// (a multiple of kBits).
template <int kBits>
__device__ __forceinline__ void store_group(QLC_GLOBAL uint8_t* p, uint2 v) {
  if (kBits == 8) {
    gstore_u2(p, v);
  } else if (kBits == 4) {
    *(QLC_GLOBAL uint32_t*)p = v.x;
  } else if (((uintptr_t)p & 3u) == 0) {  // 6 bytes: word + half, or half + word
    *(QLC_GLOBAL uint32_t*)p = v.x;
    *(QLC_GLOBAL uint16_t*)(p + 4) = (uint16_t)v.y;
  } else {
    *(QLC_GLOBAL uint16_t*)p = (uint16_t)v.x;
    *(QLC_GLOBAL uint32_t*)(p + 2) = (v.x >> 16) | (v.y << 16);
  }
}

// Workgroup barrier that orders LDS accesses only: global loads in flight
// stay in flight across it (__syncthreads() would wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Copy a table (device memory, 16-byte aligned) into LDS: one 16-byte load
// per lane of the first 68 lanes, so the LUT build below reads LDS instead
// of waiting on a global load for every entry.  The caller synchronises
// before reading the copy.
static_assert(sizeof(qlc_table) % 16 == 0, "table copied in 16-byte pieces");
__device__ __forceinline__ void table_to_lds(const qlc_table* __restrict__ t, qlc_table* s,
                                             uint32_t tid) {
  if (tid < sizeof(qlc_table) / 16) ((uint4*)s)[tid] = ((const uint4*)t)[tid];
}

// Code -> symbol LUT of `table` into `lut` (2048 32-bit entries, bit 15 =
// invalid suffix) and the shift table indexed by the window's top three
// bits (byte i of sh_hi:sh_lo = 32 - prefix bits - width of the area the
// top bits name).  A table whose areas 4..7 (or 2..7) are marked 0xFF has a
// 2-bit (1-bit) area code: top bits 2a and 2a + 1 (4a .. 4a + 3) all name
// area a, so the decode chain is the same for every prefix width.  Any
// block size; every thread of the block calls it (it may synchronise the
// block), and the caller synchronises again before using the LUT.
// The per-area fields of a table (width, offset, first, count: 48
// contiguous bytes), read with three 16-byte loads.
static_assert(offsetof(qlc_table, width) == 1024 && offsetof(qlc_table, offset) == 1032 &&
                  offsetof(qlc_table, first) == 1040 && offsetof(qlc_table, count) == 1056,
              "table layout");
struct AreaFields {
  uint32_t p, na;                   // area-code bits, areas
  uint32_t w[8], off[8], first[8], cnt[8];
};
__device__ __forceinline__ AreaFields read_areas(const qlc_table* __restrict__ table) {
  const uint4* q = (const uint4*)&table->width[0];
  const uint4 a = q[0], b = q[1], c = q[2];
  AreaFields f;
  const uint32_t wd[2] = {a.x, a.y}, of[2] = {a.z, a.w};
  const uint32_t fi[4] = {b.x, b.y, b.z, b.w}, co[4] = {c.x, c.y, c.z, c.w};
  const uint32_t w4 = (wd[1] & 0xFFu), w2 = (wd[0] >> 16) & 0xFFu;
  f.p = w4 != 0xFFu ? 3u : w2 != 0xFFu ? 2u : 1u;
  f.na = 1u << f.p;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t wk = (wd[k >> 2] >> (8 * (k & 3))) & 0xFFu;
    f.w[k] = (uint32_t)k < f.na ? (wk < 8 ? wk : 8u) : 0u;  // keeps codes < 2048
    f.off[k] = (of[k >> 2] >> (8 * (k & 3))) & 0xFFu;
    f.first[k] = (fi[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
    f.cnt[k] = (uint32_t)k < f.na ? (co[k >> 1] >> (16 * (k & 1))) & 0xFFFFu : 0u;
  }
  return f;
}

__device__ __forceinline__ void build_dec_lut(const qlc_table* __restrict__ table, uint32_t* lut,
                              uint32_t& sh_lo, uint32_t& sh_hi) {
  sh_lo = 0;
  sh_hi = 0;
  const AreaFields A = read_areas(table);
  const uint32_t p = A.p, na = A.na;
  uint32_t lo[8];
  bool layered = true;  // widths non-decreasing, rank ranges back to back
  uint32_t f = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    lo[a] = (uint32_t)a << A.w[a];
    if ((uint32_t)a < na) {
      layered = layered && A.first[a] == f && (a == 0 || A.w[a] >= A.w[a - 1]);
      f += A.cnt[a];
    }
  }
  layered = layered && f <= 256;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // area named by top bits i: i >> (3 - p), selected without indexing
    // the array by a run-time value (which would put it in scratch memory)
    const uint32_t wi = p == 3 ? A.w[i] : p == 2 ? A.w[i >> 1] : A.w[i >> 2];
    const uint32_t sft = 32u - p - wi;
    if (i < 4) sh_lo |= sft << (8 * i);
    else sh_hi |= sft << (8 * (i - 4));
  }
  if (layered) {
    // Areas' code ranges are disjoint and every rank lies in one area, so
    // each rank's code is its own LUT entry: clear, then one write per rank.
    for (uint32_t c = threadIdx.x; c < 2048; c += blockDim.x) lut[c] = 0x8000;
    lds_barrier();
    for (uint32_t r = threadIdx.x; r < f; r += blockDim.x) {
      uint32_t a = 0;
#pragma unroll
      for (int k = 1; k < 8; ++k) a += ((uint32_t)k < na && A.first[k] <= r) ? 1u : 0u;
      uint32_t wa = A.w[0], oa = A.off[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        wa = a == (uint32_t)k ? A.w[k] : wa;
        oa = a == (uint32_t)k ? A.off[k] : oa;
      }
      const uint32_t suffix = r - oa;
      if (suffix < (1u << wa)) lut[(a << wa) + suffix] = table->rank_to_sym[r];
    }
  } else {
    // Any other table: per entry, the last area whose range holds the code
    // and whose rank is valid.
    for (uint32_t c = threadIdx.x; c < 2048; c += blockDim.x) {
      uint32_t e = 0x8000;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (c >= lo[a] && c < lo[a] + (1u << A.w[a])) {
          const uint32_t rank = A.off[a] + (c - lo[a]);
          if (rank >= A.first[a] && rank < A.first[a] + A.cnt[a] && rank < 256)
            e = table->rank_to_sym[rank];
        }
      }
      lut[c] = e;
    }
  }
}

// Decode chunk group `grp` of an n-symbol stream: chunks kDecThreads*grp
// onwards, one per lane (tid = threadIdx.x); S.lut holds the code -> symbol
// LUT.  Returns true in a lane whose chunk is corrupt (or whose index
// entries are inconsistent).
template <int kBits>
__device__ __forceinline__ bool decode_block(const uint8_t* __restrict__ bits, uint64_t total,
                             const uint64_t* __restrict__ index_p, uint32_t log2_chunk, uint64_t n,
                             uint8_t* __restrict__ out_p, uint64_t grp, uint32_t sh_lo,
                             uint32_t sh_hi, DecSmem& S, uint32_t tid) {
  const QLC_GLOBAL uint64_t* __restrict__ index = (const QLC_GLOBAL uint64_t*)index_p;
  QLC_GLOBAL uint8_t* __restrict__ out = (QLC_GLOBAL uint8_t*)out_p;
  const uint32_t lane = tid & 63;
  const uint32_t C = 1u << log2_chunk;
  const uint64_t nchunks = (n + C - 1) >> log2_chunk;
  const uint64_t j = grp * kDecThreads + tid;
  const uint64_t j_wave = grp * kDecThreads +
                          (uint64_t)(__builtin_amdgcn_readfirstlane(tid) & ~63u);
  bool bad = false;

  if (j_wave < nchunks) {
    // Buffer resource rebased at the wave's first superblock (32-byte aligned):
    // loads past the end of the stream, or through a corrupt index, return
    // zeros.
    const uint64_t stream_bytes = ((total + 31) >> 5) << 2;
    const uint64_t wave_bit = index[j_wave];
    const uint64_t base_sb =
        (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(wave_bit >> kSbLog2Bits)) |
        ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(wave_bit >> (32 + kSbLog2Bits))) << 32);
    const uint64_t base_byte = base_sb << (kSbLog2Bits - 3);
    uint64_t avail = stream_bytes > base_byte ? stream_bytes - base_byte : 0;
    if (avail > kOobOffset) avail = kOobOffset;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(bits + (base_byte < stream_bytes ? base_byte : 0)), (short)0,
        (int)(uint32_t)avail, 0x00020000);

    // Per-lane state.  Lanes past the last chunk, or whose index entries
    // are inconsistent, load nothing and keep none of what they decode, but
    // still take part in the wave's uniform refill / flush schedule.
    uint32_t my_groups = 0, rem = 0;
    uint64_t pos0 = 0, end = 0;
    if (j < nchunks) {
      pos0 = index[j];
      end = (j + 1 < nchunks) ? index[j + 1] : total;
      const uint64_t left = n - (j << log2_chunk);
      const uint32_t nsym = (uint32_t)(left < C ? left : C);
      if (pos0 > end || end > total || (j == 0 && pos0 != 0) || pos0 < wave_bit ||
          ((pos0 >> kSbLog2Bits) - base_sb) > (kOobOffset >> (kSbLog2Bits - 3)) - 4096) {
        bad = true;
      } else {
        my_groups = nsym >> 3;
        rem = nsym & 7;
      }
    }
    const bool live = (j < nchunks) && !bad;
    DecLane L;
    L.ring = S.ring + tid;
    L.pm1 = (live ? pos0 : 0) - 1;
    L.sh_lo = sh_lo;
    L.sh_hi = sh_hi;
    L.errbits = 0;
    const uint32_t sb0 = (uint32_t)base_sb;         // ring slots follow absolute superblocks
    uint32_t fsb = live ? (uint32_t)((pos0 >> kSbLog2Bits) - base_sb) : 0;  // next superblock (wave-relative)
    {
      constexpr uint32_t kSh = kSbLog2Bits - 3;
      const Superblock p0 = load_sb(rsrc, live ? (fsb << kSh) : kOobOffset);
      const Superblock p1 = load_sb(rsrc, live ? ((fsb + 1) << kSh) : kOobOffset);
      const Superblock p2 = load_sb(rsrc, live ? ((fsb + 2) << kSh) : kOobOffset);
      const Superblock p3 = load_sb(rsrc, live ? ((fsb + 3) << kSh) : kOobOffset);
      ring_put(L.ring, sb0 + fsb, p0);
      ring_put(L.ring, sb0 + fsb + 1, p1);
      ring_put(L.ring, sb0 + fsb + 2, p2);
      ring_put(L.ring, sb0 + fsb + 3, p3);
      fsb += 4;
    }
    const uint64_t rel0 = base_sb << kSbLog2Bits;
    Superblock pa, pb;
    uint32_t sba = 0, sbb = 0;
    bool va = false, vb = false;
    uint2* stage = S.stage + tid * kStageGroups;
    QLC_GLOBAL uint8_t* o = out + (((j << log2_chunk) * kBits) >> 3);
    // all lanes of the wave run the same number of groups
    const uint32_t wave_groups = (uint32_t)(C >> 3);

    // Waves whose 64 chunks are all whole and valid (all but at most the
    // last wave) take a branch-free path with four register sets in
    // rotation: a superblock is written to the ring four groups after its
    // load was issued.  Every kStageGroups groups the wave stores its 64
    // lanes' output runs (8 * kStageGroups bytes each), kStageGroups
    // consecutive lanes per run.
    const bool full_wave = __all(live && my_groups == wave_groups);
    if (full_wave) {
      Superblock pc_, pd_;
      uint32_t sbc = 0, sbd = 0;
      bool vc = false, vd = false;
      // bytes: R lanes per output run, one group each; sub-byte symbols: R / 2
      // lanes per run, two groups (8 or 12 bytes) each
      constexpr uint32_t R = kStageGroups;              // groups per flush
      constexpr uint32_t kGpl = kBits == 8 ? 1u : 2u;   // groups per lane per store
      constexpr uint32_t kLpr = R / kGpl;               // lanes per run
      constexpr uint32_t kRuns = 64 / kLpr;             // runs per store instruction
      const uint32_t part = lane % kLpr;
      QLC_GLOBAL uint8_t* obase =
          out + ((((j_wave + lane / kLpr) << log2_chunk) * kBits) >> 3) + part * kGpl * kBits;
      // Software pipelined: the next group's window is read right after the
      // current chain (and after the ring write it may depend on), so its
      // LDS latency overlaps the current group's LUT gathers and packing.
      // Positions are 32-bit, relative to the wave's first superblock.
      uint32_t q = (uint32_t)(L.pm1 - rel0);
      const uint32_t endr = (uint32_t)(end - rel0);  // no superblock past the chunk's end
      const uint32_t* ring = L.ring;
      const uint32_t rs = (uint32_t)base_sb & 3u;  // ring slot of relative superblock 0
      Window W = window_read(ring, q + (rs << kSbLog2Bits));
#define QLC_DEC_UNIT(GI, VAL, SBX, PX)                                                  \
  {                                                                                     \
    uint32_t e[8];                                                                      \
    q += decode_chain(W, q, L.sh_lo, L.sh_hi, S.lut, e);                                \
    if (VAL) ring_put(L.ring, sb0 + SBX, PX);                                           \
    W = window_read(ring, q + (rs << kSbLog2Bits));                                     \
    VAL = (fsb << kSbLog2Bits) < min(q + 1 + kLookaheadBits, endr);                     \
    SBX = fsb;                                                                          \
    PX = load_sb(rsrc, VAL ? (fsb << (kSbLog2Bits - 3)) : kOobOffset);                  \
    fsb += VAL ? 1u : 0u;                                                               \
    stage[stage_slot((GI), tid)] = pack_out<kBits>(pack_group(e, L.errbits));           \
  }
      // One iteration = R groups and their flush, so that the flush sits at
      // a fixed program point: the waits for loads issued before it then
      // need not wait for its stores as well.
#pragma unroll 1
      for (uint32_t g0 = 0; g0 < wave_groups; g0 += R) {
#pragma unroll
        for (uint32_t u = 0; u < R; u += 4) {
          QLC_DEC_UNIT(g0 + u + 0, va, sba, pa)
          QLC_DEC_UNIT(g0 + u + 1, vb, sbb, pb)
          QLC_DEC_UNIT(g0 + u + 2, vc, sbc, pc_)
          QLC_DEC_UNIT(g0 + u + 3, vd, sbd, pd_)
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (uint32_t k = 0; k < kLpr; ++k) {
          const uint32_t stid = (tid & ~63u) | (lane / kLpr + kRuns * k);
          QLC_GLOBAL uint8_t* dst =
              obase + ((((uint64_t)(kRuns * k) << log2_chunk) * kBits) >> 3) + g0 * kBits;
          if (kBits == 8) {
            gstore_u2(dst, S.stage[stid * R + stage_slot(g0 + part, stid)]);
          } else {
            const uint2 a = S.stage[stid * R + stage_slot(g0 + 2 * part, stid)];
            const uint2 b = S.stage[stid * R + stage_slot(g0 + 2 * part + 1, stid)];
            if (kBits == 4) {
              gstore_u2(dst, make_uint2(a.x, b.x));
            } else {  // 12 bytes at a multiple of 12
              QLC_GLOBAL uint32_t* d32 = (QLC_GLOBAL uint32_t*)dst;
              d32[0] = a.x;
              d32[1] = (a.y & 0xFFFFu) | (b.x << 16);
              d32[2] = (b.x >> 16) | (b.y << 16);
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
#undef QLC_DEC_UNIT
      L.pm1 = rel0 + q;
      if (vc) ring_put(L.ring, sb0 + sbc, pc_);
      if (vd) ring_put(L.ring, sb0 + sbd, pd_);
    } else {
      // Any other wave (chunks past the end, a short last chunk, an invalid
      // chunk): the same schedule with two register sets, every lane running
      // the wave's full count of groups but keeping only its own: its
      // position stops where its last group ends (later groups decode that
      // place again), a lane without a chunk loads nothing, and discarded
      // groups count no errors and are not stored.  The group counts are
      // wave-uniform: all (lanes in full_lanes), none, or part_groups in
      // lane part_lane (the short last chunk, the only count in between).
      constexpr uint32_t R = kStageGroups;
      constexpr uint32_t kGpl = kBits == 8 ? 1u : 2u;
      constexpr uint32_t kLpr = R / kGpl;
      constexpr uint32_t kRuns = 64 / kLpr;
      const uint32_t part = lane % kLpr;
      QLC_GLOBAL uint8_t* obase =
          out + ((((j_wave + lane / kLpr) << log2_chunk) * kBits) >> 3) + part * kGpl * kBits;
      const uint64_t full_lanes = __ballot(my_groups == wave_groups);
      const uint64_t pm = __ballot(my_groups != 0 && my_groups != wave_groups);
      const uint32_t part_lane = pm ? (uint32_t)__builtin_ctzll(pm) : 64u;
      const uint32_t part_groups =
          pm ? (uint32_t)__builtin_amdgcn_readlane((int)my_groups, (int)part_lane) : 0u;
      uint32_t q = (uint32_t)(L.pm1 - rel0);
      const uint32_t endr = live ? (uint32_t)(end - rel0) : 0u;
      const uint32_t* ring = L.ring;
      const uint32_t rs = (uint32_t)base_sb & 3u;
      Window W = window_read(ring, q + (rs << kSbLog2Bits));
#define QLC_DEC_UNIT_P(GI, VAL, SBX, PX)                                                \
  {                                                                                     \
    uint32_t e[8];                                                                      \
    const uint32_t adv = decode_chain(W, q, L.sh_lo, L.sh_hi, S.lut, e);                \
    const bool keep = (GI) < my_groups;                                                 \
    q += keep ? adv : 0u;                                                               \
    if (VAL) ring_put(L.ring, sb0 + SBX, PX);                                           \
    W = window_read(ring, q + (rs << kSbLog2Bits));                                     \
    VAL = (fsb << kSbLog2Bits) < min(q + 1 + kLookaheadBits, endr);                     \
    SBX = fsb;                                                                          \
    PX = load_sb(rsrc, VAL ? (fsb << (kSbLog2Bits - 3)) : kOobOffset);                  \
    fsb += VAL ? 1u : 0u;                                                               \
    uint32_t eb = 0;                                                                    \
    stage[stage_slot((GI), tid)] = pack_out<kBits>(pack_group(e, eb));                  \
    L.errbits |= keep ? eb : 0u;                                                        \
  }
#pragma unroll 1
      for (uint32_t g0 = 0; g0 < wave_groups; g0 += R) {
#pragma unroll
        for (uint32_t u = 0; u < R; u += 2) {
          QLC_DEC_UNIT_P(g0 + u + 0, va, sba, pa)
          QLC_DEC_UNIT_P(g0 + u + 1, vb, sbb, pb)
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (uint32_t k = 0; k < kLpr; ++k) {
          const uint32_t src = lane / kLpr + kRuns * k;  // lane (chunk) whose run is stored
          const uint32_t stid = (tid & ~63u) | src;
          const uint32_t ngrp = ((full_lanes >> src) & 1u) ? wave_groups
                                : src == part_lane ? part_groups : 0u;
          QLC_GLOBAL uint8_t* dst =
              obase + ((((uint64_t)(kRuns * k) << log2_chunk) * kBits) >> 3) + g0 * kBits;
          if (kBits == 8) {
            if (g0 + part < ngrp) gstore_u2(dst, S.stage[stid * R + stage_slot(g0 + part, stid)]);
          } else {
            // two groups (8 or 12 bytes at a multiple of 8 or 12), or only
            // the first when it is the chunk's last whole group
            const uint32_t ga = g0 + 2 * part;
            const uint2 a = S.stage[stid * R + stage_slot(ga, stid)];
            const uint2 b = S.stage[stid * R + stage_slot(ga + 1, stid)];
            QLC_GLOBAL uint32_t* d32 = (QLC_GLOBAL uint32_t*)dst;
            if (ga < ngrp) d32[0] = a.x;
            if (ga + 1 < ngrp) {
              if (kBits == 4) {
                d32[1] = b.x;
              } else {
                d32[1] = (a.y & 0xFFFFu) | (b.x << 16);
                d32[2] = (b.x >> 16) | (b.y << 16);
              }
            } else if (kBits == 6 && ga < ngrp) {
              *(QLC_GLOBAL uint16_t*)(dst + 4) = (uint16_t)a.y;
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
#undef QLC_DEC_UNIT_P
      // a lane that decoded no group keeps its 64-bit position (q holds it
      // modulo 2^32, which for the stream's first bit, pm1 = -1, is not it)
      if (my_groups) L.pm1 = rel0 + q;
    }
    if (va) ring_put(L.ring, sb0 + sba, pa);
    if (vb) ring_put(L.ring, sb0 + sbb, pb);
    if (live && rem) {  // final partial group of the last chunk
      const uint32_t q = (uint32_t)L.pm1;
      const uint32_t wi = (q >> 5) & 31u;
      const uint32_t* rr = L.ring + wi * kDecLanes;
      const uint32_t w0 = __builtin_bswap32(rr[0]), w1 = __builtin_bswap32(rr[kDecLanes]);
      const uint32_t w2 = __builtin_bswap32(rr[2 * kDecLanes]), w3 = __builtin_bswap32(rr[3 * kDecLanes]);
      uint32_t A = __builtin_amdgcn_alignbit(w0, w1, ~q);
      uint32_t B = __builtin_amdgcn_alignbit(w1, w2, ~q);
      uint32_t Cw = __builtin_amdgcn_alignbit(w2, w3, ~q);
      uint64_t acc = 0;  // the partial group, packed (sub-byte symbols)
      for (uint32_t k = 0; k < rem; ++k) {
        const uint32_t sel = __builtin_amdgcn_alignbit(kAreaSel, A, 29);
        const uint32_t s = __builtin_amdgcn_perm(sh_hi, sh_lo, sel);
        const uint32_t e = S.lut[A >> s];
        L.errbits |= e;
        if (kBits == 8) o[my_groups * 8 + k] = (uint8_t)e;
        else acc |= (uint64_t)(e & 0xFFu) << (k * kBits);
        A = __builtin_amdgcn_alignbit(A, B, s);
        B = __builtin_amdgcn_alignbit(B, Cw, s);
        Cw = __builtin_amdgcn_alignbit(Cw, 0u, s);
        L.pm1 += 32u - s;
      }
      if (kBits != 8) {  // whole bytes; the last one zero padded
        QLC_GLOBAL uint8_t* d = o + my_groups * kBits;
        for (uint32_t b = 0; b < (rem * kBits + 7) / 8; ++b) d[b] = (uint8_t)(acc >> (8 * b));
      }
    }
    if (live) bad = (L.errbits & 0x8000u) || (L.pm1 + 1 != end);
  }
  return bad;
}

template <int kBits>
__global__ __launch_bounds__(kDecThreads) void k_decode(
    const uint8_t* __restrict__ bits, const uint64_t* __restrict__ total_p,
    const uint64_t* __restrict__ index, uint32_t log2_chunk,
    const qlc_table* __restrict__ table, uint64_t n, uint8_t* __restrict__ out,
    uint32_t* __restrict__ err_out, WsHeader* __restrict__ hdr) {
  __shared__ DecSmem S;
  const uint32_t tid = threadIdx.x;
  uint32_t sh_lo, sh_hi;
  qlc_table* tl = (qlc_table*)S.ring;  // the ring is free until the decode starts
  table_to_lds(table, tl, tid);
  __syncthreads();
  build_dec_lut(tl, S.lut, sh_lo, sh_hi);
  const bool table_ok = mode_symbol_bits(tl->mode) == kBits;
  __syncthreads();
  // a table of another alphabet is refused (nothing decoded)
  if (table_ok) {
    const bool bad = decode_block<kBits>(bits, *total_p, index, log2_chunk, n, out, blockIdx.x,
                                         sh_lo, sh_hi, S, tid);
    set_error_wave(&hdr->dec_err, QLC_ERR_CORRUPT_STREAM, bad);
  } else if (tid == 0) {
    set_error(&hdr->dec_err, QLC_ERR_INVALID_ARGUMENT);
  }

  // ---- error word: first error wins; the last workgroup publishes it ----
  __syncthreads();
  if (tid == 0) {
    const uint32_t done = atomic_add_u32(&hdr->dec_done, 1u);
    if (done == gridDim.x - 1) {
      *err_out = load_relaxed_u32(&hdr->dec_err);
      store_relaxed_u32(&hdr->dec_err, 0);
      store_relaxed_u32(&hdr->dec_done, 0);
    }
  }
}

// ===========================================================================
// Split-chunk decode: several lanes per chunk.
//
// With one lane per chunk (k_decode) a tensor of few chunks leaves the
// device idle: a 1 Mi-symbol tensor at C = 2048 is 512 chunks, i.e. 512
// lanes, each walking 2048 codes one after the other.  Here a workgroup
// takes kSplitSyms (16384) symbols, i.e. 16384 / C whole chunks, and gives
// every chunk G = C / 64 lanes (C <= 16384), about 64 codes per lane:
//   1. the workgroup's stretch of the bitstream is copied into LDS with
//      coalesced 16-byte loads (each stream byte is read once);
//   2. lane g of a chunk takes the g-th of G equal pieces of the chunk's
//      bits and walks code lengths only (a code's length follows from its
//      area code alone), starting kSplitWarmBits before its piece as if a
//      code began there (a guess; exact for g = 0).  Walks of a prefix code
//      from a wrong start soon fall onto the true boundaries, so the walk
//      usually enters the piece in step with them.  The lane owns the codes
//      that start in its piece; it records where its walk enters and leaves
//      the piece and how many codes it passed in between;
//   3. correction rounds: a lane whose start differs from the point where
//      the previous lane's walk left the previous piece walks again from
//      that point, in step with its old path, until the two paths meet
//      (from there on they coincide) or the piece ends.  After round r the
//      first r + 1 lanes of every chunk are exact; the rounds stop when no
//      lane's exit changed, so after at most G + 1 rounds, and in practice
//      the two paths meet within a few codes and one round suffices;
//   4. a scan of the code counts gives every lane the position of its first
//      symbol; the lane decodes its codes through the code-word LUT into an
//      LDS copy of the workgroup's output, which is then stored with
//      coalesced stores.
// If every code length is a multiple of d (the gcd of the lengths of the
// areas in use), code starts lie d apart from the chunk's start and the
// guesses are rounded to that grid: a table whose codes all have one length
// needs no correction at all.  A chunk is reported corrupt under the same
// conditions as in k_decode: its codes do not end exactly where the next
// chunk begins (or at the stream's end) after its symbol count, a suffix
// lies outside its area, or its index entries are out of order.
// ===========================================================================
constexpr int kSplitThreads = 256;
constexpr uint32_t kSplitLog2Syms = kSplitMaxLog2Chunk;      // symbols per workgroup
constexpr uint32_t kSplitSyms = 1u << kSplitLog2Syms;
constexpr uint32_t kMaxCodeBits = 11;                         // 3-bit area code + 8-bit suffix
constexpr uint32_t kSplitCapBits = kSplitSyms * kMaxCodeBits + 128;  // + alignment of the base
constexpr uint32_t kSplitPadWords = 4;                        // zero words before the stream copy
constexpr uint32_t kSplitLoadWords = ((kSplitCapBits + 31) / 32 + 4 + 3) & ~3u;
constexpr uint32_t kSplitSpanWords = kSplitPadWords + kSplitLoadWords;
constexpr uint32_t kSplitLoadsPerLane = (kSplitLoadWords / 4 + kSplitThreads - 1) / kSplitThreads;
constexpr uint32_t kSplitQOff = kSplitPadWords * 32 - 1;      // LDS bit of stream bit 0, minus one
constexpr uint32_t kSplitMaxChunks = kSplitSyms >> 8;         // chunks per workgroup at C = 256
constexpr uint32_t kSplitWarmBits = 512;                      // walked before a piece, not counted

struct SplitSmem {
  uint32_t lut[2048];
  uint32_t span[kSplitSpanWords];         // stream words from base_bit on (memory byte order)
  uint8_t out[kSplitSyms];                // decoded symbols, one per byte
  uint32_t xs[2][kSplitThreads];          // walk exits, by round parity
  uint32_t excl[kSplitThreads];           // exclusive scan of the code counts
  uint32_t wsum[kSplitThreads / 64];
  uint32_t chunk_bad[kSplitMaxChunks];
  uint32_t any[3];                        // correction rounds: some exit changed
};

static_assert(offsetof(SplitSmem, span) % 16 == 0 && offsetof(SplitSmem, out) % 16 == 0,
              "16-byte LDS accesses");
static_assert(sizeof(SplitSmem) * 3 <= 160 * 1024, "three workgroups per CU");

// Length of the code starting at stream bit `rel` (relative to the copy).
__device__ __forceinline__ uint32_t split_code_len(const uint32_t* span, uint32_t rel,
                                                   uint32_t sh_lo, uint32_t sh_hi) {
  const uint32_t q = rel + kSplitQOff;
  const uint32_t w0 = __builtin_bswap32(span[q >> 5]), w1 = __builtin_bswap32(span[(q >> 5) + 1]);
  const uint32_t A = __builtin_amdgcn_alignbit(w0, w1, ~q);
  const uint32_t sel = __builtin_amdgcn_alignbit(kAreaSel, A, 29);
  return 32u - __builtin_amdgcn_perm(sh_hi, sh_lo, sel);
}

// The four words holding stream bits rel .. rel + 95 (and q for the chain).
__device__ __forceinline__ Window split_window(const uint32_t* span, uint32_t rel, uint32_t& q) {
  q = rel + kSplitQOff;
  const uint32_t* rr = span + (q >> 5);
  Window w;
  w.w0 = rr[0];
  w.w1 = rr[1];
  w.w2 = rr[2];
  w.w3 = rr[3];
  return w;
}

// Walk code lengths from x while x < end: returns the first code start at
// or past end and adds the codes passed to cnt.
__device__ __forceinline__ uint32_t split_walk(const uint32_t* span, uint32_t x, uint32_t end,
                                               uint32_t sh_lo, uint32_t sh_hi, uint32_t& cnt) {
  while (x < end) {
    uint32_t q;
    const Window W = split_window(span, x, q);
    const uint32_t w0 = __builtin_bswap32(W.w0), w1 = __builtin_bswap32(W.w1);
    const uint32_t w2 = __builtin_bswap32(W.w2), w3 = __builtin_bswap32(W.w3);
    uint32_t A = __builtin_amdgcn_alignbit(w0, w1, ~q);
    uint32_t B = __builtin_amdgcn_alignbit(w1, w2, ~q);
    uint32_t Cw = __builtin_amdgcn_alignbit(w2, w3, ~q);
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // at most 88 of the window's 96 bits
      const uint32_t sel = __builtin_amdgcn_alignbit(kAreaSel, A, 29);
      const uint32_t sft = __builtin_amdgcn_perm(sh_hi, sh_lo, sel);
      const bool act = x < end;  // once past the end, x stays there
      x += act ? 32u - sft : 0u;
      cnt += act ? 1u : 0u;
      A = __builtin_amdgcn_alignbit(A, B, sft);
      B = __builtin_amdgcn_alignbit(B, Cw, sft);
      Cw = __builtin_amdgcn_alignbit(Cw, 0u, sft);
    }
  }
  return x;
}

// gcd of the code lengths of the areas that hold symbols: the largest k
// that divides every length (lengths are at most kMaxCodeBits).
__device__ __forceinline__ uint32_t code_length_gcd(const qlc_table* __restrict__ table) {
  const AreaFields A = read_areas(table);
  uint32_t lens = 0;  // bit L set: some area has codes of length L
#pragma unroll
  for (uint32_t a = 0; a < 8; ++a)
    if (a < A.na && A.cnt[a] != 0) lens |= 1u << (A.p + A.w[a]);
  uint32_t d = 1;
#pragma unroll
  for (uint32_t k = 2; k <= kMaxCodeBits; ++k) {
    uint32_t mult = 0;
#pragma unroll
    for (uint32_t m = k; m <= kMaxCodeBits; m += k) mult |= 1u << m;
    if (lens != 0 && (lens & ~mult) == 0) d = k;
  }
  return d;
}

// The LUT of a split decode and what the walks need from the table.
struct SplitLut {
  uint32_t sh_lo, sh_hi;  // shift table (see build_dec_lut)
  uint32_t d;             // gcd of the code lengths in use
  bool ok;                // the table codes this alphabet
};

// Decode split unit `unit` (symbols unit * 16384 onwards) of an n-symbol
// stream with all 256 threads of the block (tid = threadIdx.x).  With
// `table` given, the LUT is built into S.lut and L set (while the stream's
// loads are in flight); with table == nullptr, S.lut and L hold a LUT built
// before.  Stores the unit's symbols; returns true in the lanes of a corrupt
// chunk.  Nothing is decoded or stored if L.ok is false.
template <int kBits>
__device__ __forceinline__ bool split_block(const uint8_t* __restrict__ bits, uint64_t total,
                                            const uint64_t* __restrict__ index_p,
                                            uint32_t log2_chunk, uint64_t n,
                                            uint8_t* __restrict__ out_p, uint64_t unit,
                                            const qlc_table* __restrict__ table, SplitLut& L,
                                            SplitSmem& S, uint32_t tid) {
  const QLC_GLOBAL uint64_t* __restrict__ index = (const QLC_GLOBAL uint64_t*)index_p;
  // a table to build the LUT from: its copy goes to the output buffer
  // (free until the decode); its load is issued first and written after the
  // stream's loads
  qlc_table* tl = (qlc_table*)S.out;
  const bool tab_lane = table != nullptr && tid < sizeof(qlc_table) / 16;
  const uint4 tv = tab_lane ? ((const uint4*)table)[tid] : make_uint4(0, 0, 0, 0);
  if (tid < kSplitPadWords) S.span[tid] = 0;
  if (tid < 3) S.any[tid] = 0;
  if (tid < kSplitMaxChunks) S.chunk_bad[tid] = 0;

  const uint32_t C = 1u << log2_chunk;
  const uint32_t log2_g = log2_chunk - 6;                 // G = C / 64 lanes per chunk
  const uint32_t G = 1u << log2_g;
  const uint32_t g = tid & (G - 1);
  const uint32_t slot = tid >> log2_g;                    // chunk slot in the workgroup
  const uint64_t nchunks = (n + C - 1) >> log2_chunk;
  const uint64_t j0 = unit << (kSplitLog2Syms - log2_chunk);
  const uint64_t j = j0 + slot;
  // this lane's index entries, loaded with the span's
  uint64_t s_abs = 0, e_abs = 0;
  if (j < nchunks) {
    s_abs = index[j];
    e_abs = j + 1 < nchunks ? index[j + 1] : total;
  }

  // ---- the workgroup's stretch of the stream ----
  uint64_t base_bit = 0, hi = 0;
  if (j0 < nchunks) {
    const uint64_t s0 = index[j0];
    base_bit = (((s0 < total ? s0 : total) >> 3) & ~15ull) << 3;
    const uint64_t jl = (j0 + (kSplitSyms >> log2_chunk) < nchunks ? j0 + (kSplitSyms >> log2_chunk)
                                                                  : nchunks) - 1;
    hi = jl + 1 < nchunks ? index[jl + 1] : total;
    if (hi < base_bit) hi = base_bit;
    if (hi - base_bit > kSplitCapBits) hi = base_bit + kSplitCapBits;
  }
  // the table's copy first, then the stream's loads, which stay in flight
  // while the LUT is built
  if (tab_lane) ((uint4*)tl)[tid] = tv;
  const uint32_t nvec =
      j0 < nchunks ? (uint32_t)((((hi - base_bit + 31) >> 5) + 4 + 3) >> 2) : 0u;
  uint4 sv[kSplitLoadsPerLane];
  {
    const uint64_t stream_bytes = ((total + 31) >> 5) << 2;
    const uint64_t base_byte = base_bit >> 3;
    uint64_t avail = stream_bytes > base_byte ? stream_bytes - base_byte : 0;
    if (avail > (1u << 20)) avail = 1u << 20;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(bits + (base_byte < stream_bytes ? base_byte : 0)), (short)0, (int)(uint32_t)avail,
        0x00020000);
#pragma unroll
    for (uint32_t k = 0; k < kSplitLoadsPerLane; ++k) {
      const uint32_t i = tid + k * kSplitThreads;
      sv[k] = bufload16(rsrc, i < nvec ? i * 16 : kOobOffset);
    }
  }
  lds_barrier();
  if (table != nullptr) {
    build_dec_lut(tl, S.lut, L.sh_lo, L.sh_hi);
    L.ok = mode_symbol_bits(tl->mode) == kBits;
    L.d = code_length_gcd(tl);
  }
  const uint32_t sh_lo = L.sh_lo, sh_hi = L.sh_hi, d = L.d;
  const bool table_ok = L.ok;
#pragma unroll
  for (uint32_t k = 0; k < kSplitLoadsPerLane; ++k) {
    const uint32_t i = tid + k * kSplitThreads;
    if (i < nvec) *(uint4*)&S.span[kSplitPadWords + 4 * i] = sv[k];
  }
  lds_barrier();

  // ---- this lane's chunk and piece ----
  bool live = false;
  uint32_t s_rel = 0, e_rel = 0, nsym = 0, lo = 0, piece_lo = 0, end = 0;
  if (table_ok && j < nchunks) {
    const uint64_t s = s_abs, e = e_abs;
    const uint64_t left = n - (j << log2_chunk);
    nsym = (uint32_t)(left < C ? left : C);
    live = s <= e && e <= total && (j != 0 || s == 0) && s >= base_bit &&
           e - base_bit <= kSplitCapBits && e - s <= (uint64_t)nsym * kMaxCodeBits;
    if (live) {
      s_rel = (uint32_t)(s - base_bit);
      e_rel = (uint32_t)(e - base_bit);
      const uint32_t len = e_rel - s_rel;
      const uint32_t piece = (len + G - 1) >> log2_g;
      const uint32_t a = min(g * piece, len), b = min((g + 1) * piece, len);
      // the walk starts kSplitWarmBits before the piece (on the d grid of
      // the chunk): by the piece's first bit it has most likely fallen in
      // step with the true code boundaries
      uint32_t u = a > kSplitWarmBits ? a - kSplitWarmBits : 0;
      if (d > 1) u = (u + d - 1) / d * d;
      lo = s_rel + u;
      piece_lo = s_rel + a;
      end = s_rel + b;
    } else {
      S.chunk_bad[slot] = 1;  // every lane of the chunk writes the same
    }
  }

  // ---- phase 1: length walks from the guessed starts ----
  uint32_t start = 0, cnt = 0, x = 0;
  if (live) {
    uint32_t warm = 0;
    start = split_walk(S.span, lo, piece_lo, sh_lo, sh_hi, warm);  // first start in the piece
    x = split_walk(S.span, start, end, sh_lo, sh_hi, cnt);
  }

  // ---- phase 2: correction rounds ----
  S.xs[0][tid] = x;
  lds_barrier();
  for (uint32_t r = 0; r <= kSplitThreads; ++r) {
    const uint32_t prev = g == 0 ? s_rel : S.xs[r & 1][tid - 1];
    bool changed = false;
    if (live && g != 0 && prev != start) {
      // new path from prev, old path from start, in step until they meet
      uint32_t a = prev, b = start, ca = 0, cb = 0;
      bool met = false;
      for (;;) {
        if (a == b) {
          met = true;
          break;
        }
        if (a < b) {
          if (a >= end) break;
          a += split_code_len(S.span, a, sh_lo, sh_hi);
          ++ca;
        } else {
          if (b >= end) break;
          b += split_code_len(S.span, b, sh_lo, sh_hi);
          ++cb;
        }
      }
      const uint32_t nx = met ? x : a;
      cnt = met ? cnt - cb + ca : ca;
      changed = nx != x;
      x = nx;
      start = prev;
    }
    // any lane changed?  (three flag words: the one read after this
    // round's barrier is cleared two rounds later)
    if (tid == 0) S.any[(r + 1) % 3] = 0;
    if (changed) S.any[r % 3] = 1;
    S.xs[(r + 1) & 1][tid] = x;
    lds_barrier();
    if (!S.any[r % 3]) break;
  }

  // ---- phase 3: first symbol of each lane (scan of the counts) ----
  const uint32_t lane = tid & 63, wave = tid >> 6;
  uint32_t incl = cnt;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const uint32_t y = __shfl_up(incl, k, 64);
    if (lane >= (uint32_t)k) incl += y;
  }
  if (lane == 63) S.wsum[wave] = incl;
  lds_barrier();
  for (uint32_t w = 0; w < wave; ++w) incl += S.wsum[w];
  S.excl[tid] = incl - cnt;
  lds_barrier();
  const uint32_t cbase = S.excl[tid - g];
  if (live && g == G - 1 && (incl - cbase != nsym || x != e_rel)) S.chunk_bad[slot] = 1;
  lds_barrier();
  bool bad = table_ok && j < nchunks && S.chunk_bad[slot] != 0;

  // ---- phase 4: decode into the LDS copy of the output ----
  if (live && !bad) {
    uint8_t* dst = S.out + (slot << log2_chunk) + (incl - cnt - cbase);
    uint32_t pos = start, errbits = 0, q;
    Window W = split_window(S.span, pos, q);
    const uint32_t full = cnt >> 3, rem = cnt & 7u;
    for (uint32_t k0 = 0; k0 < full; ++k0, dst += 8) {
      uint32_t e[8];
      pos += decode_chain(W, q, sh_lo, sh_hi, S.lut, e);
      W = split_window(S.span, pos, q);  // the next group's window, read early
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        dst[k] = (uint8_t)e[k];
        errbits |= e[k];
      }
    }
    if (rem) {
      uint32_t e[8];
      decode_chain(W, q, sh_lo, sh_hi, S.lut, e);
#pragma unroll
      for (uint32_t k = 0; k < 7; ++k) {
        if (k < rem) {
          dst[k] = (uint8_t)e[k];
          errbits |= e[k];
        }
      }
    }
    bad = (errbits & 0x8000u) != 0;
  }
  lds_barrier();

  // ---- the workgroup's output, coalesced ----
  const uint64_t sym0 = unit << kSplitLog2Syms;
  if (table_ok && sym0 < n) {
    const uint32_t nsw = (uint32_t)(n - sym0 < kSplitSyms ? n - sym0 : kSplitSyms);
    QLC_GLOBAL uint8_t* o = (QLC_GLOBAL uint8_t*)out_p + ((sym0 * kBits) >> 3);
    if (kBits == 8) {
      for (uint32_t i = tid; i < (nsw >> 4); i += kSplitThreads) {
        const uint4 v = *(const uint4*)&S.out[16 * i];
        GVec4 w;
        w.x = v.x;
        w.y = v.y;
        w.z = v.z;
        w.w = v.w;
        ((QLC_GLOBAL GVec4*)o)[i] = w;
      }
      for (uint32_t i = (nsw & ~15u) + tid; i < nsw; i += kSplitThreads) o[i] = S.out[i];
    } else {
      for (uint32_t i = tid; i < (nsw >> 3); i += kSplitThreads)
        store_group<kBits>(o + i * kBits, pack_out<kBits>(*(const uint2*)&S.out[8 * i]));
      const uint32_t rem = nsw & 7u;
      if (rem && tid == 0) {  // whole bytes; the last one zero padded
        uint64_t acc = 0;
        for (uint32_t k = 0; k < rem; ++k)
          acc |= (uint64_t)S.out[(nsw & ~7u) + k] << (k * kBits);
        QLC_GLOBAL uint8_t* t = o + (nsw >> 3) * kBits;
        for (uint32_t b = 0; b < (rem * kBits + 7) / 8; ++b) t[b] = (uint8_t)(acc >> (8 * b));
      }
    }
  }

  return bad;
}

template <int kBits>
__global__ __launch_bounds__(kSplitThreads) void k_decode_split(
    const uint8_t* __restrict__ bits, const uint64_t* __restrict__ total_p,
    const uint64_t* __restrict__ index_p, uint32_t log2_chunk,
    const qlc_table* __restrict__ table, uint64_t n, uint8_t* __restrict__ out_p,
    uint32_t* __restrict__ err_out, WsHeader* __restrict__ hdr) {
  __shared__ SplitSmem S;
  const uint32_t tid = threadIdx.x;
  SplitLut L;
  const bool bad = split_block<kBits>(bits, *total_p, index_p, log2_chunk, n, out_p, blockIdx.x,
                                      table, L, S, tid);
  set_error_wave(&hdr->dec_err, QLC_ERR_CORRUPT_STREAM, bad);
  if (!L.ok && tid == 0) set_error(&hdr->dec_err, QLC_ERR_INVALID_ARGUMENT);
  lds_barrier();

  // ---- error word: first error wins; the last workgroup publishes it ----
  if (tid == 0) {
    const uint32_t done = atomic_add_u32(&hdr->dec_done, 1u);
    if (done == gridDim.x - 1) {
      *err_out = load_relaxed_u32(&hdr->dec_err);
      store_relaxed_u32(&hdr->dec_err, 0);
      store_relaxed_u32(&hdr->dec_done, 0);
    }
  }
}

// ===========================================================================
// Batched form: many jobs of uneven sizes per launch.
//
// A one-workgroup plan kernel numbers the jobs' work units (encode
// segments of 2^log2_seg symbols, or decode groups of kDecThreads chunks), records
// which job owns each unit and resets the per-call state.  The persistent
// kernels then hand out work items from one atomic ticket counter.
//
// Encode items are, per segment g (all jobs' segments numbered jointly), a
// histogram item H(g) and an encode item E(g).  The ticket order puts the
// first `lag` histogram items first, then alternates E(0), H(lag),
// E(1), H(lag + 1), ..., then the remaining encode items.  With lag at
// least the largest job's segment count, every item an encode item waits
// for (its job's histograms and table, the preceding segments' bit counts)
// has a smaller ticket, so it was taken by a workgroup that is running and
// that waits only on smaller tickets: no deadlock, whatever the grid size.
// ===========================================================================
// threadIdx.x, hidden from loop-invariant code motion: inside the
// persistent loops, values derived from it are recomputed per item instead
// of being held in registers across the whole loop.
__device__ __forceinline__ uint32_t opaque_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ bool ptr_aligned(const void* p, uintptr_t a) {
  return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

__device__ bool job_valid(const qlc_job& jb, bool decode) {
  if (jb.n >= QLC_MAX_SYMBOLS_PER_CALL || jb.reserved != 0) return false;
  if (!jb.table || !ptr_aligned(jb.table, 16) || !jb.total_bits || !ptr_aligned(jb.total_bits, 8))
    return false;
  if (!ptr_aligned(jb.chunk_index, 8) || !ptr_aligned(jb.bits, 16)) return false;
  if (decode) {
    if (jb.n && (!jb.bits || !jb.chunk_index || !jb.out || !ptr_aligned(jb.out, 16))) return false;
  } else {
    if (jb.n && (!jb.in || !ptr_aligned(jb.in, 16) || !jb.chunk_index)) return false;
    if (jb.bits_capacity && !jb.bits) return false;
  }
  return true;
}

constexpr int kPlanThreads = 1024;
constexpr uint32_t kPlanZeroJobs = 16;  // job histograms cleared per extra plan workgroup

// Workgroup 0 plans; workgroups 1.. (encode only) clear the per-job
// histogram accumulators, kPlanZeroJobs jobs each.
__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(
    const qlc_job* __restrict__ jobs, uint32_t n_jobs, uint32_t decode, uint32_t decode_split,
    uint32_t log2_unit,
    uint64_t max_units, uint32_t lag_req, BatchHeader* __restrict__ hdr,
    BatchJobState* __restrict__ js, uint64_t* __restrict__ job_hist,
    uint32_t* __restrict__ unit_job, uint64_t* __restrict__ seg_word) {
  if (blockIdx.x > 0) {
    const uint64_t k0 = (uint64_t)(blockIdx.x - 1) * kPlanZeroJobs;
    const uint64_t k1 = k0 + kPlanZeroJobs < n_jobs ? k0 + kPlanZeroJobs : n_jobs;
    for (uint64_t i = k0 * 256 + threadIdx.x; i < k1 * 256; i += kPlanThreads) job_hist[i] = 0;
    return;
  }
  __shared__ uint64_t wsum[kPlanThreads / 64];
  __shared__ uint32_t wmax[kPlanThreads / 64];
  __shared__ uint64_t total_s;
  __shared__ uint32_t maxc_s;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t per = (n_jobs + kPlanThreads - 1) / kPlanThreads;
  const uint32_t k0 = tid * per < n_jobs ? tid * per : n_jobs;
  const uint32_t k1 = k0 + per < n_jobs ? k0 + per : n_jobs;

  // ---- symbols of the valid jobs, for the automatic work split ----
  if ((!decode && log2_unit == 0) || (decode && decode_split == 1)) {
    uint64_t syms = 0;
    for (uint32_t k = k0; k < k1; ++k) {
      const qlc_job jb = jobs[k];
      if (jb.err && ptr_aligned(jb.err, 4) && job_valid(jb, decode != 0)) syms += jb.n;
    }
    // n < 2^36 per job, and a workspace (2 KiB of histogram per job) holds
    // far fewer than 2^28 jobs: the sum stays below 2^64
    const uint64_t incl = wave_inclusive_scan_u64(syms);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t T = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) T += wsum[w];
    __syncthreads();
    if (!decode) log2_unit = batch_auto_log2_seg(T);
    else if (batch_split_all(T, log2_unit - kDecThreadsLog2)) decode_split = 2;
  }

  // ---- units per job; per-job status reset ----
  uint64_t local = 0;
  uint32_t maxc = 0;
  for (uint32_t k = k0; k < k1; ++k) {
    const qlc_job jb = jobs[k];
    uint32_t cnt = 0, split = 0;
    if (jb.err && ptr_aligned(jb.err, 4)) {
      if (job_valid(jb, decode != 0)) {
        // decode: a job of fewer chunks than one lane group fills goes to
        // split units (decode_split = 1), or every job (2); log2_unit is
        // log2 C + kDecThreadsLog2 (a lane group of kDecThreads chunks)
        const uint32_t l2c = log2_unit - kDecThreadsLog2;
        const uint64_t chunks = (jb.n + (1ull << l2c) - 1) >> l2c;
        split = decode && (decode_split == 2 || (decode_split == 1 && chunks < kDecThreads));
        const uint32_t lu = split ? kSplitLog2Syms : log2_unit;
        const uint64_t u = (jb.n + (1ull << lu) - 1) >> lu;
        cnt = (uint32_t)(decode ? u : (u ? u : 1));
        *jb.err = 0;
      } else {
        *jb.err = QLC_ERR_INVALID_ARGUMENT;
      }
    }
    js[k].count = cnt;
    js[k].hist_done = 0;  // decode: js[k].split (the same word)
    js[k].table_ready = 0;
    if (decode) js[k].split = split;
    local += cnt;
    maxc = cnt > maxc ? cnt : maxc;
  }

  // ---- exclusive scan of the unit counts over the jobs ----
  const uint64_t incl = wave_inclusive_scan_u64(local);
  uint32_t m = maxc;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t o = __shfl_xor(m, d, 64);
    m = o > m ? o : m;
  }
  if (lane == 63) wsum[wave] = incl;
  if (lane == 0) wmax[wave] = m;
  __syncthreads();
  if (tid == 0) {
    uint64_t t = 0;
    uint32_t mm = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) {
      const uint64_t v = wsum[w];
      wsum[w] = t;
      t += v;
      mm = wmax[w] > mm ? wmax[w] : mm;
    }
    total_s = t;
    maxc_s = mm;
  }
  __syncthreads();
  const uint64_t total = total_s;
  if (total > max_units) {
    // workspace too small for these jobs: every job fails, nothing runs
    for (uint32_t k = k0; k < k1; ++k) {
      const qlc_job jb = jobs[k];
      if (jb.err && ptr_aligned(jb.err, 4)) *jb.err = QLC_ERR_INVALID_ARGUMENT;
      js[k].count = 0;
    }
    if (tid == 0) {
      hdr->ticket = 0;
      hdr->units = 0;
      hdr->lag = 0;
      hdr->abort = 1;
      hdr->log2_seg = log2_unit;
    }
    return;
  }
  uint64_t base = wsum[wave] + incl - local;
  for (uint32_t k = k0; k < k1; ++k) {
    const uint32_t cnt = js[k].count;
    js[k].base = (uint32_t)base;
    for (uint32_t u = 0; u < cnt; ++u) unit_job[base + u] = k;
    base += cnt;
  }
  if (!decode)
    for (uint64_t u = tid; u < total; u += kPlanThreads) seg_word[u] = 0;
  if (tid == 0) {
    uint64_t lag = lag_req == 0 ? total : (lag_req > maxc_s ? lag_req : maxc_s);
    hdr->ticket = 0;
    hdr->units = (uint32_t)total;
    hdr->lag = (uint32_t)(lag < total ? lag : total);
    hdr->abort = 0;
    hdr->log2_seg = log2_unit;
  }
}

// Ticket p of the encode queue -> (histogram item?, segment).
__device__ __forceinline__ bool encode_item(uint32_t p, uint32_t G, uint32_t L, uint32_t& g) {
  if (p < L) {
    g = p;
    return true;
  }
  if (p < 2 * G - L) {
    const uint32_t q = p - L;
    g = (q & 1u) ? L + (q >> 1) : (q >> 1);
    return (q & 1u) != 0;
  }
  g = p - G;
  return false;
}

union BatchEncSmem {
  uint32_t sub[256 * kHistCopies];
  TableSmem table;
  EncSmem enc;
};

// At most 128 VGPRs, so that four workgroups share a CU (LDS allows it).
template <int kBits>
__global__ __launch_bounds__(kEncThreads, 4) void k_encode_batched(
    const qlc_job* __restrict__ jobs, uint32_t mode, uint32_t log2_chunk,
    BatchHeader* __restrict__ hdr, BatchJobState* __restrict__ js,
    uint64_t* __restrict__ job_hist, const uint32_t* __restrict__ seg_job,
    uint64_t* __restrict__ seg_word, uint32_t* __restrict__ seg_hist) {
  __shared__ BatchEncSmem S;
  __shared__ uint32_t s_ticket, s_flag;
  const uint32_t tid = threadIdx.x;
  const uint32_t G = hdr->units;
  const uint32_t L = hdr->lag;
  const uint32_t log2_seg = hdr->log2_seg;  // the plan's (given or automatic) segment size
  // A workgroup beyond the number of work items takes no ticket: the queue
  // is drained by the lower-numbered ones, and a small batch does not queue
  // every resident workgroup's atomic on the one ticket word.
  if ((uint64_t)blockIdx.x >= 2ull * G) return;
  for (;;) {
    if (tid == 0) s_ticket = atomic_add_u32(&hdr->ticket, 1u);
    __syncthreads();
    const uint32_t p = __builtin_amdgcn_readfirstlane(s_ticket);
    if (p >= 2 * G) break;
    uint32_t g;
    const bool hist = encode_item(p, G, L, g);
    const uint32_t k = __builtin_amdgcn_readfirstlane(seg_job[g]);
    const uint32_t base = js[k].base, cnt = js[k].count;
    const qlc_job jb = jobs[k];
    const uint32_t s = g - base;
    const uint64_t seg0 = (uint64_t)s << log2_seg;
    const uint64_t seg1 = (seg0 + (1ull << log2_seg)) < jb.n ? seg0 + (1ull << log2_seg) : jb.n;

    if (hist) {
      // ---- H(g): the segment's histogram; the job's last one builds the table ----
      for (uint32_t i = tid; i < 256 * kHistCopies; i += kEncThreads) S.sub[i] = 0;
      __syncthreads();
      hist_segment<kBits>(jb.in, seg0, seg1, S.sub, opaque_tid());
      __syncthreads();
      const uint32_t v = hist_bin_total(S.sub, tid);
      store_relaxed_u32(&seg_hist[(uint64_t)g * 256 + tid], v);
      if (jb.build_table && v)
        __hip_atomic_fetch_add(&job_hist[(uint64_t)k * 256 + tid], (uint64_t)v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) s_flag = (atomic_add_u32(&js[k].hist_done, 1u) == cnt - 1);
      __syncthreads();
      if (s_flag) {
        if (jb.build_table) {
          S.table.h[tid] = load_relaxed_u64(&job_hist[(uint64_t)k * 256 + tid]);
          build_table_block<true>(S.table.h, mode, jb.table, S.table);
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
        }
        if (tid == 0) store_relaxed_u32(&js[k].table_ready, 1u);
      }
    } else {
      // ---- E(g): wait for the job's table, then encode the segment ----
      if (tid == 0) {
        while (load_relaxed_u32(&js[k].table_ready) == 0) __builtin_amdgcn_s_sleep(2);
        S.enc.bad_table = 0;
        S.enc.cap_hit = 0;
      }
      for (uint32_t w = tid; w < sizeof(S.enc.words) / 4; w += kEncThreads) (&S.enc.words[0][0])[w] = 0;
      __syncthreads();
      const uint32_t* tw = reinterpret_cast<const uint32_t*>(jb.table);
      if (tid < 128) {
        const uint32_t w = load_relaxed_u32(&tw[tid]);
        S.enc.lut[2 * tid] = enc_entry(w & 0xFFFFu);
        S.enc.lut[2 * tid + 1] = enc_entry(w >> 16);
      }
      if (tid == 0 &&
          mode_symbol_bits(load_relaxed_u32(&tw[offsetof(qlc_table, mode) / 4])) != kBits)
        S.enc.bad_table = 1;  // a table of another alphabet
      __syncthreads();
      const uint32_t len_t = S.enc.lut[tid] >> 16;
      if (tid < Sym<kBits>::kM && (len_t < 1 || len_t > QLC_MAX_CODE_BITS)) S.enc.bad_table = 1;
      const uint64_t my_bits = block_sum_u64(
          (uint64_t)load_relaxed_u32(&seg_hist[(uint64_t)g * 256 + tid]) * len_t, S.enc.red);
      const bool bad_table = S.enc.bad_table != 0;
      if (tid == 0) store_relaxed_u64(&seg_word[g], (1ull << 63) | my_bits);
      uint64_t pre = 0;
      for (uint32_t i = base + tid; i < g; i += kEncThreads) {
        uint64_t w;
        while (((w = load_relaxed_u64(&seg_word[i])) >> 63) == 0) __builtin_amdgcn_s_sleep(1);
        pre += w & ~(1ull << 63);
      }
      const uint64_t G0 = block_sum_u64(pre, S.enc.red);
      const bool last_seg = (s == cnt - 1);
      if (last_seg && tid == 0) *jb.total_bits = G0 + my_bits;
      bool cap = false;
      if (!bad_table)
        cap = encode_segment<kBits>(jb.in, seg0, seg1, G0, last_seg, log2_chunk,
                                    reinterpret_cast<uint32_t*>(jb.bits), jb.bits_capacity / 4,
                                    jb.chunk_index, S.enc, opaque_tid());
      if (cap) S.enc.cap_hit = 1;
      __syncthreads();
      if (tid == 0) {
        if (bad_table) set_error(jb.err, QLC_ERR_INVALID_ARGUMENT);
        else if (S.enc.cap_hit) set_error(jb.err, QLC_ERR_CAPACITY);
      }
    }
    __syncthreads();
  }
}

// Work items of a batched decode: a group of kDecThreads chunks decoded one
// lane per chunk, or, for jobs the plan marked split, a split unit of
// kSplitSyms symbols (split_block).  Both layouts start with the LUT, which
// is rebuilt only when the job changes.
union BatchDecSmem {
  DecSmem lane;
  SplitSmem split;
};
static_assert(offsetof(DecSmem, lut) == 0 && offsetof(SplitSmem, lut) == 0, "shared LUT");
static_assert(kSplitThreads == kDecThreads, "one block size");

template <int kBits>
__global__ __launch_bounds__(kDecThreads) void k_decode_batched(
    const qlc_job* __restrict__ jobs, uint32_t log2_chunk, BatchHeader* __restrict__ hdr,
    const BatchJobState* __restrict__ js, const uint32_t* __restrict__ grp_job) {
  __shared__ BatchDecSmem S;
  __shared__ uint32_t s_ticket;
  const uint32_t tid = threadIdx.x;
  const uint32_t units = hdr->units;
  if (blockIdx.x >= units) return;  // (as in the encoder: only as many workgroups as items)
  uint32_t cur = ~0u;
  SplitLut L{0, 0, 1, false};
  for (;;) {
    if (tid == 0) s_ticket = atomic_add_u32(&hdr->ticket, 1u);
    __syncthreads();
    const uint32_t p = __builtin_amdgcn_readfirstlane(s_ticket);
    if (p >= units) break;
    const uint32_t k = __builtin_amdgcn_readfirstlane(grp_job[p]);
    const qlc_job jb = jobs[k];
    if (k != cur) {
      qlc_table* tl = (qlc_table*)S.lane.ring;  // free between work items
      table_to_lds(jb.table, tl, tid);
      __syncthreads();
      build_dec_lut(tl, S.lane.lut, L.sh_lo, L.sh_hi);
      L.ok = mode_symbol_bits(tl->mode) == kBits;
      L.d = code_length_gcd(tl);
      __syncthreads();
      cur = k;
    }
    if (L.ok) {
      const uint32_t unit = p - js[k].base;
      const bool bad =
          __builtin_amdgcn_readfirstlane(js[k].split)
              ? split_block<kBits>(jb.bits, *jb.total_bits, jb.chunk_index, log2_chunk, jb.n,
                                   jb.out, unit, nullptr, L, S.split, opaque_tid())
              : decode_block<kBits>(jb.bits, *jb.total_bits, jb.chunk_index, log2_chunk, jb.n,
                                    jb.out, unit, L.sh_lo, L.sh_hi, S.lane, opaque_tid());
      set_error_wave(jb.err, QLC_ERR_CORRUPT_STREAM, bad);
    } else if (tid == 0) {
      set_error(jb.err, QLC_ERR_INVALID_ARGUMENT);  // a table of another alphabet
    }
    __syncthreads();
  }
}

// ===========================================================================
// Workspace zeroing (a fill kernel, so that callers may capture it).
// ===========================================================================
__global__ void k_zero_words(uint32_t* __restrict__ p, uint64_t nwords) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace qlc

// ===========================================================================
// Host-side launchers
// ===========================================================================
namespace qlc {

// Launch `kern<B>` for the symbol width B = bits (4, 6 or 8).
#define QLC_LAUNCH_BITS(bits, kern, grid, block, ...)                                      \
  do {                                                                                  \
    if ((bits) == 4)                                                                    \
      hipLaunchKernelGGL(kern<4>, grid, block, 0, stream, __VA_ARGS__);                 \
    else if ((bits) == 6)                                                               \
      hipLaunchKernelGGL(kern<6>, grid, block, 0, stream, __VA_ARGS__);                 \
    else                                                                                \
      hipLaunchKernelGGL(kern<8>, grid, block, 0, stream, __VA_ARGS__);                 \
  } while (0)

hipError_t launch_histogram(const uint8_t* in, uint64_t n, uint32_t bits, WsHeader* hdr,
                            uint64_t* xcd_part, uint32_t* seg_hist, uint64_t* hist_out,
                            uint32_t flags, uint32_t mode, qlc_table* table_out,
                            hipStream_t stream) {
  const uint32_t l = seg_log2(n);
  QLC_LAUNCH_BITS(bits, k_histogram, dim3((uint32_t)seg_count(n)), dim3(kHistThreads), in, n, l,
                  hdr, xcd_part, seg_hist, hist_out, flags, mode, table_out);
  return hipGetLastError();
}

hipError_t launch_table_from_hist(const uint64_t* hist, uint32_t mode, qlc_table* out,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(k_table_from_hist, dim3(1), dim3(kTableThreads), 0, stream, hist, mode, out);
  return hipGetLastError();
}

// Polls of a predecessor's published bit count before the encoder computes
// it itself: QLC_ENCODE_SPIN_POLLS (tests set 0 to take that path for every
// count not yet published), else 256 (several hundred microseconds, far more
// than co-resident workgroups take to publish).
static uint32_t encode_spin_polls() {
  static const uint32_t polls = [] {
    const char* e = getenv("QLC_ENCODE_SPIN_POLLS");
    return e ? (uint32_t)strtoul(e, nullptr, 10) : 256u;
  }();
  return polls;
}

hipError_t launch_encode(const uint8_t* in, uint64_t n, uint32_t bits, const qlc_table* table,
                         const uint32_t* seg_hist, const uint64_t* seg_bits, uint32_t log2_chunk,
                         uint32_t* bits_out, uint64_t cap_words, uint64_t* index_out,
                         uint64_t* total_out, uint32_t* err_out, WsHeader* hdr, uint64_t* seg_word,
                         hipStream_t stream) {
  const uint32_t nseg = (uint32_t)seg_count(n);
  QLC_LAUNCH_BITS(bits, k_encode, dim3(nseg), dim3(kEncThreads), in, n, seg_log2(n), table,
                  seg_hist, seg_bits, log2_chunk, bits_out, cap_words, index_out, total_out,
                  err_out, hdr, seg_word, nseg, encode_spin_polls());
  return hipGetLastError();
}

hipError_t launch_segment_bits(const uint8_t* in, uint64_t n, uint32_t bits,
                               const qlc_table* table, uint64_t* seg_bits, hipStream_t stream) {
  QLC_LAUNCH_BITS(bits, k_segment_bits, dim3((uint32_t)seg_count(n)), dim3(kHistThreads), in, n,
                  seg_log2(n), table, seg_bits);
  return hipGetLastError();
}

hipError_t launch_decode(const uint8_t* bits_in, const uint64_t* total, const uint64_t* index,
                         uint32_t log2_chunk, const qlc_table* table, uint64_t n, uint32_t bits,
                         uint8_t* out, uint32_t* err_out, WsHeader* hdr, hipStream_t stream) {
  const uint64_t nchunks = (n + (1ull << log2_chunk) - 1) >> log2_chunk;
  uint64_t blocks = (nchunks + kDecThreads - 1) / kDecThreads;
  if (blocks < 1) blocks = 1;
  QLC_LAUNCH_BITS(bits, k_decode, dim3((uint32_t)blocks), dim3(kDecThreads), bits_in, total,
                  index, log2_chunk, table, n, out, err_out, hdr);
  return hipGetLastError();
}

hipError_t launch_decode_split(const uint8_t* bits_in, const uint64_t* total, const uint64_t* index,
                               uint32_t log2_chunk, const qlc_table* table, uint64_t n,
                               uint32_t bits, uint8_t* out, uint32_t* err_out, WsHeader* hdr,
                               hipStream_t stream) {
  if (log2_chunk < 8 || log2_chunk > kSplitMaxLog2Chunk) return hipErrorInvalidValue;
  uint64_t blocks = (n + kSplitSyms - 1) >> kSplitLog2Syms;
  if (blocks < 1) blocks = 1;
  QLC_LAUNCH_BITS(bits, k_decode_split, dim3((uint32_t)blocks), dim3(kSplitThreads), bits_in,
                  total, index, log2_chunk, table, n, out, err_out, hdr);
  return hipGetLastError();
}

hipError_t launch_batch_plan(const qlc_job* jobs, uint32_t n_jobs, bool decode,
                             uint32_t decode_split, uint32_t log2_unit, uint64_t max_units,
                             uint32_t lag, BatchHeader* hdr, BatchJobState* js, uint64_t* job_hist,
                             uint32_t* unit_job, uint64_t* seg_word, hipStream_t stream) {
  const uint32_t grid = 1 + (decode ? 0u : (n_jobs + kPlanZeroJobs - 1) / kPlanZeroJobs);
  hipLaunchKernelGGL(k_batch_plan, dim3(grid), dim3(kPlanThreads), 0, stream, jobs, n_jobs,
                     decode ? 1u : 0u, decode_split, log2_unit, max_units, lag, hdr, js,
                     job_hist, unit_job, seg_word);
  return hipGetLastError();
}

hipError_t launch_encode_batched(const qlc_job* jobs, uint32_t bits, uint32_t mode,
                                 uint32_t log2_chunk, BatchHeader* hdr, BatchJobState* js,
                                 uint64_t* job_hist, const uint32_t* seg_job, uint64_t* seg_word,
                                 uint32_t* seg_hist, uint32_t grid, hipStream_t stream) {
  QLC_LAUNCH_BITS(bits, k_encode_batched, dim3(grid), dim3(kEncThreads), jobs, mode, log2_chunk,
                  hdr, js, job_hist, seg_job, seg_word, seg_hist);
  return hipGetLastError();
}

hipError_t launch_decode_batched(const qlc_job* jobs, uint32_t bits, uint32_t log2_chunk,
                                 BatchHeader* hdr, const BatchJobState* js,
                                 const uint32_t* grp_job, uint32_t grid, hipStream_t stream) {
  QLC_LAUNCH_BITS(bits, k_decode_batched, dim3(grid), dim3(kDecThreads), jobs, log2_chunk, hdr,
                  js, grp_job);
  return hipGetLastError();
}

int batched_blocks_per_cu(bool decode) {
  int nb = 0;
  hipError_t e = decode ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void*>(k_decode_batched<8>), kDecThreads, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, reinterpret_cast<const void*>(k_encode_batched<8>), kEncThreads, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t stream) {
  const uint64_t nwords = bytes / 4;
  uint64_t blocks = (nwords + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero_words, dim3((uint32_t)blocks), dim3(256), 0, stream,
                     static_cast<uint32_t*>(p), nwords);
  return hipGetLastError();
}

}  // namespace qlc
