/*
 * qlc_oracle.c -- CPU oracle for Quad Length Codes (arXiv 2602.17849).
 *
 * TEST INFRASTRUCTURE ONLY (see qlc_oracle.h): plain, slow, obviously
 * correct.  No blocking, no fusion, no bit tricks beyond writing one bit at
 * a time.  Each function names the part of the paper it follows.
 */
#include "qlc_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Histogram.  Observations section: the PMF of the 256 byte symbols.      */
/* ---------------------------------------------------------------------- */
void qref_histogram(const uint8_t* x, uint64_t n, uint64_t* h) {
  for (int s = 0; s < 256; ++s) h[s] = 0;
  for (uint64_t i = 0; i < n; ++i) h[x[i]] += 1;
}

/* ---------------------------------------------------------------------- */
/* Ranking.  Implementation section: the input symbols are sorted by      */
/* decreasing probability and mapped to 0..255 (Tables 3 and 4).  Ties    */
/* are not addressed by the paper; reading R3 breaks them by ascending    */
/* symbol value.  Selection sort: pick the best remaining symbol M times. */
/* ---------------------------------------------------------------------- */
void qref_rank(const uint64_t* h, uint32_t M, uint32_t* rank_to_sym,
               uint32_t* sym_to_rank) {
  int taken[QREF_MAX_SYMBOLS];
  for (uint32_t s = 0; s < M; ++s) taken[s] = 0;
  for (uint32_t r = 0; r < M; ++r) {
    int best = -1;
    for (uint32_t s = 0; s < M; ++s) {
      if (taken[s]) continue;
      /* strictly greater count wins; equal counts keep the smaller symbol */
      if (best < 0 || h[s] > h[best]) best = (int)s;
    }
    taken[best] = 1;
    rank_to_sym[r] = (uint32_t)best;
    sym_to_rank[best] = r;
  }
}

static uint32_t log2_exact(uint32_t M) {
  uint32_t b = 0;
  while ((1u << b) < M) ++b;
  return b;
}

/* ---------------------------------------------------------------------- */
/* Greedy fill.  Quad Length Codes section and Tables 1/2: area a holds    */
/* 2^width[a] consecutive ranks, the last area holds what remains.         */
/* ---------------------------------------------------------------------- */
int qref_fill(uint32_t M, uint32_t A, const uint32_t* width, uint32_t* first,
              uint32_t* count) {
  uint32_t next = 0;
  for (uint32_t a = 0; a < A; ++a) {
    uint32_t cap = 1u << width[a];
    uint32_t left = M - next;
    first[a] = next;
    count[a] = cap < left ? cap : left;
    next += count[a];
  }
  for (uint32_t a = 0; a < A; ++a)
    if (count[a] == 0) return 0; /* an empty area */
  return next == M;              /* all ranks covered */
}

/* ---------------------------------------------------------------------- */
/* Enumeration of admissible width tuples (reading R5).  Widths run from   */
/* 0 to the symbol width, are non-decreasing, every area must be non-empty */
/* under greedy fill and the areas must cover the alphabet.  "Quad":       */
/* Quad Length Codes section, four distinct code lengths.                  */
/* ---------------------------------------------------------------------- */
static int admissible(uint32_t M, uint32_t A, uint32_t max_distinct,
                      const uint32_t* w) {
  uint32_t first[QREF_MAX_AREAS], count[QREF_MAX_AREAS];
  uint32_t distinct = 1;
  for (uint32_t a = 1; a < A; ++a)
    if (w[a] != w[a - 1]) ++distinct;
  if (distinct > max_distinct) return 0;
  return qref_fill(M, A, w, first, count);
}

int64_t qref_enumerate(uint32_t M, uint32_t A, uint32_t max_distinct,
                       uint32_t* out, int64_t cap) {
  uint32_t maxw = log2_exact(M);
  uint32_t w[QREF_MAX_AREAS];
  int64_t n = 0;
  /* odometer over non-decreasing tuples, lexicographic order */
  for (uint32_t a = 0; a < A; ++a) w[a] = 0;
  for (;;) {
    if (admissible(M, A, max_distinct, w)) {
      if (out && n < cap)
        for (uint32_t a = 0; a < A; ++a) out[n * A + a] = w[a];
      ++n;
    }
    /* advance: rightmost position that can still grow */
    int pos = (int)A - 1;
    while (pos >= 0 && w[pos] == maxw) --pos;
    if (pos < 0) break;
    w[pos] += 1;
    for (uint32_t a = (uint32_t)pos + 1; a < A; ++a) w[a] = w[pos];
  }
  return n;
}

/* Cost of a layout: every symbol costs prefix_bits + width of its area.  */
uint64_t qref_cost(const uint64_t* ranked_counts, uint32_t M, uint32_t A,
                   uint32_t prefix_bits, const uint32_t* width) {
  uint32_t first[QREF_MAX_AREAS], count[QREF_MAX_AREAS];
  qref_fill(M, A, width, first, count);
  uint64_t cost = 0;
  for (uint32_t a = 0; a < A; ++a)
    for (uint32_t r = first[a]; r < first[a] + count[a]; ++r)
      cost += ranked_counts[r] * (uint64_t)(prefix_bits + width[a]);
  return cost;
}

int64_t qref_search(const uint64_t* ranked_counts, uint32_t M, uint32_t A,
                    uint32_t prefix_bits, uint32_t max_distinct,
                    uint32_t* width_out) {
  int64_t total = qref_enumerate(M, A, max_distinct, NULL, 0);
  if (total <= 0) return -1;
  uint32_t* all = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)total * A);
  qref_enumerate(M, A, max_distinct, all, total);
  int64_t best = -1;
  uint64_t best_cost = 0;
  for (int64_t i = 0; i < total; ++i) {
    uint64_t c = qref_cost(ranked_counts, M, A, prefix_bits, all + i * A);
    if (best < 0 || c < best_cost) { /* ties keep the earlier tuple */
      best = i;
      best_cost = c;
    }
  }
  for (uint32_t a = 0; a < A; ++a) width_out[a] = all[best * A + a];
  free(all);
  return best;
}

/* ---------------------------------------------------------------------- */
/* Table construction.  Implementation section (Table 3): rank order ->    */
/* area -> code = area code followed by the suffix; the rows are then      */
/* indexed by input symbol.  Offsets follow reading R1.                     */
/* ---------------------------------------------------------------------- */
static int fill_codes(qref_table* t) {
  if (!qref_fill(t->M, t->A, t->width, t->first, t->count))
    return QREF_ERR_INVALID_ARGUMENT;
  for (uint32_t a = 0; a < t->A; ++a)
    t->offset[a] = (t->width[a] == t->symbol_bits) ? 0 : t->first[a];
  for (uint32_t s = 0; s < t->M; ++s) {
    uint32_t r = t->sym_to_rank[s];
    uint32_t a = 0;
    while (!(r >= t->first[a] && r < t->first[a] + t->count[a])) ++a;
    t->code[s] = (a << t->width[a]) | (r - t->offset[a]);
    t->len[s] = t->prefix_bits + t->width[a];
  }
  return QREF_OK;
}

int qref_build_table_general(const uint64_t* h, uint32_t M, uint32_t A,
                             uint32_t prefix_bits, uint32_t max_distinct,
                             const uint32_t* width_fixed, qref_table* t) {
  if (M < 2 || M > QREF_MAX_SYMBOLS || (M & (M - 1)) || A < 1 ||
      A > QREF_MAX_AREAS || (1u << prefix_bits) < A)
    return QREF_ERR_INVALID_ARGUMENT;
  memset(t, 0, sizeof(*t));
  t->M = M;
  t->A = A;
  t->prefix_bits = prefix_bits;
  t->symbol_bits = log2_exact(M);
  qref_rank(h, M, t->rank_to_sym, t->sym_to_rank);
  uint64_t ranked[QREF_MAX_SYMBOLS];
  for (uint32_t r = 0; r < M; ++r) ranked[r] = h[t->rank_to_sym[r]];
  if (width_fixed) {
    for (uint32_t a = 0; a < A; ++a) t->width[a] = width_fixed[a];
  } else if (qref_search(ranked, M, A, prefix_bits, max_distinct, t->width) <
             0) {
    return QREF_ERR_INVALID_ARGUMENT;
  }
  int st = fill_codes(t);
  if (st) return st;
  t->cost_bits = qref_cost(ranked, M, A, prefix_bits, t->width);
  return QREF_OK;
}

/* Table 1 and Table 2 of the paper: the "#Symbol bits" column. */
static const uint32_t kPaperT1[8] = {3, 3, 3, 3, 3, 4, 5, 8};
static const uint32_t kPaperT2[8] = {1, 3, 3, 3, 3, 5, 5, 8};

int qref_build_table(const uint64_t* h, int mode, qref_table* t) {
  switch (mode) {
    case QREF_MODE_SEARCH_QUAD:
      return qref_build_table_general(h, 256, 8, 3, 4, NULL, t);
    case QREF_MODE_SEARCH_ANY:
      return qref_build_table_general(h, 256, 8, 3, 8, NULL, t);
    case QREF_MODE_PAPER_T1:
      return qref_build_table_general(h, 256, 8, 3, 8, kPaperT1, t);
    case QREF_MODE_PAPER_T2:
      return qref_build_table_general(h, 256, 8, 3, 8, kPaperT2, t);
    default:
      return QREF_ERR_INVALID_ARGUMENT;
  }
}

int qref_table_from_layout(const uint32_t* width, const uint32_t* rank_to_sym,
                           qref_table* t) {
  memset(t, 0, sizeof(*t));
  t->M = 256;
  t->A = 8;
  t->prefix_bits = 3;
  t->symbol_bits = 8;
  int seen[256] = {0};
  for (int r = 0; r < 256; ++r) {
    if (rank_to_sym[r] > 255 || seen[rank_to_sym[r]])
      return QREF_ERR_INVALID_ARGUMENT;
    seen[rank_to_sym[r]] = 1;
    t->rank_to_sym[r] = rank_to_sym[r];
    t->sym_to_rank[rank_to_sym[r]] = (uint32_t)r;
  }
  for (int a = 0; a < 8; ++a) {
    if (width[a] > 8 || (a > 0 && width[a] < width[a - 1]))
      return QREF_ERR_INVALID_ARGUMENT;
    t->width[a] = width[a];
  }
  return fill_codes(t);
}

/* ---------------------------------------------------------------------- */
/* Encoding.  Implementation section: look up the code of each input      */
/* symbol and concatenate the codes (reading R2: MSB first, R8: zero pad   */
/* to 32 bits, R7: chunk index every C symbols).                            */
/* ---------------------------------------------------------------------- */
static void put_bit(uint8_t* bits, uint64_t k, uint32_t v) {
  if (v) bits[k >> 3] |= (uint8_t)(0x80u >> (k & 7));
}

static uint32_t get_bit(const uint8_t* bits, uint64_t k) {
  return (bits[k >> 3] >> (7 - (k & 7))) & 1u;
}

uint64_t qref_encoded_bits(const uint8_t* x, uint64_t n, const qref_table* t) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < n; ++i) total += t->len[x[i]];
  return total;
}

uint64_t qref_encode_range(const uint8_t* x, uint64_t i0, uint64_t i1,
                           const qref_table* t, uint32_t chunk_symbols,
                           uint64_t bit0, uint8_t* bits_out,
                           uint64_t* index_out) {
  uint64_t k = bit0;
  for (uint64_t i = i0; i < i1; ++i) {
    if (i % chunk_symbols == 0) index_out[i / chunk_symbols] = k;
    uint32_t code = t->code[x[i]];
    uint32_t len = t->len[x[i]];
    for (uint32_t j = 0; j < len; ++j) /* most significant bit first */
      put_bit(bits_out, k++, (code >> (len - 1 - j)) & 1u);
  }
  return k;
}

int qref_encode(const uint8_t* x, uint64_t n, const qref_table* t,
                uint32_t chunk_symbols, uint8_t* bits_out, uint64_t cap_bytes,
                uint64_t* index_out, uint64_t* total_bits_out) {
  if (chunk_symbols == 0) return QREF_ERR_INVALID_ARGUMENT;
  uint64_t total = qref_encoded_bits(x, n, t);
  uint64_t nbytes = 4 * ((total + 31) / 32);
  if (total_bits_out) *total_bits_out = total;
  if (nbytes > cap_bytes) return QREF_ERR_CAPACITY;
  memset(bits_out, 0, (size_t)nbytes);
  qref_encode_range(x, 0, n, t, chunk_symbols, 0, bits_out, index_out);
  return QREF_OK;
}

/* ---------------------------------------------------------------------- */
/* Decoding.  Implementation section: read the 3-bit area code, which     */
/* fixes the suffix width; read the suffix; add the area offset to obtain  */
/* the rank ("encoded symbol"); map it through the 256-entry decoder LUT.  */
/* ---------------------------------------------------------------------- */
static int read_bits(const uint8_t* bits, uint64_t total, uint64_t* pos,
                     uint32_t nb, uint32_t* v) {
  uint32_t r = 0;
  for (uint32_t j = 0; j < nb; ++j) {
    if (*pos >= total) return 0; /* read past the end of the stream */
    r = (r << 1) | get_bit(bits, *pos);
    *pos += 1;
  }
  *v = r;
  return 1;
}

int qref_decode_range(const uint8_t* bits, uint64_t total_bits,
                      const uint64_t* index, uint32_t chunk_symbols,
                      const qref_table* t, uint64_t n, uint8_t* out,
                      uint64_t j0, uint64_t j1) {
  uint64_t nchunks = (n + chunk_symbols - 1) / chunk_symbols;
  for (uint64_t j = j0; j < j1; ++j) {
    uint64_t pos = index[j];
    uint64_t end = (j + 1 < nchunks) ? index[j + 1] : total_bits;
    if (j == 0 && pos != 0) return QREF_ERR_CORRUPT_STREAM;
    uint64_t i0 = j * chunk_symbols;
    uint64_t i1 = i0 + chunk_symbols < n ? i0 + chunk_symbols : n;
    for (uint64_t i = i0; i < i1; ++i) {
      uint32_t area, suffix;
      if (!read_bits(bits, total_bits, &pos, t->prefix_bits, &area))
        return QREF_ERR_CORRUPT_STREAM;
      if (area >= t->A) return QREF_ERR_CORRUPT_STREAM;
      if (!read_bits(bits, total_bits, &pos, t->width[area], &suffix))
        return QREF_ERR_CORRUPT_STREAM;
      uint32_t rank = t->offset[area] + suffix;
      if (rank < t->first[area] || rank >= t->first[area] + t->count[area])
        return QREF_ERR_CORRUPT_STREAM; /* suffix outside the area */
      out[i] = (uint8_t)t->rank_to_sym[rank];
    }
    if (pos != end) return QREF_ERR_CORRUPT_STREAM;
  }
  return QREF_OK;
}

int qref_decode(const uint8_t* bits, uint64_t total_bits,
                const uint64_t* index, uint32_t chunk_symbols,
                const qref_table* t, uint64_t n, uint8_t* out) {
  if (chunk_symbols == 0) return QREF_ERR_INVALID_ARGUMENT;
  uint64_t nchunks = (n + chunk_symbols - 1) / chunk_symbols;
  int st = qref_decode_range(bits, total_bits, index, chunk_symbols, t, n, out,
                             0, nchunks);
  if (st != QREF_OK) return st;
  if (nchunks == 0 && total_bits != 0) return QREF_ERR_CORRUPT_STREAM;
  return QREF_OK;
}
