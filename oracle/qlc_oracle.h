/*
 * qlc_oracle.h -- CPU oracle for Quad Length Codes (QLC), arXiv 2602.17849.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the QLC hot path computes, written from the paper
 * so that the GPU library can be checked against it.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the HIP library, and the
 * HIP library never calls it.
 *
 * Everything here is integer arithmetic except nothing: entropy and Huffman
 * bounds live in oracle/bounds.py (float64).
 *
 * Paper readings taken where the paper is silent (each repeated at its use):
 *   R1 offset rule   : an area whose suffix width equals the symbol width
 *                      (8 bits for 256 symbols) carries the raw rank as its
 *                      suffix (offset 0); every other area adds its first
 *                      rank as offset.  This is the only rule that reproduces
 *                      both the decode worked example (Implementation
 *                      section: area 100, suffix 010 -> 32 + 2 = 34) and the
 *                      printed codes of ranks 253..255 in Table 3.
 *   R2 bit order     : codes are written most-significant bit first; stream
 *                      bit k is bit (7 - k mod 8) of byte k / 8.
 *   R3 rank ties     : equal counts rank by ascending byte value.
 *   R4 zero counts   : every one of the 256 symbols receives a code.
 *   R5 layout choice : fixed Table 1 / Table 2 widths, or an exhaustive
 *                      search over non-decreasing width tuples filled
 *                      greedily in rank order (ties -> lexicographically
 *                      smallest tuple), optionally limited to four distinct
 *                      code lengths ("quad").
 *   R7 chunk index   : index[j] = bit offset of symbol j*C; the bitstream
 *                      itself does not depend on C.
 *   R8 padding       : zero bits up to the next 32-bit boundary.
 */
#ifndef QLC_ORACLE_H
#define QLC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QREF_MAX_AREAS 16
#define QREF_MAX_SYMBOLS 256

/* Status values (numerically equal to the library's, defined separately). */
#define QREF_OK 0
#define QREF_ERR_INVALID_ARGUMENT 1
#define QREF_ERR_CAPACITY 2
#define QREF_ERR_CORRUPT_STREAM 3

/* Layout modes. */
#define QREF_MODE_SEARCH_QUAD 0
#define QREF_MODE_SEARCH_ANY 1
#define QREF_MODE_PAPER_T1 2
#define QREF_MODE_PAPER_T2 3

typedef struct qref_table {
  uint32_t M;            /* alphabet size (256 for the codec)              */
  uint32_t A;            /* number of areas (8 for the codec)              */
  uint32_t prefix_bits;  /* bits of the area code (3 for the codec)        */
  uint32_t symbol_bits;  /* log2(M)                                         */
  uint32_t width[QREF_MAX_AREAS];   /* suffix bits of each area             */
  uint32_t first[QREF_MAX_AREAS];   /* first rank held by each area         */
  uint32_t count[QREF_MAX_AREAS];   /* number of ranks held by each area    */
  uint32_t offset[QREF_MAX_AREAS];  /* rank = offset + suffix               */
  uint32_t rank_to_sym[QREF_MAX_SYMBOLS]; /* decoder LUT (Table 4)          */
  uint32_t sym_to_rank[QREF_MAX_SYMBOLS];
  uint32_t code[QREF_MAX_SYMBOLS];  /* encoder LUT (Table 3): code bits     */
  uint32_t len[QREF_MAX_SYMBOLS];   /* code length = prefix_bits + width    */
  uint64_t cost_bits;    /* sum over symbols of count * length              */
} qref_table;

/* Histogram: h[s] = number of bytes equal to s. */
void qref_histogram(const uint8_t* x, uint64_t n, uint64_t* h);

/* Rank symbols by decreasing count, ties by ascending symbol. */
void qref_rank(const uint64_t* h, uint32_t M, uint32_t* rank_to_sym,
               uint32_t* sym_to_rank);

/* Greedy fill of ranks into areas for a width tuple.  Returns 1 when every
 * area is non-empty and the areas cover all M ranks, else 0. */
int qref_fill(uint32_t M, uint32_t A, const uint32_t* width, uint32_t* first,
              uint32_t* count);

/* Enumerate admissible non-decreasing width tuples in lexicographic order.
 * max_distinct limits the number of distinct widths (A = no limit).
 * Writes up to cap tuples (A entries each) into out (may be NULL) and
 * returns the total number of admissible tuples. */
int64_t qref_enumerate(uint32_t M, uint32_t A, uint32_t max_distinct,
                       uint32_t* out, int64_t cap);

/* Cost in bits of a width tuple for rank-ordered counts. */
uint64_t qref_cost(const uint64_t* ranked_counts, uint32_t M, uint32_t A,
                   uint32_t prefix_bits, const uint32_t* width);

/* Exhaustive layout search; returns the index of the chosen tuple in the
 * enumeration order and writes it to width_out. */
int64_t qref_search(const uint64_t* ranked_counts, uint32_t M, uint32_t A,
                    uint32_t prefix_bits, uint32_t max_distinct,
                    uint32_t* width_out);

/* Build a complete table for a general alphabet from a histogram.
 * width_fixed != NULL selects those widths instead of searching. */
int qref_build_table_general(const uint64_t* h, uint32_t M, uint32_t A,
                             uint32_t prefix_bits, uint32_t max_distinct,
                             const uint32_t* width_fixed, qref_table* t);

/* Build the codec table (M = 256, A = 8, 3 prefix bits) for a mode. */
int qref_build_table(const uint64_t* h, int mode, qref_table* t);

/* Build the codec table from a stored layout: widths + rank order. */
int qref_table_from_layout(const uint32_t* width, const uint32_t* rank_to_sym,
                           qref_table* t);

/* Encode n bytes.  bits_out receives 4*ceil(total/32) bytes (zero padded)
 * and must hold cap_bytes; index_out receives ceil(n/C) entries. */
int qref_encode(const uint8_t* x, uint64_t n, const qref_table* t,
                uint32_t chunk_symbols, uint8_t* bits_out, uint64_t cap_bytes,
                uint64_t* index_out, uint64_t* total_bits_out);

/* Total bits the encoding of x would take (sum of code lengths). */
uint64_t qref_encoded_bits(const uint8_t* x, uint64_t n, const qref_table* t);

/* Decode n symbols; returns QREF_ERR_CORRUPT_STREAM on an invalid code, a
 * read past total_bits, or a chunk that does not end where the next begins. */
int qref_decode(const uint8_t* bits, uint64_t total_bits,
                const uint64_t* index, uint32_t chunk_symbols,
                const qref_table* t, uint64_t n, uint8_t* out);

/* Building blocks of the encode / decode above, over a sub-range (used by
 * the multi-threaded variants below; no arithmetic of their own).
 * qref_encode_range writes the codes of x[i0, i1) from stream bit bit0 on
 * into a zeroed buffer and the index entries of the chunk starts inside
 * the range; returns the bit after the last code.  qref_decode_range
 * decodes chunks [j0, j1) of a stream (status as qref_decode). */
uint64_t qref_encode_range(const uint8_t* x, uint64_t i0, uint64_t i1,
                           const qref_table* t, uint32_t chunk_symbols,
                           uint64_t bit0, uint8_t* bits_out,
                           uint64_t* index_out);
int qref_decode_range(const uint8_t* bits, uint64_t total_bits,
                      const uint64_t* index, uint32_t chunk_symbols,
                      const qref_table* t, uint64_t n, uint8_t* out,
                      uint64_t j0, uint64_t j1);

/* Multi-threaded oracle (OpenMP, qlc_oracle_mt.c): the same results as the
 * single-threaded functions, byte for byte, computed over contiguous
 * slices (histogram) or ranges of whole chunks (encode, decode) by
 * `threads` threads (<= 0: OpenMP's default). */
void qref_histogram_mt(const uint8_t* x, uint64_t n, uint64_t* h, int threads);
int qref_encode_mt(const uint8_t* x, uint64_t n, const qref_table* t,
                   uint32_t chunk_symbols, uint8_t* bits_out, uint64_t cap_bytes,
                   uint64_t* index_out, uint64_t* total_bits_out, int threads);
int qref_decode_mt(const uint8_t* bits, uint64_t total_bits,
                   const uint64_t* index, uint32_t chunk_symbols,
                   const qref_table* t, uint64_t n, uint8_t* out, int threads);
/* Threads an OpenMP parallel region with `threads` (<= 0: default) runs. */
int qref_mt_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
