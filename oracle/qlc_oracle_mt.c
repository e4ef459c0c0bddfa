/*
 * qlc_oracle_mt.c -- multi-threaded CPU oracle for Quad Length Codes
 * (arXiv 2602.17849).
 *
 * TEST INFRASTRUCTURE ONLY (see qlc_oracle.h).  The single-threaded
 * oracle's own functions run on disjoint pieces of the work in OpenMP
 * threads; nothing here adds arithmetic.  The results equal the
 * single-threaded oracle's byte for byte (a test checks it), which is what
 * makes this a faithful baseline on every host core.
 *   histogram: contiguous slices counted separately, counts added;
 *   encode   : per-chunk code lengths summed in parallel, the chunk start
 *              offsets (the chunk index) by a running sum, then ranges of
 *              whole chunks written in two passes (even ranges, then odd
 *              ones), so that two ranges writing at once never share a
 *              byte of the stream;
 *   decode   : ranges of whole chunks decoded independently (each chunk
 *              starts at its index entry); the status is that of the first
 *              failing range, i.e. of the first failing chunk.
 */
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "qlc_oracle.h"

int qref_mt_threads(int threads) {
  return threads > 0 ? threads : omp_get_max_threads();
}

void qref_histogram_mt(const uint8_t* x, uint64_t n, uint64_t* h, int threads) {
  const int T = qref_mt_threads(threads);
  uint64_t* part = (uint64_t*)calloc((size_t)T * 256, sizeof(uint64_t));
#pragma omp parallel for num_threads(T) schedule(static, 1)
  for (int r = 0; r < T; ++r) {
    const uint64_t lo = n * (uint64_t)r / (uint64_t)T;
    const uint64_t hi = n * (uint64_t)(r + 1) / (uint64_t)T;
    qref_histogram(x + lo, hi - lo, part + (size_t)r * 256);
  }
  for (int s = 0; s < 256; ++s) {
    h[s] = 0;
    for (int r = 0; r < T; ++r) h[s] += part[(size_t)r * 256 + s];
  }
  free(part);
}

int qref_encode_mt(const uint8_t* x, uint64_t n, const qref_table* t,
                   uint32_t chunk_symbols, uint8_t* bits_out, uint64_t cap_bytes,
                   uint64_t* index_out, uint64_t* total_bits_out, int threads) {
  if (chunk_symbols == 0) return QREF_ERR_INVALID_ARGUMENT;
  const int T = qref_mt_threads(threads);
  const uint64_t C = chunk_symbols;
  const uint64_t nchunks = (n + C - 1) / C;
  uint64_t* bits_of = (uint64_t*)malloc(sizeof(uint64_t) * (nchunks ? nchunks : 1));
#pragma omp parallel for num_threads(T) schedule(static)
  for (int64_t j = 0; j < (int64_t)nchunks; ++j) {
    const uint64_t i0 = (uint64_t)j * C;
    const uint64_t i1 = i0 + C < n ? i0 + C : n;
    bits_of[j] = qref_encoded_bits(x + i0, i1 - i0, t);
  }
  uint64_t total = 0;
  for (uint64_t j = 0; j < nchunks; ++j) {
    index_out[j] = total;
    total += bits_of[j];
  }
  free(bits_of);
  const uint64_t nbytes = 4 * ((total + 31) / 32);
  if (total_bits_out) *total_bits_out = total;
  if (nbytes > cap_bytes) return QREF_ERR_CAPACITY;
  memset(bits_out, 0, (size_t)nbytes);
  if (nchunks == 0) return QREF_OK;

  /* Two ranges written at the same time are never neighbours, and a range
   * between them holds whole chunks of at least 8 bits each, so they share
   * no byte.  With codes too short for that, one range. */
  uint32_t min_len = ~0u;
  for (uint32_t s = 0; s < t->M; ++s) min_len = t->len[s] < min_len ? t->len[s] : min_len;
  uint64_t R = (uint64_t)T * 2;
  if (R > nchunks) R = nchunks;
  if (C * min_len < 8) R = 1;
  for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
    for (int64_t r = pass; r < (int64_t)R; r += 2) {
      const uint64_t j0 = nchunks * (uint64_t)r / R;
      const uint64_t j1 = nchunks * (uint64_t)(r + 1) / R;
      const uint64_t i1 = j1 * C < n ? j1 * C : n;
      qref_encode_range(x, j0 * C, i1, t, chunk_symbols, index_out[j0], bits_out,
                        index_out);
    }
  }
  return QREF_OK;
}

int qref_decode_mt(const uint8_t* bits, uint64_t total_bits,
                   const uint64_t* index, uint32_t chunk_symbols,
                   const qref_table* t, uint64_t n, uint8_t* out, int threads) {
  if (chunk_symbols == 0) return QREF_ERR_INVALID_ARGUMENT;
  const int T = qref_mt_threads(threads);
  const uint64_t nchunks = (n + chunk_symbols - 1) / chunk_symbols;
  if (nchunks == 0) return total_bits != 0 ? QREF_ERR_CORRUPT_STREAM : QREF_OK;
  uint64_t R = (uint64_t)T * 4;
  if (R > nchunks) R = nchunks;
  int* st = (int*)malloc(sizeof(int) * R);
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
  for (int64_t r = 0; r < (int64_t)R; ++r) {
    const uint64_t j0 = nchunks * (uint64_t)r / R;
    const uint64_t j1 = nchunks * (uint64_t)(r + 1) / R;
    st[r] = qref_decode_range(bits, total_bits, index, chunk_symbols, t, n, out, j0, j1);
  }
  int res = QREF_OK;
  for (uint64_t r = 0; r < R && res == QREF_OK; ++r) res = st[r];
  free(st);
  return res;
}
