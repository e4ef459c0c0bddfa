/*
 * qlc.h -- C ABI of libqlc, an MI355X (gfx950) implementation of Quad Length
 * Codes (QLC), the lossless code for e4m3 byte streams of arXiv 2602.17849.
 *
 * The method (Quad Length Codes and Implementation sections of the paper):
 *   1. count the 256 byte symbols (histogram);
 *   2. rank the symbols by decreasing count;
 *   3. split the ranks into 8 areas named by a 3-bit area code, area a
 *      holding 2^width[a] ranks (the last one what remains), so a code is
 *      the area code followed by width[a] suffix bits (Tables 1 and 2);
 *   4. emit a 256-entry encoder LUT (symbol -> code, length) and a 256-entry
 *      decoder LUT (rank -> symbol) (Tables 3 and 4);
 *   5. encode: look up each symbol's code and concatenate the codes;
 *   6. decode: read 3 bits, which fix the suffix width, read the suffix, add
 *      the area offset to get the rank, map the rank through the decoder LUT.
 *
 * Readings of points the paper leaves open (the stream format):
 *   - suffix/offset: an area whose width is 8 stores the raw rank as its
 *     suffix (offset 0); any other area stores rank - first rank of the area
 *     (reproduces both the decode example, 100|010 -> 34, and the printed
 *     codes 111_11111101..111_11111111 of ranks 253..255 in Table 3);
 *   - bit order: each code is written most significant bit first, stream bit
 *     k is bit (7 - k mod 8) of byte k/8; the stream is zero padded to a
 *     multiple of 32 bits, so it occupies 4*ceil(total_bits/32) bytes;
 *   - rank ties: equal counts rank by ascending symbol value; every symbol,
 *     also one of count 0, gets a code;
 *   - chunk index: index[j] is the bit offset of symbol j*C; the stream does
 *     not depend on C (no per-chunk alignment);
 *   - layout choice: the widths of Table 1 or Table 2, or the cheapest
 *     non-decreasing width tuple (3639 candidates; 1308 when limited to four
 *     distinct code lengths), filled greedily in rank order, ties to the
 *     lexicographically smallest tuple.
 *
 * Conventions for every entry point below:
 *   - Pointers named h_* are host pointers; every other pointer is a DEVICE
 *     pointer (hipMalloc'd or torch CUDA/ROCm tensor storage).
 *   - Work is enqueued asynchronously on `stream`; results are valid after
 *     the stream is synchronised.  The library never allocates or frees on
 *     these paths; the caller owns every buffer.
 *   - Argument errors are detected on the host before any launch and are
 *     returned synchronously (nothing is enqueued).
 *   - Data-dependent errors (capacity exceeded, corrupt stream) are written
 *     by the device to *err_out (0 = success, otherwise a qlc_status value;
 *     the first error found wins).  Outputs are undefined when *err_out != 0.
 *   - Workspaces: a buffer of at least qlc_workspace_bytes() bytes, zeroed
 *     once before its first use (qlc_workspace_init or any memset to 0);
 *     the kernels leave it zeroed-equivalent for the next call.  Calls that
 *     run concurrently (different streams) need different workspaces.
 *   - Alignment: `in`, `out`, `bits` and `bits_out` 16 bytes; index and
 *     total pointers 8 bytes; tables 16 bytes.
 *   - n < 2^36 symbols per call.
 */
#ifndef QLC_H
#define QLC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QLC_ABI_VERSION 1u
#define QLC_NUM_SYMBOLS 256
#define QLC_NUM_AREAS 8
#define QLC_MAX_CODE_BITS 11
#define QLC_SERIALIZED_TABLE_BYTES 264
#define QLC_MIN_CHUNK 256u
#define QLC_MAX_CHUNK 65536u
#define QLC_MAX_SYMBOLS_PER_CALL (1ull << 36)

typedef enum qlc_status {
  QLC_OK = 0,
  QLC_ERR_INVALID_ARGUMENT = 1,
  QLC_ERR_CAPACITY = 2,
  QLC_ERR_CORRUPT_STREAM = 3,
  QLC_ERR_UNSUPPORTED = 4,
  QLC_ERR_HIP = 5,
  QLC_ERR_BUSY = 6
} qlc_status;

typedef enum qlc_layout_mode {
  QLC_LAYOUT_SEARCH_QUAD = 0, /* cheapest tuple with <= 4 distinct lengths   */
  QLC_LAYOUT_SEARCH_ANY = 1,  /* cheapest tuple, any number of lengths       */
  QLC_LAYOUT_PAPER_T1 = 2,    /* Table 1: widths 3,3,3,3,3,4,5,8             */
  QLC_LAYOUT_PAPER_T2 = 3,    /* Table 2: widths 1,3,3,3,3,5,5,8             */
  /* Cheapest tuple with at most k distinct code lengths, k = 1..8 (the
   * number of distinct lengths is one of the knobs the Conclusion section
   * leaves open; k = 4 gives SEARCH_QUAD's table, k = 8 SEARCH_ANY's). */
  QLC_LAYOUT_SEARCH_DISTINCT_1 = 17,
  QLC_LAYOUT_SEARCH_DISTINCT_2 = 18,
  QLC_LAYOUT_SEARCH_DISTINCT_3 = 19,
  QLC_LAYOUT_SEARCH_DISTINCT_4 = 20,
  QLC_LAYOUT_SEARCH_DISTINCT_5 = 21,
  QLC_LAYOUT_SEARCH_DISTINCT_6 = 22,
  QLC_LAYOUT_SEARCH_DISTINCT_7 = 23,
  QLC_LAYOUT_SEARCH_DISTINCT_8 = 24,
  /* Four areas named by a 2-bit area code (the number of areas is another
   * knob the Conclusion section leaves open): cheapest non-decreasing
   * 4-tuple of widths, greedy fill, codes of 2 + width bits.  The table's
   * areas 4..7 get width 0xFF, no ranks. */
  QLC_LAYOUT_SEARCH_AREAS4 = 32,
  /* Small alphabets (the eXmY family's 4- and 6-bit types, Experimental
   * Setup; areas and symbols per area are the knobs the Conclusion leaves
   * open): the cheapest non-decreasing width tuple, greedy fill, for 16
   * symbols (4-bit codes such as e2m1) in 2 areas (1-bit area code, codes
   * of 1..5 bits) or 4 areas (2-bit area code, 2..6 bits), and for 64
   * symbols (6-bit codes such as e3m2) in 4 areas (2..8 bits) or 8 areas
   * (3-bit area code, 3..9 bits).  An area whose width is the symbol width
   * stores the raw rank.  Used with the *_sym entry points below. */
  QLC_LAYOUT_M16_AREAS2 = 48,
  QLC_LAYOUT_M16_AREAS4 = 49,
  QLC_LAYOUT_M64_AREAS4 = 50,
  QLC_LAYOUT_M64_AREAS8 = 51
} qlc_layout_mode;
#define QLC_LAYOUT_SEARCH_DISTINCT(k) ((qlc_layout_mode)(16 + (k)))

/* A complete QLC table (Tables 1-4 in one record).  Plain old data, 1088
 * bytes, device resident when passed to the codec entry points. */
typedef struct qlc_table {
  uint16_t enc[256];        /* encoder LUT by input symbol: (len << 11) | code,
                               code right aligned, len = 3 + width[area]    */
  uint8_t rank_to_sym[256]; /* decoder LUT (Table 4)                         */
  uint8_t sym_to_rank[256]; /* inverse of rank_to_sym                        */
  uint8_t width[8];         /* suffix bits of each area, non-decreasing;
                               0xFF in areas 4..7 of a 4-area table          */
  uint8_t offset[8];        /* rank = offset[a] + suffix                     */
  uint16_t first[8];        /* first rank of each area                       */
  uint16_t count[8];        /* ranks held by each area, >= 1 in every area
                               used, sum 256                                 */
  uint64_t cost_bits;       /* sum of count*length over the histogram used   */
  uint32_t mode;            /* qlc_layout_mode it was built with             */
  uint32_t version;         /* QLC_ABI_VERSION                               */
} qlc_table;

/* Human-readable name of a status. */
const char* qlc_status_string(qlc_status s);

/* Number of chunk-index entries for n symbols: ceil(n / chunk_symbols). */
uint64_t qlc_chunk_count(uint64_t n, uint32_t chunk_symbols);

/* Bitstream bytes that suffice for any table: 11 bits per symbol rounded up
 * to 32-bit words, then to 16 bytes. */
uint64_t qlc_encode_bound_bytes(uint64_t n);

/* Workspace bytes for a call on n symbols with the given chunk size (the
 * same workspace serves histogram, table, encode and decode calls). */
size_t qlc_workspace_bytes(uint64_t n, uint32_t chunk_symbols);

/* Zero a workspace on `stream` (needed once, before its first use). */
qlc_status qlc_workspace_init(void* ws, size_t ws_bytes, hipStream_t stream);

/* Step 1 (Observations section): hist_out[s] = number of bytes equal to s,
 * as 256 uint64 counts. */
qlc_status qlc_histogram(const uint8_t* in, uint64_t n, uint64_t* hist_out,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* Step 1 for a table shared by many tensors (Implementation section: one
 * LUT per tensor type, obtained a priori): hist_inout[s] += number of
 * bytes of `in` equal to s.  hist_inout (256 uint64 counts, device, 8-byte
 * aligned) is read and written by the last workgroup on `stream`, so calls
 * on one stream accumulate in order; the caller zeroes it before the first
 * call.  Same argument rules and errors as qlc_histogram.  Feeding the sum
 * to qlc_table_from_histogram gives one table for every tensor summed
 * (while the sum stays below 2^48 symbols). */
qlc_status qlc_histogram_accumulate(const uint8_t* in, uint64_t n, uint64_t* hist_inout,
                                    void* ws, size_t ws_bytes, hipStream_t stream);

/* Steps 2-4 (Implementation section, Tables 1-4): build *table_out from a
 * device histogram of 256 uint64 counts.  The counts must sum to less than
 * 2^48 (every single-call histogram does: n < 2^36); from a larger sum the
 * table comes out marked unusable (every code length 0, every width 0xFF),
 * and an encode with it fails with QLC_ERR_INVALID_ARGUMENT.  Scale such a
 * histogram down first. */
qlc_status qlc_table_from_histogram(const uint64_t* hist, qlc_layout_mode mode,
                                    qlc_table* table_out, hipStream_t stream);

/* Steps 1-4 fused: histogram of `in`, then the table. */
qlc_status qlc_build_table(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                           qlc_table* table_out, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/* Step 5 (Implementation section, encoding): bits_out receives the
 * concatenated codes (4*ceil(total/32) bytes, zero padded), chunk_index_out
 * the ceil(n/C) chunk start offsets, *total_bits_out the stream length in
 * bits.  chunk_symbols C: a power of two in [256, 65536].  If the stream
 * would exceed bits_capacity_bytes nothing past the capacity is written and
 * *err_out = QLC_ERR_CAPACITY. */
qlc_status qlc_encode(const uint8_t* in, uint64_t n, const qlc_table* table,
                      uint32_t chunk_symbols, uint8_t* bits_out,
                      uint64_t bits_capacity_bytes, uint64_t* chunk_index_out,
                      uint64_t* total_bits_out, uint32_t* err_out, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* Steps 1-5 fused for one tensor: its histogram, a table built from it
 * with `mode` (written to *table_out), then the encoding as qlc_encode.
 * Reads the input twice (histogram, then codes) and never re-reads the
 * table from the host.  (The encoder's workgroups exchange their segments'
 * bit counts; one that has waited QLC_ENCODE_SPIN_POLLS polls (an
 * environment variable read once per process, default 256) for a
 * predecessor's count computes it itself from that segment's histogram.
 * The result is the same either way.) */
qlc_status qlc_compress(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                        qlc_table* table_out, uint32_t chunk_symbols,
                        uint8_t* bits_out, uint64_t bits_capacity_bytes,
                        uint64_t* chunk_index_out, uint64_t* total_bits_out,
                        uint32_t* err_out, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* qlc_compress for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results as qlc_compress without a workspace.
 * Instead of `ws`, the call uses a workspace of
 * QLC_COMPRESS_NOALLOC_SCRATCH_BYTES held in a device array inside the
 * library (one per device, kept until the process ends; looked up and
 * zeroed by the first call on each device, on that call's stream).  No
 * hipMalloc, hipFree or allocating library routine is called.
 *   - n <= QLC_COMPRESS_NOALLOC_MAX_SYMBOLS (2^30), else
 *     QLC_ERR_INVALID_ARGUMENT and nothing is launched; every other
 *     argument rule and error is that of qlc_compress.
 *   - Every call on one device shares that device's array: calls whose
 *     work overlaps on the device (different streams, or host threads
 *     without ordering between them) race and give undefined results.
 *     Calls in stream order are safe; each leaves the array ready for the
 *     next. */
#define QLC_COMPRESS_NOALLOC_MAX_SYMBOLS (1ull << 30)
#define QLC_COMPRESS_NOALLOC_SCRATCH_BYTES 1074688u
qlc_status qlc_compress_noalloc(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                                qlc_table* table_out, uint32_t chunk_symbols,
                                uint8_t* bits_out, uint64_t bits_capacity_bytes,
                                uint64_t* chunk_index_out, uint64_t* total_bits_out,
                                uint32_t* err_out, hipStream_t stream);

/* Step 6 (Implementation section, decoding): decode n symbols of the stream
 * `bits` (4*ceil(*total_bits/32) readable bytes) into out.  Each chunk is
 * decoded independently from its index entry.  *err_out =
 * QLC_ERR_CORRUPT_STREAM for a suffix outside its area, a chunk that does
 * not end where the next begins (the last one at *total_bits) or an index
 * entry out of order. */
qlc_status qlc_decode(const uint8_t* bits, const uint64_t* total_bits,
                      const uint64_t* chunk_index, uint32_t chunk_symbols,
                      const qlc_table* table, uint64_t n, uint8_t* out,
                      uint32_t* err_out, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* Step 6 with a choice of decoder.  Both give the same output and errors
 * (the decoding section of the paper: each code's length follows from its
 * area code, so a chunk can also be cut into pieces whose code boundaries
 * are found by walking lengths alone):
 *   QLC_DECODER_LANE   one lane walks each chunk from its index entry; the
 *                      rate for tensors of many chunks (n / C >= 2^17);
 *   QLC_DECODER_SPLIT  C / 64 lanes per chunk (C <= 16384, else
 *                      QLC_ERR_INVALID_ARGUMENT): each lane walks the code
 *                      lengths of one piece of the chunk's bits from a
 *                      guessed start, the lanes correct their starts from
 *                      their neighbours' exits, then each decodes about 64
 *                      codes; latency for tensors of few chunks;
 *   QLC_DECODER_AUTO   the one qlc_decode / qlc_decode_sym use: the decoder
 *                      with the shorter estimated time, from models of both
 *                      fitted on MI355X (256 MiB down to 1 Mi symbols):
 *                      LANE  max(14.6 us + 36.7 ns * C, 0.615 ps * n),
 *                      SPLIT 21.3 us + 1.235 ps * n (only for C <= 16384).
 * symbol_bits as in the *_sym entry points below (8 for bytes); other
 * arguments and errors as qlc_decode. */
typedef enum qlc_decoder {
  QLC_DECODER_AUTO = 0,
  QLC_DECODER_LANE = 1,
  QLC_DECODER_SPLIT = 2
} qlc_decoder;
/* The decoder QLC_DECODER_AUTO takes for n symbols at chunk size C:
 * QLC_DECODER_LANE or QLC_DECODER_SPLIT (QLC_DECODER_AUTO for an invalid C).
 * Host only, no device call. */
qlc_decoder qlc_decoder_choice(uint64_t n, uint32_t chunk_symbols);
qlc_status qlc_decode_ex(const uint8_t* bits, const uint64_t* total_bits,
                         const uint64_t* chunk_index, uint32_t chunk_symbols,
                         const qlc_table* table, uint64_t n, uint32_t symbol_bits,
                         qlc_decoder decoder, uint8_t* out, uint32_t* err_out,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- Small alphabets: 4-bit and 6-bit symbols, packed ----
 *
 * The *_sym entry points take `symbol_bits` = 4, 6 or 8 and otherwise the
 * arguments of the byte entry points above (which are the symbol_bits = 8
 * case).  n counts symbols; a buffer of n symbols holds
 * ceil(n * symbol_bits / 8) bytes:
 *   - 4 bits: two symbols per byte, symbol 2k in the low nibble of byte k
 *     (the usual packing of e2m1 pairs);
 *   - 6 bits: symbol i in bits 6i .. 6i + 5 of the buffer read as a
 *     little-endian bit string (bit b of byte k is string bit 8k + b), four
 *     symbols per three bytes.
 * Decoded buffers follow the same packing; pad bits of the last byte are
 * written as zeros.  Layout modes must be for the same alphabet
 * (QLC_LAYOUT_M16_* for 4 bits, QLC_LAYOUT_M64_* for 6 bits, the others
 * for 8 bits), else QLC_ERR_INVALID_ARGUMENT before any launch; an encode
 * or decode given a table built for another alphabet reports
 * QLC_ERR_INVALID_ARGUMENT in *err_out and writes nothing.  The stream,
 * chunk index and table formats are those of the byte codec: a table of M
 * symbols uses enc / sym_to_rank entries 0..M-1 and rank_to_sym entries
 * 0..M-1 (the other entries are 0 / identity), and marks the areas it
 * does not use with width 0xFF. */
qlc_status qlc_histogram_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                             uint64_t* hist_out, void* ws, size_t ws_bytes, hipStream_t stream);
qlc_status qlc_histogram_accumulate_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                                        uint64_t* hist_inout, void* ws, size_t ws_bytes,
                                        hipStream_t stream);
qlc_status qlc_build_table_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                               qlc_layout_mode mode, qlc_table* table_out, void* ws,
                               size_t ws_bytes, hipStream_t stream);
qlc_status qlc_compress_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                            qlc_layout_mode mode, qlc_table* table_out, uint32_t chunk_symbols,
                            uint8_t* bits_out, uint64_t bits_capacity_bytes,
                            uint64_t* chunk_index_out, uint64_t* total_bits_out,
                            uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream);
qlc_status qlc_encode_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                          const qlc_table* table, uint32_t chunk_symbols, uint8_t* bits_out,
                          uint64_t bits_capacity_bytes, uint64_t* chunk_index_out,
                          uint64_t* total_bits_out, uint32_t* err_out, void* ws, size_t ws_bytes,
                          hipStream_t stream);
qlc_status qlc_decode_sym(const uint8_t* bits, const uint64_t* total_bits,
                          const uint64_t* chunk_index, uint32_t chunk_symbols,
                          const qlc_table* table, uint64_t n, uint32_t symbol_bits, uint8_t* out,
                          uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- Batched form: many tensors (shards) of uneven sizes per launch ----
 *
 * The same steps as qlc_compress / qlc_decode applied to every job of a
 * device array; each job's table, bitstream, index and total are
 * byte-identical to what the single-tensor entry points produce for it with
 * the same mode and C.  A call is a small planning kernel followed by one
 * persistent launch whose workgroups take work items (segment histograms,
 * table builds, segment encodes, 256-chunk decode groups or split units) from a shared
 * queue, so small shards do not leave the device idle.  Neither call
 * allocates, synchronises or sets memory from the host, so both may be
 * captured in a hipGraph and replayed. */
typedef struct qlc_job {
  const uint8_t* in;       /* encode: n input symbols (16-B aligned)           */
  uint8_t* out;            /* decode: n output symbols (16-B aligned)          */
  uint64_t n;              /* symbols of the job (< 2^36)                      */
  qlc_table* table;        /* encode: built when build_table, else read;
                              decode: read (16-B aligned)                      */
  uint8_t* bits;           /* encode: written; decode: read (16-B aligned)     */
  uint64_t bits_capacity;  /* encode: bytes writable at bits                   */
  uint64_t* chunk_index;   /* ceil(n / C) entries (8-B aligned)                */
  uint64_t* total_bits;    /* encode: written; decode: read (8-B aligned)      */
  uint32_t* err;           /* the job's status, set by every call (4-B aligned) */
  uint32_t build_table;    /* encode: 1 = build *table from `in` with `mode`   */
  uint32_t reserved;       /* 0 */
} qlc_job;                 /* 80 bytes */

/* Work split of a batched call; zero fields take the defaults. */
typedef struct qlc_batch_tuning {
  uint32_t log2_segment; /* encode work item = 2^log2_segment symbols, 13..24;
                            0: chosen on the device from T, the symbols of
                            the call's valid jobs: floor(log2 T)/2 + 4
                            clamped to 13..19 (about sqrt(T)/16 items) */
  uint32_t lag_segments; /* encode: histogram items handed out ahead of the
                            encode items, raised to the largest job's segment
                            count (0: every histogram first) */
  uint32_t workgroups;   /* persistent workgroups (0: fill the device)        */
  uint32_t decoder;      /* decode: QLC_DECODER_AUTO (0) = every job in split
                            units of 2^14 symbols (C/64 lanes per chunk,
                            C <= 16384) when a time model of the two
                            decoders favours split for T symbols at this C
                            (26 us + 2.5 ps/symbol against the larger of
                            19.4 us + 44 ns * C and 0.46 ps/symbol), else
                            only the jobs of fewer than 256 chunks, the
                            others one lane per chunk; QLC_DECODER_LANE =
                            every job one lane per chunk; QLC_DECODER_SPLIT =
                            every job split (C <= 16384).  Ignored by
                            encode.                                         */
} qlc_batch_tuning;

/* Workspace bytes for batched calls over n_jobs jobs holding at most
 * total_symbols symbols together (h_tuning may be NULL).  Every batched call
 * resets the state it uses, so a batched workspace needs no zeroing; a
 * workspace handed to the single-tensor entry points after batched calls
 * must be zeroed (qlc_workspace_init) first. */
size_t qlc_batched_workspace_bytes(uint32_t n_jobs, uint64_t total_symbols,
                                   uint32_t chunk_symbols,
                                   const qlc_batch_tuning* h_tuning);

/* Steps 1-5 for every job of the device array `jobs` (n_jobs entries).  Per
 * job: *err = 0 on success; QLC_ERR_INVALID_ARGUMENT for a job whose
 * pointers are NULL or misaligned, n >= 2^36, reserved != 0, or (for every
 * job) when the workspace is too small for the jobs' total size; a job
 * whose err pointer is NULL or misaligned is skipped.  QLC_ERR_CAPACITY as
 * qlc_encode.  A table written by a build_table job must not be another
 * job's table in the same call. */
qlc_status qlc_encode_batched(const qlc_job* jobs, uint32_t n_jobs,
                              qlc_layout_mode mode, uint32_t chunk_symbols,
                              const qlc_batch_tuning* h_tuning, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* Step 6 for every job of `jobs` (bits, chunk_index, total_bits and table
 * in, out written); per-job err as qlc_decode. */
qlc_status qlc_decode_batched(const qlc_job* jobs, uint32_t n_jobs,
                              uint32_t chunk_symbols,
                              const qlc_batch_tuning* h_tuning, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* The batched calls for jobs of `symbol_bits`-bit symbols (4, 6 or 8; all
 * jobs of one call share it; packing and mode rules as the *_sym entry
 * points above). */
qlc_status qlc_encode_batched_sym(const qlc_job* jobs, uint32_t n_jobs, uint32_t symbol_bits,
                                  qlc_layout_mode mode, uint32_t chunk_symbols,
                                  const qlc_batch_tuning* h_tuning, void* ws, size_t ws_bytes,
                                  hipStream_t stream);
qlc_status qlc_decode_batched_sym(const qlc_job* jobs, uint32_t n_jobs, uint32_t symbol_bits,
                                  uint32_t chunk_symbols, const qlc_batch_tuning* h_tuning,
                                  void* ws, size_t ws_bytes, hipStream_t stream);

/* Host-side persisted table form: width[8] followed by rank_to_sym[256]. */
qlc_status qlc_table_serialize(const qlc_table* h_table,
                               uint8_t h_out[QLC_SERIALIZED_TABLE_BYTES]);
/* Rebuild a full table on the host: 8, 4 or 2 areas (the widths after the
 * last area are 0xFF), over the alphabet of 256, 64 or 16 symbols that the
 * widths fill greedily with every area non-empty (at most one does; 8
 * areas are never a 16-symbol table).  Rejects widths that are not
 * non-decreasing in 0..8 or fit no alphabet, and rank orders that are not
 * a permutation of the alphabet (identity beyond it).  A 16- or 64-symbol
 * table gets its QLC_LAYOUT_M* mode, so the *_sym calls accept it; a byte
 * table gets mode 0xFFFFFFFF. */
qlc_status qlc_table_deserialize(const uint8_t h_in[QLC_SERIALIZED_TABLE_BYTES],
                                 qlc_table* h_table);

#ifdef __cplusplus
}
#endif
#endif /* QLC_H */
