/*
 * qlc_server.h -- serving form of libqlc: a request loop that admits
 * compress / decompress requests of mixed sizes against a device-memory
 * budget and runs them with continuous batching.
 *
 * Not a step of the paper: this is the deployment form around its codec.
 * Each request is one job of the batched entry points (qlc_encode_batched /
 * qlc_decode_batched), or, in a tick of one request, a call of the
 * single-tensor entry points (qlc_compress / qlc_encode / qlc_decode_ex,
 * whose fixed costs are lower for one tensor); either way its result is
 * byte-identical to what the single-tensor entry points give for it alone,
 * whatever else shares its tick.
 *
 * Model:
 *   - qlc_server_create reserves, once, a device pool of
 *     memory_budget_bytes plus per-tick buffers (job arrays, workspaces,
 *     pinned status words) for max_ticks_in_flight ticks; nothing is
 *     allocated afterwards.
 *   - qlc_server_submit queues a request (any thread).  A request reserves
 *     its outputs in the pool when admitted: compress = table + total/err +
 *     chunk index + bitstream (n + 16 bytes when the server searches the
 *     table, whose cost never exceeds 8 bits per symbol; the 11-bit bound
 *     for a caller's table and for the fixed PAPER_T1 / PAPER_T2 widths,
 *     which spend up to 9.6 bits per symbol); decompress = the n output
 *     bytes + err.  A
 *     request whose reservation exceeds the whole budget is rejected at
 *     submit with QLC_ERR_CAPACITY.
 *   - A server thread admits queued requests in arrival order while they
 *     fit the budget and a tick slot is free, and launches them as one tick
 *     (batched encode for the compress jobs, batched decode for the
 *     decompress jobs; the single-tensor call for a tick of one request)
 *     on the slot's stream; up to max_ticks_in_flight
 *     ticks overlap on the device, and requests arriving meanwhile join the
 *     next tick.  A request waiting for memory holds back those behind it
 *     (no overtaking).
 *   - qlc_server_poll returns completed requests; their outputs stay in the
 *     pool until qlc_server_release.
 * Inputs (compress `in`, decompress bits/index/total/table) are caller
 * device memory that must stay valid until the request completes.
 * Timestamps are steady-clock nanoseconds.
 */
#ifndef QLC_SERVER_H
#define QLC_SERVER_H

#include "qlc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qlc_server qlc_server;

typedef struct qlc_server_config {
  uint64_t memory_budget_bytes; /* device pool for admitted requests' outputs */
  uint64_t max_tick_symbols;    /* symbols per tick (0: the budget)         */
  uint32_t chunk_symbols;       /* C of every stream the server writes/reads */
  uint32_t layout_mode;         /* qlc_layout_mode of server-built tables     */
  uint32_t max_jobs_per_tick;   /* 0: 256                                     */
  uint32_t max_ticks_in_flight; /* streams / tick slots, 0: 2 (at most 8)     */
  uint32_t log2_segment;        /* batched work split (0: automatic, per tick) */
  uint32_t decoder;             /* qlc_batch_tuning.decoder of the decode
                                   ticks (0: QLC_DECODER_AUTO)                */
} qlc_server_config;

typedef enum qlc_request_kind {
  QLC_REQUEST_COMPRESS = 0,
  QLC_REQUEST_DECOMPRESS = 1
} qlc_request_kind;

typedef struct qlc_request {
  uint32_t kind;                /* qlc_request_kind                            */
  uint32_t reserved;            /* 0 */
  uint64_t n;                   /* symbols                                     */
  const uint8_t* in;            /* compress: n device bytes, 16-B aligned      */
  const qlc_table* table;       /* compress: NULL = build from `in`, else use;
                                   decompress: the stream's table               */
  const uint8_t* bits;          /* decompress: the bitstream                   */
  const uint64_t* chunk_index;  /* decompress: ceil(n / C) entries             */
  const uint64_t* total_bits;   /* decompress: device word                     */
  uint64_t user_tag;            /* returned unchanged                          */
} qlc_request;

typedef struct qlc_result {
  uint64_t id;                  /* from qlc_server_submit                      */
  uint64_t user_tag;
  uint32_t kind;
  uint32_t status;              /* the job's qlc_status                        */
  uint64_t n;
  uint64_t total_bits;          /* compress: stream length in bits             */
  /* device pointers into the pool, valid until qlc_server_release(id):      */
  qlc_table* table;             /* compress (the caller's table if given)      */
  uint8_t* bits;                /* compress: 4*ceil(total_bits/32) bytes       */
  uint64_t* chunk_index;        /* compress                                    */
  uint64_t* total_bits_dev;     /* compress                                    */
  uint8_t* out;                 /* decompress: n bytes                         */
  uint64_t submit_ns, admit_ns, complete_ns;
} qlc_result;

typedef struct qlc_server_stats {
  uint64_t budget_bytes;
  uint64_t bytes_in_use;        /* reserved by admitted, unreleased requests  */
  uint64_t peak_bytes_in_use;
  uint64_t submitted, rejected, completed, ticks;
  uint32_t max_jobs_in_tick;
  uint32_t max_ticks_in_flight; /* most ticks seen on the device at once       */
  uint32_t queued;              /* waiting for admission now                  */
  uint32_t reserved;
} qlc_server_stats;

/* Create a server on the current device.  QLC_ERR_INVALID_ARGUMENT for a
 * bad config, QLC_ERR_HIP if the pool or the tick buffers cannot be
 * allocated. */
qlc_status qlc_server_create(const qlc_server_config* h_config, qlc_server** out);

/* Queue a request; *id_out receives its id.  Synchronous errors: NULL or
 * misaligned pointers, n >= 2^36, unknown kind (QLC_ERR_INVALID_ARGUMENT);
 * a reservation larger than the budget (QLC_ERR_CAPACITY); a server that
 * is shutting down (QLC_ERR_BUSY). */
qlc_status qlc_server_submit(qlc_server* s, const qlc_request* h_req, uint64_t* id_out);

/* Move up to max_results completed requests into out (oldest first),
 * waiting up to timeout_us microseconds for the first one (0: do not
 * wait).  Returns the number written. */
uint32_t qlc_server_poll(qlc_server* s, qlc_result* out, uint32_t max_results,
                         int64_t timeout_us);

/* Return a completed request's outputs to the pool. */
qlc_status qlc_server_release(qlc_server* s, uint64_t id);

qlc_status qlc_server_get_stats(qlc_server* s, qlc_server_stats* out);

/* Finish every queued and running request, then free the server. */
qlc_status qlc_server_destroy(qlc_server* s);

#ifdef __cplusplus
}
#endif
#endif /* QLC_SERVER_H */
