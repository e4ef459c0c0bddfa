// libqlc C ABI: argument validation, workspace carving, kernel launches.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string.h>

#include "qlc_internal.h"
#include "qlc_kernels.h"

namespace qlc {
namespace {

constexpr int kMaxDevices = 64;
// Per device, queried once: compute units and the resident workgroups per
// CU of the two persistent kernels (the occupancy query costs microseconds
// of host time, which a small batched call would otherwise pay every time).
struct DeviceInfo {
  int cus;
  int enc_blocks_per_cu;
  int dec_blocks_per_cu;
};
DeviceInfo g_dev_info[kMaxDevices];
std::once_flag g_dev_once[kMaxDevices];

const DeviceInfo& device_info() {
  static const DeviceInfo fallback = {256, 1, 1};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return fallback;
  std::call_once(g_dev_once[dev], [dev] {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    g_dev_info[dev] = {cus, batched_blocks_per_cu(false), batched_blocks_per_cu(true)};
  });
  return g_dev_info[dev];
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool valid_chunk(uint32_t c, uint32_t* log2c) {
  if (c < QLC_MIN_CHUNK || c > QLC_MAX_CHUNK || (c & (c - 1))) return false;
  uint32_t l = 0;
  while ((1u << l) < c) ++l;
  *log2c = l;
  return true;
}

qlc_status hip_status(hipError_t e) { return e == hipSuccess ? QLC_OK : QLC_ERR_HIP; }

struct WsView {
  WsHeader* hdr;
  uint64_t* xcd_part;
  uint32_t* seg_hist;
  uint64_t* seg_word;
};

WsView carve(void* ws, uint64_t n) {
  char* b = static_cast<char*>(ws);
  const uint64_t s = seg_count(n);
  WsView v;
  v.hdr = reinterpret_cast<WsHeader*>(b);
  v.xcd_part = reinterpret_cast<uint64_t*>(b + kWsHistOffset);
  v.seg_hist = reinterpret_cast<uint32_t*>(b + kWsSegOffset);
  v.seg_word = reinterpret_cast<uint64_t*>(b + kWsSegOffset + s * 256 * sizeof(uint32_t));
  return v;
}

// ---- batched calls ----
constexpr uint64_t kMaxBatchUnits = 1ull << 30;

struct BatchView {
  BatchHeader* hdr;
  BatchJobState* js;
  uint64_t* job_hist;
  uint32_t* seg_hist;   // encode
  uint64_t* seg_word;   // encode
  uint32_t* unit_job;   // seg_job (encode) or grp_job (decode)
  uint64_t max_units;
};

BatchView carve_batch(void* ws, size_t ws_bytes, uint32_t n_jobs, bool decode) {
  char* b = static_cast<char*>(ws);
  BatchView v{};
  v.hdr = reinterpret_cast<BatchHeader*>(b);
  v.js = reinterpret_cast<BatchJobState*>(b + batch_js_offset());
  v.job_hist = reinterpret_cast<uint64_t*>(b + batch_hist_offset(n_jobs));
  const size_t u0 = batch_units_offset(n_jobs);
  const size_t room = ws_bytes > u0 ? ws_bytes - u0 : 0;
  uint64_t mu = room / (decode ? kBatchGroupBytes : kBatchSegBytes);
  if (mu > kMaxBatchUnits) mu = kMaxBatchUnits;
  v.max_units = mu;
  if (decode) {
    v.unit_job = reinterpret_cast<uint32_t*>(b + u0);
  } else {
    v.seg_hist = reinterpret_cast<uint32_t*>(b + u0);
    v.seg_word = reinterpret_cast<uint64_t*>(b + u0 + mu * 256 * sizeof(uint32_t));
    v.unit_job = reinterpret_cast<uint32_t*>(b + u0 + mu * (256 * sizeof(uint32_t) + 8));
  }
  return v;
}

bool batch_tuning(const qlc_batch_tuning* t, uint32_t* log2_seg, uint32_t* lag, uint32_t* wgs,
                  uint32_t* decoder = nullptr) {
  *log2_seg = 0;  // automatic (chosen by the plan kernel)
  *lag = 0;
  *wgs = 0;
  if (decoder) *decoder = QLC_DECODER_AUTO;
  if (!t) return true;
  if (t->decoder != QLC_DECODER_AUTO && t->decoder != QLC_DECODER_LANE &&
      t->decoder != QLC_DECODER_SPLIT)
    return false;
  if (decoder) *decoder = t->decoder;
  if (t->log2_segment) {
    if (t->log2_segment < kBatchMinLog2Seg || t->log2_segment > kBatchMaxLog2Seg) return false;
    *log2_seg = t->log2_segment;
  }
  *lag = t->lag_segments;
  *wgs = t->workgroups;
  return true;
}

uint32_t persistent_grid(bool decode, uint32_t requested) {
  if (requested) return requested;
  const DeviceInfo& d = device_info();
  const uint32_t g = (uint32_t)(d.cus * (decode ? d.dec_blocks_per_cu : d.enc_blocks_per_cu));
  return g ? g : 1;
}

// ---- the allocation-free compress: a file-scope device workspace ----------
// Sized for the largest single-tensor workspace up to kStaticMaxSymbols
// symbols (at most 1025 segments: header, per-XCD histograms, 1025 segment
// histograms and bit-count words).  Each device the library runs on holds
// its own copy until the process ends.
constexpr uint64_t kStaticMaxSymbols = 1ull << 30;
constexpr size_t kStaticWsBytes =
    (kWsSegOffset + 1025 * (256 * sizeof(uint32_t) + sizeof(uint64_t)) + 255) & ~size_t(255);
static_assert(kStaticWsBytes == QLC_COMPRESS_NOALLOC_SCRATCH_BYTES, "scratch size in qlc.h");

static __device__ __align__(256) uint8_t scratch[kStaticWsBytes];

// Device address of `scratch` on each device, looked up (and the array
// zeroed, on the caller's stream) by the first call on that device.  The
// array's name is a host-side stand-in: only these addresses reach kernels.
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

hipError_t static_workspace(hipStream_t stream, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[dev], [dev, stream] {
    void* p = nullptr;
    hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    // a fill kernel rather than a memset node, so that a first call under
    // graph capture records a plain kernel
    if (r == hipSuccess) r = launch_zero(p, kStaticWsBytes, stream);
    g_scratch_ptr[dev] = r == hipSuccess ? p : nullptr;
    g_scratch_err[dev] = r;
  });
  if (g_scratch_err[dev] != hipSuccess) return g_scratch_err[dev];
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace qlc

using namespace qlc;

extern "C" {

const char* qlc_status_string(qlc_status s) {
  switch (s) {
    case QLC_OK: return "ok";
    case QLC_ERR_INVALID_ARGUMENT: return "invalid argument";
    case QLC_ERR_CAPACITY: return "bitstream capacity exceeded";
    case QLC_ERR_CORRUPT_STREAM: return "corrupt stream";
    case QLC_ERR_UNSUPPORTED: return "unsupported";
    case QLC_ERR_HIP: return "HIP runtime error";
    case QLC_ERR_BUSY: return "busy";
  }
  return "unknown status";
}

uint64_t qlc_chunk_count(uint64_t n, uint32_t chunk_symbols) {
  if (chunk_symbols == 0) return 0;
  return (n + chunk_symbols - 1) / chunk_symbols;
}

uint64_t qlc_encode_bound_bytes(uint64_t n) {
  const uint64_t words = (n * QLC_MAX_CODE_BITS + 31) / 32;
  return (words * 4 + 15) & ~uint64_t(15);
}

size_t qlc_workspace_bytes(uint64_t n, uint32_t chunk_symbols) {
  (void)chunk_symbols;
  return ws_bytes_for(n);
}

qlc_status qlc_workspace_init(void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ws || ws_bytes < kWsSegOffset || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  return hip_status(launch_zero(ws, ws_bytes, stream));
}

qlc_status qlc_histogram_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                             uint64_t* hist_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if ((n && !in) || !hist_out || !ws || n >= QLC_MAX_SYMBOLS_PER_CALL ||
      !valid_symbol_bits(symbol_bits))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(hist_out, 8) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, n);
  return hip_status(launch_histogram(in, n, symbol_bits, v.hdr, v.xcd_part, v.seg_hist, hist_out,
                                     kHistGlobal, 0, nullptr, stream));
}

qlc_status qlc_histogram(const uint8_t* in, uint64_t n, uint64_t* hist_out, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  return qlc_histogram_sym(in, n, 8, hist_out, ws, ws_bytes, stream);
}

qlc_status qlc_histogram_accumulate_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                                        uint64_t* hist_inout, void* ws, size_t ws_bytes,
                                        hipStream_t stream) {
  if ((n && !in) || !hist_inout || !ws || n >= QLC_MAX_SYMBOLS_PER_CALL ||
      !valid_symbol_bits(symbol_bits))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(hist_inout, 8) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, n);
  return hip_status(launch_histogram(in, n, symbol_bits, v.hdr, v.xcd_part, v.seg_hist,
                                     hist_inout, kHistGlobal | kHistAccumulate, 0, nullptr,
                                     stream));
}

qlc_status qlc_histogram_accumulate(const uint8_t* in, uint64_t n, uint64_t* hist_inout, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  return qlc_histogram_accumulate_sym(in, n, 8, hist_inout, ws, ws_bytes, stream);
}

qlc_status qlc_table_from_histogram(const uint64_t* hist, qlc_layout_mode mode,
                                    qlc_table* table_out, hipStream_t stream) {
  if (!hist || !table_out || !valid_layout_mode((uint32_t)mode)) return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(hist, 8) || !aligned(table_out, 16)) return QLC_ERR_INVALID_ARGUMENT;
  return hip_status(launch_table_from_hist(hist, (uint32_t)mode, table_out, stream));
}

namespace {
// a layout mode for symbols of `symbol_bits` bits
bool mode_for(qlc_layout_mode mode, uint32_t symbol_bits) {
  return valid_layout_mode((uint32_t)mode) && mode_symbol_bits((uint32_t)mode) == symbol_bits;
}
}  // namespace

qlc_status qlc_build_table_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                               qlc_layout_mode mode, qlc_table* table_out, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  if ((n && !in) || !table_out || !ws || !mode_for(mode, symbol_bits) ||
      n >= QLC_MAX_SYMBOLS_PER_CALL)
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(table_out, 16) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, n);
  return hip_status(launch_histogram(in, n, symbol_bits, v.hdr, v.xcd_part, v.seg_hist, nullptr,
                                     kHistGlobal | kHistBuildTable, (uint32_t)mode, table_out,
                                     stream));
}

qlc_status qlc_build_table(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                           qlc_table* table_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return qlc_build_table_sym(in, n, 8, mode, table_out, ws, ws_bytes, stream);
}

namespace {
qlc_status check_encode_args(const uint8_t* in, uint64_t n, const void* table, uint32_t chunk_symbols,
                             uint8_t* bits_out, uint64_t cap, uint64_t* index_out,
                             uint64_t* total_out, uint32_t* err_out, void* ws, size_t ws_bytes,
                             uint32_t* log2c) {
  if (!valid_chunk(chunk_symbols, log2c) || n >= QLC_MAX_SYMBOLS_PER_CALL)
    return QLC_ERR_INVALID_ARGUMENT;
  if ((n && (!in || !index_out)) || !table || !total_out || !err_out || !ws || (cap && !bits_out))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(table, 16) || !aligned(bits_out, 16) || !aligned(index_out, 8) ||
      !aligned(total_out, 8) || !aligned(err_out, 4) || !aligned(ws, 256))
    return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  return QLC_OK;
}
}  // namespace

qlc_status qlc_encode_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                          const qlc_table* table, uint32_t chunk_symbols, uint8_t* bits_out,
                          uint64_t bits_capacity_bytes, uint64_t* chunk_index_out,
                          uint64_t* total_bits_out, uint32_t* err_out, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  uint32_t log2c = 0;
  if (!valid_symbol_bits(symbol_bits)) return QLC_ERR_INVALID_ARGUMENT;
  qlc_status st = check_encode_args(in, n, table, chunk_symbols, bits_out, bits_capacity_bytes,
                                    chunk_index_out, total_bits_out, err_out, ws, ws_bytes, &log2c);
  if (st != QLC_OK) return st;
  WsView v = carve(ws, n);
  // segment bit counts straight from the table's lengths (the segment
  // histograms' region holds them)
  uint64_t* seg_bits = reinterpret_cast<uint64_t*>(v.seg_hist);
  hipError_t e = launch_segment_bits(in, n, symbol_bits, table, seg_bits, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_encode(in, n, symbol_bits, table, nullptr, seg_bits, log2c,
                                  reinterpret_cast<uint32_t*>(bits_out), bits_capacity_bytes / 4,
                                  chunk_index_out, total_bits_out, err_out, v.hdr, v.seg_word,
                                  stream));
}

qlc_status qlc_encode(const uint8_t* in, uint64_t n, const qlc_table* table,
                      uint32_t chunk_symbols, uint8_t* bits_out, uint64_t bits_capacity_bytes,
                      uint64_t* chunk_index_out, uint64_t* total_bits_out, uint32_t* err_out,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
  return qlc_encode_sym(in, n, 8, table, chunk_symbols, bits_out, bits_capacity_bytes,
                        chunk_index_out, total_bits_out, err_out, ws, ws_bytes, stream);
}

qlc_status qlc_compress_sym(const uint8_t* in, uint64_t n, uint32_t symbol_bits,
                            qlc_layout_mode mode, qlc_table* table_out, uint32_t chunk_symbols,
                            uint8_t* bits_out, uint64_t bits_capacity_bytes,
                            uint64_t* chunk_index_out, uint64_t* total_bits_out,
                            uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0;
  if (!mode_for(mode, symbol_bits)) return QLC_ERR_INVALID_ARGUMENT;
  qlc_status st = check_encode_args(in, n, table_out, chunk_symbols, bits_out, bits_capacity_bytes,
                                    chunk_index_out, total_bits_out, err_out, ws, ws_bytes, &log2c);
  if (st != QLC_OK) return st;
  WsView v = carve(ws, n);
  hipError_t e = launch_histogram(in, n, symbol_bits, v.hdr, v.xcd_part, v.seg_hist, nullptr,
                                  kHistSegment | kHistGlobal | kHistBuildTable, (uint32_t)mode,
                                  table_out, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_encode(in, n, symbol_bits, table_out, v.seg_hist, nullptr, log2c,
                                  reinterpret_cast<uint32_t*>(bits_out), bits_capacity_bytes / 4,
                                  chunk_index_out, total_bits_out, err_out, v.hdr, v.seg_word,
                                  stream));
}

qlc_status qlc_compress(const uint8_t* in, uint64_t n, qlc_layout_mode mode, qlc_table* table_out,
                        uint32_t chunk_symbols, uint8_t* bits_out, uint64_t bits_capacity_bytes,
                        uint64_t* chunk_index_out, uint64_t* total_bits_out, uint32_t* err_out,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  return qlc_compress_sym(in, n, 8, mode, table_out, chunk_symbols, bits_out, bits_capacity_bytes,
                          chunk_index_out, total_bits_out, err_out, ws, ws_bytes, stream);
}

qlc_status qlc_compress_noalloc(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                                qlc_table* table_out, uint32_t chunk_symbols, uint8_t* bits_out,
                                uint64_t bits_capacity_bytes, uint64_t* chunk_index_out,
                                uint64_t* total_bits_out, uint32_t* err_out,
                                hipStream_t stream) {
  if (n > kStaticMaxSymbols) return QLC_ERR_INVALID_ARGUMENT;
  void* ws = nullptr;
  if (static_workspace(stream, &ws) != hipSuccess) return QLC_ERR_HIP;
  return qlc_compress(in, n, mode, table_out, chunk_symbols, bits_out, bits_capacity_bytes,
                      chunk_index_out, total_bits_out, err_out, ws, kStaticWsBytes, stream);
}

// The decoder with the shorter estimated time (ns), from two-term models
// fitted to measured decode times on MI355X: one lane per chunk walks C
// codes in sequence (a fixed cost plus 36.7 ns per code) unless the chunks
// fill the device, where it takes 0.615 ps per symbol (1.63 TB/s); the
// split decoder costs 21.3 us plus 1.235 ps per symbol (1 to 128 Mi
// symbols, 512-bit warm-up).
static qlc_decoder auto_decoder(uint64_t n, uint32_t log2c) {
  if (log2c > kSplitMaxLog2Chunk) return QLC_DECODER_LANE;
  const uint64_t C = 1ull << log2c;
  const uint64_t lane_walk = 14600 + C * 367 / 10, lane_rate = n * 615 / 1000000;
  const uint64_t lane = lane_walk > lane_rate ? lane_walk : lane_rate;
  const uint64_t split = 21300 + n * 1235 / 1000000;
  return split < lane ? QLC_DECODER_SPLIT : QLC_DECODER_LANE;
}

qlc_decoder qlc_decoder_choice(uint64_t n, uint32_t chunk_symbols) {
  uint32_t log2c = 0;
  if (!valid_chunk(chunk_symbols, &log2c)) return QLC_DECODER_AUTO;
  return auto_decoder(n, log2c);
}

qlc_status qlc_decode_ex(const uint8_t* bits, const uint64_t* total_bits,
                         const uint64_t* chunk_index, uint32_t chunk_symbols,
                         const qlc_table* table, uint64_t n, uint32_t symbol_bits,
                         qlc_decoder decoder, uint8_t* out, uint32_t* err_out, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0;
  if (!valid_chunk(chunk_symbols, &log2c) || n >= QLC_MAX_SYMBOLS_PER_CALL ||
      !valid_symbol_bits(symbol_bits))
    return QLC_ERR_INVALID_ARGUMENT;
  if (decoder != QLC_DECODER_AUTO && decoder != QLC_DECODER_LANE && decoder != QLC_DECODER_SPLIT)
    return QLC_ERR_INVALID_ARGUMENT;
  if (decoder == QLC_DECODER_SPLIT && log2c > kSplitMaxLog2Chunk) return QLC_ERR_INVALID_ARGUMENT;
  if (!total_bits || !table || !err_out || !ws || (n && (!bits || !chunk_index || !out)))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(bits, 16) || !aligned(total_bits, 8) || !aligned(chunk_index, 8) ||
      !aligned(table, 16) || !aligned(out, 16) || !aligned(err_out, 4) || !aligned(ws, 256))
    return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(0)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, 0);
  if (decoder == QLC_DECODER_AUTO) decoder = auto_decoder(n, log2c);
  if (decoder == QLC_DECODER_SPLIT)
    return hip_status(launch_decode_split(bits, total_bits, chunk_index, log2c, table, n,
                                          symbol_bits, out, err_out, v.hdr, stream));
  return hip_status(launch_decode(bits, total_bits, chunk_index, log2c, table, n, symbol_bits, out,
                                  err_out, v.hdr, stream));
}

qlc_status qlc_decode_sym(const uint8_t* bits, const uint64_t* total_bits,
                          const uint64_t* chunk_index, uint32_t chunk_symbols,
                          const qlc_table* table, uint64_t n, uint32_t symbol_bits, uint8_t* out,
                          uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return qlc_decode_ex(bits, total_bits, chunk_index, chunk_symbols, table, n, symbol_bits,
                       QLC_DECODER_AUTO, out, err_out, ws, ws_bytes, stream);
}

qlc_status qlc_decode(const uint8_t* bits, const uint64_t* total_bits, const uint64_t* chunk_index,
                      uint32_t chunk_symbols, const qlc_table* table, uint64_t n, uint8_t* out,
                      uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return qlc_decode_sym(bits, total_bits, chunk_index, chunk_symbols, table, n, 8, out, err_out,
                        ws, ws_bytes, stream);
}

size_t qlc_batched_workspace_bytes(uint32_t n_jobs, uint64_t total_symbols, uint32_t chunk_symbols,
                                   const qlc_batch_tuning* h_tuning) {
  uint32_t log2c = 0, log2_seg = 0, lag = 0, wgs = 0;
  if (!valid_chunk(chunk_symbols, &log2c) || !batch_tuning(h_tuning, &log2_seg, &lag, &wgs))
    return 0;
  const uint64_t segs = log2_seg ? (total_symbols >> log2_seg) + n_jobs
                                 : batch_auto_seg_bound(total_symbols, n_jobs);
  // decode units: lane groups of kDecThreads chunks (2^16 symbols or more)
  // or split units of 2^14 symbols, whichever each job gets: at most one
  // split unit per 2^14 symbols plus one per job
  static_assert(kDecThreadsLog2 + 8 >= kSplitUnitLog2, "split units outnumber lane groups");
  const uint64_t groups = (total_symbols >> kSplitUnitLog2) + n_jobs;
  const uint64_t enc = segs * kBatchSegBytes, dec = groups * kBatchGroupBytes;
  return round256(batch_units_offset(n_jobs) + (enc > dec ? enc : dec));
}

qlc_status qlc_encode_batched_sym(const qlc_job* jobs, uint32_t n_jobs, uint32_t symbol_bits,
                                  qlc_layout_mode mode, uint32_t chunk_symbols,
                                  const qlc_batch_tuning* h_tuning, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  uint32_t log2c = 0, log2_seg = 0, lag = 0, wgs = 0;
  if (!valid_chunk(chunk_symbols, &log2c) || !mode_for(mode, symbol_bits) ||
      !batch_tuning(h_tuning, &log2_seg, &lag, &wgs))
    return QLC_ERR_INVALID_ARGUMENT;
  if ((n_jobs && !jobs) || !ws || !aligned(jobs, 8) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (n_jobs == 0) return QLC_OK;
  if (ws_bytes < batch_units_offset(n_jobs)) return QLC_ERR_INVALID_ARGUMENT;
  BatchView v = carve_batch(ws, ws_bytes, n_jobs, false);
  hipError_t e = launch_batch_plan(jobs, n_jobs, false, 0, log2_seg, v.max_units, lag, v.hdr, v.js,
                                   v.job_hist, v.unit_job, v.seg_word, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_encode_batched(jobs, symbol_bits, (uint32_t)mode, log2c,
                                          v.hdr, v.js, v.job_hist, v.unit_job, v.seg_word,
                                          v.seg_hist, persistent_grid(false, wgs), stream));
}

qlc_status qlc_encode_batched(const qlc_job* jobs, uint32_t n_jobs, qlc_layout_mode mode,
                              uint32_t chunk_symbols, const qlc_batch_tuning* h_tuning, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  return qlc_encode_batched_sym(jobs, n_jobs, 8, mode, chunk_symbols, h_tuning, ws, ws_bytes,
                                stream);
}

qlc_status qlc_decode_batched_sym(const qlc_job* jobs, uint32_t n_jobs, uint32_t symbol_bits,
                                  uint32_t chunk_symbols, const qlc_batch_tuning* h_tuning,
                                  void* ws, size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0, log2_seg = 0, lag = 0, wgs = 0, decoder = 0;
  if (!valid_chunk(chunk_symbols, &log2c) || !valid_symbol_bits(symbol_bits) ||
      !batch_tuning(h_tuning, &log2_seg, &lag, &wgs, &decoder))
    return QLC_ERR_INVALID_ARGUMENT;
  if (decoder == QLC_DECODER_SPLIT && log2c > kSplitMaxLog2Chunk) return QLC_ERR_INVALID_ARGUMENT;
  if ((n_jobs && !jobs) || !ws || !aligned(jobs, 8) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (n_jobs == 0) return QLC_OK;
  if (ws_bytes < batch_units_offset(n_jobs)) return QLC_ERR_INVALID_ARGUMENT;
  BatchView v = carve_batch(ws, ws_bytes, n_jobs, true);
  // split units: every job (SPLIT), or (AUTO) jobs of fewer chunks than a
  // lane group holds, whose lanes would otherwise idle
  const uint32_t split = decoder == QLC_DECODER_SPLIT ? 2u
                         : decoder == QLC_DECODER_AUTO && log2c <= kSplitMaxLog2Chunk ? 1u
                                                                                       : 0u;
  hipError_t e = launch_batch_plan(jobs, n_jobs, true, split, log2c + kDecThreadsLog2, v.max_units,
                                   0, v.hdr, v.js, v.job_hist, v.unit_job, nullptr, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_decode_batched(jobs, symbol_bits, log2c, v.hdr, v.js, v.unit_job,
                                          persistent_grid(true, wgs), stream));
}

qlc_status qlc_decode_batched(const qlc_job* jobs, uint32_t n_jobs, uint32_t chunk_symbols,
                              const qlc_batch_tuning* h_tuning, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
  return qlc_decode_batched_sym(jobs, n_jobs, 8, chunk_symbols, h_tuning, ws, ws_bytes, stream);
}

qlc_status qlc_table_serialize(const qlc_table* h_table, uint8_t h_out[QLC_SERIALIZED_TABLE_BYTES]) {
  if (!h_table || !h_out) return QLC_ERR_INVALID_ARGUMENT;
  memcpy(h_out, h_table->width, 8);
  memcpy(h_out + 8, h_table->rank_to_sym, 256);
  return QLC_OK;
}

qlc_status qlc_table_deserialize(const uint8_t h_in[QLC_SERIALIZED_TABLE_BYTES], qlc_table* t) {
  if (!h_in || !t) return QLC_ERR_INVALID_ARGUMENT;
  // 8, 4 or 2 areas: the widths after the last area are 0xFF
  const uint32_t na = h_in[4] != 0xFFu ? 8u : h_in[2] != 0xFFu ? 4u : 2u;
  const uint32_t pbits = na == 8 ? 3u : na == 4 ? 2u : 1u;
  uint32_t w[8];
  for (uint32_t a = 0; a < 8; ++a) {
    w[a] = h_in[a];
    if (a >= na) {
      if (w[a] != 0xFFu) return QLC_ERR_INVALID_ARGUMENT;
      continue;
    }
    if (w[a] > 8 || (a && w[a] < w[a - 1])) return QLC_ERR_INVALID_ARGUMENT;
  }
  // The alphabet: the one of 16, 64 or 256 symbols (widths at most its
  // symbol width) whose greedy fill leaves every area non-empty and covers
  // it; at most one fits any width tuple.
  uint32_t M = 0, sbits = 0, first[8], count[8];
  for (uint32_t b : {4u, 6u, 8u}) {
    const uint32_t m = 1u << b;
    // the layouts that exist: 16 symbols in 2 or 4 areas, 64 or 256 in 4 or 8
    if (w[na - 1] > b || (b == 4 ? na == 8 : na == 2)) continue;
    uint32_t f = 0;
    bool ok = true;
    for (uint32_t a = 0; a < na && ok; ++a) {
      const uint32_t cap = 1u << w[a];
      first[a] = f;
      count[a] = cap < m - f ? cap : m - f;
      ok = count[a] != 0;
      f += count[a];
    }
    if (ok && f == m) {
      M = m;
      sbits = b;
      break;
    }
  }
  if (M == 0) return QLC_ERR_INVALID_ARGUMENT;
  for (uint32_t a = na; a < 8; ++a) {
    first[a] = 256;
    count[a] = 0;
  }
  // rank order: a permutation of the alphabet, identity beyond it
  bool seen[256] = {};
  for (uint32_t r = 0; r < 256; ++r) {
    const uint32_t s = h_in[8 + r];
    if (seen[s] || (r < M ? s >= M : s != r)) return QLC_ERR_INVALID_ARGUMENT;
    seen[s] = true;
  }
  memset(t, 0, sizeof(*t));
  for (uint32_t a = 0; a < 8; ++a) {
    t->width[a] = (uint8_t)w[a];
    t->first[a] = (uint16_t)first[a];
    t->count[a] = (uint16_t)count[a];
    t->offset[a] = (uint8_t)(a >= na || w[a] == sbits ? 0 : first[a]);
  }
  for (uint32_t r = 0; r < 256; ++r) {
    const uint32_t s = h_in[8 + r];
    t->rank_to_sym[r] = (uint8_t)s;
    t->sym_to_rank[s] = (uint8_t)r;
    if (r >= M) continue;  // no code outside the alphabet
    uint32_t a = 0;
    for (uint32_t k = 1; k < na; ++k) a = r >= first[k] ? k : a;
    const uint32_t code = (a << w[a]) | (r - t->offset[a]);
    t->enc[s] = (uint16_t)(((pbits + w[a]) << 11) | code);
  }
  t->cost_bits = 0;
  // the small-alphabet modes name their alphabet; a byte table's search
  // mode is not recorded
  t->mode = M == 16 ? (na == 2 ? QLC_LAYOUT_M16_AREAS2 : QLC_LAYOUT_M16_AREAS4)
            : M == 64 ? (na == 4 ? QLC_LAYOUT_M64_AREAS4 : QLC_LAYOUT_M64_AREAS8)
                      : 0xFFFFFFFFu;
  t->version = QLC_ABI_VERSION;
  return QLC_OK;
}

}  // extern "C"
