// libqlc C ABI: argument validation, workspace carving, kernel launches.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string.h>

#include "qlc_internal.h"
#include "qlc_kernels.h"

namespace qlc {
namespace {

constexpr int kMaxDevices = 64;
int g_num_cus[kMaxDevices];
std::once_flag g_cu_once[kMaxDevices];

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
  std::call_once(g_cu_once[dev], [dev] {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    g_num_cus[dev] = cus;
  });
  return g_num_cus[dev];
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

qlc_status qlc_histogram(const uint8_t* in, uint64_t n, uint64_t* hist_out, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  if ((n && !in) || !hist_out || !ws || n >= QLC_MAX_SYMBOLS_PER_CALL) return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(hist_out, 8) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, n);
  return hip_status(launch_histogram(in, n, v.hdr, v.xcd_part, v.seg_hist, hist_out, kHistGlobal,
                                     0, nullptr, stream));
}

qlc_status qlc_table_from_histogram(const uint64_t* hist, qlc_layout_mode mode,
                                    qlc_table* table_out, hipStream_t stream) {
  if (!hist || !table_out || (uint32_t)mode > QLC_LAYOUT_PAPER_T2) return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(hist, 8) || !aligned(table_out, 16)) return QLC_ERR_INVALID_ARGUMENT;
  return hip_status(launch_table_from_hist(hist, (uint32_t)mode, table_out, stream));
}

qlc_status qlc_build_table(const uint8_t* in, uint64_t n, qlc_layout_mode mode,
                           qlc_table* table_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if ((n && !in) || !table_out || !ws || (uint32_t)mode > QLC_LAYOUT_PAPER_T2 ||
      n >= QLC_MAX_SYMBOLS_PER_CALL)
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(table_out, 16) || !aligned(ws, 256)) return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(n)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, n);
  return hip_status(launch_histogram(in, n, v.hdr, v.xcd_part, v.seg_hist, nullptr,
                                     kHistGlobal | kHistBuildTable, (uint32_t)mode, table_out,
                                     stream));
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

qlc_status qlc_encode(const uint8_t* in, uint64_t n, const qlc_table* table,
                      uint32_t chunk_symbols, uint8_t* bits_out, uint64_t bits_capacity_bytes,
                      uint64_t* chunk_index_out, uint64_t* total_bits_out, uint32_t* err_out,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0;
  qlc_status st = check_encode_args(in, n, table, chunk_symbols, bits_out, bits_capacity_bytes,
                                    chunk_index_out, total_bits_out, err_out, ws, ws_bytes, &log2c);
  if (st != QLC_OK) return st;
  WsView v = carve(ws, n);
  hipError_t e = launch_histogram(in, n, v.hdr, v.xcd_part, v.seg_hist, nullptr, kHistSegment, 0,
                                  nullptr, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_encode(in, n, table, v.seg_hist, log2c,
                                  reinterpret_cast<uint32_t*>(bits_out), bits_capacity_bytes / 4,
                                  chunk_index_out, total_bits_out, err_out, v.hdr, v.seg_word,
                                  stream));
}

qlc_status qlc_compress(const uint8_t* in, uint64_t n, qlc_layout_mode mode, qlc_table* table_out,
                        uint32_t chunk_symbols, uint8_t* bits_out, uint64_t bits_capacity_bytes,
                        uint64_t* chunk_index_out, uint64_t* total_bits_out, uint32_t* err_out,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0;
  if ((uint32_t)mode > QLC_LAYOUT_PAPER_T2) return QLC_ERR_INVALID_ARGUMENT;
  qlc_status st = check_encode_args(in, n, table_out, chunk_symbols, bits_out, bits_capacity_bytes,
                                    chunk_index_out, total_bits_out, err_out, ws, ws_bytes, &log2c);
  if (st != QLC_OK) return st;
  WsView v = carve(ws, n);
  hipError_t e = launch_histogram(in, n, v.hdr, v.xcd_part, v.seg_hist, nullptr,
                                  kHistSegment | kHistGlobal | kHistBuildTable, (uint32_t)mode,
                                  table_out, stream);
  if (e != hipSuccess) return QLC_ERR_HIP;
  return hip_status(launch_encode(in, n, table_out, v.seg_hist, log2c,
                                  reinterpret_cast<uint32_t*>(bits_out), bits_capacity_bytes / 4,
                                  chunk_index_out, total_bits_out, err_out, v.hdr, v.seg_word,
                                  stream));
}

qlc_status qlc_decode(const uint8_t* bits, const uint64_t* total_bits, const uint64_t* chunk_index,
                      uint32_t chunk_symbols, const qlc_table* table, uint64_t n, uint8_t* out,
                      uint32_t* err_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  uint32_t log2c = 0;
  if (!valid_chunk(chunk_symbols, &log2c) || n >= QLC_MAX_SYMBOLS_PER_CALL)
    return QLC_ERR_INVALID_ARGUMENT;
  if (!total_bits || !table || !err_out || !ws || (n && (!bits || !chunk_index || !out)))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!aligned(bits, 16) || !aligned(total_bits, 8) || !aligned(chunk_index, 8) ||
      !aligned(table, 16) || !aligned(out, 16) || !aligned(err_out, 4) || !aligned(ws, 256))
    return QLC_ERR_INVALID_ARGUMENT;
  if (ws_bytes < ws_bytes_for(0)) return QLC_ERR_INVALID_ARGUMENT;
  WsView v = carve(ws, 0);
  return hip_status(launch_decode(bits, total_bits, chunk_index, log2c, table, n, out, err_out,
                                  v.hdr, stream));
}

qlc_status qlc_table_serialize(const qlc_table* h_table, uint8_t h_out[QLC_SERIALIZED_TABLE_BYTES]) {
  if (!h_table || !h_out) return QLC_ERR_INVALID_ARGUMENT;
  memcpy(h_out, h_table->width, 8);
  memcpy(h_out + 8, h_table->rank_to_sym, 256);
  return QLC_OK;
}

qlc_status qlc_table_deserialize(const uint8_t h_in[QLC_SERIALIZED_TABLE_BYTES], qlc_table* t) {
  if (!h_in || !t) return QLC_ERR_INVALID_ARGUMENT;
  uint32_t w[8];
  for (int a = 0; a < 8; ++a) {
    w[a] = h_in[a];
    if (w[a] > 8 || (a && w[a] < w[a - 1])) return QLC_ERR_INVALID_ARGUMENT;
  }
  uint32_t f = 0, first[8], count[8];
  for (int a = 0; a < 8; ++a) {
    const uint32_t cap = 1u << w[a];
    first[a] = f;
    count[a] = cap < 256 - f ? cap : 256 - f;
    if (count[a] == 0) return QLC_ERR_INVALID_ARGUMENT;
    f += count[a];
  }
  if (f != 256) return QLC_ERR_INVALID_ARGUMENT;
  bool seen[256] = {};
  for (int r = 0; r < 256; ++r) {
    if (seen[h_in[8 + r]]) return QLC_ERR_INVALID_ARGUMENT;
    seen[h_in[8 + r]] = true;
  }
  memset(t, 0, sizeof(*t));
  for (int a = 0; a < 8; ++a) {
    t->width[a] = (uint8_t)w[a];
    t->first[a] = (uint16_t)first[a];
    t->count[a] = (uint16_t)count[a];
    t->offset[a] = (uint8_t)(w[a] == 8 ? 0 : first[a]);
  }
  for (int r = 0; r < 256; ++r) {
    const uint32_t s = h_in[8 + r];
    t->rank_to_sym[r] = (uint8_t)s;
    t->sym_to_rank[s] = (uint8_t)r;
    uint32_t a = 0;
    for (int k = 1; k < 8; ++k) a = (uint32_t)r >= first[k] ? (uint32_t)k : a;
    const uint32_t code = (a << w[a]) | ((uint32_t)r - t->offset[a]);
    t->enc[s] = (uint16_t)(((3 + w[a]) << 11) | code);
  }
  t->cost_bits = 0;
  t->mode = 0xFFFFFFFFu;
  t->version = QLC_ABI_VERSION;
  return QLC_OK;
}

}  // extern "C"
