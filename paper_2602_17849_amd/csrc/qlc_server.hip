// libqlc serving loop: admission of compress / decompress requests against
// a device-memory budget, continuous batching of the admitted requests into
// ticks of the batched entry points, several ticks in flight on their own
// streams.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qlc.h"
#include "qlc_server.h"
#include "qlc_internal.h"
#include "qlc_kernels.h"

namespace qlc {
namespace {

constexpr uint64_t kAlign = 256;
constexpr uint32_t kDefaultJobs = 256;
constexpr uint32_t kMaxJobs = 65536;
constexpr uint32_t kDefaultTicks = 2;
constexpr uint32_t kMaxTicks = 8;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint64_t round_up(uint64_t x, uint64_t a = kAlign) { return (x + a - 1) / a * a; }

bool is_aligned(const void* p, uintptr_t a) {
  return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

// Per-job (total_bits, err) of a tick into one array of pinned, mapped host
// memory, which the host reads once the tick's event has completed (no
// device-to-host copy).
__global__ void k_gather_status(const qlc_job* __restrict__ jobs, uint32_t n,
                                uint64_t* __restrict__ status) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    status[2 * j] = *jobs[j].total_bits;
    status[2 * j + 1] = *jobs[j].err;
  }
}

// The same for a tick of one request, from its two status words.
__global__ void k_gather_one(const uint64_t* __restrict__ total, const uint32_t* __restrict__ err,
                             uint64_t* __restrict__ status) {
  if (threadIdx.x == 0) {
    status[0] = *total;
    status[1] = *err;
  }
}

// The largest ws_bytes_for(n) over 0 <= n <= N.  The segment count is not
// monotone in n (one more symbol can double the segment size), but it is
// within each stretch of equal seg_log2, so the maximum sits at N or just
// below a point where seg_log2 steps: n = 2^k (the square-root rule),
// n = 1025 * 2^l (the ~1024-segment rule) or n = (2^24 + 1) * 2^l (the cap).
inline size_t ws_bytes_upto(uint64_t N) {
  size_t m = ws_bytes_for(N);
  for (uint32_t k = 1; k < 64; ++k) {
    const uint64_t cands[3] = {
        (1ull << k) - 1,
        k <= 53 ? 1025ull * (1ull << k) - 1 : ~0ull,
        k <= 39 ? ((1ull << 24) + 1) * (1ull << k) - 1 : ~0ull};
    for (const uint64_t n : cands) {
      if (n > N) continue;
      const size_t b = ws_bytes_for(n);
      if (b > m) m = b;
    }
  }
  return m;
}

// First-fit allocator over [0, capacity) with coalescing of free blocks.
class Pool {
 public:
  void init(uint64_t cap) {
    free_.clear();
    free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(uint64_t size, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < size) continue;
      *off = it->first;
      const uint64_t rest = it->second - size, next = it->first + size;
      free_.erase(it);
      if (rest) free_[next] = rest;
      used_ += size;
      if (used_ > peak_) peak_ = used_;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t size) {
    used_ -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  uint64_t used_ = 0, peak_ = 0;
};

struct Request {
  uint64_t id = 0;
  qlc_request r{};
  uint64_t reserve = 0, off = 0;
  uint64_t submit_ns = 0, admit_ns = 0, complete_ns = 0;
  qlc_job job{};
  uint32_t status = 0;
  uint64_t total = 0;
  bool completed = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* plain_ws = nullptr;      // single-tensor workspace (ticks of one request)
  size_t plain_ws_bytes = 0;
  qlc_job* d_jobs = nullptr;   // compress jobs, then decompress jobs
  qlc_job* h_jobs = nullptr;   // pinned staging of d_jobs
  uint64_t* h_status = nullptr;      // pinned, mapped: (total_bits, err) per job
  uint64_t* h_status_dev = nullptr;  // its device-side address
  std::vector<Request*> enc, dec;
  bool busy = false;
};

}  // namespace
}  // namespace qlc

using namespace qlc;

struct qlc_server {
  qlc_server_config cfg{};
  qlc_batch_tuning tuning{};
  int device = 0;
  uint8_t* pool_base = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending, done_q;
  std::unordered_map<uint64_t, Request*> live;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread th;
  uint64_t submitted = 0, rejected = 0, completed = 0, ticks = 0;
  uint32_t max_jobs_seen = 0, max_busy_seen = 0;

  uint64_t chunks(uint64_t n) const {
    return (n + cfg.chunk_symbols - 1) / cfg.chunk_symbols;
  }
  // Bitstream bytes reserved for a compress request.  A table the server
  // searches from the request's own histogram never costs more than 8 bits
  // per symbol (every search mode has an all-equal-length candidate of 8
  // bits), so n + 16 bytes hold its stream; a caller's table, or the fixed
  // widths of Table 1 or Table 2 (9.59 bits per symbol on uniform bytes),
  // get the 11-bit bound.
  uint64_t bits_capacity(const qlc_request& r) const {
    const bool searched = cfg.layout_mode != QLC_LAYOUT_PAPER_T1 &&
                          cfg.layout_mode != QLC_LAYOUT_PAPER_T2;
    return (r.table || !searched) ? qlc_encode_bound_bytes(r.n) : round_up(r.n + 16, 16);
  }
  // Pool bytes a request holds from admission to release.
  uint64_t reservation(const qlc_request& r) const {
    if (r.kind == QLC_REQUEST_DECOMPRESS) return round_up(r.n ? r.n : 1) + kAlign;
    const uint64_t cap = bits_capacity(r);
    const uint64_t idx = 8 * (chunks(r.n) ? chunks(r.n) : 1);
    return (r.table ? 0 : round_up(sizeof(qlc_table))) + kAlign + round_up(idx) + round_up(cap);
  }

  // Point the request's job at its pool block.
  void carve(Request* q) {
    uint8_t* b = pool_base + q->off;
    const qlc_request& r = q->r;
    qlc_job& j = q->job;
    j = qlc_job{};
    j.n = r.n;
    if (r.kind == QLC_REQUEST_DECOMPRESS) {
      j.out = b;
      j.err = reinterpret_cast<uint32_t*>(b + round_up(r.n ? r.n : 1));
      j.table = const_cast<qlc_table*>(r.table);
      j.bits = const_cast<uint8_t*>(r.bits);
      j.chunk_index = const_cast<uint64_t*>(r.chunk_index);
      j.total_bits = const_cast<uint64_t*>(r.total_bits);
      return;
    }
    j.in = r.in;
    if (r.table) {
      j.table = const_cast<qlc_table*>(r.table);
      j.build_table = 0;
    } else {
      j.table = reinterpret_cast<qlc_table*>(b);
      j.build_table = 1;
      b += round_up(sizeof(qlc_table));
    }
    j.total_bits = reinterpret_cast<uint64_t*>(b);
    j.err = reinterpret_cast<uint32_t*>(b + 8);
    b += kAlign;
    j.chunk_index = reinterpret_cast<uint64_t*>(b);
    b += round_up(8 * (chunks(r.n) ? chunks(r.n) : 1));
    j.bits = b;
    j.bits_capacity = bits_capacity(r);
  }

  // Admit queued requests into a free slot (arrival order, within budget).
  bool admit(Slot& sl) {
    uint64_t syms = 0;
    const uint64_t t = now_ns();
    while (!pending.empty() && sl.enc.size() + sl.dec.size() < cfg.max_jobs_per_tick) {
      Request* q = pending.front();
      if (syms + q->r.n > cfg.max_tick_symbols) break;
      uint64_t off = 0;
      if (!pool.alloc(q->reserve, &off)) break;
      q->off = off;
      q->admit_ns = t;
      carve(q);
      pending.pop_front();
      (q->r.kind == QLC_REQUEST_COMPRESS ? sl.enc : sl.dec).push_back(q);
      syms += q->r.n;
    }
    return !sl.enc.empty() || !sl.dec.empty();
  }

  // Enqueue one tick on the slot's stream; false if a HIP call failed.
  bool launch(Slot& sl) {
    const uint32_t ne = (uint32_t)sl.enc.size(), nd = (uint32_t)sl.dec.size();
    for (uint32_t i = 0; i < ne; ++i) sl.h_jobs[i] = sl.enc[i]->job;
    for (uint32_t i = 0; i < nd; ++i) sl.h_jobs[ne + i] = sl.dec[i]->job;
    if (ne + nd == 1) {
      // A tick of one request runs the single-tensor entry points: for one
      // job they cost less than the persistent batched launch (no job-array
      // copy, plan kernel, work queue or cross-workgroup flags), with the
      // same bytes out.
      const qlc_job& j = sl.h_jobs[0];
      qlc_status st;
      if (ne && j.build_table)
        st = qlc_compress(j.in, j.n, (qlc_layout_mode)cfg.layout_mode, j.table, cfg.chunk_symbols,
                          j.bits, j.bits_capacity, j.chunk_index, j.total_bits, j.err,
                          sl.plain_ws, sl.plain_ws_bytes, sl.stream);
      else if (ne)
        st = qlc_encode(j.in, j.n, j.table, cfg.chunk_symbols, j.bits, j.bits_capacity,
                        j.chunk_index, j.total_bits, j.err, sl.plain_ws, sl.plain_ws_bytes,
                        sl.stream);
      else
        st = qlc_decode_ex(j.bits, j.total_bits, j.chunk_index, cfg.chunk_symbols, j.table, j.n,
                           8, (qlc_decoder)cfg.decoder, j.out, j.err, sl.plain_ws,
                           sl.plain_ws_bytes, sl.stream);
      if (st != QLC_OK) return false;
      hipLaunchKernelGGL(k_gather_one, dim3(1), dim3(64), 0, sl.stream, j.total_bits, j.err,
                         sl.h_status_dev);
    } else {
      if (hipMemcpyAsync(sl.d_jobs, sl.h_jobs, sizeof(qlc_job) * (ne + nd),
                         hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        return false;
      if (ne && qlc_encode_batched(sl.d_jobs, ne, (qlc_layout_mode)cfg.layout_mode,
                                   cfg.chunk_symbols, &tuning, sl.ws, sl.ws_bytes,
                                   sl.stream) != QLC_OK)
        return false;
      if (nd && qlc_decode_batched(sl.d_jobs + ne, nd, cfg.chunk_symbols, &tuning, sl.ws,
                                   sl.ws_bytes, sl.stream) != QLC_OK)
        return false;
      hipLaunchKernelGGL(k_gather_status, dim3((ne + nd + 255) / 256), dim3(256), 0, sl.stream,
                         sl.d_jobs, ne + nd, sl.h_status_dev);
    }
    if (hipGetLastError() != hipSuccess) return false;
    return hipEventRecord(sl.done, sl.stream) == hipSuccess;
  }

  void finish(Slot& sl, bool ok) {
    const uint64_t t = now_ns();
    const uint32_t ne = (uint32_t)sl.enc.size();
    auto complete = [&](Request* q, uint32_t j) {
      q->status = ok ? (uint32_t)sl.h_status[2 * j + 1] : (uint32_t)QLC_ERR_HIP;
      q->total = ok ? sl.h_status[2 * j] : 0;
      q->complete_ns = t;
      q->completed = true;
      done_q.push_back(q);
      ++completed;
    };
    for (uint32_t i = 0; i < ne; ++i) complete(sl.enc[i], i);
    for (uint32_t i = 0; i < sl.dec.size(); ++i) complete(sl.dec[i], ne + i);
    sl.enc.clear();
    sl.dec.clear();
    sl.busy = false;
    cv_done.notify_all();
  }

  void run() {
    // if the loop's thread cannot select the device, every tick fails (its
    // requests complete with QLC_ERR_HIP) instead of running elsewhere
    const bool dev_ok = hipSetDevice(device) == hipSuccess;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      uint32_t busy = 0;
      for (Slot& sl : slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) finish(sl, true);
        else if (q == hipErrorNotReady) ++busy;
        else finish(sl, false);
      }
      Slot* fs = nullptr;
      for (Slot& sl : slots)
        if (!sl.busy) {
          fs = &sl;
          break;
        }
      if (fs && !pending.empty() && admit(*fs)) {
        fs->busy = true;
        ++ticks;
        const uint32_t nj = (uint32_t)(fs->enc.size() + fs->dec.size());
        if (nj > max_jobs_seen) max_jobs_seen = nj;
        if (busy + 1 > max_busy_seen) max_busy_seen = busy + 1;
        lk.unlock();
        const bool ok = dev_ok && launch(*fs);
        // after a failed launch, let whatever was enqueued drain before the
        // requests' memory can be released
        if (!ok) (void)hipStreamSynchronize(fs->stream);
        lk.lock();
        if (!ok) finish(*fs, false);
        continue;
      }
      if (stop && pending.empty() && busy == 0) break;
      if (busy) {
        // a tick is on the device: poll its event without sleeping, so a
        // completion is seen within microseconds
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_work.wait(lk);
      }
    }
  }

  void free_all() {
    for (Slot& sl : slots) {
      if (sl.ws) (void)hipFree(sl.ws);
      if (sl.plain_ws) (void)hipFree(sl.plain_ws);
      if (sl.d_jobs) (void)hipFree(sl.d_jobs);
      if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
      if (sl.h_status) (void)hipHostFree(sl.h_status);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    slots.clear();
    if (pool_base) (void)hipFree(pool_base);
    pool_base = nullptr;
    for (auto& kv : live) delete kv.second;
    live.clear();
  }
};

extern "C" {

qlc_status qlc_server_create(const qlc_server_config* h_config, qlc_server** out) {
  if (!h_config || !out) return QLC_ERR_INVALID_ARGUMENT;
  qlc_server_config c = *h_config;
  const uint32_t C = c.chunk_symbols;
  if (c.memory_budget_bytes == 0 || C < QLC_MIN_CHUNK || C > QLC_MAX_CHUNK || (C & (C - 1)) ||
      !valid_layout_mode(c.layout_mode) || mode_symbol_bits(c.layout_mode) != 8 ||
      c.max_jobs_per_tick > kMaxJobs ||
      c.max_ticks_in_flight > kMaxTicks ||
      (c.decoder != QLC_DECODER_AUTO && c.decoder != QLC_DECODER_LANE &&
       c.decoder != QLC_DECODER_SPLIT) ||
      (c.decoder == QLC_DECODER_SPLIT && C > (1u << kSplitMaxLog2Chunk)) ||
      (c.log2_segment && (c.log2_segment < 13 || c.log2_segment > 24)))
    return QLC_ERR_INVALID_ARGUMENT;
  if (!c.max_jobs_per_tick) c.max_jobs_per_tick = kDefaultJobs;
  if (!c.max_ticks_in_flight) c.max_ticks_in_flight = kDefaultTicks;
  if (!c.max_tick_symbols || c.max_tick_symbols > c.memory_budget_bytes)
    c.max_tick_symbols = c.memory_budget_bytes;

  qlc_server* s = new (std::nothrow) qlc_server();
  if (!s) return QLC_ERR_HIP;
  s->cfg = c;
  s->tuning = qlc_batch_tuning{c.log2_segment, 0, 0, c.decoder};
  bool ok = hipGetDevice(&s->device) == hipSuccess &&
            hipMalloc((void**)&s->pool_base, c.memory_budget_bytes) == hipSuccess;
  s->pool.init(c.memory_budget_bytes);
  s->slots.resize(ok ? c.max_ticks_in_flight : 0);
  for (Slot& sl : s->slots) {
    sl.ws_bytes = qlc_batched_workspace_bytes(c.max_jobs_per_tick, c.max_tick_symbols, C,
                                              &s->tuning);
    sl.plain_ws_bytes = ws_bytes_upto(c.max_tick_symbols);  // any request size up to it
    ok = ok && sl.ws_bytes && sl.plain_ws_bytes &&
         hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
         hipMalloc(&sl.ws, sl.ws_bytes) == hipSuccess &&
         hipMalloc((void**)&sl.d_jobs, sizeof(qlc_job) * c.max_jobs_per_tick) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_jobs, sizeof(qlc_job) * c.max_jobs_per_tick) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_status, 16ull * c.max_jobs_per_tick,
                       hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
         hipHostGetDevicePointer((void**)&sl.h_status_dev, sl.h_status, 0) == hipSuccess &&
         qlc_workspace_init(sl.ws, sl.ws_bytes, sl.stream) == QLC_OK &&
         hipMalloc(&sl.plain_ws, sl.plain_ws_bytes) == hipSuccess &&
         qlc_workspace_init(sl.plain_ws, sl.plain_ws_bytes, sl.stream) == QLC_OK &&
         hipStreamSynchronize(sl.stream) == hipSuccess;
    if (!ok) break;
  }
  if (!ok) {
    s->free_all();
    delete s;
    return QLC_ERR_HIP;
  }
  try {
    s->th = std::thread([s] { s->run(); });
  } catch (...) {  // no exception may cross the C ABI
    s->free_all();
    delete s;
    return QLC_ERR_HIP;
  }
  *out = s;
  return QLC_OK;
}

qlc_status qlc_server_submit(qlc_server* s, const qlc_request* h_req, uint64_t* id_out) {
  if (!s || !h_req || !id_out) return QLC_ERR_INVALID_ARGUMENT;
  const qlc_request r = *h_req;
  if (r.reserved || r.n >= QLC_MAX_SYMBOLS_PER_CALL) return QLC_ERR_INVALID_ARGUMENT;
  if (r.kind == QLC_REQUEST_COMPRESS) {
    if ((r.n && !r.in) || !is_aligned(r.in, 16) || !is_aligned(r.table, 16))
      return QLC_ERR_INVALID_ARGUMENT;
  } else if (r.kind == QLC_REQUEST_DECOMPRESS) {
    if (!r.table || !r.total_bits || (r.n && (!r.bits || !r.chunk_index)) ||
        !is_aligned(r.table, 16) || !is_aligned(r.bits, 16) || !is_aligned(r.chunk_index, 8) ||
        !is_aligned(r.total_bits, 8))
      return QLC_ERR_INVALID_ARGUMENT;
  } else {
    return QLC_ERR_INVALID_ARGUMENT;
  }
  Request* q = new (std::nothrow) Request();
  if (!q) return QLC_ERR_HIP;
  q->r = r;
  q->reserve = s->reservation(r);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) {
    delete q;
    return QLC_ERR_BUSY;
  }
  if (q->reserve > s->cfg.memory_budget_bytes || r.n > s->cfg.max_tick_symbols) {
    ++s->rejected;
    delete q;
    return QLC_ERR_CAPACITY;
  }
  q->id = s->next_id++;
  q->submit_ns = now_ns();
  try {
    s->live[q->id] = q;
    s->pending.push_back(q);
  } catch (...) {  // out of host memory: no exception may cross the C ABI
    s->live.erase(q->id);
    delete q;
    return QLC_ERR_HIP;
  }
  ++s->submitted;
  *id_out = q->id;
  s->cv_work.notify_one();
  return QLC_OK;
}

uint32_t qlc_server_poll(qlc_server* s, qlc_result* out, uint32_t max_results, int64_t timeout_us) {
  if (!s || !out || !max_results) return 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done_q.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [s] { return !s->done_q.empty(); });
  uint32_t k = 0;
  while (k < max_results && !s->done_q.empty()) {
    Request* q = s->done_q.front();
    s->done_q.pop_front();
    qlc_result& o = out[k++];
    o = qlc_result{};
    o.id = q->id;
    o.user_tag = q->r.user_tag;
    o.kind = q->r.kind;
    o.status = q->status;
    o.n = q->r.n;
    o.submit_ns = q->submit_ns;
    o.admit_ns = q->admit_ns;
    o.complete_ns = q->complete_ns;
    if (q->r.kind == QLC_REQUEST_COMPRESS) {
      o.total_bits = q->total;
      o.table = q->job.table;
      o.bits = q->job.bits;
      o.chunk_index = q->job.chunk_index;
      o.total_bits_dev = q->job.total_bits;
    } else {
      o.out = q->job.out;
    }
  }
  return k;
}

qlc_status qlc_server_release(qlc_server* s, uint64_t id) {
  if (!s) return QLC_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) return QLC_ERR_INVALID_ARGUMENT;
  Request* q = it->second;
  if (!q->completed) return QLC_ERR_BUSY;
  s->pool.release(q->off, q->reserve);
  s->live.erase(it);
  delete q;
  s->cv_work.notify_one();
  return QLC_OK;
}

qlc_status qlc_server_get_stats(qlc_server* s, qlc_server_stats* out) {
  if (!s || !out) return QLC_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(s->mu);
  *out = qlc_server_stats{};
  out->budget_bytes = s->cfg.memory_budget_bytes;
  out->bytes_in_use = s->pool.used();
  out->peak_bytes_in_use = s->pool.peak();
  out->submitted = s->submitted;
  out->rejected = s->rejected;
  out->completed = s->completed;
  out->ticks = s->ticks;
  out->max_jobs_in_tick = s->max_jobs_seen;
  out->max_ticks_in_flight = s->max_busy_seen;
  out->queued = (uint32_t)s->pending.size();
  return QLC_OK;
}

qlc_status qlc_server_destroy(qlc_server* s) {
  if (!s) return QLC_ERR_INVALID_ARGUMENT;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  // Requests that can never be admitted (memory held by unreleased
  // results) would keep the loop waiting: release is the caller's job, so
  // destroy frees every completed result first.
  for (;;) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (auto it = s->live.begin(); it != s->live.end();) {
      Request* q = it->second;
      if (q->completed) {
        s->pool.release(q->off, q->reserve);
        delete q;
        it = s->live.erase(it);
      } else {
        ++it;
      }
    }
    s->done_q.clear();
    s->cv_work.notify_all();
    const bool idle = s->live.empty();
    lk.unlock();
    if (idle) break;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  s->th.join();
  s->free_all();
  delete s;
  return QLC_OK;
}

}  // extern "C"
