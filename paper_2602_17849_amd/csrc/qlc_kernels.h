// Host-side launchers of the libqlc kernels (defined in qlc_kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "qlc_internal.h"

namespace qlc {

// `bits`: bits per symbol of the input / output (4, 6 or 8).
hipError_t launch_histogram(const uint8_t* in, uint64_t n, uint32_t bits, WsHeader* hdr,
                            uint64_t* xcd_part, uint32_t* seg_hist, uint64_t* hist_out,
                            uint32_t flags, uint32_t mode, qlc_table* table_out,
                            hipStream_t stream);
hipError_t launch_table_from_hist(const uint64_t* hist, uint32_t mode, qlc_table* out,
                                  hipStream_t stream);
// seg_bits: precomputed segment bit counts, or null to derive them from
// the segment histograms seg_hist.
hipError_t launch_encode(const uint8_t* in, uint64_t n, uint32_t bits, const qlc_table* table,
                         const uint32_t* seg_hist, const uint64_t* seg_bits, uint32_t log2_chunk,
                         uint32_t* bits_out, uint64_t cap_words, uint64_t* index_out,
                         uint64_t* total_out, uint32_t* err_out, WsHeader* hdr, uint64_t* seg_word,
                         hipStream_t stream);
hipError_t launch_segment_bits(const uint8_t* in, uint64_t n, uint32_t bits,
                               const qlc_table* table, uint64_t* seg_bits, hipStream_t stream);
hipError_t launch_decode(const uint8_t* bits_in, const uint64_t* total, const uint64_t* index,
                         uint32_t log2_chunk, const qlc_table* table, uint64_t n, uint32_t bits,
                         uint8_t* out, uint32_t* err_out, WsHeader* hdr, hipStream_t stream);
// Several lanes per chunk (log2_chunk <= kSplitMaxLog2Chunk).
constexpr uint32_t kSplitMaxLog2Chunk = 14;
constexpr uint32_t kSplitUnitLog2 = 14;  // symbols per split unit (one workgroup)
hipError_t launch_decode_split(const uint8_t* bits_in, const uint64_t* total, const uint64_t* index,
                               uint32_t log2_chunk, const qlc_table* table, uint64_t n,
                               uint32_t bits, uint8_t* out, uint32_t* err_out, WsHeader* hdr,
                               hipStream_t stream);
// log2_unit: encode segment size (0: automatic, batch_auto_log2_seg of the
// jobs' symbols), or decode log2 C + kDecThreadsLog2.  decode_split (decode
// only): 0 every job one lane per chunk, 1 automatic (every job in split
// units when batch_split_all holds for the jobs' symbols, else the jobs of
// fewer than kDecThreads chunks), 2 every job in split units.  The plan
// records the segment size in hdr->log2_seg for the encode kernel.
hipError_t launch_batch_plan(const qlc_job* jobs, uint32_t n_jobs, bool decode,
                             uint32_t decode_split, uint32_t log2_unit, uint64_t max_units,
                             uint32_t lag, BatchHeader* hdr, BatchJobState* js, uint64_t* job_hist,
                             uint32_t* unit_job, uint64_t* seg_word, hipStream_t stream);
hipError_t launch_encode_batched(const qlc_job* jobs, uint32_t bits, uint32_t mode,
                                 uint32_t log2_chunk, BatchHeader* hdr, BatchJobState* js,
                                 uint64_t* job_hist, const uint32_t* seg_job, uint64_t* seg_word,
                                 uint32_t* seg_hist, uint32_t grid, hipStream_t stream);
hipError_t launch_decode_batched(const qlc_job* jobs, uint32_t bits, uint32_t log2_chunk,
                                 BatchHeader* hdr, const BatchJobState* js,
                                 const uint32_t* grp_job, uint32_t grid, hipStream_t stream);
// Workgroups of a batched kernel that fit on one compute unit at once.
int batched_blocks_per_cu(bool decode);
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t stream);

}  // namespace qlc
