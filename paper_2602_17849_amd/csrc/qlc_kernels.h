// Host-side launchers of the libqlc kernels (defined in qlc_kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "qlc_internal.h"

namespace qlc {

hipError_t launch_histogram(const uint8_t* in, uint64_t n, WsHeader* hdr, uint64_t* xcd_part,
                            uint32_t* seg_hist, uint64_t* hist_out, uint32_t flags, uint32_t mode,
                            qlc_table* table_out, hipStream_t stream);
hipError_t launch_table_from_hist(const uint64_t* hist, uint32_t mode, qlc_table* out,
                                  hipStream_t stream);
hipError_t launch_encode(const uint8_t* in, uint64_t n, const qlc_table* table,
                         const uint32_t* seg_hist, uint32_t log2_chunk, uint32_t* bits_out,
                         uint64_t cap_words, uint64_t* index_out, uint64_t* total_out,
                         uint32_t* err_out, WsHeader* hdr, uint64_t* seg_word, hipStream_t stream);
hipError_t launch_decode(const uint8_t* bits, const uint64_t* total, const uint64_t* index,
                         uint32_t log2_chunk, const qlc_table* table, uint64_t n, uint8_t* out,
                         uint32_t* err_out, WsHeader* hdr, hipStream_t stream);
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t stream);

}  // namespace qlc
