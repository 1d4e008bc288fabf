// Device-wide sort and scan primitives used by the event stream (own kernels
// for gfx950, in their own translation unit).  Each call with tmp == nullptr
// only stores the scratch size it needs in tmp_bytes; otherwise tmp must hold
// that many bytes (hipErrorInvalidValue if it does not).  All work is queued on
// `stream`.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace nh_sort {

// Stable sort of (key, value) pairs by the low end_bit bits of the keys.
hipError_t sort_pairs_u64(void *tmp, size_t &tmp_bytes, const uint64_t *k_in, uint64_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream);
hipError_t sort_pairs_u32(void *tmp, size_t &tmp_bytes, const uint32_t *k_in, uint32_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream);

// out[i] = sum of in[0 .. i-1].
hipError_t exclusive_sum_u64(void *tmp, size_t &tmp_bytes, const uint64_t *in, uint64_t *out, uint32_t n,
                             hipStream_t stream);
hipError_t exclusive_sum_u32(void *tmp, size_t &tmp_bytes, const uint32_t *in, uint32_t *out, uint32_t n,
                             hipStream_t stream);

} // namespace nh_sort
