// hipCUB instantiations behind stream_sort.h.
#include "stream_sort.h"

#include <hipcub/hipcub.hpp>

namespace nh_sort {

hipError_t sort_pairs_u64(void *tmp, size_t &tmp_bytes, const uint64_t *k_in, uint64_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream) {
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k_in, k_out, v_in, v_out, n, 0, end_bit, stream);
}

hipError_t sort_pairs_u32(void *tmp, size_t &tmp_bytes, const uint32_t *k_in, uint32_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream) {
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k_in, k_out, v_in, v_out, n, 0, end_bit, stream);
}

hipError_t exclusive_sum_u64(void *tmp, size_t &tmp_bytes, const uint64_t *in, uint64_t *out, uint32_t n,
                             hipStream_t stream) {
    return hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, n, stream);
}

hipError_t exclusive_sum_u32(void *tmp, size_t &tmp_bytes, const uint32_t *in, uint32_t *out, uint32_t n,
                             hipStream_t stream) {
    return hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, n, stream);
}

} // namespace nh_sort
