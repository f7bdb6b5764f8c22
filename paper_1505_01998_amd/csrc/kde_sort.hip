// kde_sort.hip -- ascending sort of a column's FP32 working copy for tile
// pruning (the pair sums do not depend on the order of the samples).  Uses
// hipCUB's device radix sort; +inf padding sorts to the end, so the padded
// copy is sorted whole.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "kde_internal.h"

namespace kde {

size_t sort_temp_bytes(int count) {
  size_t bytes = 0;
  if (hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, static_cast<const float*>(nullptr),
                                        static_cast<float*>(nullptr), count) != hipSuccess)
    return 0;
  return bytes;
}

hipError_t sort_keys(void* tmp, size_t tmp_bytes, const float* in, float* out, int count, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, in, out, count, 0, 32, s);
}

}  // namespace kde
