// Segmented sort instantiations for 64-bit keys.
#include "ms_seg_launch.hpp"

namespace ms {
MS_SEG_INSTANTIATE(uint64_t, NoVal)
MS_SEG_INSTANTIATE(uint64_t, uint32_t)
MS_SEG_INSTANTIATE(uint64_t, uint64_t)
MS_SEG_INSTANTIATE(int64_t, NoVal)
MS_SEG_INSTANTIATE(int64_t, uint32_t)
MS_SEG_INSTANTIATE(int64_t, uint64_t)
MS_DEFINE_DEV_ERRORS(dev_errors_seg64)
}  // namespace ms
