// Segmented sort instantiations for 32-bit keys.
#include "ms_seg_launch.hpp"

namespace ms {
MS_SEG_INSTANTIATE(uint32_t, NoVal)
MS_SEG_INSTANTIATE(uint32_t, uint32_t)
MS_SEG_INSTANTIATE(uint32_t, uint64_t)
MS_SEG_INSTANTIATE(int32_t, NoVal)
MS_SEG_INSTANTIATE(int32_t, uint32_t)
MS_SEG_INSTANTIATE(int32_t, uint64_t)
MS_DEFINE_DEV_ERRORS(dev_errors_seg32)
}  // namespace ms
