// Instantiations of the block-wise kernels with 8 time segments of 10, 12 or 16 steps
// (T_R 65-96 and 121-128; separate from the shorter ones so that the two compile in parallel).
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(8, 10)
ALIF_INSTANTIATE(8, 12)
ALIF_INSTANTIATE(8, 16)
}  // namespace alif
