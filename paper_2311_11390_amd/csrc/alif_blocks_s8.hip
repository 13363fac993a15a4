// Instantiations of the block-wise kernels with 8 time segment(s) per neuron.
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(8, 5)
ALIF_INSTANTIATE(8, 6)
ALIF_INSTANTIATE(8, 8)
}  // namespace alif
