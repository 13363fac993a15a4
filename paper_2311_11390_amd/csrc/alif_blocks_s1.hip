// Instantiations of the block-wise kernels with 1 time segment(s) per neuron.
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(1, 2)
ALIF_INSTANTIATE(1, 3)
ALIF_INSTANTIATE(1, 4)
}  // namespace alif
