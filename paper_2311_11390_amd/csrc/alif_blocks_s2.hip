// Instantiations of the block-wise kernels with 2 time segment(s) per neuron.
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(2, 3)
ALIF_INSTANTIATE(2, 4)
}  // namespace alif
