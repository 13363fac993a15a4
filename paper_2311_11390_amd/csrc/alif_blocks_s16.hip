// Instantiations of the block-wise kernels with 16 time segment(s) per neuron.
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(16, 6)
ALIF_INSTANTIATE(16, 8)
}  // namespace alif
