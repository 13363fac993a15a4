// Instantiations of the block-wise kernels with 4 time segment(s) per neuron.
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(4, 3)
ALIF_INSTANTIATE(4, 4)
ALIF_INSTANTIATE(4, 5)
ALIF_INSTANTIATE(4, 6)
ALIF_INSTANTIATE(4, 8)
}  // namespace alif
