// Instantiations of the block-wise kernels with 8 time segments of 13-15 steps
// (T_R 97-120; a file of their own so that it compiles in parallel with the others).
#include "alif_blocks_impl.h"

namespace alif {
ALIF_INSTANTIATE(8, 13)
ALIF_INSTANTIATE(8, 14)
ALIF_INSTANTIATE(8, 15)
}  // namespace alif
