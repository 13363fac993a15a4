// Instantiations of the one-launch recurrent layer for up to 128 neurons (two
// groups of 64 per workgroup, the block forward's segmentation of T_R).
#include "alif_recurrent_impl.h"

namespace alif {
#define ALIF_REC2(S, L) ALIF_INSTANTIATE_REC(S, L, 2)
ALIF_REC2(1, 2) ALIF_REC2(1, 3) ALIF_REC2(1, 4) ALIF_REC2(2, 3) ALIF_REC2(2, 4) ALIF_REC2(4, 3) ALIF_REC2(4, 4)
ALIF_REC2(4, 5) ALIF_REC2(4, 6) ALIF_REC2(4, 8) ALIF_REC2(8, 5) ALIF_REC2(8, 6) ALIF_REC2(8, 8) ALIF_REC2(8, 10)
ALIF_REC2(8, 12) ALIF_REC2(8, 13) ALIF_REC2(8, 14) ALIF_REC2(8, 15) ALIF_REC2(8, 16)
}  // namespace alif
