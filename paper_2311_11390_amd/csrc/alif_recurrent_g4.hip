// Instantiations of the one-launch recurrent layer for 129-256 neurons (four
// groups of 64 per workgroup, so at most four segments: T_R <= 64).
#include "alif_recurrent_impl.h"

namespace alif {
#define ALIF_REC4(S, L) ALIF_INSTANTIATE_REC(S, L, 4)
ALIF_REC4(1, 2) ALIF_REC4(1, 3) ALIF_REC4(1, 4) ALIF_REC4(2, 3) ALIF_REC4(2, 4) ALIF_REC4(4, 3) ALIF_REC4(4, 4)
ALIF_REC4(4, 5) ALIF_REC4(4, 6) ALIF_REC4(4, 8) ALIF_REC4(4, 9) ALIF_REC4(4, 10) ALIF_REC4(4, 11) ALIF_REC4(4, 12)
ALIF_REC4(4, 13) ALIF_REC4(4, 14) ALIF_REC4(4, 15) ALIF_REC4(4, 16)
}  // namespace alif
