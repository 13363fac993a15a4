// Large BF16 MFMA GEMM for gfx950: the Eq. 3 projections of wide layers and their
// gradients (current I = b + x W^T, input gradient dx = gI W, weight gradient
// dW = gI^T x) when every dimension is a few hundred or more.
//
// C[M][N] (+ bias[N]) = sum_k A(m, k) B(n, k), FP32 accumulation of bfloat16
// products. Each operand is stored either k-contiguous ([rows][k], "K-major") or
// row-contiguous ([k][rows], "R-major") and may be float, uint8 (spike counts) or
// bfloat16; it is rounded to bfloat16 (nearest even; integers up to 256 and 0/1
// spikes exactly) while it is staged through LDS.
//
// Tiling. A workgroup owns a 256 x 256 tile of C. With 512 threads (eight waves,
// two per SIMD, so one wave's MFMAs run while the other converts, stores to LDS or
// waits) each wave owns 128 x 64 as 4 x 2 accumulators of
// v_mfma_f32_32x32x16_bf16; operand pairs that need more registers (float x float,
// a row-contiguous bfloat16 B) run 256 threads, 128 x 128 per wave. K moves
// through two LDS buffers in stages of 64 (128 KiB, one workgroup per CU). LDS
// rows hold 64 k of one operand row in eight 16-byte chunks; chunk c of row r
// sits at position c ^ ((r ^ (r >> 3)) & 7), so the MFMA fragment reads (32
// consecutive rows, one chunk each) and the transposing stores of R-major
// operands (rows 4 or 8 apart per lane) both spread over all banks.
//
// Pipeline. One register stage in flight: the loads of stage s + 1 are issued
// while stage s is multiplied; they are converted and stored to the free LDS
// buffer between the MFMAs of the next stage's first half, then the loads of
// stage s + 2 go out. One barrier per stage.
//
// A split of the k range over workgroups (for the weight gradient, whose
// reduction runs over B T rows) writes partial tiles that a fixed-order reduce
// sums, so results do not depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "alif_gemm.h"

namespace alif {

// whether the large-tile BF16 path covers this call (shapes, layouts, alignment)
bool gemm_big_ok(const GemmArgs &g);
// launch it; splits the k range as g.splits asks (partials in g.C_part, reduced into g.C)
hipError_t gemm_big_launch(const GemmArgs &g, hipStream_t st);

}  // namespace alif
