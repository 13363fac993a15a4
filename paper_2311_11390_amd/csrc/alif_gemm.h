// MFMA GEMMs for the dense projections around an ALIF layer (paper Eq. 3):
// input current I~ = b + W x (forward), weight gradient dW = gI^T x and input
// gradient dx = gI W (backward). FP32 MFMA or BF16 MFMA with FP32 accumulation.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace alif {

struct GemmIn {
    int kind;         // ALIF_INPUT_SPIKES_U8 / _BF16 / _F32 (enum alif_input_kind)
    const void *ptr;  // [M][K] row-major
};

// out[M][N] = bias[N] + x[M][K] . W[N][K]^T. With bf16, a scratch of at least
// gemm_wbf16_bytes(N, K) bytes (16-byte aligned; nullptr: none) receives W rounded
// to bfloat16 once, so that the GEMM streams half the weight bytes and converts
// only x.
hipError_t gemm_input_current(size_t M, int N, int K, GemmIn x, const float *W, const float *bias,
                              float *out, bool bf16, hipStream_t st, void *scratch = nullptr,
                              size_t scratch_bytes = 0);
// bytes of the bfloat16 copy of a [N][K] weight matrix, as is or transposed, with
// rows padded to 16 bytes
size_t gemm_wbf16_bytes(int N, int K);
// gW[N][K] = sum_m gI[m][n] x[m][k]   (split over m, reduced in a fixed order);
// skip_cnt / skip_le: the device-side gate of GemmArgs. gI is float, or bfloat16
// with gi_bf16 (then bf16 must be set: the product is the BF16 one).
hipError_t gemm_weight_grad(size_t M, int N, int K, const void *gI, GemmIn x, float *gW, bool bf16,
                            void *ws, hipStream_t st, const unsigned long long *skip_cnt = nullptr,
                            unsigned long long skip_le = 0, bool gi_bf16 = false);
// gx[M][K] = gI[M][N] . W[N][K]. With bf16, a scratch of gemm_wbf16_bytes(N, K)
// bytes (as above) receives W transposed and rounded to bfloat16 once. gI as in
// gemm_weight_grad.
hipError_t gemm_input_grad(size_t M, int N, int K, const void *gI, const float *W, float *gx,
                           bool bf16, hipStream_t st, void *scratch = nullptr, size_t scratch_bytes = 0,
                           bool gi_bf16 = false);
// scratch bytes gemm_weight_grad needs for its split partial sums
size_t gemm_workspace_bytes(size_t M, int N, int K);

// Sparse spike input (alif_events.hip, alif_recurrent_wgrad.hip):
// density_flag_launch writes *flag = 0 when a fixed sample of whole rows of x
// ([rows][cols] of elem-byte elements) has at most cut_num / cut_den nonzero
// entries, else ~0 (one workgroup). events_current_launch writes W [N][n_in]
// transposed into WT (n_in x N floats; values rounded to bfloat16 with
// round_bf16) and then C = bias + x W^T from the active inputs only, its kernel
// returning at entry unless *gate == 0; false (nothing launched) for shapes or
// alignments it does not take.
hipError_t density_flag_launch(long long rows, int cols, int elem, const void *x, unsigned long long *flag,
                               int cut_num, int cut_den, hipStream_t st);
bool events_current_launch(int kind, long long M, int n_in, int N, const void *x, const float *W, float *WT,
                           bool round_bf16, const float *bias, float *C, const unsigned long long *gate,
                           hipStream_t st);

// general C[M][N] = sum_k A(m, k) B(n, k) (+ bias[n]) for tests and readout
struct GemmArgs {
    long long M;
    int N, K;
    const void *A;
    int a_dt;          // 0 float, 1 uint8, 2 bf16
    long long lda;
    int a_kc;          // 1: A(m, k) = A[m * lda + k]; 0: A(m, k) = A[k * lda + m]
    const void *B;
    int b_dt;
    long long ldb;
    int b_kc;          // 1: B(n, k) = B[n * ldb + k]; 0: B(n, k) = B[k * ldb + n]
    float *C;
    long long ldc;
    const float *bias;
    int splits;        // split of K over blockIdx.z; > 1 writes partials to C_part
    float *C_part;     // [splits][M][N]
    // Device-side gate: with skip_cnt set, every kernel of the launch returns at
    // entry when *skip_cnt <= skip_le as it starts, and C is left alone (a caller
    // that picks between this GEMM and another way of computing C on the device).
    const unsigned long long *skip_cnt;
    unsigned long long skip_le;
};
__device__ __forceinline__ bool gemm_gated_off(const unsigned long long *cnt, unsigned long long le) {
    return cnt != nullptr && *cnt <= le;
}
hipError_t gemm_launch(const GemmArgs &g, bool bf16, hipStream_t st);

}  // namespace alif
