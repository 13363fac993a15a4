// Event-driven input current of Eq. 3 for sparse spike input.
//
// I~[b][t][i] = bias[i] + sum_j W[i][j] x[b][t][j]. Spike trains are mostly zeros
// (at 10 Hz and DT 0.5 ms, 0.5% of the entries are 1), so instead of a dense GEMM
// each (b, t) row adds only the weight columns of its active inputs:
//   * one 256-thread workgroup per row compacts the nonzero inputs of the row into
//     LDS (wave ballots, in increasing input index), with their values;
//   * each thread then owns output neurons i, i + 256, ... and sums
//     value_e * WT[j_e][i] over the active inputs e in that order (FP32).
// WT is W transposed ([n_in][N], built once by alif_transpose), so that a wave's
// reads of one weight column are 64 consecutive floats. The bytes moved per row
// are the row's inputs, the active columns of WT (L2-resident for layer-sized W)
// and the N floats written.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/blockalif.h"
#include "alif_kernels.h"

namespace alif {
namespace {

constexpr int EV_THREADS = 256;
constexpr int EV_MAX_IN = 16384;   // LDS holds (index, value) for up to this many inputs per row

template <int KIND>
__device__ __forceinline__ float ev_value(const void *x, size_t e) {
    if constexpr (KIND == ALIF_INPUT_SPIKES_U8) return (float)static_cast<const uint8_t *>(x)[e];
    else if constexpr (KIND == ALIF_INPUT_SPIKES_BF16)
        return __uint_as_float((uint32_t)static_cast<const uint16_t *>(x)[e] << 16);
    else return static_cast<const float *>(x)[e];
}

template <int KIND>
__global__ __launch_bounds__(EV_THREADS) void k_events_current(long long M, int n_in, int N, const void *x,
                                                               const float *__restrict__ WT,
                                                               const float *__restrict__ bias,
                                                               float *__restrict__ C) {
    extern __shared__ int ev_smem[];
    int *act = ev_smem;                                          // [n_in]
    float *val = reinterpret_cast<float *>(ev_smem + n_in);     // [n_in]
    __shared__ int wave_cnt[EV_THREADS / 64];
    const long long row = blockIdx.x;
    if (row >= M) return;                                        // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t xrow = (size_t)row * n_in;
    int cnt = 0;
    for (int j0 = 0; j0 < n_in; j0 += EV_THREADS) {
        const int j = j0 + tid;
        const float v = j < n_in ? ev_value<KIND>(x, xrow + j) : 0.0f;
        const bool on = v != 0.0f;
        const unsigned long long m = __ballot(on);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int off = cnt;
        for (int w = 0; w < wave; w++) off += wave_cnt[w];
        if (on) {
            const int q = off + __popcll(m & ((1ull << lane) - 1ull));
            act[q] = j;
            val[q] = v;
        }
        for (int w = 0; w < EV_THREADS / 64; w++) cnt += wave_cnt[w];
        __syncthreads();
    }
    float *crow = C + (size_t)row * N;
    for (int i = tid; i < N; i += EV_THREADS) {
        float s = bias ? bias[i] : 0.0f;
        for (int e = 0; e < cnt; e++) s = fmaf(val[e], WT[(size_t)act[e] * N + i], s);
        crow[i] = s;
    }
}

// out[c][r] = in[r][c] for a rows x cols matrix, through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void k_transpose_rect(int rows, int cols, const float *__restrict__ in,
                                                        float *__restrict__ out) {
    __shared__ float tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[tx][k];
    }
}

}  // namespace
}  // namespace alif

using namespace alif;

extern "C" {

int alif_transpose(int32_t rows, int32_t cols, const float *in, float *out, void *stream) {
    if (rows < 0 || cols < 0) return alif::set_error(ALIF_EINVAL, "transpose: negative size");
    if ((long long)rows * cols == 0) return ALIF_OK;
    if (!in || !out) return alif::set_error(ALIF_EINVAL, "transpose: NULL buffer");
    if (in == out) return alif::set_error(ALIF_EINVAL, "transpose: in and out must not alias");
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)), blk(256);
    if (grid.y > 65535u) return alif::set_error(ALIF_EUNSUPPORTED, "transpose: too many rows");
    hipLaunchKernelGGL(k_transpose_rect, grid, blk, 0, (hipStream_t)stream, rows, cols, in, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

int alif_input_current_events(const alif_desc *desc, const void *input, const float *WT, const float *bias,
                              float *current, void *stream) {
    if (!desc) return alif::set_error(ALIF_EINVAL, "desc is NULL");
    const int kind = desc->input_kind;
    if (kind != ALIF_INPUT_SPIKES_U8 && kind != ALIF_INPUT_SPIKES_BF16 && kind != ALIF_INPUT_SPIKES_F32)
        return alif::set_error(ALIF_EINVAL, "alif_input_current_events needs a spike input_kind");
    if (desc->batch < 0 || desc->T < 0 || desc->n_neurons < 0 || desc->n_in < 0)
        return alif::set_error(ALIF_EINVAL, "negative size");
    if (desc->n_in > EV_MAX_IN) return alif::set_error(ALIF_EUNSUPPORTED, "event current: n_in > 16384");
    const long long M = (long long)desc->batch * desc->T;
    const int n_in = desc->n_in, N = desc->n_neurons;
    if (M == 0 || N == 0) return ALIF_OK;
    if (!current || (n_in > 0 && (!input || !WT))) return alif::set_error(ALIF_EINVAL, "NULL buffer");
    if (M > 0x7fffffffLL) return alif::set_error(ALIF_EUNSUPPORTED, "event current: B * T too large");
    const size_t sm = (size_t)(n_in > 0 ? n_in : 1) * (sizeof(int) + sizeof(float));
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)M), blk(EV_THREADS);
    if (kind == ALIF_INPUT_SPIKES_U8)
        hipLaunchKernelGGL(k_events_current<ALIF_INPUT_SPIKES_U8>, grid, blk, sm, st, M, n_in, N, input, WT, bias,
                           current);
    else if (kind == ALIF_INPUT_SPIKES_BF16)
        hipLaunchKernelGGL(k_events_current<ALIF_INPUT_SPIKES_BF16>, grid, blk, sm, st, M, n_in, N, input, WT,
                           bias, current);
    else
        hipLaunchKernelGGL(k_events_current<ALIF_INPUT_SPIKES_F32>, grid, blk, sm, st, M, n_in, N, input, WT, bias,
                           current);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

}  // extern "C"
