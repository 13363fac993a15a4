// Event-driven input current of Eq. 3 for sparse spike input.
//
// I~[b][t][i] = bias[i] + sum_j W[i][j] x[b][t][j]. Spike trains are mostly zeros
// (at 10 Hz and DT 0.5 ms, 0.5% of the entries are 1), so instead of a dense GEMM
// each (b, t) row adds only the weight rows of its active inputs. One wave owns one
// row (grid-stride over rows), with no LDS and no barrier:
//   * the wave reads the row's inputs as 32-bit words (four u8, two bf16 or one f32
//     inputs; single elements when the row is not word-aligned), EV_KW words per
//     lane per chunk, one coalesced load per k;
//   * a ballot per (word k, element b) gives the chunk's active inputs; the wave
//     walks each mask as scalar code and reads the value with readlane;
//   * lane l accumulates columns c0 + l + 64 q (q < CT) in FP32 and fetches the
//     weight rows WT[j][c0 ...] of two active inputs at a time;
//   * N beyond 64 CT is covered by further column tiles of the same row.
// WT is W transposed ([n_in][N], built once by alif_transpose), so that the weight
// row of one input is contiguous. Word loads matter: with one byte per lane the
// input read is bound by requests in flight, not by bytes. The HBM bytes per row
// are the row's inputs and the N floats written; the active rows of WT come from
// L2 (a layer-sized W fits), and the current is written with non-temporal stores
// so that streaming it out does not evict WT.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/blockalif.h"
#include "alif_gemm.h"
#include "alif_kernels.h"

namespace alif {
namespace {

constexpr int EV_WAVES = 4;        // waves (rows in flight) per workgroup
constexpr int EV_KW = 4;           // words per lane per chunk
constexpr long long EV_MAX_GROUPS = 1 << 18;

template <int KIND>
constexpr int ev_elem_bytes() {
    return KIND == ALIF_INPUT_SPIKES_U8 ? 1 : KIND == ALIF_INPUT_SPIKES_BF16 ? 2 : 4;
}

// the raw bits of element b of a unit, its activity (magnitude bits nonzero) and value
template <int KIND>
__device__ __forceinline__ uint32_t ev_bits(uint32_t u, int b) {
    if constexpr (KIND == ALIF_INPUT_SPIKES_U8) return (u >> (8 * b)) & 0xffu;
    else if constexpr (KIND == ALIF_INPUT_SPIKES_BF16) return (u >> (16 * b)) & 0xffffu;
    else return u;
}
template <int KIND>
__device__ __forceinline__ bool ev_active(uint32_t bits) {
    if constexpr (KIND == ALIF_INPUT_SPIKES_U8) return bits != 0u;
    else if constexpr (KIND == ALIF_INPUT_SPIKES_BF16) return (bits & 0x7fffu) != 0u;
    else return (bits & 0x7fffffffu) != 0u;
}
template <int KIND>
__device__ __forceinline__ float ev_float(uint32_t bits) {
    if constexpr (KIND == ALIF_INPUT_SPIKES_U8) return (float)bits;
    else if constexpr (KIND == ALIF_INPUT_SPIKES_BF16) return __uint_as_float(bits << 16);
    else return __uint_as_float(bits);
}

// WORDS: a unit is a 32-bit word of EPW elements (the row is word-aligned); else one element
template <int KIND, int CT, bool WORDS>
__global__ __launch_bounds__(64 * EV_WAVES) void k_events_current(long long M, int n_in, int N, const void *x,
                                                                   const float *__restrict__ WT,
                                                                   const float *__restrict__ bias,
                                                                   float *__restrict__ C,
                                                                   const unsigned long long *gate) {
    if (gate && *gate != 0ull) return;   // the caller's dense product runs instead
    constexpr int ES = ev_elem_bytes<KIND>();
    constexpr int EPW = WORDS ? 4 / ES : 1;          // elements per unit
    const int lane = threadIdx.x & 63;
    const int nu = n_in / EPW;                       // units per row (exact for WORDS)
    const long long stride = (long long)gridDim.x * EV_WAVES;
    for (long long row = (long long)blockIdx.x * EV_WAVES + (threadIdx.x >> 6); row < M; row += stride) {
        const char *xr = static_cast<const char *>(x) + (size_t)row * n_in * ES;
        float *crow = C + (size_t)row * N;
        for (int c0 = 0; c0 < N; c0 += 64 * CT) {
            bool ok[CT];
            float acc[CT];
#pragma unroll
            for (int q = 0; q < CT; q++) {
                const int c = c0 + lane + 64 * q;
                ok[q] = c < N;
                acc[q] = (bias && ok[q]) ? bias[c] : 0.0f;
            }
            const float *wcol = WT + c0 + lane;
            int held = -1;                           // an active input held back to fetch weight rows in pairs
            float held_v = 0.0f;
            for (int u0 = 0; u0 < nu; u0 += 64 * EV_KW) {
                uint32_t v[EV_KW];
#pragma unroll
                for (int k = 0; k < EV_KW; k++) {
                    const int u = u0 + 64 * k + lane;
                    if (u >= nu) v[k] = 0u;
                    else if constexpr (WORDS) v[k] = reinterpret_cast<const uint32_t *>(xr)[u];
                    else if constexpr (ES == 1) v[k] = reinterpret_cast<const uint8_t *>(xr)[u];
                    else if constexpr (ES == 2) v[k] = reinterpret_cast<const uint16_t *>(xr)[u];
                    else v[k] = reinterpret_cast<const uint32_t *>(xr)[u];
                }
#pragma unroll
                for (int k = 0; k < EV_KW; k++) {
                    if (!__ballot(v[k] != 0u)) continue;
#pragma unroll
                    for (int b = 0; b < EPW; b++) {
                        unsigned long long m = __ballot(ev_active<KIND>(ev_bits<KIND>(v[k], b)));
                        while (m) {
                            const int l = __builtin_ctzll(m);
                            m &= m - 1;
                            const int j = EPW * (u0 + 64 * k + l) + b;
                            const float a = ev_float<KIND>(
                                ev_bits<KIND>((uint32_t)__builtin_amdgcn_readlane((int)v[k], l), b));
                            if (held < 0) {
                                held = j;
                                held_v = a;
                                continue;
                            }
                            const float *wa = wcol + (size_t)held * N, *wb = wcol + (size_t)j * N;
                            float ra[CT], rb[CT];
#pragma unroll
                            for (int q = 0; q < CT; q++) {
                                ra[q] = ok[q] ? wa[64 * q] : 0.0f;
                                rb[q] = ok[q] ? wb[64 * q] : 0.0f;
                            }
#pragma unroll
                            for (int q = 0; q < CT; q++) acc[q] = fmaf(a, rb[q], fmaf(held_v, ra[q], acc[q]));
                            held = -1;
                        }
                    }
                }
            }
            if (held >= 0) {
                const float *wa = wcol + (size_t)held * N;
#pragma unroll
                for (int q = 0; q < CT; q++) acc[q] = fmaf(held_v, ok[q] ? wa[64 * q] : 0.0f, acc[q]);
            }
            // the current streams out once: non-temporal stores keep WT's rows in L2
#pragma unroll
            for (int q = 0; q < CT; q++)
                if (ok[q]) __builtin_nontemporal_store(acc[q], crow + c0 + lane + 64 * q);
        }
    }
}

template <int KIND, int CT>
void launch_events_ct(bool words, long long M, hipStream_t st, int n_in, int N, const void *x, const float *WT,
                      const float *bias, float *C, const unsigned long long *gate) {
    const long long groups = (M + EV_WAVES - 1) / EV_WAVES;
    const dim3 grid((unsigned)(groups < EV_MAX_GROUPS ? groups : EV_MAX_GROUPS)), blk(64 * EV_WAVES);
    if (words)
        hipLaunchKernelGGL((k_events_current<KIND, CT, true>), grid, blk, 0, st, M, n_in, N, x, WT, bias, C, gate);
    else
        hipLaunchKernelGGL((k_events_current<KIND, CT, false>), grid, blk, 0, st, M, n_in, N, x, WT, bias, C, gate);
}

template <int KIND>
void launch_events(int ct, long long M, hipStream_t st, int n_in, int N, const void *x, const float *WT,
                   const float *bias, float *C, const unsigned long long *gate = nullptr) {
    // word loads need every row to start on a 4-byte boundary
    const bool words = ((size_t)n_in * ev_elem_bytes<KIND>()) % 4 == 0 && ((uintptr_t)x & 3u) == 0;
    switch (ct) {
        case 1: launch_events_ct<KIND, 1>(words, M, st, n_in, N, x, WT, bias, C, gate); break;
        case 2: launch_events_ct<KIND, 2>(words, M, st, n_in, N, x, WT, bias, C, gate); break;
        case 4: launch_events_ct<KIND, 4>(words, M, st, n_in, N, x, WT, bias, C, gate); break;
        case 8: launch_events_ct<KIND, 8>(words, M, st, n_in, N, x, WT, bias, C, gate); break;
        default: launch_events_ct<KIND, 16>(words, M, st, n_in, N, x, WT, bias, C, gate);
    }
}

// column tile: the smallest 64 CT (CT = 1, 2, 4, 8, 16) that covers N, else 1024 columns per pass
int column_tile(int N) {
    for (int c = 1; c < 16; c *= 2)
        if (64 * c >= N) return c;
    return 16;
}

// out[c][r] = in[r][c] for a rows x cols matrix, through 32 x 32 LDS tiles (with
// round_bf16, each value rounded to the nearest bfloat16, kept as float)
__global__ __launch_bounds__(256) void k_transpose_rect(int rows, int cols, const float *__restrict__ in,
                                                        float *__restrict__ out, int round_bf16) {
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
        if (r < rows && c < cols) {
            const float v = tile[tx][k];
            out[(size_t)c * rows + r] = round_bf16 ? (float)(__bf16)v : v;
        }
    }
}

}  // namespace

bool events_current_launch(int kind, long long M, int n_in, int N, const void *x, const float *W, float *WT,
                           bool round_bf16, const float *bias, float *C, const unsigned long long *gate,
                           hipStream_t st) {
    const unsigned esz = kind == ALIF_INPUT_SPIKES_U8 ? 1u : 2u;
    if ((kind != ALIF_INPUT_SPIKES_U8 && kind != ALIF_INPUT_SPIKES_BF16) || M <= 0 || n_in <= 0 || N <= 0 ||
        ((uintptr_t)x % esz) != 0 || ((uintptr_t)WT % 4u) != 0 || ((uintptr_t)C % 4u) != 0 ||
        (bias && ((uintptr_t)bias % 4u) != 0) || (N + 31) / 32 > 65535)
        return false;
    const dim3 tg((unsigned)((n_in + 31) / 32), (unsigned)((N + 31) / 32));
    hipLaunchKernelGGL(k_transpose_rect, tg, dim3(256), 0, st, N, n_in, W, WT, round_bf16 ? 1 : 0);
    if (kind == ALIF_INPUT_SPIKES_U8)
        launch_events<ALIF_INPUT_SPIKES_U8>(column_tile(N), M, st, n_in, N, x, WT, bias, C, gate);
    else
        launch_events<ALIF_INPUT_SPIKES_BF16>(column_tile(N), M, st, n_in, N, x, WT, bias, C, gate);
    return true;
}

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
    hipLaunchKernelGGL(k_transpose_rect, grid, blk, 0, (hipStream_t)stream, rows, cols, in, out, 0);
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
    const long long M = (long long)desc->batch * desc->T;
    const int n_in = desc->n_in, N = desc->n_neurons;
    if (M == 0 || N == 0) return ALIF_OK;
    if (!current || (n_in > 0 && (!input || !WT))) return alif::set_error(ALIF_EINVAL, "NULL buffer");
    const unsigned esz = kind == ALIF_INPUT_SPIKES_U8 ? 1u : kind == ALIF_INPUT_SPIKES_BF16 ? 2u : 4u;
    if (((uintptr_t)input % esz) != 0 || ((uintptr_t)WT % 4u) != 0 || ((uintptr_t)current % 4u) != 0 ||
        (bias && ((uintptr_t)bias % 4u) != 0))
        return alif::set_error(ALIF_EINVAL, "event current: buffer not aligned to its element type");
    const int ct = column_tile(N);
    hipStream_t st = (hipStream_t)stream;
    if (kind == ALIF_INPUT_SPIKES_U8)
        launch_events<ALIF_INPUT_SPIKES_U8>(ct, M, st, n_in, N, input, WT, bias, current);
    else if (kind == ALIF_INPUT_SPIKES_BF16)
        launch_events<ALIF_INPUT_SPIKES_BF16>(ct, M, st, n_in, N, input, WT, bias, current);
    else
        launch_events<ALIF_INPUT_SPIKES_F32>(ct, M, st, n_in, N, input, WT, bias, current);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

}  // extern "C"
