// MFMA GEMMs for gfx950 (paper Eq. 3 projections and their gradients).
//
// One kernel family computes C[M][N] = sum_k A(m, k) B(n, k) (+ bias[n]) where
// each operand is read either k-contiguous or m/n-contiguous and may be float,
// uint8 (0/1 spikes) or bfloat16. A 256-thread workgroup owns a 128 x 128 tile
// of C; its four waves each own 64 x 64 as 4 x 4 MFMA 16 x 16 accumulators.
// K is staged through LDS 16 (FP32) or 32 (BF16) at a time.
//   FP32: v_mfma_f32_16x16x4_f32, operands rounded nowhere.
//   BF16: operands rounded to bfloat16 (0/1 spikes exactly), v_mfma_f32_16x16x32_bf16,
//         FP32 accumulation.
#include <hip/hip_runtime.h>

#include "../../include/blockalif.h"
#include "alif_common.h"
#include "alif_gemm.h"

namespace alif {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int GBM = 128, GBN = 128;

__device__ __forceinline__ float ld_elem(const void *p, int dt, long long i) {
    if (dt == 0) return static_cast<const float *>(p)[i];
    if (dt == 1) return (float)static_cast<const uint8_t *>(p)[i];
    const uint16_t h = static_cast<const uint16_t *>(p)[i];
    return __uint_as_float((uint32_t)h << 16);
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    constexpr int BK = BF16 ? 32 : 16;
    constexpr int APAD = BF16 ? 8 : 16;
    // BF16: [row][k] (k contiguous, 8-element MFMA fragments); FP32: [k][row]
    __shared__ __align__(16) typename std::conditional<BF16, __bf16, float>::type
        As[BF16 ? GBM : BK][BF16 ? BK + APAD : GBM + APAD],
        Bs[BF16 ? GBN : BK][BF16 ? BK + APAD : GBN + APAD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long long m0 = (long long)blockIdx.y * GBM;
    const int n0 = blockIdx.x * GBN;
    const int z = blockIdx.z;
    const int kps = (g.K + g.splits - 1) / g.splits;
    const int kb = z * kps, ke = min(g.K, kb + kps);

    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kb; k0 < ke; k0 += BK) {
        for (int idx = tid; idx < GBM * BK; idx += 256) {
            int rr, kk;
            if (g.a_kc) { kk = idx % BK; rr = idx / BK; } else { rr = idx % GBM; kk = idx / GBM; }
            const long long m = m0 + rr;
            const int k = k0 + kk;
            float v = 0.0f;
            if (m < g.M && k < ke) v = ld_elem(g.A, g.a_dt, g.a_kc ? m * g.lda + k : (long long)k * g.lda + m);
            if constexpr (BF16) As[rr][kk] = (__bf16)v; else As[kk][rr] = v;
        }
        for (int idx = tid; idx < GBN * BK; idx += 256) {
            int rr, kk;
            if (g.b_kc) { kk = idx % BK; rr = idx / BK; } else { rr = idx % GBN; kk = idx / GBN; }
            const int n = n0 + rr;
            const int k = k0 + kk;
            float v = 0.0f;
            if (n < g.N && k < ke) v = ld_elem(g.B, g.b_dt, g.b_kc ? (long long)n * g.ldb + k : (long long)k * g.ldb + n);
            if constexpr (BF16) Bs[rr][kk] = (__bf16)v; else Bs[kk][rr] = v;
        }
        __syncthreads();
        if constexpr (BF16) {
            bf16x8 a[4], b[4];
            const int kq = 8 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; i++) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 64 + i * 16 + (lane & 15)][kq]);
#pragma unroll
            for (int j = 0; j < 4; j++) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 64 + j * 16 + (lane & 15)][kq]);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int ks = 0; ks < BK / 4; ks++) {
                const int k = ks * 4 + (lane >> 4);
                float a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; i++) a[i] = As[k][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; j++) b[j] = Bs[k][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds rows 4 * (lane / 16) + r of column lane % 16 of each 16 x 16 block
    float *out = g.splits > 1 ? g.C_part + (size_t)z * g.M * g.N : g.C;
    const long long ldc = g.splits > 1 ? g.N : g.ldc;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        const float bias = (g.bias && g.splits == 1 && n < g.N) ? g.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long long m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
                if (m < g.M && n < g.N) out[m * ldc + n] = acc[i][j][r] + bias;
            }
    }
}

// fixed-order sum of split partials: C[m][n] = sum_z P[z][m][n] (+ bias)
__global__ void k_split_reduce(long long MN, int N, int splits, const float *P, float *C,
                               const float *bias) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN) return;
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += P[(size_t)z * MN + i];
    if (bias) s += bias[i % N];
    C[i] = s;
}

hipError_t gemm_launch(const GemmArgs &g, bool bf16, hipStream_t st) {
    if (g.M == 0 || g.N == 0) return hipSuccess;
    dim3 grid((g.N + GBN - 1) / GBN, (unsigned)((g.M + GBM - 1) / GBM), g.splits);
    if (grid.y > 65535) return hipErrorInvalidValue;
    if (bf16) hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.splits == 1) return e;
    const long long MN = g.M * (long long)g.N;
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, MN, g.N,
                       g.splits, g.C_part, g.C, g.bias);
    return hipGetLastError();
}

static int dt_of(int kind) {
    return kind == ALIF_INPUT_SPIKES_U8 ? 1 : (kind == ALIF_INPUT_SPIKES_BF16 ? 2 : 0);
}

hipError_t gemm_input_current(size_t M, int N, int K, GemmIn x, const float *W, const float *bias,
                              float *out, bool bf16, hipStream_t st) {
    GemmArgs g{};
    g.M = (long long)M; g.N = N; g.K = K;
    g.A = x.ptr; g.a_dt = dt_of(x.kind); g.lda = K; g.a_kc = 1;
    g.B = W; g.b_dt = 0; g.ldb = K; g.b_kc = 1;
    g.C = out; g.ldc = N; g.bias = bias; g.splits = 1;
    return gemm_launch(g, bf16, st);
}

static int wgrad_splits(size_t M, int N, int K) {
    const long long tiles = (long long)((N + GBN - 1) / GBN) * ((K + GBM - 1) / GBM);
    long long s = 1024 / (tiles > 0 ? tiles : 1);
    s = s < 1 ? 1 : (s > 64 ? 64 : s);
    const long long maxs = (long long)M / 256;
    if (s > maxs) s = maxs < 1 ? 1 : maxs;
    return (int)s;
}

size_t gemm_workspace_bytes(size_t M, int N, int K) {
    const int s = wgrad_splits(M, N, K);
    return s > 1 ? (size_t)s * N * K * sizeof(float) : 0;
}

hipError_t gemm_weight_grad(size_t M, int N, int K, const float *gI, GemmIn x, float *gW, bool bf16,
                            void *ws, hipStream_t st) {
    // C[n][k] = sum_m gI[m][n] x[m][k]: reduction over m (split), both operands m-major
    GemmArgs g{};
    g.M = N; g.N = K; g.K = (int)M;
    g.A = gI; g.a_dt = 0; g.lda = N; g.a_kc = 0;
    g.B = x.ptr; g.b_dt = dt_of(x.kind); g.ldb = K; g.b_kc = 0;
    g.C = gW; g.ldc = K; g.bias = nullptr;
    g.splits = wgrad_splits(M, N, K);
    g.C_part = (float *)ws;
    if (M > 0x7fffffff) return hipErrorInvalidValue;
    return gemm_launch(g, bf16, st);
}

hipError_t gemm_input_grad(size_t M, int N, int K, const float *gI, const float *W, float *gx,
                           bool bf16, hipStream_t st) {
    // C[m][k] = sum_n gI[m][n] W[n][k]
    GemmArgs g{};
    g.M = (long long)M; g.N = K; g.K = N;
    g.A = gI; g.a_dt = 0; g.lda = N; g.a_kc = 1;
    g.B = W; g.b_dt = 0; g.ldb = K; g.b_kc = 0;
    g.C = gx; g.ldc = K; g.bias = nullptr; g.splits = 1;
    return gemm_launch(g, bf16, st);
}

}  // namespace alif
