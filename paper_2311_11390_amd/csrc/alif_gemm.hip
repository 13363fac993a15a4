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

#include <type_traits>

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

// ---------------------------------------------------------------------------
// Fast path for C = A W^T (+ bias) with both operands k-contiguous: the Eq. 3
// current I = b + x W^T of a spike-input layer (A = x [M][K] as float, uint8 or
// bf16; W [N][K] float). A 256-thread workgroup owns a 128 x 128 tile of C (four
// waves of 64 x 64, 4 x 4 MFMA accumulators each). K moves in stages of BK:
// every thread loads half a row of A and of W (raw buffer loads: rows beyond M
// or N read 0; steps beyond K are zeroed), converts them to the MFMA operand
// type in registers and stores them to one of two LDS buffers; while a stage is
// multiplied, the next one is loaded. One barrier per stage. Workgroups are
// numbered so that the N tiles of one M tile run on one XCD and share its rows
// of A in that XCD's L2.
// ---------------------------------------------------------------------------
// BF16: 256 x 128 tiles with eight waves (W, read as float, is reused over more
// rows of A); FP32: 128 x 128 with four waves.
template <bool BF16>
struct NT {
    static constexpr int BM = BF16 ? 256 : 128, BN = 128;
    static constexpr int THREADS = BF16 ? 512 : 256;
    static constexpr int BK = BF16 ? 64 : 32;           // k per stage
    static constexpr int AH = BK * BM / THREADS;          // A elements per thread per stage
    static constexpr int BH = BK * BN / THREADS;          // W elements per thread per stage
    static constexpr int LDK = BF16 ? BK + 8 : BK + 4;   // LDS row (elements), 16-byte multiple
    using T = typename std::conditional<BF16, __bf16, float>::type;
    static constexpr size_t lds_bytes() { return (size_t)2 * (BM + BN) * LDK * sizeof(T); }
};

// HALF consecutive elements of one row, as float; k >= kmax read as 0
template <int DT, int HALF>
__device__ __forceinline__ void load_half_row(rsrc_t r, uint32_t off, int kmax, float (&v)[HALF]) {
    if constexpr (DT == 0) {            // float, rows 16-byte aligned
#pragma unroll
        for (int q = 0; q < HALF / 4; q++) {
            const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u * q, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; e++) v[4 * q + e] = __uint_as_float(w[e]);
        }
    } else if constexpr (DT == 1) {     // uint8, rows 4-byte aligned
#pragma unroll
        for (int q = 0; q < HALF / 4; q++) {
            const uint32_t w = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * q, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; e++) v[4 * q + e] = (float)((w >> (8 * e)) & 0xffu);
        }
    } else {                            // bf16, rows 4-byte aligned
#pragma unroll
        for (int q = 0; q < HALF / 2; q++) {
            const uint32_t w = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * q, 0, 0);
            v[2 * q] = __uint_as_float(w << 16);
            v[2 * q + 1] = __uint_as_float(w & 0xffff0000u);
        }
    }
#pragma unroll
    for (int e = 0; e < HALF; e++) v[e] = e < kmax ? v[e] : 0.0f;
}

template <int ADT, bool BF16>
__global__ __launch_bounds__(NT<BF16>::THREADS) void k_gemm_nt(GemmArgs g, int n_tiles, int tiles) {
    using P = NT<BF16>;
    using T = typename P::T;
    constexpr int BM = P::BM, BN = P::BN, BK = P::BK, AH = P::AH, BH = P::BH, LDK = P::LDK;
    constexpr int APR = BK / AH, BPR = BK / BH;           // threads per staged row of A, of W
    constexpr uint32_t AES = ADT == 0 ? 4 : (ADT == 1 ? 1 : 2);
    extern __shared__ __align__(16) unsigned char lds[];
    T *As = reinterpret_cast<T *>(lds);                   // [2][BM][LDK]
    T *Bs = As + 2 * BM * LDK;                            // [2][BN][LDK]

    const int work = xcd_remap(blockIdx.x, tiles);
    const long long m0 = (long long)(work / n_tiles) * BM;
    const int n0 = (work % n_tiles) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;              // wave tile (wm, wn) of 64 x 64
    const int K = g.K;

    const rsrc_t rA = make_rsrc(g.A, (uint32_t)((size_t)g.M * K * AES));
    const rsrc_t rB = make_rsrc(g.B, (uint32_t)((size_t)g.N * K * 4));
    // staged row and k part of this thread, for A and for W
    const int ra = tid / APR, ha = tid % APR, rb = tid / BPR, hb = tid % BPR;
    // byte offsets of the staged rows; a row beyond M or N uses an offset past
    // the buffer, so its loads read 0
    const bool a_in = (m0 + ra) < g.M, b_in = (n0 + rb) < g.N;
    const uint32_t arow = a_in ? (uint32_t)((m0 + ra) * K * AES) : 0u;
    const uint32_t brow = b_in ? (uint32_t)((size_t)(n0 + rb) * K * 4) : 0u;

    float va[AH], vb[BH];
    auto load_stage = [&](int k0) {
        const int ka = k0 + ha * AH, kb = k0 + hb * BH;
        load_half_row<ADT, AH>(rA, a_in ? arow + (uint32_t)ka * AES : ALIF_OOB, K - ka, va);
        load_half_row<0, BH>(rB, b_in ? brow + (uint32_t)kb * 4u : ALIF_OOB, K - kb, vb);
    };
    auto store_stage = [&](int buf) {
        T *a = As + (size_t)(buf * BM + ra) * LDK + ha * AH;
        T *b = Bs + (size_t)(buf * BN + rb) * LDK + hb * BH;
        if constexpr (BF16) {
            typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
#pragma unroll
            for (int q = 0; q < AH / 8; q++) {
                bf16x8_t pa;
#pragma unroll
                for (int e = 0; e < 8; e++) pa[e] = (__bf16)va[8 * q + e];
                *reinterpret_cast<bf16x8_t *>(a + 8 * q) = pa;
            }
#pragma unroll
            for (int q = 0; q < BH / 8; q++) {
                bf16x8_t pb;
#pragma unroll
                for (int e = 0; e < 8; e++) pb[e] = (__bf16)vb[8 * q + e];
                *reinterpret_cast<bf16x8_t *>(b + 8 * q) = pb;
            }
        } else {
#pragma unroll
            for (int q = 0; q < AH / 4; q++)
                *reinterpret_cast<floatx4 *>(a + 4 * q) = floatx4{va[4 * q], va[4 * q + 1], va[4 * q + 2], va[4 * q + 3]};
#pragma unroll
            for (int q = 0; q < BH / 4; q++)
                *reinterpret_cast<floatx4 *>(b + 4 * q) = floatx4{vb[4 * q], vb[4 * q + 1], vb[4 * q + 2], vb[4 * q + 3]};
        }
    };

    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int nk = (K + BK - 1) / BK;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) load_stage((kt + 1) * BK);
        const T *a = As + (size_t)buf * BM * LDK;
        const T *b = Bs + (size_t)buf * BN * LDK;
        if constexpr (BF16) {
#pragma unroll
            for (int kq = 0; kq < BK; kq += 32) {
                bf16x8 fa[4], fb[4];
                const int kc = kq + 8 * (lane >> 4);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    fa[i] = *reinterpret_cast<const bf16x8 *>(a + (wm * 64 + i * 16 + (lane & 15)) * LDK + kc);
#pragma unroll
                for (int j = 0; j < 4; j++)
                    fb[j] = *reinterpret_cast<const bf16x8 *>(b + (wn * 64 + j * 16 + (lane & 15)) * LDK + kc);
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                const int kc = ks + (lane >> 4);
                float fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; i++) fa[i] = a[(wm * 64 + i * 16 + (lane & 15)) * LDK + kc];
#pragma unroll
                for (int j = 0; j < 4; j++) fb[j] = b[(wn * 64 + j * 16 + (lane & 15)) * LDK + kc];
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        }
        if (more) store_stage(buf ^ 1);
        __syncthreads();
    }
    // epilogue: lane holds rows 4 * (lane / 16) + r of column lane % 16 of each 16 x 16 block
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        const float bias = (g.bias && n < g.N) ? g.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const long long m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + rr;
                if (m < g.M && n < g.N) g.C[m * g.ldc + n] = acc[i][j][rr] + bias;
            }
    }
}

// whether k_gemm_nt covers this call: both operands k-contiguous and packed,
// W float, rows aligned for its loads, byte offsets within 31 bits
static bool nt_ok(const GemmArgs &g) {
    if (!(g.a_kc && g.b_kc && g.b_dt == 0 && g.splits == 1 && g.lda == g.K && g.ldb == g.K)) return false;
    if (g.K % 4 != 0 || g.K == 0) return false;
    if ((reinterpret_cast<uintptr_t>(g.A) & 15) || (reinterpret_cast<uintptr_t>(g.B) & 15)) return false;
    const size_t aes = g.a_dt == 0 ? 4 : (g.a_dt == 1 ? 1 : 2);
    if ((size_t)g.M * g.K * aes >= ((size_t)1 << 31) || (size_t)g.N * g.K * 4 >= ((size_t)1 << 31)) return false;
    return true;
}

template <bool BF16>
static hipError_t nt_launch(const GemmArgs &g, hipStream_t st) {
    const int n_tiles = (g.N + NT<BF16>::BN - 1) / NT<BF16>::BN;
    const long long m_tiles = (g.M + NT<BF16>::BM - 1) / NT<BF16>::BM;
    const long long tiles = m_tiles * n_tiles;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t sm = NT<BF16>::lds_bytes();
    const dim3 grid((unsigned)tiles), block(NT<BF16>::THREADS);
    if (g.a_dt == 0) hipLaunchKernelGGL((k_gemm_nt<0, BF16>), grid, block, sm, st, g, n_tiles, (int)tiles);
    else if (g.a_dt == 1) hipLaunchKernelGGL((k_gemm_nt<1, BF16>), grid, block, sm, st, g, n_tiles, (int)tiles);
    else hipLaunchKernelGGL((k_gemm_nt<2, BF16>), grid, block, sm, st, g, n_tiles, (int)tiles);
    return hipGetLastError();
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
    if (nt_ok(g)) return bf16 ? nt_launch<true>(g, st) : nt_launch<false>(g, st);
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
