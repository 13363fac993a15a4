// Host-side dispatch of the block-wise kernels (alif_blocks_impl.h) plus the
// small gradient-finalize and decay-table kernels. The (segments, steps per
// segment) split of a T_R-step block is a function of T_R only, so the forward
// and the backward always run the same per-step arithmetic.
#include "alif_blocks_impl.h"

namespace alif {

// Sum the per-(b, n) FP64 partials over the batch in a fixed order and convert
// d/dbeta, d/dp to d/dtau (dbeta/dtau = beta DT / tau^2). A workgroup owns 64
// neurons; its FIN_PH phases each sum the batch rows b = ph, ph + FIN_PH, ... in
// increasing order (loads of consecutive neurons coalesce, and the phases keep
// many loads in flight), then phase 0 adds the phase sums in order 0..FIN_PH-1.
constexpr int FIN_PH = 16;

__global__ __launch_bounds__(64 * FIN_PH) void k_finalize(FinalizeArgs a) {
    __shared__ double red[FIN_PH][5][64];
    const int nl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + nl;
    const size_t BN = (size_t)a.B * a.N;
    double s[5] = {0, 0, 0, 0, 0};
    if (n < a.N) {
#pragma unroll 4
        for (int b = ph; b < a.B; b += FIN_PH)
#pragma unroll
            for (int q = 0; q < 5; q++) s[q] += a.part[q * BN + (size_t)b * a.N + n];
    }
#pragma unroll
    for (int q = 0; q < 5; q++) red[ph][q][nl] = s[q];
    __syncthreads();
    if (ph != 0 || n >= a.N) return;
#pragma unroll
    for (int q = 0; q < 5; q++) {
        double t = 0.0;
        for (int k = 0; k < FIN_PH; k++) t += red[k][q][nl];
        s[q] = t;
    }
    const double tm = a.tau_m[n], ta = a.tau_a[n];
    const double beta = exp(-a.dt / tm), p = exp(-a.dt / ta);
    if (a.g_tau_m) a.g_tau_m[n] = (float)(s[0] * beta * a.dt / (tm * tm));
    if (a.g_tau_a) a.g_tau_a[n] = (float)(s[1] * p * a.dt / (ta * ta));
    if (a.g_d) a.g_d[n] = (float)s[2];
    if (a.g_theta0) a.g_theta0[n] = (float)s[3];
    if (a.g_bias) a.g_bias[n] = (float)s[4];
}

__global__ void k_decay_tables(int N, int TR, double dt, const float *tau_m, const float *tau_a,
                               float *bp, float *pp) {
    const int TRP = TR + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * TRP) return;
    const int n = idx / TRP, k = idx - n * TRP;
    if (bp) bp[idx] = (float)exp(-dt / (double)tau_m[n] * (double)k);
    if (pp) pp[idx] = (float)exp(-dt / (double)tau_a[n] * (double)k);
}

// ---------------------------------------------------------------------------
// host-side dispatch
// ---------------------------------------------------------------------------
BlockConfig block_config(int TR) {
    if (TR <= 2) return {1, 2};
    if (TR == 3) return {1, 3};
    if (TR == 4) return {1, 4};
    if (TR <= 6) return {2, 3};
    if (TR <= 8) return {2, 4};
    if (TR <= 12) return {4, 3};
    if (TR <= 16) return {4, 4};
    if (TR <= 20) return {4, 5};
    if (TR <= 24) return {4, 6};
    if (TR <= 32) return {4, 8};
    if (TR <= 40) return {8, 5};
    if (TR <= 48) return {8, 6};
    if (TR <= 64) return {8, 8};
    if (TR <= 80) return {8, 10};
    if (TR <= 96) return {8, 12};
    if (TR <= 104) return {8, 13};
    if (TR <= 112) return {8, 14};
    if (TR <= 120) return {8, 15};
    return {8, 16};
}
int block_neurons_per_wg(int seg) { return 64 * (seg >= 4 ? 1 : 4 / seg); }

#define ALIF_CONFIGS(X) X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(4, 3) X(4, 4) X(4, 5) X(4, 6) \
    X(4, 8) X(8, 5) X(8, 6) X(8, 8) X(8, 10) X(8, 12) X(8, 13) X(8, 14) X(8, 15) X(8, 16)

#define ALIF_EXTERN(S, L)                                                                  \
    extern template hipError_t blocks_fwd_launch<S, L>(const FwdArgs &, hipStream_t);     \
    extern template hipError_t blocks_bwd_launch<S, L>(const BwdArgs &, hipStream_t);
ALIF_CONFIGS(ALIF_EXTERN)

hipError_t launch_blocks_fwd(const FwdArgs &a, hipStream_t st) {
    BlockConfig c = block_config(a.TR);
#define ALIF_F(S, L) if (c.seg == S && c.len == L) return blocks_fwd_launch<S, L>(a, st);
    ALIF_CONFIGS(ALIF_F)
#undef ALIF_F
    return hipErrorInvalidValue;
}

hipError_t launch_blocks_bwd(const BwdArgs &a, hipStream_t st) {
    BlockConfig c = block_config(a.TR);
#define ALIF_B(S, L) if (c.seg == S && c.len == L) return blocks_bwd_launch<S, L>(a, st);
    ALIF_CONFIGS(ALIF_B)
#undef ALIF_B
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// one-launch recurrent layer (alif_recurrent_impl.h)
// ---------------------------------------------------------------------------
template <int S, int L, int NG>
hipError_t recurrent_fused_launch(const RecArgs &, hipStream_t);
#define ALIF_REC_G2(X) X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(4, 8) X(8, 5) \
    X(8, 6) X(8, 8) X(8, 10) X(8, 12) X(8, 13) X(8, 14) X(8, 15) X(8, 16)
#define ALIF_REC_G4(X) X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(4, 8) X(4, 9) \
    X(4, 10) X(4, 11) X(4, 12) X(4, 13) X(4, 14) X(4, 15) X(4, 16)
#define ALIF_REC_EXT2(S, L) extern template hipError_t recurrent_fused_launch<S, L, 2>(const RecArgs &, hipStream_t);
#define ALIF_REC_EXT4(S, L) extern template hipError_t recurrent_fused_launch<S, L, 4>(const RecArgs &, hipStream_t);
ALIF_REC_G2(ALIF_REC_EXT2)
ALIF_REC_G4(ALIF_REC_EXT4)

// (neuron groups, segments, steps per segment) of the one-launch recurrent layer:
// the block forward's segmentation, capped at four segments for four groups
// (1024 threads); {0, 0, 0} if not covered.
struct RecConfig {
    int ng, seg, len;
};
static RecConfig rec_config(int N, int TR) {
    if (N < 1 || N > 256) return {0, 0, 0};
    const BlockConfig bc = block_config(TR);
    if (N <= 128) return {2, bc.seg, bc.len};
    if (bc.seg <= 4) return {4, bc.seg, bc.len};
    if (TR > 64) return {0, 0, 0};
    return {4, 4, (TR + 3) / 4};
}

int recurrent_ring_slots(int TR, int D) { return D > TR ? (D + TR - 1) / TR : 0; }

static size_t rec_smem_bytes(const RecConfig &c, int TR, int D) {
    const size_t nwg = (size_t)64 * c.ng;
    return nwg * TR * sizeof(double) + (size_t)3 * c.seg * nwg * 4 + (size_t)recurrent_ring_slots(TR, D) * nwg;
}

bool recurrent_fused_ok(int N, int TR, int D) {
    const RecConfig c = rec_config(N, TR);
    return c.ng != 0 && D >= TR && rec_smem_bytes(c, TR, D) <= (size_t)160 * 1024;
}

hipError_t launch_recurrent_fused(const RecArgs &a, hipStream_t st) {
    if (!recurrent_fused_ok(a.N, a.TR, a.D) || a.ring != recurrent_ring_slots(a.TR, a.D)) return hipErrorInvalidValue;
    const RecConfig c = rec_config(a.N, a.TR);
#define ALIF_RL2(S, L) if (c.ng == 2 && c.seg == S && c.len == L) return recurrent_fused_launch<S, L, 2>(a, st);
#define ALIF_RL4(S, L) if (c.ng == 4 && c.seg == S && c.len == L) return recurrent_fused_launch<S, L, 4>(a, st);
    ALIF_REC_G2(ALIF_RL2)
    ALIF_REC_G4(ALIF_RL4)
#undef ALIF_RL2
#undef ALIF_RL4
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// layout moves of the recurrent layer (grid-stride loops over the output)
// ---------------------------------------------------------------------------
// Recurrent current of one block from earlier spikes, event-driven (a neuron
// spikes at most once per block, so the spike rows are sparse):
//   C[b][k][i] += sum over j with S[b][t - D][j] != 0 of W_recT[j][i],  t = t0 + k,
// for b < B, k < rows; nothing where t - D < 0. The spikes come from the
// block-major staging copy (block m at byte offset m * blk_bytes, [B][TR][N] of
// element type E); D >= T_R keeps the source in a finished block. One workgroup
// per (b, k) row: the active j are compacted in increasing order (wave ballots
// and their prefix counts), then every thread sums its outputs i over them in
// that order, in FP32, reading W_recT rows (coalesced over i). C: rows of a
// [B][T][N] tensor starting at the block (batch stride bstride).
template <typename E>
__global__ __launch_bounds__(256) void k_recurrent_events(int TR, int rows, int N, long long bstride, int t0, int D,
                                                          const char *blocks, size_t blk_bytes, const float *WrecT,
                                                          float *C) {
    extern __shared__ int act[];              // [N] active presynaptic indices
    __shared__ int wave_cnt[4];
    const int row = blockIdx.x, b = row / rows, k = row - b * rows;
    const int u = t0 + k - D;                 // source step
    if (u < 0) return;                        // uniform over the workgroup
    const E *srow = reinterpret_cast<const E *>(blocks + (size_t)(u / TR) * blk_bytes) +
                    ((size_t)b * TR + (u % TR)) * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int base = 0;
    for (int j0 = 0; j0 < N; j0 += 256) {
        const int j = j0 + tid;
        const bool on = j < N && srow[j] != E(0);
        const unsigned long long m = __ballot(on);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; w++) off += wave_cnt[w];
        if (on) act[off + __popcll(m & ((1ull << lane) - 1ull))] = j;
        base += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        __syncthreads();
    }
    if (base == 0) return;
    float *crow = C + (size_t)b * bstride + (size_t)k * N;
    for (int i = tid; i < N; i += 256) {
        float s = 0.0f;
        for (int e = 0; e < base; e++) s += WrecT[(size_t)act[e] * N + i];
        crow[i] += s;
    }
}

// out[j][i] = in[i][j] for an N x N matrix
__global__ void k_transpose(int N, const float *in, float *out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)N * N) return;
    const int j = (int)(e / N), i = (int)(e - (size_t)j * N);
    out[e] = in[(size_t)i * N + j];
}

hipError_t launch_recurrent_events(int B, int TR, int rows, int N, long long bstride, int t0, int D, int elem,
                                   const void *blocks, size_t blk_bytes, const float *WrecT, float *C,
                                   hipStream_t st) {
    if (B == 0 || rows == 0 || N == 0) return hipSuccess;
    const dim3 grid((unsigned)(B * rows)), blk(256);
    const size_t sm = (size_t)N * sizeof(int);
    const char *bl = static_cast<const char *>(blocks);
    if (elem == 1)
        hipLaunchKernelGGL(k_recurrent_events<uint8_t>, grid, blk, sm, st, TR, rows, N, bstride, t0, D, bl,
                           blk_bytes, WrecT, C);
    else if (elem == 2)
        hipLaunchKernelGGL(k_recurrent_events<uint16_t>, grid, blk, sm, st, TR, rows, N, bstride, t0, D, bl,
                           blk_bytes, WrecT, C);
    else
        hipLaunchKernelGGL(k_recurrent_events<uint32_t>, grid, blk, sm, st, TR, rows, N, bstride, t0, D, bl,
                           blk_bytes, WrecT, C);
    return hipGetLastError();
}

hipError_t launch_transpose(int N, const float *in, float *out, hipStream_t st) {
    const size_t total = (size_t)N * N;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, N, in, out);
    return hipGetLastError();
}

// Both move whole neuron rows (N elements, `rb` bytes) in chunks of type C (16,
// 4 or 1 bytes, the widest that divides the row and keeps every row aligned):
// one index computation per chunk.
template <typename C>
__global__ void k_blocks_to_bt(size_t chunks, int cpr, int T, int TR, const char *blocks, size_t blk_bytes,
                               size_t rb, C *out) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < chunks; c += (size_t)gridDim.x * blockDim.x) {
        const size_t row = c / cpr;                     // output row (b, t)
        const int w = (int)(c - row * cpr);
        const size_t b = row / T;
        const int t = (int)(row - b * T);
        const int n = t / TR, k = t - n * TR;
        const C *src = reinterpret_cast<const C *>(blocks + (size_t)n * blk_bytes + (b * TR + k) * rb);
        out[c] = src[w];
    }
}

template <typename C>
__global__ void k_shift_time(size_t chunks, int cpr, int T, int D, const C *in, C *out,
                             const unsigned long long *skip_cnt, unsigned long long skip_le) {
    if (skip_cnt && *skip_cnt <= skip_le) return;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < chunks; c += (size_t)gridDim.x * blockDim.x) {
        const size_t row = c / cpr;
        const int t = (int)(row % T);
        out[c] = t >= D ? in[c - (size_t)D * cpr] : C{};
    }
}

static unsigned grid_for(size_t total) {
    const size_t g = (total + 255) / 256;
    return (unsigned)(g < ((size_t)1 << 20) ? (g ? g : 1) : ((size_t)1 << 20));
}

// widest chunk (16, 4 or 1 bytes) dividing the row bytes and every given address
static int chunk_bytes(size_t rb, const void *a, const void *b, size_t extra_align) {
    const uintptr_t m = reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | extra_align | rb;
    return (m & 15) == 0 ? 16 : ((m & 3) == 0 ? 4 : 1);
}

hipError_t launch_blocks_to_bt(int B, int T, int N, int TR, int elem, const void *blocks, size_t blk_bytes,
                               void *spikes, hipStream_t st) {
    const size_t rb = (size_t)N * elem, rows = (size_t)B * T;
    if (rows == 0 || rb == 0) return hipSuccess;
    const char *bl = static_cast<const char *>(blocks);
    const int cb = chunk_bytes(rb, blocks, spikes, blk_bytes);
    const int cpr = (int)(rb / cb);
    const size_t chunks = rows * cpr;
    if (cb == 16)
        hipLaunchKernelGGL(k_blocks_to_bt<uint4>, dim3(grid_for(chunks)), dim3(256), 0, st, chunks, cpr, T, TR, bl,
                           blk_bytes, rb, static_cast<uint4 *>(spikes));
    else if (cb == 4)
        hipLaunchKernelGGL(k_blocks_to_bt<uint32_t>, dim3(grid_for(chunks)), dim3(256), 0, st, chunks, cpr, T, TR,
                           bl, blk_bytes, rb, static_cast<uint32_t *>(spikes));
    else
        hipLaunchKernelGGL(k_blocks_to_bt<uint8_t>, dim3(grid_for(chunks)), dim3(256), 0, st, chunks, cpr, T, TR,
                           bl, blk_bytes, rb, static_cast<uint8_t *>(spikes));
    return hipGetLastError();
}

hipError_t launch_shift_time(int B, int T, int N, int D, int elem, const void *in, void *out, hipStream_t st,
                             const unsigned long long *skip_cnt, unsigned long long skip_le) {
    const size_t rb = (size_t)N * elem, rows = (size_t)B * T;
    if (rows == 0 || rb == 0) return hipSuccess;
    const int cb = chunk_bytes(rb, in, out, 0);
    const int cpr = (int)(rb / cb);
    const size_t chunks = rows * cpr;
    // a grid-stride loop over at most 2048 workgroups: enough for the copy, and a
    // gated-off launch retires in a few microseconds
    const unsigned grid = grid_for(chunks) < 2048u ? grid_for(chunks) : 2048u;
    if (cb == 16)
        hipLaunchKernelGGL(k_shift_time<uint4>, dim3(grid), dim3(256), 0, st, chunks, cpr, T, D,
                           static_cast<const uint4 *>(in), static_cast<uint4 *>(out), skip_cnt, skip_le);
    else if (cb == 4)
        hipLaunchKernelGGL(k_shift_time<uint32_t>, dim3(grid), dim3(256), 0, st, chunks, cpr, T, D,
                           static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out), skip_cnt, skip_le);
    else
        hipLaunchKernelGGL(k_shift_time<uint8_t>, dim3(grid), dim3(256), 0, st, chunks, cpr, T, D,
                           static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out), skip_cnt, skip_le);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3((a.N + 63) / 64), dim3(64 * FIN_PH), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_decay_tables(int N, int TR, double dt, const float *tau_m, const float *tau_a,
                               float *bp, float *pp, hipStream_t st) {
    const int total = N * (TR + 1);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_decay_tables, dim3((total + 255) / 256), dim3(256), 0, st, N, TR, dt,
                       tau_m, tau_a, bp, pp);
    return hipGetLastError();
}

}  // namespace alif
