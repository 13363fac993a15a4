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
#include "alif_gemm_big.h"

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
    if (gemm_gated_off(g.skip_cnt, g.skip_le)) return;
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
// Tiled fast path. C = A B^T (+ bias) on MFMA tiles fed by a two-stage register
// pipeline: while the LDS buffer of one K stage is multiplied, every thread
// loads its share of the next stage with raw buffer loads, converts it to the
// MFMA operand type and stores it to the other LDS buffer; one barrier per stage.
// Both operands sit in LDS as [row][k] (k contiguous) whatever their layout in
// memory:
//   k-contiguous operand ([row][k] in memory): a thread loads EPT consecutive k
//     of one row;
//   row-contiguous operand ([k][row] in memory): a thread loads RR consecutive
//     rows for 8 consecutive k and transposes them in registers.
// BF16 tiles are 256 x 128 over eight waves (the operand read as float is reused
// over more rows), FP32 tiles 128 x 128 over four; each wave owns 64 x 64 as
// 4 x 4 MFMA 16 x 16 accumulators. Workgroups are numbered so that the N tiles
// of one M tile (and K split) run on one XCD and share its rows of A in that
// XCD's L2. A split over K writes partial tiles that k_split_reduce sums.
// The three uses: the Eq. 3 current (A = spikes [M][K], B = W [N][K], both
// k-contiguous), the input gradient (A = gI k-contiguous, B = W row-contiguous)
// and the weight gradient (A = gI and B = spikes, both row-contiguous).
// ---------------------------------------------------------------------------
template <bool BF16>
struct Tile {
    static constexpr int BM = BF16 ? 256 : 128, BN = 128;
    static constexpr int THREADS = BF16 ? 512 : 256;
    static constexpr int BK = BF16 ? 64 : 32;           // k per stage
    static constexpr int LDK = BF16 ? BK + 8 : BK + 4;   // LDS row (elements), 16-byte multiple
    using T = typename std::conditional<BF16, __bf16, float>::type;
    static constexpr size_t lds_bytes() { return (size_t)2 * (BM + BN) * LDK * sizeof(T); }
};

template <int DT>
constexpr uint32_t elem_bytes() { return DT == 0 ? 4 : (DT == 1 ? 1 : 2); }

// A run of N consecutive elements (one buffer load of N * elem bytes). The raw
// words stay in registers until get() converts them, so that the wait for the
// load falls after the work placed between load() and get().
template <int DT, int N>
struct Run {
    static_assert(N == 2 || N == 4, "runs of 2 or 4");
    static constexpr uint32_t BYTES = N * elem_bytes<DT>();
    static constexpr int DW = BYTES < 4 ? 1 : (int)(BYTES / 4);
    uint32_t w[DW];

    __device__ __forceinline__ void load(rsrc_t r, uint32_t off) {
        if constexpr (BYTES == 16) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; e++) w[e] = x[e];
        } else if constexpr (BYTES == 8) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            w[0] = x[0];
            w[1] = x[1];
        } else if constexpr (BYTES == 4) {
            w[0] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        } else {
            w[0] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        }
    }
    __device__ __forceinline__ void get(float *v) const {
        if constexpr (DT == 0) {
#pragma unroll
            for (int e = 0; e < N; e++) v[e] = __uint_as_float(w[e]);
        } else if constexpr (DT == 1) {
#pragma unroll
            for (int e = 0; e < N; e++) v[e] = (float)((w[0] >> (8 * e)) & 0xffu);
        } else {
#pragma unroll
            for (int q = 0; q < N / 2; q++) {
                v[2 * q] = __uint_as_float(w[q] << 16);
                v[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
            }
        }
    }
};

// LDS tiles hold rows of the operand, k contiguous, in 16-byte chunks (8 bf16 or
// 4 floats). Chunk c of row r sits at chunk position c ^ ((r / 16) % 4): the
// MFMA fragment reads (16 consecutive rows, one chunk each) stay conflict-free
// and the transposing stores of row-contiguous operands, whose lanes write rows
// RR apart, spread over all banks instead of a quarter of them.
template <bool BF16>
__device__ __forceinline__ int lds_at(int row, int chunk) {
    constexpr int CE = BF16 ? 8 : 4;
    return row * Tile<BF16>::LDK + (chunk ^ ((row >> 4) & 3)) * CE;
}

// 4 values (k = 4 h .. 4 h + 3 of chunk c) to LDS row `row` in the MFMA operand type
template <bool BF16>
__device__ __forceinline__ void lds_store4(typename Tile<BF16>::T *buf, int row, int k, const float *v) {
    if constexpr (BF16) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 q;
#pragma unroll
        for (int e = 0; e < 4; e++) q[e] = (__bf16)v[e];
        *reinterpret_cast<bf16x4 *>(buf + lds_at<true>(row, k >> 3) + (k & 4)) = q;
    } else {
        *reinterpret_cast<floatx4 *>(buf + lds_at<false>(row, k >> 2)) = floatx4{v[0], v[1], v[2], v[3]};
    }
}

// 8 values (k = k0 .. k0 + 7, k0 a multiple of 8) to LDS row `row`
template <bool BF16>
__device__ __forceinline__ void lds_store8(typename Tile<BF16>::T *buf, int row, int k0, const float *v) {
    if constexpr (BF16) {
        bf16x8 q;
#pragma unroll
        for (int e = 0; e < 8; e++) q[e] = (__bf16)v[e];
        *reinterpret_cast<bf16x8 *>(buf + lds_at<true>(row, k0 >> 3)) = q;
    } else {
        *reinterpret_cast<floatx4 *>(buf + lds_at<false>(row, k0 >> 2)) = floatx4{v[0], v[1], v[2], v[3]};
        *reinterpret_cast<floatx4 *>(buf + lds_at<false>(row, (k0 >> 2) + 1)) = floatx4{v[4], v[5], v[6], v[7]};
    }
}

// One operand's ROWS x BK stage: where this thread loads it from and where it
// puts it in LDS. Loads are coalesced along memory's contiguous direction:
//   k-contiguous: BK / 4 consecutive threads read one row's BK elements of the
//     stage in runs of 4, and a thread covers NI rows RPP apart;
//   row-contiguous: RG consecutive threads read RR * RG consecutive rows of one k,
//     and a thread covers 8 consecutive k.
//   ptr, ld: operand base and elements between consecutive rows (k-contiguous)
//            or consecutive k (row-contiguous);
//   rows:    valid rows (M or N), row0 the tile's first row;
//   kb, ke:  the K range of this workgroup's split.
// Each stage gets its own buffer descriptor, starting at the stage and ending
// where the operand's valid data ends, so the per-thread offsets stay fixed:
// k-contiguous: rows beyond the valid ones read 0, and k >= ke is zeroed in the
//   last stage;
// row-contiguous: k >= ke reads 0; rows beyond the valid ones may read other
//   data, which only reaches rows of C that are never stored.
template <int DT, bool KM, int ROWS, bool BF16>
struct Stage {
    using P = Tile<BF16>;
    static constexpr int BK = P::BK;
    static constexpr int EPT = ROWS * BK / P::THREADS;   // elements per thread per stage
    static constexpr int RR = EPT / 8;                    // row-contiguous: rows per thread
    static constexpr int RG = ROWS / RR;                  // row-contiguous: row groups
    static constexpr int CPR = BK / 4;                    // k-contiguous: threads per row
    static constexpr int RPP = P::THREADS / CPR;          // k-contiguous: rows per pass
    static constexpr int NI = ROWS / RPP;                 // k-contiguous: passes
    static constexpr int NL = KM ? 8 : NI;                // loads per thread per stage
    static constexpr uint32_t ES = elem_bytes<DT>();
    static_assert(EPT % 8 == 0 && (!KM || P::THREADS / RG == BK / 8) && (KM || NI * 4 == EPT),
                  "stage shape");

    static constexpr int REG_WORDS = NL * Run<DT, KM ? RR : 4>::DW;  // registers of one stage in flight

    // one stage in flight: its raw loaded words and where it ends
    struct Regs {
        Run<DT, KM ? RR : 4> run[NL];
        int kmax;   // k-contiguous: valid k of this thread in the stage
        bool tail;  // the stage runs past ke
    };

    const char *sbase;  // the operand at stage 0 of this split and tile
    uint32_t ext;       // bytes of valid data from sbase
    uint32_t sstep;     // bytes between stages
    int kspan;          // K steps in this split
    uint32_t voff[NL];  // byte offsets of this thread's loads within a stage
    int kmax0;          // k-contiguous: valid k of this thread at stage 0
    int lrow, lk;       // LDS row and first k of this thread

    __device__ __forceinline__ void init(const void *ptr, long long ld, long long rows, long long row0, int kb,
                                         int ke, int tid) {
        const char *base = static_cast<const char *>(ptr);
        const long long vr = rows - row0;                  // valid rows from row0 (> 0)
        kspan = ke - kb;
        if constexpr (KM) {
            const int rg = tid % RG, kg = tid / RG;
            lrow = rg * RR;
            lk = kg * 8;
            sbase = base + ((size_t)kb * ld + row0) * ES;
            ext = (uint32_t)(((size_t)(ke - kb - 1) * ld + vr) * ES);
            sstep = (uint32_t)((size_t)BK * ld * ES);
#pragma unroll
            for (int j = 0; j < 8; j++) voff[j] = (uint32_t)(((size_t)(lk + j) * ld + lrow) * ES);
        } else {
            lrow = tid / CPR;
            lk = (tid % CPR) * 4;
            const long long nr = vr < ROWS ? vr : ROWS;
            sbase = base + ((size_t)row0 * ld + kb) * ES;
            ext = (uint32_t)(((size_t)nr * ld - kb) * ES);
            sstep = (uint32_t)(BK * ES);
#pragma unroll
            for (int i = 0; i < NI; i++) voff[i] = (uint32_t)(((size_t)(lrow + i * RPP) * ld + lk) * ES);
            kmax0 = kspan - lk;
        }
    }
    // issue the loads of stage s (k = kb + s * BK ...) into g; a stage past the
    // split gets an empty descriptor and reads zeros
    __device__ __forceinline__ void load(int s, Regs &g) const {
        // the descriptor is uniform; readfirstlane keeps the compiler from
        // treating it as divergent (which wraps every load in a waterfall loop)
        const uint32_t o = (uint32_t)__builtin_amdgcn_readfirstlane(s) * sstep;
        const uint64_t bp = reinterpret_cast<uint64_t>(sbase + o);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)bp);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(bp >> 32));
        const uint32_t nrec = __builtin_amdgcn_readfirstlane(o < ext ? ext - o : 0u);
        const rsrc_t r = make_rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo), nrec);
#pragma unroll
        for (int i = 0; i < NL; i++) g.run[i].load(r, voff[i]);
        g.tail = (s + 1) * BK > kspan;
        if constexpr (!KM) g.kmax = kmax0 - s * BK;
    }
    // convert a loaded stage and store it to the LDS tile buf
    __device__ __forceinline__ void store(const Regs &g, typename P::T *buf) const {
        if constexpr (KM) {
            float v[8][RR];
#pragma unroll
            for (int j = 0; j < 8; j++) g.run[j].get(v[j]);
#pragma unroll
            for (int rr = 0; rr < RR; rr++) {
                float c[8];
#pragma unroll
                for (int j = 0; j < 8; j++) c[j] = v[j][rr];
                lds_store8<BF16>(buf, lrow + rr, lk, c);
            }
        } else {
            float v[NI][4];
#pragma unroll
            for (int i = 0; i < NI; i++) g.run[i].get(v[i]);
            if (g.tail) {
#pragma unroll
                for (int i = 0; i < NI; i++)
#pragma unroll
                    for (int e = 0; e < 4; e++) v[i][e] = e < g.kmax ? v[i][e] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < NI; i++) lds_store4<BF16>(buf, lrow + i * RPP, lk, v[i]);
        }
    }
};

template <int ADT, bool AKM, int BDT, bool BKM, bool BF16>
__global__ __launch_bounds__(Tile<BF16>::THREADS) void k_gemm_tiled(GemmArgs g, int m_tiles, int n_tiles,
                                                                     int kps, int total) {
    if (gemm_gated_off(g.skip_cnt, g.skip_le)) return;
    using P = Tile<BF16>;
    using T = typename P::T;
    constexpr int BM = P::BM, BN = P::BN, BK = P::BK, LDK = P::LDK;
    extern __shared__ __align__(16) unsigned char lds[];
    T *As = reinterpret_cast<T *>(lds);                   // [2][BM][LDK]
    T *Bs = As + 2 * BM * LDK;                            // [2][BN][LDK]

    const int work = xcd_remap(blockIdx.x, total);
    const int tiles = m_tiles * n_tiles;
    const int z = work / tiles, t = work % tiles;
    const long long m0 = (long long)(t / n_tiles) * BM;
    const int n0 = (t % n_tiles) * BN;
    const int kb = z * kps, ke = min(g.K, kb + kps);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;              // wave tile (wm, wn) of 64 x 64

    Stage<ADT, AKM, BM, BF16> sa;
    Stage<BDT, BKM, BN, BF16> sb;
    sa.init(g.A, g.lda, g.M, m0, kb, ke, tid);
    sb.init(g.B, g.ldb, g.N, n0, kb, ke, tid);

    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // multiply the stage in LDS buffer buf into the accumulators
    auto mma = [&](int buf) {
        const T *a = As + (size_t)buf * BM * LDK;
        const T *b = Bs + (size_t)buf * BN * LDK;
        if constexpr (BF16) {
#pragma unroll
            for (int kq = 0; kq < BK; kq += 32) {
                bf16x8 fa[4], fb[4];
                const int kc = kq + 8 * (lane >> 4);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    fa[i] = *reinterpret_cast<const bf16x8 *>(a + lds_at<true>(wm * 64 + i * 16 + (lane & 15), kc >> 3));
#pragma unroll
                for (int j = 0; j < 4; j++)
                    fb[j] = *reinterpret_cast<const bf16x8 *>(b + lds_at<true>(wn * 64 + j * 16 + (lane & 15), kc >> 3));
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
                for (int i = 0; i < 4; i++) fa[i] = a[lds_at<false>(wm * 64 + i * 16 + (lane & 15), kc >> 2) + (kc & 3)];
#pragma unroll
                for (int j = 0; j < 4; j++) fb[j] = b[lds_at<false>(wn * 64 + j * 16 + (lane & 15), kc >> 2) + (kc & 3)];
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        }
    };

    // Loads are issued unconditionally (past the split they read zeros): a load
    // under a condition makes the compiler copy its registers, which waits for
    // it. sched_barrier keeps the compiler from moving instructions across it.
    using SA = Stage<ADT, AKM, BM, BF16>;
    using SB = Stage<BDT, BKM, BN, BF16>;
    T *const L0a = As, *const L1a = As + (size_t)BM * LDK;
    T *const L0b = Bs, *const L1b = Bs + (size_t)BN * LDK;
    const int nk = (ke - kb + BK - 1) / BK;
    if constexpr (BF16 && SA::REG_WORDS + SB::REG_WORDS <= 32) {
        // Two stages in flight. While stage kt is multiplied from one LDS
        // buffer, stage kt + 1, loaded a whole stage earlier, is converted and
        // stored to the other, interleaved with the MFMAs; then the loads of
        // stage kt + 3 go out. Stages alternate between two register sets; the
        // loop body covers an even and an odd stage so that both are addressed
        // statically. Stages past the split are stored to the buffer nobody reads.
        typename SA::Regs ra0, ra1;
        typename SB::Regs rb0, rb1;
        sa.load(0, ra0);
        sb.load(0, rb0);
        sa.load(1, ra1);
        sb.load(1, rb1);
        sa.store(ra0, L0a);
        sb.store(rb0, L0b);
        __syncthreads();
        sa.load(2, ra0);
        sb.load(2, rb0);
        int kt = 0;
        for (; kt + 2 <= nk; kt += 2) {
            __builtin_amdgcn_sched_barrier(0);
            mma(0);
            sa.store(ra1, L1a);
            sb.store(rb1, L1b);
            __syncthreads();
            sa.load(kt + 3, ra1);
            sb.load(kt + 3, rb1);
            __builtin_amdgcn_sched_barrier(0);
            mma(1);
            sa.store(ra0, L0a);
            sb.store(rb0, L0b);
            __syncthreads();
            sa.load(kt + 4, ra0);
            sb.load(kt + 4, rb0);
        }
        if (kt < nk) mma(0);
    } else {
        // One stage in flight (wide operands would not fit two in registers):
        // the loads of stage kt + 1 are issued before stage kt is multiplied and
        // converted and stored after it.
        typename SA::Regs ra;
        typename SB::Regs rb;
        sa.load(0, ra);
        sb.load(0, rb);
        sa.store(ra, L0a);
        sb.store(rb, L0b);
        __syncthreads();
        for (int kt = 0; kt + 1 < nk; kt++) {
            const int buf = kt & 1;
            sa.load(kt + 1, ra);
            sb.load(kt + 1, rb);
            __builtin_amdgcn_sched_barrier(0);
            mma(buf);
            __builtin_amdgcn_sched_barrier(0);
            sa.store(ra, buf ? L0a : L1a);
            sb.store(rb, buf ? L0b : L1b);
            __syncthreads();
        }
        mma((nk - 1) & 1);
    }
    // epilogue: lane holds rows 4 * (lane / 16) + r of column lane % 16 of each 16 x 16 block
    const bool split = total > tiles;
    float *out = split ? g.C_part + (size_t)z * g.M * g.N : g.C;
    const long long ldc = split ? g.N : g.ldc;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        const float bias = (g.bias && !split && n < g.N) ? g.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const long long m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + rr;
                if (m < g.M && n < g.N) out[m * ldc + n] = acc[i][j][rr] + bias;
            }
    }
}

// K per split of the tiled path: a multiple of the stage depth
static int tiled_kps(const GemmArgs &g, int bk) {
    const int s = g.splits < 1 ? 1 : g.splits;
    const int k = (g.K + s - 1) / s;
    return (k + bk - 1) / bk * bk;
}

// whether the tiled path covers this call: one of the three operand patterns,
// rows and bases aligned for its vector loads, every buffer extent within 31 bits
static bool tiled_ok(const GemmArgs &g, bool bf16) {
    const bool fwd = g.a_kc && g.b_kc && g.b_dt == 0;
    const bool dx = g.a_kc && (g.a_dt == 0 || g.a_dt == 2) && !g.b_kc && g.b_dt == 0;
    const bool dw = !g.a_kc && (g.a_dt == 0 || g.a_dt == 2) && !g.b_kc;
    if (!(fwd || dx || dw) || g.K <= 0) return false;
    if ((reinterpret_cast<uintptr_t>(g.A) & 15) || (reinterpret_cast<uintptr_t>(g.B) & 15)) return false;
    if (g.lda % 4 != 0 || g.ldb % 4 != 0) return false;
    if (!g.a_kc && (g.M % 4 != 0 || g.lda < g.M)) return false;
    if (!g.b_kc && (g.N % 4 != 0 || g.ldb < g.N)) return false;
    if (g.splits > 1 && (g.a_kc || g.b_kc)) return false;
    const int bk = bf16 ? Tile<true>::BK : Tile<false>::BK;
    const size_t kps = (size_t)tiled_kps(g, bk) + bk;
    const size_t lim = (size_t)1 << 31;
    const size_t aes = g.a_dt == 0 ? 4 : (g.a_dt == 1 ? 1 : 2), bes = g.b_dt == 0 ? 4 : (g.b_dt == 1 ? 1 : 2);
    const size_t a_ext = g.a_kc ? (size_t)Tile<true>::BM * g.lda * aes : kps * g.lda * aes;
    const size_t b_ext = g.b_kc ? (size_t)Tile<true>::BN * g.ldb * bes : kps * g.ldb * bes;
    return a_ext < lim && b_ext < lim;
}

template <int ADT, bool AKM, int BDT, bool BKM, bool BF16>
static void tiled_go(const GemmArgs &g, int m_tiles, int n_tiles, int kps, int total, hipStream_t st) {
    hipLaunchKernelGGL((k_gemm_tiled<ADT, AKM, BDT, BKM, BF16>), dim3((unsigned)total),
                       dim3(Tile<BF16>::THREADS), Tile<BF16>::lds_bytes(), st, g, m_tiles, n_tiles, kps, total);
}

template <bool BF16>
static hipError_t tiled_launch(const GemmArgs &g, hipStream_t st, int *splits_out) {
    using P = Tile<BF16>;
    const long long m_tiles = (g.M + P::BM - 1) / P::BM;
    const int n_tiles = (g.N + P::BN - 1) / P::BN;
    const int kps = tiled_kps(g, P::BK);
    const int splits = (g.K + kps - 1) / kps;
    const long long total = m_tiles * n_tiles * splits;
    if (total > 0x7fffffffLL || m_tiles * n_tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    const int mt = (int)m_tiles, tt = (int)total;
    *splits_out = splits;
    if (g.a_kc && g.b_kc) {
        if (g.a_dt == 0) tiled_go<0, false, 0, false, BF16>(g, mt, n_tiles, kps, tt, st);
        else if (g.a_dt == 1) tiled_go<1, false, 0, false, BF16>(g, mt, n_tiles, kps, tt, st);
        else tiled_go<2, false, 0, false, BF16>(g, mt, n_tiles, kps, tt, st);
    } else if (g.a_kc) {
        if (g.a_dt == 2) tiled_go<2, false, 0, true, BF16>(g, mt, n_tiles, kps, tt, st);
        else tiled_go<0, false, 0, true, BF16>(g, mt, n_tiles, kps, tt, st);
    } else if (g.a_dt == 2) {
        if (g.b_dt == 0) tiled_go<2, true, 0, true, BF16>(g, mt, n_tiles, kps, tt, st);
        else if (g.b_dt == 1) tiled_go<2, true, 1, true, BF16>(g, mt, n_tiles, kps, tt, st);
        else tiled_go<2, true, 2, true, BF16>(g, mt, n_tiles, kps, tt, st);
    } else {
        if (g.b_dt == 0) tiled_go<0, true, 0, true, BF16>(g, mt, n_tiles, kps, tt, st);
        else if (g.b_dt == 1) tiled_go<0, true, 1, true, BF16>(g, mt, n_tiles, kps, tt, st);
        else tiled_go<0, true, 2, true, BF16>(g, mt, n_tiles, kps, tt, st);
    }
    return hipGetLastError();
}

// fixed-order sum of split partials: C[m][n] = sum_z P[z][m][n] (+ bias)
__global__ void k_split_reduce(long long MN, int N, int splits, const float *P, float *C,
                               const float *bias, const unsigned long long *skip_cnt, unsigned long long skip_le) {
    if (gemm_gated_off(skip_cnt, skip_le)) return;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN) return;
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += P[(size_t)z * MN + i];
    if (bias) s += bias[i % N];
    C[i] = s;
}

hipError_t gemm_launch(const GemmArgs &g, bool bf16, hipStream_t st) {
    if (g.M == 0 || g.N == 0) return hipSuccess;
    if (bf16 && gemm_big_ok(g)) return gemm_big_launch(g, st);
    if (tiled_ok(g, bf16)) {
        int splits = 1;
        hipError_t e = bf16 ? tiled_launch<true>(g, st, &splits) : tiled_launch<false>(g, st, &splits);
        if (e != hipSuccess || splits == 1) return e;
        const long long MN = g.M * (long long)g.N;
        hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, MN, g.N,
                           splits, g.C_part, g.C, g.bias, g.skip_cnt, g.skip_le);
        return hipGetLastError();
    }
    dim3 grid((g.N + GBN - 1) / GBN, (unsigned)((g.M + GBM - 1) / GBM), g.splits);
    if (grid.y > 65535) return hipErrorInvalidValue;
    if (bf16) hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.splits == 1) return e;
    const long long MN = g.M * (long long)g.N;
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, MN, g.N,
                       g.splits, g.C_part, g.C, g.bias, g.skip_cnt, g.skip_le);
    return hipGetLastError();
}

static int dt_of(int kind) {
    return kind == ALIF_INPUT_SPIKES_U8 ? 1 : (kind == ALIF_INPUT_SPIKES_BF16 ? 2 : 0);
}

// W [N][K] float -> bfloat16 (round to nearest even), the same layout (TRANS = false)
// or transposed to [K][N] (TRANS = true, through a 32 x 32 LDS tile), with output
// rows of ldo >= K (resp. N) elements whose padding is zero
template <bool TRANS>
__global__ __launch_bounds__(256) void k_w_bf16(int N, int K, const float *W, __bf16 *out, int ldo) {
    if constexpr (!TRANS) {
        const long long n = (long long)N * ldo;
        for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
            const long long r = i / ldo, k = i - r * ldo;
            out[i] = (__bf16)(k < K ? W[r * K + k] : 0.0f);
        }
    } else {
        __shared__ float t[32][33];
        const int k0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
        for (int r = ty; r < 32; r += 8)
            t[r][tx] = (n0 + r < N && k0 + tx < K) ? W[(size_t)(n0 + r) * K + k0 + tx] : 0.0f;
        __syncthreads();
        // (the column tiles cover ldo: ldo <= 32 ceil(N / 32))
        for (int r = ty; r < 32; r += 8)
            if (k0 + r < K && n0 + tx < ldo) out[(size_t)(k0 + r) * ldo + n0 + tx] = (__bf16)t[tx][r];
    }
}

// bfloat16 rows padded to whole 16-byte chunks, which the large-tile kernel loads
static int ld16(int n) { return (n + 7) / 8 * 8; }

size_t gemm_wbf16_bytes(int N, int K) {
    const size_t fwd = (size_t)N * ld16(K), trans = (size_t)K * ld16(N);
    return (fwd > trans ? fwd : trans) * 2;
}

static bool scratch_fits(const void *scratch, size_t bytes, int N, int K) {
    return scratch && bytes >= gemm_wbf16_bytes(N, K) && (reinterpret_cast<uintptr_t>(scratch) & 15) == 0;
}

// Sparse spike input: a density (estimated on the device from a sample of rows) of at
// most one nonzero per ev_cut entries takes the current from the active inputs alone
// (FP32 sums of exact products; under BF16 GEMMs of W rounded to bfloat16, the GEMM's
// rounding of it); the GEMM is enqueued behind it with the opposite gate. Only for
// inputs of more than EV_MIN entries, where the sample (10 us) is small against either
// product. The cuts come from timing both on MI355X with a cold MALL: against the FP32
// GEMM the event kernel was 2-8x faster up to 5% active (K 700, N 512 and 1024);
// against the BF16 GEMM it won up to 1% at N = 1024 (0.50 against 0.61 ms) and lost at
// 2% (0.73 ms), and with N = 20 it won at 0.19% and lost at 2%.
constexpr double EV_MIN = 16777216.0;
static int ev_cut(bool bf16, int N) { return bf16 ? (N >= 256 ? 64 : 256) : 16; }

hipError_t gemm_input_current(size_t M, int N, int K, GemmIn x, const float *W, const float *bias,
                              float *out, bool bf16, hipStream_t st, void *scratch, size_t scratch_bytes) {
    GemmArgs g{};
    g.M = (long long)M; g.N = N; g.K = K;
    g.A = x.ptr; g.a_dt = dt_of(x.kind); g.lda = K; g.a_kc = 1;
    g.B = W; g.b_dt = 0; g.ldb = K; g.b_kc = 1;
    g.C = out; g.ldc = N; g.bias = bias; g.splits = 1;
    const bool spk = x.kind == ALIF_INPUT_SPIKES_U8 || x.kind == ALIF_INPUT_SPIKES_BF16;
    const size_t wt_bytes = ((size_t)K * N * 4 + 255) & ~(size_t)255;
    if (spk && M > 0 && N > 0 && K > 0 && M < ((size_t)1 << 31) && (double)M * K > EV_MIN && scratch &&
        (reinterpret_cast<uintptr_t>(scratch) & 255) == 0 &&
        scratch_bytes >= 256 + wt_bytes + gemm_wbf16_bytes(N, K)) {
        // scratch: the gate word, W transposed, then the GEMM's bfloat16 copy of W
        unsigned long long *flag = static_cast<unsigned long long *>(scratch);
        float *WT = reinterpret_cast<float *>(static_cast<char *>(scratch) + 256);
        const int elem = x.kind == ALIF_INPUT_SPIKES_U8 ? 1 : 2;
        if (density_flag_launch((long long)M, K, elem, x.ptr, flag, 1, ev_cut(bf16, N), st) == hipSuccess &&
            events_current_launch(x.kind, (long long)M, K, N, x.ptr, W, WT, bf16, bias, out, flag, st)) {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            g.skip_cnt = flag;   // the GEMM returns at entry when *flag == 0 (the event path ran)
            g.skip_le = 0;
            scratch = static_cast<char *>(scratch) + 256 + wt_bytes;
            scratch_bytes -= 256 + wt_bytes;
        }
    }
    if (bf16 && M > 0 && N > 0 && scratch_fits(scratch, scratch_bytes, N, K)) {
        GemmArgs h = g;
        h.B = scratch; h.b_dt = 2; h.ldb = ld16(K);
        if (gemm_big_ok(h)) {
            const long long n = (long long)N * h.ldb;
            const unsigned grid = (unsigned)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
            hipLaunchKernelGGL(k_w_bf16<false>, dim3(grid), dim3(256), 0, st, N, K, W, static_cast<__bf16 *>(scratch),
                               (int)h.ldb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return gemm_big_launch(h, st);
        }
    }
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

hipError_t gemm_weight_grad(size_t M, int N, int K, const void *gI, GemmIn x, float *gW, bool bf16,
                            void *ws, hipStream_t st, const unsigned long long *skip_cnt,
                            unsigned long long skip_le, bool gi_bf16) {
    // C[n][k] = sum_m gI[m][n] x[m][k]: reduction over m (split), both operands m-major
    GemmArgs g{};
    g.M = N; g.N = K; g.K = (int)M;
    g.A = gI; g.a_dt = gi_bf16 ? 2 : 0; g.lda = N; g.a_kc = 0;
    g.B = x.ptr; g.b_dt = dt_of(x.kind); g.ldb = K; g.b_kc = 0;
    g.C = gW; g.ldc = K; g.bias = nullptr;
    g.splits = wgrad_splits(M, N, K);
    g.C_part = (float *)ws;
    g.skip_cnt = skip_cnt;
    g.skip_le = skip_le;
    if (M > 0x7fffffff) return hipErrorInvalidValue;
    return gemm_launch(g, bf16, st);
}

hipError_t gemm_input_grad(size_t M, int N, int K, const void *gI, const float *W, float *gx,
                           bool bf16, hipStream_t st, void *scratch, size_t scratch_bytes, bool gi_bf16) {
    // C[m][k] = sum_n gI[m][n] W[n][k]
    GemmArgs g{};
    g.M = (long long)M; g.N = K; g.K = N;
    g.A = gI; g.a_dt = gi_bf16 ? 2 : 0; g.lda = N; g.a_kc = 1;
    g.B = W; g.b_dt = 0; g.ldb = K; g.b_kc = 0;
    g.C = gx; g.ldc = K; g.bias = nullptr; g.splits = 1;
    if (bf16 && M > 0 && K > 0 && scratch_fits(scratch, scratch_bytes, N, K)) {
        GemmArgs h = g;   // B(k, n) = W^T[k][n]: k-contiguous in the transposed copy
        h.B = scratch; h.b_dt = 2; h.ldb = ld16(N); h.b_kc = 1;
        if (gemm_big_ok(h)) {
            hipLaunchKernelGGL(k_w_bf16<true>, dim3((unsigned)((K + 31) / 32), (unsigned)((N + 31) / 32)), dim3(256), 0,
                               st, N, K, W, static_cast<__bf16 *>(scratch), (int)h.ldb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return gemm_big_launch(h, st);
        }
    }
    return gemm_launch(g, bf16, st);
}

}  // namespace alif
