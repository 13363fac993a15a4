// Large-tile BF16 MFMA GEMM for gfx950 (paper Eq. 3 projections and their
// gradients on wide layers); the design is described in alif_gemm_big.h.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "alif_common.h"
#include "alif_gemm_big.h"

namespace alif {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int TM = 256, TN = 256, TK = 64;
constexpr uint32_t ROWB = TK * 2;                                // LDS bytes per operand row (64 bf16)
constexpr uint32_t BUF_A = TM * ROWB, BUF_B = TN * ROWB;         // one LDS buffer of each operand
constexpr size_t LDS_BYTES = 2 * (size_t)(BUF_A + BUF_B);        // two buffers: 128 KiB

// byte offset of 16-byte chunk c (k = 8 c .. 8 c + 7) of row r in an LDS operand buffer:
// chunk c of row r sits at position c ^ ((r / 2) % 8). A 128-byte row covers half
// of the LDS banks, so consecutive rows alternate halves; with the position taken
// from the next three row bits, the 16 consecutive rows of one pass of a fragment
// read hit 16 different 16-byte bank groups.
__device__ __forceinline__ uint32_t lds_swz(int r) { return (uint32_t)((r >> 1) & 7); }
__device__ __forceinline__ uint32_t lds_off(int r, int c) {
    return (uint32_t)r * ROWB + (((uint32_t)c ^ lds_swz(r)) << 4);
}

// two floats -> two bfloat16 in one dword (v_cvt_pk_bf16_f32, round to nearest even)
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// One load at byte offset voff. The whole offset goes in the VGPR operand: the
// buffer range check covers the VGPR offset and the instruction's immediate but
// not the SGPR offset, so an offset carried there could read past the operand.
template <int BYTES>
__device__ __forceinline__ void ld_raw(rsrc_t r, uint32_t voff, uint32_t *w) {
    if constexpr (BYTES == 16) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
        w[0] = x[0];
        w[1] = x[1];
        w[2] = x[2];
        w[3] = x[3];
    } else {
        w[0] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0);
    }
}

// element e (0..3) of a dword holding four uint8, as float (exact)
__device__ __forceinline__ float u8f(uint32_t w, int e) { return (float)((w >> (8 * e)) & 0xffu); }

// One operand's 256 x 64 stage, loaded by the 256 threads of the workgroup and
// stored to an LDS buffer as bfloat16 rows of 64 k (chunk c of row r at position
// c ^ (r % 8)).
//   K-major ([rows][k] in memory): a unit is 8 consecutive k of one row: f32 two
//     16-byte loads, bf16 one, uint8 two 4-byte loads. Thread t takes chunk t % 8 of
//     rows t / 8 + (NT / 8) u: eight threads read a row's 64 k, and the eight
//     chunks they store land on different banks.
//   R-major ([k][rows] in memory): a unit is Q consecutive rows (16 bytes; 4 bytes
//     of uint8) at each of 8 consecutive k, transposed in registers into Q rows of
//     8 k. Thread t takes k chunk t % 8 of row groups t / 8 + (NT / 8) u (with
//     fewer units than threads, the last waves have none): per load instruction a
//     wave reads 128 contiguous bytes of each of 8 k rows, and the eight threads
//     that store one row write its eight different chunks.
// Each stage gets its own buffer descriptor starting at the stage and ending
// where the operand's valid data ends: K-major rows past the valid ones and
// R-major k past the range read zeros; K-major k past the range inside a valid
// row is zeroed after the load; R-major rows past the valid ones may read other
// data, which reaches only columns of C that are never stored.
template <int DT, bool RMAJ, int NT>
struct Op {
    static constexpr int ES = DT == 0 ? 4 : (DT == 1 ? 1 : 2);
    static constexpr int Q = RMAJ ? (DT == 2 ? 8 : 4) : 1;                   // rows per R-major unit
    static constexpr int TOTAL = RMAJ ? 8 * (256 / Q) : 8 * 256;              // units per stage
    static constexpr int UNITS = TOTAL >= NT ? TOTAL / NT : 1;                // units per thread per stage
    static constexpr bool PARTIAL = TOTAL < NT;                               // the last waves have none
    static constexpr int RSTEP = NT / 8;                                      // rows (groups) between units
    static constexpr int LB = DT == 1 ? 4 : 16;                               // bytes per load
    static constexpr int LOADS = RMAJ ? 8 : (8 * ES) / LB;                    // loads per unit
    static constexpr int LW = LB / 4;                                          // dwords per load
    static constexpr int WORDS = UNITS * LOADS * LW;                           // registers of a stage

    const char *base;   // stage 0 of this tile and split
    uint32_t ext;       // valid bytes from base
    uint32_t sstep;     // bytes between stages
    uint32_t ustep;     // bytes between this thread's consecutive units (uniform)
    uint32_t lstep;     // bytes between the loads of a unit (uniform)
    uint32_t voff0;     // byte offset of this thread's first load within a stage
    uint32_t lds0;      // LDS byte offset of this thread's first store
    int kspan;          // k steps in this split
    int kc0;            // this thread's k chunk
    bool active;        // this thread (and its whole wave) has units

    __device__ __forceinline__ void init(const void *ptr, long long ld, long long rows, long long rbase, int kb,
                                         int ke, int tid) {
        const char *p = static_cast<const char *>(ptr);
        kspan = ke - kb;
        kc0 = tid & 7;
        active = !PARTIAL || tid < TOTAL;
        if constexpr (!RMAJ) {
            const long long nr = rows - rbase < TM ? rows - rbase : TM;
            const int row0 = tid >> 3;
            base = p + ((size_t)rbase * ld + kb) * ES;
            // rounded up to the load width: a load that straddles the last valid k keeps its
            // valid part (the range check drops whole dwords); the rounding stays inside the
            // row's padding, as rows are LB-aligned and ld >= K
            ext = (uint32_t)((((size_t)(nr - 1) * ld + (size_t)(ke - kb)) * ES + LB - 1) / LB * LB);
            sstep = (uint32_t)(TK * ES);
            voff0 = (uint32_t)(((size_t)row0 * ld + (size_t)kc0 * 8) * ES);
            ustep = (uint32_t)((size_t)RSTEP * ld * ES);
            lstep = LB;
            lds0 = lds_off(row0, kc0);   // rows row0 + RSTEP u keep the position (RSTEP a multiple of 16)
        } else {
            const int rg0 = tid >> 3;
            base = p + ((size_t)kb * ld + rbase) * ES;
            // rounded up as above (rows are LB-aligned and ld >= rows)
            ext = (uint32_t)((((size_t)(ke - kb - 1) * ld + (size_t)(rows - rbase)) * ES + LB - 1) / LB * LB);
            sstep = (uint32_t)((size_t)TK * ld * ES);
            voff0 = active ? (uint32_t)(((size_t)kc0 * 8 * ld + (size_t)rg0 * Q) * ES) : ALIF_OOB;
            ustep = (uint32_t)(RSTEP * Q * ES);
            lstep = (uint32_t)((size_t)ld * ES);
            lds0 = (uint32_t)(rg0 * Q) * ROWB;
        }
    }

    // issue the loads of units [U0, U1) of stage s
    template <int U0 = 0, int U1 = UNITS>
    __device__ __forceinline__ void load(int s, uint32_t (&w)[WORDS]) const {
        // the descriptor is uniform; readfirstlane keeps the compiler from treating
        // it as divergent (which would wrap every load in a waterfall loop)
        const uint32_t o = (uint32_t)__builtin_amdgcn_readfirstlane(s) * sstep;
        const uint64_t bp = reinterpret_cast<uint64_t>(base + o);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)bp);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(bp >> 32));
        const uint32_t nrec = __builtin_amdgcn_readfirstlane(o < ext ? ext - o : 0u);
        const rsrc_t r = make_rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo), nrec);
#pragma unroll
        for (int u = U0; u < U1; u++)
#pragma unroll
            for (int l = 0; l < LOADS; l++)
                ld_raw<LB>(r, voff0 + (uint32_t)__builtin_amdgcn_readfirstlane(u * ustep + l * lstep),
                           &w[(u * LOADS + l) * LW]);
    }

    // convert units [U0, U1) of stage s from w and store them to the LDS buffer at buf
    // (MASK: zero K-major k past the range, which only a split's last stage has)
    template <int U0, int U1, bool MASK = true>
    __device__ __forceinline__ void store(int s, const uint32_t (&w)[WORDS], unsigned char *buf) const {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        if constexpr (!RMAJ) {
            const int nv = kspan - s * TK - kc0 * 8;   // valid k in this thread's units (>= 8 but in the last stage)
#pragma unroll
            for (int u = U0; u < U1; u++) {
                const uint32_t *x = &w[u * LOADS * LW];
                uint32_t q[4];
                if constexpr (DT == 0) {
#pragma unroll
                    for (int e = 0; e < 4; e++) q[e] = pk_bf16(__uint_as_float(x[2 * e]), __uint_as_float(x[2 * e + 1]));
                } else if constexpr (DT == 2) {
#pragma unroll
                    for (int e = 0; e < 4; e++) q[e] = x[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; e++) q[e] = pk_bf16(u8f(x[e >> 1], 2 * (e & 1)), u8f(x[e >> 1], 2 * (e & 1) + 1));
                }
                if constexpr (MASK) {
#pragma unroll
                    for (int e = 0; e < 4; e++) q[e] = (2 * e + 1 < nv) ? q[e] : (2 * e < nv ? q[e] & 0xffffu : 0u);
                }
                *reinterpret_cast<u32x4 *>(buf + lds0 + u * RSTEP * ROWB) = u32x4{q[0], q[1], q[2], q[3]};
            }
        } else {
            if (!active) return;   // uniform per wave
#pragma unroll
            for (int u = U0; u < U1; u++) {
                const uint32_t *x = &w[u * LOADS * LW];   // x[l * LW + ...]: k = 8 kc0 + l
#pragma unroll
                for (int e = 0; e < Q; e++) {
                    uint32_t q[4];
#pragma unroll
                    for (int h = 0; h < 4; h++) {
                        const int l0 = 2 * h, l1 = 2 * h + 1;
                        if constexpr (DT == 0) {
                            q[h] = pk_bf16(__uint_as_float(x[l0 * LW + e]), __uint_as_float(x[l1 * LW + e]));
                        } else if constexpr (DT == 2) {
                            // element e of load l: half (e & 1) of dword e >> 1
                            const uint32_t a = x[l0 * LW + (e >> 1)], b = x[l1 * LW + (e >> 1)];
                            q[h] = (e & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
                        } else {
                            q[h] = pk_bf16(u8f(x[l0], e), u8f(x[l1], e));
                        }
                    }
                    // row rg Q + e; rows RSTEP Q u further keep the position
                    const int r = (int)(lds0 / ROWB) + e;
                    *reinterpret_cast<u32x4 *>(buf + lds0 + e * ROWB + u * RSTEP * Q * ROWB +
                                               (((uint32_t)kc0 ^ lds_swz(r)) << 4)) = u32x4{q[0], q[1], q[2], q[3]};
                }
            }
        }
    }
};

struct BigArgs {
    GemmArgs g;
    int m_tiles, n_tiles, kps, total;
};

template <int ADT, bool ARM, int BDT, bool BRM, int NT>
__global__ __launch_bounds__(NT, 1) void k_gemm_big(BigArgs ba) {
    constexpr int WN = NT / 128;          // waves along n: 2 (128 x 128 each) or 4 (128 x 64 each)
    constexpr int WNE = TN / WN;          // columns per wave
    constexpr int JN = WNE / 32;          // 32-column accumulators per wave
    const GemmArgs &g = ba.g;
    if (gemm_gated_off(g.skip_cnt, g.skip_le)) return;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *const A0 = lds, *const A1 = lds + BUF_A;
    unsigned char *const B0 = lds + 2 * BUF_A, *const B1 = lds + 2 * BUF_A + BUF_B;

    const int work = xcd_remap(blockIdx.x, ba.total);
    const int tiles = ba.m_tiles * ba.n_tiles;
    const int z = work / tiles, t = work - z * tiles;
    const long long m0 = (long long)(t / ba.n_tiles) * TM;
    const int n0 = (t % ba.n_tiles) * TN;
    const int kb = z * ba.kps, ke = min(g.K, kb + ba.kps);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;             // this wave's 128 x WNE of the tile

    using OA = Op<ADT, ARM, NT>;
    using OB = Op<BDT, BRM, NT>;
    OA oa;
    OB ob;
    oa.init(g.A, g.lda, g.M, m0, kb, ke, tid);
    ob.init(g.B, g.ldb, g.N, n0, kb, ke, tid);

    floatx16 acc[4][JN];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < JN; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][j][r] = 0.0f;

    // Fragments of one 16-k step: rows 32 i apart keep their position, so a fragment's
    // position depends on the lane and kk only and the 32-row steps are immediate
    // offsets. Two register sets: the reads of step kk + 1 are issued before the
    // MFMAs of step kk.
    const int fr = lane & 31, fc = lane >> 5;
    const uint32_t fa0 = (uint32_t)(wm * 128 + fr) * ROWB, fb0 = (uint32_t)(wn * WNE + fr) * ROWB;
    bf16x8 fa[2][4], fb[2][JN];
    auto rd = [&](const unsigned char *a, const unsigned char *b, int kk, int set) __attribute__((always_inline)) {
        const uint32_t cpos = ((uint32_t)(2 * kk + fc) ^ lds_swz(fr)) << 4;
#pragma unroll
        for (int i = 0; i < 4; i++) fa[set][i] = *reinterpret_cast<const bf16x8 *>(a + fa0 + cpos + i * 32 * ROWB);
#pragma unroll
        for (int j = 0; j < JN; j++) fb[set][j] = *reinterpret_cast<const bf16x8 *>(b + fb0 + cpos + j * 32 * ROWB);
    };
    auto mrow = [&](int set, int i) __attribute__((always_inline)) {   // JN MFMAs: accumulator row i
#pragma unroll
        for (int j = 0; j < JN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[set][i], fb[set][j], acc[i][j], 0, 0, 0);
    };

    uint32_t wa[OA::WORDS], wb[OB::WORDS];
    const int nk = (ke - kb + TK - 1) / TK;
    oa.load(0, wa);
    ob.load(0, wb);
    oa.template store<0, OA::UNITS>(0, wa, A0);
    ob.template store<0, OB::UNITS>(0, wb, B0);
    __syncthreads();
    // stage 1 (past the range: zeros or data that is never multiplied), loaded in the
    // loop's unit order, so that the wait analysis at the loop head sees every unit
    // loaded as many loads before its first use as in the loop itself
    auto pre = [&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        constexpr int a0 = q * OA::UNITS / 8, a1 = (q + 1) * OA::UNITS / 8;
        constexpr int b0 = q * OB::UNITS / 8, b1 = (q + 1) * OB::UNITS / 8;
        if constexpr (a0 != a1) oa.template load<a0, a1>(1, wa);
        if constexpr (b0 != b1) ob.template load<b0, b1>(1, wb);
        __builtin_amdgcn_sched_barrier(0);
    };
    pre(std::integral_constant<int, 0>{});
    pre(std::integral_constant<int, 1>{});
    pre(std::integral_constant<int, 2>{});
    pre(std::integral_constant<int, 3>{});
    pre(std::integral_constant<int, 4>{});
    pre(std::integral_constant<int, 5>{});
    pre(std::integral_constant<int, 6>{});
    pre(std::integral_constant<int, 7>{});
    rd(A0, B0, 0, 0);
    // Iteration s multiplies stage s from LDS. Between its MFMAs, each register
    // unit of stage s + 1 (loaded during iteration s - 1) is converted and stored to
    // the other LDS buffer and at once reloaded with the same unit of stage s + 2, so
    // every load has a whole iteration to arrive. One barrier. The last iteration
    // stores and loads stages past the range into the buffer and registers nobody
    // reads.
    for (int s = 0; s < nk; s++) {
        const bool odd = s & 1;
        const unsigned char *ca = odd ? A1 : A0, *cb = odd ? B1 : B0;
        unsigned char *na = odd ? A0 : A1, *nb = odd ? B0 : B1;
        // stage s + 1 ends past the split's range (uniform; only K-major operands mask)
        const bool ragged_next = (s + 2) * TK > ke - kb;
        // steps 0 and 1: four MFMA rows each; after each row, the next eighth of the
        // units of A and of B is stored and reloaded
        auto slot = [&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            mrow((q / 4) & 1, q % 4);
            constexpr int a0 = q * OA::UNITS / 8, a1 = (q + 1) * OA::UNITS / 8;
            constexpr int b0 = q * OB::UNITS / 8, b1 = (q + 1) * OB::UNITS / 8;
            if constexpr (a0 != a1) {
                if (ragged_next) oa.template store<a0, a1, true>(s + 1, wa, na);
                else oa.template store<a0, a1, false>(s + 1, wa, na);
                oa.template load<a0, a1>(s + 2, wa);
            }
            if constexpr (b0 != b1) {
                if (ragged_next) ob.template store<b0, b1, true>(s + 1, wb, nb);
                else ob.template store<b0, b1, false>(s + 1, wb, nb);
                ob.template load<b0, b1>(s + 2, wb);
            }
            // keep the reloads here: sunk to the loop end, they would be waited for at
            // the start of the next iteration
            __builtin_amdgcn_sched_barrier(0);
        };
        using std::integral_constant;
        rd(ca, cb, 1, 1);
        slot(integral_constant<int, 0>{});
        slot(integral_constant<int, 1>{});
        slot(integral_constant<int, 2>{});
        slot(integral_constant<int, 3>{});
        rd(ca, cb, 2, 0);
        slot(integral_constant<int, 4>{});
        slot(integral_constant<int, 5>{});
        slot(integral_constant<int, 6>{});
        slot(integral_constant<int, 7>{});
        rd(ca, cb, 3, 1);
#pragma unroll
        for (int i = 0; i < 4; i++) mrow(0, i);
#pragma unroll
        for (int i = 0; i < 4; i++) mrow(1, i);
        __syncthreads();
        rd(na, nb, 0, 0);
    }

    // epilogue: lane l holds column l % 32 and rows 8 (r / 4) + 4 (l / 32) + r % 4
    // of each 32 x 32 accumulator. Stores go through a descriptor that ends at row M
    // (rows past it are dropped) and columns past N get an out-of-range offset; they
    // are non-temporal, so that the streamed result does not evict the operands' rows
    // from L2.
    const bool split = ba.total > tiles;
    float *out = split ? g.C_part + (size_t)z * g.M * g.N : g.C;
    const long long ldc = split ? g.N : g.ldc;
    const long long vrows = g.M - m0 < TM ? g.M - m0 : TM;
    const rsrc_t rc = make_rsrc(out + m0 * ldc, (uint32_t)(((vrows - 1) * ldc + g.N) * 4));
    const uint32_t ldc4 = __builtin_amdgcn_readfirstlane((uint32_t)ldc * 4u);
    // this lane's first row of its wave's 128 rows; rows step by whole 4-row groups below
    const uint32_t lrow = (uint32_t)(wm * 128 + 4 * fc);
#pragma unroll
    for (int j = 0; j < JN; j++) {
        const int n = n0 + wn * WNE + j * 32 + fr;
        const float bias = (g.bias && !split && n < g.N) ? g.bias[n] : 0.0f;
        const uint32_t cb = n < g.N ? lrow * ldc4 + (uint32_t)n * 4u : ALIF_OOB;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                // uniform part of the row: i * 32 + 8 (r / 4) + r % 4 rows. It is added to the
                // VGPR offset (rows past M then fall past the descriptor's end; an SGPR offset
                // would not be range-checked)
                const uint32_t so = (uint32_t)(i * 32 + 8 * (r >> 2) + (r & 3)) * ldc4;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[i][j][r] + bias), rc,
                                                      cb + (uint32_t)__builtin_amdgcn_readfirstlane(so), 0, 2);
            }
    }
}

// fixed-order sum of split partials: C[m][n] = sum_z P[z][m][n]
__global__ void k_big_split_reduce(long long MN, int splits, const float *P, float *C, const float *bias, int N,
                                   const unsigned long long *skip_cnt, unsigned long long skip_le) {
    if (gemm_gated_off(skip_cnt, skip_le)) return;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN) return;
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += P[(size_t)z * MN + i];
    if (bias) s += bias[i % N];
    C[i] = s;
}

// 512 threads (two waves per SIMD) unless the operand pair needs more registers than
// two waves per SIMD can hold: float x float (the input gradient against float W
// among them) and a row-contiguous bfloat16 B in the weight gradient run with 256
template <int ADT, bool ARM, int BDT, bool BRM>
hipError_t go(const BigArgs &ba, hipStream_t st) {
    constexpr bool wide = !(ADT == 0 && BDT == 0) && !(ARM && BDT == 2);
    constexpr int NT = wide ? 512 : 256;
    hipLaunchKernelGGL((k_gemm_big<ADT, ARM, BDT, BRM, NT>), dim3((unsigned)ba.total), dim3(NT), LDS_BYTES, st, ba);
    return hipGetLastError();
}

size_t elem_size(int dt) { return dt == 0 ? 4 : (dt == 1 ? 1 : 2); }

bool aligned_for(int dt, const void *p, long long ld) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if (dt == 1) return a % 4 == 0 && ld % 4 == 0;
    return a % 16 == 0 && (ld * (long long)elem_size(dt)) % 16 == 0;
}

}  // namespace

bool gemm_big_ok(const GemmArgs &g) {
    if (g.M < TM || g.N < TN || g.K < TK) return false;
    const bool fwd = g.a_kc && g.b_kc && (g.b_dt == 0 || g.b_dt == 2);
    const bool dx = g.a_kc && g.a_dt == 0 && !g.b_kc && g.b_dt == 0;
    const bool dw = !g.a_kc && (g.a_dt == 0 || g.a_dt == 2) && !g.b_kc;
    if (!(fwd || dx || dw)) return false;
    if (!aligned_for(g.a_dt, g.A, g.lda) || !aligned_for(g.b_dt, g.B, g.ldb)) return false;
    if (!g.a_kc && g.lda < g.M) return false;
    if (!g.b_kc && g.ldb < g.N) return false;
    if (g.a_kc && g.lda < g.K) return false;
    if (g.b_kc && g.ldb < g.K) return false;
    if (g.splits > 1 && (g.a_kc || g.b_kc)) return false;
    // every per-tile and per-split byte extent within 31 bits
    const size_t lim = (size_t)1 << 31;
    // (the loads run up to two stages past a split's range: K spans of a split plus 4 stages)
    const size_t kspan = (size_t)(g.K + (g.splits > 1 ? g.splits : 1) - 1) / (g.splits > 1 ? g.splits : 1) + 4 * TK;
    const size_t ea = g.a_kc ? (size_t)TM * g.lda * elem_size(g.a_dt) : kspan * g.lda * elem_size(g.a_dt);
    const size_t eb = g.b_kc ? (size_t)TN * g.ldb * elem_size(g.b_dt) : kspan * g.ldb * elem_size(g.b_dt);
    // the C tile's extent, with the column offset of an out-of-range lane added on top
    const size_t ldc = (size_t)(g.splits > 1 ? g.N : g.ldc);
    const size_t ec = (size_t)TM * ldc * 4;
    return ea < lim && eb < lim && ec < lim;
}

hipError_t gemm_big_launch(const GemmArgs &g, hipStream_t st) {
    BigArgs ba;
    ba.g = g;
    const long long mt = (g.M + TM - 1) / TM;
    ba.n_tiles = (g.N + TN - 1) / TN;
    const int s = g.splits < 1 ? 1 : g.splits;
    const int k = (g.K + s - 1) / s;
    ba.kps = (k + TK - 1) / TK * TK;
    const int splits = (g.K + ba.kps - 1) / ba.kps;
    const long long total = mt * ba.n_tiles * splits;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
    ba.m_tiles = (int)mt;
    ba.total = (int)total;
    if (splits > 1) ba.g.bias = nullptr;
    hipError_t e;
    if (g.a_kc && g.b_kc && g.b_dt == 0) {
        if (g.a_dt == 0) e = go<0, false, 0, false>(ba, st);
        else if (g.a_dt == 1) e = go<1, false, 0, false>(ba, st);
        else e = go<2, false, 0, false>(ba, st);
    } else if (g.a_kc && g.b_kc) {   // B already in bfloat16
        if (g.a_dt == 0) e = go<0, false, 2, false>(ba, st);
        else if (g.a_dt == 1) e = go<1, false, 2, false>(ba, st);
        else e = go<2, false, 2, false>(ba, st);
    } else if (g.a_kc) {
        e = go<0, false, 0, true>(ba, st);
    } else if (g.a_dt == 2) {   // the weight gradient from a bfloat16 input-current gradient
        if (g.b_dt == 1) e = go<2, true, 1, true>(ba, st);
        else if (g.b_dt == 2) e = go<2, true, 2, true>(ba, st);
        else e = go<2, true, 0, true>(ba, st);
    } else {
        if (g.b_dt == 0) e = go<0, true, 0, true>(ba, st);
        else if (g.b_dt == 1) e = go<0, true, 1, true>(ba, st);
        else e = go<0, true, 2, true>(ba, st);
    }
    if (e != hipSuccess || splits == 1) return e;
    const long long MN = g.M * (long long)g.N;
    hipLaunchKernelGGL(k_big_split_reduce, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, MN, splits,
                       g.C_part, g.C, g.bias, g.N, g.skip_cnt, g.skip_le);
    return hipGetLastError();
}

}  // namespace alif
