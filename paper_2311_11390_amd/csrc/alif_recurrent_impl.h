// Recurrent ALIF layer in one launch: Eq. 3 with the recurrent current
// W_rec S[t - D] (D >= T_R, so a block's recurrent input comes from finished
// blocks only; Prop. 3 keeps one spike per neuron per block).
//
// One workgroup per batch element holds the whole layer: NG groups of 64
// neurons (lane = neuron) x SEG segment-waves, exactly the per-block arithmetic
// of the block forward (seg_scan / seg_horner / seg_membrane, the same FP64
// carry), so only the segmentation of a block can differ from the per-block
// launches. The blocks of the layer run one after another inside the kernel and
// meet at the workgroup barriers the block integrate already has:
//
//   1. x = feed-forward current of block nb (prefetched) + the recurrent sums
//      gathered at the end of block nb - 1;
//   2. scan, Horner stitch (barrier), membrane, first-crossing candidates (barrier);
//   3. from the candidates in LDS every wave knows the spike step of every
//      neuron of block nb; the spikes whose target step t + D falls into block
//      nb + 1 and into this wave's segment are found with a ballot per neuron
//      group, and for each one, in increasing presynaptic index, the lane adds
//      W_rec[i][j] (one 256-byte row of W_rec^T, L2-resident) to the target step.
//      Older source blocks (D > T_R) come from a small ring of spike steps in LDS;
//   4. stores of block nb (spikes, traces, carries, the whole current), then the
//      prefetch of block nb + DEPTH.
// Every row of the whole current is written (the same values again where the
// input-current GEMM wrote the feed-forward current in place). No store sits
// behind a branch, so the compiler's count of memory operations in flight is
// exact and the wait for a prefetched block never waits for younger stores.
//
// Stores cost the loop more than anything else (a workgroup issues them for
// every step of every neuron while one block runs), so with CHUNKED (N a
// multiple of 16 and room in LDS) they go out as 16-byte chunks: the block's
// current through a wave-private LDS tile, three chunk stores a wave instead of
// L per-lane ones, and the spikes packed from one ballot per step, one chunk
// store instead of L byte stores. Both are issued at the end of the block, after
// its barriers.
//
// Summation order: per target step the recurrent term is a sum in FP32 from zero
// over the active presynaptic neurons in increasing index, added once to the
// feed-forward current: the order of the per-block recurrent-current kernel.
#pragma once
#include "alif_blocks_impl.h"

namespace alif {

// LDS: pd [NWG][T_R] f64 | X [SEG][NWG] f32 | C [2][SEG][NWG] i32 | ring [R][NWG] u8
template <int SEG, int NG>
__host__ __device__ constexpr size_t rec_smem_fixed(int TR) {
    return (size_t)64 * NG * TR * sizeof(double) + (size_t)3 * SEG * 64 * NG * 4;
}

// LDS of the CHUNKED staging tile: [waves][L][64] floats after the 16-byte aligned fixed part
template <int SEG, int L, int NG>
__host__ __device__ constexpr size_t rec_stage_bytes() {
    return (size_t)NG * SEG * L * 64 * 4;
}
__host__ __device__ constexpr size_t rec_stage_offset(size_t fixed_and_ring) { return (fixed_and_ring + 15) & ~(size_t)15; }

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Non-temporal (streamed) access for the feed-forward current read once and the
// whole current and spikes written once, so that they pass through L2 without
// evicting the W_rec^T rows the gather reads every block (about 1% of the loop).
constexpr int REC_NT = 2;
__device__ __forceinline__ float ld_f32_nt(rsrc_t r, uint32_t byte_off) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, REC_NT));
}

template <int SEG, int L, bool EVEN, int NG, bool TRACES, bool CHUNKED>
__global__ __launch_bounds__(64 * NG * SEG) void k_recurrent_fused(RecArgs a) {
    constexpr int NWG = 64 * NG;
    constexpr int DEPTH = 2;
    constexpr int EV = 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, N = a.N, T = a.T, D = a.D, R = a.ring;
    double *pd_tab = reinterpret_cast<double *>(smem);
    float *exX = reinterpret_cast<float *>(smem + (size_t)NWG * TR * sizeof(double));
    int *exC = reinterpret_cast<int *>(exX + SEG * NWG);
    uint8_t *ring = reinterpret_cast<uint8_t *>(exC + 2 * SEG * NWG);
    // this wave's staging tile [L][64] (CHUNKED)
    float *stg = reinterpret_cast<float *>(
                     smem + rec_stage_offset(rec_smem_fixed<SEG, NG>(TR) + (size_t)R * NWG)) +
                 (size_t)(threadIdx.x >> 6) * L * 64;

    const int b = blockIdx.x;
    build_p_tables<SEG, L, NWG>(pd_tab, nullptr, 0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L, EVEN> c;
    lane_setup<SEG, L, EVEN, NG>(c, N, TR, a.dt, 0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    if (c.valid && c.w == 0 && !params_ok(a.tau_m[c.n], a.tau_a[c.n], c.dd, c.th0))
        atomicOr(a.status, 1u);
    const int pdrow = c.nl * TR;
    const int lane = threadIdx.x & 63;

    const size_t TN = (size_t)T * N;
    const int SB = spike_bytes(a.spike_dtype);
    const rsrc_t rIn = make_rsrc(a.I_ff + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rS = make_rsrc((char *)a.spikes + b * TN * SB, (uint32_t)(TN * SB));
    const rsrc_t rV = make_rsrc(a.V ? a.V + b * TN : nullptr, a.V ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rT = make_rsrc(a.TH ? a.TH + b * TN : nullptr, a.TH ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rW = make_rsrc(a.WrecT, (uint32_t)((size_t)N * N * 4));
    const size_t CN = (size_t)(a.NB + 1) * N;
    const bool ck = a.ck.v != nullptr;
    const rsrc_t rCv = make_rsrc(ck ? a.ck.v + b * CN : nullptr, ck ? (uint32_t)(CN * 4) : 0u);
    const rsrc_t rCa = make_rsrc(ck ? a.ck.a + b * CN : nullptr, ck ? (uint32_t)(CN * 4) : 0u);
    const rsrc_t rCt = make_rsrc(ck ? a.ck.ts + b * CN : nullptr, ck ? (uint32_t)CN : 0u);
    const uint32_t ck4 = (c.valid && c.w == 0) ? (uint32_t)c.n * 4u : ALIF_OOB;
    const uint32_t ck1 = (c.valid && c.w == 0) ? (uint32_t)c.n : ALIF_OOB;
    // this lane's column of W_rec^T (byte offset within a row), or out of range
    const uint32_t wcol = c.valid ? (uint32_t)c.n * 4u : ALIF_OOB;
    const uint32_t wrow = (uint32_t)N * 4u;
    const int spk_shift = SB == 1 ? 2 : (SB == 2 ? 1 : 0);

    double v0d = 0.0, a0d = 0.0;
    int cts = 0;
    const uint32_t blk4 = (uint32_t)(TR * N) * 4u;
    float buf[DEPTH][L];
#pragma unroll
    for (int i = 0; i < DEPTH; i++)
#pragma unroll
        for (int k = 0; k < L; k++) buf[i][k] = ld_f32_nt(rIn, c.off(k, (uint32_t)min((size_t)i * blk4, TN * 4)));

    // recurrent sums of the next block at this lane's steps; hit: steps with a term (wave-uniform)
    float acc[L];
#pragma unroll
    for (int k = 0; k < L; k++) acc[k] = 0.0f;
    uint32_t hit = 0;
    const int qD = (D + TR - 1) / TR;   // source blocks lie qD or qD - 1 blocks back

    // Gather the recurrent input of block nt from the spikes of blocks < nt
    // (block nt - 1 from the candidate array Cp, older ones from the ring).
    auto gather = [&](int nt, const int *Cp) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < L; k++) acc[k] = 0.0f;
        hit = 0;
        for (int q = 0; q < 2; q++) {
            const int m = nt - qD + q;   // uniform
            if (m < 0 || m >= nt || (q == 1 && D % TR == 0)) continue;
            const int base = (m - nt) * TR + D - 1;   // target offset in block nt = base + t_s
#pragma unroll
            for (int g = 0; g < NG; g++) {
                const int j = g * 64 + lane;
                int tsj;
                if (m == nt - 1) {
                    tsj = ALIF_NO_SPIKE;
#pragma unroll
                    for (int s = 0; s < SEG; s++) tsj = min(tsj, Cp[s * NWG + j]);
                    tsj = tsj <= TR ? tsj : 0;
                } else {
                    tsj = ring[(m % R) * NWG + j];
                }
                const int r = base + tsj;
                // steps past T (padding of a ragged last block) get no recurrent term
                const bool mine = tsj > 0 && j < N && r >= c.t0 && r < c.t0 + c.len && nt * TR + r < T;
                uint64_t mk = __ballot(mine);
                while (mk) {   // EV active inputs at a time: their loads are in flight together
                    int kk[EV];
                    float w[EV];
#pragma unroll
                    for (int e = 0; e < EV; e++) {
                        kk[e] = -1;
                        w[e] = 0.0f;
                        if (mk) {
                            const int l = __builtin_ctzll(mk);
                            mk &= mk - 1;
                            kk[e] = __builtin_amdgcn_readlane(r, l) - c.t0;
                            w[e] = ld_f32(rW, (uint32_t)(g * 64 + l) * wrow + wcol);
                        }
                    }
#pragma unroll
                    for (int e = 0; e < EV; e++) {
#pragma unroll
                        for (int k = 0; k < L; k++) acc[k] = k == kk[e] ? acc[k] + w[e] : acc[k];
                        hit |= kk[e] >= 0 ? 1u << kk[e] : 0u;
                    }
                }
            }
        }
    };

    auto do_block = [&](float (&bi)[L], int nb) __attribute__((always_inline)) {
        const uint32_t bo = (uint32_t)nb * blk4;
        float x[L];
#pragma unroll
        for (int k = 0; k < L; k++) {
            x[k] = (hit >> k) & 1u ? bi[k] + acc[k] : bi[k];   // uniform: a row with a recurrent term
            if constexpr (CHUNKED) stg[k * 64 + lane] = x[k];
            else st_f32(rI, c.off(k, bo), x[k]);
        }
        const float cv = (float)v0d, ca = (float)a0d;
        const int mpre = cts > 0 ? cts - 1 : 0;
        const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
        float uu[L];
        seg_scan(c, x, mpre, uu);
        float E = 0.0f, uTR;
        if constexpr (SEG > 1) {
            exX[c.w * NWG + c.nl] = uu[L - 1];
            __syncthreads();
            seg_horner<SEG, L, EVEN, NWG>(c, exX, E, uTR);
        } else {
            uTR = uu[L - 1];
        }
        float vt[L], th[L];
        const int cand = seg_membrane(c, cv, E, a1, uu, vt, th);
        int *Cp = exC + (nb & 1) * SEG * NWG;
        Cp[c.w * NWG + c.nl] = cand;
        __syncthreads();
        int ts = ALIF_NO_SPIKE;
#pragma unroll
        for (int s = 0; s < SEG; s++) ts = min(ts, Cp[s * NWG + c.nl]);
        if (nb + 1 < a.NB) gather(nb + 1, Cp);   // uniform

        // outputs of block nb (reset after t_s, Eqs. 2 and 5) and its carry-in
        {
            const uint32_t e = (uint32_t)(nb * N);
            st_f32(rCv, ck4 + e * 4u, cv);
            st_f32(rCa, ck4 + e * 4u, ca);
            st_u8(rCt, ck1 + e, (uint8_t)cts);
        }
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int t = c.t0 + k + 1;
            const uint32_t o4 = c.off(k, bo);
            if constexpr (!CHUNKED) st_spike(rS, a.spike_dtype, o4 >> spk_shift | (o4 & ALIF_OOB), t == ts);
            if constexpr (TRACES) {
                const bool after = t > ts;
                st_f32(rV, o4, after ? 0.0f : vt[k]);
                // p^(t - 1 - t_s) when after (clamped into the row for the steps that are not)
                const float pa = (float)pd_tab[pdrow + min(TR - 1, max(0, t - 1 - ts))];
                st_f32(rT, o4, after ? fmaf(c.dd, pa, th[k]) : th[k]);
            }
        }
        const bool spk = ts <= TR;
        const double e1 = cts == TR ? c.pTm1 : 0.0;
        const double e2 = pd_tab[pdrow + max(0, TR - 1 - min(ts, TR))];
        const double extra = e1 + ((spk && ts < TR) ? e2 : 0.0);
        v0d = spk ? 0.0 : fma(c.betaT, v0d, (double)uTR);
        a0d = fma(c.pT, a0d, extra);
        cts = spk ? ts : 0;
        if (R > 0 && c.w == 0) ring[(nb % R) * NWG + c.nl] = (uint8_t)(spk ? ts : 0);
        if constexpr (CHUNKED) {
            const int nw0 = c.n - lane;                     // first neuron of this wave's group
            const int row0 = nb * TR + c.t0;                // first step of this wave's segment
            // spikes: a ballot per step; 16-byte chunks of NPC = 16 / SB neurons, 4 SB per step row
            uint64_t m[L];
#pragma unroll
            for (int k = 0; k < L; k++) m[k] = __ballot(c.t0 + k + 1 == ts);
            const int CPR = 4 * SB, NPC = 16 / SB;
            // a fixed number of store instructions (the f32 count; chunks past CPR L are dropped)
#pragma unroll
            for (int ci0 = 0; ci0 < 16 * L; ci0 += 64) {
                const int ci = ci0 + lane, k = ci / CPR, q = ci - k * CPR;
                uint64_t mk = 0;
#pragma unroll
                for (int kk = 0; kk < L; kk++) mk = k == kk ? m[kk] : mk;
                const uint32_t bits = (uint32_t)(mk >> (q * NPC));
                u32x4_t v;
                if (SB == 1) {   // bytes 0 / 1: spread each nibble to four bytes
                    v.x = ((bits & 15u) * 0x204081u) & 0x01010101u;
                    v.y = (((bits >> 4) & 15u) * 0x204081u) & 0x01010101u;
                    v.z = (((bits >> 8) & 15u) * 0x204081u) & 0x01010101u;
                    v.w = (((bits >> 12) & 15u) * 0x204081u) & 0x01010101u;
                } else if (SB == 2) {   // bfloat16 1.0 = 0x3F80
                    v.x = (bits & 1u ? 0x3F80u : 0u) | (bits & 2u ? 0x3F800000u : 0u);
                    v.y = (bits & 4u ? 0x3F80u : 0u) | (bits & 8u ? 0x3F800000u : 0u);
                    v.z = (bits & 16u ? 0x3F80u : 0u) | (bits & 32u ? 0x3F800000u : 0u);
                    v.w = (bits & 64u ? 0x3F80u : 0u) | (bits & 128u ? 0x3F800000u : 0u);
                } else {
                    v.x = bits & 1u ? 0x3F800000u : 0u;
                    v.y = bits & 2u ? 0x3F800000u : 0u;
                    v.z = bits & 4u ? 0x3F800000u : 0u;
                    v.w = bits & 8u ? 0x3F800000u : 0u;
                }
                const bool ok = ci < CPR * L && k < c.len && nw0 + q * NPC < N;
                const uint32_t off = ok ? (uint32_t)(((size_t)(row0 + k) * N + nw0 + q * NPC) * SB) : ALIF_OOB;
                __builtin_amdgcn_raw_buffer_store_b128(v, rS, off, 0, REC_NT);
            }
            // the whole current of the block from the staging tile: 16 chunks of 4 neurons per step row
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int ci0 = 0; ci0 < 16 * L; ci0 += 64) {
                const int ci = ci0 + lane, k = ci >> 4, q = ci & 15;
                const bool ok = ci < 16 * L && k < c.len && nw0 + 4 * q < N;
                const u32x4_t v = *reinterpret_cast<const u32x4_t *>(&stg[(ok ? k : 0) * 64 + 4 * q]);
                const uint32_t off = ok ? (uint32_t)(((size_t)(row0 + k) * N + nw0 + 4 * q) * 4) : ALIF_OOB;
                __builtin_amdgcn_raw_buffer_store_b128(v, rI, off, 0, REC_NT);
            }
            __builtin_amdgcn_wave_barrier();
        }
        const uint32_t nxt = (uint32_t)min((size_t)(nb + DEPTH) * blk4, TN * 4);
#pragma unroll
        for (int k = 0; k < L; k++) bi[k] = ld_f32_nt(rIn, c.off(k, nxt));
    };

    wait_vmem_all();
    int nb0 = 0;
    for (; nb0 + DEPTH <= a.NB; nb0 += DEPTH) {
#pragma unroll
        for (int i = 0; i < DEPTH; i++) do_block(buf[i], nb0 + i);
    }
#pragma unroll
    for (int i = 0; i < DEPTH; i++)
        if (nb0 + i < a.NB) do_block(buf[i], nb0 + i);   // uniform
    {   // the final carry
        const uint32_t e = (uint32_t)(a.NB * N);
        st_f32(rCv, ck4 + e * 4u, (float)v0d);
        st_f32(rCa, ck4 + e * 4u, (float)a0d);
        st_u8(rCt, ck1 + e, (uint8_t)cts);
    }
}

template <int SEG, int L, int NG>
hipError_t recurrent_fused_launch(const RecArgs &a, hipStream_t st) {
    if (a.B == 0) return hipSuccess;
    const size_t base = rec_smem_fixed<SEG, NG>(a.TR) + (size_t)a.ring * 64 * NG;
    const size_t smc = rec_stage_offset(base) + rec_stage_bytes<SEG, L, NG>();
    const bool tr = a.V || a.TH;
    // chunked stores: whole 16-neuron chunks in every row and room for the staging tile
    const bool chunked = !tr && a.N % 16 == 0 && smc <= (size_t)160 * 1024;
    const size_t sm = chunked ? smc : base;
    const bool even = a.TR == SEG * L;
#define ALIF_LR(EV, TRC, CH) \
    hipLaunchKernelGGL((k_recurrent_fused<SEG, L, EV, NG, TRC, CH>), dim3(a.B), dim3(64 * NG * SEG), sm, st, a)
    if (even) {
        if (tr) ALIF_LR(true, true, false); else if (chunked) ALIF_LR(true, false, true); else ALIF_LR(true, false, false);
    } else {
        if (tr) ALIF_LR(false, true, false); else if (chunked) ALIF_LR(false, false, true); else ALIF_LR(false, false, false);
    }
#undef ALIF_LR
    return hipGetLastError();
}

#define ALIF_INSTANTIATE_REC(S, L, NG) \
    template hipError_t recurrent_fused_launch<S, L, NG>(const RecArgs &, hipStream_t);

}  // namespace alif
