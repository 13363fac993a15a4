// Block-wise ALIF kernels for gfx950: forward (integrate + first crossing +
// persistent block-boundary carry) and surrogate-gradient backward.
//
// Method (paper Section 3): time is cut into blocks of T_R steps. Inside a block a
// neuron fires at most once, so with the reset ignored the membrane is a linear
// filter of the (refractory-masked) input (Prop. 1, Eq. 6):
//   V~[t] = beta^t V0 + (1 - beta) sum_{j<=t} beta^(t-j) Im[j],   t = 1..T_R,
// the threshold inside the block is theta0 + d p^(t-1) a1 (Prop. 5, written with
// a1 = a[1] of the block so that no 1/p appears), and the block's only real
// spike is the first crossing V~[t] > theta[t] (Eqs. 7-9, Prop. 2: phi marks the
// first faulty spike; here it is found directly as a min-reduce). Across blocks
// only (V0, a, t_s) are carried (Props. 3-5): the next block's first t_s - 1
// steps are masked, V0 = 0 after a spike, and a follows Eq. 5.
//
// GPU mapping. The T_R steps of a block are split into SEG segments of L
// steps. A wavefront owns one segment of 64 consecutive neurons (lane = neuron),
// so every load and store instruction of the hot loop moves one contiguous
// 64-neuron row of a [T][N] tensor (256 bytes of float, 64 bytes of uint8
// spikes). A workgroup holds the SEG segment-waves of NG neuron groups; the
// segments of a block are stitched together in LDS: each wave publishes its
// segment's partial sum, then every wave combines the partial sums in order
// (Horner) to get the membrane at its segment start and at the block end; the
// block's spike step is the minimum of the segment candidates. Each wave is
// persistent over all T / T_R blocks; the carry (V0 and a in FP64) is kept,
// identically, by every wave of a neuron, and input loads run DEPTH blocks
// ahead (more blocks for short blocks, see fwd_depth / bwd_depth). The loop body has no data-dependent branches around memory
// operations; blocks that follow a spike take a wave-uniform branch to the
// masked / reset arithmetic.
//
// Precision. Inputs and per-step arithmetic are FP32. Decay powers beta^k, p^k
// are evaluated in FP64 (exp(-k DT / tau)) and rounded once. The block-boundary
// carry is FP64: the no-spike membrane is V0 <- beta^T_R V0 + U[T_R] and the
// adaptation a <- p^T_R a + (spike term), so rounding does not accumulate over
// the T / T_R boundaries.
#pragma once
#include "alif_common.h"
#include "alif_kernels.h"

namespace alif {

#define ALIF_NO_SPIKE 0x7fff  // "no crossing" marker for the per-block spike step

// workgroup geometry: NG groups of 64 neurons x SEG segment-waves
template <int SEG>
struct Geo {
    static constexpr int NG = SEG >= 4 ? 1 : 4 / SEG;
    static constexpr int WAVES = NG * SEG;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int NWG = 64 * NG;  // neurons per workgroup
};

// row length of the padded FP32 p^e table (e in [-T_R, T_R + L))
__host__ __device__ constexpr int ptab_row(int TR, int L) { return 2 * TR + L; }

template <int SEG>
struct Exch {  // LDS exchange arrays, each [SEG][NWG]
    float *X;
    int *C;
    float *M, *R, *RA, *VL;
    // floats in one copy of the arrays; the backward keeps two copies (block parity)
    static constexpr int SIZE = 6 * SEG * Geo<SEG>::NWG;
};

template <int SEG>
__device__ __forceinline__ Exch<SEG> exch_at(unsigned char *base) {
    constexpr int SZ = SEG * Geo<SEG>::NWG;
    float *f = reinterpret_cast<float *>(base);
    return Exch<SEG>{f, reinterpret_cast<int *>(f + SZ), f + 2 * SZ, f + 3 * SZ, f + 4 * SZ, f + 5 * SZ};
}

// LDS layouts. Forward: pd [NWG][TR] f64 | pfp [NWG][RL] f32 | one or two copies of the exchange arrays.
// Backward (no carry, so no pd): pfp | two copies of the exchange arrays.
// whether the forward runs as a two-stage pipeline (see k_blocks_fwd)
template <int SEG>
__host__ __device__ constexpr bool fwd_pipelined() { return SEG == 4 || SEG == 8; }

template <int SEG, int L>
size_t fwd_smem_bytes(int TR) {   // two exchange copies when the forward is pipelined
    constexpr int NWG = Geo<SEG>::NWG;
    const size_t ex = SEG > 1 ? (size_t)(fwd_pipelined<SEG>() ? 2 : 1) * Exch<SEG>::SIZE * sizeof(float) : 0;
    return (size_t)NWG * TR * sizeof(double) + (size_t)NWG * ptab_row(TR, L) * sizeof(float) + ex;
}
template <int SEG, int L>
size_t bwd_smem_bytes(int TR) {
    constexpr int NWG = Geo<SEG>::NWG;
    const size_t ex = SEG > 1 ? (size_t)2 * Exch<SEG>::SIZE * sizeof(float) : 0;
    return (size_t)NWG * ptab_row(TR, L) * sizeof(float) + ex;
}

// Per-lane constants of the block recurrence. EVEN (T_R == SEG * L) means no
// segment has padding, so the per-step padding arrays collapse to scalars.
template <int SEG, int L, bool EVEN>
struct Lane {
    static constexpr int LP = EVEN ? 1 : L;
    int w, nl, n, t0, len;
    bool valid;
    float beta, omb, pf, th0, dd, ob;  // ob = (1 - beta) * bias
    double betaT, pT, pTm1;            // beta^T_R, p^T_R, p^(T_R - 1) in FP64
    float bsL;                         // beta^t0: decay of V0 to this segment's start
    float bL, bPart, pL, pPart;        // beta / p over a full segment and over the partial one
    int sfull;                         // segments before sfull are full, sfull is partial, later empty
    float bk[L];                       // beta^(k + 1)
    float pk[L];                       // p^(k + 1)
    float pt[L];                       // p^(t_k - 1),  t_k = t0 + k + 1
    float ptm1;                        // p^(t0 - 1)
    uint32_t off0;                     // byte offset of (t0, n) in a [T][N] float row block, or OOB
    uint32_t stepN4;                   // N * 4
    float bdec_[LP], pdec_[LP], obk_[LP], thk_[LP], PB_[LP], PP_[LP];
    uint32_t off_[LP];

    __device__ __forceinline__ float bdec(int k) const { return EVEN ? beta : bdec_[k]; }
    __device__ __forceinline__ float pdec(int k) const { return EVEN ? pf : pdec_[k]; }
    __device__ __forceinline__ float obk(int k) const { return EVEN ? ob : obk_[k]; }
    __device__ __forceinline__ float thk(int k) const { return EVEN ? th0 : thk_[k]; }
    // beta^(valid steps in [k, L)), p^(same)
    __device__ __forceinline__ float PB(int k) const { return EVEN ? bk[L - 1 - k] : PB_[k]; }
    __device__ __forceinline__ float PP(int k) const { return EVEN ? pk[L - 1 - k] : PP_[k]; }
    __device__ __forceinline__ bool kvalid(int k) const { return EVEN ? true : k < len; }
    // decay across segment s (full or last)
    __device__ __forceinline__ float bseg(int s) const { return (EVEN || s < sfull) ? bL : (s == sfull ? bPart : 1.0f); }
    __device__ __forceinline__ float pseg(int s) const { return (EVEN || s < sfull) ? pL : (s == sfull ? pPart : 1.0f); }
    __device__ __forceinline__ uint32_t off(int k, uint32_t bo) const {
        return EVEN ? off0 + (bo + (uint32_t)k * stepN4) : off_[k] + bo;
    }
};

// NG: neuron groups of 64 per workgroup (wave = segment * NG + group)
template <int SEG, int L, bool EVEN, int NG = Geo<SEG>::NG>
__device__ __forceinline__ void lane_setup(Lane<SEG, L, EVEN> &c, int N, int TR, double dt, int n0,
                                           const float *tau_m, const float *tau_a, const float *d,
                                           const float *theta0, const float *bias) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // uniform over the wave (and the constant 0 with one segment per block)
    c.w = SEG == 1 ? 0 : __builtin_amdgcn_readfirstlane(wave / NG);
    c.nl = (wave % NG) * 64 + lane;
    c.n = n0 + c.nl;
    c.valid = c.n < N;
    const int nc = c.valid ? c.n : N - 1;
    const float tm = tau_m[nc], ta = tau_a[nc];
    c.dd = d[nc];
    c.th0 = theta0[nc];
    const float b = bias ? bias[nc] : 0.0f;
    const double lb = -dt / (double)tm, lp = -dt / (double)ta;
    c.beta = (float)exp(lb);
    c.omb = (float)(-expm1(lb));
    c.ob = (float)(-expm1(lb) * (double)b);
    c.pf = (float)exp(lp);
    c.betaT = exp(lb * TR);
    c.pT = exp(lp * TR);
    c.pTm1 = exp(lp * (TR - 1));
    c.t0 = c.w * L;
    c.len = max(0, min(L, TR - c.t0));
    c.bsL = (float)exp(lb * (double)c.t0);
    c.sfull = TR / L;
    const int part = TR - c.sfull * L;
    c.bL = (float)exp(lb * (double)L);
    c.pL = (float)exp(lp * (double)L);
    c.bPart = (float)exp(lb * (double)part);
    c.pPart = (float)exp(lp * (double)part);
    c.stepN4 = (uint32_t)N * 4u;
    c.off0 = c.valid ? (uint32_t)(c.t0 * N + c.n) * 4u : ALIF_OOB;
#pragma unroll
    for (int k = 0; k < L; k++) {
        c.bk[k] = (float)exp(lb * (double)(k + 1));
        c.pk[k] = (float)exp(lp * (double)(k + 1));
        c.pt[k] = (float)exp(lp * (double)(c.t0 + k));
    }
    if constexpr (!EVEN) {
#pragma unroll
        for (int k = 0; k < L; k++) {
            const bool v = k < c.len;
            c.bdec_[k] = v ? c.beta : 1.0f;
            c.pdec_[k] = v ? c.pf : 1.0f;
            c.obk_[k] = v ? c.ob : 0.0f;
            c.thk_[k] = v ? c.th0 : __int_as_float(0x7f800000);
            const int nv = max(0, c.len - k);
            c.PB_[k] = (float)exp(lb * (double)nv);
            c.PP_[k] = (float)exp(lp * (double)nv);
            c.off_[k] = (c.valid && v) ? (uint32_t)((c.t0 + k) * N + c.n) * 4u : ALIF_OOB;
        }
    }
    c.ptm1 = (float)exp(lp * (double)max(0, c.t0 - 1));
}

// Tables for data-dependent exponents: pd[j][k] = p^k (FP64, k < T_R) for the
// carry; pfp[j][T_R + e] = p^e (FP32, e >= 0; 0 for e < 0) for post-spike values.
template <int SEG, int L, int NWG = Geo<SEG>::NWG>
__device__ __forceinline__ void build_p_tables(double *pd, float *pfp, int n0, int N, int TR,
                                               double dt, const float *tau_a) {
    const int RL = ptab_row(TR, L);
    if (pd) {
        for (int idx = threadIdx.x; idx < NWG * TR; idx += blockDim.x) {
            const int jj = idx / TR, k = idx - jj * TR;
            pd[idx] = exp(-dt / (double)tau_a[min(n0 + jj, N - 1)] * (double)k);
        }
    }
    if (pfp) {
        for (int idx = threadIdx.x; idx < NWG * RL; idx += blockDim.x) {
            const int jj = idx / RL, e = idx - jj * RL - TR;
            pfp[idx] = e < 0 ? 0.0f : (float)exp(-dt / (double)tau_a[min(n0 + jj, N - 1)] * (double)e);
        }
    }
    __syncthreads();
}

// Local part of the no-reset membrane over this lane's segment (Prop. 1): the
// input decayed from the segment start, uu[k] = sum over the valid, unmasked
// steps j <= k of beta^(k - j) (1 - beta) (I[t_j] + b), where the first
// mpre steps of the block are masked (the refractory steps, Prop. 3).
template <int SEG, int L, bool EVEN>
__device__ __forceinline__ void seg_scan(const Lane<SEG, L, EVEN> &c, const float (&x)[L], int mpre,
                                         float (&uu)[L]) {
    float u = 0.0f;
    if (__any(mpre > 0)) {
        const int kmin = mpre - c.t0;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const float in = k >= kmin ? fmaf(c.omb, x[k], c.obk(k)) : 0.0f;
            u = fmaf(c.bdec(k), u, in);
            uu[k] = u;
        }
    } else {
#pragma unroll
        for (int k = 0; k < L; k++) {
            u = fmaf(c.bdec(k), u, fmaf(c.omb, x[k], c.obk(k)));
            uu[k] = u;
        }
    }
}

// From the segment ends X[s] of one block (each lane's own neuron): the input
// part of the membrane at this lane's segment start (E) and at the block end (U),
// combined in segment order (Horner).
template <int SEG, int L, bool EVEN, int NWG = Geo<SEG>::NWG>
__device__ __forceinline__ void seg_horner(const Lane<SEG, L, EVEN> &c, const float *X, float &E, float &U) {
    float e = 0.0f, u = 0.0f;
#pragma unroll
    for (int s = 0; s < SEG; s++) {
        const float xs = X[s * NWG + c.nl];
        e = (s == c.w) ? u : e;
        u = fmaf(c.bseg(s), u, xs);
    }
    E = e;
    U = u;
}

// The no-reset membrane V~[t_k] = beta^(t_k) V0 + U[t_k] (Prop. 1) and the
// threshold theta0 + d p^(t_k - 1) a1 (Prop. 5) over this lane's steps, and the
// first step where V~ > theta (Eq. 7, strict; ALIF_NO_SPIKE if none).
template <int SEG, int L, bool EVEN>
__device__ __forceinline__ int seg_membrane(const Lane<SEG, L, EVEN> &c, float cv, float E, float a1,
                                            const float (&uu)[L], float (&vt)[L], float (&th)[L]) {
    const float C = fmaf(c.bsL, cv, E);                              // V~ at the segment start
    const float da1 = c.dd * a1;
    int cand = ALIF_NO_SPIKE;
#pragma unroll
    for (int k = L - 1; k >= 0; k--) {
        vt[k] = fmaf(c.bk[k], C, uu[k]);
        th[k] = fmaf(c.pt[k], da1, c.thk(k));
        cand = vt[k] > th[k] ? c.t0 + k + 1 : cand;
    }
    return cand;
}

// One block of the forward, for every segment-wave of the workgroup:
//   x[k]  input current at t_k, a1 = a[1] of the block, cv = V0 (float),
//   mpre  = masked leading steps (t_s of the previous block - 1).
// Returns the block's spike step t_s (ALIF_NO_SPIKE if none; the minimum of the
// segments' candidates, Eqs. 8-9 / Prop. 2), the no-reset membrane vt[k], the
// threshold th[k] (valid up to t_s), and U[T_R] (the input part of the membrane
// at the block end). Two workgroup barriers if SEG > 1. The backward recomputes
// blocks with the same helpers, so its V~ and theta are the forward's.
template <int SEG, int L, bool EVEN>
__device__ __forceinline__ int block_integrate(const Lane<SEG, L, EVEN> &c, const Exch<SEG> &ex,
                                               const float (&x)[L], float cv, float a1, int mpre,
                                               float (&vt)[L], float (&th)[L], float &uTR) {
    constexpr int NWG = Geo<SEG>::NWG;
    float uu[L];
    seg_scan(c, x, mpre, uu);
    float E = 0.0f;
    if constexpr (SEG > 1) {
        ex.X[c.w * NWG + c.nl] = uu[L - 1];
        __syncthreads();
        seg_horner(c, ex.X, E, uTR);
    } else {
        uTR = uu[L - 1];
    }
    const int cand = seg_membrane(c, cv, E, a1, uu, vt, th);
    if constexpr (SEG > 1) {
        ex.C[c.w * NWG + c.nl] = cand;
        __syncthreads();
        int ts = ALIF_NO_SPIKE;
#pragma unroll
        for (int s = 0; s < SEG; s++) ts = min(ts, ex.C[s * NWG + c.nl]);
        return ts;
    } else {
        return cand;
    }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
template <int SEG, int L, bool EVEN, int DEPTH, bool TRACES, int SDT>
__global__ __launch_bounds__(Geo<SEG>::THREADS) void k_blocks_fwd(FwdArgs a) {
    constexpr int NWG = Geo<SEG>::NWG;
    constexpr uint32_t SB = SDT == 0 ? 1u : (SDT == 1 ? 2u : 4u);
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, N = a.N, T = a.T, RL = ptab_row(TR, L);
    double *pd_tab = reinterpret_cast<double *>(smem);
    float *pf_tab = reinterpret_cast<float *>(smem + (size_t)NWG * TR * sizeof(double));
    const Exch<SEG> ex = exch_at<SEG>(reinterpret_cast<unsigned char *>(pf_tab + (size_t)NWG * RL));

    const int work = xcd_remap(blockIdx.x, gridDim.x);
    const int b = work / a.n_groups, g = work - b * a.n_groups;
    const int n0 = g * NWG;
    build_p_tables<SEG, L>(pd_tab, pf_tab, n0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L, EVEN> c;
    lane_setup(c, N, TR, a.dt, n0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    if (c.valid && c.w == 0 && !params_ok(a.tau_m[c.n], a.tau_a[c.n], c.dd, c.th0))
        atomicOr(a.status, 1u);
    const int pdrow = c.nl * TR;
    const int pfrow = c.nl * RL + TR + c.t0;

    const size_t TN = (size_t)T * N;
    const size_t bsi = a.bs_i ? a.bs_i : TN, bss = a.bs_s ? a.bs_s : TN;
    const rsrc_t rI = make_rsrc(a.I + b * bsi, (uint32_t)(TN * 4));
    const rsrc_t rS = make_rsrc((const char *)a.spikes + b * bss * SB, (uint32_t)(TN * SB));
    const rsrc_t rV = make_rsrc(a.V ? a.V + b * bsi : nullptr, a.V ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rT = make_rsrc(a.TH ? a.TH + b * bsi : nullptr, a.TH ? (uint32_t)(TN * 4) : 0u);
    // carry-in of every block, then the final carry; a sub-range run writes its
    // entries at block ck_off of arrays with ck_nb blocks
    const size_t CN = (size_t)((a.ck_nb ? a.ck_nb : a.NB) + 1) * N, CE = (size_t)(a.NB + 1) * N;
    const size_t CO = b * CN + (size_t)a.ck_off * N;
    const bool ck = a.ck.v != nullptr;
    const rsrc_t rCv = make_rsrc(ck ? a.ck.v + CO : nullptr, ck ? (uint32_t)(CE * 4) : 0u);
    const rsrc_t rCa = make_rsrc(ck ? a.ck.a + CO : nullptr, ck ? (uint32_t)(CE * 4) : 0u);
    const rsrc_t rCt = make_rsrc(ck ? a.ck.ts + CO : nullptr, ck ? (uint32_t)CE : 0u);
    // checkpoint offsets (bytes); only the segment-0 wave stores
    const uint32_t ck4 = (c.valid && c.w == 0) ? (uint32_t)c.n * 4u : ALIF_OOB;
    const uint32_t ck1 = (c.valid && c.w == 0) ? (uint32_t)c.n : ALIF_OOB;

    // carry-in of block 0
    double v0d = 0.0, a0d = 0.0;
    int cts = 0;
    if (a.init_v && c.valid) {
        const size_t i = (size_t)b * N + c.n;
        v0d = a.init_v[i];
        a0d = a.init_a[i];
        cts = a.init_ts[i];
        if (cts < 0 || cts > TR) { if (c.w == 0) atomicOr(a.status, 1u); cts = 0; }
    }

    const uint32_t blk4 = (uint32_t)(TR * N) * 4u;    // bytes per block in a float [T][N] row
    float buf[DEPTH][L];
#pragma unroll
    for (int i = 0; i < DEPTH; i++)
#pragma unroll
        for (int k = 0; k < L; k++) buf[i][k] = ld_f32(rI, c.off(k, (uint32_t)min((size_t)i * blk4, TN * 4)));

    // The block's outputs (spikes and corrected traces: reset after t_s, Eqs. 2
    // and 5) and the carry to the next block (Props. 4-5, FP64).
    auto finish_block = [&](int nb, int ts, const float (&vt)[L], const float (&th)[L], float uTR)
        __attribute__((always_inline)) {
        const bool spk = ts <= TR;
        const uint32_t bo = (uint32_t)nb * blk4;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int t = c.t0 + k + 1;
            const uint32_t o4 = c.off(k, bo);
            const bool sk = t == ts;
            if constexpr (SDT == 0) st_u8(rS, o4 >> 2 | (o4 & ALIF_OOB), sk ? 1 : 0);
            else if constexpr (SDT == 1) st_u16(rS, o4 >> 1 | (o4 & ALIF_OOB), sk ? (uint16_t)0x3F80 : (uint16_t)0);
            else st_f32(rS, o4, sk ? 1.0f : 0.0f);
            if constexpr (TRACES) {
                const bool after = t > ts;
                st_f32(rV, o4, after ? 0.0f : vt[k]);
                const float pa = pf_tab[pfrow - min(ts, TR) + k];
                st_f32(rT, o4, after ? fmaf(c.dd, pa, th[k]) : th[k]);
            }
        }
        const double e1 = cts == TR ? c.pTm1 : 0.0;
        const double e2 = pd_tab[pdrow + max(0, TR - 1 - min(ts, TR))];
        const double extra = e1 + ((spk && ts < TR) ? e2 : 0.0);
        v0d = spk ? 0.0 : fma(c.betaT, v0d, (double)uTR);
        a0d = fma(c.pT, a0d, extra);
        cts = spk ? ts : 0;
    };
    // carry-in of block nb, for the backward pass
    auto store_carry_in = [&](int nb, float cv, float ca) __attribute__((always_inline)) {
        const uint32_t e = (uint32_t)(nb * N);
        st_f32(rCv, ck4 + e * 4u, cv);
        st_f32(rCa, ck4 + e * 4u, ca);
        st_u8(rCt, ck1 + e, (uint8_t)cts);
    };

    // One block: integrate, find the crossing, write the outputs, carry on.
    // buf[i] holds block nb's input and receives block nb + DEPTH's.
    auto do_block = [&](float (&bi)[L], int nb) __attribute__((always_inline)) {
        float x[L];
#pragma unroll
        for (int k = 0; k < L; k++) x[k] = bi[k];
        const float cv = (float)v0d, ca = (float)a0d;
        const int mpre = cts > 0 ? cts - 1 : 0;
        const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
        store_carry_in(nb, cv, ca);
        float vt[L], th[L], uTR;
        const int ts = block_integrate<SEG, L, EVEN>(c, ex, x, cv, a1, mpre, vt, th, uTR);
        // prefetch block nb + DEPTH into the registers block nb has just finished
        // with (beyond the end of the row: out of range -> 0). Issued only now,
        // after the last use of x, so that the load can target bi's own
        // registers: loading earlier makes the compiler load into temporaries and
        // copy them back at the end of the block, which waits for the load.
        {
            const uint32_t nxt = (uint32_t)min((size_t)(nb + DEPTH) * blk4, TN * 4);
#pragma unroll
            for (int k = 0; k < L; k++) bi[k] = ld_f32(rI, c.off(k, nxt));
        }
        finish_block(nb, ts, vt, th, uTR);
    };

    // Pipelined form (SEG 4 or 8: every wave of a workgroup holds the same 64
    // neurons, so a vote over one wave is a vote over the workgroup). The
    // iteration for block nb integrates block nb from its scan and Horner sums,
    // done one iteration earlier, and scans block nb + 1 assuming no refractory
    // mask; both results go through LDS behind a single barrier. Once t_s of
    // block nb is known, block nb + 1 is rescanned (with a second barrier) only if
    // some neuron of the workgroup needs the mask; otherwise the assumption held
    // and the scan took exactly the unmasked path. The exchange arrays come in
    // two copies selected by block parity. Slot (i + 1) mod DEPTH holds block
    // nb + 1 and is refilled with block nb + 1 + DEPTH after its scan.
    constexpr bool PIPE = fwd_pipelined<SEG>();
    const auto par = [](int nb) { return (nb & 1) * Exch<SEG>::SIZE; };
    float uuc[L];               // scan of the block the next iteration integrates
    float Ec = 0.0f, Uc = 0.0f; // its input part at this segment's start and at the block end
    auto do_block_pipe = [&](float (&bj)[L], int nb, bool has_next) __attribute__((always_inline)) {
        constexpr int NWG_ = Geo<SEG>::NWG;
        const float cv = (float)v0d, ca = (float)a0d;
        const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
        store_carry_in(nb, cv, ca);
        float vt[L], th[L];
        const int cand = seg_membrane(c, cv, Ec, a1, uuc, vt, th);
        const float uTR = Uc;
        ex.C[par(nb) + c.w * NWG_ + c.nl] = cand;
        float uun[L];
        if (has_next) {
            seg_scan(c, bj, 0, uun);
            ex.X[par(nb + 1) + c.w * NWG_ + c.nl] = uun[L - 1];
        }
        __syncthreads();
        int ts = ALIF_NO_SPIKE;
#pragma unroll
        for (int s2 = 0; s2 < SEG; s2++) ts = min(ts, ex.C[par(nb) + s2 * NWG_ + c.nl]);
        finish_block(nb, ts, vt, th, uTR);
        if (has_next) {
            const int mpren = cts > 0 ? cts - 1 : 0;
            if (__any(mpren > 0)) {   // uniform over the workgroup
                seg_scan(c, bj, mpren, uun);
                ex.X[par(nb + 1) + c.w * NWG_ + c.nl] = uun[L - 1];
                __syncthreads();
            }
            seg_horner(c, ex.X + par(nb + 1), Ec, Uc);
#pragma unroll
            for (int k = 0; k < L; k++) uuc[k] = uun[k];
            // prefetch block nb + 1 + DEPTH into the slot block nb + 1 has left
            const uint32_t nxt = (uint32_t)min((size_t)(nb + 1 + DEPTH) * blk4, TN * 4);
#pragma unroll
            for (int k = 0; k < L; k++) bj[k] = ld_f32(rI, c.off(k, nxt));
        }
    };

    // Full groups of DEPTH blocks with no per-block guard: a guard would give the
    // loop paths from an early block straight to its latch, and the compiler's
    // wait analysis at the loop head would then assume the shortest distance to
    // every prefetch. The remaining blocks run after the loop.
    if constexpr (PIPE) {
        {   // block 0's scan and Horner sums
            seg_scan(c, buf[0], cts > 0 ? cts - 1 : 0, uuc);
            ex.X[par(0) + c.w * NWG + c.nl] = uuc[L - 1];
            __syncthreads();
            seg_horner(c, ex.X + par(0), Ec, Uc);
            const uint32_t nxt = (uint32_t)min((size_t)DEPTH * blk4, TN * 4);
#pragma unroll
            for (int k = 0; k < L; k++) buf[0][k] = ld_f32(rI, c.off(k, nxt));
        }
        wait_vmem_all();
        int nb0 = 0;
        for (; nb0 + DEPTH < a.NB; nb0 += DEPTH) {   // block nb + 1 always exists here
#pragma unroll
            for (int i = 0; i < DEPTH; i++) do_block_pipe(buf[(i + 1) % DEPTH], nb0 + i, true);
        }
#pragma unroll
        for (int i = 0; i < DEPTH; i++)
            if (nb0 + i < a.NB) do_block_pipe(buf[(i + 1) % DEPTH], nb0 + i, nb0 + i + 1 < a.NB);   // uniform
    } else {
        wait_vmem_all();
        int nb0 = 0;
        for (; nb0 + DEPTH <= a.NB; nb0 += DEPTH) {
#pragma unroll
            for (int i = 0; i < DEPTH; i++) do_block(buf[i], nb0 + i);
        }
#pragma unroll
        for (int i = 0; i < DEPTH; i++)
            if (nb0 + i < a.NB) do_block(buf[i], nb0 + i);   // uniform over the workgroup
    }
    {   // the final carry, after the carry-in of the last block
        const uint32_t e = (uint32_t)(a.NB * N);
        st_f32(rCv, ck4 + e * 4u, (float)v0d);
        st_f32(rCa, ck4 + e * 4u, (float)a0d);
        st_u8(rCt, ck1 + e, (uint8_t)cts);
    }
    if (a.fin_v && c.valid && c.w == 0) {
        const size_t i = (size_t)b * N + c.n;
        a.fin_v[i] = v0d;
        a.fin_a[i] = a0d;
        a.fin_ts[i] = cts;
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// Reverse adjoint of the detached-policy recurrence (the oracle's sequential
// surrogate gradient), one block at a time from the last to the first:
//   lamV[t]  = gV[t] + gS[t] s'(u) + beta (1 - S[t]) lamV[t+1]
//   lamTh[t] = gTh[t] - gS[t] s'(u),   lamA[t] = d lamTh[t] + p lamA[t+1]
//   gI[t] = (1 - beta) gate[t] lamV[t];  dbeta += (1 - S[t-1]) (V[t-1] - gate I[t]) lamV[t]
//   dp += a[t-1] lamA[t];  dd += a[t] lamTh[t];  dtheta0 += lamTh[t]
// Each block's V, theta, a and spike are recomputed from its saved carry with
// the forward's arithmetic. Within a block each segment-wave runs the two
// reverse recurrences over its L steps from zero, publishes the resulting
// affine map (lam_start = R + M lam_in) in LDS, and every wave composes the
// maps from the block end (Horner) to get its own incoming lambda and the
// block's lambda at step 1 (the carry to the previous block).
// The input-current gradient out of the backward: GI = 1 float, GI = 2 bfloat16
// (rounded to nearest even, the rounding the BF16 GEMMs apply to it) at half the
// byte offset; an out-of-range offset stays out of range.
template <int GI>
__device__ __forceinline__ void st_gi(rsrc_t r, uint32_t off4, float v) {
    if constexpr (GI == 1) st_f32(r, off4, v);
    else st_u16(r, (off4 >> 1) | (off4 & ALIF_OOB), __builtin_bit_cast(uint16_t, (__bf16)v));
}

template <int SEG, int L, bool EVEN, int DEPTH, bool GVT, int GI, int SG>
__global__ __launch_bounds__(Geo<SEG>::THREADS) void k_blocks_bwd(BwdArgs a) {
    constexpr int NWG = Geo<SEG>::NWG;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, N = a.N, T = a.T, RL = ptab_row(TR, L);
    float *pf_tab = reinterpret_cast<float *>(smem);
    const Exch<SEG> ex = exch_at<SEG>(reinterpret_cast<unsigned char *>(pf_tab + (size_t)NWG * RL));

    const int work = xcd_remap(blockIdx.x, gridDim.x);
    const int b = work / a.n_groups, g = work - b * a.n_groups;
    const int n0 = g * NWG;
    build_p_tables<SEG, L>(nullptr, pf_tab, n0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L, EVEN> c;
    lane_setup(c, N, TR, a.dt, n0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    const int pfrow = c.nl * RL + TR + c.t0;
    const float bias = (a.bias_k && c.valid) ? a.bias_k[c.n] : 0.0f;

    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rGS = make_rsrc(a.gS ? a.gS + b * TN : nullptr, a.gS ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGV = make_rsrc(a.gV ? a.gV + b * TN : nullptr, a.gV ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGT = make_rsrc(a.gTH ? a.gTH + b * TN : nullptr, a.gTH ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGI = GI == 2 ? make_rsrc(a.gI16 + b * TN, (uint32_t)(TN * 2))
                                : make_rsrc(a.gI ? a.gI + b * TN : nullptr, a.gI ? (uint32_t)(TN * 4) : 0u);
    const size_t CN = (size_t)(a.NB + 1) * N;   // carry-in of every block, then the final carry
    const rsrc_t rCv = make_rsrc(a.ck.v + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCa = make_rsrc(a.ck.a + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCt = make_rsrc(a.ck.ts + b * CN, (uint32_t)CN);
    const uint32_t ck4 = c.valid ? (uint32_t)c.n * 4u : ALIF_OOB;
    const uint32_t ck1 = c.valid ? (uint32_t)c.n : ALIF_OOB;
    const uint32_t blk4 = (uint32_t)(TR * N) * 4u;
    const uint32_t TN4 = (uint32_t)(TN * 4);

    struct Slot {
        float x[L], gs[L], gv[L], gt[L];
        float cv, ca;
        int cts, tsn;   // spike step of the previous block (carry-in) and of this block
    };
    Slot buf[DEPTH];
    auto load_block = [&](Slot &dst, int nb) {   // nb < 0: everything out of range
        const uint32_t bo = nb >= 0 ? (uint32_t)nb * blk4 : TN4;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const uint32_t o = c.off(k, bo);
            dst.x[k] = ld_f32(rI, o);
            dst.gs[k] = ld_f32(rGS, o);
            if constexpr (GVT) {
                dst.gv[k] = ld_f32(rGV, o);
                dst.gt[k] = ld_f32(rGT, o);
            }
        }
        const uint32_t e = nb >= 0 ? (uint32_t)(nb * N) : (uint32_t)CN;
        dst.cv = ld_f32(rCv, ck4 + e * 4u);
        dst.ca = ld_f32(rCa, ck4 + e * 4u);
        dst.cts = ld_u8(rCt, ck1 + e);
        dst.tsn = ld_u8(rCt, ck1 + (nb >= 0 ? e + (uint32_t)N : (uint32_t)CN));
    };
#pragma unroll
    for (int i = 0; i < DEPTH; i++) load_block(buf[i], a.NB - 1 - i);

    // The blocks are processed last to first, as a two-stage pipeline with one
    // workgroup barrier per block: the iteration for block nb runs the masked
    // scan of block nb - 1 (which needs only that block's input and saved
    // carry-in) and the reverse scans of block nb, publishes both through LDS,
    // waits once, then finishes block nb (lambda composition, parameter sums)
    // and block nb - 1's membrane, which the next iteration uses. The exchange
    // arrays come in two copies selected by block parity: a copy is rewritten
    // two iterations later, after a barrier that follows its last read.
    // With one segment per block there is no barrier to share, and each block's
    // membrane is computed in its own iteration instead.
    constexpr bool PIPE = SEG > 1;
    // recompute instead of store (see below): long segments, and 6-8 steps when the
    // dL/dV, dL/dtheta inputs take the registers (T_R 64: 0.79 against 1.74 ms)
    constexpr bool RECOMP = L > 8 || (GVT && L > 5);
    const auto par = [](int nb) { return (nb & 1) * Exch<SEG>::SIZE; };
    float vtn[L], thn[L];   // V~ and theta of the block the next iteration finishes
    if constexpr (PIPE) {
        const Slot &s0 = buf[0];
        const int cts0 = min(s0.cts, TR);
        float uu[L];
        seg_scan(c, s0.x, cts0 > 0 ? cts0 - 1 : 0, uu);
        float E = 0.0f, U;
        if constexpr (SEG > 1) {
            ex.X[par(a.NB - 1) + c.w * NWG + c.nl] = uu[L - 1];
            __syncthreads();
            seg_horner(c, ex.X + par(a.NB - 1), E, U);
        }
        seg_membrane(c, s0.cv, E, fmaf(c.pf, s0.ca, cts0 == TR ? 1.0f : 0.0f), uu, vtn, thn);
    }

    // lambda_V and lambda_a' at step 1 of the block after the current one. The
    // adaptation adjoint is carried without its factor d (lambda_a = d lambda_a',
    // exact by linearity, also for d = 0), so the per-step recurrence has no
    // multiply by d; d is applied once per block to its parameter-gradient sum.
    float lamV_c = 0.0f, lamA_c = 0.0f;
    double acc_b = 0.0, acc_p = 0.0, acc_d = 0.0, acc_th = 0.0, acc_bias = 0.0;

    // One block, from its saved carry-in: reverse adjoint and parameter sums for
    // block nb (slot bi), and the membrane of block nb - 1 (slot bj).
    auto do_block = [&](Slot &bi, const Slot &bj, int nb) __attribute__((always_inline)) {
        const bool has_prev = PIPE && nb >= 1;   // uniform over the workgroup
        if constexpr (!PIPE) {   // this block's membrane, now
            const int cts0 = min(bi.cts, TR);
            float uu[L];
            seg_scan(c, bi.x, cts0 > 0 ? cts0 - 1 : 0, uu);
            seg_membrane(c, bi.cv, 0.0f, fmaf(c.pf, bi.ca, cts0 == TR ? 1.0f : 0.0f), uu, vtn, thn);
        }
        // stage 1a: masked scan of block nb - 1
        float uun[L];
        float a1n = 0.0f;
        if (has_prev) {
            const int ctsn = min(bj.cts, TR);
            a1n = fmaf(c.pf, bj.ca, ctsn == TR ? 1.0f : 0.0f);
            seg_scan(c, bj.x, ctsn > 0 ? ctsn - 1 : 0, uun);
            if constexpr (SEG > 1) ex.X[par(nb - 1) + c.w * NWG + c.nl] = uun[L - 1];
        }

        // stage 1b: block nb, with V~ and theta from the previous iteration
        const Slot &cur = bi;
        const int cts = min(cur.cts, TR);
        // the block's spike step, as the forward decided it (carry-in of block nb + 1)
        const int ts = cur.tsn > 0 ? min(cur.tsn, TR) : ALIF_NO_SPIKE;
        const float cv = cur.cv, ca = cur.ca;
        const int mpre = cts > 0 ? cts - 1 : 0;
        const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
        const float (&vt)[L] = vtn;
        const float (&th)[L] = thn;
        const int tsc = min(ts, TR);
        // quiet block: no spike in this block and none at the end of the previous
        // one anywhere in the wave -> no reset, no mask, no post-spike terms
        const bool quiet = !__any(ts <= TR || mpre > 0);

        // local reverse recurrences over this segment's steps, from zero:
        //   rv: lambda_V (source dL/dV + dL/dS s'), pv: its decay across the segment,
        //   ra: lambda_a' (source lambda_theta = dL/dtheta - dL/dS s').
        // Short segments keep every step's lambdas, membrane, adaptation and gate in
        // registers for the gradient pass. Long ones (RECOMP) keep only dL/dS s' per
        // step; the gradient pass reruns the same recurrences step by step (the same
        // operations, so the same values), which frees about 6 L registers per lane.
        float Vk[L], ak[L], lt[L], rV[L], PVk[L], rA[L], gsv[L];
        bool gate[L];
        float rv = 0.0f, pv = 1.0f, ra = 0.0f;
        float VLast = vt[L - 1];   // V of this segment's last step (after a spike: 0)
        if constexpr (!RECOMP) {
            if (quiet) {
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const float gsk = cur.gs[k] * surrogate_grad<SG>(vt[k] - th[k], a.slope);
                    float src;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        lt[k] = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        lt[k] = -gsk;
                    }
                    rv = fmaf(c.bdec(k), rv, src);
                    ra = fmaf(c.pdec(k), ra, lt[k]);
                    rV[k] = rv;
                    rA[k] = ra;
                }
                pv = c.PB(0);
            } else {
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const int t = c.t0 + k + 1;
                    const bool after = t > ts;
                    const float pa = pf_tab[pfrow - tsc + k];   // p^(t - 1 - t_s)
                    Vk[k] = after ? 0.0f : vt[k];
                    ak[k] = after ? fmaf(c.pt[k], a1, pa) : c.pt[k] * a1;
                    const float thk = after ? fmaf(c.dd, pa, th[k]) : th[k];
                    gate[k] = (t > mpre) && !after;
                    const float gsk = cur.gs[k] * surrogate_grad<SG>(Vk[k] - thk, a.slope);
                    float src;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        lt[k] = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        lt[k] = -gsk;
                    }
                    const float fV = t == ts ? 0.0f : c.bdec(k);
                    rv = fmaf(fV, rv, src);
                    pv = pv * fV;
                    ra = fmaf(c.pdec(k), ra, lt[k]);
                    rV[k] = rv;
                    PVk[k] = pv;
                    rA[k] = ra;
                }
            }

            VLast = quiet ? vt[L - 1] : Vk[L - 1];
        } else {
            if (quiet) {
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const float gsk = cur.gs[k] * surrogate_grad<SG>(vt[k] - th[k], a.slope);
                    gsv[k] = gsk;
                    float src, ltk;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        ltk = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        ltk = -gsk;
                    }
                    rv = fmaf(c.bdec(k), rv, src);
                    ra = fmaf(c.pdec(k), ra, ltk);
                }
                pv = c.PB(0);
            } else {
                VLast = c.t0 + L > ts ? 0.0f : vt[L - 1];
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const int t = c.t0 + k + 1;
                    const bool after = t > ts;
                    const float pa = pf_tab[pfrow - tsc + k];   // p^(t - 1 - t_s)
                    const float Vkk = after ? 0.0f : vt[k];
                    const float thk = after ? fmaf(c.dd, pa, th[k]) : th[k];
                    const float gsk = cur.gs[k] * surrogate_grad<SG>(Vkk - thk, a.slope);
                    gsv[k] = gsk;
                    float src, ltk;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        ltk = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        ltk = -gsk;
                    }
                    const float fV = t == ts ? 0.0f : c.bdec(k);
                    rv = fmaf(fV, rv, src);
                    pv = pv * fV;
                    ra = fmaf(c.pdec(k), ra, ltk);
                }
            }

        }

        // stage 2: one barrier, then the incoming lambdas at this segment's end
        // (composing the later segments' maps lam_start = R + M lam_end from the
        // block end) and the block's lambdas at step 1
        float lVin, lAin, Vprev0, nlV, nlA;
        if constexpr (SEG > 1) {
            const int po = par(nb);
            ex.M[po + c.w * NWG + c.nl] = pv;
            ex.R[po + c.w * NWG + c.nl] = rv;
            ex.RA[po + c.w * NWG + c.nl] = ra;
            ex.VL[po + c.w * NWG + c.nl] = VLast;
            __syncthreads();
            float lv = lamV_c, la = lamA_c;
            lVin = lv;
            lAin = la;
#pragma unroll
            for (int s = SEG - 1; s >= 0; s--) {
                lVin = (s == c.w) ? lv : lVin;
                lAin = (s == c.w) ? la : lAin;
                lv = fmaf(ex.M[po + s * NWG + c.nl], lv, ex.R[po + s * NWG + c.nl]);
                la = fmaf(c.pseg(s), la, ex.RA[po + s * NWG + c.nl]);
            }
            nlV = lv;
            nlA = la;
            Vprev0 = c.w > 0 ? ex.VL[po + (c.w - 1) * NWG + c.nl] : cv;
        } else {
            lVin = lamV_c;
            lAin = lamA_c;
            nlV = fmaf(pv, lamV_c, rv);
            nlA = fmaf(c.pseg(0), lamA_c, ra);
            Vprev0 = cv;
        }

        // gradient contributions of this lane's steps:
        //   d/dbeta   += (1 - S[t-1]) (V[t-1] - gate I[t]) lambda_V[t]
        //   d/dp      += a[t-1] lambda_a[t] = d a[t-1] lambda_a'[t]
        //   d/dd      += a[t] lambda_theta[t],   d/dtheta0 += lambda_theta[t]
        //   d/dbias   += (1 - beta) gate lambda_V[t]
        float pb = 0.0f, pp = 0.0f, pdd = 0.0f, pth = 0.0f, pbias = 0.0f;
        const uint32_t bo = (uint32_t)nb * blk4;
        if constexpr (!RECOMP) {
            if (quiet) {
                // a[t] = p^(t-1) a1 throughout a quiet block, so a1 factors out of the
                // d and p sums; the bias term of I factors out of the beta sum
                const float aprev0 = c.w == 0 ? ca : c.ptm1 * a1;
                float slV = 0.0f, qd = 0.0f, qp = 0.0f, lA0 = 0.0f;
#pragma unroll
                for (int k = 0; k < L; k++) {
                    const float lV = c.kvalid(k) ? fmaf(c.PB(k), lVin, rV[k]) : 0.0f;
                    const float lA = c.kvalid(k) ? fmaf(c.PP(k), lAin, rA[k]) : 0.0f;
                    const float Vprev = (k == 0) ? Vprev0 : vt[k > 0 ? k - 1 : 0];
                    slV += lV;
                    pb = fmaf(Vprev - cur.x[k], lV, pb);
                    qd = fmaf(c.pt[k], lt[k], qd);
                    if (k == 0) lA0 = lA;
                    else qp = fmaf(c.pt[k > 0 ? k - 1 : 0], lA, qp);
                    pth += lt[k];
                    if constexpr (GI != 0) st_gi<GI>(rGI, c.off(k, bo), c.omb * lV);
                }
                pb = fmaf(-bias, slV, pb);
                pp = c.dd * fmaf(a1, qp, aprev0 * lA0);
                pdd = a1 * qd;
                pbias = c.omb * slV;
            } else {
                const float pa0 = pf_tab[pfrow - tsc - 1];     // p^(t0 - 1 - t_s)
                const float aprev0 = c.w == 0 ? ca : (c.t0 > ts ? fmaf(c.ptm1, a1, pa0) : c.ptm1 * a1);
                float sglV = 0.0f;
#pragma unroll
                for (int k = 0; k < L; k++) {
                    const float lV = c.kvalid(k) ? fmaf(PVk[k], lVin, rV[k]) : 0.0f;
                    const float lA = c.kvalid(k) ? fmaf(c.PP(k), lAin, rA[k]) : 0.0f;
                    const int t = c.t0 + k + 1;
                    const bool sprev = (t == 1) ? (cts == TR) : (t - 1 == ts);
                    const float Vprev = (k == 0) ? Vprev0 : Vk[k > 0 ? k - 1 : 0];
                    const float aprev = (k == 0) ? aprev0 : ak[k > 0 ? k - 1 : 0];
                    const float glV = gate[k] ? lV : 0.0f;
                    const float im = gate[k] ? cur.x[k] + bias : 0.0f;
                    pb = fmaf(sprev ? 0.0f : Vprev - im, lV, pb);
                    pp = fmaf(aprev, lA, pp);
                    pdd = fmaf(ak[k], lt[k], pdd);
                    pth += lt[k];
                    sglV += glV;
                    if constexpr (GI != 0) st_gi<GI>(rGI, c.off(k, bo), c.omb * glV);
                }
                pp *= c.dd;
                pbias = c.omb * sglV;
            }
        } else {   // steps last to first, rerunning the local recurrences
            if (quiet) {
                // a[t] = p^(t-1) a1 throughout a quiet block, so a1 factors out of the
                // d and p sums; the bias term of I factors out of the beta sum
                const float aprev0 = c.w == 0 ? ca : c.ptm1 * a1;
                float slV = 0.0f, qd = 0.0f, qp = 0.0f, lA0 = 0.0f, rv2 = 0.0f, ra2 = 0.0f;
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const float gsk = gsv[k];
                    float src, ltk;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        ltk = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        ltk = -gsk;
                    }
                    rv2 = fmaf(c.bdec(k), rv2, src);
                    ra2 = fmaf(c.pdec(k), ra2, ltk);
                    const float lV = c.kvalid(k) ? fmaf(c.PB(k), lVin, rv2) : 0.0f;
                    const float lA = c.kvalid(k) ? fmaf(c.PP(k), lAin, ra2) : 0.0f;
                    const float Vprev = (k == 0) ? Vprev0 : vt[k > 0 ? k - 1 : 0];
                    slV += lV;
                    pb = fmaf(Vprev - cur.x[k], lV, pb);
                    qd = fmaf(c.pt[k], ltk, qd);
                    if (k == 0) lA0 = lA;
                    else qp = fmaf(c.pt[k > 0 ? k - 1 : 0], lA, qp);
                    pth += ltk;
                    if constexpr (GI != 0) st_gi<GI>(rGI, c.off(k, bo), c.omb * lV);
                }
                pb = fmaf(-bias, slV, pb);
                pp = c.dd * fmaf(a1, qp, aprev0 * lA0);
                pdd = a1 * qd;
                pbias = c.omb * slV;
            } else {
                const float pa0 = pf_tab[pfrow - tsc - 1];     // p^(t0 - 1 - t_s)
                const float aprev0 = c.w == 0 ? ca : (c.t0 > ts ? fmaf(c.ptm1, a1, pa0) : c.ptm1 * a1);
                float sglV = 0.0f, rv2 = 0.0f, pv2 = 1.0f, ra2 = 0.0f;
                // a at step k (corrected after the spike), carried down to the next step
                float ak_c;
                {
                    const int t = c.t0 + L;
                    const float pa = pf_tab[pfrow - tsc + L - 1];
                    ak_c = t > ts ? fmaf(c.pt[L - 1], a1, pa) : c.pt[L - 1] * a1;
                }
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const int t = c.t0 + k + 1;
                    const bool after = t > ts;
                    const float gsk = gsv[k];
                    float src, ltk;
                    if constexpr (GVT) {
                        src = cur.gv[k] + gsk;
                        ltk = cur.gt[k] - gsk;
                    } else {
                        src = gsk;
                        ltk = -gsk;
                    }
                    const float fV = t == ts ? 0.0f : c.bdec(k);
                    rv2 = fmaf(fV, rv2, src);
                    pv2 = pv2 * fV;
                    ra2 = fmaf(c.pdec(k), ra2, ltk);
                    const float lV = c.kvalid(k) ? fmaf(pv2, lVin, rv2) : 0.0f;
                    const float lA = c.kvalid(k) ? fmaf(c.PP(k), lAin, ra2) : 0.0f;
                    const bool sprev = (t == 1) ? (cts == TR) : (t - 1 == ts);
                    float Vprev, aprev;
                    if (k == 0) {
                        Vprev = Vprev0;
                        aprev = aprev0;
                    } else {
                        const bool afterp = t - 1 > ts;
                        const float pap = pf_tab[pfrow - tsc + k - 1];
                        Vprev = afterp ? 0.0f : vt[k > 0 ? k - 1 : 0];
                        aprev = afterp ? fmaf(c.pt[k > 0 ? k - 1 : 0], a1, pap) : c.pt[k > 0 ? k - 1 : 0] * a1;
                    }
                    const bool gate = (t > mpre) && !after;
                    const float glV = gate ? lV : 0.0f;
                    const float im = gate ? cur.x[k] + bias : 0.0f;
                    pb = fmaf(sprev ? 0.0f : Vprev - im, lV, pb);
                    pp = fmaf(aprev, lA, pp);
                    pdd = fmaf(ak_c, ltk, pdd);
                    pth += ltk;
                    sglV += glV;
                    if constexpr (GI != 0) st_gi<GI>(rGI, c.off(k, bo), c.omb * glV);
                    ak_c = aprev;
                }
                pp *= c.dd;
                pbias = c.omb * sglV;
            }
        }
        acc_b += (double)pb;
        acc_p += (double)pp;
        acc_d += (double)pdd;
        acc_th += (double)pth;
        acc_bias += (double)pbias;
        lamV_c = nlV;
        lamA_c = nlA;

        // stage 2b: the membrane of block nb - 1, for the next iteration
        if (has_prev) {
            float E = 0.0f, U;
            if constexpr (SEG > 1) seg_horner(c, ex.X + par(nb - 1), E, U);
            seg_membrane(c, bj.cv, E, a1n, uun, vtn, thn);
        }
        // prefetch block nb - DEPTH into this slot, after the last use of cur (so
        // the loads can target the slot's own registers; see the forward)
        load_block(bi, nb - DEPTH);
    };
    // Full groups of DEPTH blocks without per-block guards, then the remainder
    // (the reason is given at the forward's loop). Slot i holds block nb, slot
    // i + 1 (mod DEPTH) block nb - 1; DEPTH >= 3 keeps a whole iteration between
    // a slot's prefetch and its first use by the masked scan.
    // Depth 2 is still correct (the masked scan then waits on a load issued one
    // block earlier); it is used only for 13-16-step segments, whose per-block work
    // covers more of the latency and whose registers cannot hold a third slot.
    static_assert(!PIPE || DEPTH >= 3 || L >= 13, "the backward pipeline reads the next block's slot one iteration early");
    wait_vmem_all();
    int r0 = 0;
    for (; r0 + DEPTH <= a.NB; r0 += DEPTH) {
#pragma unroll
        for (int i = 0; i < DEPTH; i++) do_block(buf[i], buf[(i + 1) % DEPTH], a.NB - 1 - (r0 + i));
    }
#pragma unroll
    for (int i = 0; i < DEPTH; i++)
        if (r0 + i < a.NB) do_block(buf[i], buf[(i + 1) % DEPTH], a.NB - 1 - (r0 + i));   // uniform
    // per-(b, n) sums over this neuron's segment-waves, in a fixed order
    if constexpr (SEG > 1) {
        double *red = reinterpret_cast<double *>(ex.X);   // reuse the exchange area
        __syncthreads();
        const int q = c.w * NWG + c.nl;
        double vals[5] = {acc_b, acc_p, acc_d, acc_th, acc_bias};
#pragma unroll
        for (int j = 0; j < 5; j++) {
            red[q] = vals[j];
            __syncthreads();
            if (c.w == 0) {
                double s = 0.0;
                for (int w = 0; w < SEG; w++) s += red[w * NWG + c.nl];
                vals[j] = s;
            }
            __syncthreads();
        }
        acc_b = vals[0]; acc_p = vals[1]; acc_d = vals[2]; acc_th = vals[3]; acc_bias = vals[4];
    }
    if (c.valid && c.w == 0) {
        const size_t BN = (size_t)a.B * N, i = (size_t)b * N + c.n;
        a.part[i] = acc_b;
        a.part[BN + i] = acc_p;
        a.part[2 * BN + i] = acc_d;
        a.part[3 * BN + i] = acc_th;
        a.part[4 * BN + i] = acc_bias;
    }
}

// ---------------------------------------------------------------------------
// backward, attached gradient policy
// ---------------------------------------------------------------------------
// Supplementary "Detaching gradients" sets the detached policy against one where
// the spike's own effects stay in the gradient: its reset of the next step's
// membrane, dV[t+1]/dS[t] = -(beta V[t] + (1 - beta) Im[t+1]) = -c[t] (Im: the
// gated input), and its adaptation jump, da[t+1]/dS[t] = 1. The adjoint of the
// spike then collects lamS[t] = dL/dS[t] - c[t] lamV[t+1] + lamA[t+1], and with
// s = the surrogate derivative at V[t] - theta[t]:
//   lamV[t]  = dL/dV[t] + s lamS[t] + beta (1 - S[t]) lamV[t+1]
//   lamTh[t] = dL/dtheta[t] - s lamS[t],   lamA[t] = d lamTh[t] + p lamA[t+1],
// an affine map of the pair (lamV, lamA)[t+1]:
//   (lamV, lamA)[t] = r[t] + M[t] (lamV, lamA)[t+1],
//   M[t] = [[beta (1 - S[t]) - s c[t], s], [d s c[t], p - d s]],
//   r[t] = (dL/dV + s dL/dS, d (dL/dtheta - s dL/dS)).
// The ARP gate counts steps and passes no gradient under either policy.
//
// Block form: as in the detached backward, each block is recomputed from its saved
// carry-in with the forward's helpers (so V~ and theta are the forward's FP32
// values) and the spike step is read from the next block's carry. Each
// segment-wave composes its steps' maps from zero (P = M[t0+1] ... M[t0+L],
// R the matching offset), the (P, R) pairs meet in LDS, and every wave composes
// them from the block end, starting from the lambdas at step 1 of the block after.
// The coupled recurrence can amplify rounding by orders of magnitude (the
// multi-Gaussian surrogate at T_R = 2 grows gradients by 1e9 over a few hundred
// steps), so the surrogate, the maps, the lambdas and the sums are FP64; only V,
// theta and a are the forward's FP32 values. Two barriers per block, two-block
// register prefetch. dL/dV, dL/dtheta may be absent (their buffers then read 0) and
// so may dL/dI (its stores are dropped).
template <int SEG>
__host__ __device__ constexpr int att_exch_doubles() { return 6 * SEG * Geo<SEG>::NWG; }

template <int SEG, int L>
size_t bwd_att_smem_bytes(int TR) {
    constexpr int NWG = Geo<SEG>::NWG;
    return (size_t)att_exch_doubles<SEG>() * sizeof(double) + (size_t)NWG * ptab_row(TR, L) * sizeof(float) +
           (size_t)2 * SEG * NWG * sizeof(float);
}

template <int SEG, int L, bool EVEN, int SG>
__global__ __launch_bounds__(Geo<SEG>::THREADS) void k_blocks_bwd_att(BwdArgs a) {
    constexpr int NWG = Geo<SEG>::NWG;
    constexpr int SN = SEG * NWG;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, N = a.N, T = a.T, RL = ptab_row(TR, L);
    double *exP = reinterpret_cast<double *>(smem);             // [6][SEG][NWG]: P00 P01 P10 P11 R0 R1
    float *pf_tab = reinterpret_cast<float *>(exP + att_exch_doubles<SEG>());
    float *exX = pf_tab + (size_t)NWG * RL;                       // [SEG][NWG] segment ends of the scan
    float *exVL = exX + SN;                                       // [SEG][NWG] V at each segment's last step

    const int work = xcd_remap(blockIdx.x, gridDim.x);
    const int b = work / a.n_groups, g = work - b * a.n_groups;
    const int n0 = g * NWG;
    build_p_tables<SEG, L>(nullptr, pf_tab, n0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L, EVEN> c;
    lane_setup(c, N, TR, a.dt, n0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    const int pfrow = c.nl * RL + TR + c.t0;
    const float bias = (a.bias_k && c.valid) ? a.bias_k[c.n] : 0.0f;
    const int nc = c.valid ? c.n : N - 1;
    const double beta = exp(-a.dt / (double)a.tau_m[nc]);
    const double omb = 1.0 - beta;
    const double p = exp(-a.dt / (double)a.tau_a[nc]);
    const double dd = (double)c.dd;
    const double slope = (double)a.slope;
    // FP64 powers for the adaptation variable at this segment's start (step t0)
    const double lpd = -a.dt / (double)a.tau_a[nc];
    const double pt0 = exp(lpd * (double)c.t0), pt0m1 = c.t0 > 0 ? exp(lpd * (double)(c.t0 - 1)) : 0.0;

    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rGS = make_rsrc(a.gS ? a.gS + b * TN : nullptr, a.gS ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGV = make_rsrc(a.gV ? a.gV + b * TN : nullptr, a.gV ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGT = make_rsrc(a.gTH ? a.gTH + b * TN : nullptr, a.gTH ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGI = make_rsrc(a.gI ? a.gI + b * TN : nullptr, a.gI ? (uint32_t)(TN * 4) : 0u);
    const size_t CN = (size_t)(a.NB + 1) * N;
    const rsrc_t rCv = make_rsrc(a.ck.v + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCa = make_rsrc(a.ck.a + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCt = make_rsrc(a.ck.ts + b * CN, (uint32_t)CN);
    const uint32_t ck4 = c.valid ? (uint32_t)c.n * 4u : ALIF_OOB;
    const uint32_t ck1 = c.valid ? (uint32_t)c.n : ALIF_OOB;
    const uint32_t blk4 = (uint32_t)(TR * N) * 4u;
    const uint32_t TN4 = (uint32_t)(TN * 4);
    // The step after this segment's last valid one: the next segment's first step,
    // or, for the block's last non-empty segment, step 1 of the next block.
    const int lastw = (TR - 1) / L;
    const uint32_t xn_own = (c.valid && c.w < lastw) ? (uint32_t)((c.t0 + L) * N + c.n) * 4u : ALIF_OOB;
    const uint32_t xn_nxt = (c.valid && c.w == lastw) ? (uint32_t)c.n * 4u : ALIF_OOB;

    struct Slot {
        float x[L], gs[L], gv[L], gt[L];
        float xn;       // input at the step after the segment
        float cv, ca;
        int cts, tsn;
    };
    auto load_block = [&](Slot &dst, int nb) {   // nb < 0: everything out of range
        const uint32_t bo = nb >= 0 ? (uint32_t)nb * blk4 : TN4;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const uint32_t o = c.off(k, bo);
            dst.x[k] = ld_f32(rI, o);
            dst.gs[k] = ld_f32(rGS, o);
            dst.gv[k] = ld_f32(rGV, o);
            dst.gt[k] = ld_f32(rGT, o);
        }
        const uint32_t bn = nb >= 0 ? (uint32_t)min((size_t)(nb + 1) * blk4, TN * 4) : TN4;
        dst.xn = ld_f32(rI, c.w < lastw ? xn_own + bo : xn_nxt + bn);
        const uint32_t e = nb >= 0 ? (uint32_t)(nb * N) : (uint32_t)CN;
        dst.cv = ld_f32(rCv, ck4 + e * 4u);
        dst.ca = ld_f32(rCa, ck4 + e * 4u);
        dst.cts = ld_u8(rCt, ck1 + e);
        dst.tsn = ld_u8(rCt, ck1 + (nb >= 0 ? e + (uint32_t)N : (uint32_t)CN));
    };
    Slot buf[2];
    load_block(buf[0], a.NB - 1);
    load_block(buf[1], a.NB - 2);

    double lamVc = 0.0, lamAc = 0.0;   // lambdas at step 1 of the block after the current one
    double acc_b = 0.0, acc_p = 0.0, acc_d = 0.0, acc_th = 0.0, acc_bias = 0.0;

    auto do_block = [&](Slot &cur, int nb) __attribute__((always_inline)) {
        const int cts = min(cur.cts, TR);
        const int mpre = cts > 0 ? cts - 1 : 0;
        const float a1 = fmaf(c.pf, cur.ca, cts == TR ? 1.0f : 0.0f);
        float uu[L];
        seg_scan(c, cur.x, mpre, uu);
        float E = 0.0f, U = 0.0f;
        if constexpr (SEG > 1) {
            exX[c.w * NWG + c.nl] = uu[L - 1];
            __syncthreads();
            seg_horner(c, exX, E, U);
        }
        float vt[L], th[L];
        seg_membrane(c, cur.cv, E, a1, uu, vt, th);
        const int ts = cur.tsn > 0 ? min(cur.tsn, TR) : ALIF_NO_SPIKE;
        const int tsc = min(ts, TR);

        // The adaptation variable in FP64, Eq. 5 run from the block's saved carry-in:
        // a[t0] in closed form, then a[t] = p a[t-1] + S[t-1] over the segment. It
        // enters the d and p sums, which the attached adjoint can make ill-conditioned.
        double A0 = (double)cur.ca;
        if (c.t0 > 0) {
            A0 = pt0 * A0 + (cts == TR ? pt0m1 : 0.0);
            if (ts < c.t0) A0 += exp(lpd * (double)(c.t0 - 1 - ts));
        }
        double a64[L];
        {
            double av = A0;
#pragma unroll
            for (int k = 0; k < L; k++) {
                const int t = c.t0 + k + 1;
                const bool sp = (t == 1) ? (cts == TR) : (t - 1 == ts);
                av = fma(p, av, sp ? 1.0 : 0.0);
                a64[k] = av;
            }
        }
        // corrected traces (reset after t_s, Eqs. 2 and 5), gate, surrogate and c[t]
        float Vk[L];
        bool gk[L];
        double sk[L], ckk[L];
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int t = c.t0 + k + 1;
            const bool after = t > ts;
            const float pa = pf_tab[pfrow - tsc + k];   // p^(t - 1 - t_s)
            Vk[k] = after ? 0.0f : vt[k];
            const float thk = after ? fmaf(c.dd, pa, th[k]) : th[k];
            gk[k] = (t > mpre) && !after;
            sk[k] = c.kvalid(k) ? surrogate_grad_f64<SG>((double)Vk[k] - (double)thk, slope) : 0.0;
        }
        {   // gate at the step after the segment: inside the block, or step 1 of the next
            // block, which a spike at t_s >= 2 masks (Prop. 3)
            const int tn = c.t0 + L + 1;
            const bool gn = c.w == lastw ? !(ts <= TR && ts >= 2) : (tn > mpre && !(tn > ts));
            const double imn = gn ? (double)(cur.xn + bias) : 0.0;
#pragma unroll
            for (int k = 0; k < L; k++) {
                const double im = (k + 1 < c.len) ? (gk[k + 1 < L ? k + 1 : k] ? (double)(cur.x[k + 1 < L ? k + 1 : k] + bias) : 0.0)
                                                  : imn;
                ckk[k] = fma(beta, (double)Vk[k], omb * im);
            }
        }

        // this segment's maps composed from zero: lam_start = R + P lam_after
        double P00 = 1.0, P01 = 0.0, P10 = 0.0, P11 = 1.0, R0 = 0.0, R1 = 0.0;
#pragma unroll
        for (int k = L - 1; k >= 0; k--) {
            if (c.kvalid(k)) {
                const int t = c.t0 + k + 1;
                const double s = sk[k], sc = s * ckk[k];
                const double m00 = (t == ts ? 0.0 : beta) - sc, m01 = s, m10 = dd * sc, m11 = p - dd * s;
                const double gs = cur.gs[k];
                const double r0 = fma(s, gs, (double)cur.gv[k]);
                const double r1 = dd * ((double)cur.gt[k] - s * gs);
                const double nR0 = r0 + m00 * R0 + m01 * R1, nR1 = r1 + m10 * R0 + m11 * R1;
                const double n00 = m00 * P00 + m01 * P10, n01 = m00 * P01 + m01 * P11;
                const double n10 = m10 * P00 + m11 * P10, n11 = m10 * P01 + m11 * P11;
                R0 = nR0; R1 = nR1; P00 = n00; P01 = n01; P10 = n10; P11 = n11;
            }
        }
        float VLast = 0.0f;   // V at this segment's last valid step
#pragma unroll
        for (int k = 0; k < L; k++) VLast = (k == c.len - 1) ? Vk[k] : VLast;
        double lVin, lAin, lv, la;
        float Vprev0;
        if constexpr (SEG > 1) {
            const int q = c.w * NWG + c.nl;
            exP[q] = P00; exP[SN + q] = P01; exP[2 * SN + q] = P10; exP[3 * SN + q] = P11;
            exP[4 * SN + q] = R0; exP[5 * SN + q] = R1;
            exVL[q] = VLast;
            __syncthreads();
            lv = lamVc; la = lamAc;
            lVin = lv; lAin = la;
#pragma unroll
            for (int s2 = SEG - 1; s2 >= 0; s2--) {
                const int o = s2 * NWG + c.nl;
                lVin = (s2 == c.w) ? lv : lVin;
                lAin = (s2 == c.w) ? la : lAin;
                const double nv = exP[4 * SN + o] + exP[o] * lv + exP[SN + o] * la;
                const double na = exP[5 * SN + o] + exP[2 * SN + o] * lv + exP[3 * SN + o] * la;
                lv = nv; la = na;
            }
            Vprev0 = c.w > 0 ? exVL[(c.w - 1) * NWG + c.nl] : cur.cv;
        } else {
            lVin = lamVc; lAin = lamAc;
            lv = R0 + P00 * lamVc + P01 * lamAc;
            la = R1 + P10 * lamVc + P11 * lamAc;
            Vprev0 = cur.cv;
        }

        // the lambdas step by step from the segment end, and the gradient terms:
        //   dI += (1 - beta) gate lamV;  d/dbeta += (1 - S[t-1]) (V[t-1] - Im[t]) lamV
        //   d/dp += a[t-1] lamA;  d/dd += a[t] lamTh;  d/dtheta0 += lamTh
        const uint32_t bo = (uint32_t)nb * blk4;
        double lV1 = lVin, lA1 = lAin;
        double pb = 0.0, pp = 0.0, pdd = 0.0, pth = 0.0, pbias = 0.0;
#pragma unroll
        for (int k = L - 1; k >= 0; k--) {
            if (c.kvalid(k)) {
                const int t = c.t0 + k + 1;
                const double s = sk[k];
                const double gs = cur.gs[k];
                const double lamS = gs - ckk[k] * lV1 + lA1;
                const double lamV = (double)cur.gv[k] + s * lamS + (t == ts ? 0.0 : beta) * lV1;
                const double lamTh = (double)cur.gt[k] - s * lamS;
                const double lamA = dd * lamTh + p * lA1;
                const bool sprev = (t == 1) ? (cts == TR) : (t - 1 == ts);
                const float Vprev = (k == 0) ? Vprev0 : Vk[k > 0 ? k - 1 : 0];
                const double aprev = (k == 0) ? A0 : a64[k > 0 ? k - 1 : 0];
                const double im = gk[k] ? (double)(cur.x[k] + bias) : 0.0;
                pb += sprev ? 0.0 : ((double)Vprev - im) * lamV;
                pp += aprev * lamA;
                pdd += a64[k] * lamTh;
                pth += lamTh;
                const double glV = gk[k] ? omb * lamV : 0.0;
                pbias += glV;
                st_f32(rGI, c.off(k, bo), (float)glV);
                lV1 = lamV;
                lA1 = lamA;
            }
        }
        acc_b += pb; acc_p += pp; acc_d += pdd; acc_th += pth; acc_bias += pbias;
        lamVc = lv;
        lamAc = la;
        load_block(cur, nb - 2);   // after the last use of this slot
    };

    wait_vmem_all();
    int r0 = 0;
    for (; r0 + 2 <= a.NB; r0 += 2) {
        do_block(buf[0], a.NB - 1 - r0);
        do_block(buf[1], a.NB - 2 - r0);
    }
    if (r0 < a.NB) do_block(buf[0], a.NB - 1 - r0);   // uniform over the workgroup
    // per-(b, n) sums over this neuron's segment-waves, in a fixed order
    if constexpr (SEG > 1) {
        double *red = exP;
        __syncthreads();
        const int q = c.w * NWG + c.nl;
        double vals[5] = {acc_b, acc_p, acc_d, acc_th, acc_bias};
#pragma unroll
        for (int j = 0; j < 5; j++) {
            red[q] = vals[j];
            __syncthreads();
            if (c.w == 0) {
                double sm = 0.0;
                for (int w = 0; w < SEG; w++) sm += red[w * NWG + c.nl];
                vals[j] = sm;
            }
            __syncthreads();
        }
        acc_b = vals[0]; acc_p = vals[1]; acc_d = vals[2]; acc_th = vals[3]; acc_bias = vals[4];
    }
    if (c.valid && c.w == 0) {
        const size_t BN = (size_t)a.B * N, i = (size_t)b * N + c.n;
        a.part[i] = acc_b;
        a.part[BN + i] = acc_p;
        a.part[2 * BN + i] = acc_d;
        a.part[3 * BN + i] = acc_th;
        a.part[4 * BN + i] = acc_bias;
    }
}

// Register prefetch depth, in blocks. Between two blocks a wave does only the
// block's arithmetic and the carry update, so short blocks need more of them in
// flight to cover the HBM latency: the depth targets a number of time steps
// ahead, at least ALIF_*_MIN_DEPTH blocks and within a register budget of
// prefetched values per lane.
#ifndef ALIF_FWD_AHEAD
#define ALIF_FWD_AHEAD 64
#endif
#ifndef ALIF_BWD_AHEAD
#define ALIF_BWD_AHEAD 32
#endif
#define ALIF_FWD_MIN_DEPTH 4
#define ALIF_BWD_MIN_DEPTH (SEG > 1 ? 3 : 2)   // the pipelined backward needs 3

constexpr int clamp_depth(int want, int lo, int hi) { return want < lo ? lo : (want > hi ? hi : want); }
template <int SEG, int L>
constexpr int fwd_depth() {   // <= 64 prefetched floats per lane
    return clamp_depth((ALIF_FWD_AHEAD + SEG * L - 1) / (SEG * L), ALIF_FWD_MIN_DEPTH, 64 / L);
}
template <int SEG, int L>
constexpr int bwd_depth() {   // <= 12 prefetched steps (x, dL/dS and maybe dL/dV, dL/dtheta) per lane
    // 13-16-step segments: two slots (a third would spill; measured 0.84 against 1.46 ms
    // at T_R = 128 on 4 x 2048 x 20000). 10-12 steps keep three (0.63 against 0.71 ms).
    return L >= 13 ? 2 : clamp_depth((ALIF_BWD_AHEAD + SEG * L - 1) / (SEG * L), ALIF_BWD_MIN_DEPTH, 12 / L);
}

template <int SEG, int L>
hipError_t blocks_fwd_launch(const FwdArgs &a, hipStream_t st) {
    const int grid = a.B * a.n_groups;
    if (grid == 0) return hipSuccess;
    const size_t sm = fwd_smem_bytes<SEG, L>(a.TR);
    constexpr int TH = Geo<SEG>::THREADS;
    const bool tr = a.V || a.TH;
#define ALIF_LF(TRC, SD)                                                                          \
    do {                                                                                          \
        if (a.TR == SEG * L)                                                                      \
            hipLaunchKernelGGL((k_blocks_fwd<SEG, L, true, fwd_depth<SEG, L>(), TRC, SD>), dim3(grid), \
                               dim3(TH), sm, st, a);                                              \
        else                                                                                      \
            hipLaunchKernelGGL((k_blocks_fwd<SEG, L, false, fwd_depth<SEG, L>(), TRC, SD>), dim3(grid),\
                               dim3(TH), sm, st, a);                                              \
    } while (0)
    if (tr) {
        if (a.spike_dtype == 0) ALIF_LF(true, 0);
        else if (a.spike_dtype == 1) ALIF_LF(true, 1);
        else ALIF_LF(true, 2);
    } else {
        if (a.spike_dtype == 0) ALIF_LF(false, 0);
        else if (a.spike_dtype == 1) ALIF_LF(false, 1);
        else ALIF_LF(false, 2);
    }
#undef ALIF_LF
    return hipGetLastError();
}

template <int SEG, int L>
hipError_t blocks_bwd_launch(const BwdArgs &a, hipStream_t st) {
    const int grid = a.B * a.n_groups;
    if (grid == 0) return hipSuccess;
    constexpr int TH = Geo<SEG>::THREADS;
    if (a.attached) {
        const size_t sma = bwd_att_smem_bytes<SEG, L>(a.TR);
#define ALIF_LA(SG)                                                                                     \
    do {                                                                                                \
        if (a.TR == SEG * L)                                                                            \
            hipLaunchKernelGGL((k_blocks_bwd_att<SEG, L, true, SG>), dim3(grid), dim3(TH), sma, st, a); \
        else                                                                                            \
            hipLaunchKernelGGL((k_blocks_bwd_att<SEG, L, false, SG>), dim3(grid), dim3(TH), sma, st, a);\
    } while (0)
        if (a.surrogate == 1) ALIF_LA(1);
        else if (a.surrogate == 2) ALIF_LA(2);
        else ALIF_LA(0);
#undef ALIF_LA
        return hipGetLastError();
    }
    const size_t sm = bwd_smem_bytes<SEG, L>(a.TR);
    const bool gvt = a.gV || a.gTH;
    const int gi = a.gI ? 1 : (a.gI16 ? 2 : 0);   // (a bfloat16 gI comes without gV / gTH)
#define ALIF_LB3(G1, G2, SG)                                                                      \
    do {                                                                                          \
        if (a.TR == SEG * L)                                                                      \
            hipLaunchKernelGGL((k_blocks_bwd<SEG, L, true, bwd_depth<SEG, L>(), G1, G2, SG>), dim3(grid), \
                               dim3(TH), sm, st, a);                                              \
        else                                                                                      \
            hipLaunchKernelGGL((k_blocks_bwd<SEG, L, false, bwd_depth<SEG, L>(), G1, G2, SG>), dim3(grid),\
                               dim3(TH), sm, st, a);                                              \
    } while (0)
#define ALIF_LB(G1, G2)                                                                           \
    do {                                                                                          \
        if (a.surrogate == 1) ALIF_LB3(G1, G2, 1);                                                \
        else if (a.surrogate == 2) ALIF_LB3(G1, G2, 2);                                           \
        else ALIF_LB3(G1, G2, 0);                                                                 \
    } while (0)
    if (gvt) { if (gi == 1) ALIF_LB(true, 1); else ALIF_LB(true, 0); }
    else { if (gi == 1) ALIF_LB(false, 1); else if (gi == 2) ALIF_LB(false, 2); else ALIF_LB(false, 0); }
#undef ALIF_LB
#undef ALIF_LB3
    return hipGetLastError();
}

#define ALIF_INSTANTIATE(SEG, L)                                                        \
    template hipError_t blocks_fwd_launch<SEG, L>(const FwdArgs &, hipStream_t);       \
    template hipError_t blocks_bwd_launch<SEG, L>(const BwdArgs &, hipStream_t);

}  // namespace alif
