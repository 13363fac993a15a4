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
// GPU mapping. A wavefront holds 64/SEG neurons x SEG time segments of L steps
// (lane = neuron * SEG + segment), so the T_R steps of a block are spread over
// SEG lanes and each lane integrates only L = ceil(T_R / SEG) steps
// sequentially. Segments are combined by an affine prefix scan in DPP (row_shr)
// and the first crossing by a DPP min-reduce, so no shared memory round trip
// sits in the per-block dependency chain. Each wave is persistent over all
// T / T_R blocks of its neurons; the carry (V0 and a in FP64) stays in
// registers and input loads run DEPTH blocks ahead. HBM access is
// neuron-innermost: lanes of one segment read consecutive neurons of a step.
//
// Precision. Inputs and per-step arithmetic are FP32. Decay powers beta^k, p^k
// are evaluated in FP64 (exp(-k DT / tau)) and rounded once. The block-boundary
// carry is FP64: the no-spike membrane is V0 <- beta^T_R V0 + U[T_R] and the
// adaptation a <- p^T_R a + (spike term), so rounding does not accumulate over
// the T / T_R boundaries.
#include "alif_common.h"
#include "alif_kernels.h"

namespace alif {

#define ALIF_NO_SPIKE 0x7fff  // "no crossing" marker for the per-block spike step

// Per-lane constants of the block recurrence.
template <int SEG, int L>
struct Lane {
    int s, j, n, t0, len;
    bool valid;
    float beta, omb, pf, th0, dd, bias;
    double betaT, pT;
    float bt[L];  // beta^(t_k)      t_k = t0 + k + 1 (block-local step)
    float bk[L];  // beta^(k + 1)
    float pt[L];  // p^(t_k - 1)
    float D[4];   // prefix-scan decays across 1, 2, 4, 8 segments ending here
    float ptm1;   // p^(t0 - 1) (s >= 1), for a[t-1] at the lane's first step
};

template <int SEG, int L>
__device__ __forceinline__ void lane_setup(Lane<SEG, L> &c, int N, int TR, double dt, int n0,
                                           const float *tau_m, const float *tau_a,
                                           const float *d, const float *theta0,
                                           const float *bias) {
    constexpr int NPW = 64 / SEG;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    c.s = lane & (SEG - 1);
    c.j = wave * NPW + lane / SEG;
    c.n = n0 + c.j;
    c.valid = c.n < N;
    const int nc = c.valid ? c.n : N - 1;
    const float tm = tau_m[nc], ta = tau_a[nc];
    c.dd = d[nc];
    c.th0 = theta0[nc];
    c.bias = bias ? bias[nc] : 0.0f;
    const double lb = -dt / (double)tm, lp = -dt / (double)ta;
    c.beta = (float)exp(lb);
    c.omb = (float)(-expm1(lb));
    c.pf = (float)exp(lp);
    c.betaT = exp(lb * TR);
    c.pT = exp(lp * TR);
    c.t0 = c.s * L;
    c.len = max(0, min(L, TR - c.t0));
#pragma unroll
    for (int k = 0; k < L; k++) {
        c.bt[k] = (float)exp(lb * (double)(c.t0 + k + 1));
        c.bk[k] = (float)exp(lb * (double)(k + 1));
        c.pt[k] = (float)exp(lp * (double)(c.t0 + k));
    }
    c.ptm1 = (float)exp(lp * (double)max(0, c.t0 - 1));
    const int cum = min(TR, (c.s + 1) * L);
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int off = 1 << r;
        const int prev = min(TR, max(0, c.s + 1 - off) * L);
        c.D[r] = (float)exp(lb * (double)(cum - prev));
    }
}

// p^k tables for data-dependent exponents: FP64 (carry) and FP32 (traces)
template <int NWG>
__device__ __forceinline__ void build_p_tables(double *pd, float *pf, int n0, int N, int TR,
                                               double dt, const float *tau_a) {
    const int TRP = TR + 1;
    for (int idx = threadIdx.x; idx < NWG * TRP; idx += blockDim.x) {
        const int jj = idx / TRP, k = idx - jj * TRP;
        const int nn = min(n0 + jj, N - 1);
        const double v = exp(-dt / (double)tau_a[nn] * (double)k);
        pd[idx] = v;
        pf[idx] = (float)v;
    }
    __syncthreads();
}

// The per-block integration shared by forward and backward (identical
// arithmetic, so the backward recovers exactly the forward's spike steps).
//   x[k]  input current at t_k (bias included), a1 = a[1] of the block,
//   cv    V0 as float, mpre = masked leading steps (t_s of the previous block - 1).
// Returns the block's spike step t_s (ALIF_NO_SPIKE if none), the no-reset
// membrane vt[k], the threshold th[k] (valid up to t_s) and P (inclusive
// segment prefix; on the group's last lane it is U[T_R]).
template <int SEG, int L>
__device__ __forceinline__ int block_integrate(const Lane<SEG, L> &c, const float (&x)[L],
                                               float cv, float a1, int mpre, float (&vt)[L],
                                               float (&th)[L], float &P) {
    float uu[L];
    float u = 0.0f;
#pragma unroll
    for (int k = 0; k < L; k++) {
        const float im = (c.t0 + k + 1 > mpre) ? x[k] : 0.0f;     // Prop. 3 mask
        u = fmaf(c.beta, u, c.omb * im);                          // Prop. 1, local part
        uu[k] = u;
    }
    float X = 0.0f;
#pragma unroll
    for (int k = 0; k < L; k++) X = (k == c.len - 1) ? uu[k] : X;
    P = group_prefix<SEG>(X, c.s, c.D);
    const float E = from_prev<SEG>(P, c.s, 0.0f);                 // U at segment start
    const float da1 = c.dd * a1;
    int cand = ALIF_NO_SPIKE;
#pragma unroll
    for (int k = L - 1; k >= 0; k--) {
        const float U = fmaf(c.bk[k], E, uu[k]);
        vt[k] = fmaf(c.bt[k], cv, U);                             // V~[t]
        th[k] = fmaf(c.pt[k], da1, c.th0);                        // Prop. 5
        const int t = c.t0 + k + 1;
        if (k < c.len && t > mpre && vt[k] > th[k]) cand = t;     // Eq. 7, strict
    }
    return group_min<SEG>(cand);                                  // Eqs. 8-9 / Prop. 2
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
template <int SEG, int L, int DEPTH>
__global__ __launch_bounds__(256) void k_blocks_fwd(FwdArgs a) {
    constexpr int NPW = 64 / SEG, NWG = 4 * NPW;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, TRP = TR + 1, N = a.N, T = a.T;
    double *pd_tab = reinterpret_cast<double *>(smem);
    float *pf_tab = reinterpret_cast<float *>(smem + (size_t)NWG * TRP * sizeof(double));

    const int work = xcd_remap(blockIdx.x, gridDim.x);
    const int b = work / a.n_groups, g = work - b * a.n_groups;
    const int n0 = g * NWG;
    build_p_tables<NWG>(pd_tab, pf_tab, n0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L> c;
    lane_setup(c, N, TR, a.dt, n0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    if (c.valid && c.s == 0 && !params_ok(a.tau_m[c.n], a.tau_a[c.n], c.dd, c.th0))
        atomicOr(a.status, 1u);
    const int ptab = c.j * TRP;

    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const int sb = spike_bytes(a.spike_dtype);
    const rsrc_t rS = make_rsrc((const char *)a.spikes + b * TN * sb, (uint32_t)(TN * sb));
    const rsrc_t rV = make_rsrc(a.V ? a.V + b * TN : nullptr, a.V ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rT = make_rsrc(a.TH ? a.TH + b * TN : nullptr, a.TH ? (uint32_t)(TN * 4) : 0u);
    const size_t CN = (size_t)a.NB * N;
    const bool ck = a.ck.v != nullptr;
    const rsrc_t rCv = make_rsrc(ck ? a.ck.v + b * CN : nullptr, ck ? (uint32_t)(CN * 4) : 0u);
    const rsrc_t rCa = make_rsrc(ck ? a.ck.a + b * CN : nullptr, ck ? (uint32_t)(CN * 4) : 0u);
    const rsrc_t rCt = make_rsrc(ck ? a.ck.ts + b * CN : nullptr, ck ? (uint32_t)CN : 0u);

    // carry-in of block 0
    double v0d = 0.0, a0d = 0.0;
    int cts = 0;
    if (a.init_v && c.valid) {
        const size_t i = (size_t)b * N + c.n;
        v0d = a.init_v[i];
        a0d = a.init_a[i];
        cts = a.init_ts[i];
        if (cts < 0 || cts > TR) { if (c.s == 0) atomicOr(a.status, 1u); cts = 0; }
    }

    float buf[DEPTH][L];
    auto load_block = [&](float (&dst)[L], int nb) {
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int tg = nb * TR + c.t0 + k;
            const bool ok = c.valid && k < c.len && tg < T && nb < a.NB;
            dst[k] = ld_f32(rI, ok ? (uint32_t)(tg * N + c.n) * 4u : ALIF_OOB);
        }
    };
#pragma unroll
    for (int i = 0; i < DEPTH; i++) load_block(buf[i], i);

    for (int nb0 = 0; nb0 < a.NB; nb0 += DEPTH) {
#pragma unroll
        for (int i = 0; i < DEPTH; i++) {
            const int nb = nb0 + i;
            const bool live = nb < a.NB;
            float x[L];
#pragma unroll
            for (int k = 0; k < L; k++) x[k] = buf[i][k] + c.bias;
            load_block(buf[i], nb + DEPTH);

            const float cv = (float)v0d, ca = (float)a0d;
            const int mpre = cts > 0 ? cts - 1 : 0;
            const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
            if (ck && c.s == 0) {   // carry-in of this block, for the backward pass
                const bool ok = c.valid && live;
                const uint32_t e = (uint32_t)(nb * N + c.n);
                st_f32(rCv, ok ? e * 4u : ALIF_OOB, cv);
                st_f32(rCa, ok ? e * 4u : ALIF_OOB, ca);
                st_u8(rCt, ok ? e : ALIF_OOB, (uint8_t)cts);
            }
            float vt[L], th[L], P;
            const int ts = block_integrate<SEG, L>(c, x, cv, a1, mpre, vt, th, P);
            const bool spk = ts <= TR;

            // outputs: spikes and corrected traces (reset after t_s, Eqs. 2 and 5)
#pragma unroll
            for (int k = 0; k < L; k++) {
                const int t = c.t0 + k + 1;
                const int tg = nb * TR + t - 1;
                const bool ok = c.valid && live && k < c.len && tg < T;
                const uint32_t e = (uint32_t)(tg * N + c.n);
                st_spike(rS, a.spike_dtype, ok ? e * (uint32_t)sb : ALIF_OOB, t == ts);
                if (a.V) st_f32(rV, ok ? e * 4u : ALIF_OOB, t <= ts ? vt[k] : 0.0f);
                if (a.TH) {
                    const bool after = t > ts;
                    const float pa = pf_tab[ptab + (after ? min(t - 1 - ts, TR) : 0)];
                    st_f32(rT, ok ? e * 4u : ALIF_OOB, after ? fmaf(c.dd, pa, th[k]) : th[k]);
                }
            }
            // carry to the next block (Props. 4-5), FP64
            const float uTR = group_bcast<SEG>(P, c.s, SEG - 1);
            double extra = 0.0;
            if (cts == TR) extra += pd_tab[ptab + TR - 1];
            if (spk && ts < TR) extra += pd_tab[ptab + TR - 1 - ts];
            const double nv = spk ? 0.0 : fma(c.betaT, v0d, (double)uTR);
            const double na = fma(c.pT, a0d, extra);
            v0d = live ? nv : v0d;
            a0d = live ? na : a0d;
            cts = live ? (spk ? ts : 0) : cts;
        }
    }
    if (a.fin_v && c.valid && c.s == 0) {
        const size_t i = (size_t)b * N + c.n;
        a.fin_v[i] = v0d;
        a.fin_a[i] = a0d;
        a.fin_ts[i] = cts;
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
template <int SEG, int L, int DEPTH, bool GVT>
__global__ __launch_bounds__(256) void k_blocks_bwd(BwdArgs a) {
    constexpr int NPW = 64 / SEG, NWG = 4 * NPW;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TR = a.TR, TRP = TR + 1, N = a.N, T = a.T;
    double *pd_tab = reinterpret_cast<double *>(smem);
    float *pf_tab = reinterpret_cast<float *>(smem + (size_t)NWG * TRP * sizeof(double));

    const int work = xcd_remap(blockIdx.x, gridDim.x);
    const int b = work / a.n_groups, g = work - b * a.n_groups;
    const int n0 = g * NWG;
    build_p_tables<NWG>(pd_tab, pf_tab, n0, N, TR, a.dt, a.tau_a);
    Lane<SEG, L> c;
    lane_setup(c, N, TR, a.dt, n0, a.tau_m, a.tau_a, a.d, a.theta0, a.bias_k);
    const int ptab = c.j * TRP;

    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rGS = make_rsrc(a.gS ? a.gS + b * TN : nullptr, a.gS ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGV = make_rsrc(a.gV ? a.gV + b * TN : nullptr, a.gV ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGT = make_rsrc(a.gTH ? a.gTH + b * TN : nullptr, a.gTH ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGI = make_rsrc(a.gI ? a.gI + b * TN : nullptr, a.gI ? (uint32_t)(TN * 4) : 0u);
    const size_t CN = (size_t)a.NB * N;
    const rsrc_t rCv = make_rsrc(a.ck.v + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCa = make_rsrc(a.ck.a + b * CN, (uint32_t)(CN * 4));
    const rsrc_t rCt = make_rsrc(a.ck.ts + b * CN, (uint32_t)CN);

    struct Slot {
        float x[L], gs[L], gv[L], gt[L];
        float cv, ca;
        int cts;
    };
    Slot buf[DEPTH];
    auto load_block = [&](Slot &dst, int nb) {
        const bool blk = nb >= 0;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int tg = nb * TR + c.t0 + k;
            const bool ok = blk && c.valid && k < c.len && tg < T;
            const uint32_t off = ok ? (uint32_t)(tg * N + c.n) * 4u : ALIF_OOB;
            dst.x[k] = ld_f32(rI, off);
            dst.gs[k] = ld_f32(rGS, off);
            if constexpr (GVT) {
                dst.gv[k] = ld_f32(rGV, off);
                dst.gt[k] = ld_f32(rGT, off);
            } else {
                dst.gv[k] = 0.0f;
                dst.gt[k] = 0.0f;
            }
        }
        const bool ok = blk && c.valid;
        const uint32_t e = (uint32_t)(max(nb, 0) * N + c.n);
        dst.cv = ld_f32(rCv, ok ? e * 4u : ALIF_OOB);
        dst.ca = ld_f32(rCa, ok ? e * 4u : ALIF_OOB);
        dst.cts = ld_u8(rCt, ok ? e : ALIF_OOB);
    };
#pragma unroll
    for (int i = 0; i < DEPTH; i++) load_block(buf[i], a.NB - 1 - i);

    float lamV_c = 0.0f, lamA_c = 0.0f;  // lambda_V, lambda_a at step 1 of the next block
    double acc_b = 0.0, acc_p = 0.0, acc_d = 0.0, acc_th = 0.0, acc_bias = 0.0;

    for (int r0 = 0; r0 < a.NB; r0 += DEPTH) {
#pragma unroll
        for (int i = 0; i < DEPTH; i++) {
            const int nb = a.NB - 1 - (r0 + i);
            const bool live = nb >= 0;
            Slot cur = buf[i];
            load_block(buf[i], nb - DEPTH);
            float x[L];
#pragma unroll
            for (int k = 0; k < L; k++) x[k] = cur.x[k] + c.bias;
            const int cts = min(cur.cts, TR);
            const float cv = cur.cv, ca = cur.ca;
            const int mpre = cts > 0 ? cts - 1 : 0;
            const float a1 = fmaf(c.pf, ca, cts == TR ? 1.0f : 0.0f);
            float vt[L], th[L], P;
            const int ts = block_integrate<SEG, L>(c, x, cv, a1, mpre, vt, th, P);

            // corrected forward quantities and the local reverse scans
            float Vk[L], ak[L], lt[L], rV[L], PV[L], rA[L], PA[L];
            bool gate[L];
#pragma unroll
            for (int k = 0; k < L; k++) {
                const int t = c.t0 + k + 1;
                const int tg = nb * TR + t - 1;
                const bool vk = k < c.len && tg < T;
                const bool after = t > ts;
                const float pa = pf_tab[ptab + (after ? min(t - 1 - ts, TR) : 0)];
                Vk[k] = after ? 0.0f : vt[k];
                ak[k] = after ? fmaf(c.pt[k], a1, pa) : c.pt[k] * a1;
                const float thk = after ? fmaf(c.dd, pa, th[k]) : th[k];
                gate[k] = (t > mpre) && !after;
                const float sg = fast_sigmoid_grad(Vk[k] - thk, a.slope);
                const float gsk = cur.gs[k] * sg;
                lt[k] = vk ? cur.gt[k] - gsk : 0.0f;
                const float cV = vk ? cur.gv[k] + gsk : 0.0f;
                (void)cV;
                rV[k] = cV;   // scanned below
            }
            {
                float rv = 0.0f, pv = 1.0f, ra = 0.0f, pa = 1.0f;
#pragma unroll
                for (int k = L - 1; k >= 0; k--) {
                    const int t = c.t0 + k + 1;
                    const int tg = nb * TR + t - 1;
                    const bool vk = k < c.len && tg < T;
                    const float fV = vk ? (t == ts ? 0.0f : c.beta) : 1.0f;
                    const float fA = vk ? c.pf : 1.0f;
                    rv = fmaf(fV, rv, rV[k]);
                    pv = pv * fV;
                    ra = fmaf(fA, ra, c.dd * lt[k]);
                    pa = pa * fA;
                    rV[k] = rv;
                    PV[k] = pv;
                    rA[k] = ra;
                    PA[k] = pa;
                }
            }
            float MV = PV[0], RV = rV[0], MA = PA[0], RA = rA[0];
            group_suffix<SEG>(MV, RV, c.s);
            group_suffix<SEG>(MA, RA, c.s);
            const float lVin = fmaf(from_next<SEG>(MV, c.s, 1.0f), lamV_c, from_next<SEG>(RV, c.s, 0.0f));
            const float lAin = fmaf(from_next<SEG>(MA, c.s, 1.0f), lamA_c, from_next<SEG>(RA, c.s, 0.0f));
            const float Vprev0 = from_prev<SEG>(Vk[L - 1], c.s, cv);

            float pb = 0.0f, pp = 0.0f, pdd = 0.0f, pth = 0.0f, pbias = 0.0f;
            float lV0 = 0.0f, lA0 = 0.0f;
#pragma unroll
            for (int k = 0; k < L; k++) {
                const int t = c.t0 + k + 1;
                const int tg = nb * TR + t - 1;
                const bool vk = k < c.len && tg < T;
                const float lV = fmaf(PV[k], lVin, rV[k]);
                const float lA = fmaf(PA[k], lAin, rA[k]);
                if (k == 0) { lV0 = lV; lA0 = lA; }
                const bool sprev = (t == 1) ? (cts == TR) : (t - 1 == ts);
                const float Vprev = (k == 0) ? Vprev0 : Vk[k > 0 ? k - 1 : 0];
                float aprev;
                if (t == 1) {
                    aprev = ca;
                } else {
                    const float pbase = (k == 0) ? c.ptm1 : c.pt[k > 0 ? k - 1 : 0];
                    const bool aft = t - 1 > ts;
                    const float pa = pf_tab[ptab + (aft ? min(t - 2 - ts, TR) : 0)];
                    aprev = aft ? fmaf(pbase, a1, pa) : pbase * a1;
                }
                const float gI = gate[k] ? c.omb * lV : 0.0f;
                if (vk) {
                    pb = fmaf(sprev ? 0.0f : (Vprev - (gate[k] ? x[k] : 0.0f)), lV, pb);
                    pp = fmaf(aprev, lA, pp);
                    pdd = fmaf(ak[k], lt[k], pdd);
                    pth += lt[k];
                    pbias += gI;
                }
                if (a.gI) {
                    const bool ok = c.valid && live && vk;
                    st_f32(rGI, ok ? (uint32_t)(tg * N + c.n) * 4u : ALIF_OOB, gI);
                }
            }
            if (live) {
                acc_b += (double)pb;
                acc_p += (double)pp;
                acc_d += (double)pdd;
                acc_th += (double)pth;
                acc_bias += (double)pbias;
                lamV_c = group_bcast<SEG>(lV0, c.s, 0);
                lamA_c = group_bcast<SEG>(lA0, c.s, 0);
            }
        }
    }
    acc_b = group_sum<SEG>(acc_b);
    acc_p = group_sum<SEG>(acc_p);
    acc_d = group_sum<SEG>(acc_d);
    acc_th = group_sum<SEG>(acc_th);
    acc_bias = group_sum<SEG>(acc_bias);
    if (c.valid && c.s == 0) {
        const size_t BN = (size_t)a.B * N, i = (size_t)b * N + c.n;
        a.part[i] = acc_b;
        a.part[BN + i] = acc_p;
        a.part[2 * BN + i] = acc_d;
        a.part[3 * BN + i] = acc_th;
        a.part[4 * BN + i] = acc_bias;
    }
}

// Sum the per-(b, n) FP64 partials over the batch in a fixed order and convert
// d/dbeta, d/dp to d/dtau (dbeta/dtau = beta DT / tau^2).
__global__ void k_finalize(FinalizeArgs a) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const size_t BN = (size_t)a.B * a.N;
    double s[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < a.B; b++)
        for (int q = 0; q < 5; q++) s[q] += a.part[q * BN + (size_t)b * a.N + n];
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
    if (TR <= 96) return {16, 6};
    return {16, 8};
}
int block_neurons_per_wg(int seg) { return 4 * (64 / seg); }
size_t block_smem_bytes(int seg, int TR) {
    return (size_t)block_neurons_per_wg(seg) * (TR + 1) * (sizeof(double) + sizeof(float));
}

#define ALIF_FWD_DEPTH 4
#define ALIF_BWD_DEPTH 3

template <int SEG, int L>
static hipError_t fwd_t(const FwdArgs &a, hipStream_t st) {
    const int grid = a.B * a.n_groups;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_blocks_fwd<SEG, L, ALIF_FWD_DEPTH>), dim3(grid), dim3(256),
                       block_smem_bytes(SEG, a.TR), st, a);
    return hipGetLastError();
}
template <int SEG, int L>
static hipError_t bwd_t(const BwdArgs &a, hipStream_t st) {
    const int grid = a.B * a.n_groups;
    if (grid == 0) return hipSuccess;
    if (a.gV || a.gTH)
        hipLaunchKernelGGL((k_blocks_bwd<SEG, L, ALIF_BWD_DEPTH, true>), dim3(grid), dim3(256),
                           block_smem_bytes(SEG, a.TR), st, a);
    else
        hipLaunchKernelGGL((k_blocks_bwd<SEG, L, ALIF_BWD_DEPTH, false>), dim3(grid), dim3(256),
                           block_smem_bytes(SEG, a.TR), st, a);
    return hipGetLastError();
}

#define ALIF_DISPATCH(FN, ARGS, ST)                          \
    do {                                                     \
        BlockConfig cfg = block_config((ARGS).TR);           \
        switch (cfg.seg * 100 + cfg.len) {                   \
        case 102: return FN<1, 2>(ARGS, ST);                 \
        case 103: return FN<1, 3>(ARGS, ST);                 \
        case 104: return FN<1, 4>(ARGS, ST);                 \
        case 203: return FN<2, 3>(ARGS, ST);                 \
        case 204: return FN<2, 4>(ARGS, ST);                 \
        case 403: return FN<4, 3>(ARGS, ST);                 \
        case 404: return FN<4, 4>(ARGS, ST);                 \
        case 405: return FN<4, 5>(ARGS, ST);                 \
        case 406: return FN<4, 6>(ARGS, ST);                 \
        case 408: return FN<4, 8>(ARGS, ST);                 \
        case 805: return FN<8, 5>(ARGS, ST);                 \
        case 806: return FN<8, 6>(ARGS, ST);                 \
        case 808: return FN<8, 8>(ARGS, ST);                 \
        case 1606: return FN<16, 6>(ARGS, ST);               \
        case 1608: return FN<16, 8>(ARGS, ST);               \
        default: return hipErrorInvalidValue;                \
        }                                                    \
    } while (0)

hipError_t launch_blocks_fwd(const FwdArgs &a, hipStream_t st) { ALIF_DISPATCH(fwd_t, a, st); }
hipError_t launch_blocks_bwd(const BwdArgs &a, hipStream_t st) { ALIF_DISPATCH(bwd_t, a, st); }

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3((a.N + 255) / 256), dim3(256), 0, st, a);
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
