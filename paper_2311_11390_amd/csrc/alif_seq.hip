// Sequential ALIF baselines for gfx950: the plain per-step recurrence of the
// standard model (paper Section 2, Eqs. 1-5), one thread per (batch, neuron).
//
//  * k_seq_fwd: one launch, each thread loops over all T steps (input loads run
//    DEPTH steps ahead). Writes block-boundary checkpoints every T_R steps so
//    that the sequential backward moves the same bytes as the block backward.
//  * k_seq_step: one launch per time step (state round-trips through HBM), the
//    cost structure of a framework-level "standard" implementation.
//  * k_seq_bwd: reverse over the T_R-step intervals; each interval is
//    recomputed forward from its checkpoint into shared memory, then the
//    adjoint recurrence runs backwards over it step by step, under the detached
//    gradient policy or the attached one (supplementary "Detaching gradients").
//
// The membrane and adaptation state are FP64. That is a parity requirement, not
// a speed choice: an FP32 per-step recurrence drifts by ~1e-5 over thousands of
// small steps (DT = 0.05 ms, beta ~ 0.9975), enough to flip crossings well outside
// the 1e-6 band the parity tests excuse. FP64 vector arithmetic costs this kernel
// about half the FP32 vector rate (78.6 against 157.3 TFLOP/s on MI355X); at the
// fine-DT size the 16384 (batch, neuron) rows are 256 waves, one per CU, so the
// per-step dependence chain rather than the arithmetic rate sets the time.
#include <type_traits>

#include "alif_common.h"
#include "alif_kernels.h"

namespace alif {

struct SeqLane {
    double beta, omb, p, th0, d;
    float bias;
    int n;
    bool valid;
};

__device__ __forceinline__ SeqLane seq_lane(const SeqArgs &a, int n) {
    SeqLane L;
    L.n = n;
    L.valid = n < a.N;
    const int nc = L.valid ? n : a.N - 1;
    const double lb = -a.dt / (double)a.tau_m[nc], lp = -a.dt / (double)a.tau_a[nc];
    L.beta = exp(lb);
    L.omb = -expm1(lb);
    L.p = exp(lp);
    L.th0 = a.theta0[nc];
    L.d = a.d[nc];
    L.bias = a.bias_k ? a.bias_k[nc] : 0.0f;
    return L;
}

// One step of Eqs. 1-5. c = steps since the last spike (capped at T_R);
// returns the spike and leaves V, a, theta of this step in v, av, th.
__device__ __forceinline__ bool seq_step(const SeqLane &L, int TR, float x, double &v, double &av,
                                         int &c, bool &sprev, double &th, bool &pass) {
    c = min(c + 1, TR);
    pass = c >= TR;                                           // Eq. 4
    const double im = pass ? (double)x : 0.0;
    v = sprev ? 0.0 : fma(L.beta, v, L.omb * im);             // Eq. 2
    av = fma(L.p, av, sprev ? 1.0 : 0.0);                     // Eq. 5
    th = fma(L.d, av, L.th0);
    const bool s = v > th;                                    // Eq. 1
    if (s) c = 0;
    sprev = s;
    return s;
}

__device__ __forceinline__ void seq_work(int &b, int &n, int N) {
    const int per_b = (N + 63) / 64;
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    b = w / per_b;
    n = (w - b * per_b) * 64 + (int)threadIdx.x;
}

template <int DEPTH>
__global__ __launch_bounds__(64) void k_seq_fwd(SeqArgs a) {
    int b, n;
    seq_work(b, n, a.N);
    const SeqLane L = seq_lane(a, n);
    const int N = a.N, T = a.T, TR = a.TR;
    if (L.valid && !params_ok(a.tau_m[n], a.tau_a[n], (float)L.d, (float)L.th0)) atomicOr(a.status, 1u);
    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const int sb = spike_bytes(a.spike_dtype);
    const rsrc_t rS = make_rsrc((const char *)a.spikes + b * TN * sb, (uint32_t)(TN * sb));
    const rsrc_t rV = make_rsrc(a.V ? a.V + b * TN : nullptr, a.V ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rT = make_rsrc(a.TH ? a.TH + b * TN : nullptr, a.TH ? (uint32_t)(TN * 4) : 0u);

    double v = 0.0, av = 0.0;
    int c = TR;
    bool sprev = false;
    if (a.init_v && L.valid) {
        const size_t i = (size_t)b * N + n;
        v = a.init_v[i];
        av = a.init_a[i];
        int ts = a.init_ts[i];
        ts = (ts < 0 || ts > TR) ? 0 : ts;
        c = ts > 0 ? TR - ts : TR;
        sprev = ts == TR;
    }
    const size_t CN = (size_t)a.NB * N;
    double *ckv = a.ck.v ? a.ck.v + b * CN : nullptr;
    double *cka = a.ck.v ? a.ck.a + b * CN : nullptr;
    int32_t *ckc = a.ck.v ? a.ck.c + b * CN : nullptr;

    float ring[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; i++)
        ring[i] = ld_f32(rI, (L.valid && i < T) ? (uint32_t)(i * N + n) * 4u : ALIF_OOB);
    int kb = 0, nb = 0;  // step within the current T_R interval, interval index
    for (int t0 = 0; t0 < T; t0 += DEPTH) {
#pragma unroll
        for (int i = 0; i < DEPTH; i++) {
            const int t = t0 + i;
            const bool live = t < T;
            const float x = ring[i] + L.bias;
            const int tn = t + DEPTH;
            ring[i] = ld_f32(rI, (L.valid && tn < T) ? (uint32_t)(tn * N + n) * 4u : ALIF_OOB);
            if (live && kb == 0 && ckv && L.valid) {
                ckv[(size_t)nb * N + n] = v;
                cka[(size_t)nb * N + n] = av;
                ckc[(size_t)nb * N + n] = sprev ? 0 : c;
            }
            if (live) {
                double th;
                bool pass;
                const bool s = seq_step(L, TR, x, v, av, c, sprev, th, pass);
                const bool ok = L.valid;
                const uint32_t e = (uint32_t)(t * N + n);
                st_spike(rS, a.spike_dtype, ok ? e * (uint32_t)sb : ALIF_OOB, s);
                if (a.V) st_f32(rV, ok ? e * 4u : ALIF_OOB, (float)v);
                if (a.TH) st_f32(rT, ok ? e * 4u : ALIF_OOB, (float)th);
                if (++kb == TR) { kb = 0; nb++; }
            }
        }
    }
    if (a.fin_v && L.valid) {
        const size_t i = (size_t)b * N + n;
        const bool spiked_last_block = c < TR;
        a.fin_v[i] = spiked_last_block ? 0.0 : v;
        a.fin_a[i] = av;
        a.fin_ts[i] = spiked_last_block ? TR - c : 0;
    }
}

// one step for all (b, n); state in HBM
__global__ __launch_bounds__(256) void k_seq_step(SeqArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N;
    if (idx >= a.B * N) return;
    const int b = idx / N, n = idx - b * N;
    const SeqLane L = seq_lane(a, n);
    const int TR = a.TR, t = a.step;
    double v, av;
    int c;
    if (t == 0) {
        v = a.init_v ? a.init_v[idx] : 0.0;
        av = a.init_a ? a.init_a[idx] : 0.0;
        int ts = a.init_ts ? a.init_ts[idx] : 0;
        ts = (ts < 0 || ts > TR) ? 0 : ts;
        c = ts > 0 ? TR - ts : TR;
    } else {
        v = a.st_v[idx];
        av = a.st_a[idx];
        c = a.st_c[idx];
    }
    bool sprev = c == 0;
    const size_t e = ((size_t)b * a.T + t) * N + n;
    const float x = a.I[e] + L.bias;
    double th;
    bool pass;
    const bool s = seq_step(L, TR, x, v, av, c, sprev, th, pass);
    a.st_v[idx] = v;
    a.st_a[idx] = av;
    a.st_c[idx] = c;
    const int sb = spike_bytes(a.spike_dtype);
    if (sb == 1) ((uint8_t *)a.spikes)[e] = s;
    else if (sb == 2) ((uint16_t *)a.spikes)[e] = s ? 0x3F80 : 0;
    else ((float *)a.spikes)[e] = s ? 1.0f : 0.0f;
    if (a.V) a.V[e] = (float)v;
    if (a.TH) a.TH[e] = (float)th;
    if (t == a.T - 1 && a.fin_v) {
        const bool spk = c < TR;
        a.fin_v[idx] = spk ? 0.0 : v;
        a.fin_a[idx] = av;
        a.fin_ts[idx] = spk ? TR - c : 0;
    }
}

__device__ __forceinline__ float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return fma(a, b, c); }

// Sequential backward. Shared memory per lane and step of the current interval:
// V, theta, a, x, gS (+ gV, gTheta) as float and a flag byte. ATT: attached
// gradient policy, where dL/dS[t] also takes -c[t] lambda_V[t+1] + lambda_a[t+1]
// with c[t] = beta V[t] + (1 - beta) gate[t+1] x[t+1] (the membrane the reset removes).
template <bool GVT, int SG, bool ATT>
__global__ __launch_bounds__(64) void k_seq_bwd(SeqArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    int b, n;
    seq_work(b, n, a.N);
    const SeqLane L = seq_lane(a, n);
    const int N = a.N, T = a.T, TR = a.TR, lane = threadIdx.x;
    float *sV = reinterpret_cast<float *>(smem);
    float *sTh = sV + TR * 64;
    float *sA = sTh + TR * 64;
    float *sX = sA + TR * 64;
    float *sGS = sX + TR * 64;
    float *sGV = sGS + TR * 64;
    float *sGT = sGV + (GVT ? TR * 64 : 0);
    uint8_t *sF = reinterpret_cast<uint8_t *>(sGT + (GVT ? TR * 64 : 0));

    const size_t TN = (size_t)T * N;
    const rsrc_t rI = make_rsrc(a.I + b * TN, (uint32_t)(TN * 4));
    const rsrc_t rGS = make_rsrc(a.gS ? a.gS + b * TN : nullptr, a.gS ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGV = make_rsrc(a.gV ? a.gV + b * TN : nullptr, a.gV ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGT = make_rsrc(a.gTH ? a.gTH + b * TN : nullptr, a.gTH ? (uint32_t)(TN * 4) : 0u);
    const rsrc_t rGI = make_rsrc(a.gI ? a.gI + b * TN : nullptr, a.gI ? (uint32_t)(TN * 4) : 0u);
    const size_t CN = (size_t)a.NB * N;
    const int nc = L.valid ? n : N - 1;
    const float fbeta = (float)L.beta, fomb = (float)L.omb, fp = (float)L.p, fd = (float)L.d;

    // The attached adjoint couples lambda_V and lambda_a at every step where the
    // surrogate is nonzero and can grow by orders of magnitude (the wide
    // multi-Gaussian); in FP32 its rounding reaches ~1e-3 relative. That policy
    // therefore evaluates the surrogate, the coefficients, the recurrence and the
    // sums in FP64 from the FP32-staged V, theta, a and x.
    using R = typename std::conditional<ATT, double, float>::type;
    const R rbeta = ATT ? (R)L.beta : (R)fbeta, romb = ATT ? (R)L.omb : (R)fomb;
    const R rp = ATT ? (R)L.p : (R)fp, rd = ATT ? (R)L.d : (R)fd;
    R lamV = 0, lamA = 0;
    float x_next = 0.0f;   // attached: input (with bias) of the step after this block's last
    bool pass_next = false;
    double acc[5] = {0, 0, 0, 0, 0};
    constexpr int CH = 8;  // loads issued a chunk at a time
    for (int nb = a.NB - 1; nb >= 0; nb--) {
        double v = a.ck.v[b * CN + (size_t)nb * N + nc];
        double av = a.ck.a[b * CN + (size_t)nb * N + nc];
        int c = a.ck.c[b * CN + (size_t)nb * N + nc];
        bool sprev = c == 0;
        const float v_in = (float)v, a_in = (float)av;
        const int tb = nb * TR;
        const int len = min(TR, T - tb);
        for (int k0 = 0; k0 < len; k0 += CH) {
            float xs[CH], gs[CH], gv[CH], gt[CH];
#pragma unroll
            for (int i = 0; i < CH; i++) {
                const int k = k0 + i;
                const bool ok = L.valid && k < len;
                const uint32_t off = ok ? (uint32_t)((tb + k) * N + n) * 4u : ALIF_OOB;
                xs[i] = ld_f32(rI, off);
                gs[i] = ld_f32(rGS, off);
                if constexpr (GVT) { gv[i] = ld_f32(rGV, off); gt[i] = ld_f32(rGT, off); }
            }
#pragma unroll
            for (int i = 0; i < CH; i++) {
                const int k = k0 + i;
                if (k < len) {
                    const float x = xs[i] + L.bias;
                    double th;
                    bool pass;
                    const bool sp = sprev;
                    const bool s = seq_step(L, TR, x, v, av, c, sprev, th, pass);
                    const int q = k * 64 + lane;
                    sV[q] = (float)v;
                    sTh[q] = (float)th;
                    sA[q] = (float)av;
                    sX[q] = x;
                    sGS[q] = gs[i];
                    if constexpr (GVT) { sGV[q] = gv[i]; sGT[q] = gt[i]; }
                    sF[q] = (uint8_t)((s ? 1 : 0) | (pass ? 2 : 0) | (sp ? 4 : 0));
                }
            }
        }
        R pb = 0, pp = 0, pd = 0, pth = 0, pbias = 0;
        for (int k = len - 1; k >= 0; k--) {
            const int q = k * 64 + lane;
            const uint8_t f = sF[q];
            const bool s = f & 1, pass = f & 2, sp = f & 4;
            const float V = sV[q], th = sTh[q], av_k = sA[q], x = sX[q];
            R sg;
            if constexpr (ATT) sg = surrogate_grad_f64<SG>((double)V - (double)th, (double)a.slope);
            else sg = surrogate_grad<SG>(V - th, a.slope);
            R lamS = sGS[q];
            if constexpr (ATT) {
                // lamV, lamA still hold step t + 1's values here (0 after the last step)
                const float xn = k + 1 < len ? sX[q + 64] : x_next;
                const bool pn = k + 1 < len ? (sF[q + 64] & 2) != 0 : pass_next;
                const R c = rfma(rbeta, (R)V, pn ? romb * (R)xn : (R)0);
                lamS = rfma(-c, lamV, lamS + lamA);
            }
            const R gsk = lamS * sg;
            const R cV = (GVT ? (R)sGV[q] : (R)0) + gsk;
            const R lt = (GVT ? (R)sGT[q] : (R)0) - gsk;
            lamV = rfma(s ? (R)0 : rbeta, lamV, cV);
            lamA = rfma(rp, lamA, rd * lt);
            const bool gate = pass && !sp;
            const R gI = gate ? romb * lamV : (R)0;
            const float Vprev = k > 0 ? sV[q - 64] : v_in;
            const float aprev = k > 0 ? sA[q - 64] : a_in;
            pb = rfma(sp ? (R)0 : (R)(Vprev - (pass ? x : 0.0f)), lamV, pb);
            pp = rfma((R)aprev, lamA, pp);
            pd = rfma((R)av_k, lt, pd);
            pth += lt;
            pbias += gI;
            if (a.gI) st_f32(rGI, L.valid ? (uint32_t)((tb + k) * N + n) * 4u : ALIF_OOB, (float)gI);
            if constexpr (ATT) {
                if (k == 0) {
                    x_next = x;
                    pass_next = pass;
                }
            }
        }
        acc[0] += pb;
        acc[1] += pp;
        acc[2] += pd;
        acc[3] += pth;
        acc[4] += pbias;
    }
    if (L.valid) {
        const size_t BN = (size_t)a.B * N, i = (size_t)b * N + n;
        for (int q = 0; q < 5; q++) a.part[q * BN + i] = acc[q];
    }
}

#define ALIF_SEQ_DEPTH 16

hipError_t launch_seq_fwd(const SeqArgs &a, hipStream_t st) {
    const int grid = a.B * ((a.N + 63) / 64);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_seq_fwd<ALIF_SEQ_DEPTH>), dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_seq_step_fwd(SeqArgs a, hipStream_t st) {
    const int total = a.B * a.N;
    if (total == 0) return hipSuccess;
    for (int t = 0; t < a.T; t++) {
        a.step = t;
        hipLaunchKernelGGL(k_seq_step, dim3((total + 255) / 256), dim3(256), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// LDS holds one block of T_R steps x 64 neurons: V, theta, a, x, dL/dS (and dL/dV,
// dL/dtheta) in FP32 plus the step flags, within the 160 KiB of a gfx950 CU.
static size_t seq_bwd_lds_bytes(int TR, bool gvt) { return (size_t)TR * 64 * ((gvt ? 7 : 5) * sizeof(float) + 1); }
int seq_bwd_max_tr(bool gvt) { return (int)((size_t)160 * 1024 / seq_bwd_lds_bytes(1, gvt)); }

hipError_t launch_seq_bwd(const SeqArgs &a, hipStream_t st) {
    const int grid = a.B * ((a.N + 63) / 64);
    if (grid == 0) return hipSuccess;
    const bool gvt = a.gV || a.gTH;
    const size_t smem = seq_bwd_lds_bytes(a.TR, gvt);
#define ALIF_SB(G, A)                                                                             \
    do {                                                                                          \
        if (a.surrogate == 1) hipLaunchKernelGGL((k_seq_bwd<G, 1, A>), dim3(grid), dim3(64), smem, st, a); \
        else if (a.surrogate == 2) hipLaunchKernelGGL((k_seq_bwd<G, 2, A>), dim3(grid), dim3(64), smem, st, a); \
        else hipLaunchKernelGGL((k_seq_bwd<G, 0, A>), dim3(grid), dim3(64), smem, st, a);        \
    } while (0)
    if (a.attached) {
        if (gvt) ALIF_SB(true, true);
        else ALIF_SB(false, true);
    } else {
        if (gvt) ALIF_SB(true, false);
        else ALIF_SB(false, false);
    }
#undef ALIF_SB
    return hipGetLastError();
}

}  // namespace alif
