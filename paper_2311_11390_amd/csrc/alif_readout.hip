// Leaky non-spiking readout (paper supplementary, "Readout neurons"):
//   I_r = W_r S,  V_r[t] = beta_r V_r[t-1] + (1 - beta_r) I_r[t],  o = sum_t V_r[t],
// beta_r = exp(-DT / tau_r). The projection runs on the MFMA GEMM; the
// integration runs in FP64, each (batch, readout neuron) row on 16 threads that take
// a chunk of time each and join their carries through LDS.
// Workspace layout (kept by the caller from forward to backward):
//   I_r [B*T][C] f32 | V_r [B*T][C] f32 | gI_r [B*T][C] f32 | part [B][C] f64 | GEMM split scratch
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/blockalif.h"
#include "alif_common.h"
#include "alif_gemm.h"
#include "alif_kernels.h"

namespace alif {
namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct RoWs {
    float *Ir, *Vr, *gIr;
    double *part;
    void *gemm;
};
RoWs ro_ws(void *ws, int B, int T, int C) {
    const size_t mc = (size_t)B * T * C * sizeof(float);
    char *p = (char *)ws;
    RoWs w;
    w.Ir = (float *)p;
    w.Vr = (float *)(p + a256(mc));
    w.gIr = (float *)(p + 2 * a256(mc));
    w.part = (double *)(p + 3 * a256(mc));
    w.gemm = p + 3 * a256(mc) + a256((size_t)B * C * sizeof(double));
    return w;
}

// Each (b, c) row's recurrence over T is cut into RK chunks of Lc = ceil(T / RK)
// steps. A workgroup holds batch element b = blockIdx.x and CG classes (blockIdx.y
// picks which): thread (k, cl) = (tid / CG, tid % CG) takes chunk k of class cl,
// so consecutive threads read consecutive classes of one step. A chunk first runs
// from zero to get its local end value; through LDS every thread then forms its
// true carry-in,
//   V_in(k) = sum over k' < k of beta^(Lc (k - 1 - k')) e(k')   (Horner over k'),
// and reruns its chunk from it, writing V_r and summing it; the chunk sums are added
// in chunk order. Loads go 32 steps at a time. The backward is the same with the
// reverse recurrence (its local pass needs no loads) and the carry from the chunks
// after. Every chunk before the last non-empty one is full, so beta^Lc is the only
// decay across chunks.
constexpr int RK = 16;   // chunks a row
constexpr int RU = 32;   // steps whose loads are issued together
constexpr int RCG = 32;  // classes a workgroup at most (512 threads: no register spills)

// Run v <- beta v + omb I[t] over t in [t0, t1) from v; with STORE, write V_r and sum v.
template <bool STORE>
__device__ __forceinline__ double run_fwd(const float *__restrict__ ir, float *__restrict__ vr, int C, int t0,
                                          int t1, double beta, double omb, double v, double &sum) {
    for (int tb = t0; tb < t1; tb += RU) {
        float x[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) x[u] = tb + u < t1 ? ir[(size_t)(tb + u) * C] : 0.0f;
#pragma unroll
        for (int u = 0; u < RU; u++)
            if (tb + u < t1) {
                v = fma(beta, v, omb * (double)x[u]);
                if constexpr (STORE) {
                    vr[(size_t)(tb + u) * C] = (float)v;
                    sum += v;
                }
            }
    }
    return v;
}

__global__ __launch_bounds__(RK * RCG) void k_readout_fwd(int B, int T, int C, double dt,
                                                          const float *__restrict__ tau_r,
                                                          const float *__restrict__ Ir, float *__restrict__ Vr,
                                                          float *__restrict__ o) {
    __shared__ double sh[RK][RCG];
    const int CG = blockDim.x / RK;
    const int k = threadIdx.x / CG, cl = threadIdx.x - k * CG;
    const int b = blockIdx.x, c = blockIdx.y * CG + cl;
    const bool ok = c < C;
    const double lb = -dt / (double)tau_r[ok ? c : 0];
    const double beta = exp(lb), omb = -expm1(lb);
    const int Lc = (T + RK - 1) / RK;
    const int t0 = min(T, k * Lc), t1 = min(T, t0 + Lc);
    const float *ir = Ir + (size_t)b * T * C + c;
    float *vr = Vr + (size_t)b * T * C + c;
    double unused = 0.0;
    sh[k][cl] = ok ? run_fwd<false>(ir, vr, C, t0, t1, beta, omb, 0.0, unused) : 0.0;
    __syncthreads();
    const double dk = exp(lb * (double)Lc);
    double vin = 0.0;
    for (int kk = 0; kk < k; kk++) vin = fma(dk, vin, sh[kk][cl]);
    double sum = 0.0;
    if (ok) run_fwd<true>(ir, vr, C, t0, t1, beta, omb, vin, sum);
    __syncthreads();
    sh[k][cl] = sum;
    __syncthreads();
    if (ok && k == 0) {
        double tot = 0.0;
        for (int kk = 0; kk < RK; kk++) tot += sh[kk][cl];
        o[(size_t)b * C + c] = (float)tot;
    }
}

// Run lam <- g + beta lam over t = t1 - 1 down to t0 from lam; with ACC, write gI_r
// and accumulate d/dbeta (V_r[t - 1] - I_r[t]) lam.
template <bool ACC>
__device__ __forceinline__ double run_bwd(const float *__restrict__ ir, const float *__restrict__ vr,
                                          float *__restrict__ gi, int C, int t0, int t1, double beta, double omb,
                                          double g, double lam, double &gb) {
    for (int tb = t1 - 1; tb >= t0; tb -= RU) {
        float xi[RU], xv[RU];
        if constexpr (ACC) {
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int t = tb - u;
                xi[u] = t >= t0 ? ir[(size_t)t * C] : 0.0f;
                xv[u] = (t >= t0 && t > 0) ? vr[(size_t)(t - 1) * C] : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int t = tb - u;
            if (t >= t0) {
                lam = fma(beta, lam, g);
                if constexpr (ACC) {
                    gi[(size_t)t * C] = (float)(omb * lam);
                    gb = fma((double)xv[u] - (double)xi[u], lam, gb);
                }
            }
        }
    }
    return lam;
}

// reverse recurrence lam[t] = go + beta lam[t+1]; gI_r[t] = (1 - beta) lam[t];
// d/dbeta = sum_t (V_r[t-1] - I_r[t]) lam[t]
__global__ __launch_bounds__(RK * RCG) void k_readout_bwd(int B, int T, int C, double dt,
                                                          const float *__restrict__ tau_r,
                                                          const float *__restrict__ Ir, const float *__restrict__ Vr,
                                                          const float *__restrict__ go, float *__restrict__ gIr,
                                                          double *__restrict__ part) {
    __shared__ double sh[RK][RCG];
    const int CG = blockDim.x / RK;
    const int k = threadIdx.x / CG, cl = threadIdx.x - k * CG;
    const int b = blockIdx.x, c = blockIdx.y * CG + cl;
    const bool ok = c < C;
    const double lb = -dt / (double)tau_r[ok ? c : 0];
    const double beta = exp(lb), omb = -expm1(lb);
    const double g = ok ? (double)go[(size_t)b * C + c] : 0.0;
    const int Lc = (T + RK - 1) / RK;
    const int t0 = min(T, k * Lc), t1 = min(T, t0 + Lc);
    const size_t base = (size_t)b * T * C + c;
    const float *ir = Ir + base, *vr = Vr + base;
    float *gi = gIr + base;
    double unused = 0.0;
    // lambda at this chunk's first step from a zero carry at its end
    sh[k][cl] = ok ? run_bwd<false>(ir, vr, gi, C, t0, t1, beta, omb, g, 0.0, unused) : 0.0;
    __syncthreads();
    // the carry at this chunk's end: the later chunks' values, Horner from the last
    const double dk = exp(lb * (double)Lc);
    double lin = 0.0;
    for (int kk = RK - 1; kk > k; kk--) lin = fma(dk, lin, sh[kk][cl]);
    double gb = 0.0;
    if (ok) run_bwd<true>(ir, vr, gi, C, t0, t1, beta, omb, g, lin, gb);
    __syncthreads();
    sh[k][cl] = gb;
    __syncthreads();
    if (ok && k == 0) {
        double tot = 0.0;
        for (int kk = 0; kk < RK; kk++) tot += sh[kk][cl];
        part[(size_t)b * C + c] = tot;
    }
}

__global__ void k_readout_tau(int B, int C, double dt, const float *tau_r, const double *part, float *g_tau) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int b = 0; b < B; b++) s += part[(size_t)b * C + c];
    const double tau = tau_r[c];
    g_tau[c] = (float)(s * exp(-dt / tau) * dt / (tau * tau));
}

int dt_code(int spike_dtype) { return spike_dtype == ALIF_SPIKES_U8 ? 1 : (spike_dtype == ALIF_SPIKES_BF16 ? 2 : 0); }

int wsplits(long long M, int N, int K) {
    const long long tiles = (long long)((N + 127) / 128) * ((K + 127) / 128);
    long long s = 512 / (tiles > 0 ? tiles : 1);
    s = s < 1 ? 1 : (s > 64 ? 64 : s);
    if (s > M / 256) s = M / 256 < 1 ? 1 : M / 256;
    return (int)s;
}

}  // namespace
}  // namespace alif

using namespace alif;

extern "C" {

int alif_readout_workspace_bytes(int32_t B, int32_t T, int32_t n_hidden, int32_t C, size_t *bytes) {
    if (B < 0 || T < 0 || n_hidden <= 0 || C <= 0 || !bytes) return alif::set_error(ALIF_EINVAL, "bad readout sizes");
    const size_t mc = (size_t)B * T * C * sizeof(float);
    const long long M = (long long)B * T;
    const int s = wsplits(M, C, n_hidden);
    *bytes = 3 * a256(mc) + a256((size_t)B * C * sizeof(double)) +
             (s > 1 ? (size_t)s * C * n_hidden * sizeof(float) : 0);
    return ALIF_OK;
}

int alif_readout_forward(int32_t B, int32_t T, int32_t n_hidden, int32_t C, double dt_ms,
                         int32_t spike_dtype, const void *spikes, const float *W_r,
                         const float *tau_r, float *o, void *workspace, void *stream) {
    if (B < 0 || T < 0 || n_hidden <= 0 || C <= 0 || !(dt_ms > 0))
        return alif::set_error(ALIF_EINVAL, "bad readout sizes or dt");
    if (spike_dtype < ALIF_SPIKES_U8 || spike_dtype > ALIF_SPIKES_F32)
        return alif::set_error(ALIF_EINVAL, "unknown spike_dtype");
    if (!spikes || !W_r || !tau_r || !o || !workspace)
        return alif::set_error(ALIF_EINVAL, "NULL readout argument");
    if ((C + RCG - 1) / RCG > 65535)
        return alif::set_error(ALIF_EUNSUPPORTED, "too many readout neurons (C / 32 must stay within 65535)");
    hipStream_t st = (hipStream_t)stream;
    RoWs w = ro_ws(workspace, B, T, C);
    GemmArgs g{};
    g.M = (long long)B * T; g.N = C; g.K = n_hidden;
    g.A = spikes; g.a_dt = dt_code(spike_dtype); g.lda = n_hidden; g.a_kc = 1;
    g.B = W_r; g.b_dt = 0; g.ldb = n_hidden; g.b_kc = 1;
    g.C = w.Ir; g.ldc = C; g.splits = 1;
    hipError_t e = gemm_launch(g, false, st);
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    if (B == 0) return ALIF_OK;
    const int cg = C < RCG ? C : RCG;
    hipLaunchKernelGGL(k_readout_fwd, dim3((unsigned)B, (unsigned)((C + cg - 1) / cg)), dim3(RK * cg), 0, st, B, T,
                       C, dt_ms, tau_r, w.Ir, w.Vr, o);
    e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

int alif_readout_backward(int32_t B, int32_t T, int32_t n_hidden, int32_t C, double dt_ms,
                          int32_t spike_dtype, const void *spikes, const float *W_r,
                          const float *tau_r, const float *go, float *grad_spikes,
                          float *grad_W_r, float *grad_tau_r, void *workspace, void *stream) {
    if (B < 0 || T < 0 || n_hidden <= 0 || C <= 0 || !(dt_ms > 0))
        return alif::set_error(ALIF_EINVAL, "bad readout sizes or dt");
    if (!spikes || !W_r || !tau_r || !go || !workspace)
        return alif::set_error(ALIF_EINVAL, "NULL readout argument");
    if ((C + RCG - 1) / RCG > 65535)
        return alif::set_error(ALIF_EUNSUPPORTED, "too many readout neurons (C / 32 must stay within 65535)");
    hipStream_t st = (hipStream_t)stream;
    RoWs w = ro_ws(workspace, B, T, C);
    if (B > 0) {
        const int cg = C < RCG ? C : RCG;
        hipLaunchKernelGGL(k_readout_bwd, dim3((unsigned)B, (unsigned)((C + cg - 1) / cg)), dim3(RK * cg), 0, st, B,
                           T, C, dt_ms, tau_r, w.Ir, w.Vr, go, w.gIr, w.part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    if (grad_tau_r) {
        hipLaunchKernelGGL(k_readout_tau, dim3((C + 127) / 128), dim3(128), 0, st, B, C, dt_ms, tau_r,
                           w.part, grad_tau_r);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    const long long M = (long long)B * T;
    if (grad_spikes) {  // gS[m][h] = sum_c gI_r[m][c] W_r[c][h]
        GemmArgs g{};
        g.M = M; g.N = n_hidden; g.K = C;
        g.A = w.gIr; g.a_dt = 0; g.lda = C; g.a_kc = 1;
        g.B = W_r; g.b_dt = 0; g.ldb = n_hidden; g.b_kc = 0;
        g.C = grad_spikes; g.ldc = n_hidden; g.splits = 1;
        hipError_t e = gemm_launch(g, false, st);
        if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    if (grad_W_r) {  // gW_r[c][h] = sum_m gI_r[m][c] S[m][h]
        if (M > 0x7fffffff) return alif::set_error(ALIF_EUNSUPPORTED, "B*T too large");
        GemmArgs g{};
        g.M = C; g.N = n_hidden; g.K = (int)M;
        g.A = w.gIr; g.a_dt = 0; g.lda = C; g.a_kc = 0;
        g.B = spikes; g.b_dt = dt_code(spike_dtype); g.ldb = n_hidden; g.b_kc = 0;
        g.C = grad_W_r; g.ldc = n_hidden;
        g.splits = wsplits(M, C, n_hidden);
        g.C_part = (float *)w.gemm;
        hipError_t e = gemm_launch(g, false, st);
        if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    return ALIF_OK;
}

}  // extern "C"
