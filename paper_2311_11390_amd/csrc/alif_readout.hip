// Leaky non-spiking readout (paper supplementary, "Readout neurons"):
//   I_r = W_r S,  V_r[t] = beta_r V_r[t-1] + (1 - beta_r) I_r[t],  o = sum_t V_r[t],
// beta_r = exp(-DT / tau_r). The projection runs on the MFMA GEMM; the
// integration is one thread per (batch, readout neuron) in FP64, its loads issued a
// chunk of steps ahead.
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

// One thread per (b, c) runs the recurrence over T in FP64. The loads of I_r (and,
// backward, of V_r) for the next RU steps are issued before this chunk's
// arithmetic, so the loop waits for a chunk of loads once instead of one L2 round
// trip per step; the arithmetic and its order are the plain recurrence's.
constexpr int RU = 32;

__global__ __launch_bounds__(64) void k_readout_fwd(int B, int T, int C, double dt, const float *__restrict__ tau_r,
                                                    const float *__restrict__ Ir, float *__restrict__ Vr,
                                                    float *__restrict__ o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * C) return;
    const int b = i / C, c = i - b * C;
    const double lb = -dt / (double)tau_r[c];
    const double beta = exp(lb), omb = -expm1(lb);
    const float *ir = Ir + (size_t)b * T * C + c;
    float *vr = Vr + (size_t)b * T * C + c;
    double v = 0.0, sum = 0.0;
    float nxt[RU];
#pragma unroll
    for (int u = 0; u < RU; u++) nxt[u] = u < T ? ir[(size_t)u * C] : 0.0f;
    for (int t0 = 0; t0 < T; t0 += RU) {
        float cur[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) cur[u] = nxt[u];
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int t = t0 + RU + u;
            nxt[u] = t < T ? ir[(size_t)t * C] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int t = t0 + u;
            if (t < T) {
                v = fma(beta, v, omb * (double)cur[u]);
                vr[(size_t)t * C] = (float)v;
                sum += v;
            }
        }
    }
    o[i] = (float)sum;
}

// reverse recurrence lam[t] = go + beta lam[t+1]; gI_r[t] = (1 - beta) lam[t];
// d/dbeta = sum_t (V_r[t-1] - I_r[t]) lam[t]
__global__ __launch_bounds__(64) void k_readout_bwd(int B, int T, int C, double dt, const float *__restrict__ tau_r,
                                                    const float *__restrict__ Ir, const float *__restrict__ Vr,
                                                    const float *__restrict__ go, float *__restrict__ gIr,
                                                    double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * C) return;
    const int b = i / C, c = i - b * C;
    const double lb = -dt / (double)tau_r[c];
    const double beta = exp(lb), omb = -expm1(lb);
    const double g = go[i];
    const size_t base = (size_t)b * T * C + c;
    const float *ir = Ir + base, *vr = Vr + base;
    float *gi = gIr + base;
    double lam = 0.0, gb = 0.0;
    // steps t = t0 - u of a chunk, last to first; V_r[t - 1] is 0 at t = 0
    float ni[RU], nv[RU];
#pragma unroll
    for (int u = 0; u < RU; u++) {
        const int t = T - 1 - u;
        ni[u] = t >= 0 ? ir[(size_t)t * C] : 0.0f;
        nv[u] = t > 0 ? vr[(size_t)(t - 1) * C] : 0.0f;
    }
    for (int t0 = T - 1; t0 >= 0; t0 -= RU) {
        float ci[RU], cv[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) {
            ci[u] = ni[u];
            cv[u] = nv[u];
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int t = t0 - RU - u;
            ni[u] = t >= 0 ? ir[(size_t)t * C] : 0.0f;
            nv[u] = t > 0 ? vr[(size_t)(t - 1) * C] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int t = t0 - u;
            if (t >= 0) {
                lam = fma(beta, lam, g);
                gi[(size_t)t * C] = (float)(omb * lam);
                gb = fma((double)cv[u] - (double)ci[u], lam, gb);
            }
        }
    }
    part[i] = gb;
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
    hipStream_t st = (hipStream_t)stream;
    RoWs w = ro_ws(workspace, B, T, C);
    GemmArgs g{};
    g.M = (long long)B * T; g.N = C; g.K = n_hidden;
    g.A = spikes; g.a_dt = dt_code(spike_dtype); g.lda = n_hidden; g.a_kc = 1;
    g.B = W_r; g.b_dt = 0; g.ldb = n_hidden; g.b_kc = 1;
    g.C = w.Ir; g.ldc = C; g.splits = 1;
    hipError_t e = gemm_launch(g, false, st);
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    if (B * C == 0) return ALIF_OK;
    hipLaunchKernelGGL(k_readout_fwd, dim3((B * C + 63) / 64), dim3(64), 0, st, B, T, C, dt_ms, tau_r,
                       w.Ir, w.Vr, o);
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
    hipStream_t st = (hipStream_t)stream;
    RoWs w = ro_ws(workspace, B, T, C);
    if (B * C > 0) {
        hipLaunchKernelGGL(k_readout_bwd, dim3((B * C + 63) / 64), dim3(64), 0, st, B, T, C, dt_ms,
                           tau_r, w.Ir, w.Vr, go, w.gIr, w.part);
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
