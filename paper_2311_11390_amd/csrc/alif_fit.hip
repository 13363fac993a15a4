// Neural-fit loss and optimiser step (paper supplementary, "Neural fits").
//
// Van Rossum distance, supplementary "Supervised training loss": for a model train
// x and a target train y on the simulation grid,
//   e[t] = sum_{s <= t} a^(t - s) (x[s] - y[s]),   a = exp(-DT / tau_R),
//   D    = sqrt((DT / tau_R) sum_t e[t]^2),
//   dD/dx[s] = (DT / (tau_R D)) sum_{t >= s} a^(t - s) e[t]   (0 where D = 0).
// Both sums are first-order linear recurrences along time, so the time axis is
// cut into chunks that run in parallel and are stitched by their carries:
//   k_vr_chunks  one thread per (b, chunk, 1 or 4 neurons): runs e from a zero
//                carry over its chunk and keeps, per repeat, the end value E, the
//                sums P = sum e_loc^2 and Q = sum a^(j+1) e_loc[t0 + j] (FP64),
//                plus e_loc every 16 steps (checkpoints). With the true carry C
//                into the chunk, e = e_loc + a^(j+1) C, so the chunk adds
//                P + 2 C Q + C^2 G to sum e^2, G = sum_{j=1..L} a^(2j).
//   k_vr_combine one thread per (b, repeat, neuron): walks the chunks left to
//                right for the carries of e and for D, then right to left for
//                the carries of the reverse recurrence g[s] = e[s] + a g[s + 1].
//   k_vr_grad    one thread per (b, chunk, 1 or 4 neurons): the gradient is the
//                reverse recurrence of c = sum_r w_r e_r, w_r = scale DT /
//                (tau_R D_r), so the carries combine with the same weights. It
//                walks its chunk's 16-step pieces last to first; each piece
//                rebuilds c forward from its checkpoint into registers, then runs
//                g backward and stores it.
// Data read: the spike bytes twice (x once per group of up to four repeats in
// the first pass), the gradient written once; checkpoints and chunk sums add
// about 4 R / 16 bytes per element each way.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/blockalif.h"
#include "alif_common.h"
#include "alif_kernels.h"

namespace alif {
namespace {

constexpr int VR_SUB = 16;          // steps per checkpointed piece
constexpr int VR_MAX_R = 8;         // repeats per model train (the error messages say 8)
#ifndef ALIF_VR_THREADS_LOG2
#define ALIF_VR_THREADS_LOG2 17   // threads the chunking aims at
#endif
constexpr long long VR_TARGET_THREADS = 1LL << ALIF_VR_THREADS_LOG2;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct VrPlan {
    int vec, ng, K, Lc, S;          // neurons per thread, thread columns per row, chunks, chunk length, pieces
    size_t off_sum, off_cp, off_w, off_ce, off_cg, total;
};

VrPlan vr_plan(int B, int R, int T, int N) {
    VrPlan p{};
    p.vec = (N % 4 == 0) ? 4 : 1;
    p.ng = N / p.vec;
    const long long cols = (long long)B * p.ng;
    const int max_k = (T + VR_SUB - 1) / VR_SUB;
    long long K = cols > 0 ? (VR_TARGET_THREADS + cols - 1) / cols : 1;
    if (K > max_k) K = max_k;
    if (K < 1) K = 1;
    int Lc = (int)((T + K - 1) / K);
    Lc = (Lc + VR_SUB - 1) / VR_SUB * VR_SUB;
    if (Lc < VR_SUB) Lc = VR_SUB;
    p.Lc = Lc;
    p.K = T > 0 ? (T + Lc - 1) / Lc : 0;
    p.S = Lc / VR_SUB;
    const size_t bkn = (size_t)B * p.K * N;
    p.off_sum = 0;
    p.off_cp = a256(bkn * R * 3 * sizeof(double));
    p.off_w = p.off_cp + a256(bkn * p.S * R * sizeof(float));
    p.off_ce = p.off_w + a256((size_t)B * R * N * sizeof(float));
    p.off_cg = p.off_ce + a256(bkn * R * sizeof(double));
    p.total = p.off_cg + a256(bkn * R * sizeof(double));
    return p;
}

template <int VEC>
struct Bytes;
template <>
struct Bytes<4> {
    using W = uint32_t;
    __device__ static float get(W w, int v) { return (float)((w >> (8 * v)) & 0xffu); }
};
template <>
struct Bytes<1> {
    using W = uint8_t;
    __device__ static float get(W w, int) { return (float)w; }
};

template <int VEC>
__device__ __forceinline__ typename Bytes<VEC>::W load_w(const uint8_t *p, size_t e) {
    return *reinterpret_cast<const typename Bytes<VEC>::W *>(p + e);
}

// Summaries of one chunk for repeats [r0, r0 + RG).
template <int VEC, int RG>
__global__ void __launch_bounds__(256) k_vr_chunks(int B, int R, int r0, int T, int N, int ng, int K, int Lc,
                                                   int S, double a, const uint8_t *__restrict__ x,
                                                   const uint8_t *__restrict__ y, double *__restrict__ sums,
                                                   float *__restrict__ cp) {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long long)B * K * ng) return;
    const int j = (int)(tid % ng);
    tid /= ng;
    const int k = (int)(tid % K);
    const int b = (int)(tid / K);
    const int n0 = j * VEC;
    const int t0 = k * Lc, t1 = min(T, t0 + Lc);
    double c[RG][VEC], P[RG][VEC], Q[RG][VEC];
#pragma unroll
    for (int r = 0; r < RG; r++)
#pragma unroll
        for (int v = 0; v < VEC; v++) c[r][v] = P[r][v] = Q[r][v] = 0.0;
    double ap = 1.0;
    const size_t xrow = (size_t)b * T * N + n0;
    const size_t ytr = (size_t)T * N;
    const size_t yrow = ((size_t)b * R + r0) * ytr + n0;
    for (int s = 0; t0 + s * VR_SUB < t1; s++) {
        const int ts = t0 + s * VR_SUB;
        const int len = min(VR_SUB, t1 - ts);
        if (s > 0) {
#pragma unroll
            for (int r = 0; r < RG; r++) {
                float *o = cp + ((((size_t)b * K + k) * S + s) * R + r0 + r) * N + n0;
#pragma unroll
                for (int v = 0; v < VEC; v++) o[v] = (float)c[r][v];
            }
        }
        typename Bytes<VEC>::W wx[VR_SUB], wy[RG][VR_SUB];
#pragma unroll
        for (int i = 0; i < VR_SUB; i++) {
            const int t = i < len ? ts + i : ts;
            wx[i] = load_w<VEC>(x, xrow + (size_t)t * N);
#pragma unroll
            for (int r = 0; r < RG; r++) wy[r][i] = load_w<VEC>(y, yrow + r * ytr + (size_t)t * N);
        }
#pragma unroll
        for (int i = 0; i < VR_SUB; i++) {
            if (i < len) {
                ap *= a;
#pragma unroll
                for (int r = 0; r < RG; r++)
#pragma unroll
                    for (int v = 0; v < VEC; v++) {
                        const double z = (double)(Bytes<VEC>::get(wx[i], v) - Bytes<VEC>::get(wy[r][i], v));
                        c[r][v] = fma(a, c[r][v], z);
                        P[r][v] = fma(c[r][v], c[r][v], P[r][v]);
                        Q[r][v] = fma(ap, c[r][v], Q[r][v]);
                    }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RG; r++) {
        double *o = sums + ((((size_t)b * K + k) * R + r0 + r) * 3) * N + n0;
#pragma unroll
        for (int v = 0; v < VEC; v++) {
            o[v] = c[r][v];
            o[N + v] = P[r][v];
            o[2 * N + v] = Q[r][v];
        }
    }
}

// Per (b, repeat, neuron): the distance, the repeat's weight w_r, and per chunk
// k the carries of e_r and of g_r = sum_{t >= s} a^(t - s) e_r[t] (unweighted;
// the gradient kernel forms sum_r w_r of both). All chunks but the last have
// length Lc: their decay a^Lc and sum G are passed in (aL, G; aLl, Gl for the last).
__global__ void __launch_bounds__(256) k_vr_combine(int B, int R, int N, int K, double a, double aL, double G,
                                                    double aLl, double Gl, double dt_over_tau, double scale,
                                                    const double *__restrict__ sums, float *__restrict__ dist,
                                                    float *__restrict__ wts, double *__restrict__ ce,
                                                    double *__restrict__ cg, int want_grad) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)B * R * N) return;
    const int n = (int)(i % N);
    const int r = (int)((i / N) % R);
    const int b = (int)(i / ((long long)N * R));
    const size_t kstride = (size_t)R * 3 * N;
    const double *col = sums + (size_t)b * K * kstride + (size_t)(3 * r) * N + n;   // [k][r][E, P, Q][N]
    double *cec = ce + ((size_t)b * K * R + r) * N + n;                           // [b][k][r][N]
    double *cgc = cg + ((size_t)b * K * R + r) * N + n;
    const size_t ko = (size_t)R * N;
    double C = 0.0, D2 = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; k++) {
        const bool last = k == K - 1;
        const double *s = col + k * kstride;
        const double E = s[0], P = s[N], Q = s[2 * N];
        if (want_grad) cec[k * ko] = C;
        D2 += P + 2.0 * C * Q + C * C * (last ? Gl : G);
        C = fma(last ? aLl : aL, C, E);
    }
    const double d = sqrt(fmax(0.0, dt_over_tau * D2));
    if (dist) dist[((size_t)b * R + r) * N + n] = (float)d;
    if (!want_grad) return;
    wts[((size_t)b * R + r) * N + n] = d > 0.0 ? (float)(scale * dt_over_tau / d) : 0.0f;
    // g_r at the first step of each chunk, from the right:
    // g[t0] = sum_j a^j e[t0 + j] + a^L g[t0 + L], sum_j a^j e[t0 + j] = (Q + G C) / a
    const double inv_a = 1.0 / a;
    double g = 0.0;
#pragma unroll 4
    for (int k = K - 1; k >= 0; k--) {
        const bool last = k == K - 1;
        const double A = (col[k * kstride + 2 * N] + (last ? Gl : G) * cec[k * ko]) * inv_a;
        cgc[k * ko] = g;
        g = fma(last ? aLl : aL, g, A);
    }
}

// RM: compile-time bound on the repeats (4 or 8), so that the weights and one
// piece's target words sit in registers and every load of a piece is issued
// before its arithmetic.
template <int VEC, int RM>
__global__ void __launch_bounds__(256) k_vr_grad(int B, int R, int T, int N, int ng, int K, int Lc, int S,
                                                 double lna, const uint8_t *__restrict__ x,
                                                 const uint8_t *__restrict__ y, const float *__restrict__ wts,
                                                 const double *__restrict__ ce, const double *__restrict__ cg,
                                                 const float *__restrict__ cp, float *__restrict__ grad) {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long long)B * K * ng) return;
    const int j = (int)(tid % ng);
    tid /= ng;
    const int k = (int)(tid % K);
    const int b = (int)(tid / K);
    const int n0 = j * VEC;
    const int t0 = k * Lc, t1 = min(T, t0 + Lc);
    const float a = (float)exp(lna);
    float w[RM][VEC], W[VEC];
#pragma unroll
    for (int v = 0; v < VEC; v++) W[v] = 0.f;
#pragma unroll
    for (int r = 0; r < RM; r++)
#pragma unroll
        for (int v = 0; v < VEC; v++) {
            w[r][v] = r < R ? wts[((size_t)b * R + r) * N + n0 + v] : 0.f;
            W[v] += w[r][v];
        }
    // carries into this chunk of c = sum_r w_r e_r and of g = sum_r w_r g_r
    double cmk[VEC];
    float g[VEC];
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const size_t o = ((size_t)b * K + k) * R * N + n0 + v;
        double cc = 0.0, gg = 0.0;
#pragma unroll
        for (int r = 0; r < RM; r++)
            if (r < R) {
                cc = fma((double)w[r][v], ce[o + (size_t)r * N], cc);
                gg = fma((double)w[r][v], cg[o + (size_t)r * N], gg);
            }
        cmk[v] = cc;
        g[v] = (float)gg;
    }
    const size_t xrow = (size_t)b * T * N + n0;
    const size_t ytr = (size_t)T * N;
    const size_t yrow = (size_t)b * R * ytr + n0;
    const int s_last = (t1 - t0 - 1) / VR_SUB;
    const double inv_a16 = exp(-(double)VR_SUB * lna);
    double pw = exp((double)(s_last * VR_SUB) * lna);   // a^(16 s), divided by a^16 per piece
    for (int s = s_last; s >= 0; s--, pw *= inv_a16) {
        const int ts = t0 + s * VR_SUB;
        const int len = min(VR_SUB, t1 - ts);
        // all loads of the piece first: model spikes, every target, the checkpoints
        typename Bytes<VEC>::W wx[VR_SUB], wy[RM][VR_SUB];
#pragma unroll
        for (int i = 0; i < VR_SUB; i++) {
            const int t = i < len ? ts + i : ts;
            wx[i] = load_w<VEC>(x, xrow + (size_t)t * N);
#pragma unroll
            for (int r = 0; r < RM; r++)
                wy[r][i] = r < R ? load_w<VEC>(y, yrow + r * ytr + (size_t)t * N) : (typename Bytes<VEC>::W)0;
        }
        float c[VEC];
#pragma unroll
        for (int v = 0; v < VEC; v++) {
            double cc = pw * cmk[v];
            if (s > 0) {
                const float *q = cp + (((size_t)b * K + k) * S + s) * R * N + n0 + v;
#pragma unroll
                for (int r = 0; r < RM; r++)
                    if (r < R) cc = fma((double)w[r][v], (double)q[(size_t)r * N], cc);
            }
            c[v] = (float)cc;
        }
        // drive m[t] = W x[t] - sum_r w_r y_r[t], then c[t] in place
        float cs[VR_SUB][VEC];
#pragma unroll
        for (int i = 0; i < VR_SUB; i++)
#pragma unroll
            for (int v = 0; v < VEC; v++) {
                float m = W[v] * Bytes<VEC>::get(wx[i], v);
#pragma unroll
                for (int r = 0; r < RM; r++) m = fmaf(-w[r][v], Bytes<VEC>::get(wy[r][i], v), m);
                c[v] = fmaf(a, c[v], m);
                cs[i][v] = c[v];
            }
#pragma unroll
        for (int i = VR_SUB - 1; i >= 0; i--) {
            if (i < len) {
                float o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; v++) {
                    g[v] = fmaf(a, g[v], cs[i][v]);
                    o[v] = g[v];
                }
                float *dst = grad + xrow + (size_t)(ts + i) * N;
                if constexpr (VEC == 4)
                    *reinterpret_cast<float4 *>(dst) = make_float4(o[0], o[1], o[2], o[3]);
                else
                    dst[0] = o[0];
            }
        }
    }
}

template <int VEC, int RG>
hipError_t launch_chunks(const VrPlan &p, int B, int R, int r0, int T, int N, double a, const uint8_t *x,
                         const uint8_t *y, double *sums, float *cp, hipStream_t st) {
    const long long n = (long long)B * p.K * p.ng;
    hipLaunchKernelGGL((k_vr_chunks<VEC, RG>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, R, r0, T, N,
                       p.ng, p.K, p.Lc, p.S, a, x, y, sums, cp);
    return hipGetLastError();
}

template <int VEC>
hipError_t launch_chunks_rg(int rg, const VrPlan &p, int B, int R, int r0, int T, int N, double a,
                            const uint8_t *x, const uint8_t *y, double *sums, float *cp, hipStream_t st) {
    switch (rg) {
        case 1: return launch_chunks<VEC, 1>(p, B, R, r0, T, N, a, x, y, sums, cp, st);
        case 2: return launch_chunks<VEC, 2>(p, B, R, r0, T, N, a, x, y, sums, cp, st);
        case 3: return launch_chunks<VEC, 3>(p, B, R, r0, T, N, a, x, y, sums, cp, st);
        default: return launch_chunks<VEC, 4>(p, B, R, r0, T, N, a, x, y, sums, cp, st);
    }
}

__global__ void __launch_bounds__(256) k_fill_zero(long long n, float *__restrict__ p) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void __launch_bounds__(256) k_adam(int n, float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float b1, float omb1,
                                              float b2, float omb2, float lr_c1, float inv_c2, float eps, float lo,
                                              float hi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], omb1 * gi);
    const float vi = fmaf(b2, v[i], omb2 * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float q = p[i] - lr_c1 * mi / (sqrtf(vi * inv_c2) + eps);
    p[i] = fminf(fmaxf(q, lo), hi);
}

}  // namespace
}  // namespace alif

using namespace alif;

extern "C" {

int alif_van_rossum_workspace_bytes(int32_t B, int32_t R, int32_t T, int32_t N, size_t *bytes) {
    if (B < 0 || R < 1 || T < 0 || N < 0 || !bytes) return alif::set_error(ALIF_EINVAL, "bad van Rossum sizes");
    if (R > VR_MAX_R) return alif::set_error(ALIF_EUNSUPPORTED, "van Rossum: at most 8 repeats");
    *bytes = vr_plan(B, R, T, N).total;
    return ALIF_OK;
}

int alif_van_rossum(int32_t B, int32_t R, int32_t T, int32_t N, double dt_ms, double tau_ms,
                    const uint8_t *spikes, const uint8_t *targets, float scale, float *dist, float *grad,
                    void *workspace, void *stream) {
    if (B < 0 || R < 1 || T < 0 || N < 0) return alif::set_error(ALIF_EINVAL, "bad van Rossum sizes");
    if (R > VR_MAX_R) return alif::set_error(ALIF_EUNSUPPORTED, "van Rossum: at most 8 repeats");
    if (!(dt_ms > 0) || !(tau_ms > 0) || !std::isfinite(dt_ms) || !std::isfinite(tau_ms))
        return alif::set_error(ALIF_EINVAL, "van Rossum: dt_ms and tau_ms must be finite and > 0");
    if (!std::isfinite(scale)) return alif::set_error(ALIF_EINVAL, "van Rossum: scale must be finite");
    if (!dist && !grad) return ALIF_OK;
    const size_t elems = (size_t)B * T * N;
    if (elems == 0) {  // T = 0: every distance is 0 (no gradient elements)
        const long long nd = (long long)B * R * N;
        if (dist && nd > 0) {
            hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                               nd, dist);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
        }
        return ALIF_OK;
    }
    if (!spikes || !targets || !workspace) return alif::set_error(ALIF_EINVAL, "van Rossum: NULL argument");
    if ((size_t)B * R * T * N >= ((size_t)1 << 46)) return alif::set_error(ALIF_EUNSUPPORTED, "van Rossum: too large");
    const VrPlan p = vr_plan(B, R, T, N);
    if (p.vec == 4 && (((uintptr_t)spikes | (uintptr_t)targets) & 3))
        return alif::set_error(ALIF_EINVAL, "van Rossum: spikes and targets must be 4-byte aligned when N % 4 == 0");
    if (grad && p.vec == 4 && ((uintptr_t)grad & 15))
        return alif::set_error(ALIF_EINVAL, "van Rossum: grad must be 16-byte aligned when N % 4 == 0");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    double *sums = (double *)(ws + p.off_sum);
    float *cp = (float *)(ws + p.off_cp);
    float *wts = (float *)(ws + p.off_w);
    double *ce = (double *)(ws + p.off_ce);
    double *cg = (double *)(ws + p.off_cg);
    const double lna = -dt_ms / tau_ms;
    const double a = exp(lna);
    hipError_t e = hipSuccess;
    for (int r0 = 0; r0 < R && e == hipSuccess; r0 += 4) {
        const int rg = R - r0 < 4 ? R - r0 : 4;
        e = p.vec == 4 ? launch_chunks_rg<4>(rg, p, B, R, r0, T, N, a, spikes, targets, sums, cp, st)
                       : launch_chunks_rg<1>(rg, p, B, R, r0, T, N, a, spikes, targets, sums, cp, st);
    }
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    const long long cols = (long long)B * R * N;
    const int Ll = T - (p.K - 1) * p.Lc;   // length of the last chunk
    const double den = expm1(2.0 * lna);
    const double aL = exp(p.Lc * lna), G = a * a * expm1(2.0 * p.Lc * lna) / den;
    const double aLl = exp(Ll * lna), Gl = a * a * expm1(2.0 * Ll * lna) / den;
    hipLaunchKernelGGL(k_vr_combine, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, B, R, N, p.K, a, aL, G,
                       aLl, Gl, dt_ms / tau_ms, (double)scale, sums, dist, wts, ce, cg, grad ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    if (!grad) return ALIF_OK;
    const long long n = (long long)B * p.K * p.ng;
    const dim3 gg((unsigned)((n + 255) / 256)), bb(256);
#define ALIF_VRG(V, RM) hipLaunchKernelGGL((k_vr_grad<V, RM>), gg, bb, 0, st, B, R, T, N, p.ng, p.K, p.Lc, p.S, lna, \
                                           spikes, targets, wts, ce, cg, cp, grad)
    if (p.vec == 4) {
        if (R <= 4) ALIF_VRG(4, 4);
        else ALIF_VRG(4, 8);
    } else {
        if (R <= 4) ALIF_VRG(1, 4);
        else ALIF_VRG(1, 8);
    }
#undef ALIF_VRG
    e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

int alif_adam_step(int32_t n, float *param, const float *grad, float *m, float *v, int32_t step, double lr,
                   double beta1, double beta2, double eps, float lo, float hi, void *stream) {
    if (n < 0 || step < 1) return alif::set_error(ALIF_EINVAL, "adam: n >= 0 and step >= 1 required");
    if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || !std::isfinite(lr) || !(lo <= hi))
        return alif::set_error(ALIF_EINVAL, "adam: bad hyperparameters");
    if (n == 0) return ALIF_OK;
    if (!param || !grad || !m || !v) return alif::set_error(ALIF_EINVAL, "adam: NULL argument");
    // 1 - beta and the bias corrections in FP64, each rounded once to FP32
    const double c1 = -expm1(step * log(beta1)), c2 = -expm1(step * log(beta2));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, param, grad, m, v,
                       (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)(lr / c1),
                       (float)(1.0 / c2), (float)eps, lo, hi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return alif::set_error(ALIF_EHIP, hipGetErrorString(e));
    return ALIF_OK;
}

}  // extern "C"
