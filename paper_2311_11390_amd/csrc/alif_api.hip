// C-ABI of libblockalif: argument validation, buffer layouts, kernel dispatch.
// Every entry point catches its own failures and reports them as a status code
// plus a thread-local message; nothing throws across the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/blockalif.h"
#include "alif_gemm.h"
#include "alif_kernels.h"

using namespace alif;

// Device scratch of alif_backward_noalloc: the block backward's FP64 partial sums
// and the weight-gradient GEMM's split-K partial tiles. One copy per device (a
// module-scope device array exists on every device the library runs on). Host code
// never uses the name itself, which is only a host-side stand-in: it asks the
// runtime for the array's address on the current device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[ALIF_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
int hip_fail(hipError_t e, const char *what) {
    return fail(ALIF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// one status word per device, allocated on first use
std::mutex g_status_mu;
unsigned *g_status[64] = {nullptr};

int status_word(unsigned **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(ALIF_EINVAL, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_status_mu);
    if (!g_status[dev]) {
        unsigned *p = nullptr;
        e = hipMalloc(&p, 256);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(status)");
        e = hipMemset(p, 0, 256);
        if (e != hipSuccess) return hip_fail(e, "hipMemset(status)");
        g_status[dev] = p;
    }
    *out = g_status[dev];
    return ALIF_OK;
}

// The address of `scratch` on the current device, looked up once per device with
// that device current (each device holds its own copy at its own address).
std::mutex g_scratch_mu;
void *g_scratch[64] = {nullptr};

int noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(ALIF_EINVAL, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(ALIF_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return ALIF_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int tr_of(double dt, double arp) {
    if (!(dt > 0.0) || !(arp > 0.0) || !std::isfinite(dt) || !std::isfinite(arp)) return -1;
    const double r = arp / dt;
    const double n = std::floor(r + 0.5);
    if (n < 1.0 || std::fabs(r - n) > 1e-9 * n) return -1;
    if (n > 1e9) return -1;
    return (int)n;
}

struct Prob {
    int B, T, N, n_in, TR, NB;
    bool spikes_in;
};

int check_desc(const alif_desc *d, Prob *p) {
    if (!d) return fail(ALIF_EINVAL, "desc is NULL");
    if (d->batch < 0 || d->n_neurons < 0 || d->T < 0)
        return fail(ALIF_EINVAL, "negative size (batch=%d n_neurons=%d T=%d)", d->batch, d->n_neurons, d->T);
    const int TR = tr_of(d->dt_ms, d->arp_ms);
    if (TR < 0)
        return fail(ALIF_EINVAL, "arp_ms/dt_ms = %g/%g is not a whole number of steps", d->arp_ms, d->dt_ms);
    if (TR < 2)
        return fail(ALIF_EINVAL, "T_R = %d: blocks need T_R >= 2 (Eq. 2's reset already blanks the step after a spike)", TR);
    if (TR > ALIF_MAX_TR) return fail(ALIF_EUNSUPPORTED, "T_R = %d exceeds ALIF_MAX_TR = %d", TR, ALIF_MAX_TR);
    if (d->input_kind < ALIF_INPUT_CURRENT_F32 || d->input_kind > ALIF_INPUT_SPIKES_F32)
        return fail(ALIF_EINVAL, "unknown input_kind %d", d->input_kind);
    if (d->spike_dtype < ALIF_SPIKES_U8 || d->spike_dtype > ALIF_SPIKES_F32)
        return fail(ALIF_EINVAL, "unknown spike_dtype %d", d->spike_dtype);
    if (d->algo < ALIF_ALGO_BLOCKS || d->algo > ALIF_ALGO_SEQUENTIAL_STEP)
        return fail(ALIF_EINVAL, "unknown algo %d", d->algo);
    if (d->surrogate != ALIF_SG_FAST_SIGMOID && d->surrogate != ALIF_SG_BOXCAR &&
        d->surrogate != ALIF_SG_MULTI_GAUSSIAN)
        return fail(ALIF_EINVAL, "unknown surrogate %d", d->surrogate);
    if (d->grad_policy != ALIF_GRAD_DETACHED && d->grad_policy != ALIF_GRAD_ATTACHED)
        return fail(ALIF_EINVAL, "unknown grad_policy %d", d->grad_policy);
    if (!(d->sg_slope >= 0.0f) || !std::isfinite(d->sg_slope)) return fail(ALIF_EINVAL, "bad sg_slope");
    const bool sp = d->input_kind != ALIF_INPUT_CURRENT_F32;
    if (sp) {
        if (d->n_in <= 0) return fail(ALIF_EINVAL, "spike input needs n_in > 0 (got %d)", d->n_in);
        if (d->gemm_precision != ALIF_GEMM_FP32 && d->gemm_precision != ALIF_GEMM_BF16)
            return fail(ALIF_EINVAL, "unknown gemm_precision %d", d->gemm_precision);
    }
    const size_t TN = (size_t)d->T * (size_t)d->n_neurons;
    if (TN * 4 >= ((size_t)1 << 31))
        return fail(ALIF_EUNSUPPORTED, "T * n_neurons = %zu: one batch row must stay below 2 GiB of float", TN);
    if (sp && (size_t)d->T * (size_t)d->n_in * 4 >= ((size_t)1 << 31))
        return fail(ALIF_EUNSUPPORTED, "T * n_in too large");
    p->B = d->batch;
    p->T = d->T;
    p->N = d->n_neurons;
    p->n_in = sp ? d->n_in : 0;
    p->TR = TR;
    p->NB = (d->T + TR - 1) / TR;
    p->spikes_in = sp;
    if ((size_t)p->NB * (size_t)p->N * 8 >= ((size_t)1 << 31))
        return fail(ALIF_EUNSUPPORTED, "T / T_R * n_neurons too large");
    return ALIF_OK;
}

int check_params(const alif_params *prm) {
    if (!prm) return fail(ALIF_EINVAL, "params is NULL");
    if (!prm->tau_mem_ms || !prm->tau_adapt_ms || !prm->d || !prm->theta0)
        return fail(ALIF_EINVAL, "tau_mem_ms, tau_adapt_ms, d and theta0 are required");
    return ALIF_OK;
}

// Block path: the carry-in of every block plus the final carry, [B][NB + 1][N]
// (the backward reads block n's spike step from the carry-in of block n + 1).
size_t carry_bytes(const alif_desc *d, const Prob &p) {
    if (d->algo == ALIF_ALGO_BLOCKS) {
        const size_t cn = (size_t)p.B * (p.NB + 1) * p.N;
        return align256(cn * 4) * 2 + align256(cn);
    }
    const size_t cn = (size_t)p.B * p.NB * p.N;
    if (d->algo == ALIF_ALGO_SEQUENTIAL) return align256(cn * 8) * 2 + align256(cn * 4);
    const size_t bn = (size_t)p.B * p.N;  // per-step launch: state only
    return align256(bn * 8) * 2 + align256(bn * 4);
}

CarryView carry_view(void *base, const Prob &p) {
    const size_t cn = (size_t)p.B * (p.NB + 1) * p.N;
    char *c = (char *)base;
    CarryView v;
    v.v = (float *)c;
    v.a = (float *)(c + align256(cn * 4));
    v.ts = (uint8_t *)(c + 2 * align256(cn * 4));
    return v;
}
SeqCarryView seq_carry_view(void *base, size_t cn) {
    char *c = (char *)base;
    SeqCarryView v;
    v.v = (double *)c;
    v.a = (double *)(c + align256(cn * 8));
    v.c = (int32_t *)(c + 2 * align256(cn * 8));
    return v;
}

}  // namespace

namespace alif {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
// Backward workspace: FP64 partial sums [5][B][N]; for spike input the weight-gradient
// GEMM's split partials and the event path's count, masks and partials (both are
// enqueued, one runs); with BF16 GEMMs, W transposed and rounded to bfloat16 once
// for the input gradient, then the input-current gradient as bfloat16 [B][T][N] for
// a call that passes no grad_current.
struct BwdWs {
    size_t part, gemm, wgev, wt, gi16, total;
};
BwdWs bwd_ws_layout(const alif_desc *desc, const Prob &p) {
    BwdWs w;
    w.part = 0;
    w.gemm = align256((size_t)5 * p.B * p.N * sizeof(double));
    w.wgev = w.gemm + (p.spikes_in ? align256(gemm_workspace_bytes((size_t)p.B * p.T, p.N, p.n_in)) : 0);
    w.wt = w.wgev + (p.spikes_in ? align256(wgrad_event_bytes(p.B, p.T, p.n_in, p.N)) : 0);
    const bool bf = p.spikes_in && desc->gemm_precision == ALIF_GEMM_BF16;
    w.gi16 = w.wt + (bf ? align256(gemm_wbf16_bytes(p.N, p.n_in)) : 0);
    w.total = w.gi16 + (bf ? align256((size_t)p.B * p.T * p.N * 2) : 0);
    return w;
}
// Whether a backward call keeps the input-current gradient as bfloat16 in its
// workspace: spike input, BF16 GEMMs, the detached block backward, no gV / gTheta,
// the projections' gradients asked for and no grad_current to fill. N % 8 == 0
// keeps the bfloat16 rows 16-byte aligned, so the GEMMs take the same kernels as
// from a float gI (and give the same bits).
bool bwd_gi16(const alif_desc *desc, const Prob &p, bool grad_current, bool grad_vt, bool proj) {
    return p.spikes_in && desc->gemm_precision == ALIF_GEMM_BF16 && desc->algo == ALIF_ALGO_BLOCKS &&
           desc->grad_policy != ALIF_GRAD_ATTACHED && !grad_vt && proj && !grad_current && p.N % 8 == 0;
}

}  // namespace alif

extern "C" {

const char *alif_last_error(void) { return g_err.c_str(); }

int alif_refractory_steps(double dt_ms, double arp_ms) {
    const int TR = tr_of(dt_ms, arp_ms);
    if (TR < 0) return fail(ALIF_EINVAL, "arp/dt is not a whole number of steps");
    if (TR < 2) return fail(ALIF_EINVAL, "T_R must be >= 2");
    if (TR > ALIF_MAX_TR) return fail(ALIF_EUNSUPPORTED, "T_R > ALIF_MAX_TR");
    return TR;
}

int alif_carry_bytes(const alif_desc *desc, size_t *bytes) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!bytes) return fail(ALIF_EINVAL, "bytes is NULL");
    *bytes = carry_bytes(desc, p);
    return ALIF_OK;
}

int alif_backward_workspace_bytes(const alif_desc *desc, size_t *bytes) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!bytes) return fail(ALIF_EINVAL, "bytes is NULL");
    *bytes = bwd_ws_layout(desc, p).total;
    return ALIF_OK;
}

int alif_decay_tables(const alif_desc *desc, const alif_params *prm, float *beta_pow, float *p_pow,
                      void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!prm || !prm->tau_mem_ms || !prm->tau_adapt_ms) return fail(ALIF_EINVAL, "tau pointers required");
    hipError_t e = launch_decay_tables(p.N, p.TR, desc->dt_ms, prm->tau_mem_ms, prm->tau_adapt_ms,
                                       beta_pow, p_pow, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "decay tables launch");
    return ALIF_OK;
}

int alif_input_current(const alif_desc *desc, const void *input, const float *W, const float *bias,
                       float *current, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!p.spikes_in) return fail(ALIF_EINVAL, "alif_input_current needs a spike input_kind");
    if (!input || !W || !current) return fail(ALIF_EINVAL, "input, W and current are required");
    GemmIn in;
    in.kind = desc->input_kind;
    in.ptr = input;
    hipError_t e = gemm_input_current((size_t)p.B * p.T, p.N, p.n_in, in, W, bias, current,
                                      desc->gemm_precision == ALIF_GEMM_BF16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "input-current GEMM");
    return ALIF_OK;
}

int alif_weight_grad_workspace_bytes(const alif_desc *desc, size_t *bytes) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!bytes) return fail(ALIF_EINVAL, "bytes is NULL");
    *bytes = p.spikes_in ? gemm_workspace_bytes((size_t)p.B * p.T, p.N, p.n_in) : 0;
    return ALIF_OK;
}

int alif_weight_grad(const alif_desc *desc, const float *grad_current, const void *input, float *grad_W,
                     void *workspace, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!p.spikes_in) return fail(ALIF_EINVAL, "alif_weight_grad needs a spike input_kind");
    if (!grad_current || !input || !grad_W) return fail(ALIF_EINVAL, "grad_current, input and grad_W are required");
    if (!workspace && gemm_workspace_bytes((size_t)p.B * p.T, p.N, p.n_in) > 0)
        return fail(ALIF_EINVAL, "workspace is NULL");
    GemmIn in;
    in.kind = desc->input_kind;
    in.ptr = input;
    hipError_t e = gemm_weight_grad((size_t)p.B * p.T, p.N, p.n_in, grad_current, in, grad_W,
                                    desc->gemm_precision == ALIF_GEMM_BF16, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "weight-gradient GEMM");
    return ALIF_OK;
}

int alif_input_grad(const alif_desc *desc, const float *grad_current, const float *W, float *grad_input,
                    void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!p.spikes_in) return fail(ALIF_EINVAL, "alif_input_grad needs a spike input_kind");
    if (!grad_current || !W || !grad_input) return fail(ALIF_EINVAL, "grad_current, W and grad_input are required");
    hipError_t e = gemm_input_grad((size_t)p.B * p.T, p.N, p.n_in, grad_current, W, grad_input,
                                   desc->gemm_precision == ALIF_GEMM_BF16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "input-gradient GEMM");
    return ALIF_OK;
}

int alif_forward(const alif_desc *desc, const alif_params *prm, const void *input, const float *W,
                 float *current, const alif_state *init, alif_state *final, void *spikes, float *v,
                 float *theta, void *carries, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (!input && p.B * (size_t)p.T * p.N > 0) return fail(ALIF_EINVAL, "input is NULL");
    if (!spikes && p.B * (size_t)p.T * p.N > 0) return fail(ALIF_EINVAL, "spikes output is NULL");
    if (p.spikes_in) {
        if (!W || !current) return fail(ALIF_EINVAL, "spike input needs W and the current workspace");
    } else if (current) {
        return fail(ALIF_EINVAL, "current workspace must be NULL for current input");
    }
    if (init && (!init->v || !init->a || !init->ts)) return fail(ALIF_EINVAL, "init state has NULL arrays");
    if (final) {
        if (!final->v || !final->a || !final->ts) return fail(ALIF_EINVAL, "final state has NULL arrays");
        if (p.T % p.TR != 0) return fail(ALIF_EINVAL, "final state needs T %% T_R == 0 (T=%d, T_R=%d)", p.T, p.TR);
    }
    if (desc->algo == ALIF_ALGO_SEQUENTIAL_STEP && !carries)
        return fail(ALIF_EINVAL, "the per-step baseline keeps its state in the carries buffer");
    unsigned *status = nullptr;
    if ((rc = status_word(&status))) return rc;
    hipStream_t st = (hipStream_t)stream;

    const float *I = (const float *)input;
    const float *bias_k = prm->bias;
    if (p.spikes_in) {
        GemmIn in;
        in.kind = desc->input_kind;
        in.ptr = input;
        // the spike output, written only after the GEMM, holds the bfloat16 weights meanwhile
        const size_t sbytes = (size_t)p.B * p.T * p.N *
                              (desc->spike_dtype == ALIF_SPIKES_U8 ? 1 : (desc->spike_dtype == ALIF_SPIKES_BF16 ? 2 : 4));
        hipError_t e = gemm_input_current((size_t)p.B * p.T, p.N, p.n_in, in, W, prm->bias, current,
                                          desc->gemm_precision == ALIF_GEMM_BF16, st, spikes, sbytes);
        if (e != hipSuccess) return hip_fail(e, "input-current GEMM");
        I = current;
        bias_k = nullptr;
    }
    if (p.B == 0 || p.N == 0 || p.T == 0) return ALIF_OK;

    if (desc->algo == ALIF_ALGO_BLOCKS) {
        FwdArgs a{};
        a.B = p.B; a.T = p.T; a.N = p.N; a.TR = p.TR; a.NB = p.NB;
        a.n_groups = (p.N + block_neurons_per_wg(block_config(p.TR).seg) - 1) /
                     block_neurons_per_wg(block_config(p.TR).seg);
        a.dt = desc->dt_ms;
        a.I = I;
        a.bias_k = bias_k;
        a.tau_m = prm->tau_mem_ms; a.tau_a = prm->tau_adapt_ms; a.d = prm->d; a.theta0 = prm->theta0;
        if (init) { a.init_v = init->v; a.init_a = init->a; a.init_ts = init->ts; }
        if (final) { a.fin_v = final->v; a.fin_a = final->a; a.fin_ts = final->ts; }
        a.spikes = spikes;
        a.spike_dtype = desc->spike_dtype;
        a.V = v;
        a.TH = theta;
        if (carries) a.ck = carry_view(carries, p);
        a.status = status;
        hipError_t e = launch_blocks_fwd(a, st);
        if (e != hipSuccess) return hip_fail(e, "block forward launch");
        return ALIF_OK;
    }
    SeqArgs a{};
    a.B = p.B; a.T = p.T; a.N = p.N; a.TR = p.TR; a.NB = p.NB;
    a.dt = desc->dt_ms;
    a.slope = desc->sg_slope;
    a.surrogate = desc->surrogate;
    a.I = I;
    a.bias_k = bias_k;
    a.tau_m = prm->tau_mem_ms; a.tau_a = prm->tau_adapt_ms; a.d = prm->d; a.theta0 = prm->theta0;
    if (init) { a.init_v = init->v; a.init_a = init->a; a.init_ts = init->ts; }
    if (final) { a.fin_v = final->v; a.fin_a = final->a; a.fin_ts = final->ts; }
    a.spikes = spikes;
    a.spike_dtype = desc->spike_dtype;
    a.V = v;
    a.TH = theta;
    a.status = status;
    hipError_t e;
    if (desc->algo == ALIF_ALGO_SEQUENTIAL) {
        if (carries) a.ck = seq_carry_view(carries, (size_t)p.B * p.NB * p.N);
        e = launch_seq_fwd(a, st);
    } else {
        SeqCarryView sv = seq_carry_view(carries, (size_t)p.B * p.N);
        a.st_v = sv.v;
        a.st_a = sv.a;
        a.st_c = sv.c;
        e = launch_seq_step_fwd(a, st);
    }
    if (e != hipSuccess) return hip_fail(e, "sequential forward launch");
    return ALIF_OK;
}

int alif_backward(const alif_desc *desc, const alif_params *prm, const void *input, const float *W,
                  const float *current, const void *carries, const float *grad_spikes,
                  const float *grad_v, const float *grad_theta, float *grad_current,
                  float *grad_input, float *grad_W, float *grad_bias, float *grad_tau_mem,
                  float *grad_tau_adapt, float *grad_d, float *grad_theta0, void *workspace,
                  void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (desc->algo == ALIF_ALGO_SEQUENTIAL_STEP)
        return fail(ALIF_EUNSUPPORTED, "the per-step-launch baseline is forward only");
    if (desc->algo == ALIF_ALGO_SEQUENTIAL && p.TR > seq_bwd_max_tr(grad_v || grad_theta))
        return fail(ALIF_EUNSUPPORTED, "sequential backward supports T_R <= %d here",
                    seq_bwd_max_tr(grad_v || grad_theta));
    const size_t work = (size_t)p.B * p.T * p.N;
    if (work == 0) {
        // nothing to differentiate: parameter gradients are zero
        hipStream_t st = (hipStream_t)stream;
        float *outs[5] = {grad_bias, grad_tau_mem, grad_tau_adapt, grad_d, grad_theta0};
        for (float *o : outs)
            if (o && p.N > 0) {
                hipError_t e = hipMemsetAsync(o, 0, (size_t)p.N * 4, st);
                if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
            }
        if (grad_W && p.spikes_in && p.N > 0) {
            hipError_t e = hipMemsetAsync(grad_W, 0, (size_t)p.N * p.n_in * 4, st);
            if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        }
        return ALIF_OK;
    }
    if (!input || !carries || !workspace) return fail(ALIF_EINVAL, "input, carries and workspace are required");
    const bool gi16 = bwd_gi16(desc, p, grad_current != nullptr, grad_v || grad_theta, grad_W || grad_input);
    if (p.spikes_in) {
        if (!current || !W) return fail(ALIF_EINVAL, "spike input: pass W and the current workspace alif_forward filled");
        if ((grad_W || grad_input) && !grad_current && !gi16)
            return fail(ALIF_EINVAL, "grad_W / grad_input need the grad_current buffer (it may be NULL only with "
                                     "BF16 GEMMs, the detached block backward, no grad_v / grad_theta and a "
                                     "multiple of 8 neurons)");
    } else {
        if (grad_input || grad_W) return fail(ALIF_EINVAL, "current input: its gradient is grad_current");
    }
    hipStream_t st = (hipStream_t)stream;
    const float *I = p.spikes_in ? current : (const float *)input;
    const float *bias_k = p.spikes_in ? nullptr : prm->bias;
    double *part = (double *)workspace;

    hipError_t e;
    if (desc->algo == ALIF_ALGO_BLOCKS) {
        BwdArgs a{};
        a.B = p.B; a.T = p.T; a.N = p.N; a.TR = p.TR; a.NB = p.NB;
        const int nwg = block_neurons_per_wg(block_config(p.TR).seg);
        a.n_groups = (p.N + nwg - 1) / nwg;
        a.dt = desc->dt_ms;
        a.slope = desc->sg_slope;
        a.surrogate = desc->surrogate;
        a.attached = desc->grad_policy == ALIF_GRAD_ATTACHED;
        a.I = I;
        a.bias_k = bias_k;
        a.tau_m = prm->tau_mem_ms; a.tau_a = prm->tau_adapt_ms; a.d = prm->d; a.theta0 = prm->theta0;
        a.ck = carry_view(const_cast<void *>(carries), p);
        a.gS = grad_spikes; a.gV = grad_v; a.gTH = grad_theta;
        a.gI = grad_current;
        a.gI16 = gi16 ? reinterpret_cast<uint16_t *>((char *)workspace + bwd_ws_layout(desc, p).gi16) : nullptr;
        a.part = part;
        e = launch_blocks_bwd(a, st);
        if (e != hipSuccess) return hip_fail(e, "block backward launch");
    } else {
        SeqArgs a{};
        a.B = p.B; a.T = p.T; a.N = p.N; a.TR = p.TR; a.NB = p.NB;
        a.dt = desc->dt_ms;
        a.slope = desc->sg_slope;
        a.surrogate = desc->surrogate;
        a.attached = desc->grad_policy == ALIF_GRAD_ATTACHED;
        a.I = I;
        a.bias_k = bias_k;
        a.tau_m = prm->tau_mem_ms; a.tau_a = prm->tau_adapt_ms; a.d = prm->d; a.theta0 = prm->theta0;
        a.ck = seq_carry_view(const_cast<void *>(carries), (size_t)p.B * p.NB * p.N);
        a.gS = grad_spikes; a.gV = grad_v; a.gTH = grad_theta;
        a.gI = grad_current;
        a.part = part;
        e = launch_seq_bwd(a, st);
        if (e != hipSuccess) return hip_fail(e, "sequential backward launch");
    }
    FinalizeArgs f{};
    f.B = p.B; f.N = p.N; f.dt = desc->dt_ms;
    f.tau_m = prm->tau_mem_ms; f.tau_a = prm->tau_adapt_ms;
    f.part = part;
    f.g_tau_m = grad_tau_mem; f.g_tau_a = grad_tau_adapt; f.g_d = grad_d; f.g_theta0 = grad_theta0;
    f.g_bias = grad_bias;
    e = launch_finalize(f, st);
    if (e != hipSuccess) return hip_fail(e, "gradient finalize launch");

    if (p.spikes_in) {
        GemmIn in;
        in.kind = desc->input_kind;
        in.ptr = input;
        const BwdWs lay = bwd_ws_layout(desc, p);
        void *gws = (char *)workspace + lay.gemm;
        const void *gI = gi16 ? (const void *)((char *)workspace + lay.gi16) : (const void *)grad_current;
        const bool bf = desc->gemm_precision == ALIF_GEMM_BF16;
        if (grad_W) {
            // sparse input: dW summed over the active inputs (exact products, FP32 sums in a
            // fixed order; gI rounded to bfloat16 as the BF16 GEMM rounds it); the dense GEMM
            // behind it runs instead when the device-side count of active inputs is above
            // one per 256 entries
            unsigned long long *cnt = nullptr, thr = 0;
            e = launch_wgrad_events(p.B, p.T, p.n_in, p.N, 0, desc->input_kind == ALIF_INPUT_SPIKES_U8 ? 1 : 2,
                                    input, gI, gi16 ? 2 : (bf ? 1 : 0), grad_W, (char *)workspace + lay.wgev, &cnt,
                                    &thr, st);
            if (e != hipSuccess) return hip_fail(e, "weight-gradient event launch");
            e = gemm_weight_grad((size_t)p.B * p.T, p.N, p.n_in, gI, in, grad_W, bf, gws, st, cnt, thr, gi16);
            if (e != hipSuccess) return hip_fail(e, "weight-gradient GEMM");
        }
        if (grad_input) {
            e = gemm_input_grad((size_t)p.B * p.T, p.N, p.n_in, gI, W, grad_input, bf, st,
                                (char *)workspace + lay.wt, lay.gi16 - lay.wt, gi16);
            if (e != hipSuccess) return hip_fail(e, "input-gradient GEMM");
        }
    }
    return ALIF_OK;
}

int alif_backward_noalloc(const alif_desc *desc, const alif_params *prm, const void *input, const float *W,
                          const float *current, const void *carries, const float *grad_spikes,
                          const float *grad_v, const float *grad_theta, float *grad_current,
                          float *grad_input, float *grad_W, float *grad_bias, float *grad_tau_mem,
                          float *grad_tau_adapt, float *grad_d, float *grad_theta0, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    // the scratch alif_backward would take as its workspace: the partial sums, the
    // split-K tiles only when the weight gradient is asked for, the rounded W^T only
    // for the input gradient, the bfloat16 gI only when it stands in for grad_current
    const BwdWs lay = bwd_ws_layout(desc, p);
    size_t need = grad_W ? lay.wt : lay.gemm;
    if (grad_input && lay.gi16 > lay.wt) need = lay.gi16;   // W transposed and rounded
    if (bwd_gi16(desc, p, grad_current != nullptr, grad_v || grad_theta, grad_W || grad_input)) need = lay.total;
    if (need > (size_t)ALIF_NOALLOC_SCRATCH_BYTES)
        return fail(ALIF_EUNSUPPORTED,
                    "alif_backward_noalloc: this problem needs %zu bytes of scratch, more than the %u-byte "
                    "static scratch; use alif_backward with a workspace",
                    need, (unsigned)ALIF_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((rc = noalloc_scratch(&ws))) return rc;
    // every scratch byte the kernels read they have written earlier in the same call
    // (the partial sums of every (b, neuron), every split's tile), so nothing is cleared
    return alif_backward(desc, prm, input, W, current, carries, grad_spikes, grad_v, grad_theta, grad_current,
                         grad_input, grad_W, grad_bias, grad_tau_mem, grad_tau_adapt, grad_d, grad_theta0, ws,
                         stream);
}

// ---------------------------------------------------------------------------
// recurrent layer (Eq. 3's recurrent current with delay D = T_R; Prop. 3)
// ---------------------------------------------------------------------------
namespace {

int spike_elem_bytes(int sdt) { return sdt == ALIF_SPIKES_U8 ? 1 : (sdt == ALIF_SPIKES_BF16 ? 2 : 4); }
int spike_gemm_kind(int sdt) {
    return sdt == ALIF_SPIKES_U8 ? ALIF_INPUT_SPIKES_U8
                                 : (sdt == ALIF_SPIKES_BF16 ? ALIF_INPUT_SPIKES_BF16 : ALIF_INPUT_SPIKES_F32);
}

// Forward scratch: the spikes of every block, block-major [NB][B][T_R][N] (each
// block 256-byte aligned; the next block's recurrent current reads them), then
// two FP64 carry states [B][N] (v, a) and their int32 spike steps, then W_rec
// transposed.
struct RecLayout {
    size_t blk, spikes, state, wt, total;
};
RecLayout rec_layout(const alif_desc *d, const Prob &p) {
    RecLayout L{};
    const size_t sb = (size_t)spike_elem_bytes(d->spike_dtype);
    L.blk = align256((size_t)p.B * p.TR * p.N * sb);
    L.spikes = L.blk * p.NB;
    L.state = align256((size_t)p.B * p.N * 8) * 4 + align256((size_t)p.B * p.N * 4) * 2;
    L.wt = align256((size_t)p.N * p.N * 4);
    const size_t fwd = L.spikes + L.state + L.wt;
    // weight gradient: the event path's count, masks and partials; the dense path's
    // shifted spikes and GEMM partial sums from byte 256 on (over the masks: the
    // two never both run)
    const size_t ev = wgrad_event_bytes(p.B, p.T, p.N, p.N);
    const size_t dense = 256 + align256((size_t)p.B * p.T * p.N * sb) +
                         gemm_workspace_bytes((size_t)p.B * p.T, p.N, p.N);
    const size_t wg = ev > dense ? ev : dense;
    L.total = fwd > wg ? fwd : wg;
    return L;
}

}  // namespace

int alif_recurrent_workspace_bytes(const alif_desc *desc, size_t *bytes) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if (!bytes) return fail(ALIF_EINVAL, "bytes is NULL");
    *bytes = rec_layout(desc, p).total;
    return ALIF_OK;
}

int alif_forward_recurrent(const alif_desc *desc, const alif_params *prm, const void *input, const float *W,
                           const float *W_rec, int32_t delay, float *current, void *spikes, float *v,
                           float *theta, void *carries, void *workspace, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (desc->algo != ALIF_ALGO_BLOCKS) return fail(ALIF_EUNSUPPORTED, "the recurrent layer runs the blocks algorithm");
    const int D = delay == 0 ? p.TR : delay;
    if (D < p.TR) return fail(ALIF_EINVAL, "recurrent delay %d < T_R = %d", D, p.TR);
    const size_t BTN = (size_t)p.B * p.T * p.N;
    if (BTN == 0) return ALIF_OK;
    if (!input || !W_rec || !current || !spikes || !workspace)
        return fail(ALIF_EINVAL, "input, W_rec, current, spikes and workspace are required");
    if (p.spikes_in && !W) return fail(ALIF_EINVAL, "spike input needs W");
    unsigned *status = nullptr;
    if ((rc = status_word(&status))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool bf16 = desc->gemm_precision == ALIF_GEMM_BF16;
    const float *bias_k = prm->bias;
    hipError_t e;
    // the current without its recurrent part: b + W x (spike input) or the input
    // itself (current input; the bias is then added in-kernel, as alif_forward does)
    const bool fused = recurrent_fused_ok(p.N, p.TR, D);
    if (p.spikes_in) {
        GemmIn in;
        in.kind = desc->input_kind;
        in.ptr = input;
        // the spike output, written only at the end, holds the bfloat16 weights meanwhile
        e = gemm_input_current((size_t)p.B * p.T, p.N, p.n_in, in, W, prm->bias, current, bf16, st, spikes,
                               BTN * (size_t)spike_elem_bytes(desc->spike_dtype));
        if (e != hipSuccess) return hip_fail(e, "input-current GEMM");
        bias_k = nullptr;
    } else if (!fused) {   // the one-launch layer reads the input and writes the whole current itself
        e = hipMemcpyAsync(current, input, BTN * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "current copy");
    }
    const RecLayout L = rec_layout(desc, p);
    char *ws = (char *)workspace;
    char *sblk = ws;
    char *stb = ws + L.spikes;
    const size_t s8 = align256((size_t)p.B * p.N * 8), s4 = align256((size_t)p.B * p.N * 4);
    double *sv[2] = {(double *)stb, (double *)(stb + s8)};
    double *sa[2] = {(double *)(stb + 2 * s8), (double *)(stb + 3 * s8)};
    int32_t *sts[2] = {(int32_t *)(stb + 4 * s8), (int32_t *)(stb + 4 * s8 + s4)};
    float *wrt = (float *)(stb + L.state);
    e = launch_transpose(p.N, W_rec, wrt, st);
    if (e != hipSuccess) return hip_fail(e, "W_rec transpose launch");
    if (fused) {   // the whole block loop in one launch
        RecArgs r{};
        r.B = p.B; r.T = p.T; r.N = p.N; r.TR = p.TR; r.NB = p.NB; r.D = D;
        r.ring = recurrent_ring_slots(p.TR, D);
        r.dt = desc->dt_ms;
        r.I_ff = p.spikes_in ? current : (const float *)input;
        r.I = current;
        r.bias_k = bias_k;
        r.tau_m = prm->tau_mem_ms; r.tau_a = prm->tau_adapt_ms; r.d = prm->d; r.theta0 = prm->theta0;
        r.WrecT = wrt;
        r.spikes = spikes;
        r.spike_dtype = desc->spike_dtype;
        r.V = v;
        r.TH = theta;
        if (carries) r.ck = carry_view(carries, p);
        r.status = status;
        e = launch_recurrent_fused(r, st);
        if (e != hipSuccess) return hip_fail(e, "recurrent layer launch");
        return ALIF_OK;
    }
    const int nwg = block_neurons_per_wg(block_config(p.TR).seg);
    const size_t TN = (size_t)p.T * p.N, TRN = (size_t)p.TR * p.N;
    const int sb = spike_elem_bytes(desc->spike_dtype);
    for (int n = 0; n < p.NB; n++) {
        const int rows = p.T - n * p.TR < p.TR ? p.T - n * p.TR : p.TR;
        float *cur_n = current + n * TRN;
        if ((n + 1) * p.TR > D) {   // block n's recurrent current from spikes D steps back
            e = launch_recurrent_events(p.B, p.TR, rows, p.N, (long long)TN, n * p.TR, D, sb, sblk, L.blk, wrt,
                                        cur_n, st);
            if (e != hipSuccess) return hip_fail(e, "recurrent current launch");
        }
        FwdArgs a{};
        a.B = p.B; a.T = rows; a.N = p.N; a.TR = p.TR; a.NB = 1;
        a.n_groups = (p.N + nwg - 1) / nwg;
        a.dt = desc->dt_ms;
        a.I = cur_n;
        a.bias_k = bias_k;
        a.tau_m = prm->tau_mem_ms; a.tau_a = prm->tau_adapt_ms; a.d = prm->d; a.theta0 = prm->theta0;
        if (n > 0) { a.init_v = sv[(n - 1) & 1]; a.init_a = sa[(n - 1) & 1]; a.init_ts = sts[(n - 1) & 1]; }
        a.fin_v = sv[n & 1]; a.fin_a = sa[n & 1]; a.fin_ts = sts[n & 1];
        a.spikes = sblk + (size_t)n * L.blk;
        a.spike_dtype = desc->spike_dtype;
        a.V = v ? v + n * TRN : nullptr;
        a.TH = theta ? theta + n * TRN : nullptr;
        if (carries) a.ck = carry_view(carries, p);
        a.status = status;
        a.bs_i = TN;
        a.bs_s = TRN;
        a.ck_nb = p.NB;
        a.ck_off = n;
        e = launch_blocks_fwd(a, st);
        if (e != hipSuccess) return hip_fail(e, "block forward launch");
    }
    e = launch_blocks_to_bt(p.B, p.T, p.N, p.TR, sb, sblk, L.blk, spikes, st);
    if (e != hipSuccess) return hip_fail(e, "spike layout launch");
    return ALIF_OK;
}

int alif_recurrent_weight_grad(const alif_desc *desc, int32_t delay, const float *grad_current,
                               const void *spikes, float *grad_W_rec, void *workspace, void *stream) {
    Prob p;
    int rc = check_desc(desc, &p);
    if (rc) return rc;
    const int D = delay == 0 ? p.TR : delay;
    if (D < p.TR) return fail(ALIF_EINVAL, "recurrent delay %d < T_R = %d", D, p.TR);
    if (!grad_current || !spikes || !grad_W_rec || !workspace)
        return fail(ALIF_EINVAL, "grad_current, spikes, grad_W_rec and workspace are required");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(ALIF_EINVAL, "workspace not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int sb = spike_elem_bytes(desc->spike_dtype);
    // the event path, then the dense path gated on the event count it leaves
    unsigned long long *count = nullptr, thr = 0;
    hipError_t e = launch_wgrad_events(p.B, p.T, p.N, p.N, D, sb, spikes, grad_current, 0, grad_W_rec, workspace,
                                       &count, &thr, st);
    if (e != hipSuccess) return hip_fail(e, "recurrent weight-gradient event launch");
    const size_t shb = align256((size_t)p.B * p.T * p.N * sb);
    char *shifted = (char *)workspace + 256;
    e = launch_shift_time(p.B, p.T, p.N, D, sb, spikes, shifted, st, count, thr);
    if (e != hipSuccess) return hip_fail(e, "spike shift launch");
    GemmIn x;
    x.kind = spike_gemm_kind(desc->spike_dtype);
    x.ptr = shifted;
    e = gemm_weight_grad((size_t)p.B * p.T, p.N, p.N, grad_current, x, grad_W_rec,
                         desc->gemm_precision == ALIF_GEMM_BF16, shifted + shb, st, count, thr);
    if (e != hipSuccess) return hip_fail(e, "recurrent weight-gradient GEMM");
    return ALIF_OK;
}

int alif_device_status(uint32_t *bits, void *stream) {
    if (!bits) return fail(ALIF_EINVAL, "bits is NULL");
    unsigned *s = nullptr;
    int rc = status_word(&s);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    unsigned h = 0;
    hipError_t e = hipMemcpyAsync(&h, s, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemsetAsync(s, 0, sizeof(unsigned), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading the device status word");
    *bits = h;
    return ALIF_OK;
}

}  // extern "C"
