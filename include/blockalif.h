/*
 * libblockalif -- block-wise ALIF simulation and surrogate-gradient training on
 * one AMD Instinct MI355X (gfx950).
 *
 * The library implements the "Blocks" reformulation of the adaptive leaky
 * integrate-and-fire (ALIF) network of Taylor, King & Harper, "Addressing the
 * speed-accuracy simulation trade-off for adaptive spiking neurons" (NeurIPS 2023,
 * arXiv 2311.11390): time is cut into blocks of T_R steps (T_R = ARP / DT, the
 * absolute refractory period in steps), inside which a neuron fires at most once,
 * so that each block is integrated in parallel over its T_R steps (Section 3,
 * "Block", Eqs. 6-9, Props. 1-2) and only the block-boundary state is carried
 * sequentially, T / T_R times (Section 3, "Blocks", Props. 3-5). The dynamics
 * are exactly those of the standard ALIF model (Section 2, Eqs. 1-5):
 *
 *   S[t]  = 1[V[t] > th[t]]                                  (Eq. 1, strict)
 *   V[t]  = (beta V[t-1] + (1 - beta) I[t]) (1 - S[t-1])     (Eq. 2)
 *   I~[t] = b + W x[t]                                       (Eq. 3, feedforward)
 *   I[t]  = I~[t] if the last spike is >= T_R steps back, else 0   (Eq. 4)
 *   th[t] = theta0 + d a[t],  a[t] = p a[t-1] + S[t-1]       (Eq. 5)
 *
 * with beta = exp(-DT / tau_mem), p = exp(-DT / tau_adapt) (supplementary,
 * "Weight initialisation"), V = a = 0 and no earlier spike at t = 0. The paper's
 * baseline threshold 1 is generalised to a per-neuron theta0. NOTE: the parameter
 * called `d` here is the paper's adaptation scalar d; some workload descriptions
 * call it "beta", which is NOT the membrane decay beta above.
 *
 * Conventions shared by every entry point:
 *  - Status: 0 = ALIF_OK, 1 = ALIF_PENDING, negative = error. After an error,
 *    alif_last_error() returns a message (thread-local). No C++ exception ever
 *    crosses this boundary.
 *  - Memory: every pointer argument is caller-owned. Pointers documented as
 *    "device" must be device memory of the current HIP device; "host" pointers
 *    are ordinary host memory. The library keeps no pointer after a call returns,
 *    except where a server request says otherwise.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream). alif_forward / alif_backward and the other compute calls only
 *    enqueue work on that stream and never synchronise the device.
 *  - Layout: every per-step tensor is row-major [B][T][N] (batch, step, neuron),
 *    neuron innermost, so that 64 lanes of a wavefront read 64 consecutive
 *    neurons of one step.
 *  - T_R = round(arp_ms / dt_ms) must be a whole number of steps (within 1e-9
 *    relative) and 2 <= T_R <= ALIF_MAX_TR. With T_R = 1 the block model is not
 *    the standard model (the reset of Eq. 2 already silences the step after a
 *    spike, which a one-step block cannot express), so it is rejected.
 *  - T need not be a multiple of T_R: the last block is zero-padded (footnote to
 *    Section 3, "Blocks") and padded steps are never written.
 *  - Parameter VALUES live in device memory, so they are checked on the device:
 *    a neuron with tau_mem <= 0, tau_adapt <= 0, theta0 <= 0, d < 0 or a NaN
 *    parameter produces unspecified outputs and sets ALIF_STATUS_BAD_PARAM in the
 *    device status word, read with alif_device_status(). (theta0 > 0 and d >= 0
 *    keep the threshold positive, so a reset neuron at V = 0 cannot fire during
 *    its refractory steps -- the premise of "at most one spike per block".)
 */
#ifndef BLOCKALIF_H
#define BLOCKALIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define ALIF_OK            0
#define ALIF_PENDING       1
#define ALIF_EINVAL       (-1)  /* bad size, pointer, enum or T_R */
#define ALIF_ENOMEM       (-2)  /* host or device allocation failed */
#define ALIF_EHIP         (-3)  /* a HIP runtime call failed (message has the HIP error) */
#define ALIF_EBUDGET      (-4)  /* serving: request footprint exceeds the server budget */
#define ALIF_ENOTFOUND    (-5)  /* serving: unknown ticket */
#define ALIF_EUNSUPPORTED (-6)  /* valid request the build does not cover (e.g. T_R too large) */
#define ALIF_ESHUTDOWN    (-7)  /* serving: server is shutting down */

#define ALIF_MAX_TR 128          /* largest block length (steps) the kernels are built for */

/* device status word bits (alif_device_status) */
#define ALIF_STATUS_BAD_PARAM 1u

/* ---- enums ----------------------------------------------------------------- */
enum alif_input_kind {
    ALIF_INPUT_CURRENT_F32 = 0, /* input is the current I~ itself, float [B][T][N] */
    ALIF_INPUT_SPIKES_U8   = 1, /* input is presynaptic spikes x, uint8 0/1 [B][T][n_in] */
    ALIF_INPUT_SPIKES_BF16 = 2, /* x as bfloat16 0/1 [B][T][n_in] (exact) */
    ALIF_INPUT_SPIKES_F32  = 3  /* x as float 0/1 [B][T][n_in] */
};
enum alif_gemm_precision {
    ALIF_GEMM_FP32 = 0,  /* I~ = b + W x with FP32 MFMA (v_mfma_f32_16x16x4_f32) */
    ALIF_GEMM_BF16 = 1   /* W and x rounded to bfloat16, FP32 accumulation (MFMA) */
};
enum alif_spike_dtype { ALIF_SPIKES_U8 = 0, ALIF_SPIKES_BF16 = 1, ALIF_SPIKES_F32 = 2 };
enum alif_algo {
    ALIF_ALGO_BLOCKS          = 0, /* the block-wise method (default) */
    ALIF_ALGO_SEQUENTIAL      = 1, /* baseline: one thread per (b, neuron), fused loop over t */
    ALIF_ALGO_SEQUENTIAL_STEP = 2  /* baseline: one kernel launch per time step */
};
/* Surrogate derivative dS/du of the backward, u = V - th (supplementary
 * "Surrogate gradient"; the multi-Gaussian constants as printed there). */
enum alif_surrogate {
    ALIF_SG_FAST_SIGMOID   = 0, /* (k|u| + 1)^-2, k = sg_slope */
    ALIF_SG_BOXCAR         = 1, /* 0.5 where |u| <= 0.5, else 0 */
    ALIF_SG_MULTI_GAUSSIAN = 2  /* 1.15 N(u|0, 0.5^2) - 0.15 N(u|3, 3^2) - 0.15 N(u|-3, 3^2) */
};

/* Gradient policy of the backward (supplementary "Detaching gradients"). Detached:
 * the spike's uses in the reset of V[t+1] and in the adaptation jump of a[t+1] are
 * constants; gradient flows through the feedforward connections only. Attached:
 * those uses stay in the gradient, dV[t+1]/dS[t] = -(beta V[t] + (1 - beta) I[t+1])
 * (the membrane the reset removes) and da[t+1]/dS[t] = 1. The ARP gate is a step
 * function of the spike history under both. */
enum alif_grad_policy {
    ALIF_GRAD_DETACHED = 0,
    ALIF_GRAD_ATTACHED = 1   /* ALIF_ALGO_SEQUENTIAL backward only; blocks: ALIF_EUNSUPPORTED */
};

/* ---- problem descriptor ------------------------------------------------------ */
typedef struct alif_desc {
    int32_t batch;          /* B >= 0 */
    int32_t n_in;           /* presynaptic channels (spike input); ignored for current input */
    int32_t n_neurons;      /* N >= 0 */
    int32_t T;              /* steps >= 0 */
    double  dt_ms;          /* step size DT > 0 */
    double  arp_ms;         /* absolute refractory period; T_R = round(arp_ms / dt_ms) */
    int32_t input_kind;     /* enum alif_input_kind */
    int32_t gemm_precision; /* enum alif_gemm_precision (spike input only) */
    int32_t spike_dtype;    /* enum alif_spike_dtype of the spike output */
    int32_t algo;           /* enum alif_algo */
    int32_t surrogate;      /* enum alif_surrogate */
    float   sg_slope;       /* fast-sigmoid slope k (supplementary uses 10); >= 0 */
    int32_t grad_policy;    /* enum alif_grad_policy (0 = detached) */
} alif_desc;

/* Per-neuron parameters, device float [N] each (Eqs. 2-5). bias may be NULL (= 0). */
typedef struct alif_params {
    const float *tau_mem_ms;   /* > 0;  beta = exp(-DT / tau_mem) */
    const float *tau_adapt_ms; /* > 0;  p = exp(-DT / tau_adapt) */
    const float *d;            /* >= 0; adaptation scalar: threshold jump per spike */
    const float *theta0;       /* > 0;  baseline threshold */
    const float *bias;         /* b of Eq. 3, or NULL */
} alif_params;

/*
 * Complete simulation state at a block boundary (Props. 4-5: the membrane carried
 * into the next block, the adaptation variable and where the last block's spike
 * fell, which fixes the next block's refractory mask, Prop. 3). Device [B][N] each.
 * Running T steps in one call equals running it in pieces whose lengths are
 * multiples of T_R, passing `final` of one piece as `init` of the next.
 */
typedef struct alif_state {
    double  *v;   /* membrane potential at the boundary; 0 if the last block spiked */
    double  *a;   /* adaptation a at the boundary */
    int32_t *ts;  /* 1..T_R: step of the last block's spike, 0: none */
} alif_state;

/* ---- sizes ----------------------------------------------------------------- */

/* T_R for dt/arp, or a negative status if they do not give 2 <= T_R <= ALIF_MAX_TR. */
int alif_refractory_steps(double dt_ms, double arp_ms);

/* Bytes of the block-carry buffer alif_forward writes for alif_backward.
 * ALIF_ALGO_BLOCKS: the carry-in (V0 float, a float, previous spike step u8)
 * of every block plus the final carry, 9 bytes per (b, block + 1, neuron);
 * ALIF_ALGO_SEQUENTIAL: FP64 state checkpoints every T_R steps, 20 bytes per
 * (b, block, neuron); ALIF_ALGO_PER_STEP: the state of one step. Each part is
 * 256-byte aligned. */
int alif_carry_bytes(const alif_desc *desc, size_t *bytes);

/* Bytes of device scratch alif_backward needs (per-(b, neuron) FP64 partial sums). */
int alif_backward_workspace_bytes(const alif_desc *desc, size_t *bytes);

/* ---- compute ----------------------------------------------------------------- */

/*
 * Decay tables (supplementary "Weight initialisation": beta = exp(-DT/tau_mem),
 * p = exp(-DT/tau_adapt); Props. 1 and 5 use their powers). Computes in FP64
 * and rounds once to FP32: beta_pow[n][k] = beta_n^k, p_pow[n][k] = p_n^k for
 * k = 0..T_R. Device outputs float [N][T_R + 1], either may be NULL. The
 * forward and backward kernels build the same tables in their prologue; this
 * entry point exposes them for checking.
 */
int alif_decay_tables(const alif_desc *desc, const alif_params *prm,
                      float *beta_pow, float *p_pow, void *stream);

/*
 * Input current of Eq. 3 (feedforward part plus bias), the dense projection
 * I~[b][t][:] = bias + W x[b][t][:], as an MFMA GEMM on gfx950.
 *   input   device spikes [B][T][n_in] of desc->input_kind (0/1 values)
 *   W       device float [N][n_in]; bias device float [N] or NULL
 *   current device float [B][T][N] output
 * FP32 precision uses FP32 MFMA; BF16 rounds W to bfloat16 (x is exact) and
 * accumulates in FP32.
 */
int alif_input_current(const alif_desc *desc, const void *input, const float *W,
                       const float *bias, float *current, void *stream);

/*
 * The same input current of Eq. 3, I~[b][t][i] = bias[i] + sum_j W[i][j] x[b][t][j],
 * computed from the active inputs only: for each (b, t) row the nonzero entries
 * of x are found and their weight columns summed (FP32, value times weight; the
 * order is fixed by n_in, the input kind and the row alignment, so results are
 * reproducible), instead of a dense MFMA GEMM. For sparse spike
 * trains (a few percent of the entries or fewer) this moves the bytes the
 * result needs instead of doing n_in multiply-adds per output.
 *   desc     B, T, n_in, n_neurons and a spike input_kind (gemm_precision ignored)
 *   input    device spikes [B][T][n_in] of desc->input_kind (any values, 0 skipped)
 *   WT       device float [n_in][N]: W transposed (alif_transpose(N, n_in, W, WT))
 *   bias     device float [N] or NULL;  current  device float [B][T][N] output
 * Pass `current` to alif_forward as ALIF_INPUT_CURRENT_F32 input (with bias NULL
 * in that call's params, or computed here with bias NULL). The dW and dx of the
 * backward are alif_weight_grad and alif_input_grad as for the GEMM path.
 * Entries whose magnitude is zero (+0 and -0) are skipped. Buffers must be aligned
 * to their element type (ALIF_EINVAL otherwise); rows that start on 4-byte
 * boundaries are read as 32-bit words.
 *
 * alif_transpose: out[c][r] = in[r][c] for a device float rows x cols matrix
 * (out must not alias in; ALIF_EUNSUPPORTED for rows > 65535 * 32).
 */
int alif_transpose(int32_t rows, int32_t cols, const float *in, float *out, void *stream);
int alif_input_current_events(const alif_desc *desc, const void *input, const float *WT, const float *bias,
                              float *current, void *stream);

/*
 * Gradients of the Eq. 3 projection for a spike-input layer, given the gradient
 * of the loss with respect to its input current (what alif_backward writes to
 * grad_current), as MFMA GEMMs in desc->gemm_precision (BF16 rounds
 * grad_current and W to bfloat16 and accumulates in FP32):
 *   alif_weight_grad  grad_W[n][i] = sum over b, t of grad_current[b][t][n] x[b][t][i]
 *                     (device float [N][n_in]); the sum over b, t is split into
 *                     partial sums in `workspace` (device, of
 *                     alif_weight_grad_workspace_bytes() bytes; NULL when that is 0)
 *                     and reduced in a fixed order, so results are reproducible
 *   alif_input_grad   grad_input[b][t][i] = sum over n of grad_current[b][t][n] W[n][i]
 *                     (device float [B][T][n_in]), the gradient passed to the layer
 *                     below as its spike gradient
 * input: device spikes [B][T][n_in] of desc->input_kind; W device float
 * [N][n_in]; grad_current device float [B][T][N]. alif_backward makes the same
 * two calls when given grad_W / grad_input.
 */
int alif_weight_grad_workspace_bytes(const alif_desc *desc, size_t *bytes);
int alif_weight_grad(const alif_desc *desc, const float *grad_current, const void *input,
                     float *grad_W, void *workspace, void *stream);
int alif_input_grad(const alif_desc *desc, const float *grad_current, const float *W,
                    float *grad_input, void *stream);

/*
 * Forward pass of one ALIF layer over T steps (Eqs. 1-5 computed by Blocks,
 * Props. 1-5; or, with desc->algo, by the sequential baselines).
 *   input    device: current float [B][T][N] (ALIF_INPUT_CURRENT_F32; the bias is
 *            still added) or spikes [B][T][n_in] (then W is required)
 *   W        device float [N][n_in] or NULL for current input
 *   current  device float [B][T][N] workspace receiving b + W x for spike input
 *            (keep it for alif_backward); must be NULL for current input. It is
 *            the GEMM of desc->gemm_precision, or, for inputs of more than 2^24
 *            entries that a device-side sample of rows puts at most one in 16
 *            (FP32 GEMMs), one in 64 (BF16, N >= 256) or one in 256 (BF16, smaller
 *            N) nonzero, the sum over the nonzero inputs in FP32 (W rounded to
 *            bfloat16 under BF16 GEMMs, as the GEMM rounds it), computed in
 *            `spikes` as scratch before the block kernel writes it
 *   init     initial state or NULL (= zeros, no earlier spike)
 *   final    state after step T or NULL; requires T % T_R == 0
 *   spikes   device [B][T][N] of desc->spike_dtype (required)
 *   v, theta device float [B][T][N] membrane / threshold traces, or NULL
 *   carries  device buffer of alif_carry_bytes() for alif_backward, or NULL
 * Returns ALIF_OK after enqueueing; errors are reported before any work is queued.
 */
int alif_forward(const alif_desc *desc, const alif_params *prm,
                 const void *input, const float *W, float *current,
                 const alif_state *init, alif_state *final,
                 void *spikes, float *v, float *theta,
                 void *carries, void *stream);

/*
 * Surrogate-gradient backward pass of alif_forward under the paper's "detached"
 * policy (supplementary "Detaching gradients"; surrogate desc->surrogate,
 * supplementary "Surrogate gradient"): spikes pass gradient to the loss and to
 * downstream layers; their uses in reset, adaptation and refractory gate are
 * constants. Each block is recomputed from the input and its saved carry, then
 * the reverse recurrences run over blocks in reverse order.
 *   desc, prm, input, W, current  exactly as given to alif_forward (current:
 *            the workspace alif_forward filled, NULL for current input)
 *   carries  the buffer alif_forward filled (it holds every block's carry-in,
 *            including the init state's)
 *   grad_spikes, grad_v, grad_theta  device float [B][T][N] upstream gradients,
 *            each nullable (= 0)
 *   grad_current  device float [B][T][N]: gradient w.r.t. I~ (the input current);
 *            required when grad_W or grad_input (spike input) is requested,
 *            otherwise nullable. Exception: with BF16 GEMMs, the blocks
 *            algorithm, the detached policy, no grad_v / grad_theta and
 *            n_neurons a multiple of 8 it may be NULL; the block backward then
 *            writes the gradient as bfloat16 (round to nearest even, the
 *            rounding the BF16 GEMMs apply to it) into the workspace, and
 *            grad_W and grad_input are bit for bit the same as with a float
 *            grad_current, at half its bytes and with no conversion in the
 *            GEMMs
 *   grad_input    spike input only: device float [B][T][n_in] = grad_current W;
 *            nullable. (For current input the gradient is grad_current.)
 *   grad_W        device float [N][n_in] = sum_{b,t} grad_current^T x; nullable.
 *            With at most one nonzero per 256 entries of x (counted on the
 *            device, after a sampled estimate on inputs above 2^24 entries) it is
 *            summed over the nonzero entries (FP32, fixed order; grad_current
 *            rounded to bfloat16 under BF16 GEMMs), else it is the GEMM of
 *            desc->gemm_precision; deterministic either way
 *   grad_bias, grad_tau_mem, grad_tau_adapt, grad_d, grad_theta0
 *            device float [N], summed over the batch; each nullable
 *   workspace device scratch of alif_backward_workspace_bytes() bytes (with
 *            spike input and BF16 GEMMs it includes 2 B T N bytes for the
 *            bfloat16 gradient above)
 * desc->grad_policy ALIF_GRAD_ATTACHED keeps the spike's reset and adaptation uses
 * in the gradient (supplementary "Detaching gradients"): the block backward then
 * composes the per-step adjoint as 2 x 2 affine maps of (lambda_V, lambda_a) in
 * FP64 (the coupled recurrence can amplify rounding by many orders of magnitude);
 * the sequential backward evaluates it step by step in FP64. The sequential
 * backward stages one block in LDS and takes T_R <= 121 (<= 88 with grad_v or
 * grad_theta). The per-step-launch algorithm has no backward. Both limits are
 * ALIF_EUNSUPPORTED, reported before any work is queued.
 */
int alif_backward(const alif_desc *desc, const alif_params *prm,
                  const void *input, const float *W, const float *current,
                  const void *carries,
                  const float *grad_spikes, const float *grad_v, const float *grad_theta,
                  float *grad_current, float *grad_input, float *grad_W,
                  float *grad_bias, float *grad_tau_mem, float *grad_tau_adapt,
                  float *grad_d, float *grad_theta0,
                  void *workspace, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving or training loops, harnesses that forbid hipMalloc): the same
 * backward as alif_backward, same arguments and results, without the workspace
 * argument. Its scratch (the FP64 partial sums, 40 bytes per (b, neuron), plus the
 * weight-gradient GEMM's split-K tiles when grad_W is requested for spike input)
 * lives in a static device array of ALIF_NOALLOC_SCRATCH_BYTES inside the library,
 * one per device, held until the process ends. This call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine. A problem whose scratch
 * exceeds the array (the parts of alif_backward_workspace_bytes the call uses:
 * the partial sums, the GEMM split tiles with grad_W, the rounded W with BF16
 * grad_input, the bfloat16 gradient without grad_current) is rejected with
 * ALIF_EUNSUPPORTED before any work is queued. Every call on one device shares that device's array and leaves the
 * last call's contents in it, so calls that overlap on one device (on different
 * streams, or from different threads) race and give wrong gradients; serialise
 * them on one stream. Each call writes every scratch byte it reads, so nothing
 * needs clearing between calls.
 */
#define ALIF_NOALLOC_SCRATCH_BYTES (16u << 20)
int alif_backward_noalloc(const alif_desc *desc, const alif_params *prm,
                          const void *input, const float *W, const float *current,
                          const void *carries, const float *grad_spikes,
                          const float *grad_v, const float *grad_theta,
                          float *grad_current, float *grad_input, float *grad_W,
                          float *grad_bias, float *grad_tau_mem, float *grad_tau_adapt,
                          float *grad_d, float *grad_theta0, void *stream);

/*
 * Recurrent layer: Eq. 3's input current with the recurrent term
 * sum_j W_rec[i][j] S_j[t - D] and transmission delay D (Section 2 takes
 * D = T_R, which Prop. 3 turns into block n + 1 receiving W_rec times the
 * spikes of block n; any D >= T_R keeps the source in a finished block).
 * The blocks run one after another. Each block's recurrent current is the sum of
 * the columns of W_rec of the neurons that spiked D steps earlier, in FP32 and in
 * increasing neuron order, added to `current`; the block then runs from the
 * previous block's FP64 carry. Layers of up to 256 neurons whose workgroup state
 * fits the LDS run the whole block loop in one launch (a workgroup per batch
 * element, spikes passed between blocks in LDS); others take two launches per
 * block (the recurrent current, then the block kernel). Both give the same
 * values. No initial or final state: the run starts from rest with no earlier
 * spike.
 *   desc, prm   as alif_forward; desc->algo must be ALIF_ALGO_BLOCKS;
 *               desc->gemm_precision applies to the feedforward GEMM
 *   input, W    as alif_forward (current input: float [B][T][N]; spike input:
 *               spikes [B][T][n_in] and W [N][n_in])
 *   W_rec       device float [N][N]
 *   delay       D in steps; 0 means T_R; D < T_R is rejected (ALIF_EINVAL)
 *   current     device float [B][T][N], required: receives the whole current,
 *               b + W x + W_rec S[t - T_R] for spike input, input + W_rec S[t - T_R]
 *               for current input (the bias then added in-kernel, as
 *               alif_forward does). Pass it to alif_backward as `current` (spike
 *               input) or as `input` (current input): under the detached policy
 *               the recurrent current is a constant of the spike path, so the
 *               ordinary backward applies.
 *   spikes, v, theta, carries   as alif_forward
 *   workspace   device scratch of alif_recurrent_workspace_bytes() bytes,
 *               256-byte aligned (as hipMalloc returns)
 * alif_recurrent_weight_grad: grad_W_rec[i][j] = sum over b, t >= D of
 * grad_current[b][t][i] S[b][t - D][j] (device float [N][N]), from the spikes
 * alif_forward_recurrent wrote (desc->spike_dtype), the same delay and the same
 * workspace size (ALIF_EINVAL if it is not 256-byte aligned). The spikes are
 * counted on the device first. With at most one nonzero per 256 entries of the
 * source steps (B (T - D) N of them) the sum runs over the nonzero spikes only:
 * each adds its
 * value times a row of grad_current, in FP32, in increasing (b, t) order per
 * segment of the run and the segments' sums in order (no GEMM; gemm_precision
 * does not apply). Otherwise it is the GEMM of desc->gemm_precision over the
 * shifted spikes. Either way the result is deterministic. Asynchronous on
 * `stream`; the choice is made on the device.
 */
int alif_recurrent_workspace_bytes(const alif_desc *desc, size_t *bytes);
int alif_forward_recurrent(const alif_desc *desc, const alif_params *prm,
                           const void *input, const float *W, const float *W_rec,
                           int32_t delay, float *current, void *spikes, float *v,
                           float *theta, void *carries, void *workspace, void *stream);
int alif_recurrent_weight_grad(const alif_desc *desc, int32_t delay,
                               const float *grad_current, const void *spikes,
                               float *grad_W_rec, void *workspace, void *stream);

/*
 * Leaky non-spiking readout (supplementary "Readout neurons"): the membrane of
 * Eq. 2 without spike, reset or refractory gate, driven by I_r = W_r S, with
 * output o[b][c] = sum_t V_r[b][t][c].
 *   spikes  device [B][T][n_hidden] of spike_dtype (0/1)
 *   W_r     device float [C][n_hidden]; tau_r device float [C] (> 0)
 *   o       device float [B][C] output
 * Backward: given go [B][C] returns grad_spikes [B][T][n_hidden] (float),
 * grad_W_r [C][n_hidden] and grad_tau_r [C] (each nullable). workspace is device
 * memory of alif_readout_workspace_bytes() bytes; alif_readout_forward stores the
 * readout current and membrane there and alif_readout_backward reads them, so
 * the same workspace must be passed to both, unchanged in between.
 */
int alif_readout_workspace_bytes(int32_t B, int32_t T, int32_t n_hidden, int32_t C,
                                 size_t *bytes);
int alif_readout_forward(int32_t B, int32_t T, int32_t n_hidden, int32_t C, double dt_ms,
                         int32_t spike_dtype, const void *spikes, const float *W_r,
                         const float *tau_r, float *o, void *workspace, void *stream);
int alif_readout_backward(int32_t B, int32_t T, int32_t n_hidden, int32_t C, double dt_ms,
                          int32_t spike_dtype, const void *spikes, const float *W_r,
                          const float *tau_r, const float *go, float *grad_spikes,
                          float *grad_W_r, float *grad_tau_r, void *workspace, void *stream);

/* ---- neural fits: van Rossum loss and Adam (supplementary "Neural fits") ------ */

/*
 * Van Rossum distance (supplementary "Supervised training loss") between model
 * spike trains and recorded ones, with its gradient for alif_backward's
 * grad_spikes. On the simulation grid a spike (or a count) at step s is an
 * impulse of unit area, the exponential kernel is H(t) exp(-t / tau_R) with
 * H(0) = 1, and the integral over the T steps is DT times a sum:
 *   e[t] = sum_{s <= t} a^(t - s) (x[s] - y[s]),  a = exp(-dt_ms / tau_ms),
 *   D    = sqrt((dt_ms / tau_ms) sum_{t < T} e[t]^2).
 *   B, R, T, N  batch, repeats per model train (1..8), steps, neurons; any may be 0
 *   spikes      device uint8 [B][T][N]: the model's trains (0/1 or counts)
 *   targets     device uint8 [B][R][T][N]: R recorded trains per model train
 *               (repeats of the same stimulus), spike counts per step
 *   dist        device float [B][R][N]: D of each (model train, repeat, neuron),
 *               or NULL
 *   grad        device float [B][T][N] = scale * sum_r dD[b][r][n] / dx[b][t][n],
 *               or NULL; where D = 0 that term's gradient is 0 (subgradient)
 *   workspace   device scratch of alif_van_rossum_workspace_bytes(B, R, T, N)
 * With N % 4 == 0, spikes and targets must be 4-byte and grad 16-byte aligned.
 * Sums run in FP64 per time chunk, the gradient recurrence in FP32.
 * ALIF_EINVAL for bad sizes, dt_ms or tau_ms <= 0, or NULL buffers;
 * ALIF_EUNSUPPORTED for R > 8. Errors are reported before any work is queued.
 */
int alif_van_rossum_workspace_bytes(int32_t B, int32_t R, int32_t T, int32_t N, size_t *bytes);
int alif_van_rossum(int32_t B, int32_t R, int32_t T, int32_t N, double dt_ms, double tau_ms,
                    const uint8_t *spikes, const uint8_t *targets, float scale,
                    float *dist, float *grad, void *workspace, void *stream);

/*
 * One Adam step (Kingma and Ba, Algorithm 1; the neural fits' optimiser) over n
 * device floats, in place, then the parameter is clamped to [lo, hi] (keeps time
 * constants and thresholds valid). step counts from 1; m and v start at 0 and
 * are kept by the caller between steps. The update runs in FP32; 1 - beta and
 * the bias corrections are formed in FP64 from the given values and rounded once.
 * ALIF_EINVAL for step < 1, beta outside [0, 1), eps <= 0, lo > hi or NULL buffers.
 */
int alif_adam_step(int32_t n, float *param, const float *grad, float *m, float *v, int32_t step,
                   double lr, double beta1, double beta2, double eps, float lo, float hi, void *stream);

/* Copies the device status word (ALIF_STATUS_* bits OR-ed by kernels on the
 * current device since the last call) to *bits and clears it. Synchronises
 * `stream`. */
int alif_device_status(uint32_t *bits, void *stream);

/* Message for the last error on this thread (empty string if none). */
const char *alif_last_error(void);

/* ---- Ornstein-Uhlenbeck input current --------------------------------------- */

/*
 * Writes the device float [T][N] current I[t] = mean + X[t] of independent OU
 * processes, discretised exactly with e = exp(-dt_ms / tau_ms):
 *   X[0] = sd z_0,  X[t] = e X[t-1] + sd sqrt(1 - e^2) z_t,
 * evaluated in FP64 and rounded once to float. z_t of neuron n is a standard
 * normal from Philox4x32-10 (Salmon et al., SC 2011; key = seed, low word
 * first; counter (t / 4, n, 0, 0)) through Box-Muller in FP64: with output
 * words (w0, w1, w2, w3), u1 = (w_2j + 1) / 2^32, u2 = w_2j+1 / 2^32 and
 * r = sqrt(-2 ln u1), step 4q + 2j takes r cos(2 pi u2) and step 4q + 2j + 1
 * takes r sin(2 pi u2). The same (seed, n, t) always gives the same value,
 * independent of T and N. workspace: device, alif_ou_workspace_bytes(T, N)
 * bytes. Needs tau_ms > 0, sd >= 0, dt_ms > 0.
 */
int alif_ou_workspace_bytes(int32_t T, int32_t n_neurons, size_t *bytes);
int alif_ou_current(int32_t T, int32_t n_neurons, double dt_ms, float tau_ms, float mean, float sd,
                    uint64_t seed, float *current, void *workspace, size_t workspace_bytes,
                    void *stream);

/* ---- serving: continuous batching of independent simulations ---------------- */

typedef struct alif_server alif_server;

enum alif_request_input {
    ALIF_REQ_HOST_CURRENT = 0, /* host float [T][N] current, caller-owned until done */
    ALIF_REQ_OU           = 1  /* Ornstein-Uhlenbeck current drawn on the device */
};

/*
 * One single-layer simulation request (forward only, batch 1). Parameters are
 * host float [N] arrays copied at submit. ALIF_REQ_OU draws the current on the
 * device exactly as alif_ou_current does (with the request's dt_ms, ou_tau_ms,
 * ou_mean, ou_sd and seed).
 *
 * Outputs (either, both or neither):
 *  - host_spikes: the dense uint8 [T][N] spike raster;
 *  - host_events: the spikes as flat indices t * N + n (uint32, ascending, so
 *    ordered by step, then neuron), at most events_capacity of them; the result
 *    says how many spikes there were and whether the list was cut short. At
 *    these firing rates this is orders of magnitude smaller than the raster, and
 *    it is what crosses PCIe.
 * host_current (if used), host_spikes and host_events must stay valid until
 * alif_poll has returned the request's result.
 */
typedef struct alif_request {
    int32_t n_neurons;
    int32_t T;
    double  dt_ms;
    double  arp_ms;
    const float *tau_mem_ms, *tau_adapt_ms, *d, *theta0, *bias; /* host [N]; bias nullable */
    int32_t input;             /* enum alif_request_input */
    const float *host_current; /* ALIF_REQ_HOST_CURRENT: host [T][N] */
    float ou_tau_ms, ou_mean, ou_sd;
    uint64_t seed;
    uint8_t *host_spikes;      /* host [T][N] raster, caller-owned, nullable */
    uint32_t *host_events;     /* host [events_capacity] spike indices, caller-owned, nullable */
    int64_t events_capacity;
} alif_request;

typedef struct alif_result {
    int32_t status;            /* ALIF_OK, or the request's error */
    int32_t events_truncated;  /* 1 if n_spikes > events_capacity (host_events holds the first ones) */
    int64_t n_spikes;
    double  t_submit_s, t_admit_s, t_done_s; /* server clock (CLOCK_MONOTONIC), seconds */
} alif_result;

/*
 * Continuous batching: a scheduler thread admits queued requests in arrival
 * order whenever one of max_slots slots is free and the request's footprint
 * fits in what is left of hbm_budget_bytes, and runs each on its slot's own
 * stream on `device` (default priority), so that requests that arrive while
 * others run overlap on the GPU. A request's result does not depend on what
 * else is resident. 1 <= max_slots <= 64. Device memory for a request is taken
 * from HIP's stream-ordered allocator at admission and returned on completion;
 * each slot also keeps pinned host staging, grown to the largest request it
 * has served.
 */
int alif_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t device,
                       alif_server **out);
/* Device bytes a request holds while resident (its admission footprint). */
int alif_request_footprint(const alif_request *req, size_t *bytes);
/* Validates and enqueues; returns at once. ALIF_EBUDGET if it can never fit. */
int alif_submit(alif_server *srv, const alif_request *req, uint64_t *ticket);
/* ALIF_PENDING until the request is done; then fills *res and forgets the ticket. */
int alif_poll(alif_server *srv, uint64_t ticket, alif_result *res);
/* Blocks until every submitted request is done, then stops the scheduler. */
int alif_server_destroy(alif_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* BLOCKALIF_H */
