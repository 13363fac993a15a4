// Internal launcher interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace alif {

// Records a message for alif_last_error() and returns `code`.
int set_error(int code, const char *msg);

// Block-carry checkpoint layout written by the block forward for the backward:
// three arrays [B][NB][N]: v0 (float), a0 (float), ts (uint8), 256-byte aligned.
struct CarryView {
    float *v;
    float *a;
    uint8_t *ts;
};
// Sequential-baseline checkpoint: [B][NB][N] of v (double), a (double), c (int32 =
// steps since the last spike, capped at T_R).
struct SeqCarryView {
    double *v;
    double *a;
    int32_t *c;
};

struct FwdArgs {
    int B, T, N, TR, NB, n_groups;
    double dt;
    const float *I;       // [B][T][N] current (without bias if bias_k != nullptr)
    const float *bias_k;  // added in-kernel, nullable
    const float *tau_m, *tau_a, *d, *theta0;
    const double *init_v, *init_a;
    const int32_t *init_ts;
    double *fin_v, *fin_a;
    int32_t *fin_ts;
    void *spikes;
    int spike_dtype;
    float *V, *TH;
    CarryView ck;
    unsigned *status;
    // Sub-range runs (0 = the defaults of a whole-tensor run): elements between
    // consecutive batch elements of I, V, TH (bs_i) and of spikes (bs_s), the
    // block dimension of the carry arrays (ck_nb) and the block index of this
    // run's first carry in them (ck_off).
    size_t bs_i, bs_s;
    int ck_nb, ck_off;
};

struct BwdArgs {
    int B, T, N, TR, NB, n_groups;
    double dt;
    int surrogate;  // enum alif_surrogate
    int attached;   // gradient policy: 1 = attached (reset and adaptation uses of the spike carry gradient)
    float slope;
    const float *I;
    const float *bias_k;
    const float *tau_m, *tau_a, *d, *theta0;
    CarryView ck;
    const float *gS, *gV, *gTH;
    float *gI;
    uint16_t *gI16;  // the same gradient as bfloat16 (round to nearest even), in place of gI
                     // (detached policy, no gV / gTH); nullptr: none
    double *part;  // [5][B][N]
};

// Recurrent layer in one launch (one workgroup per batch element)
struct RecArgs {
    int B, T, N, TR, NB;
    int D;                // recurrent delay in steps, >= T_R
    int ring;             // slots of the LDS ring of older blocks' spike steps (0 when D == T_R)
    double dt;
    const float *I_ff;    // [B][T][N] feed-forward current (may equal I)
    float *I;             // [B][T][N] the whole current (every row written)
    const float *bias_k;  // added in-kernel, nullable
    const float *tau_m, *tau_a, *d, *theta0;
    const float *WrecT;   // [N][N], WrecT[j][i] = W_rec[i][j]
    void *spikes;         // [B][T][N]
    int spike_dtype;
    float *V, *TH;
    CarryView ck;
    unsigned *status;
};

struct SeqArgs {
    int B, T, N, TR, NB;
    double dt;
    int surrogate;  // enum alif_surrogate (backward)
    int attached;   // gradient policy of the backward: 1 = attached
    float slope;
    const float *I;
    const float *bias_k;
    const float *tau_m, *tau_a, *d, *theta0;
    const double *init_v, *init_a;
    const int32_t *init_ts;
    double *fin_v, *fin_a;
    int32_t *fin_ts;
    void *spikes;
    int spike_dtype;
    float *V, *TH;
    SeqCarryView ck;
    const float *gS, *gV, *gTH;
    float *gI;
    double *part;
    unsigned *status;
    // per-step-launch baseline state [B][N]
    double *st_v, *st_a;
    int32_t *st_c;
    int step;
};

struct FinalizeArgs {
    int B, N;
    double dt;
    const float *tau_m, *tau_a;
    const double *part;  // [5][B][N]
    float *g_tau_m, *g_tau_a, *g_d, *g_theta0, *g_bias;
};

// (SEG, L) segmentation of a block of T_R steps over lanes; same for fwd and bwd.
struct BlockConfig {
    int seg, len;
};
BlockConfig block_config(int TR);
int block_neurons_per_wg(int seg);

hipError_t launch_blocks_fwd(const FwdArgs &a, hipStream_t st);
// spikes[b][n T_R + k][i] = blocks[n][b][k][i] (block n at byte offset n * blk_bytes), for n T_R + k < T
hipError_t launch_blocks_to_bt(int B, int T, int N, int TR, int elem, const void *blocks, size_t blk_bytes,
                               void *spikes, hipStream_t st);
// C[b][k][i] += sum_{j: S[b][t0 + k - D][j] != 0} WrecT[j][i] (b < B, k < rows; spikes from
// the block-major staging [NB][B][TR][N] of `elem`-byte elements, block m at m * blk_bytes;
// C rows of a [B][T][N] tensor at batch stride bstride; nothing where t0 + k < D)
hipError_t launch_recurrent_events(int B, int TR, int rows, int N, long long bstride, int t0, int D, int elem,
                                   const void *blocks, size_t blk_bytes, const float *WrecT, float *C,
                                   hipStream_t st);
// Whether the one-launch recurrent layer covers (N, T_R, D) (N <= 256 and the
// workgroup's LDS); launch it (alif_forward_recurrent's whole block loop).
bool recurrent_fused_ok(int N, int TR, int D);
int recurrent_ring_slots(int TR, int D);
hipError_t launch_recurrent_fused(const RecArgs &a, hipStream_t st);
// The weight gradient of a spike-driven projection from the spike events
// (dW[i][j] = sum over b and u < T - D of S[b][u][j] gI[b][u + D][i], Nj spike
// columns j, Ni gradient columns i; D = 0 for a feed-forward projection) into the
// workspace ws (256-byte aligned, wgrad_event_bytes(B, T, Nj, Ni) bytes, which
// bound every D >= 0). gI [B][T][Ni] is float (gi_mode 0), float rounded to
// bfloat16 as it is read (1) or bfloat16 (2). It counts the events into a device
// word first and computes dW only when they are few; *count and *thr (nullptr
// when the event path cannot take the shape) give the gate of the dense path
// enqueued behind it: dense runs when *count > *thr.
size_t wgrad_event_bytes(int B, int T, int Nj, int Ni);
hipError_t launch_wgrad_events(int B, int T, int Nj, int Ni, int D, int elem, const void *spikes, const void *gI,
                               int gi_mode, float *dW, void *ws, unsigned long long **count, unsigned long long *thr,
                               hipStream_t st);
// out[j][i] = in[i][j], N x N float
hipError_t launch_transpose(int N, const float *in, float *out, hipStream_t st);
// out[b][t][i] = in[b][t - D][i] for t >= D, else 0 (elements of `elem` bytes); with
// skip_cnt set the kernel returns at entry when *skip_cnt <= skip_le as it starts
hipError_t launch_shift_time(int B, int T, int N, int D, int elem, const void *in, void *out, hipStream_t st,
                             const unsigned long long *skip_cnt = nullptr, unsigned long long skip_le = 0);
hipError_t launch_blocks_bwd(const BwdArgs &a, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st);
hipError_t launch_decay_tables(int N, int TR, double dt, const float *tau_m, const float *tau_a,
                               float *beta_pow, float *p_pow, hipStream_t st);

hipError_t launch_seq_fwd(const SeqArgs &a, hipStream_t st);
hipError_t launch_seq_step_fwd(SeqArgs a, hipStream_t st);
hipError_t launch_seq_bwd(const SeqArgs &a, hipStream_t st);
int seq_bwd_max_tr(bool with_v_theta_grads);

}  // namespace alif
