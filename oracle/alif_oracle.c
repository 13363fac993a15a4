/*
 * FP64 CPU oracle for the standard ALIF network -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library. The GPU library never links, includes or calls it, and
 * it shares no code with the GPU library.
 *
 * What it computes: the plain, step-by-step standard ALIF neuron of the paper's
 * Section 2 ("Standard ALIF model", Equations 1-5), one independent row
 * (one (batch, neuron) pair) at a time, in double precision:
 *
 *   I~[t] = b + sum_j W[j] x_j[t]                     (Eq. 3, feedforward part)
 *   I[t]  = I~[t] if C[t] >= T_R else 0               (Eq. 4; C = steps since last spike)
 *   V[t]  = (beta V[t-1] + (1-beta) I[t]) (1 - S[t-1]) (Eq. 2)
 *   a[t]  = p a[t-1] + S[t-1]                         (Eq. 5)
 *   th[t] = theta0 + d a[t]                           (Eq. 5, baseline threshold theta0)
 *   S[t]  = 1[V[t] > th[t]]                           (Eq. 1, strict)
 *
 * with beta = exp(-DT/tau_mem), p = exp(-DT/tau_adapt) (supplementary "Weight
 * initialisation"), V = a = 0 and no earlier spike (C = infinity) before t = 1.
 *
 * The adjoint (oracle_alif_backward) is the sequential surrogate gradient of the
 * same recurrence under the paper's "detached" policy (supplementary "Detaching
 * gradients"): the spike enters the loss and the next layer through a surrogate
 * derivative (supplementary "Surrogate gradient"), while its uses in the reset
 * factor (1 - S[t-1]), in the adaptation increment and in the refractory mask are
 * constants. The leak path beta*V and the threshold path stay attached.
 *
 * Readings where the paper is silent:
 *   - T_R = round(ARP/DT) steps; C[t] = t - t_last, input passes iff C >= T_R.
 *   - The surrogate argument is u = V - th for every surrogate.
 *   - dS/dth = -sigma'(u) (the threshold is learnable here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of refractory steps T_R for an ARP and a step size (footnote to the
 * contributions list: T_R is a count of steps). Returns -1 when ARP/DT is not
 * within 1e-9 (relative) of a whole number or an argument is not positive. */
int oracle_refractory_steps(double dt_ms, double arp_ms)
{
    if (!(dt_ms > 0.0) || !(arp_ms > 0.0)) return -1;
    double r = arp_ms / dt_ms;
    double n = floor(r + 0.5);
    if (n < 1.0 || fabs(r - n) > 1e-9 * n) return -1;
    return (int)n;
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. 3, feedforward current with bias, for binary presynaptic spikes.
 * x: [M][n_in] (0/1 bytes), W: [n][n_in], bias: [n] or NULL, out: [M][n]. */
void oracle_input_current(int64_t M, int64_t n, int64_t n_in, const uint8_t *x,
                          const double *W, const double *bias, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; m++) {
        const uint8_t *xm = x + m * n_in;
        for (int64_t i = 0; i < n; i++) {
            const double *wi = W + i * n_in;
            double acc = bias ? bias[i] : 0.0;
            for (int64_t j = 0; j < n_in; j++)
                if (xm[j]) acc += wi[j];
            out[m * n + i] = acc;
        }
    }
}

/*
 * Standard ALIF forward, Eqs. 1-5, R independent rows of T steps.
 *   I      [R][T]  input current before the refractory mask (Eq. 3 output)
 *   tau_m, tau_a, d, theta0  [R]  per-row parameters (d is the adaptation scalar)
 *   force  [R][T]  optional: -1 = let Eq. 1 decide, 0/1 = impose that spike decision
 *                  (used to re-run the oracle on the decisions another
 *                  implementation took where the margin |V - th| is tiny)
 * Outputs [R][T]: S (0/1), V, TH, A (adaptation a[t]), MASK (1 if the input passed
 * the refractory gate at t).
 */
void oracle_alif_forward(int64_t R, int64_t T, const double *I,
                         const double *tau_m, const double *tau_a,
                         const double *d, const double *theta0,
                         double dt, int TR, const int8_t *force,
                         uint8_t *S, double *V, double *TH, double *A, uint8_t *MASK)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < R; r++) {
        const double beta = exp(-dt / tau_m[r]);
        const double p = exp(-dt / tau_a[r]);
        const double *Ir = I + r * T;
        double v = 0.0, a = 0.0;
        int s_prev = 0;
        int spiked_before = 0;
        int64_t t_last = 0;
        for (int64_t t = 0; t < T; t++) {
            /* Eq. 4: C = steps since the last spike, infinite before the first. */
            int pass = !spiked_before || (t - t_last) >= (int64_t)TR;
            double in = pass ? Ir[t] : 0.0;
            /* Eq. 2 */
            v = (beta * v + (1.0 - beta) * in) * (1.0 - (double)s_prev);
            /* Eq. 5 */
            a = p * a + (double)s_prev;
            double th = theta0[r] + d[r] * a;
            /* Eq. 1 */
            int s = v > th;
            if (force) {
                int8_t f = force[r * T + t];
                if (f >= 0) s = f;
            }
            if (s) { spiked_before = 1; t_last = t; }
            S[r * T + t] = (uint8_t)s;
            V[r * T + t] = v;
            TH[r * T + t] = th;
            A[r * T + t] = a;
            MASK[r * T + t] = (uint8_t)pass;
            s_prev = s;
        }
    }
}

/*
 * The recurrent network of Eqs. 1-5: Eq. 3's input current gains the recurrent
 * term sum_j W_rec[i][j] S_j[t - D] with transmission delay D (the paper takes
 * D = T_R; no spikes before t = 1, so the term is 0 for t <= D). All N neurons
 * of one batch element advance together, step by step.
 *   Iff   [B][T][N] the rest of the current (bias + feedforward), FP64
 *   Wrec  [N][N]    recurrent weights
 *   force [B][T][N] or NULL: as in oracle_alif_forward
 * Outputs [B][T][N]: S, V, TH, A, MASK and Itot (the whole Eq. 3 current).
 */
void oracle_alif_forward_recurrent(int64_t B, int64_t T, int64_t N, const double *Iff,
                                   const double *Wrec, const double *tau_m, const double *tau_a,
                                   const double *d, const double *theta0, double dt, int TR, int D,
                                   const int8_t *force, uint8_t *S, double *V, double *TH,
                                   double *A, uint8_t *MASK, double *Itot)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < B; b++) {
        double *v = calloc((size_t)N, sizeof(double));
        double *a = calloc((size_t)N, sizeof(double));
        int *s_prev = calloc((size_t)N, sizeof(int));
        int *spiked = calloc((size_t)N, sizeof(int));
        int64_t *t_last = calloc((size_t)N, sizeof(int64_t));
        for (int64_t t = 0; t < T; t++) {
            const int64_t o = (b * T + t) * N;
            const int64_t od = (b * T + t - D) * N;   /* step t - D of the same batch element */
            for (int64_t i = 0; i < N; i++) {
                const double beta = exp(-dt / tau_m[i]);
                const double p = exp(-dt / tau_a[i]);
                /* Eq. 3 with the recurrent current */
                double cur = Iff[o + i];
                if (t - D >= 0)
                    for (int64_t j = 0; j < N; j++)
                        if (S[od + j]) cur += Wrec[i * N + j];
                Itot[o + i] = cur;
                /* Eq. 4 */
                const int pass = !spiked[i] || (t - t_last[i]) >= (int64_t)TR;
                const double in = pass ? cur : 0.0;
                /* Eq. 2 */
                v[i] = (beta * v[i] + (1.0 - beta) * in) * (1.0 - (double)s_prev[i]);
                /* Eq. 5 */
                a[i] = p * a[i] + (double)s_prev[i];
                const double th = theta0[i] + d[i] * a[i];
                /* Eq. 1 */
                int s1 = v[i] > th;
                if (force && force[o + i] >= 0) s1 = force[o + i];
                if (s1) { spiked[i] = 1; t_last[i] = t; }
                S[o + i] = (uint8_t)s1;
                V[o + i] = v[i];
                TH[o + i] = th;
                A[o + i] = a[i];
                MASK[o + i] = (uint8_t)pass;
            }
            for (int64_t i = 0; i < N; i++) s_prev[i] = S[o + i];
        }
        free(v); free(a); free(s_prev); free(spiked); free(t_last);
    }
}

/* Normal density N(u | m, s^2). */
static double normal_pdf(double u, double m, double s)
{
    const double z = (u - m) / s;
    const double pi = 3.14159265358979323846;
    return exp(-0.5 * z * z) / (s * sqrt(2.0 * pi));
}

/*
 * The three surrogate derivatives dS/du the supplementary ("Surrogate gradient")
 * compares, with u = V - th for all of them:
 *   kind 0, fast sigmoid:   (k |u| + 1)^-2
 *   kind 1, boxcar:         0.5 where |u| <= 0.5, else 0
 *   kind 2, multi-Gaussian: 1.15 N(u | 0, 0.5^2) - 0.15 N(u | 3, 3^2) - 0.15 N(u | -3, 3^2)
 * The multi-Gaussian constants are the ones printed there.
 */
double oracle_surrogate(int kind, double u, double k)
{
    if (kind == 1) return fabs(u) <= 0.5 ? 0.5 : 0.0;
    if (kind == 2)
        return 1.15 * normal_pdf(u, 0.0, 0.5) - 0.15 * normal_pdf(u, 3.0, 3.0) -
               0.15 * normal_pdf(u, -3.0, 3.0);
    const double q = k * fabs(u) + 1.0;
    return 1.0 / (q * q);
}

/*
 * Adjoint of oracle_alif_forward, reverse over t with lambda_V[T+1] =
 * lambda_a[T+1] = 0 (sigma' is oracle_surrogate of `surrogate`):
 *   s        = sigma'(V[t] - th[t])
 *   lamS[t]  = gS[t]                                   (detached policy)
 *            = gS[t] - c[t] lamV[t+1] + lamA[t+1]      (attached: the spike also
 *              acts through the reset of V[t+1] and the jump of a[t+1], with
 *              c[t] = beta V[t] + (1 - beta) MASK[t+1] I[t+1], the membrane the
 *              reset removes, and dV[t+1]/dS[t] = -c[t], da[t+1]/dS[t] = 1)
 *   lamV[t]  = gV[t] + lamS[t] s + beta (1 - S[t]) lamV[t+1]
 *   lamTh[t] = gTh[t] - lamS[t] s
 *   lamA[t]  = d lamTh[t] + p lamA[t+1]
 *   gI[t]    = (1 - beta) MASK[t] (1 - S[t-1]) lamV[t]        (gradient w.r.t. I~[t])
 *   gbeta   += (1 - S[t-1]) (V[t-1] - MASK[t] I[t]) lamV[t]
 *   gp      += a[t-1] lamA[t];  gd += a[t] lamTh[t];  gtheta0 += lamTh[t]
 * then g_tau_m = gbeta beta DT / tau_m^2 and g_tau_a = gp p DT / tau_a^2.
 * The ARP gate MASK is a step function of the spike history: no gradient in
 * either policy. gS, gV, gTH: [R][T], each may be NULL (= zero). Outputs: gI
 * [R][T] (may be NULL), g_tau_m, g_tau_a, g_d, g_theta0 [R] (each may be NULL).
 */
void oracle_alif_backward(int64_t R, int64_t T, const double *I,
                          const double *tau_m, const double *tau_a,
                          const double *d, const double *theta0,
                          double dt, int surrogate, double slope, int attached,
                          const uint8_t *S, const double *V, const double *TH,
                          const double *A, const uint8_t *MASK,
                          const double *gS, const double *gV, const double *gTH,
                          double *gI, double *g_tau_m, double *g_tau_a,
                          double *g_d, double *g_theta0)
{
    (void)theta0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < R; r++) {
        const double beta = exp(-dt / tau_m[r]);
        const double p = exp(-dt / tau_a[r]);
        const int64_t o = r * T;
        double lamV_next = 0.0, lamA_next = 0.0;
        double gbeta = 0.0, gp = 0.0, gd = 0.0, gth0 = 0.0;
        for (int64_t t = T - 1; t >= 0; t--) {
            double sg = oracle_surrogate(surrogate, V[o + t] - TH[o + t], slope);
            double lamS = gS ? gS[o + t] : 0.0;
            if (attached && t + 1 < T) {
                double in_next = MASK[o + t + 1] ? I[o + t + 1] : 0.0;
                double c = beta * V[o + t] + (1.0 - beta) * in_next;
                lamS += -c * lamV_next + lamA_next;
            }
            double lamV = (gV ? gV[o + t] : 0.0) + lamS * sg
                        + beta * (1.0 - (double)S[o + t]) * lamV_next;
            double lamTh = (gTH ? gTH[o + t] : 0.0) - lamS * sg;
            double lamA = d[r] * lamTh + p * lamA_next;
            double s_prev = t > 0 ? (double)S[o + t - 1] : 0.0;
            double v_prev = t > 0 ? V[o + t - 1] : 0.0;
            double a_prev = t > 0 ? A[o + t - 1] : 0.0;
            double in = MASK[o + t] ? I[o + t] : 0.0;
            if (gI) gI[o + t] = (1.0 - beta) * (double)MASK[o + t] * (1.0 - s_prev) * lamV;
            gbeta += (1.0 - s_prev) * (v_prev - in) * lamV;
            gp += a_prev * lamA;
            gd += A[o + t] * lamTh;
            gth0 += lamTh;
            lamV_next = lamV;
            lamA_next = lamA;
        }
        if (g_tau_m) g_tau_m[r] = gbeta * beta * dt / (tau_m[r] * tau_m[r]);
        if (g_tau_a) g_tau_a[r] = gp * p * dt / (tau_a[r] * tau_a[r]);
        if (g_d) g_d[r] = gd;
        if (g_theta0) g_theta0[r] = gth0;
    }
}

/*
 * Leaky non-spiking readout (supplementary "Readout neurons"): the membrane of
 * Eq. 2 without spike, reset or refractory gate, summed over time.
 *   Vr[t] = beta_r Vr[t-1] + (1 - beta_r) Ir[t],  o = sum_t Vr[t]
 * Ir: [R][T] rows; out o: [R]. Backward with go[R]: lam[t] = go + beta_r lam[t+1],
 * gIr[t] = (1 - beta_r) lam[t], gbeta_r = sum_t (Vr[t-1] - Ir[t]) lam[t],
 * g_tau_r = gbeta_r beta_r DT / tau_r^2.
 */
void oracle_readout_forward(int64_t R, int64_t T, const double *Ir, const double *tau_r,
                            double dt, double *Vr, double *o)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; r++) {
        const double beta = exp(-dt / tau_r[r]);
        double v = 0.0, sum = 0.0;
        for (int64_t t = 0; t < T; t++) {
            v = beta * v + (1.0 - beta) * Ir[r * T + t];
            if (Vr) Vr[r * T + t] = v;
            sum += v;
        }
        o[r] = sum;
    }
}

void oracle_readout_backward(int64_t R, int64_t T, const double *Ir, const double *tau_r,
                             double dt, const double *go, double *gIr, double *g_tau_r)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; r++) {
        const double beta = exp(-dt / tau_r[r]);
        double *lam = (double *)malloc((size_t)(T > 0 ? T : 1) * sizeof(double));
        double *v = (double *)malloc((size_t)(T > 0 ? T : 1) * sizeof(double));
        double vt = 0.0;
        for (int64_t t = 0; t < T; t++) {           /* forward trace */
            vt = beta * vt + (1.0 - beta) * Ir[r * T + t];
            v[t] = vt;
        }
        double next = 0.0;
        for (int64_t t = T - 1; t >= 0; t--) {      /* reverse recurrence */
            lam[t] = go[r] + beta * next;
            next = lam[t];
        }
        double gbeta = 0.0;
        for (int64_t t = 0; t < T; t++) {
            double v_prev = t > 0 ? v[t - 1] : 0.0;
            if (gIr) gIr[r * T + t] = (1.0 - beta) * lam[t];
            gbeta += (v_prev - Ir[r * T + t]) * lam[t];
        }
        if (g_tau_r) g_tau_r[r] = gbeta * beta * dt / (tau_r[r] * tau_r[r]);
        free(lam);
        free(v);
    }
}
