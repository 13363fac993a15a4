// Serving: continuous batching of independent single-layer ALIF simulations,
// and the on-device Ornstein-Uhlenbeck current generator it uses.
//
// alif_submit copies a request into a FIFO queue and returns a ticket. A
// scheduler thread admits queued requests in arrival order whenever a slot is
// free and the request's device footprint fits in what is left of the HBM
// budget, and runs each admitted request on its slot's own stream, so that the
// work of requests that arrive while others are running overlaps on the device:
//   device allocation (stream-ordered) -> parameters H2D -> input current
//   (H2D from the slot's pinned staging, or OU drawn on the device) ->
//   block-wise forward (the kernels behind alif_forward) -> spike compaction
//   (count, scan, and a scatter of the spike indices straight into the slot's
//   pinned event staging) -> raster D2H if asked for -> free -> completion event.
// When the event has fired, the scheduler copies the results into the caller's
// buffers, releases the slot and the budget, and files the result for
// alif_poll. Every bulk host buffer the device touches is pinned: an async copy
// to pageable memory would block the scheduler thread until the copy ran, which
// would serialise the requests.
//
// OU current (exact discretisation of dX = -X/tau dt + noise, e = exp(-DT/tau)):
//   X[0] = sd z_0,  X[t] = e X[t-1] + sd sqrt(1 - e^2) z_t,  I[t] = mu + X[t],
// X in FP64, I rounded once to float. The standard normals come from
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011) with the 64-bit seed as key (low word first) and
// counter (t / 4, n, 0, 0) for neuron n; the output words (w0, w1) give the
// Box-Muller pair of steps 4q and 4q + 1, (w2, w3) that of 4q + 2 and 4q + 3:
//   u1 = (w_even + 1) / 2^32, u2 = w_odd / 2^32, r = sqrt(-2 ln u1),
//   z_{even step} = r cos(2 pi u2), z_{odd step} = r sin(2 pi u2)   (FP64).
// The linear recurrence is evaluated in chunks of OU_CHUNK steps: a first pass
// gives each chunk's end value started from zero, a second pass combines the
// ends of the earlier chunks into the chunk's start value and regenerates the
// chunk's normals to write I.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/blockalif.h"
#include "alif_kernels.h"

using namespace alif;

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10, Box-Muller, OU kernels
// ---------------------------------------------------------------------------
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   // round multipliers
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   // Weyl key increments
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// the four standard normals of steps 4q .. 4q + 3 of neuron n
__device__ __forceinline__ void ou_normals4(uint64_t seed, int q, int n, double z[4]) {
    const u32x4 w = philox4x32_10(u32x4{(uint32_t)q, (uint32_t)n, 0u, 0u}, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    constexpr double INV32 = 1.0 / 4294967296.0, TWO_PI = 6.283185307179586476925;
    const double r0 = sqrt(-2.0 * log(((double)w.x + 1.0) * INV32));
    const double r1 = sqrt(-2.0 * log(((double)w.z + 1.0) * INV32));
    const double a0 = TWO_PI * ((double)w.y * INV32), a1 = TWO_PI * ((double)w.w * INV32);
    z[0] = r0 * cos(a0);
    z[1] = r0 * sin(a0);
    z[2] = r1 * cos(a1);
    z[3] = r1 * sin(a1);
}

constexpr int OU_CHUNK = 256;   // steps per chunk (a multiple of 4)

struct OuArgs {
    int T, N;
    double e, s, sd, mu, eC;    // e = exp(-DT/tau), s = sd sqrt(1 - e^2), eC = e^OU_CHUNK
    uint64_t seed;
    double *ends;               // [NC][N]
    float *I;                   // [T][N]
};

// X over steps [t0, t1) of one chunk, starting from x (the value at t0 - 1)
template <bool WRITE>
__device__ __forceinline__ double ou_chunk(const OuArgs &a, int n, int t0, int t1, double x) {
    for (int t = t0; t < t1; t += 4) {
        double z[4];
        ou_normals4(a.seed, t >> 2, n, z);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (t + j >= t1) break;
            x = (t + j == 0) ? a.sd * z[j] : fma(a.e, x, a.s * z[j]);
            if constexpr (WRITE) a.I[(size_t)(t + j) * a.N + n] = (float)(a.mu + x);
        }
    }
    return x;
}

__global__ void k_ou_chunk_ends(OuArgs a) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int ch = blockIdx.y;
    if (n >= a.N) return;
    const int t0 = ch * OU_CHUNK, t1 = min(a.T, t0 + OU_CHUNK);
    a.ends[(size_t)ch * a.N + n] = ou_chunk<false>(a, n, t0, t1, 0.0);
}

__global__ void k_ou_fill(OuArgs a) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int ch = blockIdx.y;
    if (n >= a.N) return;
    double x = 0.0;   // X at the last step of chunk ch - 1
    for (int c = 0; c < ch; c++) x = fma(a.eC, x, a.ends[(size_t)c * a.N + n]);
    const int t0 = ch * OU_CHUNK, t1 = min(a.T, t0 + OU_CHUNK);
    ou_chunk<true>(a, n, t0, t1, x);
}

size_t ou_chunks(int T) { return ((size_t)T + OU_CHUNK - 1) / OU_CHUNK; }
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

int ou_check(int T, int N, double dt, float tau, float sd) {
    if (T < 0 || N < 0) return set_error(ALIF_EINVAL, "OU current: T and N must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ALIF_EINVAL, "OU current: dt must be > 0");
    if (!(tau > 0.0f) || !std::isfinite(tau) || !(sd >= 0.0f) || !std::isfinite(sd))
        return set_error(ALIF_EINVAL, "OU current: need tau > 0 and sd >= 0");
    if (ou_chunks(T) > 65535) return set_error(ALIF_EUNSUPPORTED, "OU current: T too long");
    return ALIF_OK;
}

hipError_t ou_launch(int T, int N, double dt, float tau, float mean, float sd, uint64_t seed, double *ends,
                     float *I, hipStream_t st) {
    if (T == 0 || N == 0) return hipSuccess;
    OuArgs a{};
    a.T = T;
    a.N = N;
    a.e = std::exp(-dt / (double)tau);
    a.s = (double)sd * std::sqrt(1.0 - a.e * a.e);
    a.sd = sd;
    a.mu = mean;
    a.eC = std::pow(a.e, (double)OU_CHUNK);
    a.seed = seed;
    a.ends = ends;
    a.I = I;
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)ou_chunks(T));
    hipLaunchKernelGGL(k_ou_chunk_ends, grid, dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_ou_fill, grid, dim3(64), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spike-raster compaction: count per chunk -> exclusive scan -> scatter. The
// events come out in ascending flat index (t * N + n), the same on every run.
// ---------------------------------------------------------------------------
constexpr int CMP_THREADS = 256;
constexpr int CMP_BYTES = 32;                                   // raster bytes per thread
constexpr size_t CMP_CHUNK = (size_t)CMP_THREADS * CMP_BYTES;   // raster bytes per workgroup

// spikes among this thread's 32 raster bytes (each byte is 0 or 1)
__device__ __forceinline__ int thread_spikes(const uint8_t *s, size_t n, size_t i0, uint32_t w[8]) {
    if (i0 + CMP_BYTES <= n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(s + i0);   // 32-byte aligned
        const uint4 a = p[0], b = p[1];
        w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
        w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            uint32_t v = 0;
            for (int j = 0; j < 4; j++) {
                const size_t i = i0 + 4 * k + j;
                if (i < n) v |= (uint32_t)(s[i] != 0) << (8 * j);
            }
            w[k] = v;
        }
    }
    int c = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) c += __popc(w[k] & 0x01010101u);
    return c;
}

// exclusive prefix over the workgroup's threads; returns the workgroup total in *total
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < CMP_THREADS / 64; k++) {
        base += k < wv ? lds[k] : 0;
        tot += lds[k];
    }
    *total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(CMP_THREADS) void k_cmp_count(const uint8_t *s, size_t n, uint32_t *counts) {
    __shared__ int lds[CMP_THREADS / 64];
    uint32_t w[8];
    const size_t i0 = (size_t)blockIdx.x * CMP_CHUNK + (size_t)threadIdx.x * CMP_BYTES;
    int tot;
    block_exclusive_scan(thread_spikes(s, n, i0, w), lds, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = (uint32_t)tot;
}

// one workgroup: offsets[g] = sum of counts[0..g), *total = sum of all
__global__ __launch_bounds__(1024) void k_cmp_scan(const uint32_t *counts, uint32_t G, uint32_t *offsets,
                                                   unsigned long long *total) {
    __shared__ int lds[16];
    const uint32_t per = (G + 1023) / 1024;
    const uint32_t g0 = threadIdx.x * per, g1 = min(G, g0 + per);
    uint32_t mine = 0;
    for (uint32_t g = g0; g < g1; g++) mine += counts[g];
    // workgroup scan of the per-thread sums (16 waves)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wv] = (int)x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < 16; k++) {
        base += k < wv ? (uint32_t)lds[k] : 0u;
        tot += (uint32_t)lds[k];
    }
    uint32_t run = base + x - mine;
    for (uint32_t g = g0; g < g1; g++) {
        offsets[g] = run;
        run += counts[g];
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(CMP_THREADS) void k_cmp_scatter(const uint8_t *s, size_t n, const uint32_t *offsets,
                                                             uint32_t *events, uint32_t cap) {
    __shared__ int lds[CMP_THREADS / 64];
    uint32_t w[8];
    const size_t i0 = (size_t)blockIdx.x * CMP_CHUNK + (size_t)threadIdx.x * CMP_BYTES;
    int tot;
    const int c = thread_spikes(s, n, i0, w);
    uint32_t pos = offsets[blockIdx.x] + (uint32_t)block_exclusive_scan(c, lds, &tot);
    if (c == 0) return;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        uint32_t m = w[k] & 0x01010101u;
        while (m) {
            const int bit = __ffs(m) - 1;
            if (pos < cap) events[pos] = (uint32_t)(i0 + 4 * k + (bit >> 3));
            pos++;
            m &= m - 1;
        }
    }
}

// ---------------------------------------------------------------------------
// server state
// ---------------------------------------------------------------------------
double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Layout {   // offsets into a request's one device allocation
    size_t prm, cur, spk, ends, counts, offsets, cnt, total;
    uint32_t chunks;   // compaction workgroups
};
Layout layout(const alif_request &r) {
    Layout l;
    const size_t N = (size_t)r.n_neurons, T = (size_t)r.T;
    size_t o = 0;
    l.prm = o; o += a256(5 * N * sizeof(float));
    l.cur = o; o += a256(T * N * sizeof(float));
    l.spk = o; o += a256(T * N);
    l.ends = o; o += r.input == ALIF_REQ_OU ? a256(ou_chunks((int)T) * N * sizeof(double)) : 0;
    l.chunks = (uint32_t)((T * N + CMP_CHUNK - 1) / CMP_CHUNK);
    l.counts = o; o += a256((size_t)l.chunks * 4);
    l.offsets = o; o += a256((size_t)l.chunks * 4);
    l.cnt = o; o += 256;
    l.total = o;
    return l;
}

struct Req {
    uint64_t ticket = 0;
    alif_request r{};
    uint32_t ev_cap = 0;       // events the scatter may write (<= the caller's capacity)
    std::vector<float> prm;    // tau_mem | tau_adapt | d | theta0 | bias, each [N]
    bool has_bias = false;
    int TR = 0;
    Layout lay{};
    char *dmem = nullptr;
    hipEvent_t ev = nullptr;
    alif_result res{};
};

struct Slot {
    hipStream_t st = nullptr;
    Req *q = nullptr;
    float *h_in = nullptr;   // pinned staging, grown on demand
    uint8_t *h_out = nullptr;
    uint32_t *h_ev = nullptr;   // written by the scatter kernel through its device mapping
    unsigned long long *h_cnt = nullptr;
    size_t cap_in = 0, cap_out = 0, cap_ev = 0;
};

}  // namespace

struct alif_server {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> done;
    std::unordered_set<uint64_t> live;   // queued or running
    std::vector<Slot> slots;
    size_t budget = 0, used = 0;
    int device = 0;
    unsigned *status = nullptr;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
};

namespace {

hipError_t grow_pinned(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    const size_t sz = std::max(need, *cap * 2);
    if (*p) {
        hipError_t e = hipHostFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
        *cap = 0;
    }
    hipError_t e = hipHostMalloc(p, sz, hipHostMallocDefault);
    if (e == hipSuccess) *cap = sz;
    return e;
}

// enqueue one admitted request on its slot's stream
int start_request(alif_server *s, Slot &sl) {
    Req *q = sl.q;
    const alif_request &r = q->r;
    const int N = r.n_neurons, T = r.T;
    const size_t TN = (size_t)T * N;
    hipStream_t st = sl.st;
    hipError_t e = hipSuccess;
    if (r.host_spikes) e = grow_pinned((void **)&sl.h_out, &sl.cap_out, std::max<size_t>(TN, 1));
    if (e == hipSuccess && q->ev_cap > 0)
        e = grow_pinned((void **)&sl.h_ev, &sl.cap_ev, (size_t)q->ev_cap * sizeof(uint32_t));
    if (e == hipSuccess && r.input == ALIF_REQ_HOST_CURRENT)
        e = grow_pinned((void **)&sl.h_in, &sl.cap_in, std::max<size_t>(TN * sizeof(float), 1));
    if (e != hipSuccess) return set_error(ALIF_ENOMEM, "pinned staging allocation failed");
    uint32_t *ev_dev = nullptr;   // the events staging as the device sees it
    if (q->ev_cap > 0 && hipHostGetDevicePointer((void **)&ev_dev, sl.h_ev, 0) != hipSuccess)
        return set_error(ALIF_EHIP, "no device mapping of the pinned event staging");
    e = hipMallocAsync((void **)&q->dmem, q->lay.total, st);
    if (e != hipSuccess) {
        q->dmem = nullptr;
        return set_error(ALIF_ENOMEM, "device allocation for a request failed");
    }
    float *prm = (float *)(q->dmem + q->lay.prm);
    float *cur = (float *)(q->dmem + q->lay.cur);
    uint8_t *spk = (uint8_t *)(q->dmem + q->lay.spk);
    unsigned long long *cnt = (unsigned long long *)(q->dmem + q->lay.cnt);
    // the parameters stay in the request (host memory that is not touched until
    // the request is done); the copy is small
    e = hipMemcpyAsync(prm, q->prm.data(), q->prm.size() * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess && TN > 0) {
        if (r.input == ALIF_REQ_HOST_CURRENT) {
            std::memcpy(sl.h_in, r.host_current, TN * sizeof(float));
            e = hipMemcpyAsync(cur, sl.h_in, TN * sizeof(float), hipMemcpyHostToDevice, st);
        } else {
            e = ou_launch(T, N, r.dt_ms, r.ou_tau_ms, r.ou_mean, r.ou_sd, r.seed,
                          (double *)(q->dmem + q->lay.ends), cur, st);
        }
        if (e == hipSuccess) {
            FwdArgs a{};
            a.B = 1; a.T = T; a.N = N; a.TR = q->TR; a.NB = (T + q->TR - 1) / q->TR;
            const int nwg = block_neurons_per_wg(block_config(q->TR).seg);
            a.n_groups = (N + nwg - 1) / nwg;
            a.dt = r.dt_ms;
            a.I = cur;
            a.bias_k = q->has_bias ? prm + 4 * (size_t)N : nullptr;
            a.tau_m = prm; a.tau_a = prm + N; a.d = prm + 2 * (size_t)N; a.theta0 = prm + 3 * (size_t)N;
            a.spikes = spk;
            a.spike_dtype = 0;
            a.status = s->status;
            e = launch_blocks_fwd(a, st);
        }
        if (e == hipSuccess) {
            uint32_t *counts = (uint32_t *)(q->dmem + q->lay.counts);
            uint32_t *offsets = (uint32_t *)(q->dmem + q->lay.offsets);
            const unsigned G = q->lay.chunks;
            hipLaunchKernelGGL(k_cmp_count, dim3(G), dim3(CMP_THREADS), 0, st, spk, TN, counts);
            hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(1024), 0, st, counts, G, offsets, cnt);
            if (q->ev_cap > 0)
                hipLaunchKernelGGL(k_cmp_scatter, dim3(G), dim3(CMP_THREADS), 0, st, spk, TN, offsets, ev_dev,
                                   q->ev_cap);
            e = hipGetLastError();
        }
        if (e == hipSuccess && r.host_spikes) e = hipMemcpyAsync(sl.h_out, spk, TN, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(sl.h_cnt, cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    const hipError_t ef = hipFreeAsync(q->dmem, st);
    q->dmem = nullptr;
    if (e == hipSuccess) e = ef;
    if (e == hipSuccess) e = hipEventRecord(q->ev, st);
    return e == hipSuccess ? ALIF_OK : set_error(ALIF_EHIP, hipGetErrorString(e));
}

// called by the scheduler once the request's work has finished (or failed)
void finish(alif_server *s, Slot &sl, int status) {
    Req *q = sl.q;
    if (status == ALIF_OK) {
        const size_t TN = (size_t)q->r.T * q->r.n_neurons;
        if (q->r.host_spikes && TN) std::memcpy(q->r.host_spikes, sl.h_out, TN);
        q->res.n_spikes = TN ? (int64_t)*sl.h_cnt : 0;
        if (q->ev_cap > 0) {
            const size_t k = std::min<size_t>((size_t)q->res.n_spikes, q->ev_cap);
            std::memcpy(q->r.host_events, sl.h_ev, k * sizeof(uint32_t));
        }
        q->res.events_truncated = q->r.host_events && q->res.n_spikes > q->r.events_capacity;
    }
    q->res.status = status;
    q->res.t_done_s = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= q->lay.total;
    sl.q = nullptr;
    s->live.erase(q->ticket);
    s->done[q->ticket] = q;
}

void scheduler(alif_server *s) {
    hipSetDevice(s->device);
    std::vector<int> started;
    for (;;) {
        started.clear();
        bool busy = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // admission: arrival order, a free slot and room in the budget
            while (!s->queue.empty()) {
                Req *q = s->queue.front();
                if (s->used + q->lay.total > s->budget) break;
                int k = -1;
                for (size_t i = 0; i < s->slots.size(); i++)
                    if (!s->slots[i].q) { k = (int)i; break; }
                if (k < 0) break;
                s->queue.pop_front();
                s->slots[k].q = q;
                s->used += q->lay.total;
                q->res.t_admit_s = now_s();
                started.push_back(k);
            }
            for (const Slot &sl : s->slots) busy |= sl.q != nullptr;
            if (!busy) {
                if (s->stop && s->queue.empty()) break;
                s->cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        for (int k : started) {
            Slot &sl = s->slots[k];
            const int rc = start_request(s, sl);
            if (rc != ALIF_OK) {
                hipStreamSynchronize(sl.st);
                finish(s, sl, rc);
            }
        }
        // completions (a slot's request is only replaced by this thread)
        bool progressed = !started.empty();
        for (Slot &sl : s->slots) {
            if (!sl.q) continue;
            const hipError_t e = hipEventQuery(sl.q->ev);
            if (e == hipErrorNotReady) continue;
            finish(s, sl, e == hipSuccess ? ALIF_OK : set_error(ALIF_EHIP, hipGetErrorString(e)));
            progressed = true;
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

int validate(const alif_request *r, int *TR) {
    if (!r) return set_error(ALIF_EINVAL, "request is NULL");
    if (r->n_neurons <= 0 || r->T < 0) return set_error(ALIF_EINVAL, "request needs n_neurons > 0 and T >= 0");
    const int tr = alif_refractory_steps(r->dt_ms, r->arp_ms);
    if (tr < 0) return tr;
    *TR = tr;
    if (!r->tau_mem_ms || !r->tau_adapt_ms || !r->d || !r->theta0)
        return set_error(ALIF_EINVAL, "request: parameter arrays are required");
    if (r->input != ALIF_REQ_HOST_CURRENT && r->input != ALIF_REQ_OU)
        return set_error(ALIF_EINVAL, "request: unknown input kind");
    if (r->events_capacity < 0) return set_error(ALIF_EINVAL, "request: events_capacity < 0");
    if (r->input == ALIF_REQ_HOST_CURRENT && !r->host_current && r->T > 0)
        return set_error(ALIF_EINVAL, "request: host_current is NULL");
    if (r->input == ALIF_REQ_OU) {
        const int rc = ou_check(r->T, r->n_neurons, r->dt_ms, r->ou_tau_ms, r->ou_sd);
        if (rc) return rc;
    }
    // the forward addresses one request's [T][N] float rows with 32-bit offsets
    if ((size_t)r->T * (size_t)r->n_neurons * 4 >= ((size_t)1 << 31))
        return set_error(ALIF_EUNSUPPORTED, "request: T * n_neurons too large");
    for (int i = 0; i < r->n_neurons; i++)
        if (!(r->tau_mem_ms[i] > 0) || !(r->tau_adapt_ms[i] > 0) || !(r->d[i] >= 0) || !(r->theta0[i] > 0) ||
            !std::isfinite(r->tau_mem_ms[i]) || !std::isfinite(r->tau_adapt_ms[i]) || !std::isfinite(r->d[i]) ||
            !std::isfinite(r->theta0[i]) || (r->bias && !std::isfinite(r->bias[i])))
            return set_error(ALIF_EINVAL, "request: need finite tau_mem, tau_adapt, theta0 > 0, d >= 0, bias");
    return ALIF_OK;
}

void destroy_slots(alif_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.st) {
            hipStreamSynchronize(sl.st);
            hipStreamDestroy(sl.st);
        }
        if (sl.h_in) hipHostFree(sl.h_in);
        if (sl.h_out) hipHostFree(sl.h_out);
        if (sl.h_ev) hipHostFree(sl.h_ev);
        if (sl.h_cnt) hipHostFree(sl.h_cnt);
    }
    s->slots.clear();
}

struct DeviceGuard {   // makes `dev` current and restores the caller's device
    int prev = 0;
    explicit DeviceGuard(int dev) {
        hipGetDevice(&prev);
        hipSetDevice(dev);
    }
    ~DeviceGuard() { hipSetDevice(prev); }
};

}  // namespace

extern "C" {

int alif_ou_workspace_bytes(int32_t T, int32_t n_neurons, size_t *bytes) {
    if (!bytes || T < 0 || n_neurons < 0) return set_error(ALIF_EINVAL, "bad arguments");
    *bytes = a256(ou_chunks(T) * (size_t)n_neurons * sizeof(double));
    return ALIF_OK;
}

int alif_ou_current(int32_t T, int32_t n_neurons, double dt_ms, float tau_ms, float mean, float sd,
                    uint64_t seed, float *current, void *workspace, size_t workspace_bytes, void *stream) {
    const int rc = ou_check(T, n_neurons, dt_ms, tau_ms, sd);
    if (rc) return rc;
    if ((size_t)T * n_neurons == 0) return ALIF_OK;
    size_t need = 0;
    alif_ou_workspace_bytes(T, n_neurons, &need);
    if (!current || !workspace) return set_error(ALIF_EINVAL, "current and workspace are required");
    if (workspace_bytes < need) return set_error(ALIF_EINVAL, "workspace too small");
    const hipError_t e = ou_launch(T, n_neurons, dt_ms, tau_ms, mean, sd, seed, (double *)workspace, current,
                                   (hipStream_t)stream);
    return e == hipSuccess ? ALIF_OK : set_error(ALIF_EHIP, hipGetErrorString(e));
}

int alif_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t device, alif_server **out) {
    if (!out || max_slots <= 0 || max_slots > 64 || hbm_budget_bytes == 0)
        return set_error(ALIF_EINVAL, "server: need out, 1 <= max_slots <= 64 and a nonzero budget");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_error(ALIF_EINVAL, "server: bad device ordinal");
    alif_server *s = new (std::nothrow) alif_server();
    if (!s) return set_error(ALIF_ENOMEM, "server: out of host memory");
    s->budget = hbm_budget_bytes;
    s->device = device;
    s->slots.resize(max_slots);
    hipError_t e;
    {
        DeviceGuard g(device);
        e = hipMalloc(&s->status, 256);
        if (e == hipSuccess) e = hipMemset(s->status, 0, 256);
        for (Slot &sl : s->slots) {
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipHostMalloc((void **)&sl.h_cnt, sizeof(unsigned long long), hipHostMallocDefault);
        }
        if (e != hipSuccess) {
            destroy_slots(s);
            if (s->status) hipFree(s->status);
        }
    }
    if (e != hipSuccess) {
        delete s;
        return set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        DeviceGuard g(device);
        destroy_slots(s);
        hipFree(s->status);
        delete s;
        return set_error(ALIF_ENOMEM, "server: cannot start the scheduler thread");
    }
    *out = s;
    return ALIF_OK;
}

int alif_request_footprint(const alif_request *req, size_t *bytes) {
    int TR = 0;
    const int rc = validate(req, &TR);
    if (rc) return rc;
    if (!bytes) return set_error(ALIF_EINVAL, "bytes is NULL");
    *bytes = layout(*req).total;
    return ALIF_OK;
}

int alif_submit(alif_server *s, const alif_request *req, uint64_t *ticket) {
    if (!s || !ticket) return set_error(ALIF_EINVAL, "server and ticket are required");
    int TR = 0;
    const int rc = validate(req, &TR);
    if (rc) return rc;
    Req *q = new (std::nothrow) Req();
    if (!q) return set_error(ALIF_ENOMEM, "out of host memory");
    q->r = *req;
    q->TR = TR;
    q->lay = layout(*req);
    if (req->host_events && req->events_capacity > 0) {
        // at most one spike per neuron in each T_R-step block
        const size_t bound = (size_t)((req->T + TR - 1) / TR) * (size_t)req->n_neurons;
        q->ev_cap = (uint32_t)std::min<size_t>((size_t)req->events_capacity, bound);
    }
    if (q->lay.total > s->budget) {
        delete q;
        return set_error(ALIF_EBUDGET, "request footprint exceeds the server's HBM budget");
    }
    const size_t N = (size_t)req->n_neurons;
    q->has_bias = req->bias != nullptr;
    try {
        q->prm.assign(5 * N, 0.0f);
    } catch (...) {
        delete q;
        return set_error(ALIF_ENOMEM, "out of host memory");
    }
    std::memcpy(q->prm.data(), req->tau_mem_ms, N * sizeof(float));
    std::memcpy(q->prm.data() + N, req->tau_adapt_ms, N * sizeof(float));
    std::memcpy(q->prm.data() + 2 * N, req->d, N * sizeof(float));
    std::memcpy(q->prm.data() + 3 * N, req->theta0, N * sizeof(float));
    if (q->has_bias) std::memcpy(q->prm.data() + 4 * N, req->bias, N * sizeof(float));
    hipError_t e;
    {
        DeviceGuard g(s->device);
        e = hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        delete q;
        return set_error(ALIF_EHIP, hipGetErrorString(e));
    }
    q->res.t_submit_s = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        hipEventDestroy(q->ev);
        delete q;
        return set_error(ALIF_ESHUTDOWN, "server is shutting down");
    }
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->live.insert(q->ticket);
    s->queue.push_back(q);
    s->cv.notify_all();
    return ALIF_OK;
}

int alif_poll(alif_server *s, uint64_t ticket, alif_result *res) {
    if (!s || !res) return set_error(ALIF_EINVAL, "server and result are required");
    Req *q = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->done.find(ticket);
        if (it == s->done.end()) {
            if (s->live.count(ticket)) return ALIF_PENDING;
            return set_error(ALIF_ENOTFOUND, "unknown ticket (never issued or already collected)");
        }
        q = it->second;
        s->done.erase(it);
    }
    *res = q->res;
    hipEventDestroy(q->ev);
    delete q;
    return ALIF_OK;
}

int alif_server_destroy(alif_server *s) {
    if (!s) return ALIF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    {
        DeviceGuard g(s->device);
        destroy_slots(s);
        for (auto &kv : s->done) {
            hipEventDestroy(kv.second->ev);
            delete kv.second;
        }
        hipFree(s->status);
    }
    delete s;
    return ALIF_OK;
}

}  // extern "C"
