// Device-side helpers shared by the libblockalif kernels (gfx950 / CDNA4).
//
//  * Raw buffer descriptors: every large-array access goes through a buffer
//    resource whose range check turns an out-of-range load into 0 and drops an
//    out-of-range store, so padding steps and ragged neuron tails need no
//    branches and can never touch memory outside the tensor.
//  * DPP lane-group collectives on groups of SEG consecutive lanes
//    (SEG in {1, 2, 4, 8, 16}, aligned inside one 16-lane DPP row): all-reduce,
//    affine prefix scan (forward in time) and affine suffix scan (backward in
//    time). They replace shared-memory round trips for the per-block
//    combination of time segments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alif {

// ---------------------------------------------------------------------------
// raw buffer access
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Third descriptor dword for gfx9-family raw (untyped, stride 0) buffers.
#define ALIF_BUFFER_DWORD3 0x00020000

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             ALIF_BUFFER_DWORD3);
}

// Wait until every vector-memory operation this wave has issued is done
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt fields left at "no wait"). Issued once
// in front of a software-pipelined loop: with the loads and stores of the
// set-up code retired, the compiler's wait analysis at the loop head only sees
// the loop's own prefetches and no longer drains the queue every iteration.
__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Offset used for "no access": beyond any num_records we create (< 2^31).
#define ALIF_OOB 0x80000000u

// The b32 buffer builtins move 32-bit integers: floats cross them as bit patterns.
__device__ __forceinline__ float ld_f32(rsrc_t r, uint32_t byte_off) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ void st_f32(rsrc_t r, uint32_t byte_off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, 0);
}
__device__ __forceinline__ void st_u8(rsrc_t r, uint32_t byte_off, uint8_t v) {
    __builtin_amdgcn_raw_buffer_store_b8(v, r, byte_off, 0, 0);
}
__device__ __forceinline__ void st_u16(rsrc_t r, uint32_t byte_off, uint16_t v) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, byte_off, 0, 0);
}
__device__ __forceinline__ uint8_t ld_u8(rsrc_t r, uint32_t byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, byte_off, 0, 0);
}

// spike outputs: 0 = uint8, 1 = bfloat16 (0x3F80 = 1.0), 2 = float; byte offset
__device__ __forceinline__ void st_spike(rsrc_t r, int dtype, uint32_t byte_off, bool s) {
    if (dtype == 0) st_u8(r, byte_off, s ? 1 : 0);
    else if (dtype == 1) st_u16(r, byte_off, s ? (uint16_t)0x3F80 : (uint16_t)0);
    else st_f32(r, byte_off, s ? 1.0f : 0.0f);
}
__device__ __forceinline__ int spike_bytes(int dtype) { return dtype == 0 ? 1 : (dtype == 1 ? 2 : 4); }

// ---------------------------------------------------------------------------
// DPP (GFX9 encoding) on 32-bit values
// ---------------------------------------------------------------------------
#define DPP_QUAD(a, b, c, d) ((a) | ((b) << 2) | ((c) << 4) | ((d) << 6))
#define DPP_ROW_SHL(n) (0x100 + (n))
#define DPP_ROW_SHR(n) (0x110 + (n))
#define DPP_ROW_MIRROR 0x140
#define DPP_ROW_HALF_MIRROR 0x141

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    int2 p = *reinterpret_cast<int2 *>(&v);
    int2 q;
    q.x = dpp_i<CTRL>(p.x);
    q.y = dpp_i<CTRL>(p.y);
    return *reinterpret_cast<double *>(&q);
}

// Shift by OFF lanes within the 16-lane row: lane reads lane - OFF (up) or + OFF (down).
template <int OFF> __device__ __forceinline__ float shr_f(float v) { return dpp_f<DPP_ROW_SHR(OFF)>(v); }
template <int OFF> __device__ __forceinline__ float shl_f(float v) { return dpp_f<DPP_ROW_SHL(OFF)>(v); }

// Butterfly partner for the all-reduce round R (0: xor 1, 1: xor 2, 2: half-row
// mirror, 3: row mirror). After rounds 0..log2(SEG)-1 every lane of an aligned
// group of SEG lanes holds the reduction of the group.
template <int R, typename V> __device__ __forceinline__ V bfly(V v);
template <> __device__ __forceinline__ float bfly<0, float>(float v) { return dpp_f<DPP_QUAD(1, 0, 3, 2)>(v); }
template <> __device__ __forceinline__ float bfly<1, float>(float v) { return dpp_f<DPP_QUAD(2, 3, 0, 1)>(v); }
template <> __device__ __forceinline__ float bfly<2, float>(float v) { return dpp_f<DPP_ROW_HALF_MIRROR>(v); }
template <> __device__ __forceinline__ float bfly<3, float>(float v) { return dpp_f<DPP_ROW_MIRROR>(v); }
template <> __device__ __forceinline__ int bfly<0, int>(int v) { return dpp_i<DPP_QUAD(1, 0, 3, 2)>(v); }
template <> __device__ __forceinline__ int bfly<1, int>(int v) { return dpp_i<DPP_QUAD(2, 3, 0, 1)>(v); }
template <> __device__ __forceinline__ int bfly<2, int>(int v) { return dpp_i<DPP_ROW_HALF_MIRROR>(v); }
template <> __device__ __forceinline__ int bfly<3, int>(int v) { return dpp_i<DPP_ROW_MIRROR>(v); }
template <> __device__ __forceinline__ double bfly<0, double>(double v) { return dpp_d<DPP_QUAD(1, 0, 3, 2)>(v); }
template <> __device__ __forceinline__ double bfly<1, double>(double v) { return dpp_d<DPP_QUAD(2, 3, 0, 1)>(v); }
template <> __device__ __forceinline__ double bfly<2, double>(double v) { return dpp_d<DPP_ROW_HALF_MIRROR>(v); }
template <> __device__ __forceinline__ double bfly<3, double>(double v) { return dpp_d<DPP_ROW_MIRROR>(v); }

template <int SEG, typename V>
__device__ __forceinline__ V group_sum(V v) {
    if constexpr (SEG >= 2) v = v + bfly<0>(v);
    if constexpr (SEG >= 4) v = v + bfly<1>(v);
    if constexpr (SEG >= 8) v = v + bfly<2>(v);
    if constexpr (SEG >= 16) v = v + bfly<3>(v);
    return v;
}
template <int SEG>
__device__ __forceinline__ int group_min(int v) {
    if constexpr (SEG >= 2) v = min(v, bfly<0>(v));
    if constexpr (SEG >= 4) v = min(v, bfly<1>(v));
    if constexpr (SEG >= 8) v = min(v, bfly<2>(v));
    if constexpr (SEG >= 16) v = min(v, bfly<3>(v));
    return v;
}

// Value held by lane `src` of the group, broadcast to the whole group (exact:
// every other lane contributes +0).
template <int SEG, typename V>
__device__ __forceinline__ V group_bcast(V v, int s, int src) {
    return group_sum<SEG>(s == src ? v : V(0));
}

// Inclusive affine prefix scan over the group, s = position in the group:
//   P_s = X_s + D_s[r] * P_{s - 2^r} applied for rounds r = 0.. log2(SEG)-1,
// where D_s[r] is the decay across the 2^r segments ending at s.
template <int SEG>
__device__ __forceinline__ float group_prefix(float x, int s, const float *D) {
    if constexpr (SEG >= 2) { float y = shr_f<1>(x); if (s >= 1) x = fmaf(D[0], y, x); }
    if constexpr (SEG >= 4) { float y = shr_f<2>(x); if (s >= 2) x = fmaf(D[1], y, x); }
    if constexpr (SEG >= 8) { float y = shr_f<4>(x); if (s >= 4) x = fmaf(D[2], y, x); }
    if constexpr (SEG >= 16) { float y = shr_f<8>(x); if (s >= 8) x = fmaf(D[3], y, x); }
    return x;
}

// Inclusive affine suffix scan over the group of maps lam -> R + M lam composed
// from segment s to the group's last segment.
template <int SEG>
__device__ __forceinline__ void group_suffix(float &M, float &R, int s) {
    if constexpr (SEG >= 2) { float m = shl_f<1>(M), r = shl_f<1>(R); if (s + 1 < SEG) { R = fmaf(M, r, R); M = M * m; } }
    if constexpr (SEG >= 4) { float m = shl_f<2>(M), r = shl_f<2>(R); if (s + 2 < SEG) { R = fmaf(M, r, R); M = M * m; } }
    if constexpr (SEG >= 8) { float m = shl_f<4>(M), r = shl_f<4>(R); if (s + 4 < SEG) { R = fmaf(M, r, R); M = M * m; } }
    if constexpr (SEG >= 16) { float m = shl_f<8>(M), r = shl_f<8>(R); if (s + 8 < SEG) { R = fmaf(M, r, R); M = M * m; } }
}

// value from the next lane in the group (s + 1), or `edge` for the last lane
template <int SEG>
__device__ __forceinline__ float from_next(float v, int s, float edge) {
    if constexpr (SEG == 1) return edge;
    else { float y = shl_f<1>(v); return (s + 1 < SEG) ? y : edge; }
}
// value from the previous lane in the group (s - 1), or `edge` for the first lane
template <int SEG>
__device__ __forceinline__ float from_prev(float v, int s, float edge) {
    if constexpr (SEG == 1) return edge;
    else { float y = shr_f<1>(v); return (s >= 1) ? y : edge; }
}

// ---------------------------------------------------------------------------
// work mapping: consecutive work items on the same XCD (round-robin dispatch
// sends workgroup i to XCD i % 8), so neighbouring neuron groups share an L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int wg, int total) {
    const int X = 8;
    int q = total / X, r = total % X;
    int xcd = wg % X, idx = wg / X;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Fast-sigmoid surrogate derivative (k|u| + 1)^-2 (Supplementary, "Surrogate
// gradient"). The reciprocal is the hardware one (v_rcp_f32, within 1 ulp)
// rather than an IEEE division, which compiles to about ten instructions: the
// value only scales gradients, whose tolerance is far above 1 ulp.
__device__ __forceinline__ float fast_sigmoid_grad(float u, float k) {
    const float r = __builtin_amdgcn_rcpf(fmaf(k, fabsf(u), 1.0f));
    return r * r;
}

// The surrogate derivatives dS/du at u = V - th (Supplementary, "Surrogate
// gradient"), selected at compile time:
//   SG 0  fast sigmoid    (k|u| + 1)^-2
//   SG 1  boxcar          0.5 where |u| <= 0.5, else 0
//   SG 2  multi-Gaussian  1.15 N(u | 0, 0.5^2) - 0.15 N(u | 3, 3^2) - 0.15 N(u | -3, 3^2),
//                         with the constants as the supplementary prints them
// The exponentials are the hardware ones (v_exp_f32, a few ulp): the values only
// scale gradients.
template <int SG>
__device__ __forceinline__ float surrogate_grad(float u, float k) {
    if constexpr (SG == 1) {
        return fabsf(u) <= 0.5f ? 0.5f : 0.0f;
    } else if constexpr (SG == 2) {
        constexpr float rs2pi = 0.3989422804014327f;            // 1 / sqrt(2 pi)
        constexpr float c0 = 1.15f * rs2pi / 0.5f, c1 = 0.15f * rs2pi / 3.0f;
        const float um = u - 3.0f, up = u + 3.0f;
        return c0 * __expf(-2.0f * u * u) - c1 * (__expf(um * um * (-1.0f / 18.0f)) +
                                                   __expf(up * up * (-1.0f / 18.0f)));
    } else {
        return fast_sigmoid_grad(u, k);
    }
}

// parameter sanity for the block method (positive threshold during refractory)
__device__ __forceinline__ bool params_ok(float tm, float ta, float d, float th0) {
    return tm > 0.f && ta > 0.f && d >= 0.f && th0 > 0.f && isfinite(tm) && isfinite(ta) &&
           isfinite(d) && isfinite(th0);
}

}  // namespace alif
