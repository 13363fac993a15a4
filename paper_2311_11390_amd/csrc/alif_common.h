// Device-side helpers shared by the libblockalif kernels (gfx950 / CDNA4).
//
//  * Raw buffer descriptors: every large-array access goes through a buffer
//    resource whose range check turns an out-of-range load into 0 and drops an
//    out-of-range store, so padding steps and ragged neuron tails need no
//    branches and can never touch memory outside the tensor.
//  * XCD-aware work mapping.
//  * The surrogate derivatives of the backward.
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

// The same three surrogates in FP64 (the attached sequential backward, whose
// coupled recurrence amplifies input rounding).
template <int SG>
__device__ __forceinline__ double surrogate_grad_f64(double u, double k) {
    if constexpr (SG == 1) {
        return fabs(u) <= 0.5 ? 0.5 : 0.0;
    } else if constexpr (SG == 2) {
        const double rs2pi = 0.3989422804014327;   // 1 / sqrt(2 pi)
        const double um = u - 3.0, up = u + 3.0;
        return 1.15 * rs2pi / 0.5 * exp(-2.0 * u * u) -
               0.15 * rs2pi / 3.0 * (exp(um * um * (-1.0 / 18.0)) + exp(up * up * (-1.0 / 18.0)));
    } else {
        const double q = k * fabs(u) + 1.0;
        return 1.0 / (q * q);
    }
}

// parameter sanity for the block method (positive threshold during refractory)
__device__ __forceinline__ bool params_ok(float tm, float ta, float d, float th0) {
    return tm > 0.f && ta > 0.f && d >= 0.f && th0 > 0.f && isfinite(tm) && isfinite(ta) &&
           isfinite(d) && isfinite(th0);
}

}  // namespace alif
