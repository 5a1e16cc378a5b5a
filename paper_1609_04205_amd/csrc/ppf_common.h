// Device helpers shared by the channelisers: complex float2 arithmetic,
// 4- and 16-point DFTs, quad broadcasts, the int8 requantiser and the
// sample store into the channelised layout.
#pragma once

#include <hip/hip_fp16.h>

#include "afc_internal.h"

namespace afc {
namespace ppfk {

struct Tw64 {
    float2 w[64];                            // exp(-2 pi i m / 64), rounded from double on the host
};

__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 operator*(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 4-point DFT in place, natural order: X_k = sum_n x_n (-i)^{nk}.
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3, t3 = x1 - x3;
    x0 = t0 + t2;
    x2 = t0 - t2;
    x1 = make_float2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
    x3 = make_float2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
}

// 16-point DFT, Y[k] = sum_n a[n] exp(-2 pi i n k / 16), as 4 x 4 with
// n = al + 4 be, k = ga + 4 de.  On return Y[ga + 4 de] is in a[4 ga + de].
__device__ __forceinline__ void dft16(float2 (&a)[16]) {
    constexpr float c8 = 0.92387953251128675613f;   // cos(pi/8)
    constexpr float s8 = 0.38268343236508977173f;   // sin(pi/8)
    constexpr float r2 = 0.70710678118654752440f;   // sqrt(1/2)
#pragma unroll
    for (int al = 0; al < 4; ++al) dft4(a[al], a[al + 4], a[al + 8], a[al + 12]);
    // twiddles exp(-2 pi i al ga / 16) on a[al + 4 ga]
    a[1 + 4] = cmul(a[1 + 4], make_float2(c8, -s8));    // 1
    a[1 + 8] = cmul(a[1 + 8], make_float2(r2, -r2));    // 2
    a[1 + 12] = cmul(a[1 + 12], make_float2(s8, -c8));  // 3
    a[2 + 4] = cmul(a[2 + 4], make_float2(r2, -r2));    // 2
    a[2 + 8] = make_float2(a[2 + 8].y, -a[2 + 8].x);    // 4: -i
    a[2 + 12] = cmul(a[2 + 12], make_float2(-r2, -r2)); // 6
    a[3 + 4] = cmul(a[3 + 4], make_float2(s8, -c8));    // 3
    a[3 + 8] = cmul(a[3 + 8], make_float2(-r2, -r2));   // 6
    a[3 + 12] = cmul(a[3 + 12], make_float2(-c8, s8));  // 9
#pragma unroll
    for (int ga = 0; ga < 4; ++ga) dft4(a[4 * ga], a[4 * ga + 1], a[4 * ga + 2], a[4 * ga + 3]);
}

// value of the lane at (this lane xor M) inside the quad, M = 1 or 2
// (DPP quad_perm [1,0,3,2] or [2,3,0,1])
template <int M>
__device__ __forceinline__ float quad_xor(float v) {
    constexpr int ctrl = M == 1 ? (1 | (0 << 2) | (3 << 4) | (2 << 6)) : (2 | (3 << 2) | (0 << 4) | (1 << 6));
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
}

// clamp(rint(y * gain), -127, 127) of the exact product (one rounding, ties
// to even) as a two's-complement byte in the low 8 bits.  One fused
// multiply-add y * gain + 1.5 * 2^23 rounds the exact product to an integer
// (the result's unit in the last place is 1 while |y * gain| < 2^22; beyond
// that it is far outside the clamp) and leaves it in the low mantissa bits;
// the clamp then acts on the offset value.
__device__ __forceinline__ unsigned requant_bits(float y, float gain) {
    constexpr float kMagic = 12582912.0f;                      // 1.5 * 2^23
    const float v = __builtin_fmaf(y, gain, kMagic);
    return __float_as_uint(__builtin_amdgcn_fmed3f(v, kMagic - 127.0f, kMagic + 127.0f));
}

// store at sample index base + off (base wave-uniform, off per lane) with a
// buffer store, so the store needs no vector address arithmetic.  kOne: the
// subband's whole output is below 2^31 bytes (checked by the launch), so one
// buffer descriptor at the subband's output serves every channel, with the
// channel's byte offset as the scalar offset (16 descriptors per lane job
// otherwise cost SGPRs the kernels then spill).  Otherwise one descriptor
// per channel (a channel of samples is far below 2 GiB: one subband of input
// is bounded to 2^31 values).
template <int DT, bool kOne>
__device__ __forceinline__ void store_sample(void* zs, int64_t base, unsigned off, float2 y, float gain) {
    constexpr unsigned kB = DT == AFC_F32 ? 8 : DT == AFC_F16 ? 4 : 2;
#if defined(__HIP_DEVICE_COMPILE__)
    // raw buffer store; non-temporal (cache policy bit 1: the samples are
    // written once and not read again by this kernel)
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<char*>(zs) + (kOne ? 0 : base * kB), (short)0, 0x7FFFFFFF, 0x00020000);
    const unsigned soff = kOne ? (unsigned)(base * kB) : 0u;
    if constexpr (DT == AFC_F32) {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, y), r, off * kB, soff, 2);
    } else if constexpr (DT == AFC_F16) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, __floats2half2_rn(y.x, y.y)), r,
                                                  off * kB, soff, 2);
    } else {
        const unsigned qr = requant_bits(y.x, gain), qi = requant_bits(y.y, gain);
        // bytes: low = real, high = imaginary
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)__builtin_amdgcn_perm(qi, qr, 0x0c0c0400u), r,
                                                  off * kB, soff, 2);
    }
#endif
}

inline Tw64 make_twiddles() {
    Tw64 t;
    for (int m = 0; m < 64; ++m) {
        const double ang = -2.0 * 3.14159265358979323846 * m / 64.0;
        t.w[m] = make_float2((float)cos(ang), (float)sin(ang));
    }
    return t;
}

}  // namespace ppfk
}  // namespace afc
