// flb_device.h -- device-side building blocks of the gfx950 kernels:
// the Philox4x32-10 noise stream, the normals derived from it, and the
// population storage codecs.
#pragma once

#include "flb_internal.h"

namespace flbdev {

// a ^ b ^ c in one instruction: gfx950's three-input bit operation with the
// truth table of a three-way xor (bit abc of 0x96 is a ^ b ^ c)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11).  The key
// is wave-uniform, so its schedule lives in scalar registers; each round is
// two 32x32->64 multiplies and two three-way xors (one instruction each).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Six unit normals from one draw (the layout documented in flb.h).  The
// uniforms are exact in FP32: (2k+1) 2^-24 with k < 2^23 and (2a+1) 2^-20
// with a < 2^19.  The angle is passed to the hardware sine/cosine in
// revolutions, so 2 pi a needs no range reduction.
__device__ __forceinline__ void normals6(uint4 w, float z[6])
{
#pragma clang fp contract(off)  // the same bits in every kernel that inlines this
    const uint32_t wv[3] = {w.x, w.y, w.z};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        // r = (2 (w >> 9) + 1) 2^-24: 1 + (w >> 9) 2^-23 built from its bits,
        // less 1 - 2^-24 (exact: the operands are within a factor 2)
        const float r = __uint_as_float(0x3F800000u | (wv[p] >> 9)) - 0x1.fffffep-1f;
        const uint32_t al = ((wv[p] & 0x1FFu) << 10) | ((w.w >> (10 * p)) & 0x3FFu);
        const float a = fmaf((float)al, 0x1p-19f, 0x1p-20f);
        // r >= 2^-24 is never denormal: the hardware log2 needs no range
        // handling; -2 ln r = -2 ln(2) log2 r
        const float R = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(r));
        z[2 * p] = R * __builtin_amdgcn_cosf(a);
        z[2 * p + 1] = R * __builtin_amdgcn_sinf(a);
    }
}

// ---------------------------------------------------------------------
// Storage codecs.  FP32 keeps the deviation d = f - w rho0 itself; the
// 16-bit formats keep q = (d - feq) / scale, rounded to nearest even.
// ---------------------------------------------------------------------
template <int S> struct Codec;

template <> struct Codec<kF32> {
    using T = float;
    static __device__ __forceinline__ float decode(T v, const LatticeParams &, int) { return v; }
    static __device__ __forceinline__ T encode(float d, const LatticeParams &, int) { return d; }
};

// The FP32 value of an encode, materialised before its conversion to 16
// bits: otherwise the compiler merges the FMA and the conversion into one
// mixed-precision instruction in most contexts but not all (it rounds once,
// the separate pair twice), and results would depend on the launch shape.
// The empty statement is opaque to instruction selection but, having no side
// effects, leaves the scheduler free.
__device__ __forceinline__ float round_point(float q)
{
    asm("" : "+v"(q));
    return q;
}

// bfloat16 through the native type: gfx950 converts with one
// round-to-nearest-even instruction (v_cvt_pk_bf16_f32).
template <> struct Codec<kBF16> {
    using T = __bf16;
    static __device__ __forceinline__ float decode(T v, const LatticeParams &P, int i)
    {
        return fmaf((float)v, P.scale[i], P.feq[i]);
    }
    static __device__ __forceinline__ T encode(float d, const LatticeParams &P, int i)
    {
        return (T)round_point(fmaf(d, P.inv_scale[i], -P.feq_scaled[i]));
    }
};

template <> struct Codec<kF16> {
    using T = _Float16;
    static __device__ __forceinline__ float decode(T v, const LatticeParams &P, int i)
    {
        return fmaf((float)v, P.scale[i], P.feq[i]);
    }
    static __device__ __forceinline__ T encode(float d, const LatticeParams &P, int i)
    {
        return (T)round_point(fmaf(d, P.inv_scale[i], -P.feq_scaled[i]));
    }
};

// Plain or streaming (non-temporal) global stores and loads.
template <bool NT, typename T> __device__ __forceinline__ void gstore(T *p, T v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <bool NT, typename T> __device__ __forceinline__ T gload(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Streaming (non-temporal) access to a complex value: data written once and
// read once much later (spectra on their way to the stash and the sums),
// which would only displace other lines from the L2.
typedef float flb_v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void stream_store(float2 *p, float2 v)
{
    flb_v2f t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, (flb_v2f *)p);
}
__device__ __forceinline__ float2 stream_load(const float2 *p)
{
    const flb_v2f t = __builtin_nontemporal_load((const flb_v2f *)p);
    return make_float2(t.x, t.y);
}

// D2Q9 velocities in the order of Sec. 3.
__device__ constexpr int kVX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kVY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

__device__ __forceinline__ int wrap_add(int x, int d, int n)
{
    int r = x + d;
    r = (r < 0) ? r + n : r;
    r = (r >= n) ? r - n : r;
    return r;
}

}  // namespace flbdev
