// flb_fft.h -- LDS line transforms shared by the correlator kernels.
//
// The LDS transforms are in-place radix-2 transforms with stages fused three
// at a time (radix 8): a thread loads eight elements, runs three butterfly
// stages in registers and stores them back, so a 4096-point line takes four
// passes and four barriers.  Power-of-two lines are transformed by
// decimation in time (bit-reversed input, natural output).  Lines of other
// lengths use Bluestein's chirp-z convolution with a power-of-two work
// length: a forward decimation-in-frequency transform (natural input,
// bit-reversed output) whose last pass multiplies by the transformed chirp
// kernel, then an inverse decimation-in-time transform back to natural
// order, so that no pass only permutes.
#pragma once

#include "flb_device.h"

namespace flbdev {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bitrev(int j, int lg)
{
    return lg ? (int)(__brev((unsigned)j) >> (32 - lg)) : 0;
}

// exp(-2 pi i e / n) for 0 <= e < n, n a power of two <= kTwN, from the
// half-circle table.
__device__ __forceinline__ float2 twiddle(const float2 *tw, int e, int lgn)
{
    const int i = e << (kTwLog - lgn);
    if (i < kTwN / 2) return tw[i];
    const float2 w = tw[i - kTwN / 2];
    return make_float2(-w.x, -w.y);
}

// LDS slot of element index i.  Rows are stored contiguously, and the
// bit-reversed writes and first radix-8 passes would put a whole wave on a
// few banks; one pad slot every 16 and every 256 elements spreads every
// access pattern of the row kernel over all banks (two-way at most for
// 8-byte elements).  Column layouts interleave lines and need no padding.
template <bool PAD> __host__ __device__ __forceinline__ int lds_slot(int i)
{
    return PAD ? i + (i >> 4) + (i >> 8) : i;
}

__host__ __device__ constexpr int lds_padded_elems(int n) { return n + (n >> 4) + (n >> 8) + 1; }

// w * exp(-/+ 2 pi i m / 2^(u+1)) for the compile-time root index (u, m),
// u <= 3: multiplications by 1 and -i are free, by exp(-i pi/4) two
// multiplies; an odd multiple of pi/8 (u = 3) first takes one general
// complex multiply by exp(-/+ i pi/8).
template <int U, int M, bool INV>
__device__ __forceinline__ float2 rotate(float2 w)
{
    if constexpr (U == 3) {
        if constexpr (M % 2 == 0) {
            return rotate<2, M / 2, INV>(w);
        } else {
            constexpr float c = 0.92387953251128674f, s = 0.38268343236508977f;  // pi/8
            const float2 r = INV ? make_float2(c * w.x - s * w.y, c * w.y + s * w.x)
                                 : make_float2(c * w.x + s * w.y, c * w.y - s * w.x);
            return rotate<2, M / 2, INV>(r);
        }
    } else {
        constexpr int q = (M << (2 - U)) & 7;  // the root as a multiple of pi/4
        constexpr float c = 0.70710678118654752f;
        float2 r = w;
        if constexpr (q & 1) {  // exp(-i pi/4) (forward) or exp(+i pi/4) (inverse)
            r = INV ? make_float2(c * (w.x - w.y), c * (w.x + w.y))
                    : make_float2(c * (w.x + w.y), c * (w.y - w.x));
        }
        if constexpr (q & 2) r = INV ? make_float2(-r.y, r.x) : make_float2(r.y, -r.x);  // -/+ i
        if constexpr (q & 4) r = make_float2(-r.x, -r.y);
        return r;
    }
}

// The butterflies of one group of 2^R elements of a pass of R fused radix-2
// stages (below), in registers.  Sub-stage u pairs j and j + 2^u with twiddle
// exp(-2 pi i (k + m h) / (h 2^(u+1))), m = j mod 2^u; all are w^(2^(R-1-u))
// times a fixed 2^(u+1)-th root of unity, with w = exp(-/+ 2 pi i k / (h 2^R))
// (the sign of the inverse transform already applied).  Decimation in time
// (DIF false) runs u = 0 .. R-1 and multiplies the second operand by the
// twiddle before the sum and difference; decimation in frequency (DIF true)
// runs u = R-1 .. 0 and multiplies the difference.
// UNIT: w = 1 (the first pass of a decimation in time, the last of a
// decimation in frequency, k = 0): every twiddle is a fixed root of unity and
// is applied to the operand directly by rotate (multiplications by 1 and -i
// cost nothing, by the eighth roots two multiplies).
template <int R, bool INV, bool DIF, bool UNIT = false>
__device__ __forceinline__ void group_butterflies(float2 (&v)[1 << R], float2 w)
{
    constexpr int G = 1 << R;
    if constexpr (UNIT) {
        (void)w;
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int u = DIF ? R - 1 - uu : uu;
            const int half = 1 << u;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (j & half) continue;
                const int m = j & (half - 1);
                auto rot = [&](float2 x) -> float2 {
                    if (m == 0) return x;
                    if (u == 1) return rotate<1, 1, INV>(x);
                    if (u == 2)
                        return m == 1 ? rotate<2, 1, INV>(x) : m == 2 ? rotate<2, 2, INV>(x)
                                                                     : rotate<2, 3, INV>(x);
                    return m == 1 ? rotate<3, 1, INV>(x) : m == 2 ? rotate<3, 2, INV>(x)
                         : m == 3 ? rotate<3, 3, INV>(x) : m == 4 ? rotate<3, 4, INV>(x)
                         : m == 5 ? rotate<3, 5, INV>(x) : m == 6 ? rotate<3, 6, INV>(x)
                                                                 : rotate<3, 7, INV>(x);
                };
                if constexpr (DIF) {
                    const float2 a = v[j], c = v[j + half];
                    v[j] = make_float2(a.x + c.x, a.y + c.y);
                    v[j + half] = rot(make_float2(a.x - c.x, a.y - c.y));
                } else {
                    const float2 x = rot(v[j + half]);
                    v[j + half] = make_float2(v[j].x - x.x, v[j].y - x.y);
                    v[j] = make_float2(v[j].x + x.x, v[j].y + x.y);
                }
            }
        }
        return;
    }
    float2 base[4];
    if constexpr (R == 4) {
        base[3] = w;
        base[2] = cmul(w, w);
        base[1] = cmul(base[2], base[2]);
        base[0] = cmul(base[1], base[1]);
    } else {
        base[R - 1] = w;
        if constexpr (R >= 2) base[R - 2] = cmul(w, w);
        if constexpr (R >= 3) base[0] = cmul(base[1], base[1]);
    }
#pragma unroll
    for (int uu = 0; uu < R; ++uu) {
        const int u = DIF ? R - 1 - uu : uu;
        const int half = 1 << u;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (j & half) continue;
            const int m = j & (half - 1);
            float2 t;
            if (u == 0) t = base[0];
            else if (u == 1) t = m ? rotate<1, 1, INV>(base[1]) : base[1];
            else if (u == 2)
                t = m == 0 ? base[2] : m == 1 ? rotate<2, 1, INV>(base[2])
                  : m == 2 ? rotate<2, 2, INV>(base[2]) : rotate<2, 3, INV>(base[2]);
            else
                t = m == 0 ? base[3] : m == 1 ? rotate<3, 1, INV>(base[3])
                  : m == 2 ? rotate<3, 2, INV>(base[3]) : m == 3 ? rotate<3, 3, INV>(base[3])
                  : m == 4 ? rotate<3, 4, INV>(base[3]) : m == 5 ? rotate<3, 5, INV>(base[3])
                  : m == 6 ? rotate<3, 6, INV>(base[3]) : rotate<3, 7, INV>(base[3]);
            if constexpr (DIF) {
                const float2 a = v[j], c = v[j + half];
                v[j] = make_float2(a.x + c.x, a.y + c.y);
                v[j + half] = cmul(t, make_float2(a.x - c.x, a.y - c.y));
            } else {
                const float2 x = cmul(t, v[j + half]);
                v[j + half] = make_float2(v[j].x - x.x, v[j].y - x.y);
                v[j] = make_float2(v[j].x + x.x, v[j].y + x.y);
            }
        }
    }
}

// One pass of R fused radix-2 stages s .. s+R-1 (1-based; stage s pairs
// elements h = 2^(s-1) apart) over `nlines` lines of length 2^lg; element e
// of line l at slot(l * ls + e * es).  A thread takes the 2^R elements
// b + k + j h (j < 2^R) of one group and runs group_butterflies on them with
// w = exp(-2 pi i k / (h 2^R)), the one value read from the table.  With
// `post`, every output of the pass is multiplied by post[e] (e the element's
// index in its line).
template <int R, bool PAD, bool INV, bool DIF = false, bool UNIT = false>
__device__ __forceinline__ void fused_pass(float2 *buf, int lg, int s, int nlines, int ls, int es,
                                         const float2 *tw, const float2 *post = nullptr)
{
    constexpr int G = 1 << R;
    const int h = 1 << (s - 1);
    const int lgg = lg - R;  // log2 of groups per line
    const int total = nlines << lgg;
    // Lines stored contiguously (ls > 1): neighbouring threads take
    // neighbouring groups of one line.  Lines interleaved (ls == 1): they
    // take the same group of neighbouring lines.  Either way a wave's LDS
    // accesses are consecutive addresses.
    const bool interleaved = (ls == 1);
    const int st = h * es;
    const bool linear = !PAD || (st & 255) == 0;  // padded slots advance uniformly
    const int sst = PAD ? st + (st >> 4) + (st >> 8) : st;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int l, g;
        if (interleaved) {
            g = idx / nlines;
            l = idx - g * nlines;
        } else {
            l = idx >> lgg;
            g = idx & ((1 << lgg) - 1);
        }
        const int k = g & (h - 1);
        const int b = (g >> (s - 1)) << (s - 1 + R);
        const int e0 = l * ls + (b + k) * es;
        int slot[G];
        if (linear) {
            const int s0 = lds_slot<PAD>(e0);
#pragma unroll
            for (int j = 0; j < G; ++j) slot[j] = s0 + j * sst;
        } else {
#pragma unroll
            for (int j = 0; j < G; ++j) slot[j] = lds_slot<PAD>(e0 + j * st);
        }
        float2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = buf[slot[j]];
        float2 w = make_float2(1.f, 0.f);
        if constexpr (!UNIT) {
            w = tw[k << (kTwLog - (s + R - 1))];
            if (INV) w.y = -w.y;
        }
        group_butterflies<R, INV, DIF, UNIT>(v, w);
        if (post) {
#pragma unroll
            for (int j = 0; j < G; ++j) v[j] = cmul(v[j], post[b + k + j * h]);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) buf[slot[j]] = v[j];
    }
}

// In-place transform of lines given in bit-reversed order; natural order out.
// RMAX: at most that many stages per pass (3, or 4 for kernels with the
// registers to hold sixteen elements per thread).
template <bool PAD, bool INV, int RMAX = 3>
__device__ __forceinline__ void lds_fft_dit(float2 *buf, int lg, int nlines, int ls, int es, const float2 *tw)
{
    if (lg < 1) return;
    // the first pass (stages 1 .. r, k = 0) has fixed twiddles only
    int s = 1;
    {
        const int r = lg < RMAX ? lg : RMAX;
        if (RMAX >= 4 && r >= 4) fused_pass<(RMAX >= 4 ? 4 : 3), PAD, INV, false, true>(buf, lg, 1, nlines, ls, es, tw);
        else if (r == 3) fused_pass<3, PAD, INV, false, true>(buf, lg, 1, nlines, ls, es, tw);
        else if (r == 2) fused_pass<2, PAD, INV, false, true>(buf, lg, 1, nlines, ls, es, tw);
        else fused_pass<1, PAD, INV, false, true>(buf, lg, 1, nlines, ls, es, tw);
        s += r;
        __syncthreads();
    }
    while (s <= lg) {
        const int r = lg - s + 1;
        if constexpr (RMAX >= 4) {
            if (r >= 4) {
                fused_pass<4, PAD, INV>(buf, lg, s, nlines, ls, es, tw);
                s += 4;
                __syncthreads();
                continue;
            }
        }
        if (r >= 3) {
            fused_pass<3, PAD, INV>(buf, lg, s, nlines, ls, es, tw);
            s += 3;
        } else if (r == 2) {
            fused_pass<2, PAD, INV>(buf, lg, s, nlines, ls, es, tw);
            s += 2;
        } else {
            fused_pass<1, PAD, INV>(buf, lg, s, nlines, ls, es, tw);
            s += 1;
        }
        __syncthreads();
    }
}

// In-place forward transform of lines given in natural order; bit-reversed
// order out, each output (at line element e) multiplied by post[e].  The
// widest stages go first, the radix-2 or radix-4 remainder last.
template <bool PAD, int RMAX = 3>
__device__ __forceinline__ void lds_fft_dif(float2 *buf, int lg, int nlines, int ls, int es,
                                            const float2 *tw, const float2 *post)
{
    int top = lg;  // stages 1 .. top are left
    while (top >= 1) {
        const int r = top >= RMAX ? RMAX : top;
        const int s = top - r + 1;
        if (s == 1) {  // the last pass: k = 0, fixed twiddles only
            if (RMAX >= 4 && r == 4)
                fused_pass<(RMAX >= 4 ? 4 : 3), PAD, false, true, true>(buf, lg, 1, nlines, ls, es, tw, post);
            else if (r == 3) fused_pass<3, PAD, false, true, true>(buf, lg, 1, nlines, ls, es, tw, post);
            else if (r == 2) fused_pass<2, PAD, false, true, true>(buf, lg, 1, nlines, ls, es, tw, post);
            else fused_pass<1, PAD, false, true, true>(buf, lg, 1, nlines, ls, es, tw, post);
            __syncthreads();
            break;
        }
        if constexpr (RMAX >= 4) {
            if (r == 4) {
                fused_pass<4, PAD, false, true>(buf, lg, s, nlines, ls, es, tw);
                top -= 4;
                __syncthreads();
                continue;
            }
        }
        if (r == 3) fused_pass<3, PAD, false, true>(buf, lg, s, nlines, ls, es, tw);
        else if (r == 2) fused_pass<2, PAD, false, true>(buf, lg, s, nlines, ls, es, tw);
        else fused_pass<1, PAD, false, true>(buf, lg, s, nlines, ls, es, tw);
        top -= r;
        __syncthreads();
    }
}

// Where a line transform expects element x of a line: bit-reversed for
// power-of-two lengths (lds_fft_dit), natural order for Bluestein work
// lengths (lds_bluestein_dft).
__device__ __forceinline__ int line_in_pos(const LinePlan &L, int x)
{
    return L.bluestein ? x : bitrev(x, L.log2m);
}

// Length-n DFT of Bluestein lines (L.bluestein) whose element x was written
// in natural order, already multiplied by the chirp, in place; on exit
// element k < n holds X_k in natural order.  The transformed chirp kernel is
// stored in bit-reversed order, the order of the forward transform's output.
// With CHIRP false the lines are left without their final chirp factor: the
// caller multiplies element k by the chirp's k-th value as it reads it.
// Kernels that know a plan's kind at compile time call this or lds_fft_dit
// directly, so that a power-of-two instantiation carries no Bluestein code.
template <bool PAD, bool CHIRP = true, int RMAX = 3>
__device__ __forceinline__ void lds_bluestein_dft(float2 *buf, const LinePlan &L, int nlines,
                                                  int ls, int es, const float2 *tables)
{
    const float2 *tw = tables;
    lds_fft_dif<PAD, RMAX>(buf, L.log2m, nlines, ls, es, tw, tables + L.kernel_off);
    lds_fft_dit<PAD, true, RMAX>(buf, L.log2m, nlines, ls, es, tw);
    if constexpr (!CHIRP) return;
    const float2 *C = tables + L.chirp_off;
    for (int idx = threadIdx.x; idx < nlines * L.n; idx += blockDim.x) {
        const int l = idx / L.n, j = idx - l * L.n;
        float2 *p = buf + lds_slot<PAD>(l * ls + j * es);
        *p = cmul(*p, C[j]);
    }
    __syncthreads();
}

// Either kind of plan, chosen at run time: lines whose element x was written
// at line_in_pos(L, x).
template <bool PAD>
__device__ __forceinline__ void lds_line_dft(float2 *buf, const LinePlan &L, int nlines, int ls,
                                             int es, const float2 *tables)
{
    if (L.bluestein) lds_bluestein_dft<PAD>(buf, L, nlines, ls, es, tables);
    else lds_fft_dit<PAD, false>(buf, L.log2m, nlines, ls, es, tables);
}

constexpr int kFftThreads = 512;  // threads of the transform kernels
// Global loads of the transform kernels are issued kBatch per thread before
// any of them is used, so that each thread keeps several requests in flight
// (one load per loop iteration leaves the kernels latency-bound).
constexpr int kBatch = 8;

}  // namespace flbdev
