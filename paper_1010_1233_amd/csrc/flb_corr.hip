// flb_corr.hip -- correlator sample: spatial transforms of the fluctuation
// fields and FP64 accumulation of Eqs. (11)-(12).
//
// Fields (FP32): d rho = rho - rho0, d j = j - rho0 u0, d u = j / rho - u0.
// Subtracting the constant reference instead of the spatial mean changes the
// transform only at k = 0, which is not accumulated (the paper's fluctuation
// dM = M - <M> has no k = 0 component), and keeps the FP32 transforms free of
// a large mean.
//
// Per sample:
//   rows   one block per group of rows gathers the state once, keeps rho and
//          j of its sites in registers and transforms three packed complex
//          lines per row (jx + i jy, ux + i uy, rho) along x through one LDS
//          buffer; it writes the half spectra kx = 0..nx/2 of the five real
//          fields and the FP64 conservation partials of its rows.  (The
//          optional moment set goes through FP32 field planes and a separate
//          row kernel.)
//   columns: whole columns are transformed in LDS (Bluestein's convolution
//          for lengths that are not powers of two; power-of-two columns of
//          512 to 4096 points in a persistent, pipelined kernel) and the
//          spectra go to one of kDeferK (32) stash slots, column-tiled;
//          with every kDeferK-th sample a second kernel adds the products
//          of all the stashed samples to the FP64 sums, one thread per k.
// The line transforms themselves are in flb_fft.h.
#include <algorithm>
#include <type_traits>

#include "flb_corr_internal.h"
#include "flb_fft.h"

namespace flbdev {

struct CorrArgs {
    const void *pops;
    const LatticeParams *params;
    const LinePlan *plans;
    const float2 *tables;
    const CorrItem *items;
    float2 *spec;
    float2 *stash;  // spectra of samples whose products are not yet added (stash_offset)
    int arg;        // stash slot (stash mode) or number of slots (pair mode, flush)
    double *acc;
    float *fields;
    double *csum_part;
    double *csum;
    int set;  // field set: 0 = rho, j, u; 1 = moments 3..8
};

// Block sum of five doubles into out[0..4] (deterministic order), for
// blocks of NT threads.
template <int NT> __device__ __forceinline__ void block_sum5(double (&v)[5], double *out)
{
    __shared__ double red[5][NT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) red[q][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double x = 0;
        for (int w = 0; w < NT / 64; ++w) x += red[threadIdx.x][w];
        out[threadIdx.x] = x;
    }
}

// Deviations f_i - w_i rho0 arriving at site (x, y): the current state
// pulled along each velocity (streaming, Eq. 1).
template <int S>
__device__ __forceinline__ void pull_site(const typename Codec<S>::T *p, const LatticeParams &P,
                                          int x, int y, float (&d)[9])
{
    const int nx = P.nx, ny = P.ny, px = P.px, plane = (int)P.plane;
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int rc = y * px, rm = ym * px, rp = yp * px;
    d[0] = Codec<S>::decode(p[rc + x], P, 0);
    d[1] = Codec<S>::decode(p[1 * plane + rc + xm], P, 1);
    d[2] = Codec<S>::decode(p[2 * plane + rm + x], P, 2);
    d[3] = Codec<S>::decode(p[3 * plane + rc + xp], P, 3);
    d[4] = Codec<S>::decode(p[4 * plane + rp + x], P, 4);
    d[5] = Codec<S>::decode(p[5 * plane + rm + xm], P, 5);
    d[6] = Codec<S>::decode(p[6 * plane + rm + xp], P, 6);
    d[7] = Codec<S>::decode(p[7 * plane + rp + xp], P, 7);
    d[8] = Codec<S>::decode(p[8 * plane + rp + xm], P, 8);
}

// Non-conserved moments M^3..M^8 (rows of Eq. 9) at site (x, y).  The rows
// are orthogonal to M^0 under the weights, so the moments of the deviations
// are the moments themselves.
template <int S>
__device__ __forceinline__ void site_moments(const typename Codec<S>::T *p,
                                             const LatticeParams &P, int x, int y,
                                             float (&M)[6])
{
    float d[9];
    pull_site<S>(p, P, x, y, d);
    const float axis = (d[1] + d[3]) + (d[2] + d[4]);
    const float diag = (d[5] + d[7]) + (d[6] + d[8]);
    const float s32 = 1.2247448713915890f, s6 = 2.4494897427831781f;
    M[0] = 1.5f * ((d[1] + d[3]) - (d[2] + d[4]));
    M[1] = 3.0f * ((d[5] + d[7]) - (d[6] + d[8]));
    M[2] = fmaf(0.5f, axis, fmaf(2.0f, diag, -d[0]));
    M[3] = fmaf(s32, d[3] - d[1], s6 * ((d[5] - d[7]) + (d[8] - d[6])));
    M[4] = fmaf(s32, d[4] - d[2], s6 * ((d[5] - d[7]) + (d[6] - d[8])));
    M[5] = fmaf(0.5f, d[0], fmaf(2.0f, diag, -axis));
}

// Writes the packed half spectra of one group of transformed lines: for the
// pair z = a + i b of two real sequences, a_k = (z_k + conj z_{-k}) / 2 and
// b_k = (z_k - conj z_{-k}) / (2i) go to fields fa and fa + 1; a single real
// sequence (pair false) goes to field fa as is.  kx = 0..nx/2, padding
// columns up to kxp zeroed.  With `chirp`, line element k is first
// multiplied by chirp[k] (a Bluestein line left without its output chirp).
// The spectra are streamed: the column transforms read them back only
// after the whole launch has written them.
__device__ __forceinline__ void store_row_spectra(const float2 *lds, const LatticeParams &P,
                                                  float2 *spec, int y0, int nl, int m, int fa,
                                                  bool pair, const float2 *chirp = nullptr)
{
    const int nx = P.nx, nkx = P.nkx, kxp = P.kxp;
    const int64_t fstride = (int64_t)P.ny * kxp;
    float2 *sa = spec + fa * fstride, *sb = sa + fstride;
    // line l = e / kxp by a float reciprocal: (e + 1/2) / kxp stays at least
    // 1/(2 kxp) away from an integer, far beyond the rounding of the product
    // (e < 8192, kxp < 4096)
    const float rkxp = 1.0f / (float)kxp;
    for (int e = threadIdx.x; e < nl * kxp; e += kFftThreads) {
        const int l = (int)(((float)e + 0.5f) * rkxp), k = e - l * kxp;
        const int64_t row = (int64_t)(y0 + l) * kxp + k;
        if (k >= nkx) {  // padding columns: keep them finite
            sa[row] = make_float2(0.f, 0.f);
            if (pair) sb[row] = make_float2(0.f, 0.f);
            continue;
        }
        float2 zk = lds[lds_slot<true>(l * m + k)];
        if (chirp) zk = cmul(zk, chirp[k]);
        if (!pair) {
            stream_store(&sa[row], zk);
        } else {
            const int km = k == 0 ? 0 : nx - k;
            float2 zm = lds[lds_slot<true>(l * m + km)];
            if (chirp) zm = cmul(zm, chirp[km]);
            stream_store(&sa[row], make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)));
            stream_store(&sb[row], make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x)));
        }
    }
}

// Field set 0, fields and row transforms in one pass: a block takes a group
// of rows (nl * m <= 4096 line elements), gathers the state of its sites once
// (pull along each velocity, Eq. 1), keeps rho - rho0 and j in registers and
// transforms three packed lines through one LDS buffer: jx + i jy and
// ux + i uy of the fluctuations d j = j - rho0 u0, d u = j / rho - u0, then
// rho - rho0 alone.  It also writes the FP64 conservation sums of its rows
// (mass, momentum, staggered momenta) as one partial.  BLUE: the lattice's
// rows use Bluestein's transform (other lengths than powers of two); the two
// cases are separate instantiations so that the power-of-two one carries no
// chirp state in registers.
// item: lattice, first row, rows, index of the block's partial.
// At most 80 VGPRs (six waves per SIMD, three blocks per CU): the kernel is
// bound by the latency of its transforms, and the third block hides more of
// it.  Measured at 4096^2 (sample alone, whole path, row-kernel HBM bytes
// over the algorithmic ones): 93 VGPRs 0.79 ms, 82.5 GLUPS, 1.00; 80 VGPRs
// (6 values spilled) 0.77 ms, 83.4 GLUPS, 1.17; 64 VGPRs (28 spilled)
// 0.80 ms, 84.1 GLUPS, 1.64, the spills' scratch traffic not worth the last
// percent.
template <int S, bool BLUE>
__global__ __launch_bounds__(kFftThreads, 6) void corr_rows_kernel(CorrArgs g)
{
    using T = typename Codec<S>::T;
    constexpr int E = 4096 / kFftThreads;  // line elements per thread
    extern __shared__ float2 lds[];
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_x];
    const int nx = P.nx;
    const int y0 = it.a, nl = min(it.b, P.ny - y0);
    const int m = L.m, lg = L.log2m, ne = nl * m;
    const T *p = (const T *)g.pops + P.base;

    float r[E], jx[E], jy[E];
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int e = (int)threadIdx.x + j * kFftThreads, l = e >> lg, x = e & (m - 1);
        r[j] = jx[j] = jy[j] = 0.f;
        if (e < ne && x < nx) {
            float d[9];
            pull_site<S>(p, P, x, y0 + l, d);
            r[j] = d[0] + (d[1] + d[3]) + (d[2] + d[4]) + (d[5] + d[7]) + (d[6] + d[8]);
            jx[j] = (d[1] - d[3]) + (d[5] - d[7]) - (d[6] - d[8]);
            jy[j] = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
            const double Jx = jx[j], Jy = jy[j];
            acc[0] += r[j];
            acc[1] += Jx;
            acc[2] += Jy;
            acc[3] += (x & 1) ? -Jx : Jx;
            acc[4] += ((y0 + l) & 1) ? -Jy : Jy;
        }
    }
    block_sum5<kFftThreads>(acc, g.csum_part + 5 * (int64_t)it.c);

    const float2 *chirp = g.tables + L.chirp_off;
    float2 *spec = g.spec + P.spec_base;
    const float rho0 = P.rho0, u0x = P.u0x, u0y = P.u0y;
    const float jx0 = rho0 * u0x, jy0 = rho0 * u0y;
#pragma unroll 1
    for (int sig = 0; sig < 3; ++sig) {
        // (the block sum and every earlier signal's reads of LDS are behind a
        // barrier before the lines are written)
        __syncthreads();
        // the line indices are recomputed for every signal rather than kept
        // in registers through the transforms
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        // (no branch per element: sites past a row's end, where the line
        // is zero padding, are set to zero by a select)
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = tid + j * kFftThreads, l = e >> lg, x = e & (m - 1);
            float2 v;
            if (sig == 0) {
                v = make_float2(jx[j] - jx0, jy[j] - jy0);
            } else if (sig == 1) {
                // u = j / rho with the hardware reciprocal (1 ulp)
                const float ir = __builtin_amdgcn_rcpf(rho0 + r[j]);
                v = make_float2(fmaf(jx[j], ir, -u0x), fmaf(jy[j], ir, -u0y));
            } else {
                v = make_float2(r[j], 0.f);
            }
            if (BLUE) v = cmul(v, chirp[x < nx ? x : 0]);
            if (x >= nx) v = make_float2(0.f, 0.f);
            if (e < ne) lds[lds_slot<true>(l * m + (BLUE ? x : bitrev(x, lg)))] = v;
        }
        __syncthreads();
        if (BLUE) lds_bluestein_dft<true, false>(lds, L, nl, m, 1, g.tables);
        else lds_fft_dit<true, false>(lds, lg, nl, m, 1, g.tables);
        // spectra: 1, 2 = jx, jy; 3, 4 = ux, uy; 0 = rho
        store_row_spectra(lds, P, spec, y0, nl, m, sig == 0 ? 1 : sig == 1 ? 3 : 0, sig != 2,
                          BLUE ? chirp : nullptr);
    }
}

// store_row_spectra for the blocks of corr_rows_p2_kernel, sizes fixed at
// compile time: the columns kx < 2^LG/2 of all lines four per thread (a
// line's half spans whole waves), then the Nyquist column and the padding
// columns up to k_xp = 2^LG/2 + 16.  The spectra of one lattice stay below
// 2^31 elements, so offsets from the field's base are 32-bit.
template <int LG>
__device__ __forceinline__ void store_row_spectra_p2(const float2 *lds, float2 *sa, float2 *sb,
                                                     int y0, int nl, bool pair, int tid)
{
    constexpr int M = 1 << LG, HALF = M / 2, KXP = HALF + 16, NL = 4096 >> LG;
    auto put = [&](int l, int k) {
        const uint32_t o = (uint32_t)((y0 + l) * KXP + k);
        const float2 zk = lds[lds_slot<true>(l * M + k)];
        if (!pair) {
            stream_store(&sa[o], zk);
        } else {
            const float2 zm = lds[lds_slot<true>(l * M + ((M - k) & (M - 1)))];
            stream_store(&sa[o], make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)));
            stream_store(&sb[o], make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x)));
        }
    };
#pragma unroll
    for (int q = 0; q < (NL * HALF) / kFftThreads; ++q) {
        const int e = tid + q * kFftThreads, l = e >> (LG - 1);
        if (l < nl) put(l, e & (HALF - 1));
    }
    if (tid < 16 * NL) {
        const int l = tid >> 4, k = HALF + (tid & 15);
        if (l < nl) {
            if (k == HALF) {
                put(l, k);
            } else {  // padding columns: keep them finite
                const uint32_t o = (uint32_t)((y0 + l) * KXP + k);
                sa[o] = make_float2(0.f, 0.f);
                if (pair) sb[o] = make_float2(0.f, 0.f);
            }
        }
    }
}

// One pass of R fused radix-2 stages S0 .. S0+R-1 (as fused_pass; inverse
// and decimation in frequency as there) over the 4096 >> LG lines of 2^LG
// elements in a row block's LDS, every size fixed at compile time.  The
// first decimation-in-time pass and the last decimation-in-frequency pass
// (S0 = 1) have fixed roots of unity only.
template <int LG, int S0, int R, bool INV = false, bool DIF = false>
__device__ __forceinline__ void row_fft_pass(float2 *buf, const float2 *tw, int tid)
{
    constexpr int M = 1 << LG, G = 1 << R, H = 1 << (S0 - 1);
    constexpr int PER = (4096 >> R) / kFftThreads;  // groups per thread
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * kFftThreads;
        const int l = idx >> (LG - R), gi = idx & ((1 << (LG - R)) - 1);
        const int k = gi & (H - 1);
        const int e0 = l * M + ((gi >> (S0 - 1)) << (S0 - 1 + R)) + k;
        float2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = buf[lds_slot<true>(e0 + j * H)];
        if constexpr (S0 == 1) {
            group_butterflies<R, INV, DIF, true>(v, make_float2(1.f, 0.f));
        } else {
            float2 w = tw[k << (kTwLog - (S0 + R - 1))];
            if (INV) w.y = -w.y;
            group_butterflies<R, INV, DIF>(v, w);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) buf[lds_slot<true>(e0 + j * H)] = v[j];
    }
}
template <int LG, int S0, int R>
__device__ __forceinline__ void row_dit_pass(float2 *buf, const float2 *tw, int tid)
{
    row_fft_pass<LG, S0, R>(buf, tw, tid);
}

// A block of corr_rows_p2_kernel for lattices whose rows are powers of
// two of 2^LG = 512 .. 4096 points: what corr_rows_kernel computes, with the
// line length fixed at compile time.  Thread t takes the eight sites x = c + j 2^LG/8 (j < 8) of
// line t / (2^LG/8) of the block, c = t mod 2^LG/8.  In bit-reversed order
// these sites are the eight consecutive elements 8 rev(c) .. 8 rev(c) + 7 of
// a line, one group of the first decimation-in-time pass (stages 1..3, no
// twiddles), so that pass runs on the gathered values in registers and
// writes eight consecutive LDS slots; stages 4..LG follow in LDS.  A line
// spans whole waves, so the rows a wave reads are wave-uniform and the
// gather addresses are scalar bases plus 32-bit offsets; the periodic wrap
// along x is a mask.
template <int S, int LG>
__device__ __forceinline__ void rows_p2_block(const CorrArgs &g, const CorrItem &it)
{
    using T = typename Codec<S>::T;
    constexpr int M = 1 << LG, H = M >> 3;
    static_assert(LG >= 9 && LG <= 12, "a line spans whole waves; a block holds 4096 elements");
    extern __shared__ float2 lds[];
    const LatticeParams &P = g.params[it.lattice];
    const int y0 = it.a, nl = min(it.b, P.ny - y0);
    const int t = (int)threadIdx.x, c = t & (H - 1);
    const int l = __builtin_amdgcn_readfirstlane(t >> (LG - 3));
    const T *p = (const T *)g.pops + P.base;

    float r[8], jx[8], jy[8];
    double acc[5] = {0, 0, 0, 0, 0};
    if (l < nl) {
        // wave-uniform plane rows: scalar bases, 32-bit offsets
        const int ny = P.ny, y = y0 + l;
        const int ym = __builtin_amdgcn_readfirstlane(y == 0 ? ny - 1 : y - 1);
        const int yp = __builtin_amdgcn_readfirstlane(y == ny - 1 ? 0 : y + 1);
        const int64_t px = P.px, pl = P.plane;
        const T *rc = p + y * px, *rm = p + ym * px, *rp = p + yp * px;
        const T *__restrict__ q0 = rc, *__restrict__ q1 = rc + pl, *__restrict__ q2 = rm + 2 * pl;
        const T *__restrict__ q3 = rc + 3 * pl, *__restrict__ q4 = rp + 4 * pl;
        const T *__restrict__ q5 = rm + 5 * pl, *__restrict__ q6 = rm + 6 * pl;
        const T *__restrict__ q7 = rp + 7 * pl, *__restrict__ q8 = rp + 8 * pl;
        double sx = 0, sy = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t x = (uint32_t)(c + j * H), xm = (x - 1) & (M - 1), xp = (x + 1) & (M - 1);
            float d[9];
            d[0] = Codec<S>::decode(q0[x], P, 0);
            d[1] = Codec<S>::decode(q1[xm], P, 1);
            d[2] = Codec<S>::decode(q2[x], P, 2);
            d[3] = Codec<S>::decode(q3[xp], P, 3);
            d[4] = Codec<S>::decode(q4[x], P, 4);
            d[5] = Codec<S>::decode(q5[xm], P, 5);
            d[6] = Codec<S>::decode(q6[xp], P, 6);
            d[7] = Codec<S>::decode(q7[xp], P, 7);
            d[8] = Codec<S>::decode(q8[xm], P, 8);
            r[j] = d[0] + (d[1] + d[3]) + (d[2] + d[4]) + (d[5] + d[7]) + (d[6] + d[8]);
            jx[j] = (d[1] - d[3]) + (d[5] - d[7]) - (d[6] - d[8]);
            jy[j] = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
            acc[0] += r[j];
            sx += jx[j];
            sy += jy[j];
        }
        // the thread's sites share the parity of x (c) and of y
        acc[1] = sx;
        acc[2] = sy;
        acc[3] = (c & 1) ? -sx : sx;
        acc[4] = (y & 1) ? -sy : sy;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = jx[j] = jy[j] = 0.f;
    }
    block_sum5<kFftThreads>(acc, g.csum_part + 5 * (int64_t)it.c);

    const float2 *tw = g.tables;
    float2 *spec = g.spec + P.spec_base;
    const int64_t fstride = (int64_t)P.ny * P.kxp;
    const float rho0 = P.rho0, u0x = P.u0x, u0y = P.u0y;
    const float jx0 = rho0 * u0x, jy0 = rho0 * u0y;
    // (unrolled, so that the sites' j die after the second field pair and
    // the kernel keeps to 80 registers without spilling; rolled up, the
    // loop held every site value to its end and spilled)
#pragma unroll
    for (int sig = 0; sig < 3; ++sig) {
        // LDS addresses are recomputed for every signal rather than kept in
        // registers through the loop
        int tid = t;
        asm volatile("" : "+v"(tid));
        // first slot of the thread's group: eight consecutive slots (a pad
        // slot falls only at multiples of 16)
        const int base = lds_slot<true>(l * M + 8 * bitrev(tid & (H - 1), LG - 3));
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (sig == 0) {
                v[j] = make_float2(jx[j] - jx0, jy[j] - jy0);
            } else if (sig == 1) {
                const float ir = __builtin_amdgcn_rcpf(rho0 + r[j]);
                v[j] = make_float2(fmaf(jx[j], ir, -u0x), fmaf(jy[j], ir, -u0y));
            } else {
                v[j] = make_float2(r[j], 0.f);
            }
            if (l >= nl) v[j] = make_float2(0.f, 0.f);
        }
        // element 8 rev(c) + i of the line is site x = c + rev3(i) H
        float2 u[8] = {v[0], v[4], v[2], v[6], v[1], v[5], v[3], v[7]};
        group_butterflies<3, false, false, true>(u, make_float2(1.f, 0.f));
        // (the block sum and the previous signal's reads of LDS are behind
        // this barrier)
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[base + i] = u[i];
        __syncthreads();
        row_dit_pass<LG, 4, 3>(lds, tw, tid);
        __syncthreads();
        if constexpr (LG >= 10) {
            row_dit_pass<LG, 7, 3>(lds, tw, tid);
            __syncthreads();
            row_dit_pass<LG, 10, LG - 9>(lds, tw, tid);
        } else {
            row_dit_pass<LG, 7, 3>(lds, tw, tid);
        }
        __syncthreads();
        // spectra: 1, 2 = jx, jy; 3, 4 = ux, uy; 0 = rho
        float2 *sa = spec + (sig == 0 ? 1 : sig == 1 ? 3 : 0) * fstride;
        store_row_spectra_p2<LG>(lds, sa, sa + fstride, y0, nl, sig != 2, tid);
    }
}


// The middle of a Bluestein convolution in a row block, on groups of 2^R
// consecutive elements: the last stages of the forward decimation in
// frequency (stages R .. 1, fixed roots), the product with the transformed
// chirp kernel (bit-reversed order, as the forward transform leaves it) and
// the first stages of the inverse decimation in time (1 .. R) in registers,
// one LDS round trip for the three.
template <int LG, int R>
__device__ __forceinline__ void row_blue_middle(float2 *buf, const float2 *kern, int tid)
{
    constexpr int G = 1 << R, PER = (4096 >> R) / kFftThreads;
    constexpr int M = 1 << LG;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e0 = (tid + q * kFftThreads) << R;  // line l = e0 / M, element e0 % M
        const int s0 = lds_slot<true>(e0);            // G <= 8 consecutive slots
        float2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = buf[s0 + j];
        group_butterflies<R, false, true, true>(v, make_float2(1.f, 0.f));
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = cmul(v[j], kern[(e0 & (M - 1)) + j]);
        group_butterflies<R, true, false, true>(v, make_float2(1.f, 0.f));
#pragma unroll
        for (int j = 0; j < G; ++j) buf[s0 + j] = v[j];
    }
}

// A block of corr_rows_blue_kernel for lattices whose rows take
// Bluestein's transform with a work length of 2^LG = 256 .. 2048 (rows of n
// points, 2n - 1 <= 2^LG, n not a power of two): what corr_rows_kernel<S,
// true> computes, with the work length fixed at compile time.  A block holds 4096 >> LG lines; thread t
// takes the elements x = c + j 2^LG/8 (j < 8) of line t / (2^LG/8),
// c = t mod 2^LG/8, which are one group of the forward transform's first
// radix-8 pass (decimation in frequency, natural order); as 2^LG >= 2n - 1,
// only j < 4 can hold sites, the rest are the convolution's zero padding.
// That pass runs on the gathered, chirp-multiplied values in registers; the
// forward transform's last pass, the product with the chirp kernel's
// transform and the inverse transform's first pass share one LDS round
// trip.  Passes per field pair: 6 (2^11), 6 (2^10), 4 (2^9), 4 (2^8), and
// one store.
template <int S, int LG>
__device__ __forceinline__ void rows_blue_block(const CorrArgs &g, const CorrItem &it)
{
    using T = typename Codec<S>::T;
    constexpr int M = 1 << LG, H = M >> 3;
    static_assert(LG >= 8 && LG <= 11, "work lengths 256 .. 2048");
    extern __shared__ float2 lds[];
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_x];
    const int nx = P.nx;
    const int y0 = it.a, nl = min(it.b, P.ny - y0);
    const int t = (int)threadIdx.x, c = t & (H - 1);
    // a line spans whole waves from 2^9 on
    const int l = LG >= 9 ? __builtin_amdgcn_readfirstlane(t >> (LG - 3)) : t >> (LG - 3);
    const T *p = (const T *)g.pops + P.base;
    const float2 *chirp = g.tables + L.chirp_off;

    float r[4], jx[4], jy[4];
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = jx[j] = jy[j] = 0.f;
    if (l < nl) {
        const int y = y0 + l;
        double sx = 0, sy = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = c + j * H;
            if (x < nx) {
                float d[9];
                pull_site<S>(p, P, x, y, d);
                r[j] = d[0] + (d[1] + d[3]) + (d[2] + d[4]) + (d[5] + d[7]) + (d[6] + d[8]);
                jx[j] = (d[1] - d[3]) + (d[5] - d[7]) - (d[6] - d[8]);
                jy[j] = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
                acc[0] += r[j];
                sx += jx[j];
                sy += jy[j];
            }
        }
        // the thread's sites share the parity of x (c) and of y
        acc[1] = sx;
        acc[2] = sy;
        acc[3] = (c & 1) ? -sx : sx;
        acc[4] = (y & 1) ? -sy : sy;
    }
    block_sum5<kFftThreads>(acc, g.csum_part + 5 * (int64_t)it.c);

    const float2 *tw = g.tables;
    const float2 *kern = g.tables + L.kernel_off;
    float2 *spec = g.spec + P.spec_base;
    const float rho0 = P.rho0, u0x = P.u0x, u0y = P.u0y;
    const float jx0 = rho0 * u0x, jy0 = rho0 * u0y;
#pragma unroll
    for (int sig = 0; sig < 3; ++sig) {
        int tid = t;
        asm volatile("" : "+v"(tid));
        const int cc = tid & (H - 1), base = (l * M) + cc;
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = cc + j * H;
            float2 z;
            if (sig == 0) {
                z = make_float2(jx[j] - jx0, jy[j] - jy0);
            } else if (sig == 1) {
                const float ir = __builtin_amdgcn_rcpf(rho0 + r[j]);
                z = make_float2(fmaf(jx[j], ir, -u0x), fmaf(jy[j], ir, -u0y));
            } else {
                z = make_float2(r[j], 0.f);
            }
            z = cmul(z, chirp[x < nx ? x : 0]);
            v[j] = (x < nx && l < nl) ? z : make_float2(0.f, 0.f);
            v[j + 4] = make_float2(0.f, 0.f);
        }
        // forward stages LG .. LG-2 (decimation in frequency), twiddle
        // exp(-2 pi i c / 2^LG)
        group_butterflies<3, false, true>(v, tw[cc << (kTwLog - LG)]);
        // (the block sum and the previous signal's reads of LDS are behind
        // this barrier)
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) lds[lds_slot<true>(base + j * H)] = v[j];
        __syncthreads();
        // the rest of the forward transform, the kernel product, the
        // inverse transform (decimation in time) back to natural order
        if constexpr (LG == 11) {
            row_fft_pass<LG, 6, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 3, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_blue_middle<LG, 2>(lds, kern, tid);
            __syncthreads();
            row_fft_pass<LG, 3, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 6, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 9, 3, true>(lds, tw, tid);
        } else if constexpr (LG == 10) {
            row_fft_pass<LG, 5, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 2, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_blue_middle<LG, 1>(lds, kern, tid);
            __syncthreads();
            row_fft_pass<LG, 2, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 5, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 8, 3, true>(lds, tw, tid);
        } else if constexpr (LG == 9) {
            row_fft_pass<LG, 4, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_blue_middle<LG, 3>(lds, kern, tid);
            __syncthreads();
            row_fft_pass<LG, 4, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 7, 3, true>(lds, tw, tid);
        } else {
            row_fft_pass<LG, 3, 3, false, true>(lds, tw, tid);
            __syncthreads();
            row_blue_middle<LG, 2>(lds, kern, tid);
            __syncthreads();
            row_fft_pass<LG, 3, 3, true>(lds, tw, tid);
            __syncthreads();
            row_fft_pass<LG, 6, 3, true>(lds, tw, tid);
        }
        __syncthreads();
        // spectra: 1, 2 = jx, jy; 3, 4 = ux, uy; 0 = rho (the output chirp
        // applied as they are read)
        store_row_spectra(lds, P, spec, y0, nl, M, sig == 0 ? 1 : sig == 1 ? 3 : 0, sig != 2,
                          chirp);
    }
}


// Field set 0 for lattices whose rows have a length-specialised block: one
// kernel per power-of-two length (corr_rows_p2_kernel; the lattices of a
// batch usually share one), one for every Bluestein work length together
// (corr_rows_blue_kernel: each block takes the code of its lattice's plan,
// so that the lengths of an uneven batch share the device instead of
// queueing as launches of their own; a kernel holding the power-of-two
// blocks too took their registers and was slower for them).
template <int S, int LG>
__global__ __launch_bounds__(kFftThreads, 6) void corr_rows_p2_kernel(CorrArgs g)
{
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    rows_p2_block<S, LG>(g, it);
}

// (64 registers, four blocks per compute unit: 20 bytes of each thread
// spill, and the uneven batch's sample is still 2 % faster than with three
// blocks and no spill)
template <int S>
__global__ __launch_bounds__(kFftThreads, 8) void corr_rows_blue_kernel(CorrArgs g)
{
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    switch (g.plans[g.params[it.lattice].line_x].log2m) {
    case 8: rows_blue_block<S, 8>(g, it); break;
    case 9: rows_blue_block<S, 9>(g, it); break;
    case 10: rows_blue_block<S, 10>(g, it); break;
    case 11: rows_blue_block<S, 11>(g, it); break;
    default: break;
    }
}

__global__ __launch_bounds__(kThreads) void corr_csum_kernel(CorrArgs g, int nlat)
{
    const int l = blockIdx.x;
    if (l >= nlat) return;
    const LatticeParams &P = g.params[l];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < P.fld_nparts; b += kThreads)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += g.csum_part[5 * ((int64_t)P.fld_part0 + b) + q];
    block_sum5<kThreads>(acc, g.csum + 5 * (int64_t)l);
}

// Field set 1: the six non-conserved moments of the current state as FP32
// planes [6][ny][nx], one thread per column of a tile of 256 sites x
// kFieldRows rows.  item: lattice, tile.
template <int S>
__global__ __launch_bounds__(kThreads) void corr_moment_fields_kernel(CorrArgs g)
{
    using T = typename Codec<S>::T;
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int nx = P.nx, ny = P.ny;
    const int tx = it.a % P.fld_tiles_x, ty = it.a / P.fld_tiles_x;
    const int x = tx * kThreads + (int)threadIdx.x;
    if (x >= nx) return;
    const T *p = (const T *)g.pops + P.base;
    const int64_t fs = (int64_t)nx * ny;
    const int y1 = min(ny, (ty + 1) * kFieldRows);
    for (int y = ty * kFieldRows; y < y1; ++y) {
        float M[6];
        site_moments<S>(p, P, x, y, M);
        float *f = g.fields + P.fld_base + (int64_t)y * nx + x;
#pragma unroll
        for (int q = 0; q < 6; ++q) f[q * fs] = M[q];
    }
}

// Field set 1, row transforms: one block per (lattice, group of rows,
// signal s), s packing M^(3+2s) + i M^(4+2s).
// item: lattice, first row, rows in this block, signal
__global__ __launch_bounds__(kFftThreads) void corr_moment_rows_kernel(CorrArgs g)
{
    extern __shared__ float2 lds[];
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_x];
    const int nx = P.nx, ny = P.ny;
    const int y0 = it.a, nl = min(it.b, ny - y0), fa = 2 * it.c;
    const int m = L.m, lg = L.log2m;
    const float2 *chirp = g.tables + L.chirp_off;
    const int64_t fs = (int64_t)nx * ny;
    const float *fa_p = g.fields + P.fld_base + fa * fs;
    const float *fb_p = fa_p + fs;

    const int ne = nl * m;
    for (int e0 = threadIdx.x; e0 < ne; e0 += kBatch * kFftThreads) {
        float va[kBatch], vb[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int e = e0 + j * kFftThreads, l = e >> lg, x = e & (m - 1);
            va[j] = vb[j] = 0.f;
            if (e < ne && x < nx) {
                const int64_t o = (int64_t)(y0 + l) * nx + x;
                va[j] = fa_p[o];
                vb[j] = fb_p[o];
            }
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int e = e0 + j * kFftThreads, l = e >> lg, x = e & (m - 1);
            if (e >= ne) break;
            float2 v = make_float2(va[j], vb[j]);
            if (L.bluestein && x < nx) v = cmul(v, chirp[x]);
            lds[lds_slot<true>(l * m + line_in_pos(L, x))] = v;
        }
    }
    __syncthreads();
    lds_line_dft<true>(lds, L, nl, m, 1, g.tables);
    store_row_spectra(lds, P, g.spec + P.spec_base, y0, nl, m, fa, true);
}

// Fifteen products of the five spectra at one k, in FP64.
__device__ __forceinline__ void products_k(double (&val)[kKinds], const float2 (&X)[5])
{
    double re[5], im[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        re[f] = X[f].x;
        im[f] = X[f].y;
    }
    // a b* = (ar br + ai bi) + i (ai br - ar bi)
#define FLB_RE(u, v) (re[u] * re[v] + im[u] * im[v])
#define FLB_IM(u, v) (im[u] * re[v] - re[u] * im[v])
    const double p[kKinds] = {FLB_RE(0, 0), FLB_RE(1, 1), FLB_RE(2, 2), FLB_RE(3, 3),
                              FLB_RE(4, 4), FLB_RE(3, 4), FLB_IM(3, 4), FLB_RE(0, 1),
                              FLB_IM(0, 1), FLB_RE(0, 2), FLB_IM(0, 2), FLB_RE(0, 3),
                              FLB_IM(0, 3), FLB_RE(0, 4), FLB_IM(0, 4)};
#undef FLB_RE
#undef FLB_IM
#pragma unroll
    for (int q = 0; q < kKinds; ++q) val[q] = p[q];
}

// One read-modify-write of NK FP64 sums at one k (stride kstride): every
// old value is read before any is written, so the reads are in flight
// together (read and write addresses are the same, so the compiler may not
// reorder a later read before an earlier write on its own).
template <int NK, bool NT = false>
__device__ __forceinline__ void add_to_sums(double *a, int64_t kstride, const double (&u)[NK])
{
    double old[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q) old[q] = gload<NT>(&a[q * kstride]);
#pragma unroll
    for (int q = 0; q < NK; ++q) gstore<NT>(&a[q * kstride], old[q] + u[q]);
}

// Adds the products of one sample at one k to the sums.
__device__ __forceinline__ void accumulate_k(double *a, int64_t kstride, const float2 (&X)[5])
{
    double val[kKinds];
    products_k(val, X);
    add_to_sums(a, kstride, val);
}

// Stash slots read per batch: the slots of a cycle are whole batches, each
// with all its reads in flight at once.
constexpr int kSlotBatch = 4;
static_assert(kDeferK % kSlotBatch == 0, "whole batches per cycle");

// The products of the n >= 1 stashed samples at st (field f of slot j at
// st + (5 j + f) * fs), summed in slot order and added to the sums (kind q
// at a + q * kstride) in one read-modify-write; stash and sums are streamed
// (each is read once per cycle, far more than the L2 holds).
__device__ __forceinline__ void accumulate_stashed_k(double *a, int64_t kstride, const float2 *st,
                                                     int64_t fs, int n)
{
    double u[kKinds];
#pragma unroll
    for (int q = 0; q < kKinds; ++q) u[q] = 0.0;
    for (int j0 = 0; j0 < n; j0 += kSlotBatch) {
        // slots past the last are read again (in bounds) and not added
        float2 Y[kSlotBatch][5];
#pragma unroll
        for (int b = 0; b < kSlotBatch; ++b) {
            const int j = min(j0 + b, n - 1);
#pragma unroll
            for (int f = 0; f < 5; ++f) Y[b][f] = stream_load(&st[(j * 5 + f) * fs]);
        }
        // (a select, not a branch: the reads of a batch must not be sunk
        // into per-slot branches, which would serialise them again)
#pragma unroll
        for (int b = 0; b < kSlotBatch; ++b) {
            const bool on = j0 + b < n;
            double w[kKinds];
            products_k(w, Y[b]);
#pragma unroll
            for (int q = 0; q < kKinds; ++q) u[q] += on ? w[q] : 0.0;
        }
    }
    add_to_sums<kKinds, true>(a, kstride, u);
}

// Squared moduli of the six moment spectra at one k, added to kinds
// kKinds .. kKinds + 5.
__device__ __forceinline__ void accumulate_moments_k(double *a, int64_t kstride,
                                                     const float2 (&X)[6])
{
    double u[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const double re = X[f].x, im = X[f].y;
        u[f] = re * re + im * im;
    }
    add_to_sums<6>(a + kKinds * kstride, kstride, u);
}

template <int SET, int NF>
__device__ __forceinline__ void accumulate_set(double *a, int64_t kstride, const float2 (&X)[NF])
{
    if constexpr (SET == 0)
        accumulate_k(a, kstride, X);
    else
        accumulate_moments_k(a, kstride, X);
}

// Column transforms, whole columns in LDS: Bluestein's convolution for
// lengths that are not powers of two, the plain transform otherwise.  item:
// lattice, field, first column, log2 of the columns per block (at most 16,
// so that a block's lines take at most kColsElems LDS elements, or
// kColsLargeElems in the large blocks of NT = kColsLargeThreads threads that
// power-of-two lengths from 1024 on take).  LDS [j][c], padded (the small-stride
// passes of a few interleaved lines would otherwise share banks).  The
// transforms fuse four radix-2 stages per pass, sixteen elements per thread:
// the registers that takes are free at the occupancy the LDS allows.  A
// Bluestein line's output chirp is applied as the result is stored.
// Whole 4096-point columns in blocks of four (1024 threads, one block per
// CU) against a two-pass split into 64 x 64 points (16 columns per pass, an
// HBM round trip of the spectra between the passes), 4096^2 whole path:
// 87.3 against 83.4 GLUPS; in blocks of two (512 threads): 80.0.
template <int NT>
__global__ __launch_bounds__(NT) void corr_cols_kernel(CorrArgs g)
{
    extern __shared__ float2 lds[];
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_y];
    const int ny = P.ny, nkx = P.nkx, kxp = P.kxp;
    const int f = it.a, c0 = it.b, lgc = it.c, cb = 1 << lgc;
    const int ncol = min(cb, nkx - c0);
    const float2 *col = g.spec + P.spec_base + (int64_t)f * ny * kxp;
    // the transformed column goes back in place (row order), or to stash
    // slot g.arg >= 0
    const bool tiled = g.arg >= 0;
    float2 *out = g.spec + P.spec_base + (int64_t)f * ny * kxp;
    const int64_t plane = (int64_t)ny * kxp;
    const float2 *chirp = g.tables + L.chirp_off;
    const bool blue = L.bluestein != 0;
    // a Bluestein work length's zero padding, rows ny .. m-1
    for (int idx = ny * cb + (int)threadIdx.x; idx < L.m * cb; idx += NT)
        lds[lds_slot<true>(idx)] = make_float2(0.f, 0.f);
    const int ne = ny * cb;
    for (int i0 = threadIdx.x; i0 < ne; i0 += kBatch * NT) {
        float2 v[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int idx = i0 + b * NT, j = idx >> lgc, c = idx & (cb - 1);
            v[b] = make_float2(0.f, 0.f);
            if (idx < ne && c < ncol) v[b] = col[(int64_t)j * kxp + c0 + c];
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int idx = i0 + b * NT, j = idx >> lgc, c = idx & (cb - 1);
            if (idx >= ne) continue;
            if (blue) lds[lds_slot<true>(idx)] = cmul(v[b], chirp[j]);
            else lds[lds_slot<true>((bitrev(j, L.log2m) << lgc) + c)] = v[b];
        }
    }
    __syncthreads();
    if (blue) lds_bluestein_dft<true, false, 4>(lds, L, cb, 1, cb, g.tables);
    else lds_fft_dit<true, false, 4>(lds, L.log2m, cb, 1, cb, g.tables);
    for (int idx = threadIdx.x; idx < ne; idx += NT) {
        const int j = idx >> lgc, c = idx & (cb - 1);
        if (c >= ncol) continue;
        const float2 x = lds[lds_slot<true>(idx)];
        const float2 y = blue ? cmul(x, chirp[j]) : x;
        if (tiled)
            stream_store(&g.stash[stash_offset(P.spec_base, plane, spec_offset(j, c0 + c, ny),
                                               g.arg, f)], y);
        else
            out[(int64_t)j * kxp + c0 + c] = y;
    }
}

// Column transforms of power-of-two lengths N = 2^LG, 512 <= N <= 4096, in
// persistent blocks of NT threads.  A group is CB = 16384 / N (at most 16)
// adjacent columns of one field of one lattice (item: lattice, field, first
// column, log2 CB); each block works through the groups the host scheduled
// for it (sched[it * gridDim.x + blockIdx.x], it < niter, lattice -1 =
// none), and issues the global loads of its next group as soon as the
// current one has left its registers, so that they run under the current
// group's LDS passes and stores.
// The transform is the in-place decimation in time of lds_fft_dit with
// passes of R1, R2, R3 fused radix-2 stages, but its first pass works on the
// registers the global loads fill (first-pass group g of a column holds rows
// bitrev(g) + r N / 2^R1 at position bitrev(r), the bit-reversed input
// order) and its last pass stores the natural-order result straight to
// global memory, so only the middle pass reads and writes LDS in between.
// LDS [element][column] interleaved, padded as the other column layouts.
// 1024 to 4096 points take 512 threads, each with two groups per pass:
// with 1024 threads a radix-16 pass alone fills the 128 registers a thread
// may hold, and the prefetched group did not fit beside it.

// bit reversal of r < 2^bits at compile time (register array indices)
__host__ __device__ constexpr int rev_bits(int r, int bits)
{
    int o = 0;
    for (int b = 0; b < bits; ++b) o |= ((r >> b) & 1) << (bits - 1 - b);
    return o;
}

// a[0] <- a[1] <- ... <- a[n-1] <- a[0]: a register array cycled with
// static indices only
template <int NA> __device__ __forceinline__ void rotate_left(float2 (&a)[NA])
{
    const float2 t = a[0];
#pragma unroll
    for (int i = 0; i + 1 < NA; ++i) a[i] = a[i + 1];
    a[NA - 1] = t;
}

__host__ __device__ constexpr int cols_pipe_threads(int lg) { return lg >= 10 ? 512 : 1024; }

template <int LG, int R1, int R2, int R3>
__global__ __launch_bounds__(cols_pipe_threads(LG)) void corr_cols_pipe_kernel(
    CorrArgs g, const PipeItem *__restrict__ sched, int niter)
{
    static_assert(R1 + R2 + R3 == LG && R1 <= 4 && R2 <= 4 && R3 <= 4, "pass plan");
    constexpr int NT = cols_pipe_threads(LG);
    constexpr int N = 1 << LG;
    constexpr int G1 = 1 << R1, G2 = 1 << R2, G3 = 1 << R3;
    constexpr int CB = (16384 >> LG) < 16 ? (16384 >> LG) : 16;  // columns per group
    constexpr int LGC = (CB == 16) ? 4 : (CB == 8) ? 3 : (CB == 4) ? 2 : (CB == 2) ? 1 : 0;
    static_assert((1 << LGC) == CB, "columns per group");
    // groups of the first, middle and last pass per thread
    constexpr int NG1 = (CB << (LG - R1)) / NT, NG2 = (CB << (LG - R2)) / NT;
    constexpr int NG3 = (CB << (LG - R3)) / NT;
    static_assert(NG1 >= 1 && NG1 * NT == (CB << (LG - R1)) && NG2 * NT == (CB << (LG - R2)) &&
                  NG3 * NT == (CB << (LG - R3)) && NT % CB == 0, "passes");
    constexpr int S2 = R1 + 1, H2 = 1 << (S2 - 1);  // the middle pass's first stage, distance
    constexpr int H3 = N >> R3;                     // element distance of the last pass
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int c = tid & (CB - 1);                   // this thread's column in its group

    // The twiddles of the middle and last passes depend on the thread alone:
    // read once, before any load whose completion the loop waits for (the
    // vector memory counter is in order, so a twiddle read behind the
    // prefetched loads would wait for them).
    float2 tw2[NG2], tw3[NG3];
#pragma unroll
    for (int i = 0; i < NG2; ++i)
        tw2[i] = g.tables[((tid + i * NT) >> LGC & (H2 - 1)) << (kTwLog - (S2 + R2 - 1))];
#pragma unroll
    for (int i = 0; i < NG3; ++i) tw3[i] = g.tables[((tid + i * NT) >> LGC) << (kTwLog - LG)];
    // vmcnt(0), other counters untouched: the twiddles have arrived before
    // the first prefetch is issued, so no wait inside the loop is held up by
    // them (otherwise the wait analysis, not telling the first iteration
    // from later ones, orders them behind the prefetched loads)
    __builtin_amdgcn_s_waitcnt(0x0F70);

    float2 v[NG1][G1];
    // global loads of rows r0 .. r1-1 (of the G1 of each first-pass group the
    // thread takes) of one group of columns into v, bit-reversed order within
    // a first-pass group; a wave-uniform base and 32-bit offsets (a field's
    // spectra are far below 2^32 elements).  Threads past the group's last
    // column read that column again and store nothing.
    auto load = [&](const PipeItem &it, auto r0, auto r1) {
        const float2 *col = g.spec + it.off;
        const uint32_t kxp = (uint32_t)it.kxp, cl = (uint32_t)min(c, it.ncol - 1);
#pragma unroll
        for (int q = 0; q < NG1; ++q) {
            const int g1 = (tid + q * NT) >> LGC;
            const uint32_t o0 = (uint32_t)bitrev(g1, LG - R1) * kxp + cl;
#pragma unroll
            for (int r = decltype(r0)::value; r < decltype(r1)::value; ++r)
                v[q][rev_bits(r, R1)] = col[o0 + ((uint32_t)r << (LG - R1)) * kxp];
        }
    };
    using Zero = std::integral_constant<int, 0>;
    using Half = std::integral_constant<int, G1 / 2>;
    using All = std::integral_constant<int, G1>;

    PipeItem cur = sched[blockIdx.x];
    if (cur.ncol <= 0) return;
    load(cur, Zero{}, All{});
    for (int it = 0;; ++it) {
        __syncthreads();  // the previous item's last pass has read LDS
        // first pass: stages 1 .. R1 (h = 1, so every twiddle is a fixed root)
#pragma unroll
        for (int q = 0; q < NG1; ++q) {
            const int g1 = (tid + q * NT) >> LGC;
            group_butterflies<R1, false, false, true>(v[q], make_float2(1.f, 0.f));
#pragma unroll
            for (int j = 0; j < G1; ++j) lds[lds_slot<true>((((g1 << R1) + j) << LGC) + c)] = v[q][j];
        }
        const PipeItem next = it + 1 < niter ? sched[(it + 1) * gridDim.x + blockIdx.x]
                                             : PipeItem{0, 0, 0};
        // the next item's loads, half before the middle pass and half after
        // it
        if (next.ncol > 0) load(next, Zero{}, Half{});
        __syncthreads();
        // middle pass: stages S2 .. S2 + R2 - 1, as fused_pass on the
        // interleaved layout
        // (one group at a time: interleaving two would need twice the
        // registers; the twiddles rotate so that the one in use is tw2[0])
#pragma unroll 1
        for (int i = 0; i < NG2; ++i) {
            const int idx = tid + i * NT, gg = idx >> LGC, l = idx & (CB - 1);
            const int k = gg & (H2 - 1);
            const int e0 = ((((gg >> (S2 - 1)) << (S2 - 1 + R2)) + k) << LGC) + l;
            float2 x[G2];
#pragma unroll
            for (int j = 0; j < G2; ++j) x[j] = lds[lds_slot<true>(e0 + ((j * H2) << LGC))];
            group_butterflies<R2, false, false>(x, tw2[0]);
#pragma unroll
            for (int j = 0; j < G2; ++j) lds[lds_slot<true>(e0 + ((j * H2) << LGC))] = x[j];
            rotate_left(tw2);
        }
        if (next.ncol > 0) load(next, Half{}, All{});
        __syncthreads();
        // last pass: stages LG - R3 + 1 .. LG, groups k < H3 of elements
        // k + j H3, which are in natural order when they leave it
        {
            // in place (row order), or to a stash slot (column-tiled: rows
            // of a tile kTileCols apart, positions placed by stash_offset)
            static_assert(kTileCols == 4, "tile offsets below");
            const bool tiled = g.arg >= 0;
            float2 *out = g.spec + cur.off;
            const uint32_t rs = tiled ? 4u : (uint32_t)cur.kxp;
            const uint32_t ts = (uint32_t)cur.ts;
#pragma unroll 1
            for (int i = 0; i < NG3; ++i) {
                const int idx = tid + i * NT, k = idx >> LGC, cc = idx & (CB - 1);
                float2 x[G3];
#pragma unroll
                for (int j = 0; j < G3; ++j) x[j] = lds[lds_slot<true>(((k + j * H3) << LGC) + cc)];
                group_butterflies<R3, false, false>(x, tw3[0]);
                rotate_left(tw3);
                if (cc < cur.ncol) {
                    const uint32_t o0 = (uint32_t)k * rs + (tiled ? ((uint32_t)cc >> 2) * ts + (cc & 3)
                                                                   : (uint32_t)cc);
#pragma unroll
                    for (int j = 0; j < G3; ++j) {
                        const uint32_t o = o0 + (uint32_t)(j * H3) * rs;
                        if (tiled)
                            stream_store(&g.stash[stash_offset(cur.sbase, cur.plane,
                                                               (int64_t)cur.o0 + o, g.arg, cur.f)],
                                         x[j]);
                        else
                            out[o] = x[j];
                    }
                }
            }
        }
        if (next.ncol <= 0) break;
        cur = next;
    }
}

// Accumulation.  item: lattice, first k of the (ny, nkx) plane.
// Bluestein column transforms with the work length 2^LG = 256 .. 2048 fixed
// at compile time: a block takes CB = 8192 / 2^LG columns of one field
// (8192 complex values of LDS, two blocks per compute unit), interleaved in
// LDS as the generic column kernel has them (element e of column c at
// e * CB + c).  One pass of R radix-2 stages S0 .. S0+R-1 over all of them:
template <int LG, int S0, int R, bool INV = false, bool DIF = false>
__device__ __forceinline__ void col_fft_pass(float2 *buf, const float2 *tw, int tid)
{
    constexpr int LGC = 13 - LG, G = 1 << R, H = 1 << (S0 - 1);
    constexpr int PER = (8192 >> R) / kFftThreads;  // groups per thread
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * kFftThreads;
        const int l = idx & ((1 << LGC) - 1), gg = idx >> LGC;
        const int k = gg & (H - 1);
        const int e0 = ((gg >> (S0 - 1)) << (S0 - 1 + R)) + k;
        float2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = buf[lds_slot<true>(((e0 + j * H) << LGC) + l)];
        if constexpr (S0 == 1) {
            group_butterflies<R, INV, DIF, true>(v, make_float2(1.f, 0.f));
        } else {
            float2 w = tw[k << (kTwLog - (S0 + R - 1))];
            if (INV) w.y = -w.y;
            group_butterflies<R, INV, DIF>(v, w);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) buf[lds_slot<true>(((e0 + j * H) << LGC) + l)] = v[j];
    }
}

// ... the last forward stages R .. 1, the product with the chirp kernel's
// transform (bit-reversed order) and the first inverse stages 1 .. R on
// groups of 2^R consecutive elements of a column (as row_blue_middle):
template <int LG, int R>
__device__ __forceinline__ void col_blue_middle(float2 *buf, const float2 *kern, int tid)
{
    constexpr int LGC = 13 - LG, G = 1 << R, PER = (8192 >> R) / kFftThreads;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * kFftThreads;
        const int l = idx & ((1 << LGC) - 1), e0 = (idx >> LGC) << R;
        float2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = buf[lds_slot<true>(((e0 + j) << LGC) + l)];
        group_butterflies<R, false, true, true>(v, make_float2(1.f, 0.f));
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = cmul(v[j], kern[e0 + j]);
        group_butterflies<R, true, false, true>(v, make_float2(1.f, 0.f));
#pragma unroll
        for (int j = 0; j < G; ++j) buf[lds_slot<true>(((e0 + j) << LGC) + l)] = v[j];
    }
}

// ... and the block: what corr_cols_kernel computes for such columns.  Each
// thread reads the column elements e = k + j 2^LG/16 (j < 16) of its column,
// one group of the forward transform's first radix-16 pass (decimation in
// frequency, natural order); as 2^LG >= 2 ny - 1 only j < 8 can hold rows,
// and that pass runs in registers on the loaded, chirp-multiplied values.
// The inverse transform's last radix-16 pass leaves the elements in natural
// order and stores them (times the output chirp) from registers.  LDS
// round trips per block: 4 (2^11, 2^10, 2^9) or 2 (2^8).
template <int LG>
__device__ __forceinline__ void cols_blue_block(const CorrArgs &g, const CorrItem &it)
{
    constexpr int M = 1 << LG, LGC = 13 - LG, CB = 1 << LGC, H = M >> 4;
    static_assert(LG >= 8 && LG <= 11, "work lengths 256 .. 2048");
    extern __shared__ float2 lds[];
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_y];
    const int ny = P.ny, nkx = P.nkx, kxp = P.kxp;
    const int f = it.a, c0 = it.b;
    const int ncol = min(CB, nkx - c0);
    const int tid = (int)threadIdx.x, c = tid & (CB - 1), k = tid >> LGC;
    const float2 *chirp = g.tables + L.chirp_off;
    const float2 *tw = g.tables;
    const float2 *col = g.spec + P.spec_base + (int64_t)f * ny * kxp + c0 + min(c, ncol - 1);

    float2 v[16];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int e = k + j * H;
        v[j] = e < ny ? col[(int64_t)e * kxp] : make_float2(0.f, 0.f);
        v[j + 8] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int e = k + j * H;
        v[j] = cmul(v[j], chirp[e < ny ? e : 0]);
    }
    // forward stages LG .. LG-3 (decimation in frequency), twiddle
    // exp(-2 pi i k / 2^LG)
    group_butterflies<4, false, true>(v, tw[k << (kTwLog - LG)]);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds[lds_slot<true>(((k + j * H) << LGC) + c)] = v[j];
    __syncthreads();
    const float2 *kern = g.tables + L.kernel_off;
    if constexpr (LG == 11) {
        col_fft_pass<LG, 5, 3, false, true>(lds, tw, tid);
        __syncthreads();
        col_blue_middle<LG, 4>(lds, kern, tid);
        __syncthreads();
        col_fft_pass<LG, 5, 3, true>(lds, tw, tid);
    } else if constexpr (LG == 10) {
        col_fft_pass<LG, 4, 3, false, true>(lds, tw, tid);
        __syncthreads();
        col_blue_middle<LG, 3>(lds, kern, tid);
        __syncthreads();
        col_fft_pass<LG, 4, 3, true>(lds, tw, tid);
    } else if constexpr (LG == 9) {
        col_fft_pass<LG, 3, 3, false, true>(lds, tw, tid);
        __syncthreads();
        col_blue_middle<LG, 2>(lds, kern, tid);
        __syncthreads();
        col_fft_pass<LG, 3, 3, true>(lds, tw, tid);
    } else {
        col_blue_middle<LG, 4>(lds, kern, tid);
    }
    __syncthreads();
    // inverse stages LG-3 .. LG: groups k of elements k + j 2^LG/16, natural
    // order when they leave; rows e < ny are kept (e < 2^LG/2: j < 8)
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds[lds_slot<true>(((k + j * H) << LGC) + c)];
    float2 w = tw[k << (kTwLog - LG)];
    w.y = -w.y;
    group_butterflies<4, true, false>(v, w);
    if (c >= ncol) return;
    // the transformed column goes back in place, or to stash slot g.arg >= 0
    const bool tiled = g.arg >= 0;
    float2 *out = g.spec + P.spec_base + (int64_t)f * ny * kxp;
    const int64_t plane = (int64_t)ny * kxp;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int e = k + j * H;
        if (e >= ny) break;
        const float2 y = cmul(v[j], chirp[e]);
        if (tiled)
            stream_store(&g.stash[stash_offset(P.spec_base, plane, spec_offset(e, c0 + c, ny),
                                               g.arg, f)], y);
        else
            out[(int64_t)e * kxp + c0 + c] = y;
    }
}

// All Bluestein columns of work length 2^8 .. 2^11 (corr_cols_blue_supported)
// in one launch, each block taking the code of its lattice's plan.
__global__ __launch_bounds__(kFftThreads, 4) void corr_cols_blue_kernel(CorrArgs g)
{
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    switch (g.plans[g.params[it.lattice].line_y].log2m) {
    case 8: cols_blue_block<8>(g, it); break;
    case 9: cols_blue_block<9>(g, it); break;
    case 10: cols_blue_block<10>(g, it); break;
    case 11: cols_blue_block<11>(g, it); break;
    default: break;
    }
}

// Row and column (ky, kx) of position o of a column-tiled plane; whether it
// holds a k that is accumulated: not a padding column (kx >= nkx), not k = 0
// (which carries no fluctuation).
__device__ __forceinline__ bool tiled_k(const LatticeParams &P, uint32_t o, uint32_t &ky,
                                        uint32_t &kx)
{
    const uint32_t q = o / kTileCols, tile = q / (uint32_t)P.ny;
    ky = q - tile * (uint32_t)P.ny;
    kx = tile * kTileCols + o % kTileCols;
    return kx < (uint32_t)P.nkx && (kx | ky) != 0;
}

template <int SET>
__global__ __launch_bounds__(kThreads) void corr_accum_kernel(CorrArgs g)
{
    constexpr int NF = SET ? 6 : 5;
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int64_t fstride = (int64_t)P.ny * P.kxp;
    const int64_t o = (int64_t)it.a + threadIdx.x;  // position in a tiled sum plane
    uint32_t ky, kx;
    if (o >= fstride || !tiled_k(P, (uint32_t)o, ky, kx)) return;
    // this sample's spectra, in place in row order
    const float2 *sp = g.spec + P.spec_base + (int64_t)ky * P.kxp + kx;
    float2 X[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) X[f] = sp[f * fstride];
    accumulate_set<SET, NF>(g.acc + P.acc_base + o, fstride, X);
}

// Reads a sample's stashed spectra back: the products of the first g.arg
// stash slots added to the sums (the layout and items of
// corr_accum_kernel<0>).
__global__ __launch_bounds__(kThreads) void corr_flush_kernel(CorrArgs g)
{
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int64_t fstride = (int64_t)P.ny * P.kxp;
    const int64_t o = (int64_t)it.a + threadIdx.x;  // tiled stash and sum planes
    uint32_t ky, kx;
    if (o >= fstride || !tiled_k(P, (uint32_t)o, ky, kx)) return;
    // this position's chunk of the stash: every slot and field in turn,
    // chunk-wide apart
    const int64_t c = o / kStashChunk, left = fstride - c * kStashChunk;
    const int64_t w = left < kStashChunk ? left : kStashChunk;
    accumulate_stashed_k(g.acc + P.acc_base + o, fstride,
                         g.stash + stash_offset(P.spec_base, fstride, o, 0, 0), w, g.arg);
}

static CorrArgs make_args(const DeviceView &v, const CorrItem *items, int set)
{
    CorrArgs g;
    g.pops = v.pops[v.cur];
    g.params = v.params;
    g.plans = v.plans;
    g.tables = v.tables;
    g.items = items;
    g.spec = v.spec;
    g.stash = v.stash;
    g.arg = 0;
    g.acc = v.acc;
    g.fields = v.fields;
    g.csum_part = v.csum_part;
    g.csum = v.csum;
    g.set = set;
    return g;
}

template <bool BLUE>
static void rows_for(const DeviceView &v, const CorrArgs &g, int nitems, int lds_bytes,
                     hipStream_t s)
{
    const dim3 grid(nitems), block(kFftThreads);
    if (v.storage == kF32)
        hipLaunchKernelGGL((corr_rows_kernel<kF32, BLUE>), grid, block, lds_bytes, s, g);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL((corr_rows_kernel<kBF16, BLUE>), grid, block, lds_bytes, s, g);
    else
        hipLaunchKernelGGL((corr_rows_kernel<kF16, BLUE>), grid, block, lds_bytes, s, g);
}

bool corr_rows_p2_supported(int lg) { return lg >= 9 && lg <= 12; }
bool corr_rows_blue_supported(int lg) { return lg >= 8 && lg <= 11; }

template <int LG>
static void rows_p2_for(const DeviceView &v, const CorrArgs &g, int nitems, int lds_bytes,
                        hipStream_t s)
{
    const dim3 grid(nitems), block(kFftThreads);
    if (v.storage == kF32)
        hipLaunchKernelGGL((corr_rows_p2_kernel<kF32, LG>), grid, block, lds_bytes, s, g);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL((corr_rows_p2_kernel<kBF16, LG>), grid, block, lds_bytes, s, g);
    else
        hipLaunchKernelGGL((corr_rows_p2_kernel<kF16, LG>), grid, block, lds_bytes, s, g);
}

hipError_t launch_corr_rows(const DeviceView &v, const CorrItem *items, int nitems,
                            const RowLaunch *fixed, int nfixed, const CorrItem *blue_items,
                            int nblue, int lds_bytes, hipStream_t s)
{
    // the length-specialised blocks first (Bluestein, the most expensive,
    // ahead of the power-of-two lengths)
    for (int q = 0; q < nfixed; ++q) {
        const CorrArgs g = make_args(v, items + fixed[q].off, 0);
        const dim3 grid(fixed[q].n), block(kFftThreads);
        switch (fixed[q].lg) {
        case 0:  // every Bluestein work length of corr_rows_blue_supported
            if (v.storage == kF32)
                hipLaunchKernelGGL(corr_rows_blue_kernel<kF32>, grid, block, lds_bytes, s, g);
            else if (v.storage == kBF16)
                hipLaunchKernelGGL(corr_rows_blue_kernel<kBF16>, grid, block, lds_bytes, s, g);
            else
                hipLaunchKernelGGL(corr_rows_blue_kernel<kF16>, grid, block, lds_bytes, s, g);
            break;
        case 9: rows_p2_for<9>(v, g, fixed[q].n, lds_bytes, s); break;
        case 10: rows_p2_for<10>(v, g, fixed[q].n, lds_bytes, s); break;
        case 11: rows_p2_for<11>(v, g, fixed[q].n, lds_bytes, s); break;
        case 12: rows_p2_for<12>(v, g, fixed[q].n, lds_bytes, s); break;
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nitems) {
        rows_for<false>(v, make_args(v, items, 0), nitems, lds_bytes, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nblue) {
        rows_for<true>(v, make_args(v, blue_items, 0), nblue, lds_bytes, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_corr_csum(const DeviceView &v, hipStream_t s)
{
    const CorrArgs g = make_args(v, nullptr, 0);
    hipLaunchKernelGGL(corr_csum_kernel, dim3(v.nlat), dim3(kThreads), 0, s, g, v.nlat);
    return hipGetLastError();
}

hipError_t launch_corr_moment_fields(const DeviceView &v, const CorrItem *items, int nitems,
                                     hipStream_t s)
{
    const CorrArgs g = make_args(v, items, 1);
    const dim3 grid(nitems), block(kThreads);
    if (v.storage == kF32)
        hipLaunchKernelGGL(corr_moment_fields_kernel<kF32>, grid, block, 0, s, g);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(corr_moment_fields_kernel<kBF16>, grid, block, 0, s, g);
    else
        hipLaunchKernelGGL(corr_moment_fields_kernel<kF16>, grid, block, 0, s, g);
    return hipGetLastError();
}

hipError_t launch_corr_moment_rows(const DeviceView &v, const CorrItem *items, int nitems,
                                   int lds_bytes, hipStream_t s)
{
    const CorrArgs g = make_args(v, items, 1);
    hipLaunchKernelGGL(corr_moment_rows_kernel, dim3(nitems), dim3(kFftThreads), lds_bytes, s,
                       g);
    return hipGetLastError();
}

hipError_t launch_corr_flush(const DeviceView &v, const CorrItem *items, int nitems, int nslots,
                             hipStream_t s)
{
    CorrArgs g = make_args(v, items, 0);
    g.arg = nslots;
    hipLaunchKernelGGL(corr_flush_kernel, dim3(nitems), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

bool corr_cols_blue_supported(int lg) { return lg >= 8 && lg <= 11; }
int corr_cols_blue_lds_bytes() { return lds_padded_elems(8192) * (int)sizeof(float2); }

hipError_t launch_corr_cols_blue(const DeviceView &v, const CorrItem *items, int nitems, int slot,
                                 hipStream_t s)
{
    CorrArgs g = make_args(v, items, 0);
    g.arg = slot;
    hipLaunchKernelGGL(corr_cols_blue_kernel, dim3(nitems), dim3(kFftThreads),
                       corr_cols_blue_lds_bytes(), s, g);
    return hipGetLastError();
}

hipError_t launch_corr_cols(const DeviceView &v, const CorrItem *items, int nitems, int slot,
                            bool large, int lds_bytes, hipStream_t s)
{
    CorrArgs g = make_args(v, items, 0);
    g.arg = slot;
    if (large)
        hipLaunchKernelGGL(corr_cols_kernel<kColsLargeThreads>, dim3(nitems),
                           dim3(kColsLargeThreads), lds_bytes, s, g);
    else
        hipLaunchKernelGGL(corr_cols_kernel<kFftThreads>, dim3(nitems), dim3(kFftThreads),
                           lds_bytes, s, g);
    return hipGetLastError();
}

bool corr_cols_pipe_supported(int lg) { return lg >= 9 && lg <= 12; }

int corr_cols_pipe_lds_bytes(int lg)
{
    const int n = 1 << lg, cb = std::min(16, 16384 / n);
    return (lds_slot<true>(n * cb - 1) + 1) * (int)sizeof(float2);
}

hipError_t launch_corr_cols_pipe(const DeviceView &v, const PipeItem *sched, int niter, int grid,
                                 int lg, int slot, hipStream_t s)
{
    CorrArgs g = make_args(v, nullptr, 0);
    g.arg = slot;
    const int lds = corr_cols_pipe_lds_bytes(lg);
    const dim3 gr(grid), bl(cols_pipe_threads(lg));
    switch (lg) {
    case 9:
        hipLaunchKernelGGL((corr_cols_pipe_kernel<9, 3, 3, 3>), gr, bl, lds, s, g, sched, niter);
        break;
    case 10:
        hipLaunchKernelGGL((corr_cols_pipe_kernel<10, 4, 3, 3>), gr, bl, lds, s, g, sched, niter);
        break;
    case 11:
        hipLaunchKernelGGL((corr_cols_pipe_kernel<11, 4, 4, 3>), gr, bl, lds, s, g, sched, niter);
        break;
    case 12:
        hipLaunchKernelGGL((corr_cols_pipe_kernel<12, 4, 4, 4>), gr, bl, lds, s, g, sched, niter);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_corr_accum(const DeviceView &v, const CorrItem *items, int nitems, int set,
                             hipStream_t s)
{
    CorrArgs g = make_args(v, items, set);
    if (set == 1)
        hipLaunchKernelGGL(corr_accum_kernel<1>, dim3(nitems), dim3(kThreads), 0, s, g);
    else
        hipLaunchKernelGGL(corr_accum_kernel<0>, dim3(nitems), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

}  // namespace flbdev
