// flb_dq.hip -- the fluctuating lattice Boltzmann step and its structure
// factors on the velocity sets of flb_dq.h (D1Q3, D2Q9, D3Q15), and their
// C ABI.
//
// One step per site (Sec. 2): pull f_i(x) = f*_i(x - v_i) (Eq. 1), moments
// of the FP32 deviations (Eq. 3), equilibrium stress moments of Eq. (2)
// (the ghost equilibria vanish), relaxation of every non-conserved moment
// with its own rate and noise of amplitude Eq. (8) (Eq. 5), and the change
// of the non-conserved moments back-transformed with n_i^a = w_i m_i^a
// (Eq. 4).  What the FP32 tables let leak into mass and momentum is
// projected out (zero in exact arithmetic), so both stay conserved.
//
// The equilibrium moment of a stress mode a is the projection of Eq. (2):
//   M^{a,0} = 4.5 rho sum_ab T^a_ab u_a u_b,  T^a_ab = sum_i w_i m_i^a v_ia v_ib,
// since the stress rows are orthogonal to 1 and v.
//
// Correlators per sample: an FP32 field kernel (rho, j, u, the non-conserved
// moments), packed real-pair line transforms along x into half spectra,
// strided line transforms along y and z in place, and an FP64 accumulation of
// the kinds of flb_dq.h.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/flb.h"
#include "../../include/flb_dq.h"
#include "flb_fft.h"

namespace flbdev {

constexpr int kDqMaxQ = FLB_DQ_MAXQ;
constexpr int kDqThreads = 256;

// Velocity sets in the order of flb_dq.h.
template <int MODEL> struct DqSet;
template <> struct DqSet<FLB_DQ_D1Q3> {
    static constexpr int D = 1, Q = 3;
    static constexpr int v[3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
};
template <> struct DqSet<FLB_DQ_D2Q9> {
    static constexpr int D = 2, Q = 9;
    static constexpr int v[9][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},  {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0}};
};
template <> struct DqSet<FLB_DQ_D3Q15> {
    static constexpr int D = 3, Q = 15;
    static constexpr int v[15][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},   {0, 1, 0},
                                     {0, -1, 0},  {0, 0, 1},   {0, 0, -1},   {1, 1, 1},
                                     {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},  {1, 1, -1},
                                     {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
};

struct DqParams {
    int32_t n[3];
    int32_t tiles_x;            // blocks of kDqThreads sites along x
    uint32_t stream_id;
    float rho0;
    float u0[3];
    float m[kDqMaxQ][kDqMaxQ];  // m[a][i]
    float nw[kDqMaxQ][kDqMaxQ]; // w_i m_i^a, as nw[a][i]
    float w[kDqMaxQ];
    float T[6][3][3];           // stress tensors of the stress modes, in order
    float omega[kDqMaxQ];       // 1/tau^a
    float amp[kDqMaxQ];         // sigma_a (Eq. 8)
    float therm[kDqMaxQ];       // sqrt(mu rho0 w_i)
    int32_t nkx, kxp;           // half-space extent along x and its pitch
};

__device__ __forceinline__ int wrapi(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Site of a thread: tiles of kDqThreads sites along x, one row (y, z) per
// block row.  Returns false past the end of the row.
__device__ __forceinline__ bool dq_site(const DqParams &P, int &x, int &y, int &z)
{
    const int row = (int)(blockIdx.x / (uint32_t)P.tiles_x);
    const int tile = (int)blockIdx.x - row * P.tiles_x;
    x = tile * kDqThreads + (int)threadIdx.x;
    y = row % P.n[1];
    z = row / P.n[1];
    return x < P.n[0];
}

// Element `off` of a buffer through a 32-bit byte offset from a wave-uniform
// base (a buffer is below 4 GiB).
__device__ __forceinline__ const float *dq_at(const float *base, uint32_t off)
{
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off * 4u);
}
__device__ __forceinline__ float *dq_at(float *base, uint32_t off)
{
    return reinterpret_cast<float *>(reinterpret_cast<char *>(base) + off * 4u);
}

template <int MODEL, bool NT = false>
__device__ __forceinline__ void dq_pull(const float *__restrict__ src, const DqParams &P, int x, int y,
                                        int z, uint32_t V, float (&d)[DqSet<MODEL>::Q])
{
    using S = DqSet<MODEL>;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
        const int xs = S::v[i][0] ? wrapi(x - S::v[i][0], nx) : x;
        const int ys = S::v[i][1] ? wrapi(y - S::v[i][1], ny) : y;
        const int zs = S::v[i][2] ? wrapi(z - S::v[i][2], nz) : z;
        d[i] = gload<NT>(dq_at(src, (uint32_t)i * V + (uint32_t)xs +
                                        (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * (uint32_t)zs)));
    }
}

template <int MODEL>
__device__ __forceinline__ void dq_moments(const DqParams &P, const float (&d)[DqSet<MODEL>::Q],
                                           float (&M)[DqSet<MODEL>::Q])
{
    constexpr int Q = DqSet<MODEL>::Q;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) s = fmaf(P.m[a][i], d[i], s);
        M[a] = s;
    }
}

// NT: streaming (non-temporal) loads and stores, for buffers well beyond the
// last-level cache.
template <int MODEL, bool NOISE, bool NT>
__global__ __launch_bounds__(kDqThreads) void dq_step_kernel(const float *__restrict__ src,
                                                             float *__restrict__ dst,
                                                             const DqParams *__restrict__ Pp,
                                                             uint32_t t, uint32_t key0, uint32_t key1)
{
    using S = DqSet<MODEL>;
    constexpr int D = S::D, Q = S::Q, NM = Q - D - 1, NS = D * (D + 1) / 2;
    const DqParams &P = *Pp;
    int x, y, z;
    if (!dq_site(P, x, y, z)) return;
    const uint32_t V = (uint32_t)P.n[0] * (uint32_t)P.n[1] * (uint32_t)P.n[2];
    const uint32_t site = (uint32_t)x + (uint32_t)P.n[0] * ((uint32_t)y + (uint32_t)P.n[1] * (uint32_t)z);
    float d[Q], M[Q];
    dq_pull<MODEL, NT>(src, P, x, y, z, V, d);
    dq_moments<MODEL>(P, d, M);
    const float rho = P.rho0 + M[0];
    const float ir = 1.0f / rho;
    float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = M[1 + a] * 0.57735026918962576f * ir;
    float zn[6 * ((NM + 5) / 6)];
#pragma unroll
    for (int k = 0; k < 6 * ((NM + 5) / 6); ++k) zn[k] = 0.f;
    if constexpr (NOISE) {
#pragma unroll
        for (int dd = 0; dd < (NM + 5) / 6; ++dd)
            normals6(philox4x32_10(make_uint4(site, t, P.stream_id, (uint32_t)dd), key0, key1),
                     zn + 6 * dd);
    }
    float dM[Q];
#pragma unroll
    for (int a = D + 1; a < Q; ++a) {
        float eq = 0.f;
        if (a < D + 1 + NS) {
            const int s = a - D - 1;
            float q = 0.f;
#pragma unroll
            for (int al = 0; al < D; ++al)
#pragma unroll
                for (int be = 0; be < D; ++be) q = fmaf(P.T[s][al][be], u[al] * u[be], q);
            eq = 4.5f * rho * q;
        }
        dM[a] = fmaf(P.omega[a], eq - M[a], P.amp[a] * zn[a - D - 1]);
    }
    float inc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float s = 0.f;
#pragma unroll
        for (int a = D + 1; a < Q; ++a) s = fmaf(P.nw[a][i], dM[a], s);
        inc[i] = s;
    }
    // leakage into mass and momentum through the rounded tables
    float lr = 0.f, lj[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        lr += inc[i];
#pragma unroll
        for (int al = 0; al < D; ++al)
            if (S::v[i][al]) lj[al] += S::v[i][al] > 0 ? inc[i] : -inc[i];
    }
    const uint32_t out = site;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float c = lr;
#pragma unroll
        for (int al = 0; al < D; ++al)
            if (S::v[i][al]) c += S::v[i][al] > 0 ? 3.f * lj[al] : -3.f * lj[al];
        gstore<NT>(dq_at(dst, (uint32_t)i * V + out), d[i] + fmaf(-P.w[i], c, inc[i]));
    }
}

// Thermal start, first half: adds sqrt(mu rho0 w_i) z_i(x) to the value
// that streams into x (stored at x - v_i), with per-block FP64 sums of the
// additions per population.
template <int MODEL>
__global__ __launch_bounds__(kDqThreads) void dq_thermal_add_kernel(float *__restrict__ buf,
                                                                    const DqParams *__restrict__ Pp,
                                                                    uint32_t key0, uint32_t key1,
                                                                    double *__restrict__ part)
{
    using S = DqSet<MODEL>;
    constexpr int Q = S::Q;
    const DqParams &P = *Pp;
    __shared__ double red[Q][kDqThreads / 64];
    int x, y, z;
    const bool on = dq_site(P, x, y, z);
    double a[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) a[i] = 0.0;
    if (on) {
        const uint32_t V = (uint32_t)P.n[0] * (uint32_t)P.n[1] * (uint32_t)P.n[2];
        const uint32_t site =
            (uint32_t)x + (uint32_t)P.n[0] * ((uint32_t)y + (uint32_t)P.n[1] * (uint32_t)z);
        float zn[18];
#pragma unroll
        for (int dd = 0; dd < (Q + 5) / 6; ++dd)
            normals6(philox4x32_10(make_uint4(site, 0xFFFFFFFFu, P.stream_id, (uint32_t)dd), key0, key1),
                     zn + 6 * dd);
        const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int xs = S::v[i][0] ? wrapi(x - S::v[i][0], nx) : x;
            const int ys = S::v[i][1] ? wrapi(y - S::v[i][1], ny) : y;
            const int zs = S::v[i][2] ? wrapi(z - S::v[i][2], nz) : z;
            const float add = P.therm[i] * zn[i];
            float *p = buf + (uint32_t)i * V + (uint32_t)xs + (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * (uint32_t)zs);
            *p += add;
            a[i] = add;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double s = a[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if (lane == 0) red[i][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < Q) {
        double s = 0.0;
        for (int w = 0; w < kDqThreads / 64; ++w) s += red[threadIdx.x][w];
        part[(size_t)blockIdx.x * Q + threadIdx.x] = s;
    }
}

// Sums nparts rows of `width` doubles in a fixed order; out[c] = sum * scale.
__global__ __launch_bounds__(kDqThreads) void dq_reduce_kernel(const double *__restrict__ part,
                                                               int nparts, int width, double scale,
                                                               double *__restrict__ out)
{
    __shared__ double red[kDqThreads];
    for (int c = 0; c < width; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kDqThreads) s += part[(size_t)b * width + c];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = kDqThreads / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0] * scale;
        __syncthreads();
    }
}

// Thermal start, second half: each population's mean addition removed.
__global__ __launch_bounds__(kDqThreads) void dq_thermal_sub_kernel(float *__restrict__ buf, int Q,
                                                                    uint32_t V,
                                                                    const double *__restrict__ mean)
{
    const uint64_t e = (uint64_t)blockIdx.x * kDqThreads + threadIdx.x;
    if (e >= (uint64_t)Q * V) return;
    buf[e] -= (float)mean[e / V];
}

// FP64 per-block sums of mass and momentum deviations of the stored state
// (sums are unchanged by streaming).
template <int MODEL>
__global__ __launch_bounds__(kDqThreads) void dq_conservation_kernel(const float *__restrict__ buf,
                                                                     const DqParams *__restrict__ Pp,
                                                                     double *__restrict__ part)
{
    using S = DqSet<MODEL>;
    const DqParams &P = *Pp;
    __shared__ double red[4][kDqThreads / 64];
    int x, y, z;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (dq_site(P, x, y, z)) {
        const uint32_t V = (uint32_t)P.n[0] * (uint32_t)P.n[1] * (uint32_t)P.n[2];
        const uint32_t s = (uint32_t)x + (uint32_t)P.n[0] * ((uint32_t)y + (uint32_t)P.n[1] * (uint32_t)z);
#pragma unroll
        for (int i = 0; i < S::Q; ++i) {
            const double f = buf[(uint32_t)i * V + s];
            a[0] += f;
#pragma unroll
            for (int al = 0; al < S::D; ++al) a[1 + al] += S::v[i][al] * f;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double s = a[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if (lane == 0) red[q][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < kDqThreads / 64; ++w) s += red[threadIdx.x][w];
        part[(size_t)blockIdx.x * 4 + threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------
// Correlators
// ---------------------------------------------------------------------
// Fields of the current state as FP32 planes [nf][V]: d rho, d j_a (D),
// d u_a (D), the non-conserved moments; the constant references rho0,
// rho0 u0, u0 are subtracted instead of the spatial means (k = 0 is never
// accumulated).
template <int MODEL>
__global__ __launch_bounds__(kDqThreads) void dq_fields_kernel(const float *__restrict__ src,
                                                               const DqParams *__restrict__ Pp,
                                                               float *__restrict__ fld)
{
    using S = DqSet<MODEL>;
    constexpr int D = S::D, Q = S::Q;
    const DqParams &P = *Pp;
    int x, y, z;
    if (!dq_site(P, x, y, z)) return;
    const uint32_t V = (uint32_t)P.n[0] * (uint32_t)P.n[1] * (uint32_t)P.n[2];
    const uint32_t s = (uint32_t)x + (uint32_t)P.n[0] * ((uint32_t)y + (uint32_t)P.n[1] * (uint32_t)z);
    float d[Q], M[Q];
    dq_pull<MODEL>(src, P, x, y, z, V, d);
    dq_moments<MODEL>(P, d, M);
    const float ir = 1.0f / (P.rho0 + M[0]);
    fld[s] = M[0];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float j = M[1 + a] * 0.57735026918962576f;
        fld[(uint32_t)(1 + a) * V + s] = j - P.rho0 * P.u0[a];
        fld[(uint32_t)(1 + D + a) * V + s] = j * ir - P.u0[a];
    }
#pragma unroll
    for (int a = D + 1; a < Q; ++a) fld[(uint32_t)(a + D) * V + s] = M[a];
}

struct DqCorrArgs {
    const float *fld;
    float2 *spec;
    double *acc;
    const LinePlan *plans;
    const float2 *tables;
    int n[3];
    int nkx, kxp;
    int nf;
    int line_x, line_y, line_z;
    int D;
};

// The transform kernels below are instantiated for power-of-two lines
// (BLUE false) and for Bluestein lines (BLUE true); the host picks the one
// that matches the axis's line plan.

// Transforms along x: one block per (field pair, group of rows); pair p packs
// fields 2p + i (2p+1) (the last field alone if nf is odd) and writes the
// half spectra kx = 0..nx/2 of both, rows of pitch kxp.
template <bool BLUE>
__global__ __launch_bounds__(kFftThreads) void dq_rows_kernel(DqCorrArgs g, int rb)
{
    extern __shared__ float2 lds[];
    const int nx = g.n[0], nrows = g.n[1] * g.n[2];
    const int ngroups = (nrows + rb - 1) / rb;
    const int p = (int)blockIdx.x / ngroups, grp = (int)blockIdx.x - p * ngroups;
    const int fa = 2 * p;
    const bool pair = fa + 1 < g.nf;
    const LinePlan &L = g.plans[g.line_x];
    const int m = L.m, lg = L.log2m;
    const int r0 = grp * rb, nl = min(rb, nrows - r0);
    const size_t V = (size_t)nx * nrows;
    const float *A = g.fld + (size_t)fa * V, *B = A + V;
    const float2 *chirp = g.tables + L.chirp_off;
    // loads kBatch per thread in flight before any is stored to LDS
    const int ne = nl * m;
    for (int e0 = threadIdx.x; e0 < ne; e0 += kBatch * kFftThreads) {
        float va[kBatch], vb[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int e = e0 + i * kFftThreads, l = e >> lg, x = e & (m - 1);
            va[i] = vb[i] = 0.f;
            if (e < ne && x < nx) {
                const size_t o = (size_t)(r0 + l) * nx + x;
                va[i] = A[o];
                if (pair) vb[i] = B[o];
            }
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int e = e0 + i * kFftThreads, l = e >> lg, x = e & (m - 1);
            if (e >= ne) break;
            float2 v = make_float2(va[i], vb[i]);
            if (BLUE && x < nx) v = cmul(v, chirp[x]);
            lds[lds_slot<true>(l * m + (BLUE ? x : bitrev(x, lg)))] = v;
        }
    }
    __syncthreads();
    if (BLUE) lds_bluestein_dft<true>(lds, L, nl, m, 1, g.tables);
    else lds_fft_dit<true, false>(lds, lg, nl, m, 1, g.tables);
    const size_t fstride = (size_t)nrows * g.kxp;
    float2 *sa = g.spec + (size_t)fa * fstride, *sb = sa + fstride;
    for (int e = threadIdx.x; e < nl * g.kxp; e += kFftThreads) {
        const int l = e / g.kxp, k = e - l * g.kxp;
        const size_t o = (size_t)(r0 + l) * g.kxp + k;
        if (k >= g.nkx) {
            sa[o] = make_float2(0.f, 0.f);
            if (pair) sb[o] = make_float2(0.f, 0.f);
            continue;
        }
        const float2 zk = lds[lds_slot<true>(l * m + k)];
        if (!pair) {
            sa[o] = zk;
        } else {
            const float2 zm = lds[lds_slot<true>(l * m + (k == 0 ? 0 : nx - k))];
            sa[o] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            sb[o] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
        }
    }
}

// Transforms along y (axis 1) or z (axis 2), in place: one block per
// (field, position along the other axis, group of cb adjacent kx).
template <bool BLUE>
__global__ __launch_bounds__(kFftThreads) void dq_lines_kernel(DqCorrArgs g, int axis, int cb)
{
    extern __shared__ float2 lds[];
    const int ny = g.n[1], nz = g.n[2];
    const int n = axis == 1 ? ny : nz, nouter = axis == 1 ? nz : ny;
    const size_t stride = axis == 1 ? (size_t)g.kxp : (size_t)ny * g.kxp;
    const size_t ostride = axis == 1 ? (size_t)ny * g.kxp : (size_t)g.kxp;
    const int ncg = (g.nkx + cb - 1) / cb;
    int b = (int)blockIdx.x;
    const int cgi = b % ncg;
    b /= ncg;
    const int o = b % nouter, f = b / nouter;
    const int c0 = cgi * cb, ncol = min(cb, g.nkx - c0);
    const LinePlan &L = g.plans[axis == 1 ? g.line_y : g.line_z];
    const float2 *chirp = g.tables + L.chirp_off;
    float2 *col = g.spec + (size_t)f * ((size_t)nz * ny * g.kxp) + (size_t)o * ostride + c0;
    const int ne = L.m * cb;
    for (int i0 = threadIdx.x; i0 < ne; i0 += kBatch * kFftThreads) {
        float2 v[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int idx = i0 + i * kFftThreads, j = idx / cb, c = idx - j * cb;
            v[i] = make_float2(0.f, 0.f);
            if (idx < ne && j < n && c < ncol) v[i] = col[(size_t)j * stride + c];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int idx = i0 + i * kFftThreads, j = idx / cb, c = idx - j * cb;
            if (idx >= ne) break;
            if (BLUE && j < n) v[i] = cmul(v[i], chirp[j]);
            lds[(BLUE ? j : bitrev(j, L.log2m)) * cb + c] = v[i];
        }
    }
    __syncthreads();
    if (BLUE) lds_bluestein_dft<false>(lds, L, cb, 1, cb, g.tables);
    else lds_fft_dit<false, false>(lds, L.log2m, cb, 1, cb, g.tables);
    for (int idx = threadIdx.x; idx < n * cb; idx += kFftThreads) {
        const int j = idx / cb, c = idx - j * cb;
        if (c < ncol) col[(size_t)j * stride + c] = lds[idx];
    }
}

// Kind index of field f's auto-correlation: the two u_x u_y* kinds come
// just before the first non-conserved moment (D >= 2).
__device__ __forceinline__ int dq_auto_kind(int f, int D)
{
    return (D >= 2 && f >= 1 + 2 * D) ? f + 2 : f;
}

// Last transform axis with the accumulation fused in: one block per (field,
// position along the other axis, group of cb adjacent kx), every field alone
// except u_x, u_y, which are transformed together for their cross kinds
// (upair: one launch of that pair alone); the spectra are added to the FP64
// sums as they leave LDS, never written back.
template <bool BLUE>
__global__ __launch_bounds__(kFftThreads) void dq_last_kernel(DqCorrArgs g, int axis, int cb,
                                                              int upair)
{
    extern __shared__ float2 lds[];
    const int D = g.D, ny = g.n[1], nz = g.n[2];
    const int n = axis == 1 ? ny : nz, nouter = axis == 1 ? nz : ny;
    const size_t stride = axis == 1 ? (size_t)g.kxp : (size_t)ny * g.kxp;
    const size_t ostride = axis == 1 ? (size_t)ny * g.kxp : (size_t)g.kxp;
    const int ncg = (g.nkx + cb - 1) / cb;
    int b = (int)blockIdx.x;
    const int cgi = b % ncg;
    b /= ncg;
    const int o = b % nouter, grp = b / nouter;
    // single fields skip u_x, u_y (fields 1 + D, 2 + D)
    const int f0 = upair ? 1 + D : (grp < 1 + D ? grp : grp + 2), nfg = upair ? 2 : 1;
    const int c0 = cgi * cb, ncol = min(cb, g.nkx - c0);
    const LinePlan &L = g.plans[axis == 1 ? g.line_y : g.line_z];
    const float2 *chirp = g.tables + L.chirp_off;
    const size_t fstride = (size_t)ny * nz * g.kxp;
    const size_t base = (size_t)o * ostride + c0;
    const int nl = nfg * cb;  // interleaved lines: field q, column c at q * cb + c
    const int ne = L.m * nl;
    for (int i0 = threadIdx.x; i0 < ne; i0 += kBatch * kFftThreads) {
        float2 v[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int idx = i0 + i * kFftThreads, j = idx / nl, r = idx - j * nl, q = r / cb,
                      c = r - q * cb;
            v[i] = make_float2(0.f, 0.f);
            if (idx < ne && j < n && c < ncol)
                v[i] = g.spec[(size_t)(f0 + q) * fstride + base + (size_t)j * stride + c];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int idx = i0 + i * kFftThreads, j = idx / nl, r = idx - j * nl;
            if (idx >= ne) break;
            if (BLUE && j < n) v[i] = cmul(v[i], chirp[j]);
            lds[(BLUE ? j : bitrev(j, L.log2m)) * nl + r] = v[i];
        }
    }
    __syncthreads();
    if (BLUE) lds_bluestein_dft<false>(lds, L, nl, 1, nl, g.tables);
    else lds_fft_dit<false, false>(lds, L.log2m, nl, 1, nl, g.tables);
    for (int idx = threadIdx.x; idx < n * cb; idx += kFftThreads) {
        const int j = idx / cb, c = idx - j * cb;
        if (c >= ncol || (j == 0 && o == 0 && c0 + c == 0)) continue;  // k = 0
        const size_t off = base + (size_t)j * stride + c;
        const float2 X = lds[j * nl + c];
        const double xr = X.x, xi = X.y;
        g.acc[(size_t)dq_auto_kind(f0, D) * fstride + off] += xr * xr + xi * xi;
        if (upair) {
            const float2 Y = lds[j * nl + cb + c];
            const double yr = Y.x, yi = Y.y;
            g.acc[(size_t)dq_auto_kind(f0 + 1, D) * fstride + off] += yr * yr + yi * yi;
            g.acc[(size_t)(1 + 2 * D) * fstride + off] += xr * yr + xi * yi;
            g.acc[(size_t)(2 + 2 * D) * fstride + off] += xi * yr - xr * yi;
        }
    }
}

// FP64 accumulation of the kinds of flb_dq.h at every k of the half space.
__global__ __launch_bounds__(kDqThreads) void dq_accum_kernel(DqCorrArgs g)
{
    const int nrows = g.n[1] * g.n[2];
    const int64_t nk = (int64_t)nrows * g.nkx;
    const int64_t k = (int64_t)blockIdx.x * kDqThreads + threadIdx.x;
    if (k >= nk || k == 0) return;
    const int row = (int)(k / g.nkx), kx = (int)(k - (int64_t)row * g.nkx);
    const size_t o = (size_t)row * g.kxp + kx;
    const size_t fstride = (size_t)nrows * g.kxp;
    const int D = g.D;
    int kind = 0;
    for (int f = 0; f < g.nf; ++f) {
        if (f == 1 + 2 * D && D >= 2) {
            // u_x u_y* between the velocity fields and the moments
            const float2 a = g.spec[(size_t)(1 + D) * fstride + o];
            const float2 c = g.spec[(size_t)(2 + D) * fstride + o];
            const double ar = a.x, ai = a.y, br = c.x, bi = c.y;
            g.acc[(size_t)kind++ * fstride + o] += ar * br + ai * bi;
            g.acc[(size_t)kind++ * fstride + o] += ai * br - ar * bi;
        }
        const float2 X = g.spec[(size_t)f * fstride + o];
        const double re = X.x, im = X.y;
        g.acc[(size_t)kind++ * fstride + o] += re * re + im * im;
    }
}

}  // namespace flbdev

using namespace flbdev;

// ---------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------
struct flb_dq {
    int model = 0, D = 0, Q = 0, nm = 0, nf = 0, nkinds = 0;
    int n[3] = {1, 1, 1};
    uint32_t V = 0;
    double w[kDqMaxQ] = {0}, m[kDqMaxQ][kDqMaxQ] = {{0}};
    int v[kDqMaxQ][3] = {{0}};
    double rho0 = 1.0, theta = 0.0;
    uint64_t seed = 0;
    bool noise = false;
    bool nontemporal = false;  // streaming accesses (buffers beyond 256 MB)
    DqParams P;
    DqParams *d_P = nullptr;
    float *pops[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t t = 0;
    double *d_part = nullptr;   // reduction partials
    double *d_red = nullptr;    // reduction results (means, sums)
    int nblocks = 0;
    hipStream_t own = nullptr, stream = nullptr;
    // correlators
    bool corr_ready = false;
    LinePlan *d_plans = nullptr;
    float2 *d_tables = nullptr;
    float *d_fld = nullptr;
    float2 *d_spec = nullptr;
    double *d_acc = nullptr;
    int line[3] = {0, 0, 0};
    bool blue[3] = {false, false, false};  // the axis's line plan is a Bluestein one
    int rows_lds = 0, lines_lds = 0, rb = 1, cb = 1;
    // fused last pass: columns per block for single fields and for the u
    // pair (0: a separate accumulation)
    int last_cb = 0, last_cb_pair = 0, last_lds = 0;
    int64_t nsamples = 0;
};

namespace {

int dq_fail(int code, const std::string &msg) { return set_error(code, msg); }

#define DQ_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return dq_fail(FLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// The velocity polynomials of flb_dq.h, in order.
double dq_poly(int D, int a, const int v[3])
{
    const double x = v[0], y = v[1], z = v[2], v2 = x * x + y * y + z * z;
    if (a == 0) return 1.0;
    if (a <= D) return (double)v[a - 1];
    if (D == 1) return x * x - 1.0 / 3.0;
    if (D == 2) {
        const double p[9] = {0, 0, 0, x * x - y * y, x * y, v2 - 2.0 / 3.0, x * v2, y * v2, v2 * v2};
        return p[a];
    }
    const double p[15] = {0, 0, 0, 0, 3 * x * x - v2, y * y - z * z, x * y, y * z, z * x, v2 - 1.0,
                          x * v2, y * v2, z * v2, x * y * z, v2 * v2};
    return p[a];
}

int dq_build(int model, int &D, int &Q, int v[kDqMaxQ][3], double w[kDqMaxQ],
             double m[kDqMaxQ][kDqMaxQ])
{
    std::memset(v, 0, sizeof(int) * kDqMaxQ * 3);
    if (model == FLB_DQ_D1Q3) {
        D = 1;
        Q = 3;
        const int vx[3] = {0, 1, -1};
        const double ww[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
        for (int i = 0; i < 3; ++i) {
            v[i][0] = vx[i];
            w[i] = ww[i];
        }
    } else if (model == FLB_DQ_D2Q9) {
        D = 2;
        Q = 9;
        for (int i = 0; i < 9; ++i) {
            v[i][0] = DqSet<FLB_DQ_D2Q9>::v[i][0];
            v[i][1] = DqSet<FLB_DQ_D2Q9>::v[i][1];
            w[i] = i == 0 ? 4.0 / 9.0 : i < 5 ? 1.0 / 9.0 : 1.0 / 36.0;
        }
    } else if (model == FLB_DQ_D3Q15) {
        D = 3;
        Q = 15;
        for (int i = 0; i < 15; ++i) {
            for (int a = 0; a < 3; ++a) v[i][a] = DqSet<FLB_DQ_D3Q15>::v[i][a];
            w[i] = i == 0 ? 2.0 / 9.0 : i < 7 ? 1.0 / 9.0 : 1.0 / 72.0;
        }
    } else {
        return dq_fail(FLB_EINVAL, "unknown model");
    }
    for (int a = 0; a < Q; ++a) {
        double h[kDqMaxQ];
        for (int i = 0; i < Q; ++i) h[i] = dq_poly(D, a, v[i]);
        for (int b = 0; b < a; ++b) {
            double p = 0.0;
            for (int i = 0; i < Q; ++i) p += w[i] * h[i] * m[b][i];
            for (int i = 0; i < Q; ++i) h[i] -= p * m[b][i];
        }
        double nrm = 0.0;
        for (int i = 0; i < Q; ++i) nrm += w[i] * h[i] * h[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < Q; ++i) m[a][i] = h[i] / nrm;
    }
    return FLB_OK;
}

template <typename F> hipError_t dispatch(int model, F f)
{
    if (model == FLB_DQ_D1Q3) return f(std::integral_constant<int, FLB_DQ_D1Q3>());
    if (model == FLB_DQ_D2Q9) return f(std::integral_constant<int, FLB_DQ_D2Q9>());
    return f(std::integral_constant<int, FLB_DQ_D3Q15>());
}

uint32_t grid_sites(const flb_dq *h) { return (uint32_t)h->P.tiles_x * h->n[1] * h->n[2]; }

int enqueue_steps(flb_dq *h, int64_t n)
{
    const uint32_t k0 = (uint32_t)(h->seed & 0xFFFFFFFFu), k1 = (uint32_t)(h->seed >> 32);
    for (int64_t s = 0; s < n; ++s) {
        const uint32_t t = (uint32_t)(h->t + s);
        const float *src = h->pops[h->cur];
        float *dst = h->pops[h->cur ^ 1];
        DQ_HIP(dispatch(h->model, [&](auto mc) {
            constexpr int MODEL = decltype(mc)::value;
            const dim3 grid(grid_sites(h)), block(kDqThreads);
            if (h->noise && h->nontemporal)
                hipLaunchKernelGGL((dq_step_kernel<MODEL, true, true>), grid, block, 0, h->stream,
                                   src, dst, h->d_P, t, k0, k1);
            else if (h->noise)
                hipLaunchKernelGGL((dq_step_kernel<MODEL, true, false>), grid, block, 0, h->stream,
                                   src, dst, h->d_P, t, k0, k1);
            else if (h->nontemporal)
                hipLaunchKernelGGL((dq_step_kernel<MODEL, false, true>), grid, block, 0, h->stream,
                                   src, dst, h->d_P, t, k0, k1);
            else
                hipLaunchKernelGGL((dq_step_kernel<MODEL, false, false>), grid, block, 0,
                                   h->stream, src, dst, h->d_P, t, k0, k1);
            return hipGetLastError();
        }));
        h->cur ^= 1;
    }
    h->t += n;
    return FLB_OK;
}

int setup_corr(flb_dq *h)
{
    if (h->corr_ready) return FLB_OK;
    for (int a = 0; a < h->D; ++a)
        if (!line_length_ok(h->n[a]))
            return dq_fail(FLB_ESIZE, "correlators support power-of-two sides up to 4096 and "
                                      "other sides up to 2048");
    DQ_HIP(hipStreamSynchronize(h->stream));
    LineTables lt;
    for (int a = 0; a < 3; ++a) {
        h->line[a] = lt.plan_for(h->n[a] > 1 ? h->n[a] : 2);
        h->blue[a] = lt.plans[h->line[a]].bluestein != 0;
    }
    const int mx = lt.plans[h->line[0]].m;
    h->rb = std::max(1, std::min(h->n[1] * h->n[2], 4096 / mx));
    h->rows_lds = lds_padded_elems(h->rb * mx) * (int)sizeof(float2);
    int my = 1;
    for (int a = 1; a < 3; ++a)
        if (h->n[a] > 1) my = std::max(my, lt.plans[h->line[a]].m);
    h->cb = std::max(1, std::min(16, 8192 / my));
    h->lines_lds = my * h->cb * (int)sizeof(float2);
    // the last axis carries the accumulation when the two u fields of cb >= 4
    // columns fit 32 KB of LDS; single fields take up to 16 columns (whole
    // 128-byte lines of the spectra and the sums) in the same 32 KB
    h->last_cb = h->last_cb_pair = 0;
    if (h->D >= 2) {
        const int ml = lt.plans[h->line[h->D - 1]].m;
        const int cbp = std::min(16, 32768 / (2 * ml * (int)sizeof(float2)));
        if (cbp >= 4) {
            h->last_cb_pair = cbp;
            h->last_cb = std::min(16, 2 * cbp);
            h->last_lds = 32768;
        }
    }
    const int nkx = h->n[0] / 2 + 1, kxp = (nkx + 15) / 16 * 16;
    h->P.nkx = nkx;
    h->P.kxp = kxp;
    const size_t nrows = (size_t)h->n[1] * h->n[2];
    DQ_HIP(hipMalloc((void **)&h->d_plans, lt.plans.size() * sizeof(LinePlan)));
    DQ_HIP(hipMemcpy(h->d_plans, lt.plans.data(), lt.plans.size() * sizeof(LinePlan),
                     hipMemcpyHostToDevice));
    DQ_HIP(hipMalloc((void **)&h->d_tables, lt.tables.size() * sizeof(float2)));
    DQ_HIP(hipMemcpy(h->d_tables, lt.tables.data(), lt.tables.size() * sizeof(float2),
                     hipMemcpyHostToDevice));
    DQ_HIP(hipMalloc((void **)&h->d_fld, (size_t)h->nf * h->V * sizeof(float)));
    DQ_HIP(hipMalloc((void **)&h->d_spec, (size_t)h->nf * nrows * kxp * sizeof(float2)));
    DQ_HIP(hipMalloc((void **)&h->d_acc, (size_t)h->nkinds * nrows * kxp * sizeof(double)));
    DQ_HIP(hipMemcpy(h->d_P, &h->P, sizeof(DqParams), hipMemcpyHostToDevice));
    DQ_HIP(launch_fill(h->d_acc, (size_t)h->nkinds * nrows * kxp, h->stream));
    h->nsamples = 0;
    h->corr_ready = true;
    return FLB_OK;
}

DqCorrArgs corr_args(const flb_dq *h)
{
    DqCorrArgs g;
    g.fld = h->d_fld;
    g.spec = h->d_spec;
    g.acc = h->d_acc;
    g.plans = h->d_plans;
    g.tables = h->d_tables;
    for (int a = 0; a < 3; ++a) g.n[a] = h->n[a];
    g.nkx = h->P.nkx;
    g.kxp = h->P.kxp;
    g.nf = h->nf;
    g.line_x = h->line[0];
    g.line_y = h->line[1];
    g.line_z = h->line[2];
    g.D = h->D;
    return g;
}

int enqueue_sample(flb_dq *h)
{
    const float *src = h->pops[h->cur];
    DQ_HIP(dispatch(h->model, [&](auto mc) {
        constexpr int MODEL = decltype(mc)::value;
        hipLaunchKernelGGL(dq_fields_kernel<MODEL>, dim3(grid_sites(h)), dim3(kDqThreads), 0,
                           h->stream, src, h->d_P, h->d_fld);
        return hipGetLastError();
    }));
    const DqCorrArgs g = corr_args(h);
    const int nrows = h->n[1] * h->n[2];
    const int ngroups = (nrows + h->rb - 1) / h->rb;
    const int npairs = (h->nf + 1) / 2;
    if (h->blue[0])
        hipLaunchKernelGGL(dq_rows_kernel<true>, dim3(npairs * ngroups), dim3(kFftThreads),
                           h->rows_lds, h->stream, g, h->rb);
    else
        hipLaunchKernelGGL(dq_rows_kernel<false>, dim3(npairs * ngroups), dim3(kFftThreads),
                           h->rows_lds, h->stream, g, h->rb);
    DQ_HIP(hipGetLastError());
    const int ncg = (h->P.nkx + h->cb - 1) / h->cb;
    const int last = h->D - 1;  // the last transformed axis (D >= 2)
    for (int axis = 1; axis < 3; ++axis) {
        if (h->n[axis] < 2) continue;
        const int nouter = axis == 1 ? h->n[2] : h->n[1];
        if (axis == last && h->last_cb) {
            const int ncgl = (h->P.nkx + h->last_cb - 1) / h->last_cb;
            const int ncgp = (h->P.nkx + h->last_cb_pair - 1) / h->last_cb_pair;
            auto lastk = h->blue[axis] ? dq_last_kernel<true> : dq_last_kernel<false>;
            hipLaunchKernelGGL(lastk, dim3((h->nf - 2) * nouter * ncgl), dim3(kFftThreads),
                               h->last_lds, h->stream, g, axis, h->last_cb, 0);
            DQ_HIP(hipGetLastError());
            hipLaunchKernelGGL(lastk, dim3(nouter * ncgp), dim3(kFftThreads), h->last_lds,
                               h->stream, g, axis, h->last_cb_pair, 1);
        } else {
            auto lines = h->blue[axis] ? dq_lines_kernel<true> : dq_lines_kernel<false>;
            hipLaunchKernelGGL(lines, dim3(h->nf * nouter * ncg), dim3(kFftThreads),
                               h->lines_lds, h->stream, g, axis, h->cb);
        }
        DQ_HIP(hipGetLastError());
    }
    if (!h->last_cb) {
        const int64_t nk = (int64_t)nrows * h->P.nkx;
        hipLaunchKernelGGL(dq_accum_kernel, dim3((unsigned)((nk + kDqThreads - 1) / kDqThreads)),
                           dim3(kDqThreads), 0, h->stream, g);
        DQ_HIP(hipGetLastError());
    }
    h->nsamples += 1;
    return FLB_OK;
}

int check(flb_dq *h)
{
    if (!h) return dq_fail(FLB_EINVAL, "NULL handle");
    return FLB_OK;
}

}  // namespace

extern "C" {

int flb_dq_tables(int model, int32_t *D, int32_t *Q, int32_t *v, double *w, double *m)
{
    if (!D || !Q || !v || !w || !m) return dq_fail(FLB_EINVAL, "NULL argument");
    int d, q, vv[kDqMaxQ][3];
    double ww[kDqMaxQ], mm[kDqMaxQ][kDqMaxQ];
    int rc = dq_build(model, d, q, vv, ww, mm);
    if (rc) return rc;
    *D = d;
    *Q = q;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) v[3 * i + a] = vv[i][a];
        w[i] = ww[i];
    }
    for (int a = 0; a < q; ++a)
        for (int i = 0; i < q; ++i) m[a * q + i] = mm[a][i];
    return FLB_OK;
}

flb_dq_t *flb_dq_create(int model, const int32_t n[3], const double *tau, double theta,
                        double rho0, const double u0[3], uint64_t seed, uint32_t stream_id,
                        uint32_t flags)
{
    if (!n || !tau || !u0) {
        dq_fail(FLB_EINVAL, "NULL argument");
        return nullptr;
    }
    if (flags & ~FLB_FLAG_NO_GHOST_NOISE) {
        dq_fail(FLB_EINVAL, "unknown flags");
        return nullptr;
    }
    flb_dq *h = new flb_dq();
    auto bail = [&](int code, const std::string &msg) -> flb_dq_t * {
        if (!msg.empty()) dq_fail(code, msg);
        flb_dq_destroy(h);
        return nullptr;
    };
    if (dq_build(model, h->D, h->Q, h->v, h->w, h->m)) return bail(0, "");
    h->model = model;
    const int D = h->D, Q = h->Q;
    for (int a = 0; a < 3; ++a) {
        if (a < D && n[a] < 2) return bail(FLB_EINVAL, "used sides must be >= 2");
        if (a >= D && n[a] != 1) return bail(FLB_EINVAL, "unused sides must be 1");
        h->n[a] = n[a];
    }
    const double V = (double)n[0] * n[1] * n[2];
    if (V * Q * 4.0 >= 4294967296.0)
        return bail(FLB_ESIZE, "the populations of one buffer must stay below 4 GiB");
    h->V = (uint32_t)V;
    if (!std::isfinite(theta) || theta < 0) return bail(FLB_EINVAL, "theta must be finite and >= 0");
    if (!std::isfinite(rho0) || rho0 <= 0) return bail(FLB_EINVAL, "rho0 must be finite and > 0");
    double uu = 0;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(u0[a])) return bail(FLB_EINVAL, "u0 must be finite");
        if (a >= D && u0[a] != 0.0) return bail(FLB_EINVAL, "u0 has a component along an unused axis");
        uu += u0[a] * u0[a];
    }
    if (uu >= 1.0 / 3.0) return bail(FLB_EINVAL, "|u0| must be below the sound speed");
    for (int a = D + 1; a < Q; ++a)
        if (!std::isfinite(tau[a]) || tau[a] <= 0.5)
            return bail(FLB_EINVAL, "tau[" + std::to_string(a) + "] must be finite and > 1/2");
    h->nm = Q - D - 1;
    h->nf = 1 + 2 * D + h->nm;
    h->nkinds = h->nf + (D >= 2 ? 2 : 0);
    h->rho0 = rho0;
    h->theta = theta;
    h->seed = seed;
    DqParams &P = h->P;
    std::memset(&P, 0, sizeof P);
    for (int a = 0; a < 3; ++a) P.n[a] = n[a];
    P.tiles_x = (n[0] + kDqThreads - 1) / kDqThreads;
    P.stream_id = stream_id;
    P.rho0 = (float)rho0;
    for (int a = 0; a < 3; ++a) P.u0[a] = (float)u0[a];
    const double mu = 3.0 * theta;
    const int first_ghost = 1 + D + D * (D + 1) / 2;
    for (int i = 0; i < Q; ++i) {
        P.w[i] = (float)h->w[i];
        P.therm[i] = (float)std::sqrt(mu * rho0 * h->w[i]);
    }
    for (int a = 0; a < Q; ++a)
        for (int i = 0; i < Q; ++i) {
            P.m[a][i] = (float)h->m[a][i];
            P.nw[a][i] = (float)(h->w[i] * h->m[a][i]);
        }
    for (int a = D + 1; a < Q; ++a) {
        P.omega[a] = (float)(1.0 / tau[a]);
        double sigma = std::sqrt(mu * rho0 * (2.0 * tau[a] - 1.0)) / tau[a];
        if ((flags & FLB_FLAG_NO_GHOST_NOISE) && a >= first_ghost) sigma = 0.0;
        P.amp[a] = (float)sigma;
        h->noise = h->noise || sigma != 0.0;
    }
    for (int s = 0; s < D * (D + 1) / 2; ++s) {
        const int a = D + 1 + s;
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                double t = 0;
                for (int i = 0; i < Q; ++i) t += h->w[i] * h->m[a][i] * h->v[i][al] * h->v[i][be];
                P.T[s][al][be] = (float)t;
            }
    }
    h->nblocks = (int)grid_sites(h);
    if (hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) != hipSuccess)
        return bail(FLB_EHIP, "stream creation failed");
    h->stream = h->own;
    const size_t bytes = (size_t)Q * h->V * sizeof(float);
    h->nontemporal = bytes > 256u * 1024 * 1024;
    if (hipMalloc((void **)&h->pops[0], 2 * bytes) != hipSuccess)
        return bail(FLB_ENOMEM, "population buffers: out of device memory");
    h->pops[1] = h->pops[0] + (size_t)Q * h->V;
    if (hipMalloc((void **)&h->d_P, sizeof(DqParams)) != hipSuccess ||
        hipMalloc((void **)&h->d_part, (size_t)h->nblocks * kDqMaxQ * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&h->d_red, 32 * sizeof(double)) != hipSuccess)
        return bail(FLB_ENOMEM, "scratch allocation failed");
    if (hipMemcpy(h->d_P, &P, sizeof(DqParams), hipMemcpyHostToDevice) != hipSuccess)
        return bail(FLB_EHIP, "parameter upload failed");
    // uniform f^0(rho0, u0) (Eq. 2) as deviations from w_i rho0
    std::vector<float> init((size_t)Q * h->V);
    for (int i = 0; i < Q; ++i) {
        double vu = 0;
        for (int a = 0; a < 3; ++a) vu += h->v[i][a] * u0[a];
        const double f0 = h->w[i] * rho0 * (1.0 + 3.0 * vu + 4.5 * vu * vu - 1.5 * uu);
        std::fill(init.begin() + (size_t)i * h->V, init.begin() + (size_t)(i + 1) * h->V,
                  (float)(f0 - h->w[i] * rho0));
    }
    if (hipMemcpy(h->pops[0], init.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return bail(FLB_EHIP, "initial state upload failed");
    return h;
}

void flb_dq_destroy(flb_dq_t *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own) (void)hipStreamSynchronize(h->own);
    void *ptrs[] = {h->pops[0], h->d_P, h->d_part, h->d_red, h->d_plans, h->d_tables,
                    h->d_fld, h->d_spec, h->d_acc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

int flb_dq_info(flb_dq_t *h, int32_t *D, int32_t *Q, int32_t *nkinds)
{
    if (check(h)) return FLB_EINVAL;
    if (D) *D = h->D;
    if (Q) *Q = h->Q;
    if (nkinds) *nkinds = h->nkinds;
    return FLB_OK;
}

int flb_dq_set_stream(flb_dq_t *h, void *hip_stream)
{
    if (check(h)) return FLB_EINVAL;
    DQ_HIP(hipStreamSynchronize(h->stream));
    h->stream = hip_stream ? (hipStream_t)hip_stream : h->own;
    return FLB_OK;
}

int flb_dq_synchronize(flb_dq_t *h)
{
    if (check(h)) return FLB_EINVAL;
    DQ_HIP(hipStreamSynchronize(h->stream));
    return FLB_OK;
}

int flb_dq_step(flb_dq_t *h, int64_t nsteps)
{
    if (check(h)) return FLB_EINVAL;
    if (nsteps < 0) return dq_fail(FLB_EINVAL, "nsteps must be >= 0");
    if (h->t + nsteps >= (int64_t)0xFFFFFFFF)
        return dq_fail(FLB_ESIZE, "t must stay below 2^32 - 1 (a noise counter word)");
    return enqueue_steps(h, nsteps);
}

int flb_dq_run(flb_dq_t *h, int64_t nsteps, int sample_every)
{
    if (check(h)) return FLB_EINVAL;
    if (sample_every < 0) return dq_fail(FLB_EINVAL, "sample_every must be >= 0");
    if (sample_every == 0) return flb_dq_step(h, nsteps);
    if (nsteps < 0) return dq_fail(FLB_EINVAL, "nsteps must be >= 0");
    if (h->t + nsteps >= (int64_t)0xFFFFFFFF)
        return dq_fail(FLB_ESIZE, "t must stay below 2^32 - 1 (a noise counter word)");
    int rc = setup_corr(h);
    if (rc) return rc;
    while (nsteps > 0) {
        const int64_t to = sample_every - h->t % sample_every;
        const int64_t k = std::min(nsteps, to);
        if ((rc = enqueue_steps(h, k))) return rc;
        nsteps -= k;
        if (k == to && (rc = enqueue_sample(h))) return rc;
    }
    return FLB_OK;
}

int64_t flb_dq_get_step(flb_dq_t *h) { return h ? h->t : -1; }

int flb_dq_accumulate(flb_dq_t *h)
{
    if (check(h)) return FLB_EINVAL;
    int rc = setup_corr(h);
    if (rc) return rc;
    return enqueue_sample(h);
}

int flb_dq_read(flb_dq_t *h, double *out, size_t n_doubles, int64_t *nsamples)
{
    if (check(h)) return FLB_EINVAL;
    if (!out) return dq_fail(FLB_EINVAL, "out must not be NULL");
    int rc = setup_corr(h);
    if (rc) return rc;
    const size_t nrows = (size_t)h->n[1] * h->n[2];
    if (n_doubles < (size_t)h->nkinds * nrows * h->P.nkx)
        return dq_fail(FLB_ESIZE, "output buffer too small for the correlators");
    DQ_HIP(hipStreamSynchronize(h->stream));
    DQ_HIP(hipMemcpy2D(out, (size_t)h->P.nkx * sizeof(double), h->d_acc,
                       (size_t)h->P.kxp * sizeof(double), (size_t)h->P.nkx * sizeof(double),
                       (size_t)h->nkinds * nrows, hipMemcpyDeviceToHost));
    if (nsamples) *nsamples = h->nsamples;
    return FLB_OK;
}

int flb_dq_read_normalized(flb_dq_t *h, double *out, size_t n_doubles, int64_t *nsamples)
{
    int64_t ns = 0;
    int rc = flb_dq_read(h, out, n_doubles, &ns);
    if (rc) return rc;
    if (nsamples) *nsamples = ns;
    if (ns <= 0) return dq_fail(FLB_ESTATE, "no correlator sample to normalise");
    if (!(h->theta > 0))
        return dq_fail(FLB_ESTATE, "theta = 0: no fluctuation scale to normalise by");
    // Eq. (11) (and Eq. 12 for u_x u_y*) at the noise temperature, mu = 3 theta
    const double V = (double)h->V, mu = 3.0 * h->theta, rho0 = h->rho0, theta = h->theta;
    const int D = h->D;
    const size_t plane = (size_t)h->n[1] * h->n[2] * h->P.nkx;
    for (int q = 0; q < h->nkinds; ++q) {
        double norm;
        if (q == 0) norm = 1.0 / (V * mu * rho0);                  // rho
        else if (q <= D) norm = 1.0 / (V * rho0 * theta);          // j_a
        else if (q <= 2 * D) norm = rho0 / (V * theta);            // u_a
        else if (D >= 2 && q <= 2 * D + 2) norm = rho0 / (V * theta);  // Re, Im u_x u_y*
        else norm = 1.0 / (V * mu * rho0);                         // non-conserved moments
        double *p = out + (size_t)q * plane;
        for (size_t k = 0; k < plane; ++k) p[k] = p[k] / (double)ns * norm;
    }
    return FLB_OK;
}

int flb_dq_reset(flb_dq_t *h)
{
    if (check(h)) return FLB_EINVAL;
    int rc = setup_corr(h);
    if (rc) return rc;
    const size_t nrows = (size_t)h->n[1] * h->n[2];
    DQ_HIP(launch_fill(h->d_acc, (size_t)h->nkinds * nrows * h->P.kxp, h->stream));
    h->nsamples = 0;
    return FLB_OK;
}

int flb_dq_get_populations(flb_dq_t *h, double *out, size_t n)
{
    if (check(h)) return FLB_EINVAL;
    if (!out) return dq_fail(FLB_EINVAL, "out must not be NULL");
    const size_t total = (size_t)h->Q * h->V;
    if (n < total) return dq_fail(FLB_ESIZE, "output buffer smaller than Q*nx*ny*nz");
    std::vector<float> buf(total);
    DQ_HIP(hipStreamSynchronize(h->stream));
    DQ_HIP(hipMemcpy(buf.data(), h->pops[h->cur], total * sizeof(float), hipMemcpyDeviceToHost));
    // stored: post-collision values at their source sites; f_i(x) = stored_i(x - v_i)
    const int nx = h->n[0], ny = h->n[1], nz = h->n[2];
    for (int i = 0; i < h->Q; ++i)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int xs = (x - h->v[i][0] + nx) % nx, ys = (y - h->v[i][1] + ny) % ny;
                    const int zs = (z - h->v[i][2] + nz) % nz;
                    out[(size_t)i * h->V + x + (size_t)nx * (y + (size_t)ny * z)] =
                        (double)buf[(size_t)i * h->V + xs + (size_t)nx * (ys + (size_t)ny * zs)] +
                        h->w[i] * h->rho0;
                }
    return FLB_OK;
}

int flb_dq_set_populations(flb_dq_t *h, const double *in, size_t n)
{
    if (check(h)) return FLB_EINVAL;
    if (!in) return dq_fail(FLB_EINVAL, "in must not be NULL");
    const size_t total = (size_t)h->Q * h->V;
    if (n < total) return dq_fail(FLB_ESIZE, "input buffer smaller than Q*nx*ny*nz");
    std::vector<float> buf(total);
    const int nx = h->n[0], ny = h->n[1], nz = h->n[2];
    for (int i = 0; i < h->Q; ++i)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int xs = (x - h->v[i][0] + nx) % nx, ys = (y - h->v[i][1] + ny) % ny;
                    const int zs = (z - h->v[i][2] + nz) % nz;
                    buf[(size_t)i * h->V + xs + (size_t)nx * (ys + (size_t)ny * zs)] =
                        (float)(in[(size_t)i * h->V + x + (size_t)nx * (y + (size_t)ny * z)] -
                                h->w[i] * h->rho0);
                }
    DQ_HIP(hipStreamSynchronize(h->stream));
    DQ_HIP(hipMemcpy(h->pops[h->cur], buf.data(), total * sizeof(float), hipMemcpyHostToDevice));
    return FLB_OK;
}

int flb_dq_thermalize(flb_dq_t *h)
{
    if (check(h)) return FLB_EINVAL;
    const uint32_t k0 = (uint32_t)(h->seed & 0xFFFFFFFFu), k1 = (uint32_t)(h->seed >> 32);
    float *buf = h->pops[h->cur];
    DQ_HIP(dispatch(h->model, [&](auto mc) {
        constexpr int MODEL = decltype(mc)::value;
        hipLaunchKernelGGL(dq_thermal_add_kernel<MODEL>, dim3(grid_sites(h)), dim3(kDqThreads), 0,
                           h->stream, buf, h->d_P, k0, k1, h->d_part);
        return hipGetLastError();
    }));
    hipLaunchKernelGGL(dq_reduce_kernel, dim3(1), dim3(kDqThreads), 0, h->stream, h->d_part,
                       h->nblocks, h->Q, 1.0 / (double)h->V, h->d_red);
    DQ_HIP(hipGetLastError());
    const uint64_t total = (uint64_t)h->Q * h->V;
    hipLaunchKernelGGL(dq_thermal_sub_kernel, dim3((unsigned)((total + kDqThreads - 1) / kDqThreads)),
                       dim3(kDqThreads), 0, h->stream, buf, h->Q, h->V, h->d_red);
    DQ_HIP(hipGetLastError());
    return FLB_OK;
}

int flb_dq_conservation(flb_dq_t *h, double out[4])
{
    if (check(h)) return FLB_EINVAL;
    if (!out) return dq_fail(FLB_EINVAL, "out must not be NULL");
    const float *buf = h->pops[h->cur];
    DQ_HIP(dispatch(h->model, [&](auto mc) {
        constexpr int MODEL = decltype(mc)::value;
        hipLaunchKernelGGL(dq_conservation_kernel<MODEL>, dim3(grid_sites(h)), dim3(kDqThreads),
                           0, h->stream, buf, h->d_P, h->d_part);
        return hipGetLastError();
    }));
    hipLaunchKernelGGL(dq_reduce_kernel, dim3(1), dim3(kDqThreads), 0, h->stream, h->d_part,
                       h->nblocks, 4, 1.0, h->d_red);
    DQ_HIP(hipGetLastError());
    double r[4];
    DQ_HIP(hipMemcpyAsync(r, h->d_red, sizeof r, hipMemcpyDeviceToHost, h->stream));
    DQ_HIP(hipStreamSynchronize(h->stream));
    out[0] = r[0] + h->rho0 * (double)h->V;
    for (int a = 1; a < 4; ++a) out[a] = a <= h->D ? r[a] : 0.0;
    return FLB_OK;
}

}  // extern "C"
