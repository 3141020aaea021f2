// flb_corr.hip -- correlator sample: spatial transforms of the fluctuation
// fields and FP64 accumulation of Eqs. (11)-(12).
//
// Fields (FP32): d rho = rho - rho0, d j = j - rho0 u0, d u = j / rho - u0.
// Subtracting the constant reference instead of the spatial mean changes the
// transform only at k = 0, which is not accumulated (the paper's fluctuation
// dM = M - <M> has no k = 0 component), and keeps the FP32 transforms free of
// a large mean.
//
// Three kernels per sample:
//   rows : one block per (lattice, row, signal) gathers the state, packs two
//          real sequences into one complex line (jx + i jy, ux + i uy, or the
//          density of two consecutive rows), transforms it along x in LDS and
//          writes the half spectra kx = 0..nx/2 of both real sequences;
//   cols : one block per (lattice, field, column block) transforms the half
//          spectra along y in LDS, in place;
//   accum: one thread per (ky, kx) forms the fifteen products of the five
//          spectra and adds them to the FP64 sums.
// Lines of power-of-two length use a radix-2 transform in LDS; other lengths
// use Bluestein's chirp-z convolution with a power-of-two work length.
#include "flb_device.h"

namespace flbdev {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Radix-2 transform of `nlines` lines of length 2^lg held in LDS; element j
// of line l at buf[l * ls + j * es].  Forward: exp(-2 pi i jk / m).
__device__ void lds_fft(float2 *buf, int lg, int nlines, int ls, int es, const float2 *tw,
                        bool inverse)
{
    if (lg == 0) return;
    const int m = 1 << lg, hm = m >> 1;
    for (int idx = threadIdx.x; idx < nlines * m; idx += blockDim.x) {
        const int l = idx >> lg, j = idx & (m - 1);
        const int r = (int)(__brev((unsigned)j) >> (32 - lg));
        if (j < r) {
            float2 *a = buf + l * ls + j * es, *b = buf + l * ls + r * es;
            const float2 t = *a;
            *a = *b;
            *b = t;
        }
    }
    __syncthreads();
    for (int s = 1; s <= lg; ++s) {
        const int half = 1 << (s - 1);
        const int shift = kTwLog - s;
        for (int idx = threadIdx.x; idx < nlines * hm; idx += blockDim.x) {
            const int l = idx >> (lg - 1), bb = idx & (hm - 1);
            const int k = bb & (half - 1), grp = bb >> (s - 1);
            const int i0 = grp * 2 * half + k, i1 = i0 + half;
            float2 w = tw[k << shift];
            if (inverse) w.y = -w.y;
            float2 *pa = buf + l * ls + i0 * es, *pb = buf + l * ls + i1 * es;
            const float2 a = *pa, t = cmul(w, *pb);
            *pa = make_float2(a.x + t.x, a.y + t.y);
            *pb = make_float2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
}

// Length-n DFT of lines already multiplied by the chirp (Bluestein) or plain
// (power of two), in place.  On exit element k < n of each line holds X_k.
// Expects the data written and a barrier passed before the call.
__device__ void lds_line_dft(float2 *buf, const LinePlan &L, int nlines, int ls, int es,
                             const float2 *tables)
{
    const float2 *tw = tables;
    if (!L.bluestein) {
        lds_fft(buf, L.log2m, nlines, ls, es, tw, false);
        return;
    }
    lds_fft(buf, L.log2m, nlines, ls, es, tw, false);
    const float2 *K = tables + L.kernel_off;
    for (int idx = threadIdx.x; idx < nlines * L.m; idx += blockDim.x) {
        const int l = idx / L.m, j = idx - l * L.m;
        float2 *p = buf + l * ls + j * es;
        *p = cmul(*p, K[j]);
    }
    __syncthreads();
    lds_fft(buf, L.log2m, nlines, ls, es, tw, true);
    const float2 *C = tables + L.chirp_off;
    for (int idx = threadIdx.x; idx < nlines * L.n; idx += blockDim.x) {
        const int l = idx / L.n, j = idx - l * L.n;
        float2 *p = buf + l * ls + j * es;
        *p = cmul(*p, C[j]);
    }
    __syncthreads();
}

struct CorrArgs {
    const void *pops;
    const LatticeParams *params;
    const LinePlan *plans;
    const float2 *tables;
    const CorrItem *items;
    float2 *spec;
    double *acc;
};

// Fluctuation fields at site (x, y) of the current state.
template <int S>
__device__ __forceinline__ void site_fields(const typename Codec<S>::T *p, const LatticeParams &P,
                                            int x, int y, float &drho, float &djx, float &djy,
                                            float &dux, float &duy)
{
    const int nx = P.nx, ny = P.ny, plane = (int)P.plane;
    float r = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = wrap_add(x, -kVX[i], nx), ys = wrap_add(y, -kVY[i], ny);
        const float d = Codec<S>::decode(p[i * plane + ys * nx + xs], P, i);
        r += d;
        jx += (float)kVX[i] * d;
        jy += (float)kVY[i] * d;
    }
    const float ir = 1.0f / (P.rho0 + r);
    drho = r;
    djx = jx - P.rho0 * P.u0x;
    djy = jy - P.rho0 * P.u0y;
    dux = jx * ir - P.u0x;
    duy = jy * ir - P.u0y;
}

template <int S>
__global__ __launch_bounds__(kThreads) void corr_rows_kernel(CorrArgs g)
{
    using T = typename Codec<S>::T;
    extern __shared__ float2 lds[];
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_x];
    const int nx = P.nx, ny = P.ny, nkx = P.nkx;
    const int y = it.a, sig = it.b;
    const T *p = (const T *)g.pops + P.base;
    const float2 *chirp = g.tables + L.chirp_off;

    for (int x = threadIdx.x; x < L.m; x += blockDim.x) {
        float2 v = make_float2(0.f, 0.f);
        if (x < nx) {
            float dr, jx, jy, ux, uy;
            site_fields<S>(p, P, x, y, dr, jx, jy, ux, uy);
            if (sig == 0) {
                v = make_float2(jx, jy);
            } else if (sig == 1) {
                v = make_float2(ux, uy);
            } else {
                v.x = dr;
                if (y + 1 < ny) {
                    site_fields<S>(p, P, x, y + 1, dr, jx, jy, ux, uy);
                    v.y = dr;
                }
            }
            if (L.bluestein) v = cmul(v, chirp[x]);
        }
        lds[x] = v;
    }
    __syncthreads();
    lds_line_dft(lds, L, 1, 0, 1, g.tables);

    // Two real sequences a, b packed as z = a + i b:
    // a_k = (z_k + conj z_{-k}) / 2, b_k = (z_k - conj z_{-k}) / (2i).
    float2 *spec = g.spec + P.spec_base;
    const int64_t fstride = (int64_t)ny * nkx;
    int fa, fb, ya = y, yb = y;
    if (sig == 0) {
        fa = 1; fb = 2;
    } else if (sig == 1) {
        fa = 3; fb = 4;
    } else {
        fa = 0; fb = 0; yb = y + 1;
    }
    for (int k = threadIdx.x; k < nkx; k += blockDim.x) {
        const float2 zk = lds[k];
        const float2 zm = lds[k == 0 ? 0 : nx - k];
        const float2 a = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 b = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
        spec[fa * fstride + (int64_t)ya * nkx + k] = a;
        if (yb < ny) spec[fb * fstride + (int64_t)yb * nkx + k] = b;
    }
}

__global__ __launch_bounds__(kThreads) void corr_cols_kernel(CorrArgs g, int cb)
{
    extern __shared__ float2 lds[];
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const LinePlan &L = g.plans[P.line_y];
    const int ny = P.ny, nkx = P.nkx;
    const int f = it.a, c0 = it.b;
    const int ncol = min(cb, nkx - c0);
    float2 *col = g.spec + P.spec_base + (int64_t)f * ny * nkx + c0;
    const float2 *chirp = g.tables + L.chirp_off;

    for (int idx = threadIdx.x; idx < L.m * cb; idx += blockDim.x) {
        const int j = idx / cb, c = idx - j * cb;
        float2 v = make_float2(0.f, 0.f);
        if (j < ny && c < ncol) {
            v = col[(int64_t)j * nkx + c];
            if (L.bluestein) v = cmul(v, chirp[j]);
        }
        lds[idx] = v;
    }
    __syncthreads();
    lds_line_dft(lds, L, cb, 1, cb, g.tables);
    for (int idx = threadIdx.x; idx < ny * cb; idx += blockDim.x) {
        const int j = idx / cb, c = idx - j * cb;
        if (c < ncol) col[(int64_t)j * nkx + c] = lds[idx];
    }
}

__global__ __launch_bounds__(kThreads) void corr_accum_kernel(CorrArgs g)
{
    const CorrItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int64_t nk = (int64_t)P.ny * P.nkx;
    const int64_t k = (int64_t)it.a + threadIdx.x;
    if (k >= nk || k == 0) return;  // k = 0 carries no fluctuation
    const float2 *sp = g.spec + P.spec_base;
    double re[5], im[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const float2 v = sp[f * nk + k];
        re[f] = v.x;
        im[f] = v.y;
    }
    double *a = g.acc + P.acc_base + k;
    // a b* = (ar br + ai bi) + i (ai br - ar bi)
#define FLB_RE(u, v) (re[u] * re[v] + im[u] * im[v])
#define FLB_IM(u, v) (im[u] * re[v] - re[u] * im[v])
    const double val[kKinds] = {FLB_RE(0, 0), FLB_RE(1, 1), FLB_RE(2, 2), FLB_RE(3, 3),
                                FLB_RE(4, 4), FLB_RE(3, 4), FLB_IM(3, 4), FLB_RE(0, 1),
                                FLB_IM(0, 1), FLB_RE(0, 2), FLB_IM(0, 2), FLB_RE(0, 3),
                                FLB_IM(0, 3), FLB_RE(0, 4), FLB_IM(0, 4)};
#undef FLB_RE
#undef FLB_IM
#pragma unroll
    for (int q = 0; q < kKinds; ++q) a[q * nk] += val[q];
}

static CorrArgs make_args(const DeviceView &v, const CorrItem *items)
{
    CorrArgs g;
    g.pops = v.pops[v.cur];
    g.params = v.params;
    g.plans = v.plans;
    g.tables = v.tables;
    g.items = items;
    g.spec = v.spec;
    g.acc = v.acc;
    return g;
}

hipError_t launch_corr_rows(const DeviceView &v, const CorrItem *items, int nitems,
                            int lds_bytes, hipStream_t s)
{
    const CorrArgs g = make_args(v, items);
    const dim3 grid(nitems), block(kThreads);
    if (v.storage == kF32)
        hipLaunchKernelGGL(corr_rows_kernel<kF32>, grid, block, lds_bytes, s, g);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(corr_rows_kernel<kBF16>, grid, block, lds_bytes, s, g);
    else
        hipLaunchKernelGGL(corr_rows_kernel<kF16>, grid, block, lds_bytes, s, g);
    return hipGetLastError();
}

hipError_t launch_corr_cols(const DeviceView &v, const CorrItem *items, int nitems, int cb,
                            int lds_bytes, hipStream_t s)
{
    const CorrArgs g = make_args(v, items);
    hipLaunchKernelGGL(corr_cols_kernel, dim3(nitems), dim3(kThreads), lds_bytes, s, g, cb);
    return hipGetLastError();
}

hipError_t launch_corr_accum(const DeviceView &v, const CorrItem *items, int nitems,
                             hipStream_t s)
{
    const CorrArgs g = make_args(v, items);
    hipLaunchKernelGGL(corr_accum_kernel, dim3(nitems), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

}  // namespace flbdev
