// flb_step.hip -- the fused noisy D2Q9 step and the state utility kernels.
//
// One thread updates one site per row it owns: it gathers the nine
// post-collision values of the previous step from the neighbours x - v_i
// (streaming, Eq. 1, in pull form), forms the moments of Eq. (3), relaxes the
// non-conserved ones towards Eq. (10) by their own 1/tau^a (Eq. 5), adds the
// noise of Eq. (8) on moments 3..8, transforms back with n_i^a = w_i m_i^a
// and stores the nine new values at x.  Population planes are SoA, so every
// wave's loads and stores are contiguous 64-site runs of one plane.  There is
// no dense contraction here: the 9x9 transforms are written out using the
// sign structure of Eq. (9), about forty adds each way.
#include "flb_device.h"

namespace flbdev {

// Eq. (5) for one site on deviations d_i = f_i - w_i rho0, in place.
// Moments are kept in a scaled basis so the back transform has unit
// coefficients: s3 = 3/2 M^3, s4 = 3 M^4, s5 = M^5, s6 = sqrt(3/2) M^6,
// s7 = sqrt(3/2) M^7, s8 = M^8; M^1 = sqrt(3) jx, M^2 = sqrt(3) jy.  The
// deviation from w_i rho0 shifts only M^0 (sum_i w_i m_i^a = 0 for a > 0).
// Only the change of moments 3..8, -(M^a - M^{a,0})/tau^a + xi^a, is
// transformed back and added to the gathered values: density and momentum
// ride along untouched, so FP32 weights such as 1/9 (not exact in binary)
// cannot bias them step after step; what remains is zero-mean rounding.
template <bool NOISE>
__device__ __forceinline__ void collide(float (&d)[9], const LatticeParams &P, const float (&z)[6])
{
    // only the written fmaf calls fuse: a multiply and an add are never
    // contracted by the compiler, whose choice could differ between the
    // kernels that inline this (their results must be the same bits)
#pragma clang fp contract(off)
    const float a = d[1] + d[3], b = d[2] + d[4];
    const float c = d[5] + d[7], e = d[6] + d[8];
    const float ab = a + b, ce = c + e;
    const float drho = d[0] + ab + ce;
    const float x13 = d[1] - d[3], y24 = d[2] - d[4];
    const float p57 = d[5] - d[7], p68 = d[6] - d[8];
    const float q68 = p57 - p68, r68 = p57 + p68;  // shared with g6, g7
    const float jx = x13 + q68;
    const float jy = y24 + r68;

    // In the scaled basis s3 = 9/4 (a - b), s4 = 9 (c - e), s5, s6 = 3/2 g6,
    // s7 = 3/2 g7, s8, and Eq. (10): e3 = 9/4 (jx^2 - jy^2)/rho,
    // e4 = 9 jx jy/rho, e5 = 3/2 (jx^2 + jy^2)/rho, the others 0.  The
    // constant factors ride in per-lattice coefficients (fcoef): t3 =
    // 9/4 omega3 ((jx^2 - jy^2)/rho - (a - b)), t4 = 9 omega4 (jx jy/rho -
    // (c - e)), and the ghost changes are kept doubled, u6 = 2 t6 =
    // -3 omega6 g6 (+ 2 amp z), u7 = 2 t7 likewise.
    const float s5 = fmaf(0.5f, ab, fmaf(2.0f, ce, -d[0]));
    const float g6 = fmaf(2.0f, q68, -x13);
    const float g7 = fmaf(2.0f, r68, -y24);
    const float s8 = fmaf(0.5f, d[0], fmaf(2.0f, ce, -ab));
    const float ir = __builtin_amdgcn_rcpf(P.rho0 + drho);
    const float jyy = jy * jy;

    // change of each scaled moment, Eq. (5) and Eq. (8)
    float t3 = P.fcoef[0] * fmaf(fmaf(jx, jx, -jyy), ir, -(a - b));
    float t4 = P.fcoef[1] * fmaf(jx * jy, ir, -(c - e));
    float t5 = P.omega[2] * fmaf(1.5f * fmaf(jx, jx, jyy), ir, -s5);
    float u6 = P.fcoef[2] * g6;
    float u7 = P.fcoef[3] * g7;
    float t8 = -P.omega[5] * s8;
    if constexpr (NOISE) {
        t3 = fmaf(P.amp[0], z[0], t3);
        t4 = fmaf(P.amp[1], z[1], t4);
        t5 = fmaf(P.amp[2], z[2], t5);
        u6 = fmaf(P.fcoef[4], z[3], u6);
        u7 = fmaf(P.fcoef[5], z[4], u7);
        t8 = fmaf(P.amp[5], z[5], t8);
    }

    // d*_i = d_i + w_i sum_{a>=3} m_i^a dM^a
    const float A = fmaf(0.5f, t5, -t8);
    const float B = 2.0f * (t5 + t8);
    const float PpQ = u6 + u7, PmQ = u6 - u7;  // 2 t6 +- 2 t7
    const float Ap = A + t3, Am = A - t3;
    constexpr float w0 = 4.0f / 9.0f, w1 = 1.0f / 9.0f, w5 = 1.0f / 36.0f;
    d[0] = fmaf(w0, fmaf(0.5f, t8, -t5), d[0]);
    d[1] = fmaf(w1, fmaf(-0.5f, u6, Ap), d[1]);
    d[3] = fmaf(w1, fmaf(0.5f, u6, Ap), d[3]);
    d[2] = fmaf(w1, fmaf(-0.5f, u7, Am), d[2]);
    d[4] = fmaf(w1, fmaf(0.5f, u7, Am), d[4]);
    d[5] = fmaf(w5, (B + t4) + PpQ, d[5]);
    d[6] = fmaf(w5, (B - t4) - PmQ, d[6]);
    d[7] = fmaf(w5, (B + t4) - PpQ, d[7]);
    d[8] = fmaf(w5, (B - t4) + PmQ, d[8]);
}

// The same collision for the 16-bit formats, on the stored scaled
// deviations q_i = (d_i - F_i) / s_i themselves (F the deviation of the
// reference state f^0(rho0, u0), s_i = sqrt(mu rho0 w_i) one scale per
// velocity class): every moment above is a linear function of the d_i, so
// it is the class-scaled sum of the q_i plus the moment of F, and the
// change of d_i, w_i sum_a m_i^a dM^a, is a change of q_i by w_i / s_i times
// that sum.  No value is decoded to d or encoded back one by one.
template <bool NOISE>
__device__ __forceinline__ void collide_q(float (&q)[9], const LatticeParams &P,
                                          const float (&z)[6])
{
#pragma clang fp contract(off)  // as in collide
    const float *C = P.qcoef, *K = P.qoff;
    const float qa = q[1] + q[3], qb = q[2] + q[4];
    const float qc = q[5] + q[7], qe = q[6] + q[8];
    const float qab = qa + qb, qce = qc + qe;
    const float qx = q[1] - q[3], qy = q[2] - q[4];
    const float qp = q[5] - q[7], qm = q[6] - q[8];
    const float pmm = qp - qm, ppm = qp + qm;
    // C: s0, s1, s5, 9/4 s1, 9 s5, s1/2, 2 s5, 3 s5, 3/2 s1, s0/2
    const float drho = fmaf(C[0], q[0], fmaf(C[1], qab, fmaf(C[2], qce, K[0])));
    const float jx = fmaf(C[1], qx, fmaf(C[2], pmm, K[1]));
    const float jy = fmaf(C[1], qy, fmaf(C[2], ppm, K[2]));
    const float s3 = fmaf(C[3], qa - qb, K[3]);
    const float s4 = fmaf(C[4], qc - qe, K[4]);
    const float s5 = fmaf(C[5], qab, fmaf(C[6], qce, fmaf(-C[0], q[0], K[5])));
    const float s6 = fmaf(C[7], pmm, fmaf(-C[8], qx, K[6]));
    const float s7 = fmaf(C[7], ppm, fmaf(-C[8], qy, K[7]));
    const float s8 = fmaf(C[9], q[0], fmaf(C[6], qce, fmaf(-C[1], qab, K[8])));

    // Eq. (10), relaxation and noise exactly as in collide()
    const float ir = __builtin_amdgcn_rcpf(P.rho0 + drho);
    const float jxx = jx * jx, jyy = jy * jy;
    const float e3 = 2.25f * (jxx - jyy) * ir;
    const float e4 = 9.0f * (jx * jy) * ir;
    const float e5 = 1.5f * (jxx + jyy) * ir;
    float t3 = P.omega[0] * (e3 - s3);
    float t4 = P.omega[1] * (e4 - s4);
    float t5 = P.omega[2] * (e5 - s5);
    float t6 = -P.omega[3] * s6;
    float t7 = -P.omega[4] * s7;
    float t8 = -P.omega[5] * s8;
    if constexpr (NOISE) {
        t3 = fmaf(P.amp[0], z[0], t3);
        t4 = fmaf(P.amp[1], z[1], t4);
        t5 = fmaf(P.amp[2], z[2], t5);
        t6 = fmaf(P.amp[3], z[3], t6);
        t7 = fmaf(P.amp[4], z[4], t7);
        t8 = fmaf(P.amp[5], z[5], t8);
    }
    // q*_i = q_i + (w_i / s_i) sum_{a>=3} m_i^a dM^a
    const float A = fmaf(0.5f, t5, -t8);
    const float B = 2.0f * (t5 + t8);
    const float P6 = 2.0f * t6, Q7 = 2.0f * t7;
    const float w0 = P.qback[0], w1 = P.qback[1], w5 = P.qback[2];
    q[0] = fmaf(w0, fmaf(0.5f, t8, -t5), q[0]);
    q[1] = fmaf(w1, (A + t3) - t6, q[1]);
    q[3] = fmaf(w1, (A + t3) + t6, q[3]);
    q[2] = fmaf(w1, (A - t3) - t7, q[2]);
    q[4] = fmaf(w1, (A - t3) + t7, q[4]);
    q[5] = fmaf(w5, (B + t4) + (P6 + Q7), q[5]);
    q[6] = fmaf(w5, (B - t4) - (P6 - Q7), q[6]);
    q[7] = fmaf(w5, (B + t4) - (P6 + Q7), q[7]);
    q[8] = fmaf(w5, (B - t4) + (P6 - Q7), q[8]);
}

// The step kernels' working value of a stored population: the FP32
// deviation itself, or for the 16-bit formats the stored scaled deviation
// (collide_q works on it); `out` rounds a working value to the storage
// format (materialised in FP32 first: see round_point).
template <int S> struct Work {
    using T = typename Codec<S>::T;
    static __device__ __forceinline__ float in(T v) { return (float)v; }
    static __device__ __forceinline__ T out(float x)
    {
        if constexpr (S == kF32) return x;
        else return (T)round_point(x);
    }
};

struct StepArgs {
    const void *src;
    void *dst;
    const LatticeParams *params;
    const StepItem *items;
    const uint32_t *step;
    uint32_t step_add;
    uint32_t key0, key1;
};

// Collision of one site, including its noise draw, on working values
// (Work<S>).
template <bool NOISE, int S>
__device__ __forceinline__ void update_site(float (&d)[9], const LatticeParams &P, uint32_t site,
                                            uint32_t t, uint32_t key0, uint32_t key1)
{
    float z[6] = {0, 0, 0, 0, 0, 0};
    if constexpr (NOISE) normals6(philox4x32_10(make_uint4(site, t, P.stream_id, 0u), key0, key1), z);
    if constexpr (S == kF32) collide<NOISE>(d, P, z);
    else collide_q<NOISE>(d, P, z);
}

// V consecutive values of one storage row, as one vector access.
template <typename T, int V> struct Vec {
    typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T> struct Vec<T, 1> {
    typedef T type;
};
template <typename T, int V>
__device__ __forceinline__ T lane(const typename Vec<T, V>::type &v, int k)
{
    if constexpr (V == 1) return v;
    else return v[k];
}

// A block covers a tile of TX threads along x by kThreads/TX rows; a thread
// updates V consecutive sites x0 .. x0+V-1 of its row.  Storage rows have a
// pitch px (a multiple of 4), so the V values of one population are one
// aligned vector access.  A population streaming along +x needs the value
// left of the group (x0 - 1, periodic) and one streaming along -x the value
// right of it (x0 + V): one extra scalar load each.  A group reaching past
// the last site of a row (nx not a multiple of V) takes the site-by-site path.
// Element `off` of a lattice's buffer through a 32-bit byte offset (a
// lattice's populations are limited to 4 GiB), so that the address is a
// scalar base plus a 32-bit vector offset.
template <typename U, typename T> __device__ __forceinline__ const U *at(const T *base, uint32_t off)
{
    return reinterpret_cast<const U *>(reinterpret_cast<const char *>(base) + off * (uint32_t)sizeof(T));
}
template <typename U, typename T> __device__ __forceinline__ U *at(T *base, uint32_t off)
{
    return reinterpret_cast<U *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(T));
}

template <int S, bool NT, bool NOISE, int TX, int V>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs g)
{
    using T = typename Codec<S>::T;
    using VT = typename Vec<T, V>::type;
    constexpr int TH = kThreads / TX;
    const StepItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int nx = P.nx, ny = P.ny;
    const uint32_t px = (uint32_t)P.px;
    const int tx = it.tile % P.tiles_x, ty = it.tile / P.tiles_x;
    const int x0 = (tx * TX + (int)(threadIdx.x % TX)) * V;
    const int y = ty * TH + (int)(threadIdx.x / TX);
    if (x0 >= nx || y >= ny) return;  // no barriers below: a thread may leave early
    // wave-uniform bases and unsigned 32-bit offsets: addresses are a scalar
    // base plus a vector offset, no 64-bit arithmetic per access
    const T *__restrict__ src = (const T *)g.src + P.base;
    T *__restrict__ dst = (T *)g.dst + P.base;
    const uint32_t plane = (uint32_t)P.plane;
    const uint32_t t = *g.step + g.step_add;
    const uint32_t ym = (y == 0) ? ny - 1 : y - 1;
    const uint32_t yp = (y == ny - 1) ? 0 : y + 1;
    const uint32_t rc = (uint32_t)y * px, rm = ym * px, rp = yp * px;
    const uint32_t ux0 = (uint32_t)x0;
    const uint32_t xm = (x0 == 0) ? nx - 1 : x0 - 1;  // left of the group
    const uint32_t site0 = (uint32_t)(y * nx + x0);   // noise counter of site x0

    if (x0 + V <= nx) {
        const uint32_t xr = (x0 + V == nx) ? 0u : (uint32_t)(x0 + V);  // right of the group
        // pull: population i arrives from x - v_i.  With streaming stores the
        // group's own values are read with the non-temporal hint too; the
        // edge values stay ordinary loads, as their lines are shared with the
        // neighbouring groups.
        const VT a0 = gload<NT>(at<VT>(src, rc + ux0));
        const VT a1 = gload<NT>(at<VT>(src, 1 * plane + rc + ux0));
        const VT a2 = gload<NT>(at<VT>(src, 2 * plane + rm + ux0));
        const VT a3 = gload<NT>(at<VT>(src, 3 * plane + rc + ux0));
        const VT a4 = gload<NT>(at<VT>(src, 4 * plane + rp + ux0));
        const VT a5 = gload<NT>(at<VT>(src, 5 * plane + rm + ux0));
        const VT a6 = gload<NT>(at<VT>(src, 6 * plane + rm + ux0));
        const VT a7 = gload<NT>(at<VT>(src, 7 * plane + rp + ux0));
        const VT a8 = gload<NT>(at<VT>(src, 8 * plane + rp + ux0));
        const T e1 = *at<T>(src, 1 * plane + rc + xm), e5 = *at<T>(src, 5 * plane + rm + xm);
        const T e8 = *at<T>(src, 8 * plane + rp + xm);
        const T e3 = *at<T>(src, 3 * plane + rc + xr), e6 = *at<T>(src, 6 * plane + rm + xr);
        const T e7 = *at<T>(src, 7 * plane + rp + xr);
        T o[9][V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            float d[9];
            d[0] = Work<S>::in(lane<T, V>(a0, k));
            d[2] = Work<S>::in(lane<T, V>(a2, k));
            d[4] = Work<S>::in(lane<T, V>(a4, k));
            d[1] = Work<S>::in(k > 0 ? lane<T, V>(a1, k - 1) : e1);
            d[5] = Work<S>::in(k > 0 ? lane<T, V>(a5, k - 1) : e5);
            d[8] = Work<S>::in(k > 0 ? lane<T, V>(a8, k - 1) : e8);
            d[3] = Work<S>::in(k < V - 1 ? lane<T, V>(a3, k + 1) : e3);
            d[6] = Work<S>::in(k < V - 1 ? lane<T, V>(a6, k + 1) : e6);
            d[7] = Work<S>::in(k < V - 1 ? lane<T, V>(a7, k + 1) : e7);
            update_site<NOISE, S>(d, P, site0 + (uint32_t)k, t, g.key0, g.key1);
#pragma unroll
            for (int i = 0; i < 9; ++i) o[i][k] = Work<S>::out(d[i]);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            VT v;
            if constexpr (V == 1) {
                v = o[i][0];
            } else {
#pragma unroll
                for (int k = 0; k < V; ++k) v[k] = o[i][k];
            }
            gstore<NT>(at<VT>(dst, i * plane + rc + ux0), v);
        }
    } else {
        for (int x = x0; x < nx; ++x) {
            const uint32_t ux = (uint32_t)x;
            const uint32_t xl = (x == 0) ? nx - 1 : x - 1, xr = (x == nx - 1) ? 0 : x + 1;
            float d[9];
            d[0] = Work<S>::in(*at<T>(src, rc + ux));
            d[1] = Work<S>::in(*at<T>(src, 1 * plane + rc + xl));
            d[2] = Work<S>::in(*at<T>(src, 2 * plane + rm + ux));
            d[3] = Work<S>::in(*at<T>(src, 3 * plane + rc + xr));
            d[4] = Work<S>::in(*at<T>(src, 4 * plane + rp + ux));
            d[5] = Work<S>::in(*at<T>(src, 5 * plane + rm + xl));
            d[6] = Work<S>::in(*at<T>(src, 6 * plane + rm + xr));
            d[7] = Work<S>::in(*at<T>(src, 7 * plane + rp + xr));
            d[8] = Work<S>::in(*at<T>(src, 8 * plane + rp + xl));
            update_site<NOISE, S>(d, P, (uint32_t)(y * nx + x), t, g.key0, g.key1);
#pragma unroll
            for (int i = 0; i < 9; ++i) gstore<NT>(at<T>(dst, i * plane + rc + ux), Work<S>::out(d[i]));
        }
    }
}

template <int S, bool NT, bool NOISE>
static hipError_t launch_step_tiles(const StepArgs &a, int nitems, int tx, int v, hipStream_t s)
{
    const dim3 grid(nitems), block(kThreads);
#define FLB_TILE(TX_, V_)                                                                     \
    if (tx == TX_ && v == V_) {                                                               \
        hipLaunchKernelGGL((step_kernel<S, NT, NOISE, TX_, V_>), grid, block, 0, s, a);       \
        return hipGetLastError();                                                             \
    }
    FLB_TILE(64, 1)
    FLB_TILE(128, 1)
    FLB_TILE(256, 1)
    FLB_TILE(64, 2)
    FLB_TILE(128, 2)
    FLB_TILE(256, 2)
    FLB_TILE(64, 4)
    FLB_TILE(128, 4)
    FLB_TILE(256, 4)
#undef FLB_TILE
    return hipErrorInvalidValue;
}

bool step_tile_supported(int tx, int v)
{
    return (tx == 64 || tx == 128 || tx == 256) && (v == 1 || v == 2 || v == 4);
}

hipError_t launch_step(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                       int sites, uint32_t step_add, bool nontemporal, bool noise, hipStream_t s)
{
    StepArgs a;
    a.src = v.pops[v.cur];
    a.dst = v.pops[v.cur ^ 1];
    a.params = v.params;
    a.items = items;
    a.step = v.step;
    a.step_add = step_add;
    a.key0 = (uint32_t)(v.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(v.seed >> 32);
#define FLB_SEL(S_)                                                                              \
    if (v.storage == S_) {                                                                       \
        if (nontemporal)                                                                         \
            return noise ? launch_step_tiles<S_, true, true>(a, nitems, tile_w, sites, s)        \
                         : launch_step_tiles<S_, true, false>(a, nitems, tile_w, sites, s);      \
        return noise ? launch_step_tiles<S_, false, true>(a, nitems, tile_w, sites, s)           \
                     : launch_step_tiles<S_, false, false>(a, nitems, tile_w, sites, s);         \
    }
    FLB_SEL(kF32)
    FLB_SEL(kBF16)
    FLB_SEL(kF16)
#undef FLB_SEL
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------
// Two steps per launch (time blocking).  A block owns a tile of TW x TH
// sites.  Phase 1 collides the tile and the one-site ring around it at time
// t (each site pulled from HBM as in the one-step kernel, the ring
// recomputed by the neighbouring blocks too) and keeps the post-collision
// values in LDS in the storage format; phase 2 pulls the tile's values from
// LDS, collides them at t + 1 and stores them.  Every site goes through the
// same update function, noise counters and storage rounding as in two
// one-step launches, so the results are the same; the populations cross HBM
// once per two steps.
//
// Each thread collides the same tile sites in both phases (and one ring
// site in phase 1), so the rest population, which streams from the site
// itself, stays in a register: LDS holds planes 1..8 only (38 KB for a
// 64 x 16 tile in FP32).  All of a thread's phase-1 loads are
// issued before its first collision.
// ---------------------------------------------------------------------
constexpr int kStep2Threads = 512;

// Tile shapes of the two-step kernel: TW x TH = 1024 sites, TW a power of
// two.  Fixed carries the shape at compile time; Dyn at run time, so that
// one kernel body serves tiles of several shapes (the kernel's registers
// stay those of one shape).
template <int TW_, int TH_> struct Fixed {
    static_assert(TW_ * TH_ == 1024 && (TW_ & (TW_ - 1)) == 0, "tile shape");
    static constexpr int tw = TW_, th = TH_, rw = TW_ + 2, rn = (TW_ + 2) * (TH_ + 2);
    static constexpr int lg = TW_ == 32 ? 5 : TW_ == 64 ? 6 : TW_ == 128 ? 7 : 8;
};
struct Dyn {
    int tw, th, rw, rn, lg;
    __device__ explicit Dyn(int lg_) : tw(1 << lg_), th(1024 >> lg_), rw(tw + 2),
                                       rn((tw + 2) * (th + 2)), lg(lg_) {}
};

// region coordinates of the h-th site of the one-site ring around a tile
template <class SH>
__device__ __forceinline__ void ring_site(const SH &sh, int h, int &rx, int &ry)
{
    const int RW = sh.rw, TH = sh.th;
    if (h < RW) {
        ry = 0;
        rx = h;
    } else if (h < 2 * RW) {
        ry = TH + 1;
        rx = h - RW;
    } else if (h < 2 * RW + TH) {
        ry = h - 2 * RW + 1;
        rx = 0;
    } else {
        ry = h - 2 * RW - TH + 1;
        rx = RW - 1;
    }
}

// One tile's two steps; mid holds 8 x sh.rn values of LDS (planes 1..8
// after phase 1, plane-major).
template <int S, bool NT, bool NOISE, class SH>
__device__ __forceinline__ void step2_tile(const StepArgs &g, StepItem it, const SH sh,
                                           typename Codec<S>::T *__restrict__ mid)
{
    using T = typename Codec<S>::T;
    const int TW = sh.tw, TH = sh.th, RW = sh.rw, RN = sh.rn;
    constexpr int NTILE = 1024;
    const int NRING = RN - NTILE;              // at most 276 (128 x 8), below the thread count
    constexpr int KT = NTILE / kStep2Threads;  // tile sites per thread
    constexpr int K = KT + 1;                  // phase-1 sites per thread: tile sites, then a ring site
    static_assert(NTILE % kStep2Threads == 0, "tile shape");
    const LatticeParams &P = g.params[it.lattice];
    const int nx = P.nx, ny = P.ny;
    const int tiles_x = (nx + TW - 1) >> sh.lg;
    const int x0 = (it.tile % tiles_x) * TW, y0 = (it.tile / tiles_x) * TH;
    const T *__restrict__ src = (const T *)g.src + P.base;
    T *__restrict__ dst = (T *)g.dst + P.base;
    const uint32_t plane = (uint32_t)P.plane, px = (uint32_t)P.px;
    const uint32_t t = *g.step + g.step_add;
    const int tid = threadIdx.x;

    // An interior tile: the region and every site it pulls from lie inside
    // the lattice, so no coordinate wraps and each plane's pull is one
    // fixed shift of the site's own offset (block-uniform test).
    const bool interior = x0 >= 2 && y0 >= 2 && x0 + TW + 2 <= nx && y0 + TH + 2 <= ny;

    // phase-1 sites: region index and (wrapped) lattice coordinates
    int xs[K], ys[K], rs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int rx, ry;
        if (k < KT) {
            const int o = tid + k * kStep2Threads;
            ry = (o >> sh.lg) + 1;
            rx = (o & (TW - 1)) + 1;
        } else {
            ring_site(sh, tid < NRING ? tid : 0, rx, ry);
        }
        rs[k] = ry * RW + rx;
        xs[k] = x0 - 1 + rx;
        ys[k] = y0 - 1 + ry;
    }
    if (!interior) {
        // wrap (x >= -1): at most one subtraction unless the lattice is
        // smaller than a tile
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int x = xs[k], y = ys[k];
            x = x < 0 ? x + nx : x;
            y = y < 0 ? y + ny : y;
            while (x >= nx) x -= nx;
            while (y >= ny) y -= ny;
            xs[k] = x;
            ys[k] = y;
        }
    }
    // per-plane bases (wave-uniform) and byte offsets within a plane
    const char *sp[9];
    char *dp[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        sp[i] = reinterpret_cast<const char *>(src) + (size_t)i * plane * sizeof(T);
        dp[i] = reinterpret_cast<char *>(dst) + (size_t)i * plane * sizeof(T);
    }
    constexpr uint32_t E = sizeof(T);
    T raw[K][9];
    if (interior) {
        // plane i pulls from x - v_i: its base shifted by -(v_iy px + v_ix)
        // values, so one vector offset serves all nine loads of a site
        const int64_t row = (int64_t)px * E;
        const char *const sh0 = sp[0];
        const char *const sh1 = sp[1] - (int64_t)E;
        const char *const sh2 = sp[2] - row;
        const char *const sh3 = sp[3] + (int64_t)E;
        const char *const sh4 = sp[4] + row;
        const char *const sh5 = sp[5] - row - (int64_t)E;
        const char *const sh6 = sp[6] - row + (int64_t)E;
        const char *const sh7 = sp[7] + row + (int64_t)E;
        const char *const sh8 = sp[8] + row - (int64_t)E;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k == KT && tid >= NRING) break;
            const uint32_t o = ((uint32_t)ys[k] * px + (uint32_t)xs[k]) * E;
            raw[k][0] = *reinterpret_cast<const T *>(sh0 + o);
            raw[k][1] = *reinterpret_cast<const T *>(sh1 + o);
            raw[k][2] = *reinterpret_cast<const T *>(sh2 + o);
            raw[k][3] = *reinterpret_cast<const T *>(sh3 + o);
            raw[k][4] = *reinterpret_cast<const T *>(sh4 + o);
            raw[k][5] = *reinterpret_cast<const T *>(sh5 + o);
            raw[k][6] = *reinterpret_cast<const T *>(sh6 + o);
            raw[k][7] = *reinterpret_cast<const T *>(sh7 + o);
            raw[k][8] = *reinterpret_cast<const T *>(sh8 + o);
        }
    } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k == KT && tid >= NRING) break;
        const int x = xs[k], y = ys[k];
        const uint32_t ux = (uint32_t)x * E;
        const uint32_t xm = (uint32_t)(x == 0 ? nx - 1 : x - 1) * E;
        const uint32_t xr = (uint32_t)(x == nx - 1 ? 0 : x + 1) * E;
        const uint32_t rc = (uint32_t)y * px * E, rm = (uint32_t)(y == 0 ? ny - 1 : y - 1) * px * E;
        const uint32_t rp = (uint32_t)(y == ny - 1 ? 0 : y + 1) * px * E;
        raw[k][0] = *reinterpret_cast<const T *>(sp[0] + (rc + ux));
        raw[k][1] = *reinterpret_cast<const T *>(sp[1] + (rc + xm));
        raw[k][2] = *reinterpret_cast<const T *>(sp[2] + (rm + ux));
        raw[k][3] = *reinterpret_cast<const T *>(sp[3] + (rc + xr));
        raw[k][4] = *reinterpret_cast<const T *>(sp[4] + (rp + ux));
        raw[k][5] = *reinterpret_cast<const T *>(sp[5] + (rm + xm));
        raw[k][6] = *reinterpret_cast<const T *>(sp[6] + (rm + xr));
        raw[k][7] = *reinterpret_cast<const T *>(sp[7] + (rp + xr));
        raw[k][8] = *reinterpret_cast<const T *>(sp[8] + (rp + xm));
    }
    }
    T own[KT];  // plane 0 of the tile sites after phase 1, in the storage format
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k == KT && tid >= NRING) break;
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Work<S>::in(raw[k][i]);
        update_site<NOISE, S>(d, P, (uint32_t)(ys[k] * nx + xs[k]), t, g.key0, g.key1);
        if (k < KT) own[k] = Work<S>::out(d[0]);
#pragma unroll
        for (int i = 1; i < 9; ++i) mid[(i - 1) * RN + rs[k]] = Work<S>::out(d[i]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        const int o = tid + k * kStep2Threads;
        const int oy = o >> sh.lg, ox = o & (TW - 1);
        const int x = x0 + ox, y = y0 + oy;
        if (x >= nx || y >= ny) continue;
        const int c = rs[k];
        float d[9];
        d[0] = Work<S>::in(own[k]);
        d[1] = Work<S>::in(mid[0 * RN + c - 1]);
        d[2] = Work<S>::in(mid[1 * RN + c - RW]);
        d[3] = Work<S>::in(mid[2 * RN + c + 1]);
        d[4] = Work<S>::in(mid[3 * RN + c + RW]);
        d[5] = Work<S>::in(mid[4 * RN + c - RW - 1]);
        d[6] = Work<S>::in(mid[5 * RN + c - RW + 1]);
        d[7] = Work<S>::in(mid[6 * RN + c + RW + 1]);
        d[8] = Work<S>::in(mid[7 * RN + c + RW - 1]);
        update_site<NOISE, S>(d, P, (uint32_t)(y * nx + x), t + 1, g.key0, g.key1);
        const uint32_t off = ((uint32_t)y * px + (uint32_t)x) * E;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            gstore<NT>(reinterpret_cast<T *>(dp[i] + off), Work<S>::out(d[i]));
    }
}

// Every tile of the launch has the shape TW x TH.  (A CU holds three
// blocks: 65-71 registers a thread; a budget of 64 for four blocks of the
// 38 KB FP32 tiles made the compiler spill, and the spills cost 5 % more
// HBM bytes than the fourth block gained.)
template <int S, bool NT, bool NOISE, int TW, int TH>
__global__ __launch_bounds__(kStep2Threads) void step2_kernel(StepArgs g)
{
    using T = typename Codec<S>::T;
    using SH = Fixed<TW, TH>;
    __shared__ T mid[8 * SH::rn];
    const StepItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    step2_tile<S, NT, NOISE>(g, it, SH{}, mid);
}

// Each work item has its own tile shape: 32 x 32 when the tile index
// carries kStep2Square, else 64 x 16 (a lattice's items all have the same
// shape).  The two shapes need about the same LDS (37 and 38 KB in FP32),
// so a batch can give each lattice the shape that fits its sides in one
// launch.
template <int S, bool NT, bool NOISE>
__global__ __launch_bounds__(kStep2Threads) void step2_mixed_kernel(StepArgs g)
{
    using T = typename Codec<S>::T;
    constexpr int RN = Fixed<32, 32>::rn > Fixed<64, 16>::rn ? Fixed<32, 32>::rn : Fixed<64, 16>::rn;
    __shared__ T mid[8 * RN];
    StepItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const bool square = (it.tile & kStep2Square) != 0;
    it.tile &= ~kStep2Square;
    step2_tile<S, NT, NOISE>(g, it, Dyn(square ? 5 : 6), mid);
}

template <int S, bool NT, bool NOISE>
static hipError_t launch_step2_tiles(const StepArgs &a, int nitems, int tw, hipStream_t s)
{
    const dim3 grid(nitems), block(kStep2Threads);
    if (tw == 64)
        hipLaunchKernelGGL((step2_kernel<S, NT, NOISE, 64, 16>), grid, block, 0, s, a);
    else if (tw == 128)
        hipLaunchKernelGGL((step2_kernel<S, NT, NOISE, 128, 8>), grid, block, 0, s, a);
    else if (tw == 32)
        hipLaunchKernelGGL((step2_kernel<S, NT, NOISE, 32, 32>), grid, block, 0, s, a);
    else if (tw == 0)
        hipLaunchKernelGGL((step2_mixed_kernel<S, NT, NOISE>), grid, block, 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

bool step2_tile_supported(int tw) { return tw == 32 || tw == 64 || tw == 128; }

hipError_t launch_step2(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                        uint32_t step_add, bool nontemporal, bool noise, hipStream_t s)
{
    StepArgs a;
    a.src = v.pops[v.cur];
    a.dst = v.pops[v.cur ^ 1];
    a.params = v.params;
    a.items = items;
    a.step = v.step;
    a.step_add = step_add;
    a.key0 = (uint32_t)(v.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(v.seed >> 32);
#define FLB_SEL(S_)                                                                              \
    if (v.storage == S_) {                                                                       \
        if (nontemporal)                                                                         \
            return noise ? launch_step2_tiles<S_, true, true>(a, nitems, tile_w, s)              \
                         : launch_step2_tiles<S_, true, false>(a, nitems, tile_w, s);            \
        return noise ? launch_step2_tiles<S_, false, true>(a, nitems, tile_w, s)                 \
                     : launch_step2_tiles<S_, false, false>(a, nitems, tile_w, s);               \
    }
    FLB_SEL(kF32)
    FLB_SEL(kBF16)
    FLB_SEL(kF16)
#undef FLB_SEL
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------
// Three steps per launch.  A block owns a TW x TH tile; its region adds two
// rings of sites.  Phase 1 collides the whole region at t (each site pulled
// from HBM), phase 2 the tile and the inner ring at t + 1 (pulled from
// phase 1's values in LDS), phase 3 the tile at t + 2, which it stores.
// Every intermediate value is rounded to the storage format, so the
// results are the bits of three one-step launches; the populations cross
// HBM once per three steps.  A thread keeps its sites across the phases
// (its two tile sites in all three, its inner-ring site in the first two,
// its outer-ring site in the first), so a site's rest population stays in a
// register and LDS holds planes 1..8 of the region.  Phase 2 reads all its
// inputs before a barrier and then overwrites them in place.
// ---------------------------------------------------------------------

// region coordinates of the h-th site of the one-site ring around a w x hh
// box whose top-left site is at region (1, 1); the ring spans [0, w + 2) x
// [0, hh + 2)
__device__ __forceinline__ void ring_box(int w, int hh, int h, int &rx, int &ry)
{
    const int RW = w + 2;
    if (h < RW) {
        ry = 0;
        rx = h;
    } else if (h < 2 * RW) {
        ry = hh + 1;
        rx = h - RW;
    } else if (h < 2 * RW + hh) {
        ry = h - 2 * RW + 1;
        rx = 0;
    } else {
        ry = h - 2 * RW - hh + 1;
        rx = RW - 1;
    }
}

// (FP32: the register budget of six waves per SIMD, three blocks per CU as
// the 51 KB of LDS of a 128 x 8 region allow.)
template <int S, bool NT, bool NOISE, int TW, int TH>
__global__ __launch_bounds__(kStep2Threads)
__attribute__((amdgpu_waves_per_eu(S == kF32 ? 6 : 4))) void step3_kernel(StepArgs g)
{
    using T = typename Codec<S>::T;
    static_assert(TW * TH == 1024 && (TW & (TW - 1)) == 0, "tile shape");
    constexpr int RW = TW + 4, RN = RW * (TH + 4);
    constexpr int N1 = 2 * (TW + 2) + 2 * TH;        // inner ring
    constexpr int N2 = 2 * (TW + 4) + 2 * (TH + 2);  // outer ring
    constexpr int KT = 1024 / kStep2Threads;        // tile sites per thread
    constexpr int K = KT + 2;                       // phase-1 slots: tile, inner, outer
    static_assert(N1 <= kStep2Threads && N2 <= kStep2Threads, "tile shape");
    constexpr int LG = TW == 32 ? 5 : TW == 64 ? 6 : 7;
    __shared__ T mid[8 * RN];  // planes 1..8 of the region
    const StepItem it = g.items[blockIdx.x];
    if (it.lattice < 0) return;
    const LatticeParams &P = g.params[it.lattice];
    const int nx = P.nx, ny = P.ny;
    const int tiles_x = (nx + TW - 1) >> LG;
    const int x0 = (it.tile % tiles_x) * TW, y0 = (it.tile / tiles_x) * TH;
    const T *__restrict__ src = (const T *)g.src + P.base;
    T *__restrict__ dst = (T *)g.dst + P.base;
    const uint32_t plane = (uint32_t)P.plane, px = (uint32_t)P.px;
    const uint32_t t = *g.step + g.step_add;
    const int tid = threadIdx.x;
    const bool has1 = tid < N1, has2 = tid >= kStep2Threads - N2;
    const bool interior = x0 >= 3 && y0 >= 3 && x0 + TW + 3 <= nx && y0 + TH + 3 <= ny;

    // slots: 0 .. KT-1 tile sites, KT the inner-ring site, KT+1 the outer
    int xs[K], ys[K], rs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int rx, ry;
        if (k < KT) {
            const int o = tid + k * kStep2Threads;
            ry = (o >> LG) + 2;
            rx = (o & (TW - 1)) + 2;
        } else if (k == KT) {
            ring_box(TW, TH, has1 ? tid : 0, rx, ry);
            rx += 1;
            ry += 1;
        } else {
            ring_box(TW + 2, TH + 2, has2 ? tid - (kStep2Threads - N2) : 0, rx, ry);
        }
        rs[k] = ry * RW + rx;
        xs[k] = x0 - 2 + rx;
        ys[k] = y0 - 2 + ry;
    }
    if (!interior) {
        // wrap (x >= -2, nx >= 2): at most one subtraction unless the
        // lattice is smaller than a tile
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int x = xs[k], y = ys[k];
            x = x < 0 ? x + nx : x;
            y = y < 0 ? y + ny : y;
            while (x >= nx) x -= nx;
            while (y >= ny) y -= ny;
            xs[k] = x;
            ys[k] = y;
        }
    }
    const char *sp[9];
    char *dp[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        sp[i] = reinterpret_cast<const char *>(src) + (size_t)i * plane * sizeof(T);
        dp[i] = reinterpret_cast<char *>(dst) + (size_t)i * plane * sizeof(T);
    }
    constexpr uint32_t E = sizeof(T);
    auto active = [&](int k) { return k < KT || (k == KT ? has1 : has2); };

    // phase 1 (t): every region site, pulled from HBM
    T raw[K][9];
    if (interior) {
        const int64_t row = (int64_t)px * E;
        const char *const sh0 = sp[0];
        const char *const sh1 = sp[1] - (int64_t)E;
        const char *const sh2 = sp[2] - row;
        const char *const sh3 = sp[3] + (int64_t)E;
        const char *const sh4 = sp[4] + row;
        const char *const sh5 = sp[5] - row - (int64_t)E;
        const char *const sh6 = sp[6] - row + (int64_t)E;
        const char *const sh7 = sp[7] + row + (int64_t)E;
        const char *const sh8 = sp[8] + row - (int64_t)E;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!active(k)) continue;
            const uint32_t o = ((uint32_t)ys[k] * px + (uint32_t)xs[k]) * E;
            raw[k][0] = *reinterpret_cast<const T *>(sh0 + o);
            raw[k][1] = *reinterpret_cast<const T *>(sh1 + o);
            raw[k][2] = *reinterpret_cast<const T *>(sh2 + o);
            raw[k][3] = *reinterpret_cast<const T *>(sh3 + o);
            raw[k][4] = *reinterpret_cast<const T *>(sh4 + o);
            raw[k][5] = *reinterpret_cast<const T *>(sh5 + o);
            raw[k][6] = *reinterpret_cast<const T *>(sh6 + o);
            raw[k][7] = *reinterpret_cast<const T *>(sh7 + o);
            raw[k][8] = *reinterpret_cast<const T *>(sh8 + o);
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!active(k)) continue;
            const int x = xs[k], y = ys[k];
            const uint32_t ux = (uint32_t)x * E;
            const uint32_t xm = (uint32_t)(x == 0 ? nx - 1 : x - 1) * E;
            const uint32_t xr = (uint32_t)(x == nx - 1 ? 0 : x + 1) * E;
            const uint32_t rc = (uint32_t)y * px * E;
            const uint32_t rm = (uint32_t)(y == 0 ? ny - 1 : y - 1) * px * E;
            const uint32_t rp = (uint32_t)(y == ny - 1 ? 0 : y + 1) * px * E;
            raw[k][0] = *reinterpret_cast<const T *>(sp[0] + (rc + ux));
            raw[k][1] = *reinterpret_cast<const T *>(sp[1] + (rc + xm));
            raw[k][2] = *reinterpret_cast<const T *>(sp[2] + (rm + ux));
            raw[k][3] = *reinterpret_cast<const T *>(sp[3] + (rc + xr));
            raw[k][4] = *reinterpret_cast<const T *>(sp[4] + (rp + ux));
            raw[k][5] = *reinterpret_cast<const T *>(sp[5] + (rm + xm));
            raw[k][6] = *reinterpret_cast<const T *>(sp[6] + (rm + xr));
            raw[k][7] = *reinterpret_cast<const T *>(sp[7] + (rp + xr));
            raw[k][8] = *reinterpret_cast<const T *>(sp[8] + (rp + xm));
        }
    }
    T own[KT + 1];  // plane 0 of the tile and inner-ring sites, storage format
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!active(k)) continue;
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Work<S>::in(raw[k][i]);
        update_site<NOISE, S>(d, P, (uint32_t)(ys[k] * nx + xs[k]), t, g.key0, g.key1);
        if (k <= KT) own[k] = Work<S>::out(d[0]);
#pragma unroll
        for (int i = 1; i < 9; ++i) mid[(i - 1) * RN + rs[k]] = Work<S>::out(d[i]);
    }
    __syncthreads();

    // phase 2 (t + 1): tile and inner ring, pulled from LDS; every read
    // before the barrier, every write after it
    T nxt[KT + 1][8];
#pragma unroll
    for (int k = 0; k <= KT; ++k) {
        if (!active(k)) continue;
        const int c = rs[k];
        float d[9];
        d[0] = Work<S>::in(own[k]);
        d[1] = Work<S>::in(mid[0 * RN + c - 1]);
        d[2] = Work<S>::in(mid[1 * RN + c - RW]);
        d[3] = Work<S>::in(mid[2 * RN + c + 1]);
        d[4] = Work<S>::in(mid[3 * RN + c + RW]);
        d[5] = Work<S>::in(mid[4 * RN + c - RW - 1]);
        d[6] = Work<S>::in(mid[5 * RN + c - RW + 1]);
        d[7] = Work<S>::in(mid[6 * RN + c + RW + 1]);
        d[8] = Work<S>::in(mid[7 * RN + c + RW - 1]);
        update_site<NOISE, S>(d, P, (uint32_t)(ys[k] * nx + xs[k]), t + 1, g.key0, g.key1);
        own[k] = Work<S>::out(d[0]);
#pragma unroll
        for (int i = 1; i < 9; ++i) nxt[k][i - 1] = Work<S>::out(d[i]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= KT; ++k) {
        if (!active(k)) continue;
#pragma unroll
        for (int i = 1; i < 9; ++i) mid[(i - 1) * RN + rs[k]] = nxt[k][i - 1];
    }
    __syncthreads();

    // phase 3 (t + 2): the tile, stored
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        const int o = tid + k * kStep2Threads;
        const int x = x0 + (o & (TW - 1)), y = y0 + (o >> LG);
        if (x >= nx || y >= ny) continue;
        const int c = rs[k];
        float d[9];
        d[0] = Work<S>::in(own[k]);
        d[1] = Work<S>::in(mid[0 * RN + c - 1]);
        d[2] = Work<S>::in(mid[1 * RN + c - RW]);
        d[3] = Work<S>::in(mid[2 * RN + c + 1]);
        d[4] = Work<S>::in(mid[3 * RN + c + RW]);
        d[5] = Work<S>::in(mid[4 * RN + c - RW - 1]);
        d[6] = Work<S>::in(mid[5 * RN + c - RW + 1]);
        d[7] = Work<S>::in(mid[6 * RN + c + RW + 1]);
        d[8] = Work<S>::in(mid[7 * RN + c + RW - 1]);
        update_site<NOISE, S>(d, P, (uint32_t)(y * nx + x), t + 2, g.key0, g.key1);
        const uint32_t off = ((uint32_t)y * px + (uint32_t)x) * E;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            gstore<NT>(reinterpret_cast<T *>(dp[i] + off), Work<S>::out(d[i]));
    }
}

template <int S, bool NT, bool NOISE>
static hipError_t launch_step3_tiles(const StepArgs &a, int nitems, int tw, hipStream_t s)
{
    const dim3 grid(nitems), block(kStep2Threads);
    if (tw == 64)
        hipLaunchKernelGGL((step3_kernel<S, NT, NOISE, 64, 16>), grid, block, 0, s, a);
    else if (tw == 128)
        hipLaunchKernelGGL((step3_kernel<S, NT, NOISE, 128, 8>), grid, block, 0, s, a);
    else if (tw == 32)
        hipLaunchKernelGGL((step3_kernel<S, NT, NOISE, 32, 32>), grid, block, 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_step3(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                        uint32_t step_add, bool nontemporal, bool noise, hipStream_t s)
{
    StepArgs a;
    a.src = v.pops[v.cur];
    a.dst = v.pops[v.cur ^ 1];
    a.params = v.params;
    a.items = items;
    a.step = v.step;
    a.step_add = step_add;
    a.key0 = (uint32_t)(v.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(v.seed >> 32);
#define FLB_SEL(S_)                                                                              \
    if (v.storage == S_) {                                                                       \
        if (nontemporal)                                                                         \
            return noise ? launch_step3_tiles<S_, true, true>(a, nitems, tile_w, s)              \
                         : launch_step3_tiles<S_, true, false>(a, nitems, tile_w, s);            \
        return noise ? launch_step3_tiles<S_, false, true>(a, nitems, tile_w, s)                 \
                     : launch_step3_tiles<S_, false, false>(a, nitems, tile_w, s);               \
    }
    FLB_SEL(kF32)
    FLB_SEL(kBF16)
    FLB_SEL(kF16)
#undef FLB_SEL
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------
// Step counter
// ---------------------------------------------------------------------
__global__ void advance_step_kernel(uint32_t *step, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += n;
}

hipError_t launch_advance_step(uint32_t *step, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, s, step, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Uniform equilibrium start, Eq. (2): every stored value is feq_i.
// ---------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(kThreads) void init_kernel(void *pops, const LatticeParams *params,
                                                        int lattice)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int64_t n = 9 * P.plane;
    T *p = (T *)pops + P.base;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / P.plane);
        p[k] = Codec<S>::encode(P.feq[i], P, i);
    }
}

static int grid_for(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

hipError_t launch_init(const DeviceView &v, int lattice, int64_t plane, hipStream_t s)
{
    const dim3 grid(grid_for(9 * plane)), block(kThreads);
    void *p = v.pops[v.cur];
    if (v.storage == kF32)
        hipLaunchKernelGGL(init_kernel<kF32>, grid, block, 0, s, p, v.params, lattice);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(init_kernel<kBF16>, grid, block, 0, s, p, v.params, lattice);
    else
        hipLaunchKernelGGL(init_kernel<kF16>, grid, block, 0, s, p, v.params, lattice);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// State export / import as full FP64 populations f_i(x) = w_i rho0 + d_i,
// with d_i(x) = stored_i(x - v_i).
// ---------------------------------------------------------------------
__device__ constexpr double kWd[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

template <int S>
__global__ __launch_bounds__(kThreads) void get_kernel(const void *pops,
                                                       const LatticeParams *params, int lattice,
                                                       double *out)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int nx = P.nx, ny = P.ny, px = P.px;
    const int64_t V = (int64_t)nx * ny, plane = P.plane;
    const T *p = (const T *)pops + P.base;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 9 * V;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / V);
        const int s = (int)(k - (int64_t)i * V);
        const int y = s / nx, x = s - y * nx;
        const int xs = wrap_add(x, -kVX[i], nx), ys = wrap_add(y, -kVY[i], ny);
        const float d = Codec<S>::decode(p[(int64_t)i * plane + ys * px + xs], P, i);
        out[k] = kWd[i] * (double)P.rho0 + (double)d;
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void set_kernel(void *pops, const LatticeParams *params,
                                                       int lattice, const double *in)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int nx = P.nx, ny = P.ny, px = P.px;
    const int64_t V = (int64_t)nx * ny, plane = P.plane;
    T *p = (T *)pops + P.base;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 9 * V;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / V);
        const int s = (int)(k - (int64_t)i * V);
        const int y = s / nx, x = s - y * nx;
        // stored_i(x) holds f_i(x + v_i)
        const int xd = wrap_add(x, kVX[i], nx), yd = wrap_add(y, kVY[i], ny);
        const double f = in[(int64_t)i * V + yd * nx + xd];
        p[(int64_t)i * plane + y * px + x] = Codec<S>::encode((float)(f - kWd[i] * (double)P.rho0), P, i);
    }
}

hipError_t launch_get(const DeviceView &v, int lattice, int nx, int ny, double *out_dev,
                      hipStream_t s)
{
    const dim3 grid(grid_for(9LL * nx * ny)), block(kThreads);
    const void *p = v.pops[v.cur];
    if (v.storage == kF32)
        hipLaunchKernelGGL(get_kernel<kF32>, grid, block, 0, s, p, v.params, lattice, out_dev);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(get_kernel<kBF16>, grid, block, 0, s, p, v.params, lattice, out_dev);
    else
        hipLaunchKernelGGL(get_kernel<kF16>, grid, block, 0, s, p, v.params, lattice, out_dev);
    return hipGetLastError();
}

hipError_t launch_set(const DeviceView &v, int lattice, int nx, int ny, const double *in_dev,
                      hipStream_t s)
{
    const dim3 grid(grid_for(9LL * nx * ny)), block(kThreads);
    void *p = v.pops[v.cur];
    if (v.storage == kF32)
        hipLaunchKernelGGL(set_kernel<kF32>, grid, block, 0, s, p, v.params, lattice, in_dev);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(set_kernel<kBF16>, grid, block, 0, s, p, v.params, lattice, in_dev);
    else
        hipLaunchKernelGGL(set_kernel<kF16>, grid, block, 0, s, p, v.params, lattice, in_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// FP64 sums: mass, momentum and the staggered momenta.  Deterministic:
// fixed per-block partials, then one block adds them in a fixed order.
// ---------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out)
{
    __shared__ double red[NV][kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) red[q][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double x = 0;
        for (int w2 = 0; w2 < kThreads / 64; ++w2) x += red[threadIdx.x][w2];
        out[threadIdx.x] = x;
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void conservation_kernel(const void *pops,
                                                                const LatticeParams *params,
                                                                int lattice, double *part)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int nx = P.nx, ny = P.ny, px = P.px;
    const int64_t V = (int64_t)nx * ny, plane = P.plane;
    const T *p = (const T *)pops + P.base;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < V;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(s / nx), x = (int)(s - (int64_t)y * nx);
        double r = 0, jx = 0, jy = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xs = wrap_add(x, -kVX[i], nx), ys = wrap_add(y, -kVY[i], ny);
            const double d = (double)Codec<S>::decode(p[(int64_t)i * plane + ys * px + xs], P, i);
            r += d;
            jx += kVX[i] * d;
            jy += kVY[i] * d;
        }
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += (x & 1) ? -jx : jx;
        acc[4] += (y & 1) ? -jy : jy;
    }
    block_sum<5>(acc, part + 5 * blockIdx.x);
}

template <int NV>
__global__ __launch_bounds__(kThreads) void reduce_parts_kernel(const double *part, int nparts,
                                                                double *out)
{
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += part[NV * b + q];
    block_sum<NV>(acc, out);
}

hipError_t launch_conservation(const DeviceView &v, int lattice, int nx, int ny, double *part,
                               int nblocks, double *out_dev, hipStream_t s)
{
    (void)nx;
    (void)ny;
    const dim3 grid(nblocks), block(kThreads);
    const void *p = v.pops[v.cur];
    if (v.storage == kF32)
        hipLaunchKernelGGL(conservation_kernel<kF32>, grid, block, 0, s, p, v.params, lattice, part);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(conservation_kernel<kBF16>, grid, block, 0, s, p, v.params, lattice,
                           part);
    else
        hipLaunchKernelGGL(conservation_kernel<kF16>, grid, block, 0, s, p, v.params, lattice, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_parts_kernel<5>, dim3(1), block, 0, s, part, nblocks, out_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Thermal start: add sqrt(mu rho0 w_i) z_i(x) to f_i(x) (stored at x - v_i),
// then subtract each population's spatial mean of what was added.
// ---------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(kThreads) void thermal_add_kernel(void *pops,
                                                               const LatticeParams *params,
                                                               int lattice, uint32_t key0,
                                                               uint32_t key1, double *part)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int nx = P.nx, ny = P.ny, px = P.px;
    const int64_t V = (int64_t)nx * ny, plane = P.plane;
    T *p = (T *)pops + P.base;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < V;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(s / nx), x = (int)(s - (int64_t)y * nx);
        float z[12];
        normals6(philox4x32_10(make_uint4((uint32_t)s, 0xFFFFFFFFu, P.stream_id, 0u), key0, key1),
                 z);
        normals6(philox4x32_10(make_uint4((uint32_t)s, 0xFFFFFFFFu, P.stream_id, 1u), key0, key1),
                 z + 6);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float add = P.therm_amp[i] * z[i];
            const int xs = wrap_add(x, -kVX[i], nx), ys = wrap_add(y, -kVY[i], ny);
            T *q = p + (int64_t)i * plane + ys * px + xs;
            *q = Codec<S>::encode(Codec<S>::decode(*q, P, i) + add, P, i);
            acc[i] += (double)add;
        }
    }
    block_sum<9>(acc, part + 9 * blockIdx.x);
}

template <int S>
__global__ __launch_bounds__(kThreads) void thermal_sub_kernel(void *pops,
                                                               const LatticeParams *params,
                                                               int lattice, const double *sums)
{
    using T = typename Codec<S>::T;
    const LatticeParams &P = params[lattice];
    const int nx = P.nx, px = P.px;
    const int64_t V = (int64_t)nx * P.ny, plane = P.plane;
    T *p = (T *)pops + P.base;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 9 * V;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / V);
        const int s = (int)(k - (int64_t)i * V);
        const int y = s / nx, x = s - y * nx;
        const float mean = (float)(sums[i] / (double)V);
        T *q = p + (int64_t)i * plane + y * px + x;
        *q = Codec<S>::encode(Codec<S>::decode(*q, P, i) - mean, P, i);
    }
}

hipError_t launch_thermalize(const DeviceView &v, int lattice, int nx, int ny, double *part,
                             int nblocks, double *sums_dev, hipStream_t s)
{
    const uint32_t k0 = (uint32_t)(v.seed & 0xFFFFFFFFu), k1 = (uint32_t)(v.seed >> 32);
    void *p = v.pops[v.cur];
    const dim3 block(kThreads);
    if (v.storage == kF32)
        hipLaunchKernelGGL(thermal_add_kernel<kF32>, dim3(nblocks), block, 0, s, p, v.params,
                           lattice, k0, k1, part);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(thermal_add_kernel<kBF16>, dim3(nblocks), block, 0, s, p, v.params,
                           lattice, k0, k1, part);
    else
        hipLaunchKernelGGL(thermal_add_kernel<kF16>, dim3(nblocks), block, 0, s, p, v.params,
                           lattice, k0, k1, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_parts_kernel<9>, dim3(1), block, 0, s, part, nblocks, sums_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(9LL * nx * ny));
    if (v.storage == kF32)
        hipLaunchKernelGGL(thermal_sub_kernel<kF32>, grid, block, 0, s, p, v.params, lattice,
                           sums_dev);
    else if (v.storage == kBF16)
        hipLaunchKernelGGL(thermal_sub_kernel<kBF16>, grid, block, 0, s, p, v.params, lattice,
                           sums_dev);
    else
        hipLaunchKernelGGL(thermal_sub_kernel<kF16>, grid, block, 0, s, p, v.params, lattice,
                           sums_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Noise words and normals as the step kernel computes them (testing).
// ---------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void debug_noise_kernel(uint32_t key0, uint32_t key1,
                                                               uint32_t stream_id, uint32_t t,
                                                               int64_t site0, int64_t n,
                                                               uint32_t *words, float *zout)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)(site0 + k), t, stream_id, 0u), key0,
                                      key1);
        float z[6];
        normals6(w, z);
        if (words) {
            words[4 * k + 0] = w.x;
            words[4 * k + 1] = w.y;
            words[4 * k + 2] = w.z;
            words[4 * k + 3] = w.w;
        }
        if (zout)
            for (int q = 0; q < 6; ++q) zout[6 * k + q] = z[q];
    }
}

hipError_t launch_debug_noise(uint64_t seed, uint32_t stream_id, uint32_t t, int64_t site0,
                              int64_t n, uint32_t *words_dev, float *z_dev, hipStream_t s)
{
    hipLaunchKernelGGL(debug_noise_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), stream_id, t,
                       site0, n, words_dev, z_dev);
    return hipGetLastError();
}

// Zero-fill without hipMemset (safe inside captured graphs).
__global__ __launch_bounds__(kThreads) void fill_kernel(double *p, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0.0;
}

hipError_t launch_fill(double *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for((int64_t)n)), dim3(kThreads), 0, s, p,
                       (int64_t)n);
    return hipGetLastError();
}

}  // namespace flbdev
