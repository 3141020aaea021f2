// flb_runtime.hip -- host runtime behind the C interface of flb.h.
//
// A handle owns: the two population buffers of all its lattices, the
// per-lattice constant table, the step-kernel work list (one item per
// (lattice, tile), ordered so that each XCD receives a contiguous run of
// tiles), the correlator work lists, line plans and tables, the FP64
// accumulators, a device step counter, and captured HIP graphs of one
// sampling period.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/flb.h"
#include "flb_corr_internal.h"

using namespace flbdev;

// Staging area of flb_get_populations_noalloc, part of the library's code
// object: every GPU the library is loaded on holds its own copy (64 MiB)
// until the process ends, so that call needs no device allocation.  Host
// code never uses the array's name as an address: it takes each device's
// address from hipGetSymbolAddress (scratch_on_device).
constexpr size_t kNoAllocDoubles = (size_t)1 << 23;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
thread_local std::string g_err;
}  // namespace

int flbdev::set_error(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

namespace {

int fail(int code, const std::string &msg) { return set_error(code, msg); }

#define FLB_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

constexpr double kCs2 = 1.0 / 3.0;
const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const int kVx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kVy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// A captured sampling period: its length, the buffer holding the state at
// its start, whether the sample of that state is due (it then runs beside
// the period's steps) and how many stashed samples are pending (which
// decides the accumulation modes of the period's samples).
struct GraphKey {
    int every, parity, pending, due;
    bool operator<(const GraphKey &o) const
    {
        if (every != o.every) return every < o.every;
        if (parity != o.parity) return parity < o.parity;
        if (pending != o.pending) return pending < o.pending;
        return due < o.due;
    }
};

}  // namespace

struct flb {
    int device = 0;
    int storage = kF32;
    int elem_bytes = 4;
    uint32_t flags = 0;
    uint64_t seed = 0;
    std::vector<flb_lattice_spec> specs;
    std::vector<LatticeParams> params;
    int64_t total_elems = 0;  // per population buffer
    bool noise = false;

    // device memory
    void *pops[2] = {nullptr, nullptr};
    int cur = 0;
    LatticeParams *d_params = nullptr;
    uint32_t *d_step = nullptr;
    double *d_red = nullptr;  // reduction scratch
    int red_blocks = 1024;

    // stepping: tiles of tile_w threads along x, `sites` sites per thread
    int tile_w = 256, sites = 1;
    bool nontemporal = false;
    StepItem *d_items = nullptr;
    int nitems = 0;
    // time blocking: steps per launch (1, 2 or 3) and the two- and
    // three-step kernels' tile width; tile2 = 0: each lattice has its own,
    // log2 of it in ltile (5 or 6)
    int tblock = 1, tile2 = 64;
    std::vector<int8_t> ltile;
    StepItem *d_items2 = nullptr;
    int nitems2 = 0;
    int64_t t = 0;

    // correlators
    bool corr_ready = false;
    std::vector<LinePlan> plans;
    LinePlan *d_plans = nullptr;
    float2 *d_tables = nullptr;
    float2 *d_spec = nullptr;
    double *d_acc = nullptr;
    int64_t spec_elems = 0, acc_elems = 0;
    // column items of the two block sizes of the column kernel (the large
    // ones for the longest work lengths)
    CorrItem *d_rows = nullptr, *d_cols = nullptr, *d_cols_l = nullptr, *d_accum = nullptr;
    CorrItem *d_fld = nullptr;
    int n_rows = 0, n_cols = 0, n_cols_l = 0, n_accum = 0, n_fld = 0;
    // moment spectra (FLB_FLAG_MOMENT_SPECTRA): a second field set of six
    // moments through the same transforms, into kinds kKinds .. kKinds + 5
    bool moments = false;
    int nkinds = kKinds, nfld = kFields;
    CorrItem *d_cols_m = nullptr, *d_cols_lm = nullptr, *d_rows_m = nullptr;
    int n_cols_m = 0, n_cols_lm = 0, n_rows_m = 0;
    CorrItem *d_rows_blue = nullptr;  // rows of lattices with Bluestein row transforms
    int n_rows_blue = 0;
    // field set 0's Bluestein columns with length-specialised blocks
    CorrItem *d_cols_blue = nullptr;
    int n_cols_blue = 0;
    // launches of the length-specialised row blocks over parts of d_rows
    // (after its first n_rows items)
    std::vector<RowLaunch> rows_fixed;
    // power-of-two columns of 512..4096 points: persistent launches of the
    // pipelined column kernel, one per work length and field set, each with
    // its host-made schedule
    struct PipeLaunch {
        int lg = 0, grid = 0, niter = 0;
        PipeItem *d_sched = nullptr;
    };
    std::vector<PipeLaunch> pipe[2];
    // deferred accumulation: samples stash their spectra (the column
    // transform's output) in kDeferK slots and every kDeferK-th one adds the
    // products of all of them at once; `pending` counts the stashed samples
    // whose products are not yet added
    bool defer = false;
    int pending = 0;
    float2 *d_stash = nullptr;
    CorrItem *d_flush = nullptr;
    int n_flush = 0;
    float *d_fields = nullptr;
    double *d_csum_part = nullptr, *d_csum = nullptr;
    int rows_lds = 0, cols_lds = 0, cols_l_lds = 0;
    int64_t nsamples = 0;

    // A registered sample is due until the next steps are enqueued: it then
    // runs on `aux` beside them, the second step launch (the first to write
    // the sampled buffer) waits until it has read the state, and the steps'
    // stream waits for its end. Every call that reads the sums or changes
    // the state enqueues a due sample on the work stream first.
    bool due = false;
    bool overlap = true;  // flb_set_sample_overlap
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_read = nullptr, ev_done = nullptr;

    // launch timing (flb_set_launch_timing): an event pair around every step
    // launch enqueued outside a graph capture, recorded after any wait so
    // that it brackets the kernel alone
    bool timing = false, capturing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed, spare_events;
    std::vector<int> timed_steps;  // steps of each timed launch

    // streams and graphs
    hipStream_t own = nullptr;
    hipStream_t stream = nullptr;  // where work is enqueued
    hipEvent_t ev = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;

    DeviceView view() const
    {
        DeviceView v;
        v.pops[0] = pops[0];
        v.pops[1] = pops[1];
        v.cur = cur;
        v.params = d_params;
        v.step = d_step;
        v.step_rw = d_step;
        v.spec = d_spec;
        v.stash = d_stash;
        v.acc = d_acc;
        v.fields = d_fields;
        v.csum_part = d_csum_part;
        v.csum = d_csum;
        v.plans = d_plans;
        v.tables = d_tables;
        v.seed = seed;
        v.storage = storage;
        v.nlat = (int)params.size();
        return v;
    }
};

namespace {

bool finite(double v) { return std::isfinite(v); }

int validate_spec(const flb_lattice_spec &s, int idx)
{
    char buf[256];
    if (s.nx < 2 || s.ny < 2) {
        snprintf(buf, sizeof buf, "lattice %d: nx and ny must be >= 2 (got %d x %d)", idx, s.nx,
                 s.ny);
        return fail(FLB_EINVAL, buf);
    }
    if ((int64_t)(s.nx + 3) * s.ny * 9 * 4 >= (int64_t)1 << 32) {
        snprintf(buf, sizeof buf, "lattice %d: its populations must fit in 4 GiB "
                 "(9*nx*ny*4 bytes, about 119M sites)", idx);
        return fail(FLB_ESIZE, buf);
    }
    for (int a = 0; a < 9; ++a)
        if (!finite(s.tau[a])) return fail(FLB_EINVAL, "tau must be finite");
    for (int a = 3; a < 9; ++a)
        if (!(s.tau[a] > 0.5)) {
            snprintf(buf, sizeof buf, "lattice %d: tau[%d] = %g must exceed 1/2", idx, a, s.tau[a]);
            return fail(FLB_EINVAL, buf);
        }
    if (!finite(s.theta) || s.theta < 0) return fail(FLB_EINVAL, "theta must be finite and >= 0");
    if (!finite(s.rho0) || !(s.rho0 > 0)) return fail(FLB_EINVAL, "rho0 must be finite and > 0");
    if (!finite(s.u0[0]) || !finite(s.u0[1])) return fail(FLB_EINVAL, "u0 must be finite");
    if (s.u0[0] * s.u0[0] + s.u0[1] * s.u0[1] >= kCs2)
        return fail(FLB_EINVAL, "|u0| must be below the sound speed 1/sqrt(3)");
    if (s.reserved != 0) return fail(FLB_EINVAL, "reserved field must be 0");
    return FLB_OK;
}

LatticeParams make_params(const flb_lattice_spec &s, uint32_t flags)
{
    LatticeParams P;
    std::memset(&P, 0, sizeof P);
    P.nx = s.nx;
    P.ny = s.ny;
    P.nkx = s.nx / 2 + 1;
    P.px = (s.nx + 3) / 4 * 4;
    P.plane = (int64_t)P.px * s.ny;
    const double mu = s.theta / kCs2;
    // scale of each stored moment relative to M^a: s3 = 3/2 M3, s4 = 3 M4,
    // s5 = M5, s6,7 = sqrt(3/2) M6,7, s8 = M8
    const double mscale[6] = {1.5, 3.0, 1.0, std::sqrt(1.5), std::sqrt(1.5), 1.0};
    for (int a = 3; a < 9; ++a) {
        const double tau = s.tau[a];
        P.omega[a - 3] = (float)(1.0 / tau);
        double sigma = std::sqrt(mu * s.rho0 * (2.0 * tau - 1.0)) / tau;  // Eq. (8)
        if ((flags & FLB_FLAG_NO_GHOST_NOISE) && a >= 6) sigma = 0.0;
        P.amp[a - 3] = (float)(mscale[a - 3] * sigma);
    }
    P.fcoef[0] = (float)(2.25 / s.tau[3]);
    P.fcoef[1] = (float)(9.0 / s.tau[4]);
    P.fcoef[2] = (float)(-3.0 / s.tau[6]);
    P.fcoef[3] = (float)(-3.0 / s.tau[7]);
    P.fcoef[4] = 2.0f * P.amp[3];
    P.fcoef[5] = 2.0f * P.amp[4];
    P.rho0 = (float)s.rho0;
    P.u0x = (float)s.u0[0];
    P.u0y = (float)s.u0[1];
    const double uu = s.u0[0] * s.u0[0] + s.u0[1] * s.u0[1];
    const double mu_store = std::max(mu, 3e-4);  // 16-bit scale when theta is tiny or zero
    for (int i = 0; i < 9; ++i) {
        const double uv = s.u0[0] * kVx[i] + s.u0[1] * kVy[i];
        // Eq. (2), c = 1, minus w_i rho0
        P.feq[i] = (float)(s.rho0 * kW[i] * (3.0 * uv + 4.5 * uv * uv - 1.5 * uu));
        P.scale[i] = (float)std::sqrt(mu_store * s.rho0 * kW[i]);
        P.inv_scale[i] = 1.0f / P.scale[i];
        P.feq_scaled[i] = P.feq[i] * P.inv_scale[i];
        P.therm_amp[i] = (float)std::sqrt(mu * s.rho0 * kW[i]);
    }
    // collide_q's constants, from the FP32 values the codec uses:
    // d_i = s_i q_i + F_i with s = scale, F = feq
    {
        double F[9];
        for (int i = 0; i < 9; ++i) F[i] = P.feq[i];
        const double s0 = P.scale[0], s1 = P.scale[1], s5 = P.scale[5];
        const double Fa = F[1] + F[3], Fb = F[2] + F[4], Fc = F[5] + F[7], Fe = F[6] + F[8];
        const double Fx = F[1] - F[3], Fy = F[2] - F[4], Fp = F[5] - F[7], Fm = F[6] - F[8];
        const double coef[11] = {s0, s1, s5, 2.25 * s1, 9.0 * s5, 0.5 * s1, 2.0 * s5,
                                 3.0 * s5, 1.5 * s1, 0.5 * s0, 0.0};
        for (int k = 0; k < 11; ++k) P.qcoef[k] = (float)coef[k];
        const double off[9] = {F[0] + Fa + Fb + Fc + Fe,                 // sum of F: delta rho
                               Fx + Fp - Fm,                              // j_x
                               Fy + Fp + Fm,                              // j_y
                               2.25 * (Fa - Fb),                          // s3 = 3/2 M3
                               9.0 * (Fc - Fe),                           // s4 = 3 M4
                               0.5 * (Fa + Fb) + 2.0 * (Fc + Fe) - F[0],  // s5 = M5
                               1.5 * (2.0 * (Fp - Fm) - Fx),              // s6
                               1.5 * (2.0 * (Fp + Fm) - Fy),              // s7
                               0.5 * F[0] + 2.0 * (Fc + Fe) - (Fa + Fb)}; // s8 = M8
        for (int k = 0; k < 9; ++k) P.qoff[k] = (float)off[k];
        P.qback[0] = (float)(kW[0] / s0);
        P.qback[1] = (float)(kW[1] / s1);
        P.qback[2] = (float)(kW[5] / s5);
    }
    P.stream_id = s.stream_id;
    return P;
}

// XCD-aware order: blocks are dispatched round-robin over the 8 XCDs, so
// block b runs on XCD b % 8.  Give each XCD a contiguous run of work items so
// that neighbouring tiles (which share cache lines and halo rows) meet in the
// same L2.
template <typename T>
std::vector<T> xcd_order(const std::vector<T> &in, const T &idle)
{
    const int nx = 8;
    const size_t n = in.size();
    const size_t per = (n + nx - 1) / nx;
    std::vector<T> out(per * nx, idle);
    for (size_t b = 0; b < out.size(); ++b) {
        const size_t j = (b % nx) * per + b / nx;
        if (j < n) out[b] = in[j];
    }
    return out;
}

template <typename T>
int upload(T **dptr, const std::vector<T> &v)
{
    if (*dptr) {
        (void)hipFree(*dptr);
        *dptr = nullptr;
    }
    if (v.empty()) return FLB_OK;
    FLB_HIP(hipMalloc((void **)dptr, v.size() * sizeof(T)));
    FLB_HIP(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return FLB_OK;
}

// The two-step kernel's work items, in XCD order: every lattice's tiles of
// width tw, or with lt, of width 2^lt[l] (the mixed kernel's items, the
// 32 x 32 ones flagged); only the lattices `only` marks, if given.
std::vector<StepItem> step2_items(const flb_t *h, const std::vector<int8_t> *lt, int tw,
                                  const std::vector<char> *only)
{
    std::vector<StepItem> items;
    for (size_t l = 0; l < h->params.size(); ++l) {
        if (only && !(*only)[l]) continue;
        const LatticeParams &P = h->params[l];
        const int w = lt ? 1 << (*lt)[l] : tw, th = 1024 / w;
        const int32_t flag = lt && w == 32 ? kStep2Square : 0;
        const int n2 = ((P.nx + w - 1) / w) * ((P.ny + th - 1) / th);
        for (int t = 0; t < n2; ++t) items.push_back({(int32_t)l, t | flag});
    }
    return xcd_order(items, StepItem{-1, 0});
}

int build_step_items(flb_t *h)
{
    const int TH = kThreads / h->tile_w;
    const int TW = h->tile_w * h->sites;  // sites per tile row
    std::vector<StepItem> items;
    for (size_t l = 0; l < h->params.size(); ++l) {
        LatticeParams &P = h->params[l];
        P.tiles_x = (P.nx + TW - 1) / TW;
        const int tiles_y = (P.ny + TH - 1) / TH;
        for (int t = 0; t < P.tiles_x * tiles_y; ++t) items.push_back({(int32_t)l, t});
    }
    items = xcd_order(items, StepItem{-1, 0});
    h->nitems = (int)items.size();
    int rc = upload(&h->d_items, items);
    if (rc) return rc;
    // the two-step kernel's tiles: tile2 x (1024 / tile2) sites, or each
    // lattice's own shape
    if (h->tile2 == 0 && h->ltile.size() != h->params.size())
        return fail(FLB_ESTATE, "per-lattice two-step tiles do not match the lattices");
    std::vector<StepItem> items2 =
        step2_items(h, h->tile2 == 0 ? &h->ltile : nullptr, h->tile2, nullptr);
    h->nitems2 = (int)items2.size();
    if ((rc = upload(&h->d_items2, items2))) return rc;
    return upload(&h->d_params, h->params);
}

// Kernel launches for n steps (the buffer parity flips once per launch).
int64_t step_launches(const flb_t *h, int64_t n)
{
    if (h->tblock == 3) return n / 3 + (n % 3 ? 1 : 0);  // a remainder of 2 takes one launch
    return h->tblock == 2 ? n / 2 + n % 2 : n;
}

void clear_graphs(flb_t *h)
{
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// In-place radix-2 transform on the host, FP64 (for the Bluestein kernel).
void host_fft(std::vector<std::complex<double>> &a)
{
    const int n = (int)a.size();
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        for (int k = 0; k < len / 2; ++k) {
            const double ang = -2.0 * M_PI * k / len;
            const std::complex<double> w(std::cos(ang), std::sin(ang));
            for (int b = 0; b < n; b += len) {
                const auto u = a[b + k], v = w * a[b + k + len / 2];
                a[b + k] = u + v;
                a[b + k + len / 2] = u - v;
            }
        }
    }
}

}  // namespace

bool flbdev::line_length_ok(int n)
{
    return is_pow2(n) ? n <= FLB_MAX_FFT_SIDE : n <= FLB_MAX_FFT_SIDE / 2;
}

flbdev::LineTables::LineTables() : tables(kTwN / 2)
{
    for (int k = 0; k < kTwN / 2; ++k) {
        const double ang = -2.0 * M_PI * k / kTwN;
        tables[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
}

int flbdev::LineTables::plan_for(int n)
{
    auto it = plan_of.find(n);
    if (it != plan_of.end()) return it->second;
    LinePlan L;
    std::memset(&L, 0, sizeof L);
    L.n = n;
    if (is_pow2(n)) {
        L.m = n;
        L.bluestein = 0;
    } else {
        L.m = 1 << log2i(2 * n - 1);
        L.bluestein = 1;
        L.chirp_off = (int64_t)tables.size();
        std::vector<std::complex<double>> c(n);
        for (int j = 0; j < n; ++j) {
            const long long q = ((long long)j * j) % (2LL * n);  // exp(-i pi j^2 / n)
            const double ang = -M_PI * (double)q / n;
            c[j] = std::complex<double>(std::cos(ang), std::sin(ang));
            tables.push_back(make_float2((float)c[j].real(), (float)c[j].imag()));
        }
        std::vector<std::complex<double>> b(L.m, 0.0);
        for (int j = 0; j < n; ++j) {
            b[j] = std::conj(c[j]);
            if (j > 0) b[L.m - j] = std::conj(c[j]);
        }
        host_fft(b);
        // bit-reversed order, the order in which the device's forward
        // transform leaves its output
        L.kernel_off = (int64_t)tables.size();
        const int lgm = log2i(L.m);
        for (int p = 0; p < L.m; ++p) {
            int j = 0;
            for (int bit = 0; bit < lgm; ++bit) j |= ((p >> bit) & 1) << (lgm - 1 - bit);
            const auto v = b[j] / (double)L.m;  // inverse transform's 1/m folded in
            tables.push_back(make_float2((float)v.real(), (float)v.imag()));
        }
    }
    L.log2m = log2i(L.m);
    const int id = (int)plans.size();
    plans.push_back(L);
    plan_of[n] = id;
    return id;
}

namespace {

// Power-of-two column lengths from which the column kernel takes its large
// blocks (kColsLargeElems elements, kColsLargeThreads threads: 16, 8 and 4
// columns of 1024, 2048 and 4096 points) instead of the kColsElems-element
// ones.  Whole path, large against small blocks: 16 x 1024^2 88.2 against
// 87.0 GLUPS, 4 x 2048^2 89.0 against 86.2, 4096^2 87.3 against 80.0 (two
// columns per block leave 16-byte runs).  Bluestein work lengths keep the
// small blocks: large ones from 1024 or 2048 on made the 64 uneven
// lattices' path 56.2 or 56.6 against 57.5.
constexpr int kColsLargeMin = 1024;

// Schedule of a persistent launch of `grid` blocks (a multiple of 8) over
// `items`, whole groups first and partial ones (fewer columns) last: each
// block takes items round after round, sched[it * grid + b].  Block b runs
// on XCD b % 8, so every XCD gets a contiguous run of the whole groups
// (neighbouring columns share cache lines in its L2) and every block the
// same number of them; the remainder, the partial groups where possible,
// goes one per block into a last round.
std::vector<CorrItem> persistent_schedule(const std::vector<CorrItem> &items, int grid,
                                          int &niter)
{
    const int F = (int)items.size(), nslot = grid / 8;
    const int q = F / grid, rem = F - q * grid;
    niter = q + (rem > 0 ? 1 : 0);
    std::vector<CorrItem> sched((size_t)niter * grid, CorrItem{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
        for (int j = 0; j < q * nslot; ++j)
            sched[(size_t)(j / nslot) * grid + x + 8 * (j % nslot)] = items[(size_t)x * q * nslot + j];
    for (int r = 0; r < rem; ++r) sched[(size_t)q * grid + r] = items[(size_t)q * grid + r];
    return sched;
}

// The pipelined column kernel's form of scheduled column groups: offsets of
// the first column in the spectra and of its tile in a stash slot, row
// pitch, tile stride and number of columns.
std::vector<PipeItem> pipe_items(const flb_t *h, const std::vector<CorrItem> &sched)
{
    std::vector<PipeItem> out(sched.size(), PipeItem{0, 0, 0, 0, 0, 0, 0, 0});
    for (size_t i = 0; i < sched.size(); ++i) {
        const CorrItem &it = sched[i];
        if (it.lattice < 0) continue;
        const LatticeParams &P = h->params[it.lattice];
        out[i].off = P.spec_base + (int64_t)it.a * P.ny * P.kxp + it.b;
        out[i].sbase = P.spec_base;
        out[i].kxp = P.kxp;
        out[i].ts = kTileCols * P.ny;
        out[i].o0 = (int32_t)spec_offset(0, it.b, P.ny);
        out[i].f = it.a;
        out[i].plane = P.ny * P.kxp;
        out[i].ncol = std::min(1 << it.c, P.nkx - it.b);
    }
    return out;
}

int setup_correlators(flb_t *h)
{
    if (h->corr_ready) return FLB_OK;
    // tables below replace device buffers that queued kernels may still read
    FLB_HIP(hipStreamSynchronize(h->stream));
    for (auto &P : h->params) {
        if (!line_length_ok(P.nx) || !line_length_ok(P.ny))
            return fail(FLB_ESIZE, "correlators support power-of-two sides up to FLB_MAX_FFT_SIDE "
                                   "and other sides up to FLB_MAX_FFT_SIDE/2");
    }

    LineTables lt;
    auto plan_for = [&](int n) { return lt.plan_for(n); };

    int64_t spec = 0, acc = 0, fld = 0;
    int nparts = 0;
    h->rows_lds = h->cols_lds = h->cols_l_lds = 0;
    for (auto &P : h->params) {
        P.line_x = plan_for(P.nx);
        P.line_y = plan_for(P.ny);
        P.kxp = (P.nkx + 15) / 16 * 16;
        // columns per block of the column kernel: at most 16, lines of at most
        // kColsElems LDS elements per block (kColsLargeElems for power-of-two
        // lengths from kColsLargeMin on, which take the large blocks)
        const int my = lt.plans[P.line_y].m;
        P.col_large = !lt.plans[P.line_y].bluestein && my >= kColsLargeMin;
        P.col_lgcb =
            log2i(std::max(1, std::min(16, (P.col_large ? kColsLargeElems : kColsElems) / my)));
        const int e = my << P.col_lgcb;  // padded like the row kernels' lines
        int &lds = P.col_large ? h->cols_l_lds : h->cols_lds;
        lds = std::max(lds, (e + (e >> 4) + (e >> 8) + 1) * (int)sizeof(float2));
        P.spec_base = spec;
        P.acc_base = acc;
        spec += (int64_t)h->nfld * P.ny * P.kxp;
        acc += (int64_t)h->nkinds * P.ny * P.kxp;
        // FP32 moment planes, only with the moment spectra
        P.fld_base = fld;
        if (h->moments) fld += ((int64_t)kMomentFields * P.nx * P.ny + 63) / 64 * 64;
        P.fld_tiles_x = (P.nx + kThreads - 1) / kThreads;
        // one conservation partial per row group of the row kernel
        const int mx = lt.plans[P.line_x].m;
        const int rb = std::max(1, std::min(P.ny, 4096 / mx));
        P.fld_part0 = nparts;
        P.fld_nparts = (P.ny + rb - 1) / rb;
        nparts += P.fld_nparts;
    }
    h->spec_elems = spec;
    h->acc_elems = acc;

    h->plans = lt.plans;
    std::vector<CorrItem> rows, cols, cols_l, accum, flds, cols_m, cols_lm, rows_m;
    std::vector<CorrItem> rows_blue, flush, cols_blue[4];
    // rows with length-specialised blocks: Bluestein rows per work length
    // (longest first, one launch for all), power-of-two rows per length
    std::vector<CorrItem> rows_fixed_blue[4];
    std::map<int, std::vector<CorrItem>> rows_fixed_p2;
    std::map<int, std::vector<CorrItem>> pipe_full[2], pipe_part[2];  // per field set and lg
    for (size_t l = 0; l < h->params.size(); ++l) {
        const LatticeParams &P = h->params[l];
        if (h->moments) {
            const int ntiles = P.fld_tiles_x * ((P.ny + kFieldRows - 1) / kFieldRows);
            for (int t = 0; t < ntiles; ++t) flds.push_back({(int32_t)l, t, 0, 0});
        }
        const int mx = lt.plans[P.line_x].m;
        // rows per block: up to 4096 line elements (32 KB of LDS), which the
        // row kernels assume
        const int rb = std::max(1, std::min(P.ny, 4096 / mx));
        if (rb * mx > 4096) return fail(FLB_ESIZE, "row transform longer than 4096 elements");
        // the row kernels pad their LDS lines (one slot per 16 and per 256);
        // the length-specialised one always transforms 4096 elements (lines
        // past the lattice's last row hold zeros)
        const LinePlan &Lx = lt.plans[P.line_x];
        const bool p2 = !Lx.bluestein && corr_rows_p2_supported(Lx.log2m) && P.kxp == mx / 2 + 16;
        const bool blue = Lx.bluestein && corr_rows_blue_supported(Lx.log2m);
        const int ne = (p2 || blue) ? 4096 : rb * mx;
        const int slots = ne + (ne >> 4) + (ne >> 8) + 1;
        h->rows_lds = std::max(h->rows_lds, slots * (int)sizeof(float2));
        for (int y = 0, part = P.fld_part0; y < P.ny; y += rb, ++part) {
            const CorrItem ri{(int32_t)l, y, rb, part};
            if (blue) rows_fixed_blue[11 - Lx.log2m].push_back(ri);
            else if (Lx.bluestein) rows_blue.push_back(ri);
            else if (p2) rows_fixed_p2[Lx.log2m].push_back(ri);
            else rows.push_back(ri);
            if (h->moments)
                for (int sig = 0; sig < 3; ++sig) rows_m.push_back({(int32_t)l, y, rb, sig});
        }
        const LinePlan &Ly = lt.plans[P.line_y];
        if (!Ly.bluestein && corr_cols_pipe_supported(Ly.log2m)) {
            // whole groups and the partial last group of each field apart
            const int cb = std::min(16, 16384 / Ly.m), lgc = log2i(cb);
            for (int f = 0; f < h->nfld; ++f)
                for (int c0 = 0; c0 < P.nkx; c0 += cb) {
                    const CorrItem it{(int32_t)l, f, c0, lgc};
                    const bool whole = c0 + cb <= P.nkx;
                    if (f < kFields) (whole ? pipe_full[0] : pipe_part[0])[Ly.log2m].push_back(it);
                    (whole ? pipe_full[1] : pipe_part[1])[Ly.log2m].push_back(it);
                }
        } else {
            // field set 0's Bluestein columns of the supported work lengths:
            // 8192 / m columns per block (longest work lengths first)
            const bool cblue = Ly.bluestein && corr_cols_blue_supported(Ly.log2m);
            if (cblue)
                for (int f = 0; f < kFields; ++f)
                    for (int c0 = 0; c0 < P.nkx; c0 += 8192 / Ly.m)
                        cols_blue[11 - Ly.log2m].push_back({(int32_t)l, f, c0, 0});
            for (int f = 0; f < h->nfld; ++f)
                for (int c0 = 0; c0 < P.nkx; c0 += 1 << P.col_lgcb) {
                    if (f < kFields && !cblue)
                        (P.col_large ? cols_l : cols).push_back({(int32_t)l, f, c0, P.col_lgcb});
                    (P.col_large ? cols_lm : cols_m).push_back({(int32_t)l, f, c0, P.col_lgcb});
                }
        }
        // the accumulation walks the tiled planes (padding columns skipped)
        const int64_t nk = (int64_t)P.ny * P.kxp;
        for (int64_t k0 = 0; k0 < nk; k0 += kThreads) {
            accum.push_back({(int32_t)l, (int32_t)k0, 0, 0});
            flush.push_back({(int32_t)l, (int32_t)k0, 0, 0});
        }
    }
    const CorrItem idle{-1, 0, 0, 0};
    flds = xcd_order(flds, idle);
    rows = xcd_order(rows, idle);
    rows_blue = xcd_order(rows_blue, idle);
    h->n_rows_blue = (int)rows_blue.size();
    cols = xcd_order(cols, idle);
    cols_l = xcd_order(cols_l, idle);
    if (h->moments) {
        cols_m = xcd_order(cols_m, idle);
        cols_lm = xcd_order(cols_lm, idle);
        rows_m = xcd_order(rows_m, idle);
    } else {
        cols_m.clear();
        cols_lm.clear();
    }
    h->n_cols_m = (int)cols_m.size();
    h->n_cols_lm = (int)cols_lm.size();
    h->n_rows_m = (int)rows_m.size();
    h->n_flush = (int)flush.size();
    int ncu = 0;
    FLB_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
    for (int set = 0; set < 2; ++set) {
        for (auto &pl : h->pipe[set])
            if (pl.d_sched) (void)hipFree(pl.d_sched);
        h->pipe[set].clear();
        if (set == 1 && !h->moments) continue;
        for (auto &kv : pipe_full[set]) {
            std::vector<CorrItem> items = kv.second;
            const auto &part = pipe_part[set][kv.first];
            items.insert(items.end(), part.begin(), part.end());
            // one block resident per CU: 140 KB of LDS from 1024 points on,
            // the registers of 1024 threads at 512 points
            int grid = std::max(8, ncu / 8 * 8);
            grid = std::min(grid, ((int)items.size() + 7) / 8 * 8);
            flb_t::PipeLaunch pl;
            pl.lg = kv.first;
            pl.grid = grid;
            int rc0 = upload(&pl.d_sched, pipe_items(h, persistent_schedule(items, grid, pl.niter)));
            if (rc0) return rc0;
            h->pipe[set].push_back(pl);
        }
        for (auto &kv : pipe_part[set])  // lengths with partial groups only
            if (!pipe_full[set].count(kv.first)) {
                const std::vector<CorrItem> &items = kv.second;
                flb_t::PipeLaunch pl;
                pl.lg = kv.first;
                pl.grid = ((int)items.size() + 7) / 8 * 8;
                int rc0 = upload(&pl.d_sched,
                                 pipe_items(h, persistent_schedule(items, pl.grid, pl.niter)));
                if (rc0) return rc0;
                h->pipe[set].push_back(pl);
            }
    }
    std::vector<CorrItem> cblue_all;
    for (const auto &part : cols_blue) {
        if (part.empty()) continue;
        const std::vector<CorrItem> o = xcd_order(part, idle);
        cblue_all.insert(cblue_all.end(), o.begin(), o.end());
    }
    h->n_cols_blue = (int)cblue_all.size();
    h->defer = !cols.empty() || !cols_l.empty() || !h->pipe[0].empty() || !cblue_all.empty();
    h->pending = 0;
    h->n_rows = (int)rows.size();
    h->rows_fixed.clear();
    {
        // Bluestein rows: each work length spread over the XCDs on its own,
        // so that every XCD gets its share of the expensive blocks
        const int off = (int)rows.size();
        for (const auto &part : rows_fixed_blue) {
            if (part.empty()) continue;
            const std::vector<CorrItem> o = xcd_order(part, idle);
            rows.insert(rows.end(), o.begin(), o.end());
        }
        if ((int)rows.size() > off) h->rows_fixed.push_back({0, off, (int)rows.size() - off});
        for (const auto &kv : rows_fixed_p2) {
            const std::vector<CorrItem> o = xcd_order(kv.second, idle);
            h->rows_fixed.push_back({kv.first, (int)rows.size(), (int)o.size()});
            rows.insert(rows.end(), o.begin(), o.end());
        }
    }
    h->n_cols = (int)cols.size();
    h->n_cols_l = (int)cols_l.size();
    h->n_accum = (int)accum.size();
    h->n_fld = (int)flds.size();
    int rc;
    if ((rc = upload(&h->d_fld, flds)) || (rc = upload(&h->d_rows, rows)) ||
        (rc = upload(&h->d_cols, cols)) || (rc = upload(&h->d_cols_l, cols_l)) ||
        (rc = upload(&h->d_accum, accum)) || (rc = upload(&h->d_cols_lm, cols_lm)) ||
        (rc = upload(&h->d_cols_m, cols_m)) || (rc = upload(&h->d_rows_m, rows_m)) ||
        (rc = upload(&h->d_rows_blue, rows_blue)) || (rc = upload(&h->d_flush, flush)) ||
        (rc = upload(&h->d_cols_blue, cblue_all)) ||
        (rc = upload(&h->d_plans, h->plans)) ||
        (rc = upload(&h->d_tables, lt.tables)) || (rc = upload(&h->d_params, h->params)))
        return rc;
    FLB_HIP(hipMalloc((void **)&h->d_spec, spec * sizeof(float2)));
    FLB_HIP(hipMalloc((void **)&h->d_acc, acc * sizeof(double)));
    if (fld > 0) FLB_HIP(hipMalloc((void **)&h->d_fields, fld * sizeof(float)));
    if (h->defer)
        FLB_HIP(hipMalloc((void **)&h->d_stash, (size_t)kDeferK * spec * sizeof(float2)));
    FLB_HIP(hipMalloc((void **)&h->d_csum_part, (size_t)nparts * 5 * sizeof(double)));
    FLB_HIP(hipMalloc((void **)&h->d_csum, h->params.size() * 5 * sizeof(double)));
    FLB_HIP(launch_fill(h->d_csum, h->params.size() * 5, h->stream));
    FLB_HIP(launch_fill(h->d_acc, (size_t)acc, h->stream));
    h->nsamples = 0;
    h->corr_ready = true;
    clear_graphs(h);
    return FLB_OK;
}

// The kernels of one sample of the current state on stream s. When ev_read
// is given it is recorded once every kernel that reads the populations has
// been enqueued.
int enqueue_sample(flb_t *h, hipStream_t s, hipEvent_t ev_read = nullptr)
{
    const DeviceView v = h->view();
    // the moment planes first, so that all reads of the state come first
    if (h->moments) FLB_HIP(launch_corr_moment_fields(v, h->d_fld, h->n_fld, s));
    for (int set = 0; set < (h->moments ? 2 : 1); ++set) {
        // the moment set reuses the spectrum buffer after set 0
        const CorrItem *cg = set ? h->d_cols_m : h->d_cols;
        const CorrItem *cl = set ? h->d_cols_lm : h->d_cols_l;
        const int ng = set ? h->n_cols_m : h->n_cols;
        const int nl = set ? h->n_cols_lm : h->n_cols_l;
        if (set == 0) {
            FLB_HIP(launch_corr_rows(v, h->d_rows, h->n_rows, h->rows_fixed.data(),
                                     (int)h->rows_fixed.size(), h->d_rows_blue, h->n_rows_blue,
                                     h->rows_lds, s));
            if (ev_read) FLB_HIP(hipEventRecord(ev_read, s));
        } else {
            FLB_HIP(launch_corr_moment_rows(v, h->d_rows_m, h->n_rows_m, h->rows_lds, s));
        }
        // field set 0: the column transforms' output goes to stash slot
        // `pending`, and every kDeferK-th sample adds the products of all
        // the slots; otherwise it stays in place and is accumulated at once
        const bool stash = !set && h->defer;
        const int slot = stash ? h->pending : -1;
        if (!set && h->n_cols_blue)
            FLB_HIP(launch_corr_cols_blue(v, h->d_cols_blue, h->n_cols_blue, slot, s));
        if (ng) FLB_HIP(launch_corr_cols(v, cg, ng, slot, false, h->cols_lds, s));
        if (nl) FLB_HIP(launch_corr_cols(v, cl, nl, slot, true, h->cols_l_lds, s));
        for (const auto &pl : h->pipe[set])
            FLB_HIP(launch_corr_cols_pipe(v, pl.d_sched, pl.niter, pl.grid, pl.lg, slot, s));
        if (stash && h->pending == kDeferK - 1)
            FLB_HIP(launch_corr_flush(v, h->d_flush, h->n_flush, kDeferK, s));
        else if (h->n_accum && !stash)
            FLB_HIP(launch_corr_accum(v, h->d_accum, h->n_accum, set, s));
    }
    if (h->defer) h->pending = (h->pending + 1) % kDeferK;
    return FLB_OK;
}

// Adds a stashed sample's products to the sums before they are read.
int flush_pending(flb_t *h)
{
    if (!h->pending) return FLB_OK;
    FLB_HIP(launch_corr_flush(h->view(), h->d_flush, h->n_flush, h->pending, h->stream));
    h->pending = 0;
    return FLB_OK;
}

// n steps from the device counter value; the counter is advanced afterwards.
// With time blocking, pairs of steps go through the two-step kernel and an
// odd last step through the one-step kernel. When wait_before_second is
// given, the second launch (the first to write the buffer that held the
// state at the start) waits for it.
int enqueue_steps(flb_t *h, int64_t n, hipStream_t s, hipEvent_t wait_before_second = nullptr)
{
    int64_t k = 0;
    int launches = 0;
    const bool timing = h->timing && !h->capturing;
    hipEvent_t stop = nullptr;
    auto before_launch = [&](int steps) -> int {
        if (launches++ == 1 && wait_before_second)
            FLB_HIP(hipStreamWaitEvent(s, wait_before_second, 0));
        if (timing) {
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (!h->spare_events.empty()) {
                ev = h->spare_events.back();
                h->spare_events.pop_back();
            } else {
                FLB_HIP(hipEventCreate(&ev.first));
                if (hipEventCreate(&ev.second) != hipSuccess) {
                    (void)hipEventDestroy(ev.first);
                    return fail(FLB_EHIP, "timing event creation failed");
                }
            }
            h->timed.push_back(ev);
            h->timed_steps.push_back(steps);
            FLB_HIP(hipEventRecord(ev.first, s));
            stop = ev.second;
        }
        return FLB_OK;
    };
    auto after_launch = [&]() -> int {
        if (timing) FLB_HIP(hipEventRecord(stop, s));
        return FLB_OK;
    };
    int rc;
    // three steps per launch: a remainder of one step after at least three
    // goes as two launches of two steps (3 + 1 -> 2 + 2), as one step per
    // launch costs a whole HBM round trip
    const int64_t n3 = h->tblock == 3 ? (n % 3 == 1 && n >= 4 ? n / 3 - 1 : n / 3) : 0;
    for (; k < 3 * n3; k += 3) {
        if ((rc = before_launch(3))) return rc;
        FLB_HIP(launch_step3(h->view(), h->d_items2, h->nitems2, h->tile2, (uint32_t)k,
                             h->nontemporal, h->noise, s));
        if ((rc = after_launch())) return rc;
        h->cur ^= 1;
    }
    if (h->tblock >= 2)
        for (; k + 2 <= n; k += 2) {
            if ((rc = before_launch(2))) return rc;
            FLB_HIP(launch_step2(h->view(), h->d_items2, h->nitems2, h->tile2, (uint32_t)k,
                                 h->nontemporal, h->noise, s));
            if ((rc = after_launch())) return rc;
            h->cur ^= 1;
        }
    for (; k < n; ++k) {
        if ((rc = before_launch(1))) return rc;
        FLB_HIP(launch_step(h->view(), h->d_items, h->nitems, h->tile_w, h->sites, (uint32_t)k,
                            h->nontemporal, h->noise, s));
        if ((rc = after_launch())) return rc;
        h->cur ^= 1;
    }
    if (n > 0) FLB_HIP(launch_advance_step(h->d_step, (uint32_t)n, s));
    return FLB_OK;
}

// n steps on stream s; a due sample of the state at their start runs on the
// side stream beside them and s waits for its end.
int enqueue_steps_overlapped(flb_t *h, int64_t n, hipStream_t s)
{
    if (!h->due || n <= 0) return enqueue_steps(h, n, s);
    FLB_HIP(hipEventRecord(h->ev_fork, s));
    FLB_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    int rc = enqueue_sample(h, h->aux, h->ev_read);
    if (rc) return rc;
    h->due = false;
    FLB_HIP(hipEventRecord(h->ev_done, h->aux));
    if ((rc = enqueue_steps(h, n, s, h->ev_read))) return rc;
    FLB_HIP(hipStreamWaitEvent(s, h->ev_done, 0));
    return FLB_OK;
}

// Enqueues a due sample on the work stream.
int settle_due(flb_t *h)
{
    if (!h->due) return FLB_OK;
    int rc = enqueue_sample(h, h->stream);
    if (rc) return rc;
    h->due = false;
    return FLB_OK;
}

int check_time(flb_t *h, int64_t n)
{
    if (n < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
    if (h->t + n >= (int64_t)0xFFFFFFFF)
        return fail(FLB_ESIZE, "the step counter is a 32-bit noise counter word; "
                               "t must stay below 2^32 - 1");
    return FLB_OK;
}

flb_t *create_impl(int n, const flb_lattice_spec *specs, uint64_t seed, int storage,
                   uint32_t flags)
{
    if (n < 1 || !specs) {
        fail(FLB_EINVAL, "need at least one lattice spec");
        return nullptr;
    }
    if (storage != FLB_STORAGE_F32 && storage != FLB_STORAGE_BF16 && storage != FLB_STORAGE_F16) {
        fail(FLB_EINVAL, "unknown storage format");
        return nullptr;
    }
    if (flags & ~(FLB_FLAG_NO_GHOST_NOISE | FLB_FLAG_MOMENT_SPECTRA)) {
        fail(FLB_EINVAL, "unknown flags");
        return nullptr;
    }
    for (int l = 0; l < n; ++l)
        if (validate_spec(specs[l], l) != FLB_OK) return nullptr;

    flb_t *h = new flb_t();
    h->storage = storage;
    h->elem_bytes = storage == FLB_STORAGE_F32 ? 4 : 2;
    h->flags = flags;
    h->moments = (flags & FLB_FLAG_MOMENT_SPECTRA) != 0;
    h->nkinds = h->moments ? FLB_NKINDS_MOMENTS : FLB_NKINDS;
    h->nfld = h->moments ? kMomentFields : kFields;
    h->seed = seed;
    h->specs.assign(specs, specs + n);
    int64_t off = 0;
    for (int l = 0; l < n; ++l) {
        LatticeParams P = make_params(specs[l], flags);
        P.base = off;
        off += 9 * P.plane;
        off = (off + 63) / 64 * 64;  // 256-byte aligned planes per lattice
        for (int a = 0; a < 6; ++a) h->noise = h->noise || P.amp[a] != 0.0f;
        h->params.push_back(P);
    }
    h->total_elems = off;
    // streaming accesses pay off once a buffer no longer fits the last-level
    // cache
    h->nontemporal = (double)off * h->elem_bytes > 256.0 * 1024 * 1024;
    // measured on MI355X at 4096^2: FP32 is best with one site per thread
    // (scalar accesses spread the 18 streams best; with the streaming hint
    // 77.9 GLUPS against at most 75.9 for other shapes), 16-bit storage with
    // four (the ALU-bound form profits from fewer address computations)
    if (h->elem_bytes == 2) {
        h->tile_w = 128;
        h->sites = 4;
    }

    auto bail = [&](int rc) -> flb_t * {
        (void)rc;
        flb_destroy(h);
        return nullptr;
    };
    if (hipGetDevice(&h->device) != hipSuccess) {
        fail(FLB_EHIP, "no HIP device");
        return bail(0);
    }
    if (hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_read, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_done, hipEventDisableTiming) != hipSuccess) {
        fail(FLB_EHIP, "stream creation failed");
        return bail(0);
    }
    h->stream = h->own;
    // both population buffers in one allocation
    const size_t bytes = (size_t)h->total_elems * h->elem_bytes;
    if (hipMalloc(&h->pops[0], 2 * bytes) != hipSuccess) {
        fail(FLB_ENOMEM, "population buffers: out of device memory");
        return bail(0);
    }
    h->pops[1] = (char *)h->pops[0] + bytes;
    if (hipMalloc((void **)&h->d_step, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&h->d_red, (size_t)(h->red_blocks * 9 + 16) * sizeof(double)) !=
            hipSuccess) {
        fail(FLB_ENOMEM, "scratch allocation failed");
        return bail(0);
    }
    if (hipMemsetAsync(h->d_step, 0, sizeof(uint32_t), h->stream) != hipSuccess) {
        fail(FLB_EHIP, "step counter reset failed");
        return bail(0);
    }
    if (build_step_items(h) != FLB_OK) return bail(0);
    for (int l = 0; l < n; ++l)
        if (launch_init(h->view(), l, h->params[l].plane, h->stream) != hipSuccess) {
            fail(FLB_EHIP, "init kernel launch failed");
            return bail(0);
        }
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        fail(FLB_EHIP, "initialisation failed");
        return bail(0);
    }
    return h;
}

// Device address of `scratch` on device `dev`, looked up once per device
// with that device current and kept.
int scratch_on_device(int dev, double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return fail(FLB_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        int cur = -1;
        FLB_HIP(hipGetDevice(&cur));
        if (cur != dev) FLB_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(FLB_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return FLB_OK;
}

int check_handle(flb_t *h)
{
    if (!h) return fail(FLB_EINVAL, "NULL handle");
    return FLB_OK;
}

int check_lattice(flb_t *h, int lattice)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (lattice < 0 || lattice >= (int)h->params.size())
        return fail(FLB_EINVAL, "lattice index out of range");
    return FLB_OK;
}

}  // namespace

extern "C" {

const char *flb_last_error(void) { return g_err.c_str(); }

flb_t *flb_create_batch(int n, const flb_lattice_spec *specs, uint64_t seed, int storage,
                        uint32_t flags)
{
    return create_impl(n, specs, seed, storage, flags);
}

flb_t *flb_create_ex(int nx, int ny, const double tau[9], double theta, double rho0,
                     const double u0[2], uint64_t seed, int storage, uint32_t stream_id,
                     uint32_t flags)
{
    if (!tau || !u0) {
        fail(FLB_EINVAL, "tau and u0 must not be NULL");
        return nullptr;
    }
    flb_lattice_spec s;
    std::memset(&s, 0, sizeof s);
    s.nx = nx;
    s.ny = ny;
    for (int a = 0; a < 9; ++a) s.tau[a] = tau[a];
    s.theta = theta;
    s.rho0 = rho0;
    s.u0[0] = u0[0];
    s.u0[1] = u0[1];
    s.stream_id = stream_id;
    return create_impl(1, &s, seed, storage, flags);
}

flb_t *flb_create(int nx, int ny, const double tau[9], double theta, double rho0,
                  const double u0[2], uint64_t seed)
{
    return flb_create_ex(nx, ny, tau, theta, rho0, u0, seed, FLB_STORAGE_F32, 0, 0);
}

void flb_destroy(flb_t *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own) (void)hipStreamSynchronize(h->own);
    if (h->aux) (void)hipStreamSynchronize(h->aux);
    clear_graphs(h);
    void *ptrs[] = {h->pops[0], h->d_params, h->d_step, h->d_red, h->d_items,
                    h->d_plans, h->d_tables, h->d_spec, h->d_acc, h->d_rows, h->d_cols,
                    h->d_accum, h->d_cols_l, h->d_fld, h->d_fields,
                    h->d_csum_part, h->d_csum, h->d_cols_lm, h->d_cols_m, h->d_rows_m,
                    h->d_rows_blue, h->d_stash, h->d_flush, h->d_items2, h->d_cols_blue};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &set : h->pipe)
        for (auto &pl : set)
            if (pl.d_sched) (void)hipFree(pl.d_sched);
    for (hipEvent_t e : {h->ev, h->ev_fork, h->ev_read, h->ev_done})
        if (e) (void)hipEventDestroy(e);
    for (auto *v : {&h->timed, &h->spare_events})
        for (auto &pr : *v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

int flb_set_stream(flb_t *h, void *hip_stream)
{
    if (check_handle(h)) return FLB_EINVAL;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->own;
    if (s != h->stream) {
        // order the new stream after everything already enqueued
        FLB_HIP(hipEventRecord(h->ev, h->stream));
        FLB_HIP(hipStreamWaitEvent(s, h->ev, 0));
        h->stream = s;
    }
    return FLB_OK;
}

int flb_synchronize(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = settle_due(h);
    if (rc) return rc;
    FLB_HIP(hipStreamSynchronize(h->stream));
    return FLB_OK;
}

int flb_step(flb_t *h, int64_t nsteps)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = check_time(h, nsteps);
    if (rc) return rc;
    rc = enqueue_steps_overlapped(h, nsteps, h->stream);
    if (rc) return rc;
    h->t += nsteps;
    return FLB_OK;
}

// Registers a sample of the current state; with sample overlap its kernels
// are enqueued with the next steps (beside them) or by the next call that
// needs them, otherwise at once.
int flb_accumulate_correlators(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = setup_correlators(h);
    if (rc) return rc;
    if ((rc = settle_due(h))) return rc;  // a second sample of the same state
    h->due = true;
    h->nsamples += 1;
    if (!h->overlap) return settle_due(h);
    return FLB_OK;
}

int flb_set_sample_overlap(flb_t *h, int on)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = settle_due(h);
    if (rc) return rc;
    if (h->overlap != (on != 0)) {
        h->overlap = on != 0;
        clear_graphs(h);
    }
    return FLB_OK;
}

int flb_get_sample_overlap(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    return h->overlap ? 1 : 0;
}

int flb_set_launch_timing(flb_t *h, int on)
{
    if (check_handle(h)) return FLB_EINVAL;
    h->timing = on != 0;
    return FLB_OK;
}

int flb_get_launch_timing_kinds(flb_t *h, int64_t launches[3], double total_ms[3])
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!launches || !total_ms) return fail(FLB_EINVAL, "launches and total_ms must not be NULL");
    FLB_HIP(hipStreamSynchronize(h->stream));
    for (int q = 0; q < 3; ++q) {
        launches[q] = 0;
        total_ms[q] = 0.0;
    }
    for (size_t i = 0; i < h->timed.size(); ++i) {
        float ms = 0.0f;
        FLB_HIP(hipEventElapsedTime(&ms, h->timed[i].first, h->timed[i].second));
        const int q = h->timed_steps[i] - 1;
        launches[q] += 1;
        total_ms[q] += ms;
    }
    h->spare_events.insert(h->spare_events.end(), h->timed.begin(), h->timed.end());
    h->timed.clear();
    h->timed_steps.clear();
    return FLB_OK;
}

int flb_get_launch_timing(flb_t *h, int64_t *launches, double *total_ms)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!launches || !total_ms) return fail(FLB_EINVAL, "launches and total_ms must not be NULL");
    int64_t n[3];
    double ms[3];
    if (int rc = flb_get_launch_timing_kinds(h, n, ms)) return rc;
    *launches = n[0] + n[1] + n[2];
    *total_ms = ms[0] + ms[1] + ms[2];
    return FLB_OK;
}

// One period of `every` steps followed by a sample, from a captured graph.
static int run_period_graph(flb_t *h, int every)
{
    const bool due0 = h->due;
    const GraphKey key{every, h->cur, h->pending, due0 ? 1 : 0};
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        // capture on the handle's own stream (capturing the legacy default
        // stream is not allowed), then launch on the current stream; a due
        // sample forks onto the side stream inside the capture and joins
        // before its end
        const int cur0 = h->cur;
        const int pending0 = h->pending;
        FLB_HIP(hipStreamBeginCapture(h->own, hipStreamCaptureModeRelaxed));
        h->capturing = true;
        int rc = enqueue_steps_overlapped(h, every, h->own);
        if (!rc && !h->overlap) rc = enqueue_sample(h, h->own);  // the period's own sample
        h->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->own, &g);
        h->cur = cur0;
        h->pending = pending0;
        h->due = due0;
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(FLB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return fail(FLB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = h->graphs.emplace(key, ex).first;
    }
    FLB_HIP(hipGraphLaunch(it->second, h->stream));
    if (step_launches(h, every) & 1) h->cur ^= 1;
    // samples the graph enqueued: the due one, and without overlap its own
    const int enqueued = (due0 ? 1 : 0) + (h->overlap ? 0 : 1);
    if (h->defer) h->pending = (h->pending + enqueued) % kDeferK;
    h->t += every;
    h->nsamples += 1;
    h->due = h->overlap;  // with overlap the period's sample runs beside the next steps
    return FLB_OK;
}

int flb_run(flb_t *h, int64_t nsteps, int sample_every)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (sample_every < 0) return fail(FLB_EINVAL, "sample_every must be >= 0");
    int rc = check_time(h, nsteps);
    if (rc) return rc;
    if (sample_every == 0) return flb_step(h, nsteps);
    rc = setup_correlators(h);
    if (rc) return rc;
    while (nsteps > 0) {
        const int64_t phase = h->t % sample_every;
        if (phase == 0 && nsteps >= sample_every) {
            rc = run_period_graph(h, sample_every);
            if (rc) return rc;
            nsteps -= sample_every;
            continue;
        }
        const int64_t to_sample = sample_every - phase;
        const int64_t n = std::min(nsteps, to_sample);
        rc = flb_step(h, n);
        if (rc) return rc;
        nsteps -= n;
        if (n == to_sample) {
            rc = flb_accumulate_correlators(h);
            if (rc) return rc;
        }
    }
    return FLB_OK;
}

int flb_read_correlators(flb_t *h, int lattice, double *out, size_t n_doubles, int64_t *nsamples)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out) return fail(FLB_EINVAL, "out must not be NULL");
    int rc = setup_correlators(h);
    if (rc) return rc;
    const LatticeParams &P = h->params[lattice];
    const size_t need = (size_t)h->nkinds * P.ny * P.nkx;
    if (n_doubles < need) return fail(FLB_ESIZE, "output buffer too small for the correlators");
    if ((rc = settle_due(h)) || (rc = flush_pending(h))) return rc;
    FLB_HIP(hipStreamSynchronize(h->stream));
    // the device planes are column-tiled with kxp >= nkx columns: copied
    // whole, then put in row order
    const int ny = P.ny, nkx = P.nkx;
    const int64_t plane = (int64_t)ny * P.kxp;
    std::vector<double> tiled((size_t)(h->nkinds * plane));
    FLB_HIP(hipMemcpy(tiled.data(), h->d_acc + P.acc_base, tiled.size() * sizeof(double),
                      hipMemcpyDeviceToHost));
    for (int q = 0; q < h->nkinds; ++q) {
        const double *src = tiled.data() + q * plane;
        double *dst = out + (size_t)q * ny * nkx;
        for (int x0 = 0; x0 < nkx; x0 += kTileCols) {
            const int w = std::min(kTileCols, nkx - x0);
            const double *t = src + spec_offset(0, x0, ny);
            for (int y = 0; y < ny; ++y)
                for (int c = 0; c < w; ++c) dst[(size_t)y * nkx + x0 + c] = t[y * kTileCols + c];
        }
    }
    if (nsamples) *nsamples = h->nsamples;
    return FLB_OK;
}

int flb_read_normalized(flb_t *h, int lattice, double *out, size_t n_doubles, int64_t *nsamples)
{
    int64_t ns = 0;
    int rc = flb_read_correlators(h, lattice, out, n_doubles, &ns);
    if (rc) return rc;
    if (nsamples) *nsamples = ns;
    const flb_lattice_spec &s = h->specs[lattice];
    if (ns <= 0) return fail(FLB_ESTATE, "no correlator sample to normalise");
    if (!(s.theta > 0)) return fail(FLB_ESTATE, "theta = 0: no fluctuation scale to normalise by");
    // Sec. 3, Eqs. (11)-(12) at the noise temperature theta (mu = 3 theta)
    const double V = (double)s.nx * (double)s.ny, mu = 3.0 * s.theta, rho0 = s.rho0;
    const double cs = 1.0 / std::sqrt(3.0), theta = s.theta;
    double norm[FLB_NKINDS_MOMENTS];
    norm[0] = 1.0 / (V * mu * rho0);
    norm[1] = norm[2] = 1.0 / (V * rho0 * theta);
    norm[3] = norm[4] = norm[5] = norm[6] = rho0 / (V * theta);
    for (int q = 7; q < 11; ++q) norm[q] = 1.0 / (V * mu * rho0 * cs);
    for (int q = 11; q < 15; ++q) norm[q] = 1.0 / (V * mu * cs);
    for (int q = 15; q < FLB_NKINDS_MOMENTS; ++q) norm[q] = 1.0 / (V * mu * rho0);
    const size_t plane = (size_t)s.ny * (size_t)(s.nx / 2 + 1);
    for (int q = 0; q < h->nkinds; ++q) {
        double *p = out + q * plane;
        for (size_t k = 0; k < plane; ++k) p[k] = p[k] / (double)ns * norm[q];
    }
    return FLB_OK;
}

int flb_flush_correlators(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!h->corr_ready) return FLB_OK;  // no sample was ever taken
    int rc = settle_due(h);
    if (rc) return rc;
    return flush_pending(h);
}

int flb_reset_correlators(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = setup_correlators(h);
    if (rc) return rc;
    FLB_HIP(launch_fill(h->d_acc, (size_t)h->acc_elems, h->stream));
    h->nsamples = 0;
    h->pending = 0;  // stashed and due samples are dropped with the sums
    h->due = false;
    return FLB_OK;
}

int flb_get_populations(flb_t *h, int lattice, double *out, size_t n)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out) return fail(FLB_EINVAL, "out must not be NULL");
    const LatticeParams &P = h->params[lattice];
    const size_t need = 9 * (size_t)P.nx * (size_t)P.ny;
    if (n < need) return fail(FLB_ESIZE, "output buffer smaller than 9*nx*ny");
    double *d = nullptr;
    FLB_HIP(hipMalloc((void **)&d, need * sizeof(double)));
    hipError_t e = launch_get(h->view(), lattice, P.nx, P.ny, d, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(out, d, need * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FLB_EHIP, std::string("get populations: ") + hipGetErrorString(e));
    return FLB_OK;
}

int flb_get_populations_noalloc(flb_t *h, int lattice, double *out, size_t n)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out) return fail(FLB_EINVAL, "out must not be NULL");
    const LatticeParams &P = h->params[lattice];
    const size_t need = 9 * (size_t)P.nx * (size_t)P.ny;
    if (n < need) return fail(FLB_ESIZE, "output buffer smaller than 9*nx*ny");
    if (need > kNoAllocDoubles)
        return fail(FLB_ESIZE, "lattice too large for the no-allocation read: 9*nx*ny must be "
                               "at most 8388608 (use flb_get_populations)");
    double *d = nullptr;
    int rc = scratch_on_device(h->device, &d);
    if (rc) return rc;
    // every value the copy reads is written by the kernel first: nothing
    // needs clearing
    FLB_HIP(launch_get(h->view(), lattice, P.nx, P.ny, d, h->stream));
    FLB_HIP(hipMemcpyAsync(out, d, need * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    FLB_HIP(hipStreamSynchronize(h->stream));
    return FLB_OK;
}

int flb_set_populations(flb_t *h, int lattice, const double *in, size_t n)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!in) return fail(FLB_EINVAL, "in must not be NULL");
    const LatticeParams &P = h->params[lattice];
    const size_t need = 9 * (size_t)P.nx * (size_t)P.ny;
    if (n < need) return fail(FLB_ESIZE, "input buffer smaller than 9*nx*ny");
    int rc = settle_due(h);
    if (rc) return rc;
    double *d = nullptr;
    FLB_HIP(hipMalloc((void **)&d, need * sizeof(double)));
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(d, in, need * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_set(h->view(), lattice, P.nx, P.ny, d, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FLB_EHIP, std::string("set populations: ") + hipGetErrorString(e));
    return FLB_OK;
}

int flb_conservation(flb_t *h, int lattice, double out[5])
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out) return fail(FLB_EINVAL, "out must not be NULL");
    const LatticeParams &P = h->params[lattice];
    const int nb = (int)std::min<int64_t>(h->red_blocks,
                                          ((int64_t)P.nx * P.ny + kThreads - 1) / kThreads);
    double *res = h->d_red + (size_t)h->red_blocks * 9;
    FLB_HIP(launch_conservation(h->view(), lattice, P.nx, P.ny, h->d_red, nb, res, h->stream));
    FLB_HIP(hipStreamSynchronize(h->stream));
    FLB_HIP(hipMemcpy(out, res, 5 * sizeof(double), hipMemcpyDeviceToHost));
    return FLB_OK;
}

int flb_sample_conservation(flb_t *h, int lattice, double out[5])
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out) return fail(FLB_EINVAL, "out must not be NULL");
    if (!h->corr_ready || h->nsamples == 0)
        return fail(FLB_ESTATE, "no correlator sample taken since the last reset");
    int rc = settle_due(h);
    if (rc) return rc;
    // the stream is ordered after the last sample's row transforms (a sample
    // beside the steps joins it at their end)
    FLB_HIP(launch_corr_csum(h->view(), h->stream));
    FLB_HIP(hipStreamSynchronize(h->stream));
    FLB_HIP(hipMemcpy(out, h->d_csum + 5 * (size_t)lattice, 5 * sizeof(double),
                      hipMemcpyDeviceToHost));
    return FLB_OK;
}

int flb_conservation_dev(flb_t *h, int lattice, double *out_dev)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (!out_dev) return fail(FLB_EINVAL, "out_dev must not be NULL");
    const LatticeParams &P = h->params[lattice];
    const int nb = (int)std::min<int64_t>(h->red_blocks,
                                          ((int64_t)P.nx * P.ny + kThreads - 1) / kThreads);
    FLB_HIP(launch_conservation(h->view(), lattice, P.nx, P.ny, h->d_red, nb, out_dev, h->stream));
    return FLB_OK;
}

int flb_thermalize(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    int rc = settle_due(h);
    if (rc) return rc;
    for (size_t l = 0; l < h->params.size(); ++l) {
        const LatticeParams &P = h->params[l];
        const int nb = (int)std::min<int64_t>(h->red_blocks,
                                          ((int64_t)P.nx * P.ny + kThreads - 1) / kThreads);
        double *sums = h->d_red + (size_t)h->red_blocks * 9;
        FLB_HIP(launch_thermalize(h->view(), (int)l, P.nx, P.ny, h->d_red, nb, sums, h->stream));
    }
    FLB_HIP(hipStreamSynchronize(h->stream));
    return FLB_OK;
}

int flb_debug_noise(flb_t *h, int lattice, uint32_t t, int64_t site0, int64_t nsites,
                    uint32_t *words_out, float *z_out)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    if (site0 < 0 || nsites < 0 || site0 + nsites > ((int64_t)1 << 32))
        return fail(FLB_EINVAL, "site range outside the 32-bit counter word");
    if (nsites == 0) return FLB_OK;
    uint32_t *dw = nullptr;
    float *dz = nullptr;
    FLB_HIP(hipMalloc((void **)&dw, (size_t)nsites * 4 * sizeof(uint32_t)));
    hipError_t e = hipMalloc((void **)&dz, (size_t)nsites * 6 * sizeof(float));
    if (e == hipSuccess)
        e = launch_debug_noise(h->seed, h->params[lattice].stream_id, t, site0, nsites, dw, dz,
                               h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && words_out)
        e = hipMemcpy(words_out, dw, (size_t)nsites * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && z_out)
        e = hipMemcpy(z_out, dz, (size_t)nsites * 6 * sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(dw);
    if (dz) (void)hipFree(dz);
    if (e != hipSuccess) return fail(FLB_EHIP, std::string("debug noise: ") + hipGetErrorString(e));
    return FLB_OK;
}

int64_t flb_get_step(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    return h->t;
}

int flb_set_step(flb_t *h, int64_t t)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (t < 0 || t >= (int64_t)0xFFFFFFFF) return fail(FLB_EINVAL, "t outside [0, 2^32 - 1)");
    const uint32_t v = (uint32_t)t;
    FLB_HIP(hipStreamSynchronize(h->stream));
    FLB_HIP(hipMemcpy(h->d_step, &v, sizeof v, hipMemcpyHostToDevice));
    h->t = t;
    return FLB_OK;
}

int flb_num_kinds(flb_t *h)
{
    if (check_handle(h)) return FLB_EINVAL;
    return h->nkinds;
}

int flb_num_lattices(flb_t *h)
{
    if (check_handle(h)) return -1;
    return (int)h->params.size();
}

int flb_lattice_info(flb_t *h, int lattice, int32_t *nx, int32_t *ny, int32_t *nkx)
{
    if (check_lattice(h, lattice)) return FLB_EINVAL;
    const LatticeParams &P = h->params[lattice];
    if (nx) *nx = P.nx;
    if (ny) *ny = P.ny;
    if (nkx) *nkx = P.nkx;
    return FLB_OK;
}

int flb_storage_info(flb_t *h, int32_t *storage, int32_t *bytes_per_value)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (storage) *storage = h->storage;
    if (bytes_per_value) *bytes_per_value = h->elem_bytes;
    return FLB_OK;
}

int flb_set_step_config(flb_t *h, int tile_w, int sites, int nontemporal)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!step_tile_supported(tile_w, sites)) return fail(FLB_EINVAL, "unsupported step tile");
    FLB_HIP(hipStreamSynchronize(h->stream));
    h->tile_w = tile_w;
    h->sites = sites;
    h->nontemporal = nontemporal != 0;
    clear_graphs(h);
    return build_step_items(h);
}

int flb_set_time_blocking(flb_t *h, int steps_per_launch, int tile_w)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (steps_per_launch < 1 || steps_per_launch > 3)
        return fail(FLB_EINVAL, "steps_per_launch must be 1, 2 or 3");
    if (!step2_tile_supported(tile_w)) return fail(FLB_EINVAL, "unsupported two-step tile");
    FLB_HIP(hipStreamSynchronize(h->stream));
    h->tblock = steps_per_launch;
    h->tile2 = tile_w;
    clear_graphs(h);
    return build_step_items(h);
}

int flb_get_time_blocking(flb_t *h, int *steps_per_launch, int *tile_w)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (steps_per_launch) *steps_per_launch = h->tblock;
    if (tile_w) *tile_w = h->tile2;
    return FLB_OK;
}

int flb_set_lattice_tiles(flb_t *h, const int *tile_w)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!tile_w) return fail(FLB_EINVAL, "tile_w must not be NULL");
    std::vector<int8_t> lt(h->params.size());
    for (size_t l = 0; l < lt.size(); ++l) {
        if (tile_w[l] != 32 && tile_w[l] != 64)
            return fail(FLB_EINVAL, "per-lattice two-step tiles are 32 or 64 sites wide");
        lt[l] = tile_w[l] == 32 ? 5 : 6;
    }
    FLB_HIP(hipStreamSynchronize(h->stream));
    h->tblock = 2;
    h->tile2 = 0;
    h->ltile = lt;
    clear_graphs(h);
    return build_step_items(h);
}

int flb_get_lattice_tiles(flb_t *h, int *tile_w)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (!tile_w) return fail(FLB_EINVAL, "tile_w must not be NULL");
    for (size_t l = 0; l < h->params.size(); ++l)
        tile_w[l] = h->tile2 ? h->tile2 : 1 << h->ltile[l];
    return FLB_OK;
}

int flb_get_step_config(flb_t *h, int *tile_w, int *sites, int *nontemporal)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (tile_w) *tile_w = h->tile_w;
    if (sites) *sites = h->sites;
    if (nontemporal) *nontemporal = h->nontemporal ? 1 : 0;
    return FLB_OK;
}

}  // extern "C"

// A step launch shape: one-step tile width, sites per thread, streaming
// accesses, steps per launch (1, 2 or 3), two- and three-step tile width
// (0: per lattice, log2 of each lattice's in lt).
struct StepShape {
    int tw, sv, nt, tb, t2;
    std::vector<int8_t> lt;
};

static void apply_shape(flb_t *h, const StepShape &c)
{
    h->tile_w = c.tw;
    h->sites = c.sv;
    h->nontemporal = c.nt != 0;
    h->tblock = c.tb;
    h->tile2 = c.t2;
    h->ltile = c.t2 == 0 ? c.lt : std::vector<int8_t>();
}

static std::string tune_key(const flb_t *h, const char *kind, int every)
{
    int64_t total = 0;
    int maxside = 0;
    for (auto &P : h->params) {
        total += (int64_t)P.nx * P.ny;
        maxside = std::max(maxside, std::max(P.nx, P.ny));
    }
    char key[160];
    snprintf(key, sizeof key, "%s:%d:%zu:%lld:%d:%d:%d", kind, h->storage, h->params.size(),
             (long long)total, maxside, h->noise ? 1 : 0, every);
    return key;
}

// A shape from the FLB_AUTOTUNE_CACHE file, if it names one for this key
// (the last such line).  Lines: key tw sv nt tb t2 ms, where t2 is a width
// or "L" followed by each lattice's log2 width (per-lattice tiles).
static bool cached_shape(const char *cache, const std::string &key, size_t nlat, StepShape &c,
                         double &ms)
{
    if (!cache) return false;
    std::ifstream in(cache);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string k, t2s;
        StepShape x{};
        double t = 0;
        if (!(ls >> k >> x.tw >> x.sv >> x.nt >> x.tb >> t2s >> t) || k != key) continue;
        if (!t2s.empty() && t2s[0] == 'L') {
            if (t2s.size() != nlat + 1) continue;
            bool ok = true;
            for (size_t l = 0; l < nlat; ++l) {
                const char ch = t2s[l + 1];
                ok = ok && (ch == '5' || ch == '6');
                x.lt.push_back((int8_t)(ch - '0'));
            }
            if (!ok || x.tb != 2) continue;
            x.t2 = 0;
        } else {
            x.t2 = atoi(t2s.c_str());
            if (!step2_tile_supported(x.t2)) continue;
        }
        if (step_tile_supported(x.tw, x.sv) && x.tb >= 1 && x.tb <= 3) {
            found = true;
            c = x;
            ms = t;
        }
    }
    return found;
}

static void cache_shape(const char *cache, const std::string &key, const StepShape &c, double ms)
{
    if (!cache) return;
    std::string t2s = std::to_string(c.t2);
    if (c.t2 == 0) {
        t2s = "L";
        for (int8_t v : c.lt) t2s += (char)('0' + v);
    }
    if (FILE *fp = fopen(cache, "a")) {
        fprintf(fp, "%s %d %d %d %d %s %.6f\n", key.c_str(), c.tw, c.sv, c.nt, c.tb, t2s.c_str(), ms);
        fclose(fp);
    }
}

// Runs body(h) between a saved and a restored state: the populations, the
// device and host step counters and the buffer parity are put back
// afterwards, and launch timing is off meanwhile (the candidates' launches
// are not the caller's).
template <typename F> static int with_saved_state(flb_t *h, F body)
{
    if (int rc0 = settle_due(h)) return rc0;
    FLB_HIP(hipStreamSynchronize(h->stream));
    const size_t bytes = (size_t)h->total_elems * h->elem_bytes;
    void *saved = nullptr;
    FLB_HIP(hipMalloc(&saved, bytes));
    uint32_t step0 = 0;
    const int cur0 = h->cur;
    const int64_t t0 = h->t;
    const bool timing0 = h->timing;
    const StepShape shape0{h->tile_w, h->sites, h->nontemporal ? 1 : 0, h->tblock, h->tile2,
                           h->ltile};
    h->timing = false;
    hipError_t e = hipMemcpyAsync(saved, h->pops[cur0], bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&step0, h->d_step, sizeof step0, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    int rc = e == hipSuccess ? body(h) : FLB_OK;
    h->timing = timing0;
    apply_shape(h, shape0);
    h->cur = cur0;
    h->t = t0;
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->pops[cur0], saved, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_step, &step0, sizeof step0, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(saved);
    clear_graphs(h);
    if (rc != FLB_OK) return rc;
    if (e != hipSuccess) return fail(FLB_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    return build_step_items(h);
}

// Times the given launch shapes alone (nsteps steps each, whole pairs for
// the two-step kernel) in kRounds round-robin passes, each shape keeping
// its fastest pass, so that a slow moment of the device does not decide; ms
// per step into best.
static int time_shapes(flb_t *h, int nsteps, const std::vector<StepShape> &shapes,
                       std::vector<float> &best)
{
    constexpr int kRounds = 3;
    best.assign(shapes.size(), 1e30f);
    return with_saved_state(h, [&](flb_t *hh) -> int {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        int rc = FLB_OK;
        for (int round = 0; round < kRounds && e == hipSuccess && rc == FLB_OK; ++round)
            for (size_t i = 0; i < shapes.size() && e == hipSuccess && rc == FLB_OK; ++i) {
                apply_shape(hh, shapes[i]);
                const int tb = shapes[i].tb;  // whole launches
                const int n = (nsteps + tb - 1) / tb * tb;
                if ((rc = build_step_items(hh)) != FLB_OK) break;
                if ((rc = enqueue_steps(hh, 2, hh->stream)) != FLB_OK) break;
                e = hipEventRecord(e0, hh->stream);
                if (e == hipSuccess && (rc = enqueue_steps(hh, n, hh->stream)) != FLB_OK) break;
                if (e == hipSuccess) e = hipEventRecord(e1, hh->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess) best[i] = std::min(best[i], ms / n);
            }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (rc != FLB_OK) return rc;
        if (e != hipSuccess) return fail(FLB_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        return FLB_OK;
    });
}

// Every supported launch shape timed alone, fastest first.
static int time_every_shape(flb_t *h, int nsteps, std::vector<std::pair<float, StepShape>> &out)
{
    std::vector<StepShape> shapes;
    for (int tw : {64, 128, 256})
        for (int sv : {1, 2, 4})
            for (int nt = 0; nt < 2; ++nt) shapes.push_back({tw, sv, nt, 1, 64, {}});
    for (int tb : {2, 3})
        for (int t2 : {32, 64, 128})
            for (int nt = 0; nt < 2; ++nt) shapes.push_back({h->tile_w, h->sites, nt, tb, t2, {}});
    std::vector<float> best;
    if (int rc = time_shapes(h, nsteps, shapes, best)) return rc;
    out.clear();
    for (size_t i = 0; i < shapes.size(); ++i) out.push_back({best[i], shapes[i]});
    std::stable_sort(out.begin(), out.end(),
                     [](const std::pair<float, StepShape> &a, const std::pair<float, StepShape> &b) {
                         return a.first < b.first;
                     });
    return FLB_OK;
}

// Collisions of the two-step kernel's phase 1 on lattice P with tiles of
// width 2^lg: tiles x (tile + ring).
static int64_t step2_collisions(const LatticeParams &P, int lg)
{
    const int w = 1 << lg, th = 1024 / w;
    return (int64_t)((P.nx + w - 1) / w) * ((P.ny + th - 1) / th) * (w + 2) * (th + 2);
}

// The two-step tile per size class of a batch: lattices whose sides round
// up to the same powers of two form a class, and each class takes the
// faster of 32 x 32 and 64 x 16 tiles, timed on its own lattices (nsteps
// steps, launches of the per-lattice kernel over that class's tiles only,
// three round-robin passes, fastest pass kept).  Where the two are within
// 1 %, the shape with fewer phase-1 collisions is kept.  Streaming accesses
// as nt says.  lt receives log2 of each lattice's tile width.
static int tune_lattice_tiles(flb_t *h, int nsteps, int nt, std::vector<int8_t> &lt)
{
    constexpr int kRounds = 3;
    const size_t nlat = h->params.size();
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (size_t l = 0; l < nlat; ++l)
        classes[{log2i(h->params[l].nx), log2i(h->params[l].ny)}].push_back((int)l);
    lt.assign(nlat, 6);
    const int launches = std::max(1, (nsteps + 1) / 2);
    return with_saved_state(h, [&](flb_t *hh) -> int {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        StepItem *d_it[2] = {nullptr, nullptr};
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        int rc = FLB_OK;
        for (auto cit = classes.begin(); cit != classes.end() && e == hipSuccess && rc == FLB_OK;
             ++cit) {
            std::vector<char> only(nlat, 0);
            for (int l : cit->second) only[l] = 1;
            int n[2];
            for (int o = 0; o < 2 && rc == FLB_OK; ++o) {
                const std::vector<int8_t> cand(nlat, (int8_t)(5 + o));
                const std::vector<StepItem> items = step2_items(hh, &cand, 0, &only);
                n[o] = (int)items.size();
                rc = upload(&d_it[o], items);
            }
            float best[2] = {1e30f, 1e30f};
            for (int round = 0; round < kRounds && e == hipSuccess && rc == FLB_OK; ++round)
                for (int o = 0; o < 2 && e == hipSuccess; ++o) {
                    // the same launch repeated on the same buffers: the
                    // state is put back afterwards
                    e = launch_step2(hh->view(), d_it[o], n[o], 0, 0, nt != 0, hh->noise, hh->stream);
                    if (e == hipSuccess) e = hipEventRecord(e0, hh->stream);
                    for (int k = 0; k < launches && e == hipSuccess; ++k)
                        e = launch_step2(hh->view(), d_it[o], n[o], 0, 0, nt != 0, hh->noise,
                                         hh->stream);
                    if (e == hipSuccess) e = hipEventRecord(e1, hh->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e == hipSuccess) best[o] = std::min(best[o], ms);
                }
            int8_t pick;
            if (best[0] < 0.99f * best[1]) pick = 5;
            else if (best[1] < 0.99f * best[0]) pick = 6;
            else {
                int64_t c5 = 0, c6 = 0;
                for (int l : cit->second) {
                    c5 += step2_collisions(hh->params[l], 5);
                    c6 += step2_collisions(hh->params[l], 6);
                }
                pick = c5 < c6 ? 5 : 6;
            }
            for (int l : cit->second) lt[l] = pick;
        }
        for (StepItem *p : d_it)
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (rc != FLB_OK) return rc;
        if (e != hipSuccess) return fail(FLB_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        return FLB_OK;
    });
}

// For a batch whose chosen shape is two-step: the per-class tiles as a
// further candidate shape (none if every class kept the chosen width).
static int lattice_tile_candidate(flb_t *h, int nsteps, const StepShape &chosen,
                                  std::vector<StepShape> &extra)
{
    extra.clear();
    if (h->params.size() < 2 || chosen.tb < 2) return FLB_OK;
    std::vector<int8_t> lt;
    if (int rc = tune_lattice_tiles(h, nsteps, chosen.nt, lt)) return rc;
    bool same = chosen.t2 == 32 || chosen.t2 == 64;
    for (int8_t v : lt) same = same && (1 << v) == chosen.t2;
    if (same) return FLB_OK;
    StepShape m = chosen;
    bool uniform = true;
    for (int8_t v : lt) uniform = uniform && v == lt[0];
    m.t2 = uniform ? 1 << lt[0] : 0;
    m.lt = uniform ? std::vector<int8_t>() : lt;
    if (!uniform) m.tb = 2;  // per-lattice tiles: the two-step kernel
    extra.push_back(m);
    return FLB_OK;
}

extern "C" {

int flb_autotune(flb_t *h, int nsteps, double *ms_out)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (nsteps < 1) return fail(FLB_EINVAL, "nsteps must be >= 1");
    const std::string key = tune_key(h, "flb-step", 0);
    const char *cache = getenv("FLB_AUTOTUNE_CACHE");
    StepShape c{};
    double ms = 0;
    if (cached_shape(cache, key, h->params.size(), c, ms)) {
        apply_shape(h, c);
        if (ms_out) *ms_out = ms;
        clear_graphs(h);
        return build_step_items(h);
    }
    std::vector<std::pair<float, StepShape>> t;
    if (int rc = time_every_shape(h, nsteps, t)) return rc;
    StepShape pick = t[0].second;
    float pick_ms = t[0].first;
    // a batch: the per-class tiles against the fastest shape, timed together
    std::vector<StepShape> extra;
    if (int rc = lattice_tile_candidate(h, nsteps, pick, extra)) return rc;
    if (!extra.empty()) {
        std::vector<StepShape> two{pick, extra[0]};
        std::vector<float> best;
        if (int rc = time_shapes(h, nsteps, two, best)) return rc;
        if (best[1] < best[0]) {
            pick = extra[0];
            pick_ms = best[1];
        }
    }
    apply_shape(h, pick);
    clear_graphs(h);
    if (ms_out) *ms_out = pick_ms;
    cache_shape(cache, key, pick, pick_ms);
    return build_step_items(h);
}

int flb_autotune_path(flb_t *h, int nsteps, int sample_every, double *ms_out)
{
    if (check_handle(h)) return FLB_EINVAL;
    if (nsteps < 1 || sample_every < 1) return fail(FLB_EINVAL, "nsteps and sample_every must be >= 1");
    if (h->nsamples != 0 || h->due || h->pending)
        return fail(FLB_ESTATE, "tune the whole path before taking correlator samples");
    const std::string key = tune_key(h, "flb-path", sample_every);
    const char *cache = getenv("FLB_AUTOTUNE_CACHE");
    StepShape c{};
    double ms = 0;
    if (cached_shape(cache, key, h->params.size(), c, ms)) {
        apply_shape(h, c);
        if (ms_out) *ms_out = ms;
        clear_graphs(h);
        return build_step_items(h);
    }
    int rc = setup_correlators(h);
    if (rc) return rc;
    std::vector<std::pair<float, StepShape>> t;
    if ((rc = time_every_shape(h, nsteps, t))) return rc;
    // the shapes within 4 % of the fastest alone (at most four), and for a
    // batch the per-class tiles, are timed on whole periods: sample_every
    // steps and a sample, the sample beside the next period's steps as with
    // the handle's own calls, in two round-robin passes of kDeferK periods
    // (a whole accumulation cycle)
    std::vector<StepShape> cand;
    for (const auto &x : t)
        if (x.first <= 1.04f * t[0].first && cand.size() < 4) cand.push_back(x.second);
    std::vector<StepShape> extra;
    if ((rc = lattice_tile_candidate(h, nsteps, cand[0], extra))) return rc;
    cand.insert(cand.end(), extra.begin(), extra.end());
    std::vector<float> best(cand.size(), 1e30f);
    if (cand.size() > 1) {
        rc = with_saved_state(h, [&](flb_t *hh) -> int {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            hipError_t e = hipEventCreate(&e0);
            if (e == hipSuccess) e = hipEventCreate(&e1);
            int r = FLB_OK;
            auto periods = [&](int n) -> int {
                for (int p = 0; p < n; ++p) {
                    if (int q = flb_step(hh, sample_every)) return q;
                    if (int q = flb_accumulate_correlators(hh)) return q;
                }
                if (int q = settle_due(hh)) return q;
                return flush_pending(hh);
            };
            for (int round = 0; round < 2 && e == hipSuccess && r == FLB_OK; ++round)
                for (size_t i = 0; i < cand.size() && e == hipSuccess && r == FLB_OK; ++i) {
                    apply_shape(hh, cand[i]);
                    clear_graphs(hh);
                    if ((r = build_step_items(hh)) != FLB_OK) break;
                    if ((r = periods(4)) != FLB_OK) break;
                    e = hipEventRecord(e0, hh->stream);
                    if (e == hipSuccess && (r = periods(kDeferK)) != FLB_OK) break;
                    if (e == hipSuccess) e = hipEventRecord(e1, hh->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float t_ms = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
                    if (e == hipSuccess)
                        best[i] = std::min(best[i], t_ms / ((float)kDeferK * sample_every));
                }
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            // the tuning's samples leave nothing behind
            const int rr = flb_reset_correlators(hh);
            if (r == FLB_OK) r = rr;
            if (r == FLB_OK && e != hipSuccess)
                r = fail(FLB_EHIP, std::string("autotune: ") + hipGetErrorString(e));
            return r;
        });
        if (rc) return rc;
    } else {
        best[0] = t[0].first;
    }
    size_t k = 0;
    for (size_t i = 1; i < cand.size(); ++i)
        if (best[i] < best[k]) k = i;
    apply_shape(h, cand[k]);
    clear_graphs(h);
    if (ms_out) *ms_out = best[k];
    cache_shape(cache, key, cand[k], best[k]);
    return build_step_items(h);
}

}  // extern "C"
