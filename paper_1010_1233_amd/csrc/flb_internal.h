// flb_internal.h -- data shared by the host runtime and the gfx950 kernels.
//
// Device layout of one handle (all lattices of a batch share each buffer):
//   pops[2]  : two population buffers (ping-pong), per lattice 9 planes of
//              ny rows of px values (px = nx rounded up to 4; the values
//              past nx are padding, never part of the lattice) in the
//              storage format, plane i at base + i*plane.
//              They hold the POST-collision state of the last step; the
//              state at time t (just after streaming) is
//              f_i(x) = stored_i(x - v_i): every kernel that needs f(x)
//              gathers, the step kernel streams by gathering ("pull").
//   step     : one uint32 on the device, the time t of the next step, so
//              that captured graphs replay with advancing noise counters.
//   spec     : complex64 scratch for the correlator transforms, per lattice
//              5 fields x ny x kxp in row order (the half spectra of the real
//              fields after the row transforms; kxp is nkx = nx/2+1 rounded
//              up to 16).
//   stash    : kDeferK spectrum-sized slots: the column transforms' output,
//              each field plane column-tiled, stored by chunks of plane
//              positions across slots and fields (spec_offset and
//              stash_offset in flb_corr_internal.h).
//   acc      : FP64 correlator sums, per lattice FLB_NKINDS x ny x kxp, each
//              kind's plane column-tiled.
//   fields   : FP32 fluctuation fields of the sampled state, 5 x ny x nx
//              per lattice, and the FP64 conservation sums of that state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

namespace flbdev {

constexpr int kThreads = 256;
constexpr int kFields = 5;   // delta rho, delta jx, delta jy, delta ux, delta uy
constexpr int kKinds = 15;
constexpr int kMomentFields = 6;  // M^3 .. M^8, with the moment spectra
constexpr int kFieldRows = 16;  // rows per block of the field kernel

// Per-lattice constants, read by every kernel through scalar loads.
struct alignas(16) LatticeParams {
    int32_t nx, ny;
    int32_t nkx;              // nx/2 + 1
    int32_t tiles_x;          // step tiles along x
    int32_t px;               // storage row pitch: nx rounded up to 4
    int32_t pad1;
    int64_t base;             // element offset of population 0 in pops[]
    int64_t plane;            // px*ny
    int64_t spec_base;        // complex offset of field 0 in spec
    int64_t acc_base;         // double offset of kind 0 in acc
    float omega[6];           // 1/tau^a, a = 3..8
    float amp[6];             // noise amplitude per scaled moment, a = 3..8
    // the FP32 collision's folded coefficients: 9/4 omega[0], 9 omega[1],
    // -3 omega[3], -3 omega[4], 2 amp[3], 2 amp[4] (see collide)
    float fcoef[6];
    float rho0, u0x, u0y;
    float feq[9];             // f_i^0(rho0,u0) - w_i rho0 (16-bit reference state)
    float scale[9];           // sqrt(mu rho0 w_i) (16-bit storage scale)
    float inv_scale[9];
    float feq_scaled[9];      // feq * inv_scale
    float therm_amp[9];       // sqrt(mu rho0 w_i) for the thermal start
    // 16-bit steps collide the stored scaled deviations q directly
    // (d = s q + feq): class scales folded into the moment coefficients,
    // the reference state's moments as offsets, w_i / s_i for the back
    // transform (see collide_q)
    float qcoef[11];
    float qoff[9];
    float qback[3];
    uint32_t stream_id;
    int32_t line_x;           // index of the x-direction line plan
    int32_t line_y;           // index of the y-direction line plan
    int32_t kxp;              // columns of the spectrum and sum planes: nkx rounded up to 16
    int32_t col_large;        // columns in the column kernel's large blocks
    int32_t col_lgcb;         // log2 of the columns per column-kernel block
    int32_t fld_tiles_x;      // field-kernel tiles (256 sites) per row band
    int64_t fld_base;         // float offset of this lattice's five field planes
    int32_t fld_part0;        // first conservation partial of this lattice
    int32_t fld_nparts;       // number of them
};

// How to transform one line of length n in LDS.  Powers of two are done
// directly; other lengths by Bluestein's chirp-z convolution of length m.
struct alignas(16) LinePlan {
    int32_t n;                // transform length
    int32_t m;                // power-of-two work length (n itself, or >= 2n-1)
    int32_t bluestein;        // 0 or 1
    int32_t log2m;
    int64_t chirp_off;        // float2 offset of exp(-i pi j^2 / n), j < n
    int64_t kernel_off;       // float2 offset of the length-m FFT of the chirp kernel
};

// Twiddle table: exp(-2 pi i k / kTwN), k < kTwN/2, for every power-of-two
// work length up to kTwN.
constexpr int kTwLog = 13;
constexpr int kTwN = 1 << kTwLog;

// Work item of the step kernel: lattice and tile index (lattice -1 = idle).
struct StepItem {
    int32_t lattice;
    int32_t tile;
};

// Work item of the row transform: lattice and row; of the column transform:
// lattice, field and first column; of the accumulation: lattice and first k.
struct CorrItem {
    int32_t lattice;
    int32_t a;
    int32_t b;
    int32_t c;
};

enum Storage : int { kF32 = 0, kBF16 = 1, kF16 = 2 };

// ---------------------------------------------------------------------
// Kernel launchers (implemented in the .hip files).
// ---------------------------------------------------------------------
struct DeviceView {
    void *pops[2];
    int cur;                          // index of the buffer holding the state
    const LatticeParams *params;      // device
    const uint32_t *step;             // device step counter
    uint32_t *step_rw;
    float2 *spec;
    float2 *stash;                    // spectra awaiting accumulation (stash_offset)
    double *acc;
    float *fields;                    // [6][ny][nx] FP32 moment planes per lattice
    double *csum_part;                // field-kernel partial sums
    double *csum;                     // [nlat][5] sums of the last sample
    const LinePlan *plans;            // device
    const float2 *tables;             // device: twiddles, chirps, kernels
    uint64_t seed;
    int storage;
    int nlat;
};

hipError_t launch_step(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                       int sites, uint32_t step_add, bool nontemporal, bool noise,
                       hipStream_t s);
bool step_tile_supported(int tw, int r);
// Two steps per launch: tiles of tile_w x (1024 / tile_w) sites, tile_w 32,
// 64 or 128; items enumerate each lattice's tiles of that shape.  tile_w 0:
// each lattice has its own shape, 32 x 32 or 64 x 16, and the tile index of
// an item of a 32 x 32 lattice carries kStep2Square.
constexpr int32_t kStep2Square = 1 << 30;
hipError_t launch_step2(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                        uint32_t step_add, bool nontemporal, bool noise, hipStream_t s);
bool step2_tile_supported(int tw);
// Three steps per launch on the two-step kernel's tiles (tile_w 32, 64 or
// 128, the same items).
hipError_t launch_step3(const DeviceView &v, const StepItem *items, int nitems, int tile_w,
                        uint32_t step_add, bool nontemporal, bool noise, hipStream_t s);
hipError_t launch_advance_step(uint32_t *step, uint32_t n, hipStream_t s);
hipError_t launch_init(const DeviceView &v, int lattice, int64_t plane, hipStream_t s);
hipError_t launch_get(const DeviceView &v, int lattice, int nx, int ny, double *out_dev,
                      hipStream_t s);
hipError_t launch_set(const DeviceView &v, int lattice, int nx, int ny, const double *in_dev,
                      hipStream_t s);
hipError_t launch_conservation(const DeviceView &v, int lattice, int nx, int ny, double *part,
                               int nblocks, double *out_dev, hipStream_t s);
hipError_t launch_thermalize(const DeviceView &v, int lattice, int nx, int ny, double *part,
                             int nblocks, double *mean_dev, hipStream_t s);
hipError_t launch_debug_noise(uint64_t seed, uint32_t stream_id, uint32_t t, int64_t site0,
                              int64_t n, uint32_t *words_dev, float *z_dev, hipStream_t s);
hipError_t launch_fill(double *p, size_t n, hipStream_t s);

// ---------------------------------------------------------------------
// Host helpers shared by the runtimes.
// ---------------------------------------------------------------------
// Records the message returned by flb_last_error(); returns code.
int set_error(int code, const std::string &msg);

// Line plans and their tables: the twiddle table first, then the chirp and
// the transformed chirp kernel of every Bluestein length.
struct LineTables {
    std::vector<LinePlan> plans;
    std::vector<float2> tables;
    std::map<int, int> plan_of;
    LineTables();
    int plan_for(int n);  // index of the plan of length n (built on first use)
};
// Lengths the LDS line transforms support: powers of two up to 4096, other
// lengths up to 2048.
bool line_length_ok(int n);

}  // namespace flbdev
