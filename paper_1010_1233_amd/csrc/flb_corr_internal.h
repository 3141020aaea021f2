// flb_corr_internal.h -- the correlator kernels' layouts and launchers,
// shared by the host runtime and flb_corr.hip (apart from flb_internal.h, so
// that the step kernels' sources do not change with them).
#pragma once

#include "flb_internal.h"

namespace flbdev {

// The column transforms' output planes and the sums (ny rows of kxp
// columns) are column-tiled: tiles of kTileCols adjacent columns, each tile
// holding all ny rows contiguously, so that the output of a group of
// kTileCols columns (what the column transforms take at 4096 points) is one
// contiguous run of memory, as is every stretch of k the accumulation
// takes.  (The row transforms' output stays in row order: their blocks hold
// one row, and a tiled store from them would write 32-byte pieces.)  Column
// kx of row y of a plane is at spec_offset.
constexpr int kTileCols = 4;
__host__ __device__ inline int64_t spec_offset(int y, int kx, int ny)
{
    return ((int64_t)(kx / kTileCols) * ny + y) * kTileCols + kx % kTileCols;
}

// Field set 0 (rho, j, u; kKinds kinds): fused fields + row transforms
// (items of power-of-two rows and of Bluestein rows), each block leaving
// its partial conservation sums of the sampled state.  Rows of 2^lg points, 9 <= lg <= 12
// (corr_rows_p2_supported), and Bluestein rows of work length 2^lg,
// 8 <= lg <= 11 (corr_rows_blue_supported), take blocks specialised per
// length: launch q of `fixed` takes items[fixed[q].off .. + fixed[q].n),
// the power-of-two rows of length 2^lg (lg = fixed[q].lg) or, for lg = 0,
// the Bluestein rows of every supported work length.  The generic kernels
// take the other power-of-two rows, items[0 .. nitems), and the other
// Bluestein rows, blue_items.  Every block of these kernels holds 4096
// complex values of LDS (lds_bytes for the padded slots).
struct RowLaunch {
    int lg, off, n;
};
bool corr_rows_p2_supported(int lg);
bool corr_rows_blue_supported(int lg);
hipError_t launch_corr_rows(const DeviceView &v, const CorrItem *items, int nitems,
                            const RowLaunch *fixed, int nfixed, const CorrItem *blue_items,
                            int nblue, int lds_bytes, hipStream_t s);
// The five conservation sums of the last sample per lattice, from the row
// blocks' partials in a fixed order (taken when they are read: the partials
// stay until the next sample's row transforms).
hipError_t launch_corr_csum(const DeviceView &v, hipStream_t s);
// Field set 1 (the six non-conserved moments, kinds kKinds .. kKinds + 5):
// FP32 field planes, then row transforms.
hipError_t launch_corr_moment_fields(const DeviceView &v, const CorrItem *items, int nitems,
                                     hipStream_t s);
hipError_t launch_corr_moment_rows(const DeviceView &v, const CorrItem *items, int nitems,
                                   int lds_bytes, hipStream_t s);
// Column transforms and accumulation; set selects the fields and kinds as
// above.  The column transform writes back in place, or to stash slot
// `slot` >= 0; `large` picks the large blocks (kColsLargeElems elements,
// kColsLargeThreads threads) over the kColsElems-element ones.  The
// accumulation adds this sample's products and, for nslots > 0 (field set
// 0), those of the first nslots stash slots.
constexpr int kColsElems = 8192;
constexpr int kColsLargeElems = 16384;
constexpr int kColsLargeThreads = 1024;
hipError_t launch_corr_cols(const DeviceView &v, const CorrItem *items, int nitems, int slot,
                            bool large, int lds_bytes, hipStream_t s);
// Column transforms of Bluestein work length 2^lg, 8 <= lg <= 11
// (corr_cols_blue_supported), field set 0, in blocks specialised per work
// length, all in one launch: items {lattice, field, first column, unused},
// 8192 / 2^lg columns per item.  `slot` as for launch_corr_cols.
bool corr_cols_blue_supported(int lg);
hipError_t launch_corr_cols_blue(const DeviceView &v, const CorrItem *items, int nitems, int slot,
                                 hipStream_t s);
// Column transforms of power-of-two lengths 2^lg, 9 <= lg <= 12, in
// persistent blocks: sched holds niter x grid groups of columns (the group
// of block b in round it at it * grid + b), each of 16384 / 2^lg (at most
// 16) adjacent columns of one field, starting at a tile: the complex offset
// of its first column in the spectra (row order, row pitch kxp), the offset
// of its first tile in a stash slot (tile stride ts = kTileCols * ny), and
// the number of columns it has (0: no group).  `slot` as for
// launch_corr_cols.
struct PipeItem {
    int64_t off;     // first column in the spectra (row order)
    int64_t sbase;   // the lattice's spec_base, for stash_offset
    int32_t kxp;     // row pitch of the spectra
    int32_t ts;      // column-tile stride of a stash plane, kTileCols * ny
    int32_t ncol;    // columns in the group (0: no group)
    int32_t o0;      // plane position of the group's first column in a stash plane
    int32_t f;       // field
    int32_t plane;   // positions per stash plane, ny * kxp
};
bool corr_cols_pipe_supported(int lg);
int corr_cols_pipe_lds_bytes(int lg);
hipError_t launch_corr_cols_pipe(const DeviceView &v, const PipeItem *sched, int niter, int grid,
                                 int lg, int slot, hipStream_t s);
// samples per read-modify-write of the FP64 sums (kDeferK stash slots, each
// the size of the spectra: 10.8 GB at 4096^2).  The sums' read-modify-write
// is most of the accumulation's bytes: 4096^2 whole path 87.5 GLUPS with 16
// against 86.4 with 8; a sample alone 0.504 ms with 32 against 0.520 with 16.
constexpr int kDeferK = 32;

// Stash layout: per lattice, kDeferK x 5 planes of ny * kxp values (each
// column-tiled as spec_offset has it) in a region of kDeferK times the
// lattice's spectra, by chunks of kStashChunk consecutive plane positions:
// chunk c holds its positions of plane (slot j, field f) for every j and f
// in turn, so that an accumulation block (one chunk) reads its kDeferK x 5
// planes as one contiguous run instead of 5 kDeferK streams.  The last
// chunk of a plane may be narrower.  Offset (complex values) of position o
// of plane (j, f) for the lattice whose spectra start at spec_base:
constexpr int kStashLog = 8, kStashChunk = 1 << kStashLog;
__host__ __device__ inline int64_t stash_offset(int64_t spec_base, int64_t plane, int64_t o,
                                                int j, int f)
{
    // (o, plane < 2^31)
    const uint32_t c = (uint32_t)o >> kStashLog, r = (uint32_t)o & (kStashChunk - 1);
    const uint32_t left = (uint32_t)plane - (c << kStashLog);
    const uint32_t w = left < (uint32_t)kStashChunk ? left : (uint32_t)kStashChunk;
    return kDeferK * spec_base + (int64_t)c * (kStashChunk * 5 * kDeferK) +
           (int64_t)((uint32_t)(j * 5 + f) * w + r);
}
// Adds the products of the first nslots stash slots to the sums (field set
// 0): every kDeferK-th sample with nslots = kDeferK, and before a read.
hipError_t launch_corr_flush(const DeviceView &v, const CorrItem *items, int nitems, int nslots,
                             hipStream_t s);
// Adds this sample's products to the sums at once (the column transforms'
// output left in place, in row order).
hipError_t launch_corr_accum(const DeviceView &v, const CorrItem *items, int nitems, int set,
                             hipStream_t s);
}  // namespace flbdev
