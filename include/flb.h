/*
 * flb.h -- C interface of the MI355X (gfx950) fluctuating ideal-gas lattice
 * Boltzmann library.
 *
 * The method is the D2Q9 scheme with noise on every non-conserved moment
 * analysed by Kaehler & Wagner, "Cross Correlators and Galilean Invariance in
 * Fluctuating Ideal Gas Lattice Boltzmann Simulations":
 *   - one time step is Eq. (1) written in moment space, Eq. (5): moments
 *     M^a = sum_i m_i^a f_i (Eq. 3, matrix Eq. 9), relaxation of every
 *     non-conserved moment by its own 1/tau^a towards the equilibrium
 *     moments of Eq. (10), Gaussian noise of amplitude Eq. (8) on the stress
 *     and ghost moments a = 3..8 (Sec. 2, last paragraph), back transform
 *     with n_i^a = w_i m_i^a (Eq. 4), then streaming on a periodic lattice;
 *   - the measurement accumulates the static structure factors of Eq. (11)
 *     and the cross correlators of Eq. (12) from spatial Fourier transforms
 *     of the density, momentum and velocity fluctuations (Sec. 3).
 *
 * Conventions used by every call:
 *   - Lattice sites x = 0..nx-1, y = 0..ny-1, periodic; site index
 *     s = y*nx + x.  Velocities in the order of Sec. 3:
 *     (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *   - Moments a = 0..8: 0 density, 1-2 momentum (x sqrt 3), 3-4 shear
 *     stress, 5 bulk stress, 6-8 ghost modes.  tau[a] for a = 0..2 is ignored
 *     (those moments are conserved).
 *   - theta is a noise temperature: the moment variance of Eq. (7) becomes
 *     mu*rho0 with mu = theta / c_s^2 = 3 theta; theta = 1/3 reproduces the
 *     paper's unit-mass noise exactly, theta = 0 switches noise off.  The
 *     noise uses the constant rho0 (the u << 1 form of Eq. 7, as in the paper).
 *   - Noise: Philox4x32-10 (Salmon et al., SC'11), key = (seed & 0xffffffff,
 *     seed >> 32), counter = (site, t, stream_id, 0) for the collision of step
 *     t -> t+1 at that site.  The four words give six unit normals: radius
 *     uniforms r_p = (2(w_p >> 9) + 1) 2^-24 and angle uniforms
 *     a_p = (2 alpha_p + 1) 2^-20, alpha_p = ((w_p & 0x1ff) << 10) |
 *     ((w_3 >> 10p) & 0x3ff), p = 0,1,2; z_2p = sqrt(-2 ln r_p) cos(2 pi a_p),
 *     z_2p+1 = sqrt(-2 ln r_p) sin(2 pi a_p); z_{a-3} drives moment a.
 *   - Populations exchanged with the caller are full values f_i (not
 *     deviations), FP64, laid out [9][ny][nx], and are the state just after
 *     streaming (before the next collision) at the current time.
 *
 * Ownership: a handle owns all of its device memory.  Every pointer argument
 * that is read or written by a call belongs to the caller and is a HOST
 * pointer unless its name ends in _dev.  Calls that return data to the host
 * synchronise the handle's stream; flb_step, flb_run and
 * flb_accumulate_correlators only enqueue work.
 *
 * Sample overlap (flb_set_sample_overlap): a sample registered by
 * flb_accumulate_correlators (or by flb_run at the end of a period) is
 * enqueued with the next steps, on an internal second stream beside them;
 * the step that would overwrite the sampled state waits until the sample has
 * read it, and the work stream waits for the sample's end before the step
 * call's work is complete.  Results are identical to enqueueing the sample
 * at once.  flb_synchronize, flb_read_correlators, flb_sample_conservation,
 * flb_set_populations, flb_thermalize and flb_autotune enqueue a sample
 * still waiting on the work stream first; flb_reset_correlators drops it with
 * the sums.  Without overlap every sample is enqueued at once.
 *
 * Errors: calls return FLB_OK (0) or a negative FLB_E* code and leave a
 * message for flb_last_error() (per thread).  Creation calls return NULL on
 * error.  A handle is not safe to use from two threads at once.
 */
#ifndef FLB_H
#define FLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLB_OK 0
#define FLB_EINVAL (-1) /* invalid argument (value, range, NULL pointer) */
#define FLB_ENOMEM (-2) /* device or host allocation failed */
#define FLB_EHIP (-3)   /* a HIP runtime call failed */
#define FLB_ESIZE (-4)  /* a buffer size or lattice size outside what is supported */
#define FLB_ESTATE (-5) /* the call does not apply to this handle's state */

/* Storage of the populations in device memory. */
#define FLB_STORAGE_F32 0  /* FP32 deviation f_i - w_i rho0 */
#define FLB_STORAGE_BF16 1 /* bfloat16 of (f_i - f_i^0(rho0,u0)) / sqrt(mu rho0 w_i) */
#define FLB_STORAGE_F16 2  /* binary16 of the same scaled deviation */

/* Creation flags. */
#define FLB_FLAG_NO_GHOST_NOISE 1u /* zero noise on moments 6..8: the older
                                      scheme Sec. 3 compares against */
#define FLB_FLAG_MOMENT_SPECTRA 2u /* also accumulate the structure factors of
                                      the six non-conserved moments (Eq. 11
                                      for every moment of Eq. 9; Sec. 3 checks
                                      all nine): kinds 15..20 */

/* Correlator kinds, first index of the accumulator array. */
#define FLB_NKINDS 15
/*  0 |rho_k|^2   1 |jx_k|^2   2 |jy_k|^2   3 |ux_k|^2   4 |uy_k|^2
 *  5,6  Re,Im ux_k uy_k*     7,8  Re,Im rho_k jx_k*    9,10 Re,Im rho_k jy_k*
 *  11,12 Re,Im rho_k ux_k*   13,14 Re,Im rho_k uy_k*
 * where X_k = sum_x (X(x) - <X>) exp(-i k.x), k = 2 pi (kx/nx, ky/ny)
 * (Sec. 3, text after Eq. 11), u = j / rho at each site.
 * With FLB_FLAG_MOMENT_SPECTRA, six more kinds follow:
 *  15 + (a - 3)  |M^a_k|^2, a = 3..8, M^a = sum_i m_i^a f_i (Eq. 3, Eq. 9)
 * (the conserved moments M^0..M^2 are rho and sqrt(3) j, kinds 0..2). */
#define FLB_NKINDS_MOMENTS 21

/* Largest side for which correlators are supported: powers of two up to
 * FLB_MAX_FFT_SIDE, other lengths up to FLB_MAX_FFT_SIDE / 2. */
#define FLB_MAX_FFT_SIDE 4096

typedef struct flb flb_t;

/* One lattice of a batch. */
typedef struct flb_lattice_spec {
    int32_t nx, ny;    /* sides, >= 2 */
    double tau[9];     /* relaxation times per moment; tau[3..8] > 1/2 */
    double theta;      /* noise temperature, >= 0 */
    double rho0;       /* mean density, > 0 */
    double u0[2];      /* imposed mean velocity, |u0| < 1/sqrt(3) */
    uint32_t stream_id; /* third Philox counter word of this lattice */
    uint32_t reserved;  /* must be 0 */
} flb_lattice_spec;

/* Creates one lattice in the uniform equilibrium f_i^0(rho0, u0) of Eq. (2)
 * (c = 1), time t = 0, FP32 storage, stream_id 0, noise on all of 3..8.
 * tau: 9 doubles (host).  u0: 2 doubles (host).  Returns NULL on invalid
 * input (nx or ny < 2, non-finite values, rho0 <= 0, theta < 0,
 * tau[a] <= 1/2 for a >= 3, |u0| >= c_s), for a lattice whose populations
 * exceed 4 GiB (9 x nx x ny x 4 bytes, about 119M sites), or on allocation
 * failure. */
flb_t *flb_create(int nx, int ny, const double tau[9], double theta, double rho0,
                  const double u0[2], uint64_t seed);

/* As flb_create, with a storage format (FLB_STORAGE_*), the Philox stream id
 * of the lattice and creation flags (FLB_FLAG_*). */
flb_t *flb_create_ex(int nx, int ny, const double tau[9], double theta, double rho0,
                     const double u0[2], uint64_t seed, int storage, uint32_t stream_id,
                     uint32_t flags);

/* Creates n >= 1 independent lattices (any mix of sizes and parameters) that
 * step together: one launch advances all of them.  specs: n entries (host).
 * All share the seed, storage and flags; each has its own stream_id, which
 * should differ between lattices for independent noise. */
flb_t *flb_create_batch(int n, const flb_lattice_spec *specs, uint64_t seed, int storage,
                        uint32_t flags);

/* Frees the handle and its device memory (after draining its stream).
 * NULL is accepted. */
void flb_destroy(flb_t *h);

/* Message of the last failed call on this thread ("" if none). */
const char *flb_last_error(void);

/* Makes the handle enqueue all later work on the HIP stream `hip_stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * handle's own stream).  The caller keeps ownership of the stream and must
 * keep it alive while the handle uses it. */
int flb_set_stream(flb_t *h, void *hip_stream);

/* Enqueues a sample still waiting for the next steps, then blocks until all
 * work enqueued by the handle has finished. */
int flb_synchronize(flb_t *h);

/* Sample overlap on (1, the default) or off (0), see above.  A sample
 * waiting for steps is enqueued first.  flb_get_sample_overlap returns the
 * setting (or a negative FLB_E* code). */
int flb_set_sample_overlap(flb_t *h, int on);
int flb_get_sample_overlap(flb_t *h);

/* Launch timing: while on, every step-kernel launch that flb_step or
 * flb_run enqueues outside a captured graph is bracketed by a pair of HIP
 * events on the work stream, recorded after any wait on the sample, so the
 * pair measures that kernel's execution.  flb_get_launch_timing
 * synchronises the work stream and writes the number of timed launches and
 * the sum of their durations (ms) since the previous call, then starts a new
 * count.  Graph-replayed periods and flb_autotune's candidates are not
 * timed; each timed launch keeps its event pair until it is read.
 * flb_get_launch_timing_kinds reads the same records split by the steps a
 * launch took: launches[q] and total_ms[q] (caller arrays of three) for the
 * launches of q + 1 steps. */
int flb_set_launch_timing(flb_t *h, int on);
int flb_get_launch_timing(flb_t *h, int64_t *launches, double *total_ms);
int flb_get_launch_timing_kinds(flb_t *h, int64_t launches[3], double total_ms[3]);

/* Advances every lattice of the handle by nsteps >= 0 steps of Eq. (5) with
 * streaming (Eq. 1).  Enqueues only. */
int flb_step(flb_t *h, int64_t nsteps);

/* Advances by nsteps and, after every step that reaches a time t with
 * t % sample_every == 0, adds a correlator sample (sample_every = 0: no
 * samples).  Whole periods of sample_every steps plus their sample are
 * replayed from a captured HIP graph (with sample overlap, each with the
 * previous period's sample beside its steps).  Enqueues only; with sample
 * overlap the last sample waits for the next steps or flb_synchronize. */
int flb_run(flb_t *h, int64_t nsteps, int sample_every);

/* Adds one sample of the current state of every lattice to its FP64
 * correlator sums (Eqs. 11-12, the kinds listed above), on the half plane
 * kx = 0..nx/2, ky = 0..ny-1; the k = 0 entry is left unchanged (the mean is
 * removed, Sec. 3).  FLB_ESIZE for sides beyond FLB_MAX_FFT_SIDE (powers
 * of two) or FLB_MAX_FFT_SIDE / 2 (other lengths).
 * Registers the sample (counted at once); with sample overlap (above) its
 * kernels are enqueued with the next steps, or by the next call that needs
 * them, otherwise at once. */
int flb_accumulate_correlators(flb_t *h);

/* Copies lattice `lattice`'s raw FP64 sums to out[kind][ky][kx] (host), with
 * kind < flb_num_kinds(h), ky < ny, kx < nx/2+1, and writes the number of
 * samples taken to *nsamples (may be NULL).  n_doubles must be at least
 * flb_num_kinds(h)*ny*(nx/2+1), else FLB_ESIZE.  Synchronises, and takes
 * host memory for one more copy of the lattice's sums (the device keeps them
 * in another order).  The library adds the FP64 products of 32 samples in
 * one pass over the sums and keeps the FP32 spectra of up to 32 samples
 * until then (32 spectrum-sized buffers of 5 x ny x (nx/2+16) complex
 * values per lattice); a read adds those first, so the sums are those of
 * adding every sample, up to FP64 rounding order. */
int flb_read_correlators(flb_t *h, int lattice, double *out, size_t n_doubles,
                         int64_t *nsamples);

/* Normalised correlators of lattice `lattice` in the layout of
 * flb_read_correlators (out[kind][ky][kx], host, n_doubles as there): the
 * sums divided by the number of samples and by each kind's normalisation
 * (Sec. 3, Eqs. 11-12), with mu = 3 theta and c_s = 1/sqrt(3):
 *   kind 0       S(rho)     = <|rho_k|^2> / (V mu rho0)
 *   kinds 1, 2   S(j_a)     = <|j_a,k|^2> / (V rho0 theta)
 *   kinds 3, 4   S(u_a)     = rho0 <|u_a,k|^2> / (V theta)
 *   kinds 5, 6   R(u_x,u_y) = rho0 <u_x,k u_y,k*> / (V theta)      (Re, Im)
 *   kinds 7..10  R(rho,j_a) = <rho_k j_a,k*> / (V mu rho0 c_s)     (Re, Im)
 *   kinds 11..14 R(rho,u_a) = <rho_k u_a,k*> / (V mu c_s)          (Re, Im)
 *   kinds 15..20 S(M^a)     = <|M^a_k|^2> / (V mu rho0), a = 3..8
 * V = nx ny.  The paper's N^rho = 1/(rho^3 V) and N^{u_a} = 1/(rho V k_B T)
 * are these at rho0 = 1, theta = k_B T = 1/3, where the equal-time moment
 * variance is rho0 (Eq. 7): at u0 = 0 every S is 1 and every R is 0 at
 * linear order.  Writes the sample count to *nsamples (may be NULL).
 * FLB_ESTATE when no sample was taken since the last reset, or when the
 * lattice's theta is 0 (no fluctuation scale to normalise by).
 * Synchronises. */
int flb_read_normalized(flb_t *h, int lattice, double *out, size_t n_doubles,
                        int64_t *nsamples);

/* Enqueues, without waiting, the work still owed to the FP64 sums: a
 * sample waiting for the next steps, then the products of the stashed
 * samples (see flb_read_correlators).  Once the handle's stream has run
 * this far, the sums hold every sample taken, as a read would find them.
 * For callers that synchronise the stream themselves and for timing a
 * whole number of samples. */
int flb_flush_correlators(flb_t *h);

/* Zeroes every lattice's correlator sums and the sample count. */
int flb_reset_correlators(flb_t *h);

/* Copies lattice `lattice`'s populations f_i(x, t) to out[9][ny][nx] (host,
 * FP64).  n must be at least 9*nx*ny.  Synchronises. */
int flb_get_populations(flb_t *h, int lattice, double *out, size_t n);

/* For callers that cannot allocate device memory (loops that read the
 * state often and may not call hipMalloc, harnesses that forbid device
 * allocation): flb_get_populations without its per-call staging
 * allocation.  Same arguments, output and errors, plus FLB_ESIZE when
 * 9*nx*ny exceeds 8388608 values (2^23).  The values pass through a 64 MiB
 * staging array in the library's code object, one per GPU, held until the
 * process ends; the call allocates nothing.  Calls on one GPU share that
 * array: calls from several host threads that overlap on one GPU race (each
 * call synchronises the handle's stream before it returns, so calls from
 * one thread never overlap).  Synchronises. */
int flb_get_populations_noalloc(flb_t *h, int lattice, double *out, size_t n);

/* Replaces lattice `lattice`'s populations by in[9][ny][nx] (host, FP64 full
 * values).  Values are rounded to the storage format.  Synchronises. */
int flb_set_populations(flb_t *h, int lattice, const double *in, size_t n);

/* FP64 sums over lattice `lattice`: out[0] = sum (rho - rho0),
 * out[1..2] = sum j, out[3] = sum (-1)^x j_x, out[4] = sum (-1)^y j_y.
 * The first three are conserved by Eq. (5); for even sides the staggered
 * sums change sign every step.  Any non-finite population makes the sums
 * non-finite.  Synchronises. */
int flb_conservation(flb_t *h, int lattice, double out[5]);

/* The same five sums, for the state of the most recent correlator sample:
 * every sample's row transforms leave FP64 partial sums of its fluctuation
 * fields (FP32 per site) at no extra pass over the populations, and this
 * call adds them up.  FLB_ESTATE if no sample was taken since creation or
 * the last reset.  Synchronises. */
int flb_sample_conservation(flb_t *h, int lattice, double out[5]);

/* As flb_conservation, but enqueue-only: the five sums are written to
 * out_dev, 5 doubles of DEVICE memory (e.g. a torch tensor's data_ptr())
 * owned by the caller. */
int flb_conservation_dev(flb_t *h, int lattice, double *out_dev);

/* Equilibrium-fluctuation start: adds sqrt(mu rho0 w_i) z_i(x) to every
 * population, z_0..z_8 being the first nine normals of the counters
 * (site, 0xffffffff, stream_id, d), d = 0, 1, then removes each
 * population's spatial mean of what was added, so totals are unchanged. */
int flb_thermalize(flb_t *h);

/* Noise of lattice `lattice` at step t for sites site0 .. site0+nsites-1:
 * words_out[4*nsites] (may be NULL) gets the Philox words, z_out[6*nsites]
 * (may be NULL) the six normals as computed by the step kernel.
 * Synchronises.  For testing. */
int flb_debug_noise(flb_t *h, int lattice, uint32_t t, int64_t site0, int64_t nsites,
                    uint32_t *words_out, float *z_out);

/* Number of correlator kinds the handle accumulates: FLB_NKINDS, or
 * FLB_NKINDS_MOMENTS with FLB_FLAG_MOMENT_SPECTRA; negative on a NULL
 * handle. */
int flb_num_kinds(flb_t *h);

/* Number of steps taken so far (the t of the next step). */
int64_t flb_get_step(flb_t *h);

/* Sets the time of the next step (0 <= t < 2^32 - 1).  With
 * flb_set_populations this resumes a run from a saved state: the noise is a
 * function of (seed, site, t, stream_id) only, so the continuation is the
 * same as an uninterrupted run (bit-identical for FP32 storage).
 * Synchronises. */
int flb_set_step(flb_t *h, int64_t t);

/* Number of lattices in the handle (-1 on error). */
int flb_num_lattices(flb_t *h);

/* Sides of lattice `lattice` and the kx extent nx/2+1 of its correlators. */
int flb_lattice_info(flb_t *h, int lattice, int32_t *nx, int32_t *ny, int32_t *nkx);

/* Storage format and bytes per population value. */
int flb_storage_info(flb_t *h, int32_t *storage, int32_t *bytes_per_value);

/* Launch shape of the step kernel: blocks of tile_w threads along x (64,
 * 128 or 256) by 256/tile_w rows, each thread updating `sites` consecutive
 * sites of its row (1, 2 or 4) with one vector access per population, and
 * the streaming (non-temporal) hint on or off for those accesses (all
 * stores, and the loads of each thread's own sites).  Results do not depend
 * on it.
 * FLB_EINVAL for an unsupported shape. */
int flb_set_step_config(flb_t *h, int tile_w, int sites, int nontemporal);
int flb_get_step_config(flb_t *h, int *tile_w, int *sites, int *nontemporal);

/* Time blocking: steps_per_launch = 2 runs pairs of steps in one kernel
 * launch (tiles of tile_w x 1024/tile_w sites, tile_w 32, 64 or 128; each
 * block collides its tile and a one-site halo at t, keeps them on chip and
 * collides the tile again at t+1), so the populations cross HBM once per two
 * steps; an odd last step uses the one-step kernel.  steps_per_launch = 3
 * runs three steps per launch on the same tiles with a two-site halo (the
 * halo at t, the tile and the inner ring at t+1, the tile at t+2); a
 * remainder of two steps takes the two-step kernel, and of one step the
 * one-step kernel if fewer than four steps are enqueued, else the last
 * three-step launch and it become two two-step launches.  Every site sees the same arithmetic, noise counters and storage
 * rounding as with one step per launch: results do not depend on it.
 * steps_per_launch = 1 (default) turns it off.  FLB_EINVAL for other values.
 * flb_get_time_blocking reports tile_w = 0 while each lattice has its own
 * tile (flb_set_lattice_tiles). */
int flb_set_time_blocking(flb_t *h, int steps_per_launch, int tile_w);
int flb_get_time_blocking(flb_t *h, int *steps_per_launch, int *tile_w);

/* Time blocking with a tile shape per lattice: tile_w[l] (32 or 64, one
 * entry per lattice of the handle, host memory, read during the call) gives
 * lattice l tiles of tile_w[l] x 1024/tile_w[l] sites; all lattices still
 * step in one launch.  Sets steps_per_launch = 2.  Results do not depend on
 * it.  FLB_EINVAL for a NULL array or another width.
 * flb_get_lattice_tiles writes each lattice's two-step tile width in
 * effect (the handle's one width, or its own) to tile_w[0 .. lattices-1]. */
int flb_set_lattice_tiles(flb_t *h, const int *tile_w);
int flb_get_lattice_tiles(flb_t *h, int *tile_w);

/* Chooses the step kernel's launch shape by timing every supported shape
 * (nsteps >= 1 steps each, HIP events on the handle's stream, in three
 * round-robin passes of which each shape keeps its fastest) on this
 * handle's own lattices, the time-blocked shapes included (per step), and
 * keeps the fastest.  For a batch whose fastest shape is time-blocked, the
 * two-step tile is then chosen per size class (the lattices whose sides
 * round up to the same powers of two): each class takes the faster of
 * 32 x 32 and 64 x 16 tiles, timed on its own lattices' tiles (the one with
 * fewer halo collisions where they are within 1 %), and these per-class tiles
 * (flb_set_lattice_tiles) replace the fastest shape if the whole batch then
 * steps faster.  The populations and the
 * step counter are restored afterwards, so results are unchanged.  When the
 * environment variable FLB_AUTOTUNE_CACHE names a file, choices are read
 * from and appended to it, keyed by storage format, lattice count, total
 * sites, largest side and noise.  Synchronises. *ms_out (may be NULL)
 * receives the chosen shape's time per step. */
int flb_autotune(flb_t *h, int nsteps, double *ms_out);

/* As flb_autotune, then for the shapes within 4 % of the fastest alone (at
 * most four), and for a batch the tile per size class as above, the whole
 * path decides: each is timed on whole periods of
 * sample_every >= 1 steps and a correlator sample (Eqs. 11-12), issued as
 * flb_step and flb_accumulate_correlators issue them (with sample overlap,
 * each sample runs beside the following steps, which a shape's time alone
 * does not show), over a full accumulation cycle in two round-robin passes,
 * and the fastest period is kept.  Only before the first sample (or after
 * flb_reset_correlators): FLB_ESTATE otherwise.  Populations, step counter
 * and correlator sums are as before the call.  Cached as flb_autotune under
 * a key that includes sample_every.  *ms_out receives the chosen shape's
 * whole-path time per step. */
int flb_autotune_path(flb_t *h, int nsteps, int sample_every, double *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* FLB_H */
