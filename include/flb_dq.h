/*
 * flb_dq.h -- C ABI of the fluctuating lattice Boltzmann method on other
 * velocity sets (libflb.so).
 *
 * Kaehler & Wagner report that the noise on every non-conserved moment gives
 * the same results on D1Q3 and D3Q15 as on D2Q9 (Sec. 3).  This interface
 * runs one periodic lattice of such a model on the GPU: the step of Eqs. (1),
 * (3), (5), (8), (4) and the structure factors of Eq. (11) (and Eq. 12 for
 * u_x u_y*), in D dimensions.  D2Q9 is available through the same generic
 * code as a cross-check of the dedicated D2Q9 interface in flb.h.
 *
 * Models (velocity order, weights, moments):
 *   FLB_DQ_D1Q3   v = 0, +1, -1; w = 2/3, 1/6, 1/6
 *   FLB_DQ_D2Q9   the velocity order and weights of Sec. 3
 *   FLB_DQ_D3Q15  rest; +x, -x, +y, -y, +z, -z; the eight corners
 *                 (c = 0..7: v = ((c&1) ? -1 : 1, (c&2) ? -1 : 1, (c&4) ? -1 : 1));
 *                 w = 2/9, 1/9 (faces), 1/72 (corners)
 * The paper prints the moment matrix only for D2Q9 (Eq. 9); for every model
 * the moments m_i^a are the velocity polynomials
 *   D1Q3:  1, v_x, v_x^2 - 1/3
 *   D2Q9:  1, v_x, v_y, v_x^2 - v_y^2, v_x v_y, v^2 - 2/3, v_x v^2, v_y v^2, v^4
 *   D3Q15: 1, v_x, v_y, v_z, 3 v_x^2 - v^2, v_y^2 - v_z^2, v_x v_y, v_y v_z,
 *          v_z v_x, v^2 - 1, v_x v^2, v_y v^2, v_z v^2, v_x v_y v_z, v^4
 * orthonormalised in this order under the weights (Gram-Schmidt, so that
 * sum_i w_i m_i^a m_i^b = delta^{ab}, Eq. 4; for D2Q9 these are the rows of
 * Eq. 9).  Moments 0..D are conserved (rho, sqrt(3) j), the next D(D+1)/2 are
 * the stress modes, the rest are ghost modes.  Noise normal z_n (n = 0, 1, ...)
 * drives non-conserved moment D+1+n; normals 6d..6d+5 of a site come from the
 * Philox4x32-10 draw with counter (site, t, stream_id, d), site =
 * x + nx (y + ny z), and the bit-to-normal mapping documented in flb.h.
 *
 * Storage: FP32 deviations f_i - w_i rho0, [Q][nz][ny][nx], two buffers
 * (ping-pong); each buffer must stay below 4 GiB.  Errors and messages as in
 * flb.h (FLB_OK, FLB_EINVAL, ...; flb_last_error()).
 */
#ifndef FLB_DQ_H
#define FLB_DQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLB_DQ_D1Q3 13
#define FLB_DQ_D2Q9 29
#define FLB_DQ_D3Q15 315
#define FLB_DQ_MAXQ 15

typedef struct flb_dq flb_dq_t;

/* The model's tables (host only, no GPU needed): dimension D, Q, velocities
 * v[Q][3], weights w[Q] and moments m[a][i] (row-major Q x Q), in FP64.
 * Arrays must hold FLB_DQ_MAXQ (v: 3 FLB_DQ_MAXQ, m: FLB_DQ_MAXQ^2) entries.
 * FLB_EINVAL for an unknown model. */
int flb_dq_tables(int model, int32_t *D, int32_t *Q, int32_t *v, double *w, double *m);

/* Creates one lattice of `model` with sides n[0..2] (unused dimensions must
 * be 1; used ones >= 2), relaxation times tau[Q] (tau[a] > 1/2 for every
 * non-conserved a; the conserved ones are ignored), noise temperature theta
 * >= 0 (mu = 3 theta, Eq. 8 amplitudes sigma_a = sqrt(mu rho0 (2 tau^a - 1)) /
 * tau^a), rho0 > 0, mean velocity u0[3] (|u0| < 1/sqrt(3), unused components
 * 0), Philox key `seed`, counter word `stream_id`, flags FLB_FLAG_NO_GHOST_NOISE
 * (flb.h) for the older scheme.  The state starts at f^0(rho0, u0) (Eq. 2),
 * t = 0.  NULL on error (flb_last_error()). */
flb_dq_t *flb_dq_create(int model, const int32_t n[3], const double *tau, double theta,
                        double rho0, const double u0[3], uint64_t seed, uint32_t stream_id,
                        uint32_t flags);
void flb_dq_destroy(flb_dq_t *h);

/* D, Q and the number of correlator kinds (see flb_dq_read). */
int flb_dq_info(flb_dq_t *h, int32_t *D, int32_t *Q, int32_t *nkinds);

/* Work is enqueued on this HIP stream (NULL: the handle's own stream). */
int flb_dq_set_stream(flb_dq_t *h, void *hip_stream);
int flb_dq_synchronize(flb_dq_t *h);

/* nsteps steps (enqueued). */
int flb_dq_step(flb_dq_t *h, int64_t nsteps);
/* nsteps steps with a correlator sample at every t with t % sample_every == 0
 * (enqueued). */
int flb_dq_run(flb_dq_t *h, int64_t nsteps, int sample_every);
int64_t flb_dq_get_step(flb_dq_t *h);

/* Adds one sample of the current state to the FP64 sums (enqueued).  Kinds:
 *   |rho_k|^2, |j_a,k|^2 (a < D), |u_a,k|^2 (a < D),
 *   Re and Im of u_x,k u_y,k* (D >= 2),
 *   |M^a_k|^2 for every non-conserved moment a = D+1 .. Q-1,
 * with X_k = sum_x (X(x) - <X>) exp(-i k.x) (Sec. 3), on the half space
 * kx = 0..nx/2; k = 0 is left unchanged.  FLB_ESIZE for a side that is not a
 * power of two up to 4096 or another length up to 2048. */
int flb_dq_accumulate(flb_dq_t *h);
/* Copies the raw sums to out[kind][nz][ny][nx/2+1] (host, FP64); n_doubles
 * must be at least nkinds*nz*ny*(nx/2+1).  Synchronises. */
int flb_dq_read(flb_dq_t *h, double *out, size_t n_doubles, int64_t *nsamples);
/* The same sums divided by the sample count and by each kind's
 * normalisation (Eq. 11, Eq. 12 for u_x u_y*; mu = 3 theta, V the number of
 * sites): V mu rho0 for rho and every moment M^a, V rho0 theta for j_a,
 * V theta / rho0 for u_a and both u_x u_y* kinds, so that each is 1 (auto)
 * or 0 (cross) at u0 = 0 to linear order.  Same layout and sizes as
 * flb_dq_read.  FLB_ESTATE when no sample was taken or theta = 0.
 * Synchronises. */
int flb_dq_read_normalized(flb_dq_t *h, double *out, size_t n_doubles, int64_t *nsamples);
int flb_dq_reset(flb_dq_t *h);

/* Populations f_i(x, t) (just after streaming, before the next collision) as
 * out[Q][nz][ny][nx] (host, FP64); n at least Q*nx*ny*nz.  Synchronises. */
int flb_dq_get_populations(flb_dq_t *h, double *out, size_t n);
int flb_dq_set_populations(flb_dq_t *h, const double *in, size_t n);

/* Equilibrium-fluctuation start: adds sqrt(mu rho0 w_i) z_i(x) to every
 * population, z from the counters (site, 0xffffffff, stream_id, d), d = 0,
 * 1, 2 (normals 0..Q-1), and removes each population's spatial mean of the
 * addition.  Enqueued. */
int flb_dq_thermalize(flb_dq_t *h);

/* FP64 sums of mass and momentum (out[0], out[1..D]; unused entries 0).
 * Synchronises. */
int flb_dq_conservation(flb_dq_t *h, double out[4]);

#ifdef __cplusplus
}
#endif

#endif /* FLB_DQ_H */
