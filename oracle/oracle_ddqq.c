/*
 * oracle_ddqq.c -- plain, slow FP64 CPU oracle of the same fluctuating
 * lattice Boltzmann method on other velocity sets: D1Q3 and D3Q15, which the
 * paper reports testing besides D2Q9 (Sec. 3), and D2Q9 itself through the
 * same generic code as a cross-check of the generic path.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; it shares nothing
 * with the GPU library.
 *
 * The paper prints the moment matrix only for D2Q9 (Eq. 9).  For any
 * velocity set the moments here are built the way Eq. (4) demands: a fixed
 * list of velocity polynomials (1, v_a, the second-order shear and bulk
 * polynomials, then higher orders) orthonormalised under the weights by
 * Gram-Schmidt in FP64, so that sum_i w_i m_i^a m_i^b = delta^{ab}.  For D2Q9
 * this reproduces the rows of Eq. (9).  Moments 0..D are conserved (rho and
 * sqrt(3) j), the next D(D+1)/2 are the stress modes (second-order
 * polynomials, non-zero equilibrium), the rest are ghost modes.
 *
 * One step, per site, in the paper's order: moments (Eq. 3), equilibrium
 * moments as the moments of Eq. (2) (c = 1, in D dimensions), relaxation of
 * every non-conserved mode with its own 1/tau^a (Eq. 5), noise of amplitude
 * Eq. (8) on every non-conserved mode (on the non-ghost ones only with the
 * older scheme's switch), back transform with n_i^a = w_i m_i^a (Eq. 4),
 * streaming (Eq. 1).  Noise normal z_n drives non-conserved moment D+1+n;
 * normals 6d..6d+5 come from the Philox draw with counter
 * (site, t, stream_id, d), site = x + nx (y + ny z), mapped to normals as in
 * oracle.c.
 *
 * State layout: f[i][z][y][x], full populations, pre-collision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from oracle.c */
void oracle_noise_words(uint64_t seed, uint32_t stream_id, uint32_t t, uint32_t site, uint32_t d,
                        uint32_t out[4]);
void oracle_normals_from_words(const uint32_t w[4], double z[6]);
void oracle_dft3(double *re, double *im, int nx, int ny, int nz);

#define DQ_MAXQ 15

typedef struct {
    int D, Q;
    int v[DQ_MAXQ][3];
    double w[DQ_MAXQ];
    double m[DQ_MAXQ][DQ_MAXQ]; /* m[a][i] */
    int nstress;                /* D (D + 1) / 2 */
} dq_model;

enum { DQ_D1Q3 = 13, DQ_D2Q9 = 29, DQ_D3Q15 = 315 };

/* Velocity polynomial number a of the model's list at velocity v. */
static double dq_poly(int D, int a, const int v[3])
{
    const double x = v[0], y = v[1], z = v[2];
    const double v2 = x * x + y * y + z * z;
    if (a == 0) return 1.0;
    if (a <= D) return (double)v[a - 1];
    if (D == 1) {
        /* the single stress mode */
        return x * x - 1.0 / 3.0;
    }
    if (D == 2) {
        /* Eq. (9) order: shear xx - yy, shear xy, bulk, then ghosts */
        switch (a) {
        case 3: return x * x - y * y;
        case 4: return x * y;
        case 5: return v2 - 2.0 / 3.0;
        case 6: return x * v2;
        case 7: return y * v2;
        case 8: return v2 * v2;
        }
    }
    /* D == 3: shear (5), bulk, then ghosts */
    switch (a) {
    case 4: return 3.0 * x * x - v2;
    case 5: return y * y - z * z;
    case 6: return x * y;
    case 7: return y * z;
    case 8: return z * x;
    case 9: return v2 - 1.0;
    case 10: return x * v2;
    case 11: return y * v2;
    case 12: return z * v2;
    case 13: return x * y * z;
    case 14: return v2 * v2;
    }
    return 0.0;
}

/* Velocity sets and weights.  D2Q9 in the order of Sec. 3; D1Q3 and D3Q15
 * with the standard weights of the isothermal c_s^2 = 1/3 models. */
int oracle_dq_model(int id, dq_model *M)
{
    memset(M, 0, sizeof *M);
    if (id == DQ_D1Q3) {
        M->D = 1;
        M->Q = 3;
        const int vx[3] = {0, 1, -1};
        const double w[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
        for (int i = 0; i < 3; ++i) {
            M->v[i][0] = vx[i];
            M->w[i] = w[i];
        }
    } else if (id == DQ_D2Q9) {
        M->D = 2;
        M->Q = 9;
        const int vx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        const int vy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        for (int i = 0; i < 9; ++i) {
            M->v[i][0] = vx[i];
            M->v[i][1] = vy[i];
            M->w[i] = i == 0 ? 4.0 / 9.0 : i < 5 ? 1.0 / 9.0 : 1.0 / 36.0;
        }
    } else if (id == DQ_D3Q15) {
        M->D = 3;
        M->Q = 15;
        /* rest, the six faces (+x, -x, +y, -y, +z, -z), the eight corners */
        int i = 0;
        M->w[i++] = 2.0 / 9.0;
        for (int a = 0; a < 3; ++a)
            for (int s = 1; s >= -1; s -= 2) {
                M->v[i][a] = s;
                M->w[i++] = 1.0 / 9.0;
            }
        for (int c = 0; c < 8; ++c) {
            M->v[i][0] = (c & 1) ? -1 : 1;
            M->v[i][1] = (c & 2) ? -1 : 1;
            M->v[i][2] = (c & 4) ? -1 : 1;
            M->w[i++] = 1.0 / 72.0;
        }
    } else {
        return -1;
    }
    M->nstress = M->D * (M->D + 1) / 2;
    /* weighted Gram-Schmidt over the polynomial list */
    for (int a = 0; a < M->Q; ++a) {
        double h[DQ_MAXQ];
        for (int i = 0; i < M->Q; ++i) h[i] = dq_poly(M->D, a, M->v[i]);
        for (int b = 0; b < a; ++b) {
            double p = 0.0;
            for (int i = 0; i < M->Q; ++i) p += M->w[i] * h[i] * M->m[b][i];
            for (int i = 0; i < M->Q; ++i) h[i] -= p * M->m[b][i];
        }
        double nrm = 0.0;
        for (int i = 0; i < M->Q; ++i) nrm += M->w[i] * h[i] * h[i];
        if (nrm < 1e-20) return -2; /* polynomial list not independent on the set */
        nrm = sqrt(nrm);
        for (int i = 0; i < M->Q; ++i) M->m[a][i] = h[i] / nrm;
    }
    return 0;
}

/* Flat exports of a model for the tests: v[Q][3], w[Q], m[Q][Q]. */
int oracle_dq_tables(int id, int *D, int *Q, int *v, double *w, double *m)
{
    dq_model M;
    int rc = oracle_dq_model(id, &M);
    if (rc) return rc;
    *D = M.D;
    *Q = M.Q;
    for (int i = 0; i < M.Q; ++i) {
        for (int a = 0; a < 3; ++a) v[3 * i + a] = M.v[i][a];
        w[i] = M.w[i];
    }
    for (int a = 0; a < M.Q; ++a)
        for (int i = 0; i < M.Q; ++i) m[a * M.Q + i] = M.m[a][i];
    return 0;
}

typedef struct {
    int model;          /* DQ_D1Q3, DQ_D2Q9 or DQ_D3Q15 */
    int n[3];           /* sides; unused ones are 1 */
    double tau[DQ_MAXQ];
    double theta, rho0;
    double u0[3];
    uint64_t seed;
    uint32_t stream_id;
    int ladd;           /* no noise on the ghost modes */
} oracle_dq_cfg;

static size_t dq_sites(const oracle_dq_cfg *c) { return (size_t)c->n[0] * c->n[1] * c->n[2]; }

/* Eq. (2) with c = 1 in D dimensions. */
static void dq_equilibrium(const dq_model *M, double rho, const double u[3], double f0[DQ_MAXQ])
{
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < M->Q; ++i) {
        const double vu = M->v[i][0] * u[0] + M->v[i][1] * u[1] + M->v[i][2] * u[2];
        f0[i] = M->w[i] * rho * (1.0 + 3.0 * vu + 4.5 * vu * vu - 1.5 * uu);
    }
}

/* Eq. (2) for the tests: f0[Q] of model `id` at rho, u[3]. */
int oracle_dq_equilibrium(int id, double rho, const double u[3], double *f0)
{
    dq_model M;
    int rc = oracle_dq_model(id, &M);
    if (rc) return rc;
    dq_equilibrium(&M, rho, u, f0);
    return 0;
}

static void dq_moments(const dq_model *M, const double *f, double *Mo)
{
    for (int a = 0; a < M->Q; ++a) {
        double s = 0.0;
        for (int i = 0; i < M->Q; ++i) s += M->m[a][i] * f[i];
        Mo[a] = s;
    }
}

void oracle_dq_init(const oracle_dq_cfg *c, double *f)
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    double f0[DQ_MAXQ];
    dq_equilibrium(&M, c->rho0, c->u0, f0);
    const size_t V = dq_sites(c);
    for (int i = 0; i < M.Q; ++i)
        for (size_t s = 0; s < V; ++s) f[i * V + s] = f0[i];
}

/* One collision of the populations f[Q] at a site with normals z. */
static void dq_collide(const dq_model *M, const oracle_dq_cfg *c, const double *f,
                       const double *z, double *fs)
{
    double Mo[DQ_MAXQ] = {0}, Meq[DQ_MAXQ] = {0}, Mp[DQ_MAXQ] = {0}, f0[DQ_MAXQ] = {0};
    dq_moments(M, f, Mo);
    const double rho = Mo[0];
    double u[3] = {0, 0, 0};
    for (int a = 0; a < M->D; ++a) u[a] = Mo[1 + a] / sqrt(3.0) / rho;
    dq_equilibrium(M, rho, u, f0);
    dq_moments(M, f0, Meq);
    const double mu = 3.0 * c->theta;
    const int first_ghost = 1 + M->D + M->nstress;
    for (int a = 0; a < M->Q; ++a) {
        if (a <= M->D) {
            Mp[a] = Mo[a];
            continue;
        }
        double sigma = sqrt(mu * c->rho0 * (2.0 * c->tau[a] - 1.0)) / c->tau[a];
        if (c->ladd && a >= first_ghost) sigma = 0.0;
        Mp[a] = Mo[a] - (Mo[a] - Meq[a]) / c->tau[a] + sigma * z[a - M->D - 1];
    }
    for (int i = 0; i < M->Q; ++i) {
        double s = 0.0;
        for (int a = 0; a < M->Q; ++a) s += M->w[i] * M->m[a][i] * Mp[a];
        fs[i] = s;
    }
}

/* Normals z[0..count-1] of a site: draws d = 0, 1, ... of the counter
 * (site, t, stream_id, d), six normals each. */
static void dq_normals(const oracle_dq_cfg *c, uint32_t t, uint32_t site, int count, double *z)
{
    for (int d = 0; 6 * d < count; ++d) {
        uint32_t w[4];
        double zz[6];
        oracle_noise_words(c->seed, c->stream_id, t, site, (uint32_t)d, w);
        oracle_normals_from_words(w, zz);
        for (int k = 0; k < 6 && 6 * d + k < count; ++k) z[6 * d + k] = zz[k];
    }
}

static int wrap(int x, int n) { return ((x % n) + n) % n; }

void oracle_dq_step(const oracle_dq_cfg *c, const double *f, double *fnew, uint32_t t)
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
    const size_t V = dq_sites(c);
    for (int zc = 0; zc < nz; ++zc)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t s = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * zc);
                double fl[DQ_MAXQ], fs[DQ_MAXQ], z[DQ_MAXQ];
                for (int i = 0; i < M.Q; ++i) fl[i] = f[i * V + s];
                dq_normals(c, t, (uint32_t)s, M.Q - M.D - 1, z);
                dq_collide(&M, c, fl, z, fs);
                for (int i = 0; i < M.Q; ++i) {
                    const int xd = wrap(x + M.v[i][0], nx), yd = wrap(y + M.v[i][1], ny);
                    const int zd = wrap(zc + M.v[i][2], nz);
                    fnew[i * V + (size_t)xd + (size_t)nx * ((size_t)yd + (size_t)ny * zd)] = fs[i];
                }
            }
}

/* FP64 sums: mass and the D momentum components. */
void oracle_dq_conservation(const oracle_dq_cfg *c, const double *f, double out[4])
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    const size_t V = dq_sites(c);
    for (int q = 0; q < 4; ++q) out[q] = 0.0;
    for (int i = 0; i < M.Q; ++i)
        for (size_t s = 0; s < V; ++s) {
            out[0] += f[i * V + s];
            for (int a = 0; a < M.D; ++a) out[1 + a] += M.v[i][a] * f[i * V + s];
        }
}

/* Equilibrium-fluctuation start: sqrt(mu rho0 w_i) z_i added to every
 * population, z from the counters (site, 0xffffffff, stream_id, d), each
 * population's spatial mean of the addition removed. */
void oracle_dq_thermalize(const oracle_dq_cfg *c, double *f)
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    const size_t V = dq_sites(c);
    const double mu = 3.0 * c->theta;
    double *add = (double *)malloc(sizeof(double) * M.Q * V);
    double mean[DQ_MAXQ] = {0};
    for (size_t s = 0; s < V; ++s) {
        double z[18];
        dq_normals(c, 0xFFFFFFFFu, (uint32_t)s, M.Q, z);
        for (int i = 0; i < M.Q; ++i) {
            add[i * V + s] = sqrt(mu * c->rho0 * M.w[i]) * z[i];
            mean[i] += add[i * V + s];
        }
    }
    for (int i = 0; i < M.Q; ++i) {
        mean[i] /= (double)V;
        for (size_t s = 0; s < V; ++s) f[i * V + s] += add[i * V + s] - mean[i];
    }
    free(add);
}

/* Number of correlator kinds: |rho|^2, |j_a|^2 (D), |u_a|^2 (D), Re and Im
 * of u_x u_y* (D >= 2), |M^a|^2 for every non-conserved moment. */
int oracle_dq_nkinds(int model)
{
    dq_model M;
    if (oracle_dq_model(model, &M)) return -1;
    return 1 + 2 * M.D + (M.D >= 2 ? 2 : 0) + (M.Q - M.D - 1);
}

/* Adds one sample of the current state to acc[kind][z][y][kx], kx = 0..nx/2,
 * with the kinds of oracle_dq_nkinds; every field X is replaced by
 * X - <X>_x before the D-dimensional transform X(k) = sum_x X(x) e^{-i k.x}
 * (Sec. 3, Eq. 11; Eq. 12 for u_x u_y*). */
void oracle_dq_sample(const oracle_dq_cfg *c, const double *f, double *acc)
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2], nh = nx / 2 + 1;
    const size_t V = dq_sites(c);
    const int D = M.D, nm = M.Q - D - 1;
    const int nf = 1 + 2 * D + nm; /* rho, j, u, moments */
    double *re = (double *)malloc(sizeof(double) * nf * V);
    double *im = (double *)calloc((size_t)nf * V, sizeof(double));
    for (size_t s = 0; s < V; ++s) {
        double fl[DQ_MAXQ], Mo[DQ_MAXQ];
        for (int i = 0; i < M.Q; ++i) fl[i] = f[i * V + s];
        dq_moments(&M, fl, Mo);
        const double rho = Mo[0];
        re[s] = rho;
        for (int a = 0; a < D; ++a) {
            double j = 0.0;
            for (int i = 0; i < M.Q; ++i) j += M.v[i][a] * fl[i];
            re[(1 + a) * V + s] = j;
            re[(1 + D + a) * V + s] = j / rho;
        }
        for (int q = 0; q < nm; ++q) re[(1 + 2 * D + q) * V + s] = Mo[D + 1 + q];
    }
    for (int q = 0; q < nf; ++q) {
        double mean = 0.0;
        for (size_t s = 0; s < V; ++s) mean += re[q * V + s];
        mean /= (double)V;
        for (size_t s = 0; s < V; ++s) re[q * V + s] -= mean;
        oracle_dft3(re + q * V, im + q * V, nx, ny, nz);
    }
    const size_t P = (size_t)nz * ny * nh;
    for (int zc = 0; zc < nz; ++zc)
        for (int y = 0; y < ny; ++y)
            for (int kx = 0; kx < nh; ++kx) {
                const size_t s = (size_t)kx + (size_t)nx * ((size_t)y + (size_t)ny * zc);
                const size_t o = (size_t)kx + (size_t)nh * ((size_t)y + (size_t)ny * zc);
                int kind = 0;
#define SQ(q) (re[(q) * V + s] * re[(q) * V + s] + im[(q) * V + s] * im[(q) * V + s])
                acc[kind++ * P + o] += SQ(0);
                for (int a = 0; a < D; ++a) acc[kind++ * P + o] += SQ(1 + a);
                for (int a = 0; a < D; ++a) acc[kind++ * P + o] += SQ(1 + D + a);
                if (D >= 2) {
                    const size_t ux = (size_t)(1 + D) * V + s, uy = (size_t)(2 + D) * V + s;
                    /* a b* = (ar br + ai bi) + i (ai br - ar bi) */
                    acc[kind++ * P + o] += re[ux] * re[uy] + im[ux] * im[uy];
                    acc[kind++ * P + o] += im[ux] * re[uy] - re[ux] * im[uy];
                }
                for (int q = 0; q < nm; ++q) acc[kind++ * P + o] += SQ(1 + 2 * D + q);
#undef SQ
            }
    free(re);
    free(im);
}

/* nsteps steps from t0 with a sample (into acc, if not NULL) at every t > t0
 * with t % sample_every == 0; returns the number of samples. */
int64_t oracle_dq_run(const oracle_dq_cfg *c, double *f, double *tmp, uint32_t t0, int64_t nsteps,
                      int sample_every, double *acc)
{
    dq_model M;
    oracle_dq_model(c->model, &M);
    const size_t n = (size_t)M.Q * dq_sites(c);
    int64_t ns = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        const uint32_t t = t0 + (uint32_t)k;
        oracle_dq_step(c, f, tmp, t);
        memcpy(f, tmp, n * sizeof(double));
        if (acc && sample_every > 0 && ((uint64_t)t + 1) % (uint64_t)sample_every == 0) {
            oracle_dq_sample(c, f, acc);
            ++ns;
        }
    }
    return ns;
}
