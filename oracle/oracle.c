/*
 * oracle.c -- plain, slow FP64 CPU oracle for the fluctuating ideal-gas
 * D2Q9 lattice Boltzmann method with noise on every non-conserved mode,
 * as stated by Kaehler & Wagner, "Cross Correlators and Galilean Invariance
 * in Fluctuating Ideal Gas Lattice Boltzmann Simulations" (Sec. 2, Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * Everything is FP64 and follows the paper's order of operations:
 *   moments (Eq. 3) -> equilibrium moments (Eq. 10) -> relaxation of every
 *   non-conserved mode by its own 1/tau^a (Eq. 5) -> noise of amplitude
 *   Eq. (8) on modes 3..8 (Sec. 2, last paragraph) -> back transform with
 *   n_i^a = w_i m_i^a (Eq. 4) -> streaming f_i(x+v_i, t+1) (Eq. 1).
 *
 * The random numbers are the one documented counter-based stream (Philox4x32
 * with 10 rounds, Salmon, Moraes, Dror & Shaw, SC'11) written here from its
 * published definition; the GPU library implements the same definition on
 * its own.
 *
 * State layout: f[i][y][x], i = 0..8, row-major, full populations (not
 * deviations), pre-collision (i.e. just after streaming) at integer times.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* D2Q9 lattice, Sec. 3: velocity order, weights and the matrix m_i^a. */
/* ------------------------------------------------------------------ */

/* Velocity set in the order listed in Sec. 3. */
static const int VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Weights: the printed list has eight entries; the missing fourth 1/9 is
 * restored so that the weights sum to one and Eq. (4) holds. */
static double W[9];
/* m[a][i]: Eq. (9), rows a = moment, columns i = velocity. */
static double M[9][9];
/* n[i][a] = w_i m_i^a (text after Eq. 9). */
static double N[9][9];
static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    const double s3 = sqrt(3.0), s32 = sqrt(1.5), s6 = sqrt(6.0);
    const double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                         1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    const double m[9][9] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, s3, 0, -s3, 0, s3, -s3, -s3, s3},
        {0, 0, s3, 0, -s3, s3, s3, -s3, -s3},
        {0, 1.5, -1.5, 1.5, -1.5, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 3, -3, 3, -3},
        {-1, 0.5, 0.5, 0.5, 0.5, 2, 2, 2, 2},
        {0, -s32, 0, s32, 0, s6, -s6, -s6, s6},
        {0, 0, -s32, 0, s32, s6, s6, -s6, -s6},
        {0.5, -1, -1, -1, -1, 2, 2, 2, 2},
    };
    for (int i = 0; i < 9; ++i) W[i] = w[i];
    for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 9; ++i) {
            M[a][i] = m[a][i];
            N[i][a] = w[i] * m[a][i];
        }
    tables_ready = 1;
}

/* Export the tables so that tests can check them against Eq. (4). */
void oracle_tables(double m_out[81], double n_out[81], double w_out[9], int v_out[18])
{
    init_tables();
    for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 9; ++i) {
            m_out[a * 9 + i] = M[a][i];
            n_out[i * 9 + a] = N[i][a];
        }
    for (int i = 0; i < 9; ++i) {
        w_out[i] = W[i];
        v_out[2 * i] = VX[i];
        v_out[2 * i + 1] = VY[i];
    }
}

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11). */
/* ------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {               /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Words of one draw.  Counter = (site, t, stream_id, d); key = the two
 * 32-bit halves of the 64-bit seed (low half first). */
void oracle_noise_words(uint64_t seed, uint32_t stream_id, uint32_t t, uint32_t site,
                        uint32_t d, uint32_t w[4])
{
    const uint32_t ctr[4] = {site, t, stream_id, d};
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* Six unit normals from the four words of one draw.
 * Radius uniforms  r_p = (2*(w_p >> 9) + 1) * 2^-24,                p = 0,1,2
 * Angle uniforms   a_p = (2*alpha_p + 1) * 2^-20,
 *                  alpha_p = ((w_p & 0x1ff) << 10) | ((w_3 >> 10p) & 0x3ff)
 * Box-Muller:      z_2p = sqrt(-2 ln r_p) cos(2 pi a_p),
 *                  z_2p+1 = sqrt(-2 ln r_p) sin(2 pi a_p).
 * The paper asks only for zero mean and unit variance (Eq. 8); the
 * Gaussian shape is the reading taken for it. */
void oracle_normals_from_words(const uint32_t w[4], double z[6])
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < 3; ++p) {
        double r = (2.0 * (double)(w[p] >> 9) + 1.0) * 0x1p-24;
        uint32_t alpha = ((w[p] & 0x1FFu) << 10) | ((w[3] >> (10 * p)) & 0x3FFu);
        double a = (2.0 * (double)alpha + 1.0) * 0x1p-20;
        double R = sqrt(-2.0 * log(r));
        z[2 * p] = R * cos(two_pi * a);
        z[2 * p + 1] = R * sin(two_pi * a);
    }
}

/* ------------------------------------------------------------------ */
/* Physics of one site                                                 */
/* ------------------------------------------------------------------ */

/* Eq. (2) with c = 1 (lattice units). */
void oracle_equilibrium(double rho, double ux, double uy, double f0[9])
{
    init_tables();
    const double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double uv = ux * VX[i] + uy * VY[i];
        f0[i] = rho * W[i] * (1.0 + 3.0 * uv + 4.5 * uv * uv - 1.5 * uu);
    }
}

/* Eq. (3): M^a = sum_i m_i^a f_i. */
void oracle_moments(const double f[9], double Mo[9])
{
    init_tables();
    for (int a = 0; a < 9; ++a) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += M[a][i] * f[i];
        Mo[a] = s;
    }
}

/* Eq. (10): equilibrium moments from rho and u = j / rho. */
void oracle_equilibrium_moments(double rho, double ux, double uy, double Meq[9])
{
    const double s3 = sqrt(3.0);
    Meq[0] = rho;
    Meq[1] = s3 * rho * ux;
    Meq[2] = s3 * rho * uy;
    Meq[3] = 1.5 * rho * (ux * ux - uy * uy);
    Meq[4] = 3.0 * rho * ux * uy;
    Meq[5] = 1.5 * rho * (ux * ux + uy * uy);
    Meq[6] = 0.0;
    Meq[7] = 0.0;
    Meq[8] = 0.0;
}

/* Eq. (8): xi^a = (1/tau^a) sqrt(rhobar (2 tau^a - 1)) N.  The paper's
 * variance rhobar is in units where k_B T = c_s^2 = 1/3; a noise temperature
 * theta scales it by mu = theta / c_s^2 = 3 theta.  rhobar is the constant
 * rho0 (the u << 1 form of Eq. 7, kept as is).  Modes 0..2 are conserved and
 * get none; with `ladd` set the ghost modes 6..8 get none either (the older
 * scheme the paper compares against). */
void oracle_noise_amplitudes(const double tau[9], double theta, double rho0, int ladd,
                             double sigma[9])
{
    const double mu = 3.0 * theta;
    for (int a = 0; a < 9; ++a) {
        if (a < 3 || (ladd && a >= 6))
            sigma[a] = 0.0;
        else
            sigma[a] = sqrt(mu * rho0 * (2.0 * tau[a] - 1.0)) / tau[a];
    }
}

/* Collision of one site, Eq. (5): returns the post-collision populations
 * f*_i = sum_a n_i^a { M^a - (M^a - M^{a,0}) / tau^a + xi^a }.
 * For the conserved modes a = 0,1,2 M^a = M^{a,0} holds exactly, so they are
 * carried over unchanged (their tau^a is irrelevant). */
void oracle_collide_site(const double f[9], const double tau[9], const double sigma[9],
                         const double z[6], double fstar[9])
{
    init_tables();
    double Mo[9], Meq[9], Mp[9];
    oracle_moments(f, Mo);
    const double rho = Mo[0];
    const double jx = Mo[1] / sqrt(3.0), jy = Mo[2] / sqrt(3.0);
    const double ux = jx / rho, uy = jy / rho;
    oracle_equilibrium_moments(rho, ux, uy, Meq);
    for (int a = 0; a < 9; ++a) {
        if (a < 3) {
            Mp[a] = Mo[a];
        } else {
            double xi = sigma[a] * z[a - 3];
            Mp[a] = Mo[a] - (Mo[a] - Meq[a]) / tau[a] + xi;
        }
    }
    for (int i = 0; i < 9; ++i) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += N[i][a] * Mp[a];
        fstar[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Whole lattice                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int nx, ny;
    double tau[9];
    double theta, rho0, u0x, u0y;
    uint64_t seed;
    uint32_t stream_id;
    int ladd;
} oracle_cfg;

static inline size_t idx(const oracle_cfg *c, int i, int y, int x)
{
    return ((size_t)i * (size_t)c->ny + (size_t)y) * (size_t)c->nx + (size_t)x;
}

/* Initial state: the uniform equilibrium f_i^0(rho0, u0) of Eq. (2). */
void oracle_init(const oracle_cfg *c, double *f)
{
    double f0[9];
    oracle_equilibrium(c->rho0, c->u0x, c->u0y, f0);
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) f[idx(c, i, y, x)] = f0[i];
}

/* One time step t -> t+1 of Eq. (1)/(5): collide every site with the noise of
 * counter (site = y*nx + x, t, stream_id, 0), then stream periodically. */
void oracle_step(const oracle_cfg *c, const double *f, double *fnew, uint32_t t)
{
    double sigma[9];
    oracle_noise_amplitudes(c->tau, c->theta, c->rho0, c->ladd, sigma);
    const int nx = c->nx, ny = c->ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fs[9], fo[9], z[6];
            uint32_t w[4];
            for (int i = 0; i < 9; ++i) fs[i] = f[idx(c, i, y, x)];
            uint32_t site = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
            oracle_noise_words(c->seed, c->stream_id, t, site, 0, w);
            oracle_normals_from_words(w, z);
            oracle_collide_site(fs, c->tau, sigma, z, fo);
            for (int i = 0; i < 9; ++i) {
                int xd = (x + VX[i] + nx) % nx;
                int yd = (y + VY[i] + ny) % ny;
                fnew[idx(c, i, yd, xd)] = fo[i];
            }
        }
}

/* Global sums: mass, momentum, and the staggered momenta
 * sum_x (-1)^x j_x and sum_y (-1)^y j_y.  out[0] is sum (rho - rho0). */
void oracle_conservation(const oracle_cfg *c, const double *f, double out[5])
{
    double s[5] = {0, 0, 0, 0, 0};
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            double rho = 0, jx = 0, jy = 0;
            for (int i = 0; i < 9; ++i) {
                double v = f[idx(c, i, y, x)];
                rho += v;
                jx += VX[i] * v;
                jy += VY[i] * v;
            }
            s[0] += rho - c->rho0;
            s[1] += jx;
            s[2] += jy;
            s[3] += (x & 1) ? -jx : jx;
            s[4] += (y & 1) ? -jy : jy;
        }
    for (int k = 0; k < 5; ++k) out[k] = s[k];
}

/* Equilibrium-fluctuation start: add sqrt(mu rho0 w_i) z_i(x) to every
 * population, z from the counters (site, 0xffffffff, stream_id, d), d = 0,1
 * (twelve normals, the first nine used), then remove each population's spatial
 * mean of what was added so that total mass and momentum are unchanged. */
void oracle_thermalize(const oracle_cfg *c, double *f)
{
    init_tables();
    const int nx = c->nx, ny = c->ny;
    const double mu = 3.0 * c->theta;
    const double V = (double)nx * (double)ny;
    double *add = (double *)malloc(sizeof(double) * 9 * (size_t)nx * (size_t)ny);
    double mean[9] = {0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            uint32_t site = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
            uint32_t w[4];
            double z[12];
            oracle_noise_words(c->seed, c->stream_id, 0xFFFFFFFFu, site, 0, w);
            oracle_normals_from_words(w, z);
            oracle_noise_words(c->seed, c->stream_id, 0xFFFFFFFFu, site, 1, w);
            oracle_normals_from_words(w, z + 6);
            for (int i = 0; i < 9; ++i) {
                double a = sqrt(mu * c->rho0 * W[i]) * z[i];
                add[idx(c, i, y, x)] = a;
                mean[i] += a;
            }
        }
    for (int i = 0; i < 9; ++i) mean[i] /= V;
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) f[idx(c, i, y, x)] += add[idx(c, i, y, x)] - mean[i];
    free(add);
}

/* ------------------------------------------------------------------ */
/* Discrete Fourier transform, Sec. 3: X(k) = sum_x X(x) exp(-i k.x).  */
/* ------------------------------------------------------------------ */

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* One line of length n, stride s, in place; re/im separate arrays.
 * Powers of two: iterative radix-2 decimation in time; any other length:
 * the direct sum.  Twiddles are taken from cos/sin of the exact angle. */
static void dft_line(double *re, double *im, int n, size_t s, double *wr, double *wi)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (is_pow2(n)) {
        /* bit-reversal permutation */
        for (int i = 1, j = 0; i < n; ++i) {
            int bit = n >> 1;
            for (; j & bit; bit >>= 1) j ^= bit;
            j ^= bit;
            if (i < j) {
                double tr = re[i * s], ti = im[i * s];
                re[i * s] = re[j * s]; im[i * s] = im[j * s];
                re[j * s] = tr; im[j * s] = ti;
            }
        }
        for (int len = 2; len <= n; len <<= 1) {
            int half = len >> 1;
            for (int k = 0; k < half; ++k) {
                double ang = -two_pi * (double)k / (double)len;
                double c = cos(ang), sn = sin(ang);
                for (int b = 0; b < n; b += len) {
                    size_t p = (size_t)(b + k) * s, q = (size_t)(b + k + half) * s;
                    double xr = re[q] * c - im[q] * sn;
                    double xi = re[q] * sn + im[q] * c;
                    re[q] = re[p] - xr; im[q] = im[p] - xi;
                    re[p] += xr; im[p] += xi;
                }
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            double sr = 0, si = 0;
            for (int j = 0; j < n; ++j) {
                long long ph = ((long long)j * (long long)k) % n;
                double ang = -two_pi * (double)ph / (double)n;
                double c = cos(ang), sn = sin(ang);
                sr += re[j * s] * c - im[j * s] * sn;
                si += re[j * s] * sn + im[j * s] * c;
            }
            wr[k] = sr; wi[k] = si;
        }
        for (int k = 0; k < n; ++k) { re[k * s] = wr[k]; im[k * s] = wi[k]; }
    }
}

/* Two-dimensional transform of an ny x nx complex field, in place. */
void oracle_dft2(double *re, double *im, int nx, int ny)
{
    int nmax = nx > ny ? nx : ny;
    double *wr = (double *)malloc(sizeof(double) * nmax);
    double *wi = (double *)malloc(sizeof(double) * nmax);
    for (int y = 0; y < ny; ++y) dft_line(re + (size_t)y * nx, im + (size_t)y * nx, nx, 1, wr, wi);
    for (int x = 0; x < nx; ++x) dft_line(re + x, im + x, ny, (size_t)nx, wr, wi);
    free(wr);
    free(wi);
}

/* Three-dimensional transform of an nz x ny x nx complex field, in place
 * (x fastest); sides of 1 are allowed, so it also serves one and two
 * dimensions. */
void oracle_dft3(double *re, double *im, int nx, int ny, int nz)
{
    int nmax = nx > ny ? nx : ny;
    if (nz > nmax) nmax = nz;
    double *wr = (double *)malloc(sizeof(double) * nmax);
    double *wi = (double *)malloc(sizeof(double) * nmax);
    const size_t pl = (size_t)nx * ny;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const size_t o = z * pl + (size_t)y * nx;
            dft_line(re + o, im + o, nx, 1, wr, wi);
        }
    if (ny > 1)
        for (int z = 0; z < nz; ++z)
            for (int x = 0; x < nx; ++x) {
                const size_t o = z * pl + x;
                dft_line(re + o, im + o, ny, (size_t)nx, wr, wi);
            }
    if (nz > 1)
        for (size_t o = 0; o < pl; ++o) dft_line(re + o, im + o, nz, pl, wr, wi);
    free(wr);
    free(wi);
}

/* ------------------------------------------------------------------ */
/* Correlator sample, Eq. (11) and Eq. (12)                            */
/* ------------------------------------------------------------------ */

/* Number of kx columns kept: 0 .. floor(nx/2) (the fields are real, so
 * X(-k) = conj X(k) and the other half carries no new information). */
int oracle_nkx(int nx) { return nx / 2 + 1; }

/* Adds one sample of the current (pre-collision) state to acc, laid out as
 * acc[kind][ky][kx], ky = 0..ny-1, kx = 0..nx/2, with kinds
 *  0 |rho|^2  1 |jx|^2  2 |jy|^2  3 |ux|^2  4 |uy|^2
 *  5,6 Re,Im ux uy*   7,8 Re,Im rho jx*   9,10 Re,Im rho jy*
 *  11,12 Re,Im rho ux*  13,14 Re,Im rho uy*
 * Each field X is replaced by dX = X - <X>_x before the transform (the
 * fluctuation of Sec. 3); u = j / rho at every site. */
void oracle_sample(const oracle_cfg *c, const double *f, double *acc)
{
    const int nx = c->nx, ny = c->ny, nh = oracle_nkx(nx);
    const size_t V = (size_t)nx * (size_t)ny;
    double *re = (double *)malloc(sizeof(double) * 5 * V);
    double *im = (double *)calloc(5 * V, sizeof(double));
    double mean[5] = {0, 0, 0, 0, 0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double rho = 0, jx = 0, jy = 0;
            for (int i = 0; i < 9; ++i) {
                double v = f[idx(c, i, y, x)];
                rho += v;
                jx += VX[i] * v;
                jy += VY[i] * v;
            }
            double fld[5] = {rho, jx, jy, jx / rho, jy / rho};
            for (int q = 0; q < 5; ++q) {
                re[q * V + (size_t)y * nx + x] = fld[q];
                mean[q] += fld[q];
            }
        }
    for (int q = 0; q < 5; ++q) {
        mean[q] /= (double)V;
        for (size_t s = 0; s < V; ++s) re[q * V + s] -= mean[q];
        oracle_dft2(re + q * V, im + q * V, nx, ny);
    }
    const size_t P = (size_t)ny * (size_t)nh;
    for (int ky = 0; ky < ny; ++ky)
        for (int kx = 0; kx < nh; ++kx) {
            size_t s = (size_t)ky * nx + kx, o = (size_t)ky * nh + kx;
            double Xr[5], Xi[5];
            for (int q = 0; q < 5; ++q) { Xr[q] = re[q * V + s]; Xi[q] = im[q * V + s]; }
            /* a b* = (ar br + ai bi) + i (ai br - ar bi) */
#define RE_AB(a, b) (Xr[a] * Xr[b] + Xi[a] * Xi[b])
#define IM_AB(a, b) (Xi[a] * Xr[b] - Xr[a] * Xi[b])
            acc[0 * P + o] += RE_AB(0, 0);
            acc[1 * P + o] += RE_AB(1, 1);
            acc[2 * P + o] += RE_AB(2, 2);
            acc[3 * P + o] += RE_AB(3, 3);
            acc[4 * P + o] += RE_AB(4, 4);
            acc[5 * P + o] += RE_AB(3, 4);
            acc[6 * P + o] += IM_AB(3, 4);
            acc[7 * P + o] += RE_AB(0, 1);
            acc[8 * P + o] += IM_AB(0, 1);
            acc[9 * P + o] += RE_AB(0, 2);
            acc[10 * P + o] += IM_AB(0, 2);
            acc[11 * P + o] += RE_AB(0, 3);
            acc[12 * P + o] += IM_AB(0, 3);
            acc[13 * P + o] += RE_AB(0, 4);
            acc[14 * P + o] += IM_AB(0, 4);
#undef RE_AB
#undef IM_AB
        }
    free(re);
    free(im);
}

/* Structure factors of the six non-conserved moments (Eq. 11 applied to
 * every moment of Eq. 9, Sec. 3): adds |dM^a(k)|^2, a = 3..8, of the current
 * (pre-collision) state to accm[a-3][ky][kx] (same k layout as
 * oracle_sample), where M^a(x) = sum_i m_i^a f_i(x) (Eq. 3) and
 * dM^a = M^a - <M^a>_x.  The conserved moments are rho and sqrt(3) j_a,
 * already covered by oracle_sample. */
void oracle_sample_moments(const oracle_cfg *c, const double *f, double *accm)
{
    init_tables();
    const int nx = c->nx, ny = c->ny, nh = oracle_nkx(nx);
    const size_t V = (size_t)nx * (size_t)ny;
    double *re = (double *)malloc(sizeof(double) * 6 * V);
    double *im = (double *)calloc(6 * V, sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fs[9], Mo[9];
            for (int i = 0; i < 9; ++i) fs[i] = f[idx(c, i, y, x)];
            oracle_moments(fs, Mo);
            for (int a = 3; a < 9; ++a) re[(size_t)(a - 3) * V + (size_t)y * nx + x] = Mo[a];
        }
    for (int q = 0; q < 6; ++q) {
        double mean = 0.0;
        for (size_t s = 0; s < V; ++s) mean += re[q * V + s];
        mean /= (double)V;
        for (size_t s = 0; s < V; ++s) re[q * V + s] -= mean;
        oracle_dft2(re + q * V, im + q * V, nx, ny);
    }
    const size_t P = (size_t)ny * (size_t)nh;
    for (int q = 0; q < 6; ++q)
        for (int ky = 0; ky < ny; ++ky)
            for (int kx = 0; kx < nh; ++kx) {
                size_t s = q * V + (size_t)ky * nx + kx;
                accm[q * P + (size_t)ky * nh + kx] += re[s] * re[s] + im[s] * im[s];
            }
    free(re);
    free(im);
}

/* Run nsteps steps from time t0, sampling (into acc, if not NULL) the state
 * at every time t > t0 with t % sample_every == 0; the moment structure
 * factors go to accm when it is not NULL.  f holds the state on entry and on
 * return; tmp is scratch of the same size.  Returns the number of samples
 * taken. */
int64_t oracle_run(const oracle_cfg *c, double *f, double *tmp, uint32_t t0, int64_t nsteps,
                   int sample_every, double *acc, double *accm)
{
    const size_t n = (size_t)9 * (size_t)c->nx * (size_t)c->ny;
    int64_t ns = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        uint32_t t = t0 + (uint32_t)s;
        oracle_step(c, f, tmp, t);
        memcpy(f, tmp, n * sizeof(double));
        if (acc && sample_every > 0 && ((uint64_t)t + 1) % (uint64_t)sample_every == 0) {
            oracle_sample(c, f, acc);
            if (accm) oracle_sample_moments(c, f, accm);
            ++ns;
        }
    }
    return ns;
}
