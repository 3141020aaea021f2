"""Pins of the oracle's moment structure factors (Eq. 11 for every moment of
Eq. 9; Sec. 3 reports S_k = 1 for all nine D2Q9 moments with ghost noise).

* A plane wave built from the Hermite-polynomial basis (not the oracle's
  table) puts exactly (c_a V / 2)^2 on its own wave vector and moment and
  nothing elsewhere; a constant offset does not reach k != 0.
* The thermal start draws independent populations of variance mu rho0 w_i,
  so every moment has per-site variance mu rho0 and S = 1 on average.
* In the paper's regime (all tau^a = 1) the stationary S(M^a) match the
  linear-response predictor: 1 everywhere with ghost noise, the large
  finite-k deficits of the older scheme without it.
"""
import numpy as np

import lyapunov
from stats_util import block_means, zscores

MKEYS = tuple("S_M%d" % a for a in range(3, 9))


def _wave(nx, ny, k0, amp, phase, offset, rho0=1.0):
    _, w, m = lyapunov.basis()
    y, x = np.mgrid[0:ny, 0:nx]
    arg = 2 * np.pi * (k0[0] * x / nx + k0[1] * y / ny)
    f = np.empty((9, ny, nx))
    for i in range(9):
        f[i] = w[i] * rho0
        for a in range(3, 9):
            f[i] += w[i] * m[a, i] * (amp[a - 3] * np.cos(arg + phase[a - 3]) + offset[a - 3])
    return f


def _sample(oracle_lib, f):
    _, ny, nx = f.shape
    L = oracle_lib.Lattice(nx, ny, [1.0] * 9, 1e-4, moments=True)
    L.set_populations(f)
    L.sample()
    return L.acc_m


def test_plane_wave_lands_on_its_own_moment_and_k(oracle_lib):
    nx, ny = 12, 10
    amp = 1e-3 * np.array([0.3, 0.5, 0.7, 1.1, 1.3, 1.7])
    phase = np.array([0.1, 0.9, 2.0, -1.2, 0.4, 3.0])
    offset = 1e-3 * np.array([2.0, -1.0, 0.5, 3.0, -2.5, 1.5])
    V = nx * ny
    for k0 in ((3, 2), (5, 7), (0, 3)):
        acc = _sample(oracle_lib, _wave(nx, ny, k0, amp, phase, offset))
        exp = np.zeros_like(acc)
        for a in range(6):
            val = (amp[a] * V / 2) ** 2
            exp[a, k0[1], k0[0]] = val
            if k0[0] == 0:  # -k0 is also on the stored half plane
                exp[a, (ny - k0[1]) % ny, 0] = val
        assert np.abs(acc - exp).max() < 1e-12 * exp.max(), k0


def test_thermal_start_has_unit_moment_variance(oracle_lib):
    nx = ny = 48
    theta = 1e-4
    vals = []
    for seed in range(4):
        L = oracle_lib.Lattice(nx, ny, [1.0] * 9, theta, seed=seed + 11, thermalize=True,
                               moments=True)
        L.sample()
        s = oracle_lib.normalized_moments(L.acc_m, 1, nx, ny, theta, 1.0)
        vals.append(np.stack([s[k] for k in MKEYS]))
    v = np.stack(vals)  # (seed, a, ky, kx)
    v[:, :, 0, 0] = np.nan  # k = 0: mean removed
    per_moment = np.nanmean(v, axis=(0, 2, 3))
    # |X_k|^2 is exponential: relative error of the mean over ~4 x 1200 k is 1.5 %
    assert np.abs(per_moment - 1.0).max() < 0.08, per_moment


def _mask(nx, ny):
    nh = nx // 2 + 1
    m = np.ones((ny, nh), dtype=bool)
    for ky in range(ny):
        for kx in range(nh):
            m[ky, kx] = not lyapunov.singular_k(nx, ny, kx, ky)
    return m


def _blocks(oracle_lib, nx, ny, tau, theta, ladd, nblocks, steps, every, seed):
    L = oracle_lib.Lattice(nx, ny, tau, theta=theta, seed=seed, ladd=ladd, thermalize=True,
                           moments=True)
    L.run(300)

    def block():
        L.acc[...] = 0.0
        L.acc_m[...] = 0.0
        L.nsamples = 0
        L.run(steps, every)
        return oracle_lib.normalized_moments(L.acc_m, L.nsamples, nx, ny, theta, 1.0)

    return block_means(block, nblocks)


def _check(mean, sem, pred, mask, mu):
    zs = []
    for k in MKEYS:
        z = zscores(mean[k], sem[k], pred[k], mask, model_err=3 * mu)
        assert np.abs(z).max() < 6.0, (k, np.abs(z).max())
        zs.append(z)
    chi = (np.concatenate(zs) ** 2).mean()
    assert 0.6 < chi < 1.7, chi


def test_moment_structure_factors_with_ghost_noise(oracle_lib):
    nx = ny = 10
    tau = [1.0] * 9
    theta = 1e-4
    mean, sem = _blocks(oracle_lib, nx, ny, tau, theta, False, 16, 1500, 3, seed=41)
    pred = lyapunov.predict(nx, ny, tau, theta)
    m = _mask(nx, ny)
    for k in MKEYS:  # the prediction is the closed form S = 1
        assert np.nanmax(np.abs(pred[k][m] - 1.0)) < 1e-12
    _check(mean, sem, pred, m, 3 * theta)


def test_moment_structure_factors_without_ghost_noise(oracle_lib):
    nx = ny = 10
    tau = [1.0] * 9
    theta = 1e-4
    mean, sem = _blocks(oracle_lib, nx, ny, tau, theta, True, 16, 1500, 3, seed=42)
    pred = lyapunov.predict(nx, ny, tau, theta, ladd=True)
    m = _mask(nx, ny)
    _check(mean, sem, pred, m, 3 * theta)
    # the deficit is large: the ghost modes sit far below 1 away from the axes
    for k in ("S_M6", "S_M7", "S_M8"):
        assert np.nanmean(mean[k][m]) < 0.6
