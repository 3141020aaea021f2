"""Oracle pins for the noise (Sec. 2, Eqs. 6-8) and its random-number stream.

The stream is Philox4x32-10 (Salmon et al., SC'11), checked against the
generator's published known-answer vectors; the normals derived from it are
checked statistically; the amplitude against the fluctuation-dissipation
relation Eq. (6) with the decoupled variance of Eq. (7).
"""
import os

import numpy as np
import pytest
import scipy.stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        h = [int(x, 16) for x in line.split()]
        rows.append((h[0:4], h[4:6], h[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle_lib.philox(ctr, key).tolist() == out


def test_noise_counter_layout(oracle_lib):
    """Counter (site, t, stream_id, d), key (seed low 32, seed high 32)."""
    seed = 0x0123456789ABCDEF
    w = oracle_lib.noise_words(seed, 7, 11, 12345, 1)
    ref = oracle_lib.philox([12345, 11, 7, 1], [0x89ABCDEF, 0x01234567])
    assert w.tolist() == ref.tolist()


@pytest.fixture(scope="module")
def zs(oracle_lib):
    """Normals of 2^16 consecutive sites of one step."""
    n = 1 << 16
    z = np.empty((n, 6))
    for s in range(n):
        z[s] = oracle_lib.normals_from_words(oracle_lib.noise_words(1, 3, 5, s, 0))
    return z


def test_normals_moments(zs):
    """Eq. (8) needs N with zero mean and unit variance; Gaussian shape (the
    reading taken) is checked by kurtosis and a KS test."""
    n = zs.shape[0]
    for c in range(6):
        x = zs[:, c]
        assert abs(x.mean()) < 5 / np.sqrt(n)
        assert abs(x.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(scipy.stats.kurtosis(x, fisher=False) - 3) < 5 * np.sqrt(24 / n)
        assert scipy.stats.kstest(x, "norm").pvalue > 1e-4
    assert np.abs(zs).max() < 5.8  # 24-bit radius uniforms bound |z|


def test_normals_independent(zs):
    """The six normals of one site and of neighbouring sites are uncorrelated
    (Eq. 7 needs independent noise on every mode)."""
    n = zs.shape[0]
    c = np.corrcoef(zs.T)
    off = c[~np.eye(6, dtype=bool)]
    assert np.abs(off).max() < 5 / np.sqrt(n)
    lag = np.array([np.corrcoef(zs[:-1, a], zs[1:, a])[0, 1] for a in range(6)])
    assert np.abs(lag).max() < 5 / np.sqrt(n)
    # squares too (a shared radius would show up here)
    sq = np.corrcoef((zs ** 2).T)
    assert np.abs(sq[~np.eye(6, dtype=bool)]).max() < 5 / np.sqrt(n)


def test_uniform_range_extremes(oracle_lib):
    """All-ones words give the largest radius uniform 1 - 2^-24, all-zero words
    the smallest 2^-24: |z| stays finite and the largest |z| is
    sqrt(-2 ln 2^-24) = 5.768."""
    z1 = oracle_lib.normals_from_words([0xFFFFFFFF] * 4)
    assert np.all(np.abs(z1) < 1e-3)
    z0 = oracle_lib.normals_from_words([0, 0, 0, 0])
    R = np.hypot(z0[0::2], z0[1::2])
    assert np.allclose(R, np.sqrt(-2 * np.log(2.0 ** -24)), rtol=1e-14)


def test_noise_adds_nothing_to_mass_and_momentum(oracle_lib):
    """Sum_i xi_i = 0 and sum_i xi_i v_i = 0 at every site (after Eq. 2): the
    difference of a noisy and a noise-free collision of the same input."""
    rng = np.random.default_rng(5)
    _, _, _, v = oracle_lib.tables()
    tau = [1, 1, 1, 0.8, 0.8, 0.9, 1.0, 1.2, 0.7]
    sigma = oracle_lib.noise_amplitudes(tau, 1e-2, 1.0)
    for _ in range(50):
        f = oracle_lib.equilibrium(1.0, 0.05, -0.02) * (1 + 0.1 * rng.standard_normal(9))
        z = rng.standard_normal(6)
        xi = oracle_lib.collide_site(f, tau, sigma, z) - oracle_lib.collide_site(f, tau, sigma, 0 * z)
        scale = np.abs(xi).sum()
        assert abs(xi.sum()) <= 1e-15 * scale + 1e-18
        assert np.abs(v.T @ xi).max() <= 1e-15 * scale + 1e-18


def test_noise_amplitude_satisfies_fdt(oracle_lib):
    """Eq. (6) with a = c and Eq. (7): a mode relaxed by (1 - 1/tau) and kicked
    by xi keeps the variance mu rho0 (mu = 3 theta) stationary:
    (1 - 1/tau)^2 mu rho0 + sigma^2 = mu rho0.  The amplitude is read off the
    collision itself (unit kick per mode) rather than from the formula."""
    _, n, _, _ = oracle_lib.tables()
    tau = [1, 1, 1, 0.55, 0.8, 1.0, 1.4, 2.0, 0.9]
    theta, rho0 = 2e-3, 1.3
    sigma = oracle_lib.noise_amplitudes(tau, theta, rho0)
    f0 = oracle_lib.equilibrium(rho0, 0.0, 0.0)
    base = oracle_lib.collide_site(f0, tau, sigma, np.zeros(6))
    mu = 3 * theta
    for a in range(3, 9):
        z = np.zeros(6); z[a - 3] = 1.0
        dM = oracle_lib.moments(oracle_lib.collide_site(f0, tau, sigma, z) - base)
        expect = np.zeros(9); expect[a] = dM[a]
        assert np.abs(dM - expect).max() < 1e-15, "noise leaked into another mode"
        s2 = dM[a] ** 2
        assert abs((1 - 1 / tau[a]) ** 2 * mu * rho0 + s2 - mu * rho0) < 1e-15
    for a in range(3):
        assert sigma[a] == 0.0


def test_ladd_switch_removes_ghost_noise(oracle_lib):
    """The comparison scheme of Sec. 3 sets the noise on M^6, M^7, M^8 to zero."""
    tau = [1.0] * 9
    s = oracle_lib.noise_amplitudes(tau, 1 / 3, 1.0, ladd=True)
    g = oracle_lib.noise_amplitudes(tau, 1 / 3, 1.0, ladd=False)
    assert np.all(s[6:] == 0) and np.all(g[6:] > 0)
    assert np.all(s[3:6] == g[3:6])
    # paper units (theta = k_B T = 1/3, rho0 = 1, tau = 1): xi^a has unit variance
    assert np.allclose(g[3:], 1.0, atol=1e-15)
