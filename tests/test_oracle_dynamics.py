"""Oracle pins for whole-lattice dynamics (Eq. 1 / Eq. 5 on a periodic lattice).

Fixed by the physics rather than by the oracle's own formulas:
  * exact conservation of mass and momentum (requirement stated after Eq. 2);
  * the noise-free uniform equilibrium is a fixed point at any mean velocity;
  * decay of shear and sound waves at the rates set by tau (hydrodynamic
    closed forms, and the exact eigenvalues of the linearised step);
  * the staggered momentum sum_x (-1)^x j_x flips sign every step (exact, also
    with noise), because streaming shifts every population with v_x = +-1 by
    one site and the collision conserves j_x at each site.
"""
import numpy as np
import pytest

import lyapunov
from paper_1010_1233_amd import workloads

TAU_C1 = workloads.tau_vector(0.8, 0.8, 1.0)


def test_mass_momentum_conserved_from_random_state(oracle_lib):
    L = oracle_lib.Lattice(16, 12, TAU_C1, theta=1e-3, rho0=1.0, u0=(0.0, 0.0), seed=9)
    f0 = oracle_lib.equilibrium(1.0, 0.02, -0.01)
    L.set_populations(workloads.perturbed(f0, 16, 12, 0.01, seed=11))
    c0 = L.conservation()
    L.step(500)
    c1 = L.conservation()
    mass = 16 * 12 * 1.0
    assert abs(c1[0] - c0[0]) <= 1e-12 * mass
    assert np.abs(c1[1:3] - c0[1:3]).max() <= 1e-12 * mass


@pytest.mark.parametrize("nx,ny", [(7, 5), (2, 2), (3, 11)])
def test_conservation_odd_and_tiny_lattices(oracle_lib, nx, ny):
    L = oracle_lib.Lattice(nx, ny, TAU_C1, theta=1e-3, seed=3)
    c0 = L.conservation()
    L.step(200)
    c1 = L.conservation()
    assert np.abs(c1[:3] - c0[:3]).max() <= 1e-12 * nx * ny


def test_noise_free_uniform_state_is_fixed(oracle_lib):
    """theta = 0: f^0(rho0, u0) is exactly stationary (M = M^0 at every site)."""
    L = oracle_lib.Lattice(16, 16, workloads.tau_vector(0.6, 0.9, 1.3), theta=0.0,
                           u0=(0.1, 0.03))
    f0 = L.f.copy()
    L.step(300)
    assert np.abs(L.f - f0).max() <= 1e-15


def _wave_series(oracle_lib, L_side, tau, field, nsteps, amp=1e-6):
    """Fourier amplitude at k = 2 pi / L along x of a small wave, theta = 0."""
    nx, ny = L_side, 2
    L = oracle_lib.Lattice(nx, ny, tau, theta=0.0)
    x = np.arange(nx)
    f = np.empty((9, ny, nx))
    for xi in range(nx):
        if field == "shear":
            f0 = oracle_lib.equilibrium(1.0, 0.0, amp * np.sin(2 * np.pi * xi / nx))
        else:
            f0 = oracle_lib.equilibrium(1.0 + amp * np.cos(2 * np.pi * xi / nx), 0.0, 0.0)
        f[:, :, xi] = f0[:, None]
    L.set_populations(f)
    _, _, _, v = oracle_lib.tables()
    ph = np.exp(-2j * np.pi * x / nx)
    out = []
    for _ in range(nsteps):
        if field == "shear":
            q = np.einsum("i,iyx->x", v[:, 1].astype(float), L.f)
        else:
            q = L.f.sum(axis=(0, 1))
            q = q / ny
        out.append((q * ph).sum())
        L.step(1)
    return np.array(out)


@pytest.mark.parametrize("L_side,tau", [(32, workloads.tau_vector(0.8, 0.8, 1.0)),
                                        (64, workloads.tau_vector(0.6, 1.0, 1.0))])
def test_shear_wave_decay(oracle_lib, L_side, tau):
    a = _wave_series(oracle_lib, L_side, tau, "shear", 120)
    ratio = (a[40:] / a[39:-1]).real
    lam = ratio.mean()
    assert ratio.std() < 1e-9
    k = 2 * np.pi / L_side
    exact, _, _ = lyapunov.exact_rates(k, tau)
    assert abs(lam - exact) < 1e-9
    hyd, _, _ = lyapunov.hydro_rates(k, tau[3], tau[5])
    # closed form holds up to O(k^4) in the exponent
    assert abs(np.log(lam) / np.log(hyd) - 1) < 0.2 * k * k + 1e-9


@pytest.mark.parametrize("L_side,tau", [(32, workloads.tau_vector(0.8, 0.8, 1.0)),
                                        (64, workloads.tau_vector(0.6, 1.0, 1.0))])
def test_sound_wave_frequency_and_damping(oracle_lib, L_side, tau):
    a = _wave_series(oracle_lib, L_side, tau, "sound", 260).real
    # a(t) = p lam^t + q conj(lam)^t  =>  a(t+2) = alpha a(t+1) + beta a(t)
    t0 = 60
    X = np.stack([a[t0 + 1:-1], a[t0:-2]], axis=1)
    y = a[t0 + 2:]
    (alpha, beta), *_ = np.linalg.lstsq(X, y, rcond=None)
    mod = np.sqrt(-beta)
    arg = np.arccos(alpha / (2 * mod))
    k = 2 * np.pi / L_side
    _, ex_mod, ex_arg = lyapunov.exact_rates(k, tau)
    assert abs(mod - ex_mod) < 1e-8
    assert abs(arg - ex_arg) < 1e-8
    _, h_mod, h_arg = lyapunov.hydro_rates(k, tau[3], tau[5])
    assert abs(np.log(mod) / np.log(h_mod) - 1) < 0.2 * k * k
    assert abs(arg / h_arg - 1) < 0.1 * k * k


def test_exact_linear_eigenvalues_at_the_first_mode():
    """Exact linear eigenvalues at k = 2 pi / 32 x, tau_s = tau_b = 0.8 (a
    number computed once, independently, by a numpy linearisation)."""
    sh, mod, arg = lyapunov.exact_rates(2 * np.pi / 32, workloads.tau_vector(0.8, 0.8, 1.0))
    assert abs(sh - 0.996150130495) < 1e-11
    assert abs(mod - 0.996147665812) < 1e-11
    assert abs(arg - 0.113306148571) < 1e-11


def test_staggered_momentum_flips(oracle_lib):
    L = oracle_lib.Lattice(12, 10, TAU_C1, theta=1e-3, u0=(0.03, 0.0), seed=4,
                           thermalize=True)
    prev = L.conservation()
    assert abs(prev[3]) > 1e-4 and abs(prev[4]) > 1e-4
    for _ in range(100):
        L.step(1)
        cur = L.conservation()
        assert abs(cur[3] + prev[3]) < 1e-13
        assert abs(cur[4] + prev[4]) < 1e-13
        prev = cur


def test_thermalize_keeps_totals_and_has_equilibrium_variance(oracle_lib):
    """Thermalised start: totals unchanged; per population the added
    deviations have variance mu rho0 w_i (the stationary covariance at linear
    order implied by Eq. 7) and no mean."""
    nx = ny = 128
    theta, rho0 = 1e-4, 1.0
    L = oracle_lib.Lattice(nx, ny, TAU_C1, theta=theta, rho0=rho0, seed=21)
    c0 = L.conservation()
    f0 = L.f.copy()
    L.thermalize()
    c1 = L.conservation()
    assert np.abs(c1[:3] - c0[:3]).max() < 1e-14 * nx * ny
    _, _, w, _ = oracle_lib.tables()
    d = (L.f - f0).reshape(9, -1)
    var = d.var(axis=1)
    expect = 3 * theta * rho0 * w
    assert np.all(np.abs(var / expect - 1) < 5 * np.sqrt(2 / d.shape[1]))
    assert np.abs(d.mean(axis=1)).max() < 1e-15
