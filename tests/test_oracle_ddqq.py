"""Pins of the generic oracle for the other velocity sets (the paper reports
D1Q3 and D3Q15 results similar to D2Q9, Sec. 3).

* Tables: weights isotropic to fourth order with c_s^2 = 1/3; the moments
  orthonormal under the weights (Eq. 4); they equal an independent numpy
  construction, the printed D2Q9 rows (Eq. 9, via the Hermite forms) and the
  closed-form D1Q3 rows; D3Q15's stress rows are second-order polynomials and
  its ghost rows are orthogonal to every polynomial of degree <= 2.
* Dynamics: generic D2Q9 equals the D2Q9 oracle step for step; exact mass and
  momentum conservation; the uniform equilibrium is a fixed point without
  noise; D3Q15 shear waves decay at the rate of the linearised operator and
  at nu = (tau_s - 1/2)/3 for small k.
* Transform: the 3-D DFT equals numpy's.
* Statistics: S = 1 for every kind at rest with noise on all modes (D1Q3,
  D3Q15), and the predicted deficits without ghost noise (D3Q15).
"""
import itertools

import numpy as np
import pytest

import lyapunov
import lyapunov_dq

MODELS = ("D1Q3", "D2Q9", "D3Q15")


@pytest.mark.parametrize("model", MODELS)
def test_weights_isotropic(oracle_lib, model):
    D, v, w, _ = oracle_lib.dq_tables(model)
    assert abs(w.sum() - 1) < 1e-15
    for a in range(3):
        assert abs((w * v[:, a]).sum()) < 1e-15
        for b in range(3):
            exp = 1 / 3 if (a == b and a < D) else 0.0
            assert abs((w * v[:, a] * v[:, b]).sum() - exp) < 1e-15
    for a, b, c, d in itertools.product(range(D), repeat=4):
        exp = ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c)) / 9.0
        assert abs((w * v[:, a] * v[:, b] * v[:, c] * v[:, d]).sum() - exp) < 1e-15


@pytest.mark.parametrize("model", MODELS)
def test_moments_orthonormal_and_independent_construction(oracle_lib, model):
    D, v, w, m = oracle_lib.dq_tables(model)
    Q = len(w)
    assert np.abs((m * w) @ m.T - np.eye(Q)).max() < 1e-14
    _, vq, wq, mq = lyapunov_dq.basis(model)
    assert np.array_equal(v, vq.astype(int)) and np.abs(w - wq).max() < 1e-16
    assert np.abs(m - mq).max() < 1e-13
    # conserved rows: 1 and sqrt(3) v_a
    assert np.abs(m[0] - 1).max() < 1e-15
    for a in range(D):
        assert np.abs(m[1 + a] - np.sqrt(3) * v[:, a]).max() < 1e-14


def test_d2q9_rows_are_eq9(oracle_lib):
    _, _, _, m = oracle_lib.dq_tables("D2Q9")
    _, _, mh = lyapunov.basis()  # the Hermite-polynomial forms of Eq. (9)
    assert np.abs(m - mh).max() < 1e-14


def test_d1q3_rows_closed_form(oracle_lib):
    _, v, _, m = oracle_lib.dq_tables("D1Q3")
    x = v[:, 0]
    assert np.abs(m[2] - (3 * x * x - 1) / np.sqrt(2)).max() < 1e-15


def test_d3q15_stress_and_ghost_structure(oracle_lib):
    D, v, w, m = oracle_lib.dq_tables("D3Q15")
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    low = np.array([np.ones(15), x, y, z, x * x, y * y, z * z, x * y, y * z, z * x]).T
    for a in range(4, 10):  # stress rows: exactly degree-2 polynomials
        coef, res, *_ = np.linalg.lstsq(low, m[a], rcond=None)
        assert np.abs(low @ coef - m[a]).max() < 1e-13
    for a in range(10, 15):  # ghost rows: orthogonal to every degree <= 2 polynomial
        assert np.abs((w * m[a]) @ low).max() < 1e-14


@pytest.mark.parametrize("model", MODELS)
def test_equilibrium_moments_closed_form(oracle_lib, model):
    """Eq. (2): sum f0 = rho, sum f0 v = rho u, sum f0 v v = rho (c_s^2 1 + u u)."""
    D, v, w, _ = oracle_lib.dq_tables(model)
    rho, u = 1.07, np.array([0.06, -0.04, 0.03])[:D]
    f0 = oracle_lib.dq_equilibrium(model, rho, u)
    uu = np.zeros(3)
    uu[:D] = u
    assert abs(f0.sum() - rho) < 1e-15
    assert np.abs(v.T @ f0 - rho * uu).max() < 1e-15
    P = (v.T * f0) @ v
    exp = rho * (np.diag([1 / 3 if a < D else 0 for a in range(3)]) + np.outer(uu, uu))
    assert np.abs(P - exp).max() < 1e-15


@pytest.mark.parametrize("model,sides,k0", [("D1Q3", (16,), (3, 0, 0)),
                                            ("D2Q9", (12, 10), (2, 3, 0)),
                                            ("D3Q15", (6, 5, 4), (1, 2, 3))])
def test_one_step_equals_linear_operator(oracle_lib, model, sides, k0):
    """A small single-k perturbation of the uniform state at u0 != 0 evolves
    in one noise-free step by the linearised operator A(k) = E(k) C of the
    independent predictor (streaming direction, relaxation per moment and the
    Jacobian of Eq. 10 at u0, quadratic terms included)."""
    D, v, w, m = oracle_lib.dq_tables(model)
    Q = len(w)
    rng = np.random.default_rng(17)
    tau = [1.0] * (D + 1) + list(rng.uniform(0.6, 1.6, Q - D - 1))
    u0 = [0.05, -0.03, 0.02][:D]
    L = oracle_lib.DqLattice(model, sides, tau, 0.0, u0=u0)
    nx, ny, nz = L.sides
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx]
    k = 2 * np.pi * np.array([k0[0] / nx, k0[1] / ny, k0[2] / nz])
    ph = np.exp(1j * (k[0] * xx + k[1] * yy + k[2] * zz))
    c = (rng.normal(size=Q) + 1j * rng.normal(size=Q)) * 1e-7
    fbar = L.f.copy()
    L.set_populations(fbar + np.real(c[:, None, None, None] * ph))
    L.step(1)
    V = nx * ny * nz
    F = 2.0 / V * ((L.f - fbar) * np.conj(ph)).sum(axis=(1, 2, 3))
    C = lyapunov_dq.collision_matrix(model, tau, 1.0, u0 + [0.0] * (3 - D))
    E = np.diag(np.exp(-1j * (v @ k)))
    assert np.abs(F - E @ C @ c).max() < 1e-6 * np.abs(c).max()


def test_generic_d2q9_equals_d2q9_oracle(oracle_lib):
    tau = [1, 1, 1, 0.7, 0.8, 0.9, 1.1, 1.2, 1.3]
    for ladd in (False, True):
        a = oracle_lib.Lattice(10, 7, tau, 1e-3, u0=(0.04, 0.02), seed=3, stream_id=2, ladd=ladd)
        b = oracle_lib.DqLattice("D2Q9", (10, 7), tau, 1e-3, u0=(0.04, 0.02), seed=3,
                                 stream_id=2, ladd=ladd)
        a.thermalize()
        b.thermalize()
        assert np.abs(a.f - b.f[:, 0]).max() == 0.0
        a.step(30)
        b.step(30)
        assert np.abs(a.f - b.f[:, 0]).max() < 1e-13
        a.sample()
        b.sample()
        # shared kinds: rho, jx, jy, ux, uy, Re/Im ux uy*
        ga = a.acc[[0, 1, 2, 3, 4, 5, 6]]
        gb = b.acc[[0, 1, 2, 3, 4, 5, 6], 0]
        assert np.abs(ga - gb).max() < 1e-12 * np.abs(ga).max()


@pytest.mark.parametrize("model,sides", [("D1Q3", (17,)), ("D3Q15", (5, 4, 3))])
def test_conservation_and_fixed_point(oracle_lib, model, sides):
    rng = np.random.default_rng(5)
    D, _, w, _ = oracle_lib.dq_tables(model)
    Q = len(w)
    tau = [1.0] * (D + 1) + list(np.linspace(0.6, 1.4, Q - D - 1))
    L = oracle_lib.DqLattice(model, sides, tau, 1e-3, u0=(0.03, -0.02, 0.01)[:D], seed=9)
    L.set_populations(L.f + rng.normal(0, 0.003, L.f.shape))
    c0 = L.conservation()
    L.step(25)
    assert np.abs(L.conservation() - c0).max() < 1e-12 * L.f[0].size
    # without noise the uniform equilibrium at u0 != 0 does not move
    E = oracle_lib.DqLattice(model, sides, tau, 0.0, u0=(0.03, -0.02, 0.01)[:D], seed=9)
    f0 = E.f.copy()
    E.step(10)
    assert np.abs(E.f - f0).max() < 1e-14


def test_d3q15_shear_wave_decay(oracle_lib):
    """u_y(x) = A sin(k x) without noise: the decay per step equals the
    eigenvalue of the linearised step operator of that k (exact up to O(A^2))
    and tends to exp(-nu k^2), nu = (tau_s - 1/2)/3."""
    nx = 32
    tau_s = 0.8
    tau = [1.0] * 4 + [tau_s] * 5 + [1.0] + [1.1] * 5
    D, v, w, m = oracle_lib.dq_tables("D3Q15")
    L = oracle_lib.DqLattice("D3Q15", (nx, 1, 1), tau, 0.0)
    A = 1e-6
    x = np.arange(nx)
    kk = 2 * np.pi / nx
    uy = A * np.sin(kk * x)
    f = np.zeros((15, 1, 1, nx))
    for i in range(15):
        vu = v[i, 1] * uy
        f[i, 0, 0] = w[i] * (1 + 3 * vu + 4.5 * vu * vu - 1.5 * uy * uy)
    L.set_populations(f)

    def amp():
        j = np.tensordot(v[:, 1], L.f[:, 0, 0], axes=1)
        return 2 * np.abs(np.fft.fft(j)[1]) / nx

    L.step(20)
    a0 = amp()
    L.step(40)
    rate = (amp() / a0) ** (1 / 40)
    C = lyapunov_dq.collision_matrix("D3Q15", tau)
    E = np.diag(np.exp(-1j * (v @ np.array([kk, 0, 0]))))
    ev = np.linalg.eigvals(E @ C)
    shear = ev[np.argmin(np.abs(ev - np.exp(-(tau_s - 0.5) / 3 * kk * kk)))]
    assert abs(rate - abs(shear)) < 1e-9
    assert abs(rate - np.exp(-(tau_s - 0.5) / 3 * kk * kk)) < 0.02 * kk * kk


@pytest.mark.parametrize("shape", [(8, 4, 2), (5, 3, 6), (1, 1, 12), (16, 1, 1)])
def test_dft3_matches_numpy(oracle_lib, shape):
    rng = np.random.default_rng(1)
    nx, ny, nz = shape
    a = rng.normal(size=(nz, ny, nx)) + 1j * rng.normal(size=(nz, ny, nx))
    assert np.abs(oracle_lib.dft3(a) - np.fft.fftn(a)).max() < 1e-12


def test_plane_wave_lands_on_its_kind(oracle_lib):
    """A wave in one non-conserved moment of D3Q15 lands on its own kind at
    its own k with (c V / 2)^2 and nowhere else (k = 0 included)."""
    D, v, w, m = oracle_lib.dq_tables("D3Q15")
    nx, ny, nz = 6, 4, 5
    L = oracle_lib.DqLattice("D3Q15", (nx, ny, nz), [1.0] * 15, 1e-4)
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx]
    k0 = (2, 1, 3)
    wave = np.cos(2 * np.pi * (k0[0] * xx / nx + k0[1] * yy / ny + k0[2] * zz / nz) + 0.3)
    V = nx * ny * nz
    names = oracle_lib.dq_kind_names(D, 15)
    for a in (4, 9, 13):
        c = 1e-3 * (a + 1)
        f = w[:, None, None, None] * (1.0 + c * m[a][:, None, None, None] * wave + 2e-3 * m[a][:, None, None, None])
        L.acc[...] = 0
        L.set_populations(f)
        L.sample()
        kind = names.index("M%d_M%d" % (a, a))
        exp = np.zeros_like(L.acc)
        exp[kind, k0[2], k0[1], k0[0]] = (c * V / 2) ** 2
        assert np.abs(L.acc - exp).max() < 1e-12 * exp.max()


def _mask(pred):
    return ~np.isnan(pred["S_rho"])


def _stat_check(oracle_lib, model, sides, tau, ladd, nblocks, steps, every, seed, theta=1e-4):
    D, _, w, _ = oracle_lib.dq_tables(model)
    Q = len(w)
    L = oracle_lib.DqLattice(model, sides, tau, theta, seed=seed, ladd=ladd, thermalize=True)
    L.run(200)
    blocks = []
    for _ in range(nblocks):
        L.acc[...] = 0
        L.nsamples = 0
        L.run(steps, every)
        blocks.append(oracle_lib.dq_normalized(L.acc, L.nsamples, D, Q, L.sides, theta, 1.0))
    pred = lyapunov_dq.predict(model, sides, tau, theta, ladd=ladd)
    mask = _mask(pred)
    zs = []
    for k in blocks[0]:
        a = np.stack([b[k] for b in blocks])
        for part in (np.real, np.imag) if np.iscomplexobj(a) else (np.real,):
            x = part(a)
            d = x.mean(0)[mask] - part(pred[k])[mask]
            s = (x.std(0, ddof=1) / np.sqrt(nblocks))[mask]
            ok = s > 1e-8
            assert np.all(np.abs(d[~ok]) < 1e-6 + 9 * theta)
            d = np.sign(d[ok]) * np.maximum(np.abs(d[ok]) - 9 * theta, 0)
            z = d / s[ok]
            assert np.abs(z).max() < 6.0, (k, np.abs(z).max())
            zs.append(z)
    chi = (np.concatenate(zs) ** 2).mean()
    assert chi < 1.7, chi
    return pred, blocks


def test_d1q3_structure_factors_are_one(oracle_lib):
    _stat_check(oracle_lib, "D1Q3", (32,), [1, 1, 0.8], False, 16, 4000, 2, seed=21)


def test_d3q15_structure_factors_are_one(oracle_lib):
    tau = [1.0] * 4 + [0.8] * 5 + [0.9] + [1.2] * 5
    pred, _ = _stat_check(oracle_lib, "D3Q15", (4, 4, 4), tau, False, 12, 600, 2, seed=22)
    for k, p in pred.items():
        exp = 0.0 if k.startswith("R_") else 1.0
        assert np.nanmax(np.abs(p - exp)) < 1e-12


def test_d3q15_without_ghost_noise_matches_linear_response(oracle_lib):
    tau = [1.0] * 15
    pred, blocks = _stat_check(oracle_lib, "D3Q15", (4, 4, 4), tau, True, 12, 600, 2, seed=23)
    m = _mask(pred)
    ghost = np.mean([np.stack([b["S_M%d" % a] for b in blocks]).mean(0)[m].mean()
                     for a in range(10, 15)])
    assert ghost < 0.7  # the ghost modes are far from equipartition
