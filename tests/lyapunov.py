"""Linear-response predictions for the fluctuating D2Q9 scheme (test pin).

This module is independent of the oracle and of the GPU library: it builds the
D2Q9 moment basis from the Hermite-polynomial forms of the rows of Eq. (9)
(not from the printed table), linearises one step of Eq. (5) plus streaming
(Eq. 1) about the uniform state f^0(rho0, u0) of Eq. (2), and solves, for every
wave vector k, the stationary discrete Lyapunov equation

    P(k) = A(k) P(k) A(k)^H + E(k) Q E(k)^H,   A(k) = E(k) N [I - Omega (I - G)] M,

with E(k) = diag(exp(-i k.v_i)) the streaming phase, Omega = diag(1/tau^a) on
the non-conserved modes, G = d M^{a,0} / d M^b the Jacobian of the equilibrium
moments (Eq. 10), and Q = N diag(sigma_a^2) N^T the per-site noise covariance
of Eq. (8) (the noise is added before streaming, hence the phases on Q).
P(k) is the per-volume covariance of the populations' Fourier
amplitudes, from which every correlator of Eq. (11)/(12) follows at linear
order in the noise.  At u0 = 0 the exact answer is P = mu rho0 diag(w) (Eq. 7),
i.e. S = 1 and vanishing cross correlators for every k; with the ghost noise
removed (the older scheme) or at u0 != 0 it gives the finite-k deviations the
paper discusses.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

CS2 = 1.0 / 3.0


def basis():
    """Velocities v[i], weights w[i] and m[a][i] from the polynomial forms."""
    v = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                  (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    vx, vy = v[:, 0], v[:, 1]
    v2 = vx * vx + vy * vy
    m = np.array([
        np.ones(9),
        np.sqrt(3.0) * vx,
        np.sqrt(3.0) * vy,
        1.5 * (vx * vx - vy * vy),
        3.0 * vx * vy,
        1.5 * v2 - 1.0,
        np.sqrt(1.5) * vx * (3.0 * v2 - 4.0),
        np.sqrt(1.5) * vy * (3.0 * v2 - 4.0),
        (9.0 * v2 * v2 - 15.0 * v2 + 2.0) / 4.0,
    ])
    return v, w, m


def _meq(Mv):
    """Equilibrium moments as a function of (M^0, M^1, M^2): Eq. (10)."""
    rho = Mv[0]
    jx = Mv[1] / np.sqrt(3.0)
    jy = Mv[2] / np.sqrt(3.0)
    ux, uy = jx / rho, jy / rho
    z = 0.0 * rho
    return np.array([rho, np.sqrt(3.0) * rho * ux, np.sqrt(3.0) * rho * uy,
                     1.5 * rho * (ux * ux - uy * uy), 3.0 * rho * ux * uy,
                     1.5 * rho * (ux * ux + uy * uy), z, z, z])


def collision_matrix(tau, rho0=1.0, u0=(0.0, 0.0)):
    """C = N [I - Omega (I - G)] M: linearised collision in population space."""
    v, w, m = basis()
    nmat = (w[:, None] * m.T)  # n[i][a]
    fbar = rho0 * w * (1 + 3 * (v @ u0) + 4.5 * (v @ u0) ** 2 - 1.5 * np.dot(u0, u0))
    Mbar = m @ fbar
    # Jacobian of Eq. (10) with respect to the moments, by complex-step
    # differentiation (exact to rounding for this analytic function).
    G = np.zeros((9, 9))
    h = 1e-30
    for b in range(9):
        Mc = Mbar.astype(complex)
        Mc[b] += 1j * h
        G[:, b] = np.imag(_meq(Mc)) / h
    omega = np.array([0.0, 0.0, 0.0] + [1.0 / tau[a] for a in range(3, 9)])
    D = np.eye(9) - np.diag(omega) @ (np.eye(9) - G)
    return nmat @ D @ m


def noise_cov(tau, theta, rho0=1.0, ladd=False):
    """Q = N diag(sigma^2) N^T, sigma_a^2 = mu rho0 (2 tau^a - 1) / tau^a^2."""
    v, w, m = basis()
    nmat = (w[:, None] * m.T)
    mu = theta / CS2
    s2 = np.zeros(9)
    for a in range(3, 9):
        if ladd and a >= 6:
            continue
        s2[a] = mu * rho0 * (2.0 * tau[a] - 1.0) / tau[a] ** 2
    return nmat @ np.diag(s2) @ nmat.T


def step_operator(k, tau, rho0=1.0, u0=(0.0, 0.0)):
    """A(k) = E(k) C for the wave vector k = (kx, ky) in radians per site."""
    v, _, _ = basis()
    E = np.diag(np.exp(-1j * (v @ np.asarray(k, dtype=float))))
    return E @ collision_matrix(tau, rho0, np.asarray(u0, dtype=float))


def _functionals(rho0, u0):
    v, _, _ = basis()
    one = np.ones(9)
    lx, ly = v[:, 0], v[:, 1]
    ux = (lx - u0[0] * one) / rho0
    uy = (ly - u0[1] * one) / rho0
    return one, lx, ly, ux, uy


def singular_k(nx, ny, kx_i, ky_i):
    """Wave vectors where A(k) has a unit-modulus eigenvalue: k = 0 (mass and
    momentum) and, for even sides, the staggered momenta (pi, 0) / (0, pi)."""
    if kx_i == 0 and ky_i == 0:
        return True
    if nx % 2 == 0 and kx_i == nx // 2 and ky_i == 0:
        return True
    if ny % 2 == 0 and ky_i == ny // 2 and kx_i == 0:
        return True
    return False


def predict(nx, ny, tau, theta, rho0=1.0, u0=(0.0, 0.0), ladd=False):
    """Stationary normalised correlators on the (ny, nx//2+1) half plane.

    Returns a dict with the same keys and normalisation as the oracle's
    ``normalized`` (plus S_M3..S_M8, the structure factors of the
    non-conserved moments, normalised by mu rho0); singular k carry NaN.
    """
    u0 = np.asarray(u0, dtype=float)
    nh = nx // 2 + 1
    mu = theta / CS2
    cs = np.sqrt(CS2)
    C = collision_matrix(tau, rho0, u0)
    Q = noise_cov(tau, theta, rho0, ladd)
    v, _, _ = basis()
    one, lx, ly, lux, luy = _functionals(rho0, u0)
    _, _, mb = basis()
    keys = ["S_rho", "S_jx", "S_jy", "S_ux", "S_uy", "R_uxuy", "R_rhojx", "R_rhojy",
            "R_rhoux", "R_rhouy"] + ["S_M%d" % a for a in range(3, 9)]
    out = {k: np.full((ny, nh), np.nan, dtype=complex) for k in keys}
    for ky_i in range(ny):
        for kx_i in range(nh):
            if singular_k(nx, ny, kx_i, ky_i):
                continue
            k = np.array([2 * np.pi * kx_i / nx, 2 * np.pi * ky_i / ny])
            E = np.diag(np.exp(-1j * (v @ k)))
            A = E @ C
            P = scipy.linalg.solve_discrete_lyapunov(A, E @ Q @ E.conj().T)

            def c(a, b):
                return a @ P @ b

            out["S_rho"][ky_i, kx_i] = c(one, one) / (mu * rho0)
            out["S_jx"][ky_i, kx_i] = c(lx, lx) / (rho0 * theta)
            out["S_jy"][ky_i, kx_i] = c(ly, ly) / (rho0 * theta)
            out["S_ux"][ky_i, kx_i] = rho0 * c(lux, lux) / theta
            out["S_uy"][ky_i, kx_i] = rho0 * c(luy, luy) / theta
            out["R_uxuy"][ky_i, kx_i] = rho0 * c(lux, luy) / theta
            out["R_rhojx"][ky_i, kx_i] = c(one, lx) / (mu * rho0 * cs)
            out["R_rhojy"][ky_i, kx_i] = c(one, ly) / (mu * rho0 * cs)
            out["R_rhoux"][ky_i, kx_i] = c(one, lux) / (mu * cs)
            out["R_rhouy"][ky_i, kx_i] = c(one, luy) / (mu * cs)
            for a in range(3, 9):
                out["S_M%d" % a][ky_i, kx_i] = c(mb[a], mb[a]) / (mu * rho0)
    for k in keys:
        if k.startswith("S_"):
            out[k] = out[k].real
    return out


def transient(nx, ny, tau, theta, times, rho0=1.0, u0=(0.0, 0.0), ladd=False, P0=None):
    """Expected estimator of S(rho) and S(u_x) averaged over sampling `times`
    from a uniform start (P_0 = 0): P_t = A P_{t-1} A^H + E Q E^H, per k."""
    u0 = np.asarray(u0, dtype=float)
    nh = nx // 2 + 1
    mu = theta / CS2
    C = collision_matrix(tau, rho0, u0)
    Q = noise_cov(tau, theta, rho0, ladd)
    v, _, _ = basis()
    one, lx, ly, lux, luy = _functionals(rho0, u0)
    times = sorted(int(t) for t in times)
    s_rho = np.zeros((ny, nh))
    s_ux = np.zeros((ny, nh))
    for ky_i in range(ny):
        for kx_i in range(nh):
            k = np.array([2 * np.pi * kx_i / nx, 2 * np.pi * ky_i / ny])
            E = np.diag(np.exp(-1j * (v @ k)))
            A = E @ C
            Qk = E @ Q @ E.conj().T
            P = np.zeros((9, 9), dtype=complex) if P0 is None else P0.astype(complex)
            t = 0
            acc_r = acc_u = 0.0
            for ts in times:
                while t < ts:
                    P = A @ P @ A.conj().T + Qk
                    t += 1
                acc_r += (one @ P @ one).real
                acc_u += (lux @ P @ lux).real
            s_rho[ky_i, kx_i] = acc_r / len(times) / (mu * rho0)
            s_ux[ky_i, kx_i] = rho0 * acc_u / len(times) / theta
    return {"S_rho": s_rho, "S_ux": s_ux}


def hydro_rates(k, tau_shear, tau_bulk):
    """Long-wavelength closed forms (isothermal, c_s^2 = 1/3):
    shear decay exp(-nu k^2), nu = (tau_s - 1/2)/3; sound exp(-Gamma k^2 +-
    i c_s k), Gamma = [(tau_s - 1/2) + (tau_b - 1/2)]/6."""
    nu = (tau_shear - 0.5) / 3.0
    gam = ((tau_shear - 0.5) + (tau_bulk - 0.5)) / 6.0
    return np.exp(-nu * k * k), np.exp(-gam * k * k), np.sqrt(CS2) * k


def exact_rates(k, tau):
    """Eigenvalues of A(k) for k along x: (shear lambda, |sound lambda|,
    arg sound lambda), picked as the eigenvalues nearest the hydrodynamic
    forms."""
    A = step_operator((k, 0.0), tau)
    ev = np.linalg.eigvals(A)
    hs, hm, hp = hydro_rates(k, tau[3], tau[5])
    shear = ev[np.argmin(np.abs(ev - hs))]
    sound = ev[np.argmin(np.abs(ev - hm * np.exp(-1j * hp)))]
    return shear.real, abs(sound), -np.angle(sound)
