"""Linear-response predictions for the other velocity sets (test pin).

Independent of the oracle and of the GPU library: the velocity sets, weights
and moment polynomials are written here, orthonormalised under the weights
with numpy (Eq. 4), and one step of Eq. (5) plus streaming (Eq. 1) is
linearised about the uniform state f^0(rho0, u0) of Eq. (2).  For every wave
vector the stationary covariance solves

    P(k) = A(k) P(k) A(k)^H + E(k) Q E(k)^H

exactly as for D2Q9 (``lyapunov.py``).  Wave vectors where A(k) keeps an
eigenvalue of modulus one (k = 0 and the lattice's staggered invariants) are
reported as NaN.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

CS2 = 1.0 / 3.0


def velocity_set(model):
    if model == "D1Q3":
        v = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0]], dtype=float)
        w = np.array([2 / 3, 1 / 6, 1 / 6])
        return 1, v, w
    if model == "D2Q9":
        v = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
                      (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)], dtype=float)
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        return 2, v, w
    if model == "D3Q15":
        v = [(0, 0, 0)]
        for a in range(3):
            for s in (1, -1):
                e = [0, 0, 0]
                e[a] = s
                v.append(tuple(e))
        for c in range(8):
            v.append(tuple(-1 if (c >> b) & 1 else 1 for b in range(3)))
        w = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)
        return 3, np.array(v, dtype=float), w
    raise ValueError(model)


def polynomials(D, v):
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    v2 = x * x + y * y + z * z
    one = np.ones(len(v))
    if D == 1:
        return [one, x, x * x - 1 / 3]
    if D == 2:
        return [one, x, y, x * x - y * y, x * y, v2 - 2 / 3, x * v2, y * v2, v2 * v2]
    return [one, x, y, z, 3 * x * x - v2, y * y - z * z, x * y, y * z, z * x, v2 - 1,
            x * v2, y * v2, z * v2, x * y * z, v2 * v2]


def basis(model):
    """(D, v, w, m) with m[a] the a-th polynomial orthonormalised (numpy QR
    in the weighted inner product)."""
    D, v, w = velocity_set(model)
    P = np.array(polynomials(D, v))  # (Q, Q): rows = polynomials at the velocities
    sw = np.sqrt(w)
    # weighted Gram-Schmidt == QR of (P * sqrt(w))^T
    q, r = np.linalg.qr((P * sw).T)
    q = q * np.sign(np.diag(r))  # positive leading coefficients
    m = (q / sw[:, None]).T
    return D, v, w, m


def _meq(M, D, m, v, w):
    """Equilibrium moments (moments of Eq. 2) from the conserved moments."""
    rho = M[0]
    u = np.zeros(3, dtype=M.dtype)
    for a in range(D):
        u[a] = M[1 + a] / np.sqrt(3.0) / rho
    vu = v @ u
    f0 = w * rho * (1 + 3 * vu + 4.5 * vu * vu - 1.5 * (u @ u))
    return m @ f0


def collision_matrix(model, tau, rho0=1.0, u0=(0.0, 0.0, 0.0)):
    D, v, w, m = basis(model)
    Q = len(w)
    u0 = np.array(list(u0) + [0.0] * (3 - len(u0)))
    vu = v @ u0
    fbar = rho0 * w * (1 + 3 * vu + 4.5 * vu * vu - 1.5 * (u0 @ u0))
    Mbar = m @ fbar
    G = np.zeros((Q, Q))
    h = 1e-30
    for b in range(Q):
        Mc = Mbar.astype(complex)
        Mc[b] += 1j * h
        G[:, b] = np.imag(_meq(Mc, D, m, v, w)) / h
    omega = np.array([0.0] * (D + 1) + [1.0 / tau[a] for a in range(D + 1, Q)])
    Dm = np.eye(Q) - np.diag(omega) @ (np.eye(Q) - G)
    nmat = w[:, None] * m.T
    return nmat @ Dm @ m


def noise_cov(model, tau, theta, rho0=1.0, ladd=False):
    D, v, w, m = basis(model)
    Q = len(w)
    first_ghost = 1 + D + D * (D + 1) // 2
    mu = theta / CS2
    s2 = np.zeros(Q)
    for a in range(D + 1, Q):
        if ladd and a >= first_ghost:
            continue
        s2[a] = mu * rho0 * (2 * tau[a] - 1) / tau[a] ** 2
    nmat = w[:, None] * m.T
    return nmat @ np.diag(s2) @ nmat.T


def predict(model, sides, tau, theta, rho0=1.0, u0=(0.0, 0.0, 0.0), ladd=False):
    """Normalised structure factors on the (nz, ny, nx//2+1) half space with
    the keys of the oracle's ``dq_normalized``."""
    D, v, w, m = basis(model)
    Q = len(w)
    sides = list(sides) + [1] * (3 - len(sides))
    nx, ny, nz = sides
    nh = nx // 2 + 1
    u0 = np.array(list(u0) + [0.0] * (3 - len(u0)))
    mu = theta / CS2
    C = collision_matrix(model, tau, rho0, u0)
    Qn = noise_cov(model, tau, theta, rho0, ladd)
    ax = "xyz"
    keys = ["S_rho"] + ["S_j" + ax[a] for a in range(D)] + ["S_u" + ax[a] for a in range(D)]
    keys += ["S_M%d" % a for a in range(D + 1, Q)]
    if D >= 2:
        keys.append("R_uxuy")
    out = {k: np.full((nz, ny, nh), np.nan, dtype=complex) for k in keys}
    one = np.ones(Q)
    lj = [v[:, a] for a in range(D)]
    lu = [(v[:, a] - u0[a]) / rho0 for a in range(D)]
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nh):
                k = 2 * np.pi * np.array([kx / nx, ky / ny, kz / nz])
                E = np.diag(np.exp(-1j * (v @ k)))
                A = E @ C
                if np.abs(np.linalg.eigvals(A)).max() > 1 - 1e-9:
                    continue
                P = scipy.linalg.solve_discrete_lyapunov(A, E @ Qn @ E.conj().T)
                o = (kz, ky, kx)
                out["S_rho"][o] = (one @ P @ one) / (mu * rho0)
                for a in range(D):
                    out["S_j" + ax[a]][o] = (lj[a] @ P @ lj[a]) / (rho0 * theta)
                    out["S_u" + ax[a]][o] = rho0 * (lu[a] @ P @ lu[a]) / theta
                if D >= 2:
                    out["R_uxuy"][o] = rho0 * (lu[0] @ P @ lu[1]) / theta
                for a in range(D + 1, Q):
                    out["S_M%d" % a][o] = (m[a] @ P @ m[a]) / (mu * rho0)
    for key in keys:
        if key.startswith("S_"):
            out[key] = out[key].real
    return out
