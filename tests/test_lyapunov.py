"""Pins of the linear-response predictor against the paper's statements.

* Eq. (7): with noise on all non-conserved modes and u0 = 0 every S_k is 1 and
  every cross correlator 0 (the stationary covariance is mu rho0 diag(w)).
* Sec. 3, without ghost noise (tau^a = 1, V = 20^2): S_k(rho) is exact on the
  k_x = 0 and k_y = 0 axes (the D1Q3 projection argument), S_k(u_x) is white
  along the k_x axis, and R_k(u_x, u_y) reaches "up to 0.25 rho" at
  intermediate k.
* Fig. 4 discussion: at u_x = 0.1 the ghost-noise scheme's cross correlator is
  non-zero but smaller than the scheme without ghost noise.
"""
import numpy as np
import pytest

import lyapunov
from paper_1010_1233_amd import workloads


def _mask(nx, ny):
    nh = nx // 2 + 1
    m = np.ones((ny, nh), dtype=bool)
    for ky in range(ny):
        for kx in range(nh):
            m[ky, kx] = not lyapunov.singular_k(nx, ny, kx, ky)
    return m


@pytest.mark.parametrize("n,tau", [(20, workloads.tau_vector(1, 1, 1)),
                                   (16, workloads.tau_vector(0.8, 0.8, 1.0)),
                                   (15, workloads.tau_vector(0.55, 1.4, 0.7))])
def test_decoupling_at_rest_is_exact(n, tau):
    p = lyapunov.predict(n, n, tau, 1e-4)
    m = _mask(n, n)
    for k, v in p.items():
        exp = 1.0 if k.startswith("S_") else 0.0
        assert np.abs(v[m] - exp).max() < 1e-12, k


def test_ladd_scheme_statements():
    n = 20
    p = lyapunov.predict(n, n, workloads.tau_vector(1, 1, 1), 1e-4, ladd=True)
    S = p["S_rho"]
    # no deficiency on the axes
    assert np.nanmax(np.abs(S[0, 1:] - 1)) < 1e-12
    assert np.nanmax(np.abs(S[1:, 0] - 1)) < 1e-12
    # drastic deficiency at large k
    assert np.nanmin(S) < 0.3
    # S(u_x) white along the k_x axis
    assert np.nanmax(np.abs(p["S_ux"][0, 1:] - 1)) < 1e-12
    # R(u_x, u_y) up to ~0.25 rho at intermediate k
    R = p["R_uxuy"].real
    assert 0.22 < np.nanmax(np.abs(R)) < 0.30
    ky, kx = np.unravel_index(np.nanargmax(np.abs(R)), R.shape)
    assert 0 < kx < n // 2 and ky not in (0, n // 2)
    assert abs(abs(R[ky, kx]) - 0.2616916331750091) < 1e-9


def test_mean_flow_errors_smaller_than_ladd():
    n = 20
    tau = workloads.tau_vector(1, 1, 1)
    g = lyapunov.predict(n, n, tau, 1e-4, u0=(0.1, 0.0))
    l0 = lyapunov.predict(n, n, tau, 1e-4, ladd=True)
    gmax = np.nanmax(np.abs(g["R_uxuy"]))
    assert 1e-3 < gmax < 0.5 * np.nanmax(np.abs(l0["R_uxuy"]))
    assert np.nanmax(np.abs(g["S_rho"] - 1)) > 1e-2


def test_gi_deviation_grows_with_velocity():
    n = 16
    tau = workloads.tau_vector(0.8, 1.0, 1.0)
    prev = 0.0
    for u in workloads.GI_VELOCITIES[1:]:
        p = lyapunov.predict(n, n, tau, 1e-4, u0=(u, 0.0))
        d = np.nanmax(np.abs(p["R_rhoux"]))
        assert d > prev
        prev = d


def test_transient_approaches_stationary():
    n = 8
    tau = workloads.tau_vector(0.8, 0.8, 1.0)
    tr = lyapunov.transient(n, n, tau, 1e-4, times=[3000])
    m = _mask(n, n)
    assert np.abs(tr["S_rho"][m] - 1).max() < 1e-6
    early = lyapunov.transient(n, n, tau, 1e-4, times=[5])
    assert early["S_rho"][m].min() < 0.9


def test_hydrodynamic_limit_of_exact_rates():
    tau = workloads.tau_vector(0.7, 1.1, 1.0)
    errs = []
    for L in (32, 64, 128):
        k = 2 * np.pi / L
        sh, mod, arg = lyapunov.exact_rates(k, tau)
        hs, hm, ha = lyapunov.hydro_rates(k, tau[3], tau[5])
        errs.append(abs(np.log(sh) / np.log(hs) - 1))
        assert abs(np.log(mod) / np.log(hm) - 1) < 0.3 * k * k
        assert abs(arg / ha - 1) < 0.1 * k * k
    assert errs[2] < errs[1] < errs[0]
