"""Oracle pins for the D2Q9 lattice and the moment transform (Sec. 3, Eqs. 2-4, 9-10).

Each test checks the oracle's tables or single-site arithmetic against a
property the paper states or that the mathematics fixes, not against a copy
of the oracle's own formula.
"""
import numpy as np
import pytest

import lyapunov


def test_weights_and_isotropy(oracle_lib):
    """Weights (Sec. 3, with the fourth 1/9 restored): they sum to one, have
    zero first moment and second moment c_s^2 = k_B T = 1/3 (Sec. 3)."""
    m, n, w, v = oracle_lib.tables()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ v, 0.0, atol=1e-16)
    second = np.einsum("i,ia,ib->ab", w, v.astype(float), v.astype(float))
    assert np.allclose(second, np.eye(2) / 3.0, atol=1e-15)
    # the velocity order of Sec. 3
    assert v.tolist() == [[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                          [1, 1], [-1, 1], [-1, -1], [1, -1]]


def test_hermite_orthonormality(oracle_lib):
    """Eq. (4): sum_i w_i m_i^a m_i^b = sum_i m_i^a n_i^b = delta^ab."""
    m, n, w, _ = oracle_lib.tables()
    assert np.abs(m @ np.diag(w) @ m.T - np.eye(9)).max() < 1e-15
    assert np.abs(m @ n - np.eye(9)).max() < 1e-15
    assert np.abs(n - (w[:, None] * m.T)).max() == 0.0


def test_table_matches_hermite_polynomials(oracle_lib):
    """The printed rows of Eq. (9) are Hermite polynomials of v: build them
    from the polynomial forms and compare with the oracle's table."""
    m, _, _, _ = oracle_lib.tables()
    _, _, mp = lyapunov.basis()
    assert np.abs(m - mp).max() < 1e-15


def test_back_transform_conserves(oracle_lib):
    """Sum_i n_i^a = delta^{a0} and sum_i n_i^a v_i = (delta^{a1}, delta^{a2})/sqrt(3):
    anything added to moments 3..8 leaves mass and momentum unchanged (the
    conservation requirement stated after Eq. 2)."""
    _, n, _, v = oracle_lib.tables()
    e0 = np.zeros(9); e0[0] = 1
    assert np.abs(n.sum(axis=0) - e0).max() < 1e-15
    mom = v.T.astype(float) @ n
    expect = np.zeros((2, 9)); expect[0, 1] = expect[1, 2] = 1 / np.sqrt(3.0)
    assert np.abs(mom - expect).max() < 1e-15


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (0.93, 0.1, -0.05), (1.2, -0.2, 0.17),
                                       (1.0, 0.05, 0.0)])
def test_equilibrium_moments_eq10_from_eq2(oracle_lib, rho, ux, uy):
    """Eq. (10) is exactly the moments (Eq. 3) of the equilibrium Eq. (2) with
    c = 1: the two are computed by different routines and must agree."""
    f0 = oracle_lib.equilibrium(rho, ux, uy)
    M = oracle_lib.moments(f0)
    Meq = oracle_lib.equilibrium_moments(rho, ux, uy)
    assert np.abs(M - Meq).max() < 2e-15
    # density and momentum of f0 (text after Eq. 2)
    _, _, _, v = oracle_lib.tables()
    assert abs(f0.sum() - rho) < 1e-15
    assert np.allclose(v.T @ f0, [rho * ux, rho * uy], atol=1e-15)


def test_collision_keeps_equilibrium(oracle_lib):
    """With no noise, Eq. (5) maps f0 to itself for any tau (M = M^0)."""
    f0 = oracle_lib.equilibrium(1.1, 0.12, -0.07)
    tau = [1, 1, 1, 0.6, 0.7, 0.9, 1.3, 0.8, 1.7]
    out = oracle_lib.collide_site(f0, tau, np.zeros(9), np.zeros(6))
    assert np.abs(out - f0).max() < 1e-15


def test_collision_relaxes_each_mode_by_its_tau(oracle_lib):
    """Eq. (5) with Lambda diagonal in moment space (text after Eq. 4): a
    perturbation of mode a decays by exactly (1 - 1/tau^a), and only mode a
    changes (at u = 0 the equilibrium moments 3..8 are second order in j)."""
    _, n, _, _ = oracle_lib.tables()
    tau = [1, 1, 1, 0.6, 0.7, 0.9, 1.3, 0.8, 1.7]
    f0 = oracle_lib.equilibrium(1.0, 0.0, 0.0)
    for a in range(3, 9):
        eps = 1e-3
        f = f0 + eps * n[:, a]
        out = oracle_lib.collide_site(f, tau, np.zeros(9), np.zeros(6))
        dM = oracle_lib.moments(out) - oracle_lib.moments(f0)
        expect = np.zeros(9); expect[a] = eps * (1 - 1 / tau[a])
        assert np.abs(dM - expect).max() < 1e-15, a
