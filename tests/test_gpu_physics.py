"""Statistical checks of the paper's claims on the GPU, against the
linear-response predictor (batched lattices give independent realisations,
so the ensemble spread is the error bar).

* The paper's regime (V = 20^2, tau^a = 1): with ghost noise every S_k and
  cross correlator agrees with Eq. (7) (the paper reports agreement "to three
  orders of magnitude" after 2e8 iterations; here 2e7 lattice-samples);
  without ghost noise R(u_x, u_y) reaches the predicted +-0.26 ("up to 0.25
  rho", Sec. 3) and S(rho) drops to 0.2 at (pi, pi).
* A mean flow breaks the decoupling by the predicted amounts (Fig. 4).
* 16-bit storage: S_k error against the prediction, stated per format.
* The structure factors of the six non-conserved moments: 1 with ghost noise
  (the paper finds the same agreement for all nine moments), the predicted
  finite-k deficits without it.
"""
import sys

import numpy as np
import pytest

import lyapunov
from stats_util import KEYS, zscores
from paper_1010_1233_amd import workloads

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mask(nx, ny):
    nh = nx // 2 + 1
    m = np.ones((ny, nh), dtype=bool)
    for ky in range(ny):
        for kx in range(nh):
            m[ky, kx] = not lyapunov.singular_k(nx, ny, kx, ky)
    return m


MKEYS = tuple("S_M%d" % a for a in range(3, 9))


def ensemble(flb, specs, steps, every, seed, ladd=False, storage="f32", burn=1000,
             moments=False):
    """Run a batch of independent lattices; return per-key ensemble mean and
    standard error over lattices of the normalised correlators."""
    b = flb.Lattice.batch(specs, seed=seed, ladd=ladd, storage=storage, moments=moments)
    b.thermalize()
    b.step(burn)
    b.reset_correlators()
    b.run(steps, every)
    per = []
    for i in range(len(specs)):
        per.append(b.read_normalized(i))
    b.close()
    mean, sem = {}, {}
    n = len(per)
    for k in per[0]:
        a = np.stack([p[k] for p in per])
        mean[k] = a.mean(axis=0)
        sd = (a.real.std(axis=0, ddof=1) + 1j * a.imag.std(axis=0, ddof=1)
              if np.iscomplexobj(a) else a.std(axis=0, ddof=1))
        sem[k] = sd / np.sqrt(n)
    return mean, sem


def _check(mean, sem, pred, mask, zmax=6.0, mu=3e-4, keys=KEYS):
    """Every correlator within zmax errors of linear response after allowing
    3 mu for the second-order terms it leaves out; the raw z-scores (no
    allowance) show the ensemble errors are not overestimated."""
    zs, raw = [], []
    for k in keys:
        z = zscores(mean[k], sem[k], pred[k], mask, model_err=3 * mu)
        r = zscores(mean[k], sem[k], pred[k], mask)
        note(f"  {k}: max|z| {np.abs(z).max():.2f} (raw {np.abs(r).max():.2f}), "
             f"max|dev| {np.nanmax(np.abs(mean[k] - pred[k])[mask]):.2e}")
        assert np.abs(z).max() < zmax, k
        zs.append(z)
        raw.append(r)
    chi = (np.concatenate(zs) ** 2).mean()
    chi_raw = (np.concatenate(raw) ** 2).mean()
    note(f"  mean z^2 {chi:.3f} (raw {chi_raw:.3f})")
    assert chi < 1.6 and chi_raw > 0.6


def test_paper_regime_with_ghost_noise(flb):
    """1024 lattices of 20^2, tau^a = 1, 2e4 steps sampled every step."""
    n, tau, theta = 20, workloads.tau_vector(1, 1, 1), 1e-4
    specs = [dict(nx=n, ny=n, tau=tau, theta=theta, stream_id=i) for i in range(1024)]
    mean, sem = ensemble(flb, specs, 20000, 1, seed=41, moments=True)
    pred = lyapunov.predict(n, n, tau, theta)
    m = _mask(n, n)
    _check(mean, sem, pred, m, keys=KEYS + MKEYS)
    for k in MKEYS:
        dev = np.abs(mean[k][m].mean() - 1)
        note(f"  <{k}> - 1 = {dev:.2e}")
        assert dev < 1e-3
    # the paper's "three orders of magnitude": k-averaged |S - 1| and |R|
    for k in ("S_rho", "S_ux", "S_jx"):
        dev = np.abs(mean[k][m].mean() - 1)
        note(f"  <{k}> - 1 = {dev:.2e}, median sem {np.median(sem[k][m]):.2e}")
        assert dev < 1e-3
    r = np.abs(mean["R_uxuy"][m].real).mean()
    note(f"  <|Re R(ux,uy)|> = {r:.2e}")
    assert r < 1e-2


def test_paper_regime_without_ghost_noise(flb):
    n, tau, theta = 20, workloads.tau_vector(1, 1, 1), 1e-4
    specs = [dict(nx=n, ny=n, tau=tau, theta=theta, stream_id=i) for i in range(512)]
    mean, sem = ensemble(flb, specs, 10000, 1, seed=42, ladd=True, moments=True)
    pred = lyapunov.predict(n, n, tau, theta, ladd=True)
    m = _mask(n, n)
    _check(mean, sem, pred, m, keys=KEYS + MKEYS)
    for k in ("S_M6", "S_M7", "S_M8"):
        note(f"  <{k}> = {mean[k][m].mean():.4f} (predicted {np.nanmean(pred[k][m]):.4f})")
        assert mean[k][m].mean() < 0.6
    R = mean["R_uxuy"].real
    note(f"  max R(ux,uy) {np.nanmax(R[m]):.4f} at {np.unravel_index(np.argmax(np.where(m, R, -9)), R.shape)}")
    assert abs(np.nanmax(R[m]) - 0.2617) < 0.01
    assert abs(mean["S_rho"][10, 10] - 0.2) < 0.01


def test_c2_shape_structure_factors(flb):
    """The 256^2 workload (tau_s = 0.8, tau_b = 1, kT = 1e-4, u0 = 0) as an
    ensemble of 64 thermalised lattices, 2e4 steps sampled every 10: every
    S = 1 and every cross correlator 0 (Eq. 7, exact at linear order for
    u0 = 0 with this start) within the ensemble errors; the k-averaged cross
    correlators are below the abstract's 0.5 %."""
    n, theta = 256, 1e-4
    tau = workloads.CONFIGS["c2_256"]["tau"]
    specs = [dict(nx=n, ny=n, tau=tau, theta=theta, stream_id=i) for i in range(64)]
    mean, sem = ensemble(flb, specs, 20000, 10, seed=2)
    m = _mask(n, n)
    pred = {k: np.ones_like(mean[k]) if k.startswith("S_") else np.zeros_like(mean[k])
            for k in KEYS}
    _check(mean, sem, pred, m)
    for k in ("R_uxuy", "R_rhojx", "R_rhojy", "R_rhoux", "R_rhouy"):
        r = abs(mean[k][m].mean())
        note(f"  |<{k}>_k| = {r:.2e}")
        assert r < 0.005


@pytest.mark.parametrize("u", [0.05, 0.1])
def test_mean_flow_deviation_matches_prediction(flb, u):
    """Fig. 4 regime and the Galilean sweep: 256 lattices of 24^2 at u_x."""
    n, tau, theta = 24, workloads.tau_vector(0.8, 1.0, 1.0), 1e-4
    specs = [dict(nx=n, ny=n, tau=tau, theta=theta, u0=(u, 0.0), stream_id=i) for i in range(256)]
    mean, sem = ensemble(flb, specs, 20000, 2, seed=43)
    pred = lyapunov.predict(n, n, tau, theta, u0=(u, 0.0))
    m = _mask(n, n)
    _check(mean, sem, pred, m)
    zero = {k: 0 * v for k, v in pred.items()}
    z0 = zscores(mean["R_rhoux"], sem["R_rhoux"], zero["R_rhoux"], m)
    assert np.abs(z0).max() > 10  # the violation itself is resolved


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_storage_formats_structure_factor_error(flb, storage):
    """S_k error of each storage format at the 4096^2 workload's parameters
    (u_x = 0.05, tau_s = 0.6, kT = 1e-4) on 64 lattices of 32^2: FP32 and
    FP16 agree with the prediction within the statistics; BF16's rounding
    (8-bit mantissa on the scaled deviation) adds a stated bias."""
    c = workloads.CONFIGS["c5_4096"]
    n = 32
    specs = [dict(nx=n, ny=n, tau=c["tau"], theta=c["theta"], u0=c["u0"], stream_id=i)
             for i in range(64)]
    mean, sem = ensemble(flb, specs, 20000, 2, seed=44, storage=storage)
    pred = lyapunov.predict(n, n, c["tau"], c["theta"], u0=c["u0"])
    m = _mask(n, n)
    err = {k: float(np.nanmax(np.abs(mean[k] - pred[k])[m])) for k in ("S_rho", "S_ux", "R_uxuy")}
    bias = {k: float(np.abs((mean[k] - pred[k])[m].mean())) for k in ("S_rho", "S_ux")}
    note(f"  {storage}: max|S - pred| {err}, |mean bias| {bias}")
    if storage in ("f32", "f16"):
        _check(mean, sem, pred, m)
    else:
        assert bias["S_rho"] < 0.05 and bias["S_ux"] < 0.05
