"""Batch-means statistics for correlator runs (test helper, no method arithmetic)."""
import numpy as np

KEYS = ("S_rho", "S_jx", "S_jy", "S_ux", "S_uy",
        "R_uxuy", "R_rhojx", "R_rhojy", "R_rhoux", "R_rhouy")


def block_means(run_block, nblocks):
    """run_block() returns a dict of per-k arrays for one independent-ish block;
    returns (mean, standard error) dicts over nblocks blocks."""
    blocks = [run_block() for _ in range(nblocks)]
    mean, sem = {}, {}
    for k in blocks[0]:
        a = np.stack([b[k] for b in blocks])
        mean[k] = a.mean(axis=0)
        if np.iscomplexobj(a):
            sem[k] = (a.real.std(axis=0, ddof=1) + 1j * a.imag.std(axis=0, ddof=1)) / np.sqrt(nblocks)
        else:
            sem[k] = a.std(axis=0, ddof=1) / np.sqrt(nblocks)
    return mean, sem


def zscores(mean, sem, expect, mask, floor=1e-8, model_err=0.0):
    """z = (mean - expect) / sem over masked k, real and imaginary parts.

    `model_err` is an absolute allowance for what the expectation leaves out
    (e.g. second-order terms of size ~mu when it comes from linear response):
    that much of the difference is not counted.

    Where the spread vanishes (a mode the dynamics keep deterministic, e.g.
    S(j_x) at (pi, pi) without ghost noise at tau = 1) the value itself must
    match to 1e-6 and is left out of the z-scores."""
    out = []
    for part in (np.real, np.imag):
        m, s, e = part(mean)[mask], part(sem)[mask], part(expect)[mask]
        ok = s > floor
        bad = ~ok
        if np.any(bad):
            assert np.abs(m[bad] - e[bad]).max() < 1e-6 + model_err
        if np.any(ok):
            d = m[ok] - e[ok]
            d = np.sign(d) * np.maximum(np.abs(d) - model_err, 0.0)
            out.append(d / s[ok])
    return np.concatenate(out) if out else np.zeros(0)
