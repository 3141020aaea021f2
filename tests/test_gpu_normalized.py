"""The library's normalised correlators (Sec. 3, Eqs. 11-12) against the
oracle's own normalisation of the same raw sums.

The library divides its FP64 sums by the sample count and by each kind's
normalisation on its side of the C interface (flb_read_normalized,
flb_dq_read_normalized); the oracle's ``normalized``, ``normalized_moments``
and ``dq_normalized`` do the same from the paper's formulas.  Non-unit rho0
and a theta other than the workloads' catch a dropped or misplaced factor.
"""
import numpy as np
import pytest

from paper_1010_1233_amd import workloads

pytestmark = pytest.mark.gpu

TAU = workloads.tau_vector(0.8, 0.9, 1.1)


def _close(a, b, rtol=1e-13):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    scale = np.abs(b).max()
    assert np.abs(a - b).max() <= rtol * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("moments", [False, True])
def test_normalized_equals_oracle_normalisation(flb, oracle_lib, moments):
    specs = [dict(nx=24, ny=18, tau=TAU, theta=2e-4, rho0=1.3, u0=(0.03, -0.01), stream_id=0),
             dict(nx=16, ny=20, tau=TAU, theta=5e-5, rho0=0.7, u0=(0.0, 0.04), stream_id=1)]
    b = flb.Lattice.batch(specs, seed=4, moments=moments)
    b.thermalize()
    b.run(70, 10)
    for i, s in enumerate(specs):
        raw, ns = b.read_correlators(i)
        assert ns == 7
        got = b.read_normalized(i)
        ref = oracle_lib.normalized(raw[:15], ns, s["nx"], s["ny"], s["theta"], s["rho0"])
        if moments:
            ref.update(oracle_lib.normalized_moments(raw[15:], ns, s["nx"], s["ny"], s["theta"],
                                                     s["rho0"]))
        assert set(got) == set(ref)
        for k in ref:
            _close(got[k], ref[k])
        # the named arrays are views of the kinds the C call returns
        arr, ns2 = b.read_normalized_raw(i)
        assert ns2 == ns and arr.shape == raw.shape
        _close(arr[5] + 1j * arr[6], ref["R_uxuy"])


def test_normalized_error_states(flb):
    g = flb.Lattice(16, 16, TAU, 1e-4)
    with pytest.raises(flb.FlbError) as e:
        g.read_normalized()  # no sample yet
    assert e.value.code == flb.ESTATE
    g.run(20, 10)
    g.read_normalized()
    g.reset_correlators()
    with pytest.raises(flb.FlbError):
        g.read_normalized()
    z = flb.Lattice(16, 16, TAU, 0.0)  # noise-free: nothing to normalise by
    z.run(10, 10)
    with pytest.raises(flb.FlbError) as e:
        z.read_normalized()
    assert e.value.code == flb.ESTATE
    raw, ns = z.read_correlators()  # the raw sums stay readable
    assert ns == 1


@pytest.mark.parametrize("model,sides", [("D1Q3", (64,)), ("D3Q15", (8, 6, 4)),
                                         ("D2Q9", (12, 10))])
def test_dq_normalized_equals_oracle_normalisation(flb, oracle_lib, model, sides):
    D, _, w, _ = flb.dq_tables(model)
    Q = len(w)
    tau = [1.0] * (D + 1) + [0.85] * (Q - D - 1)
    theta, rho0 = 3e-4, 1.2
    g = flb.DqLattice(model, sides, tau, theta, rho0=rho0, seed=5)
    g.thermalize()
    g.run(30, 5)
    raw, ns = g.read_correlators()
    assert ns == 6
    got = g.read_normalized()
    ref = oracle_lib.dq_normalized(raw, ns, D, Q, g.sides, theta, rho0)
    assert set(got) == set(ref)
    for k in ref:
        _close(got[k], ref[k])


def test_flush_correlators_is_enqueue_only_and_complete(flb):
    """flush_correlators enqueues the waiting sample and the stashed
    samples' products; the sums then equal those of a read, and a read after
    it adds nothing twice."""
    kw = dict(u0=(0.02, 0.0), seed=9)
    a = flb.Lattice(40, 36, TAU, 1e-4, **kw)
    b = flb.Lattice(40, 36, TAU, 1e-4, **kw)
    for L in (a, b):
        L.thermalize()
        L.run(70, 10)  # seven samples: six stashed, one waiting for steps
    a.flush_correlators()
    a.synchronize()
    ra, na = a.read_correlators()
    rb, nb = b.read_correlators()
    assert na == nb == 7
    assert np.array_equal(ra, rb)
    a.flush_correlators()  # nothing owed: no change
    assert np.array_equal(a.read_correlators()[0], ra)
    fresh = flb.Lattice(8, 8, TAU, 1e-4)
    fresh.flush_correlators()  # no sample ever taken
