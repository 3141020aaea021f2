"""A correlator sample runs beside the steps that follow it (on a second
stream); the step that first overwrites the sampled buffer waits until the
sample has read it.  These tests check that the overlapped order gives the
same bits as running each sample at once (the handle's synchronise call
enqueues a waiting sample on the work stream), for every step count that
puts the overwriting launch at a different place, both step kernels, all
storage formats and the moment spectra, and that calls which change the
state or the sums see a waiting sample first.  One sequence is also checked
against the oracle directly.
"""
import sys

import numpy as np
import pytest

from paper_1010_1233_amd import workloads

pytestmark = pytest.mark.gpu

TAU = workloads.tau_vector(0.7, 0.9, 1.0)
STEPS = (1, 2, 3, 5, 4, 10, 1, 7, 2, 6)


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(flb, nx, ny, storage="f32", moments=False, blocking=1):
    hs = []
    for _ in range(2):
        g = flb.Lattice(nx, ny, TAU, 1e-4, u0=(0.03, -0.01), seed=21, storage=storage,
                        moments=moments)
        g.set_time_blocking(blocking, 64)
        g.thermalize()
        hs.append(g)
    return hs


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("blocking", [1, 2, 3])
def test_overlapped_samples_equal_immediate(flb, storage, blocking):
    """1024 x 512: the sample outlasts a step launch, so the overwriting
    launch really waits; step counts 1..10 move it from absent to late."""
    note("overlap", storage, blocking)
    a, b = _pair(flb, 1024, 512, storage, blocking=blocking)
    for n in STEPS:
        a.step(n)
        b.step(n)
        a.accumulate()
        b.accumulate()
        b.synchronize()  # b's sample runs at once, before b's next steps
    a.step(3)
    b.step(3)
    assert a.t == b.t == sum(STEPS) + 3
    ra, na = a.read_correlators()
    rb, nb = b.read_correlators()
    assert na == nb == len(STEPS)
    assert np.array_equal(ra, rb)
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.sample_conservation(), b.sample_conservation())


def test_overlapped_moment_spectra_and_graphs(flb):
    """Moment spectra on (their field kernel also reads the state), graph
    periods of the two-step kernel against plain calls with immediate
    samples."""
    note("overlap moments graphs")
    a, b = _pair(flb, 512, 256, moments=True, blocking=2)
    a.run(95, 10)  # graph periods, each with the previous period's sample
    for t in range(1, 96):
        b.step(1)
        if t % 10 == 0:
            b.accumulate()
            b.synchronize()
    ra, na = a.read_correlators()
    rb, nb = b.read_correlators()
    assert na == nb == 9
    assert np.array_equal(ra, rb)
    a.run(30, 5)  # off-phase start, another period
    for t in range(96, 126):
        b.step(1)
        if t % 5 == 0:
            b.accumulate()
    assert np.array_equal(a.read_correlators()[0], b.read_correlators()[0])
    assert np.array_equal(a.get_populations(), b.get_populations())


def test_waiting_sample_precedes_state_changes(flb, oracle_lib):
    """set_populations, thermalize and autotune change the state: a sample
    registered before them reads the state it was registered on."""
    note("overlap ordering")
    a, b = _pair(flb, 256, 128)
    a.step(4)
    b.step(4)
    f_new = workloads.perturbed(oracle_lib.equilibrium(1.0, 0.03, -0.01), 256, 128, 2e-3,
                                seed=5)
    for g in (a, b):
        g.accumulate()
    b.synchronize()
    for g in (a, b):
        g.set_populations(f_new)
        g.accumulate()
    b.synchronize()
    for g in (a, b):
        g.thermalize()
        g.accumulate()
    b.synchronize()
    for g in (a, b):
        g.autotune(2)
        g.step(3)
        g.accumulate()
    ra, na = a.read_correlators()
    rb, nb = b.read_correlators()
    assert na == nb == 4
    assert np.array_equal(ra, rb)
    # two samples of one state add exactly twice one sample's products
    c, _ = _pair(flb, 256, 128)
    c.step(4)
    c.accumulate()
    one, _ = c.read_correlators()
    c.reset_correlators()
    c.accumulate()
    c.accumulate()
    two, n2 = c.read_correlators()
    assert n2 == 2 and np.array_equal(two, 2 * one)
    # a reset drops a waiting sample with the sums
    c.accumulate()
    c.reset_correlators()
    c.step(2)
    acc, ns = c.read_correlators()
    assert ns == 0 and not acc.any()


@pytest.mark.parametrize("nx,ny", [(96, 64), (70, 45)])
def test_overlapped_sequence_matches_oracle(flb, oracle_lib, nx, ny):
    """Irregular step counts between samples, overlapped on the GPU, against
    the oracle's samples of the same trajectory (70 x 45: Bluestein rows and
    columns, whose spectra go through the stash)."""
    note("overlap oracle", nx, ny)
    kw = dict(u0=(0.03, -0.01), seed=21)
    g = flb.Lattice(nx, ny, TAU, 1e-4, **kw)
    o = oracle_lib.Lattice(nx, ny, TAU, 1e-4, **kw)
    g.set_time_blocking(1, 64)
    g.thermalize()
    o.thermalize()
    for n in STEPS:
        g.step(n)
        o.step(n)
        g.accumulate()
        o.sample()
    g.step(5)
    o.step(5)
    acc, ns = g.read_correlators()
    assert ns == o.nsamples == len(STEPS)
    scale = np.abs(o.acc).reshape(15, -1).max(axis=1)
    for q in range(15):
        d = np.abs(acc[q] - o.acc[q]).max()
        assert d <= 2e-4 * max(scale[q], scale[:5].max() * 1e-3), (q, d, scale[q])


def test_overlap_switch_and_launch_timing(flb):
    """Samples enqueued at once (overlap off) give the same bits as the
    overlapped order, through plain calls and graph periods; launch timing
    counts the step launches enqueued outside graphs."""
    note("overlap switch, launch timing")
    a, b = _pair(flb, 512, 256, blocking=2)
    assert a.sample_overlap() and b.sample_overlap()
    b.set_sample_overlap(False)
    assert not b.sample_overlap()
    for g in (a, b):
        g.run(45, 10)
        for n in (3, 4):
            g.step(n)
            g.accumulate()
        g.run(20, 10)
    assert np.array_equal(a.read_correlators()[0], b.read_correlators()[0])
    assert np.array_equal(a.get_populations(), b.get_populations())
    a.set_launch_timing(True)
    assert a.launch_timing() == (0, 0.0)
    assert a.t == 72
    a.step(7)  # three two-step launches and one one-step launch
    n, ms = a.launch_timing()
    assert n == 4 and ms > 0
    a.step(1)
    a.launch_timing()
    a.run(20, 10)  # from t = 80: two graph periods, not timed
    a.accumulate()
    a.step(2)
    n, ms = a.launch_timing()
    assert n == 1 and ms > 0
    a.set_launch_timing(False)
    a.step(2)
    assert a.launch_timing() == (0, 0.0)
    # three steps per launch: ten steps are 3 + 3 + 2 + 2, seven 3 + 2 + 2,
    # two one launch of two and one a one-step launch; the records split
    # by the steps a launch took
    a.set_time_blocking(3, 64)
    a.set_launch_timing(True)
    for n, want in ((10, (0, 2, 2)), (7, (0, 2, 1)), (2, (0, 1, 0)), (1, (1, 0, 0)),
                    (9, (0, 0, 3))):
        a.step(n)
        kinds = a.launch_timing_kinds()
        assert tuple(k[0] for k in kinds) == want, (n, kinds)
        assert all((c == 0) == (ms == 0.0) for c, ms in kinds)
    a.set_launch_timing(False)
