"""GPU parity of the correlator measurement (Eqs. 11-12) against the oracle.

Paired runs (same seed and counters) follow the same trajectory to ~1e-6, so
the accumulated sums agree element by element to a small relative tolerance;
statistical runs check S_k = 1 and vanishing cross correlators at u0 = 0 on
the GPU alone (Eq. 7), with the abstract's "< 0.5 %" on the cross correlators.
"""
import sys

import numpy as np
import pytest

import lyapunov
from stats_util import KEYS, block_means, zscores
from paper_1010_1233_amd import workloads

pytestmark = pytest.mark.gpu

TAU_C1 = workloads.tau_vector(0.8, 0.8, 1.0)


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare(acc_g, acc_o, rtol):
    scale = np.abs(acc_o).reshape(15, -1).max(axis=1)
    for q in range(15):
        d = np.abs(acc_g[q] - acc_o[q]).max()
        assert d <= rtol * max(scale[q], scale[:5].max() * 1e-3), (q, d, scale[q])


@pytest.mark.parametrize("nx,ny", [(32, 32), (20, 20), (24, 18), (37, 23), (64, 8), (2, 2),
                                   (128, 96), (3, 256), (40, 600), (1000, 5), (300, 7),
                                   (1500, 3), (12, 1024), (10, 2048), (6, 4096),
                                   (512, 512), (512, 300), (300, 512),
                                   (1024, 3), (2048, 5), (4096, 3), (100, 40), (200, 12),
                                   (64, 200), (20, 1000), (512, 4096)])
def test_single_sample_matches_oracle(flb, oracle_lib, nx, ny):
    note("sample", nx, ny)
    g = flb.Lattice(nx, ny, TAU_C1, 1e-4, u0=(0.04, -0.01), seed=3)
    o = oracle_lib.Lattice(nx, ny, TAU_C1, 1e-4, u0=(0.04, -0.01), seed=3)
    g.thermalize()
    o.thermalize()
    g.step(7)
    o.step(7)
    g.accumulate()
    o.sample()
    acc, ns = g.read_correlators()
    assert ns == 1 and acc.shape == o.acc.shape
    assert np.all(acc[:, 0, 0] == 0)
    _compare(acc, o.acc, 2e-4)


def test_paired_run_config1(flb, oracle_lib):
    """32^2, 2000 steps, a sample every 10 steps, thermal start."""
    c = workloads.CONFIGS["c1_32"]
    g = flb.Lattice(32, 32, c["tau"], c["theta"], seed=c["seed"])
    o = oracle_lib.Lattice(32, 32, c["tau"], c["theta"], seed=c["seed"])
    g.thermalize()
    o.thermalize()
    g.run(2000, 10)
    o.run(2000, 10)
    acc, ns = g.read_correlators()
    assert ns == o.nsamples == 200
    _compare(acc, o.acc, 1e-3)


def test_graph_run_equals_plain_calls(flb):
    a = flb.Lattice(48, 40, TAU_C1, 1e-4, seed=8)
    b = flb.Lattice(48, 40, TAU_C1, 1e-4, seed=8)
    a.thermalize()
    b.thermalize()
    a.run(103, 10)  # graph periods plus a ragged tail
    for t in range(1, 104):
        b.step(1)
        if t % 10 == 0:
            b.accumulate()
    assert a.t == b.t == 103
    assert np.array_equal(a.get_populations(), b.get_populations())
    ra, na = a.read_correlators()
    rb, nb = b.read_correlators()
    assert na == nb == 10
    assert np.array_equal(ra, rb)
    # odd period, started off-phase
    a.run(37, 3)
    for t in range(104, 141):
        b.step(1)
        if t % 3 == 0:
            b.accumulate()
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.read_correlators()[0], b.read_correlators()[0])


def test_batch_correlators_equal_separate(flb):
    specs = [dict(nx=32, ny=32, tau=TAU_C1, theta=1e-4, stream_id=0),
             dict(nx=20, ny=12, tau=TAU_C1, theta=1e-4, u0=(0.05, 0.0), stream_id=1)]
    b = flb.Lattice.batch(specs, seed=2)
    b.thermalize()
    b.run(100, 10)
    for i, s in enumerate(specs):
        g = flb.Lattice(s["nx"], s["ny"], s["tau"], s["theta"], u0=s.get("u0", (0, 0)), seed=2,
                        stream_id=s["stream_id"])
        g.thermalize()
        g.run(100, 10)
        assert np.array_equal(b.read_correlators(i)[0], g.read_correlators()[0])


def test_reset_correlators(flb):
    g = flb.Lattice(16, 16, TAU_C1, 1e-4)
    g.run(50, 10)
    g.reset_correlators()
    acc, ns = g.read_correlators()
    assert ns == 0 and not acc.any()


def test_large_lattice_sample_matches_oracle(flb, oracle_lib):
    """4096^2: one sample against the oracle's FP64 transform."""
    c = workloads.CONFIGS["c5_4096"]
    note("4096^2 sample")
    g = flb.Lattice(4096, 4096, c["tau"], c["theta"], u0=c["u0"], seed=c["seed"])
    o = oracle_lib.Lattice(4096, 4096, c["tau"], c["theta"], u0=c["u0"], seed=c["seed"])
    f0 = workloads.perturbed(oracle_lib.equilibrium(1.0, *c["u0"]), 4096, 4096, 3e-3, seed=13)
    g.set_populations(f0)
    o.set_populations(f0)
    del f0
    g.accumulate()
    o.sample()
    acc, _ = g.read_correlators()
    _compare(acc, o.acc, 1e-3)


def _mask(nx, ny):
    nh = nx // 2 + 1
    m = np.ones((ny, nh), dtype=bool)
    for ky in range(ny):
        for kx in range(nh):
            m[ky, kx] = not lyapunov.singular_k(nx, ny, kx, ky)
    return m


def test_structure_factors_are_one_on_gpu(flb):
    """64^2 at u0 = 0 (config-2 relaxation times), thermal start: every S = 1
    and every cross correlator 0 within the batch-means error; the k-averaged
    cross correlators are below 0.5 %."""
    nx = ny = 64
    tau = workloads.CONFIGS["c2_256"]["tau"]
    theta = 1e-4
    g = flb.Lattice(nx, ny, tau, theta, seed=2)
    g.thermalize()
    g.step(2000)

    def block():
        g.reset_correlators()
        g.run(20000, 10)
        return g.read_normalized()

    mean, sem = block_means(block, 16)
    pred = lyapunov.predict(nx, ny, tau, theta)
    m = _mask(nx, ny)
    zs = []
    for k in KEYS:
        z = zscores(mean[k], sem[k], pred[k], m, model_err=9e-4)
        note(k, "max|z|", np.abs(z).max())
        assert np.abs(z).max() < 6.5
        zs.append(z)
    chi = (np.concatenate(zs) ** 2).mean()
    note("mean z^2", chi)
    assert 0.6 < chi < 1.7
    for k in ("R_uxuy", "R_rhojx", "R_rhojy", "R_rhoux", "R_rhouy"):
        assert abs(mean[k][m].mean()) < 0.005


@pytest.mark.parametrize("nx,ny", [(48, 36), (512, 12), (1024, 7), (300, 7)])
def test_sample_records_conservation_sums(flb, oracle_lib, nx, ny):
    """Each sample also returns the FP64 mass/momentum/staggered sums of the
    sampled state: they match the dedicated conservation call and the oracle
    (generic and length-specialised row kernels, power-of-two and
    Bluestein)."""
    g = flb.Lattice(nx, ny, TAU_C1, 1e-3, u0=(0.03, -0.01), seed=5)
    o = oracle_lib.Lattice(nx, ny, TAU_C1, 1e-3, u0=(0.03, -0.01), seed=5)
    with pytest.raises(flb.FlbError):
        g.sample_conservation()
    g.thermalize()
    o.thermalize()
    g.step(13)
    o.step(13)
    g.accumulate()
    cs = g.sample_conservation()
    assert np.abs(cs - g.conservation()).max() < 1e-5
    assert np.abs(cs - o.conservation()).max() < 1e-5


@pytest.mark.parametrize("nx,ny", [(32, 32), (24, 18), (37, 23), (128, 96), (256, 128), (2, 2),
                                   (8, 1024)])
def test_moment_spectra_match_oracle(flb, oracle_lib, nx, ny):
    """Kinds 15..20 (|M^a_k|^2, a = 3..8) of one sample against the oracle;
    the first fifteen kinds are unchanged by the extra field set."""
    note("moments", nx, ny)
    kw = dict(u0=(0.03, 0.01), seed=6)
    g = flb.Lattice(nx, ny, TAU_C1, 1e-4, moments=True, **kw)
    h = flb.Lattice(nx, ny, TAU_C1, 1e-4, **kw)
    o = oracle_lib.Lattice(nx, ny, TAU_C1, 1e-4, moments=True, **kw)
    for L in (g, h, o):
        L.thermalize()
        L.step(5)
    g.accumulate()
    h.accumulate()
    o.sample()
    acc, ns = g.read_correlators()
    assert ns == 1 and acc.shape[0] == flb.NKINDS_MOMENTS == g.nkinds
    assert np.array_equal(acc[:15], h.read_correlators()[0])
    assert np.all(acc[15:, 0, 0] == 0)
    scale = np.abs(o.acc_m).reshape(6, -1).max(axis=1)
    for a in range(6):
        d = np.abs(acc[15 + a] - o.acc_m[a]).max()
        assert d <= 2e-4 * scale.max(), (a, d, scale[a])


def test_moment_spectra_paired_run_and_batch(flb, oracle_lib):
    """Paired 2000-step run with a sample every 10 steps, and a batch of two
    lattices of different shapes, with the moment spectra on."""
    c = workloads.CONFIGS["c1_32"]
    g = flb.Lattice(32, 32, c["tau"], c["theta"], seed=c["seed"], moments=True)
    o = oracle_lib.Lattice(32, 32, c["tau"], c["theta"], seed=c["seed"], moments=True)
    g.thermalize()
    o.thermalize()
    g.run(2000, 10)
    o.run(2000, 10)
    acc, ns = g.read_correlators()
    assert ns == o.nsamples == 200
    _compare(acc[:15], o.acc, 1e-3)
    d = np.abs(acc[15:] - o.acc_m).max()
    assert d <= 1e-3 * np.abs(o.acc_m).max()

    specs = [dict(nx=32, ny=16, tau=TAU_C1, theta=1e-4, stream_id=0),
             dict(nx=20, ny=12, tau=TAU_C1, theta=1e-4, u0=(0.05, 0.0), stream_id=1)]
    b = flb.Lattice.batch(specs, seed=2, moments=True)
    b.thermalize()
    b.run(100, 10)
    for i, s in enumerate(specs):
        one = flb.Lattice(s["nx"], s["ny"], s["tau"], s["theta"], u0=s.get("u0", (0, 0)),
                          seed=2, stream_id=s["stream_id"], moments=True)
        one.thermalize()
        one.run(100, 10)
        assert np.array_equal(b.read_correlators(i)[0], one.read_correlators()[0])


def test_reads_between_paired_samples(flb, oracle_lib):
    """Samples stash their spectra and every 32nd adds the products of all
    32; a read with samples outstanding adds them first.  Reading after
    every sample, twice in a row, or only at the end all give the oracle's
    sums."""
    kw = dict(u0=(0.02, 0.0), seed=12)
    a = flb.Lattice(64, 32, TAU_C1, 1e-4, **kw)
    b = flb.Lattice(64, 32, TAU_C1, 1e-4, **kw)
    o = oracle_lib.Lattice(64, 32, TAU_C1, 1e-4, **kw)
    for L in (a, b, o):
        L.thermalize()
    for n in range(1, 6):
        for L in (a, b, o):
            L.step(3)
        a.accumulate()
        b.accumulate()
        o.sample()
        r1, n1 = a.read_correlators()
        r2, n2 = a.read_correlators()
        assert n1 == n2 == n and np.array_equal(r1, r2)
        _compare(r1, o.acc, 2e-4)
    rb, nb = b.read_correlators()
    assert nb == 5
    _compare(rb, o.acc, 2e-4)
    assert np.abs(rb - r1).max() <= 1e-12 * np.abs(rb).max()
    # a reset drops an outstanding sample together with the sums
    a.accumulate()
    a.reset_correlators()
    a.accumulate()
    o.acc[...] = 0
    o.sample()
    _compare(a.read_correlators()[0], o.acc, 2e-4)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("nx,ny", [(2048, 2048), (4096, 4096), (600, 300), (200, 130)])
def test_storage_formats_against_oracle(flb, oracle_lib, nx, ny):
    """The 4096^2 workload (u_x = 0.05, tau_s = 0.6, kT = 1e-4), at 4096^2
    itself and at 2048^2, and on sides whose transforms take Bluestein's
    convolution (rows and columns of work lengths 2048 and 1024, 512 and
    512): thermal start, ten steps and one sample in each storage format
    against the oracle's FP64 run of the same trajectory (one oracle run per
    shape, about a minute at 4096^2).  Per kind, the error of the sums over k
    relative to their size (cross kinds relative to the geometric mean of the
    two fields' auto sums) measures what the storage format costs the
    correlators."""
    c = workloads.CONFIGS["c5_4096"]
    side = f"{nx}x{ny}"
    note(f"{side} oracle run")
    o = oracle_lib.Lattice(nx, ny, c["tau"], c["theta"], u0=c["u0"], seed=c["seed"])
    o.thermalize()
    o.step(10)
    o.sample()
    ref = o.acc.copy()
    del o
    ref[:, 0, 0] = 0
    auto = np.sqrt((ref[:5] ** 2).reshape(5, -1).sum(axis=1))
    # fields of each product kind (rho, jx, jy, ux, uy = 0..4)
    pairs = {5: (3, 4), 6: (3, 4), 7: (0, 1), 8: (0, 1), 9: (0, 2), 10: (0, 2),
             11: (0, 3), 12: (0, 3), 13: (0, 4), 14: (0, 4)}
    # measured at 2048^2: worst kind 5e-7, 3.7e-4, 2.9e-3
    bounds = {"f32": 3e-6, "f16": 2e-3, "bf16": 1.5e-2}
    for storage, bound in bounds.items():
        note(side, storage)
        g = flb.Lattice(nx, ny, c["tau"], c["theta"], u0=c["u0"], seed=c["seed"],
                        storage=storage)
        g.thermalize()
        g.step(10)
        g.accumulate()
        acc, ns = g.read_correlators()
        g.close()
        assert ns == 1
        rel = []
        for q in range(15):
            err = np.sqrt(((acc[q] - ref[q]) ** 2).sum())
            if q < 5:
                scale = auto[q]
            else:
                a, b = pairs[q]
                scale = np.sqrt(auto[a] * auto[b])
            rel.append(err / scale)
        note(f"  {storage}: relative error per kind", " ".join(f"{r:.2e}" for r in rel))
        assert max(rel) < bound, (storage, rel)


def test_batch_of_column_block_widths_equals_separate_lattices(flb, oracle_lib):
    """Column work lengths 2048, 1024 and 256 (Bluestein, 4, 8 and 16
    columns per block) and a power-of-two side in one batch: over forty samples
    (across a 32-sample accumulation cycle, with graph-replayed periods)
    every lattice's sums are the bits of the same lattice run alone, and the
    longest columns' sums match the oracle."""
    specs = [dict(nx=40, ny=600, tau=TAU_C1, theta=1e-4, stream_id=0),
             dict(nx=30, ny=300, tau=TAU_C1, theta=1e-4, u0=(0.03, 0.0), stream_id=1),
             dict(nx=50, ny=100, tau=TAU_C1, theta=1e-4, stream_id=2),
             dict(nx=24, ny=64, tau=TAU_C1, theta=1e-4, u0=(0.0, 0.02), stream_id=3)]
    note("column block widths batch")
    b = flb.Lattice.batch(specs, seed=8)
    b.thermalize()
    b.run(160, 4)
    for i, s in enumerate(specs):
        one = flb.Lattice(s["nx"], s["ny"], s["tau"], s["theta"], u0=s.get("u0", (0, 0)),
                          seed=8, stream_id=s["stream_id"])
        one.thermalize()
        one.run(160, 4)
        acc, ns = b.read_correlators(i)
        ref, nr = one.read_correlators()
        assert ns == nr == 40
        assert np.array_equal(acc, ref), i
        one.close()
    s = specs[0]
    o = oracle_lib.Lattice(s["nx"], s["ny"], s["tau"], s["theta"], seed=8,
                           stream_id=s["stream_id"])
    o.thermalize()
    o.run(160, 4)
    assert o.nsamples == 40
    _compare(b.read_correlators(0)[0], o.acc, 1e-3)


def test_large_column_blocks_over_sample_cycles(flb, oracle_lib):
    """ny = 4096 takes the column kernel's large blocks (1024 threads, four
    whole columns): forty samples, the 32nd of which adds the products of
    the 32 stashed ones, overlapped beside the steps, with reads after the
    third and the 33rd (a read adds the stashed samples first), against
    samples enqueued at once (same bits) and against the oracle."""
    kw = dict(u0=(0.03, -0.01), seed=17)
    a = flb.Lattice(8, 4096, TAU_C1, 1e-4, **kw)
    b = flb.Lattice(8, 4096, TAU_C1, 1e-4, **kw)
    o = oracle_lib.Lattice(8, 4096, TAU_C1, 1e-4, **kw)
    b.set_sample_overlap(False)
    for L in (a, b, o):
        L.thermalize()
    for i in range(40):
        for L in (a, b, o):
            L.step(3)
        a.accumulate()
        b.accumulate()
        o.sample()
        if i in (2, 32):
            ra, na = a.read_correlators()
            assert na == i + 1
            assert np.array_equal(ra, b.read_correlators()[0])
            _compare(ra, o.acc, 2e-4)
    ra, na = a.read_correlators()
    assert na == o.nsamples == 40
    assert np.array_equal(ra, b.read_correlators()[0])
    _compare(ra, o.acc, 2e-4)


def test_galilean_batch_shape_over_sample_cycles(flb, oracle_lib):
    """The Galilean-invariance sweep's shape: 512^2 lattices (512-point rows
    and 512-point columns in the small column blocks) at four of the sweep's
    mean velocities, batched, graph-replayed periods with the samples beside
    the steps; forty samples cross a 32-sample accumulation cycle.
    Every lattice's sums match the oracle's run of the same trajectory
    element by element."""
    us = (0.0, 0.05, 0.1, 0.2)
    specs = [dict(nx=512, ny=512, tau=workloads.tau_vector(0.8, 1.0, 1.0), theta=1e-4,
                  rho0=1.0, u0=(u, 0.0), stream_id=16 * i) for i, u in enumerate(us)]
    note("4 x 512^2 batch, 40 samples")
    b = flb.Lattice.batch(specs, seed=3)
    b.thermalize()
    b.run(80, 2)
    for i, s in enumerate(specs):
        note("  oracle lattice", i)
        o = oracle_lib.Lattice(512, 512, s["tau"], s["theta"], u0=s["u0"], seed=3,
                               stream_id=s["stream_id"])
        o.thermalize()
        o.run(80, 2)
        acc, ns = b.read_correlators(i)
        assert ns == o.nsamples == 40
        assert np.all(acc[:, 0, 0] == 0)
        _compare(acc, o.acc, 1e-3)
