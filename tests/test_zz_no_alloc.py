"""flb_get_populations_noalloc, called through the C interface: the same
values as flb_get_populations, bit for bit, on two calls in a row (the
second on a smaller lattice, so that it reads a part of the staging array
the first call filled), and a clear error for a lattice beyond its limit."""
import ctypes

import numpy as np
import pytest

from paper_1010_1233_amd import workloads

pytestmark = pytest.mark.gpu

TAU = workloads.tau_vector(0.8, 1.0, 1.0)
_dp = ctypes.POINTER(ctypes.c_double)


def _noalloc(flb, g, lattice=0):
    nx, ny, _ = g.shape(lattice)
    out = np.full((9, ny, nx), np.nan)
    rc = flb.lib().flb_get_populations_noalloc(g._h, lattice, out.ctypes.data_as(_dp), out.size)
    assert rc == flb.OK, flb.last_error()
    return out


def test_noalloc_read_equals_allocating_read(flb):
    big = flb.Lattice(640, 480, TAU, 1e-4, u0=(0.03, -0.01), seed=5)
    big.thermalize()
    big.step(7)
    specs = [dict(nx=100, ny=37, tau=TAU, theta=1e-4, u0=(0.0, 0.02), stream_id=0),
             dict(nx=33, ny=64, tau=TAU, theta=1e-4, stream_id=1)]
    small = flb.Lattice.batch(specs, seed=6, storage="bf16")
    small.thermalize()
    small.step(3)
    a = _noalloc(flb, big)
    assert np.array_equal(a, big.get_populations())
    b = _noalloc(flb, small, 1)
    assert np.array_equal(b, small.get_populations(1))
    c = _noalloc(flb, small, 0)
    assert np.array_equal(c, small.get_populations(0))
    big.step(2)  # the state moved on: a new read sees it
    assert np.array_equal(_noalloc(flb, big), big.get_populations())


def test_noalloc_read_rejects_sizes_beyond_its_limit(flb):
    L = flb.lib()
    g = flb.Lattice(1000, 1000, TAU, 1e-4)  # 9e6 values > 2^23
    out = np.empty(9 * 1000 * 1000)
    rc = L.flb_get_populations_noalloc(g._h, 0, out.ctypes.data_as(_dp), out.size)
    assert rc == flb.ESIZE and "8388608" in flb.last_error()
    h = flb.Lattice(16, 16, TAU, 1e-4)
    small = np.empty(9 * 16 * 16 - 1)
    rc = L.flb_get_populations_noalloc(h._h, 0, small.ctypes.data_as(_dp), small.size)
    assert rc == flb.ESIZE
    rc = L.flb_get_populations_noalloc(h._h, 1, small.ctypes.data_as(_dp), small.size)
    assert rc == flb.EINVAL
