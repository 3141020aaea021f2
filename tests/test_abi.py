"""The C-ABI boundary, checked without a GPU.

* libflb.so loads and exports every function include/flb.h declares, and the
  Python binding declares a signature for each of them;
* the binding's mirror of flb_lattice_spec has the C layout (checked with a
  tiny program compiled by gcc against the header);
* argument validation happens on the host before any device call, so invalid
  creations fail with a message even here.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in ("flb.h", "flb_dq.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(flb_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("flb_create", "flb_step", "flb_accumulate_correlators", "flb_read_correlators",
              "flb_destroy", "flb_last_error", "flb_create_batch", "flb_run"):
        assert n in names


def test_library_exports_every_declared_symbol(flb):
    L = flb.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", flb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (flb_[a-z_0-9]+)", out))
    assert set(declared_functions()) <= exported


def test_binding_covers_header(flb):
    assert set(flb.SIGNATURES) == set(declared_functions())


def test_lattice_spec_layout_matches_c(flb, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "flb.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(flb_lattice_spec),"
        " offsetof(flb_lattice_spec, tau), offsetof(flb_lattice_spec, theta),"
        " offsetof(flb_lattice_spec, rho0), offsetof(flb_lattice_spec, u0),"
        " offsetof(flb_lattice_spec, stream_id), offsetof(flb_lattice_spec, reserved));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    S = flb.LatticeSpec
    want = [ctypes.sizeof(S), S.tau.offset, S.theta.offset, S.rho0.offset, S.u0.offset,
            S.stream_id.offset, S.reserved.offset]
    assert got == want


def _create(flb, nx=8, ny=8, tau=None, theta=1e-4, rho0=1.0, u0=(0.0, 0.0), storage=0, flags=0):
    tau = np.ascontiguousarray([1, 1, 1, .8, .8, .8, 1, 1, 1] if tau is None else tau,
                               dtype=np.float64)
    u = np.ascontiguousarray(u0, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    return flb.lib().flb_create_ex(nx, ny, tau.ctypes.data_as(dp), theta, rho0,
                                   u.ctypes.data_as(dp), 1, storage, 0, flags)


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=1), "nx and ny"),
    (dict(ny=0), "nx and ny"),
    (dict(tau=[1, 1, 1, 0.5, .8, .8, 1, 1, 1]), "tau[3]"),
    (dict(tau=[1, 1, 1, .8, .8, .8, 1, 1, 0.2]), "tau[8]"),
    (dict(tau=[1, 1, 1, .8, float("nan"), .8, 1, 1, 1]), "finite"),
    (dict(theta=-1.0), "theta"),
    (dict(theta=float("inf")), "theta"),
    (dict(rho0=0.0), "rho0"),
    (dict(u0=(0.5, 0.3)), "sound speed"),
    (dict(u0=(float("nan"), 0.0)), "u0"),
    (dict(storage=7), "storage"),
    (dict(flags=8), "flags"),
    (dict(flags=4), "flags"),
    (dict(nx=100000, ny=100000), "4 GiB"),
    (dict(nx=11000, ny=11000), "4 GiB"),
])
def test_invalid_creation_is_rejected_on_the_host(flb, kw, msg):
    h = _create(flb, **kw)
    assert not h
    assert msg in flb.last_error()


def test_null_handle_calls_fail_cleanly(flb):
    L = flb.lib()
    assert L.flb_step(None, 1) == flb.EINVAL
    assert L.flb_num_lattices(None) == -1
    assert L.flb_num_kinds(None) == flb.EINVAL
    assert L.flb_set_step(None, 0) == flb.EINVAL
    assert L.flb_set_sample_overlap(None, 1) == flb.EINVAL
    assert L.flb_get_sample_overlap(None) == flb.EINVAL
    assert L.flb_set_launch_timing(None, 1) == flb.EINVAL
    n, ms = ctypes.c_int64(), ctypes.c_double()
    assert L.flb_get_launch_timing(None, ctypes.byref(n), ctypes.byref(ms)) == flb.EINVAL
    n3, ms3 = (ctypes.c_int64 * 3)(), (ctypes.c_double * 3)()
    assert L.flb_get_launch_timing_kinds(None, n3, ms3) == flb.EINVAL
    assert L.flb_set_lattice_tiles(None, None) == flb.EINVAL
    assert L.flb_get_lattice_tiles(None, None) == flb.EINVAL
    assert "NULL" in flb.last_error()
    L.flb_destroy(None)


def test_batch_rejects_bad_spec(flb):
    specs = (flb.LatticeSpec * 2)()
    specs[0] = flb.make_spec(8, 8, [1, 1, 1, .8, .8, .8, 1, 1, 1], 1e-4)
    specs[1] = flb.make_spec(8, 1, [1, 1, 1, .8, .8, .8, 1, 1, 1], 1e-4)
    assert not flb.lib().flb_create_batch(2, specs, 1, 0, 0)
    assert "lattice 1" in flb.last_error()
    assert not flb.lib().flb_create_batch(0, specs, 1, 0, 0)


def test_dq_tables_on_the_host(flb):
    """The library's tables of the other velocity sets are orthonormal under
    the weights (Eq. 4) and D2Q9's equal the printed rows of Eq. (9)."""
    for model, q in (("D1Q3", 3), ("D2Q9", 9), ("D3Q15", 15)):
        D, v, w, m = flb.dq_tables(model)
        assert len(w) == q and abs(w.sum() - 1) < 1e-15
        assert np.abs((m * w) @ m.T - np.eye(q)).max() < 1e-14
    _, v, w, m = flb.dq_tables("D2Q9")
    s3, s32, s6 = np.sqrt(3), np.sqrt(1.5), np.sqrt(6)
    eq9_row6 = np.array([0, -s32, 0, s32, 0, s6, -s6, -s6, s6])
    assert np.abs(m[6] - eq9_row6).max() < 1e-14
    assert np.abs(m[8] - np.array([0.5, -1, -1, -1, -1, 2, 2, 2, 2])).max() < 1e-14


@pytest.mark.parametrize("kw,msg", [
    (dict(model=99), "unknown model"),
    (dict(n=(1, 8, 8)), ">= 2"),
    (dict(n=(8, 8, 2), model=29), "unused sides"),
    (dict(tau0=0.5), "tau[4]"),
    (dict(theta=-1.0), "theta"),
    (dict(u0=(0.5, 0.3, 0.2)), "sound speed"),
    (dict(u0=(0.1, 0.0, 0.0), model=13, n=(16, 1, 1), u0y=0.1), "unused axis"),
    (dict(n=(1024, 1024, 1024)), "4 GiB"),
    (dict(flags=8), "flags"),
])
def test_dq_invalid_creation_is_rejected_on_the_host(flb, kw, msg):
    model = kw.get("model", 315)
    n = np.ascontiguousarray(kw.get("n", (8, 8, 8)), dtype=np.int32)
    tau = np.ones(15)
    if "tau0" in kw:
        tau[4] = kw["tau0"]
    u0 = list(kw.get("u0", (0.0, 0.0, 0.0)))
    if "u0y" in kw:
        u0[1] = kw["u0y"]
    u = np.ascontiguousarray(u0, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    h = flb.lib().flb_dq_create(model, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                tau.ctypes.data_as(dp), kw.get("theta", 1e-4), 1.0,
                                u.ctypes.data_as(dp), 1, 0, kw.get("flags", 0))
    assert not h
    assert msg in flb.last_error()
