"""MI355X (gfx950) fluctuating ideal-gas lattice Boltzmann library.

Python binding of ``libflb.so`` (C interface in ``include/flb.h``): argument
marshalling only.  Every step of the method runs in the library: the path in
its HIP kernels, the normalisation of the correlator sums (Eqs. 11-12) on its
host side (``read_normalized``); the binding only names the kinds it returns.
PyTorch, when used, only supplies streams (``set_stream``).

The library must have been built (``python -m paper_1010_1233_amd.build``);
importing the package does not load it, the first use does, and a missing
library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflb.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "flb.h")

OK, EINVAL, ENOMEM, EHIP, ESIZE, ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "bf16": 1, "f16": 2}
FLAG_NO_GHOST_NOISE = 1
FLAG_MOMENT_SPECTRA = 2
NKINDS = 15
NKINDS_MOMENTS = 21
KINDS = ("rho_rho", "jx_jx", "jy_jy", "ux_ux", "uy_uy",
         "re_ux_uy", "im_ux_uy", "re_rho_jx", "im_rho_jx", "re_rho_jy", "im_rho_jy",
         "re_rho_ux", "im_rho_ux", "re_rho_uy", "im_rho_uy")
MOMENT_KINDS = tuple("M%d_M%d" % (a, a) for a in range(3, 9))
# Names of the normalised kinds (flb_read_normalized): one real array per
# structure factor; a cross correlator's Re and Im kinds become one complex
# array.
NORMALIZED = (("S_rho", 0), ("S_jx", 1), ("S_jy", 2), ("S_ux", 3), ("S_uy", 4),
              ("R_uxuy", 5, 6), ("R_rhojx", 7, 8), ("R_rhojy", 9, 10), ("R_rhoux", 11, 12),
              ("R_rhouy", 13, 14)) + tuple(("S_M%d" % a, 12 + a) for a in range(3, 9))


class FlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"flb error {code}: {msg}")
        self.code = code


class LatticeSpec(ctypes.Structure):
    """Mirror of ``flb_lattice_spec``."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("tau", ctypes.c_double * 9), ("theta", ctypes.c_double),
                ("rho0", ctypes.c_double), ("u0", ctypes.c_double * 2),
                ("stream_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_intp = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes)
SIGNATURES = {
    "flb_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                     ctypes.c_double, _dp, ctypes.c_uint64]),
    "flb_create_ex": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                        ctypes.c_double, _dp, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_uint32]),
    "flb_create_batch": (ctypes.c_void_p, [ctypes.c_int, ctypes.POINTER(LatticeSpec),
                                           ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32]),
    "flb_destroy": (None, [ctypes.c_void_p]),
    "flb_last_error": (ctypes.c_char_p, []),
    "flb_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "flb_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_set_sample_overlap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "flb_get_sample_overlap": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_set_launch_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "flb_get_launch_timing_kinds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                                   _dp]),
    "flb_get_launch_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_double)]),
    "flb_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "flb_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]),
    "flb_accumulate_correlators": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_read_correlators": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t,
                                            _i64p]),
    "flb_read_normalized": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t,
                                           _i64p]),
    "flb_flush_correlators": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_reset_correlators": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t]),
    "flb_get_populations_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp,
                                                   ctypes.c_size_t]),
    "flb_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t]),
    "flb_conservation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "flb_conservation_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "flb_sample_conservation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "flb_thermalize": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_debug_noise": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                       ctypes.c_int64, ctypes.c_int64, _u32p, _fp]),
    "flb_get_step": (ctypes.c_int64, [ctypes.c_void_p]),
    "flb_set_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "flb_num_kinds": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_num_lattices": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_lattice_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p, _i32p]),
    "flb_storage_info": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p]),
    "flb_set_step_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
    "flb_get_step_config": (ctypes.c_int, [ctypes.c_void_p, _intp, _intp, _intp]),
    "flb_set_time_blocking": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "flb_get_time_blocking": (ctypes.c_int, [ctypes.c_void_p, _intp, _intp]),
    "flb_set_lattice_tiles": (ctypes.c_int, [ctypes.c_void_p, _i32p]),
    "flb_get_lattice_tiles": (ctypes.c_int, [ctypes.c_void_p, _i32p]),
    "flb_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "flb_autotune_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp]),
    # other velocity sets (flb_dq.h)
    "flb_dq_tables": (ctypes.c_int, [ctypes.c_int, _i32p, _i32p, _i32p, _dp, _dp]),
    "flb_dq_create": (ctypes.c_void_p, [ctypes.c_int, _i32p, _dp, ctypes.c_double,
                                        ctypes.c_double, _dp, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32]),
    "flb_dq_destroy": (None, [ctypes.c_void_p]),
    "flb_dq_info": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p, _i32p]),
    "flb_dq_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "flb_dq_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_dq_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "flb_dq_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]),
    "flb_dq_get_step": (ctypes.c_int64, [ctypes.c_void_p]),
    "flb_dq_accumulate": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_dq_read": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t, _i64p]),
    "flb_dq_read_normalized": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t, _i64p]),
    "flb_dq_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_dq_get_populations": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "flb_dq_set_populations": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "flb_dq_thermalize": (ctypes.c_int, [ctypes.c_void_p]),
    "flb_dq_conservation": (ctypes.c_int, [ctypes.c_void_p, _dp]),
}


def lib():
    """Load libflb.so (raises if it has not been built).

    PyTorch ships its own HIP runtime under the same soname as the system
    one; whichever is loaded first serves the whole process.  torch is
    therefore imported first (when installed) so that the library and torch
    share torch's runtime, streams and events.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1010_1233_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().flb_last_error().decode()


def _check(rc):
    if rc != OK:
        raise FlbError(rc, last_error())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_dp)


def make_spec(nx, ny, tau, theta, rho0=1.0, u0=(0.0, 0.0), stream_id=0):
    s = LatticeSpec()
    s.nx, s.ny = int(nx), int(ny)
    for a in range(9):
        s.tau[a] = float(tau[a])
    s.theta, s.rho0 = float(theta), float(rho0)
    s.u0[0], s.u0[1] = float(u0[0]), float(u0[1])
    s.stream_id = int(stream_id)
    s.reserved = 0
    return s


class Lattice:
    """One handle of the library: a single lattice or a batch of lattices.

    ``Lattice(nx, ny, tau, theta, ...)`` creates one lattice;
    ``Lattice.batch(specs, ...)`` many that step together.
    """

    def __init__(self, nx=None, ny=None, tau=None, theta=None, rho0=1.0, u0=(0.0, 0.0),
                 seed=1, storage="f32", stream_id=0, ladd=False, moments=False,
                 _handle=None):
        L = lib()
        if _handle is None:
            t = np.ascontiguousarray(tau, dtype=np.float64)
            u = np.ascontiguousarray(u0, dtype=np.float64)
            flags = _flags(ladd, moments)
            _handle = L.flb_create_ex(int(nx), int(ny), _dptr(t), float(theta), float(rho0),
                                      _dptr(u), int(seed), STORAGE[storage], int(stream_id),
                                      flags)
            if not _handle:
                raise FlbError(EINVAL, last_error())
        self._h = _handle
        self.nlattices = L.flb_num_lattices(self._h)
        self._shapes = []
        for i in range(self.nlattices):
            nx_, ny_, nk_ = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _check(L.flb_lattice_info(self._h, i, ctypes.byref(nx_), ctypes.byref(ny_),
                                      ctypes.byref(nk_)))
            self._shapes.append((nx_.value, ny_.value, nk_.value))
        self.nx, self.ny, self.nkx = self._shapes[0]
        self.nkinds = L.flb_num_kinds(self._h)

    @classmethod
    def batch(cls, specs, seed=1, storage="f32", ladd=False, moments=False):
        """specs: list of dicts with nx, ny, tau, theta, rho0, u0, stream_id."""
        arr = (LatticeSpec * len(specs))()
        for i, s in enumerate(specs):
            arr[i] = make_spec(s["nx"], s["ny"], s["tau"], s["theta"], s.get("rho0", 1.0),
                               s.get("u0", (0.0, 0.0)), s.get("stream_id", i))
        h = lib().flb_create_batch(len(specs), arr, int(seed), STORAGE[storage],
                                   _flags(ladd, moments))
        if not h:
            raise FlbError(EINVAL, last_error())
        return cls(_handle=h)

    def close(self):
        if getattr(self, "_h", None):
            lib().flb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def shape(self, lattice=0):
        return self._shapes[lattice]

    # --- stepping -------------------------------------------------------
    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
        ptr = getattr(stream, "cuda_stream", stream)
        _check(lib().flb_set_stream(self._h, ctypes.c_void_p(ptr) if ptr else None))

    def synchronize(self):
        _check(lib().flb_synchronize(self._h))

    def set_sample_overlap(self, on):
        """Run each correlator sample beside the following steps (True) or
        enqueue it at once (False); results are the same."""
        _check(lib().flb_set_sample_overlap(self._h, int(bool(on))))

    def sample_overlap(self):
        v = lib().flb_get_sample_overlap(self._h)
        _check(min(v, 0))
        return bool(v)

    def set_launch_timing(self, on):
        """Bracket every step-kernel launch enqueued outside a graph with a
        pair of HIP events (see ``launch_timing``)."""
        _check(lib().flb_set_launch_timing(self._h, int(bool(on))))

    def launch_timing(self):
        """(launches, total ms) of the step-kernel launches timed since the
        previous call; synchronises the work stream."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(lib().flb_get_launch_timing(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def launch_timing_kinds(self):
        """As launch_timing, split by the steps a launch took: a list of
        (launches, total ms) for one, two and three steps per launch."""
        n = (ctypes.c_int64 * 3)()
        ms = (ctypes.c_double * 3)()
        _check(lib().flb_get_launch_timing_kinds(self._h, n, ms))
        return [(n[q], ms[q]) for q in range(3)]

    def step(self, n=1):
        _check(lib().flb_step(self._h, int(n)))

    def run(self, nsteps, sample_every=0):
        _check(lib().flb_run(self._h, int(nsteps), int(sample_every)))

    @property
    def t(self):
        return int(lib().flb_get_step(self._h))

    @t.setter
    def t(self, value):
        _check(lib().flb_set_step(self._h, int(value)))

    def set_step_config(self, tile_w, rows, nontemporal):
        _check(lib().flb_set_step_config(self._h, int(tile_w), int(rows), int(nontemporal)))

    def step_config(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().flb_get_step_config(self._h, ctypes.byref(a), ctypes.byref(b),
                                         ctypes.byref(c)))
        return a.value, b.value, bool(c.value)

    def set_time_blocking(self, steps_per_launch, tile_w=64):
        """1: one step per kernel launch; 2 or 3: that many steps per launch
        (the populations cross HBM once per launch), tiles of tile_w x
        1024/tile_w sites (tile_w 32, 64 or 128)."""
        _check(lib().flb_set_time_blocking(self._h, int(steps_per_launch), int(tile_w)))

    def time_blocking(self):
        """(steps per launch, two-step tile width); the width is 0 while
        each lattice has its own (lattice_tiles())."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().flb_get_time_blocking(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_lattice_tiles(self, tile_w):
        """Pairs of steps per launch with each lattice's own tile width (32
        or 64), one entry per lattice."""
        a = np.ascontiguousarray(tile_w, dtype=np.int32)
        if a.shape != (self.nlattices,):
            raise ValueError(f"need {self.nlattices} tile widths, got shape {a.shape}")
        _check(lib().flb_set_lattice_tiles(self._h, a.ctypes.data_as(_i32p)))

    def lattice_tiles(self):
        """Each lattice's two-step tile width in effect."""
        a = np.zeros(self.nlattices, dtype=np.int32)
        _check(lib().flb_get_lattice_tiles(self._h, a.ctypes.data_as(_i32p)))
        return a.tolist()

    def autotune_path(self, nsteps=10, sample_every=10):
        """Tune the step launch shape on whole sampling periods (see
        flb_autotune_path): returns the chosen (tile_w, sites, nontemporal)
        and the whole path's ms per step."""
        ms = ctypes.c_double()
        _check(lib().flb_autotune_path(self._h, int(nsteps), int(sample_every), ctypes.byref(ms)))
        return self.step_config(), ms.value

    def autotune(self, nsteps=10):
        """Time every step-kernel launch shape on this handle, the
        time-blocked ones included, and keep the fastest (state unchanged);
        returns the chosen (tile_w, sites, nontemporal) and its ms per step
        (``time_blocking()`` tells whether pairs of steps won)."""
        ms = ctypes.c_double()
        _check(lib().flb_autotune(self._h, int(nsteps), ctypes.byref(ms)))
        return self.step_config(), ms.value

    def storage_info(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().flb_storage_info(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # --- state ----------------------------------------------------------
    def get_populations(self, lattice=0):
        nx, ny, _ = self._shapes[lattice]
        out = np.empty((9, ny, nx), dtype=np.float64)
        _check(lib().flb_get_populations(self._h, lattice, _dptr(out), out.size))
        return out

    def set_populations(self, f, lattice=0):
        nx, ny, _ = self._shapes[lattice]
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, ny, nx):
            raise ValueError(f"expected shape (9, {ny}, {nx}), got {f.shape}")
        _check(lib().flb_set_populations(self._h, lattice, _dptr(f), f.size))

    def conservation(self, lattice=0):
        out = np.zeros(5)
        _check(lib().flb_conservation(self._h, lattice, _dptr(out)))
        return out

    def sample_conservation(self, lattice=0):
        """The five sums of the state of the most recent correlator sample."""
        out = np.zeros(5)
        _check(lib().flb_sample_conservation(self._h, lattice, _dptr(out)))
        return out

    def conservation_dev(self, out_ptr, lattice=0):
        """Enqueue the five FP64 sums into device memory at out_ptr."""
        _check(lib().flb_conservation_dev(self._h, lattice, ctypes.c_void_p(int(out_ptr))))

    def thermalize(self):
        _check(lib().flb_thermalize(self._h))

    def debug_noise(self, t, site0, nsites, lattice=0):
        w = np.zeros((int(nsites), 4), dtype=np.uint32)
        z = np.zeros((int(nsites), 6), dtype=np.float32)
        _check(lib().flb_debug_noise(self._h, lattice, int(t), int(site0), int(nsites),
                                     w.ctypes.data_as(_u32p), z.ctypes.data_as(_fp)))
        return w, z

    # --- correlators ----------------------------------------------------
    def accumulate(self):
        _check(lib().flb_accumulate_correlators(self._h))

    def reset_correlators(self):
        _check(lib().flb_reset_correlators(self._h))

    def read_correlators(self, lattice=0):
        """(raw FP64 sums [nkinds][ny][nx//2+1], number of samples); nkinds is
        15, or 21 with the moment spectra."""
        nx, ny, nk = self._shapes[lattice]
        out = np.empty((self.nkinds, ny, nk), dtype=np.float64)
        ns = ctypes.c_int64()
        _check(lib().flb_read_correlators(self._h, lattice, _dptr(out), out.size,
                                          ctypes.byref(ns)))
        return out, ns.value

    def read_normalized_raw(self, lattice=0):
        """(normalised kinds [nkinds][ny][nx//2+1] as the library computes
        them, number of samples)."""
        nx, ny, nk = self._shapes[lattice]
        out = np.empty((self.nkinds, ny, nk), dtype=np.float64)
        ns = ctypes.c_int64()
        _check(lib().flb_read_normalized(self._h, lattice, _dptr(out), out.size,
                                         ctypes.byref(ns)))
        return out, ns.value

    def read_normalized(self, lattice=0):
        """The library's normalised correlators by name (``NORMALIZED``):
        S_rho, S_jx, ..., R_uxuy (complex), ..., and S_M3..S_M8 with the
        moment spectra."""
        out, _ = self.read_normalized_raw(lattice)
        return _named(out, NORMALIZED)

    def flush_correlators(self):
        """Enqueue the work still owed to the sums (a waiting sample, the
        stashed samples' products) without waiting for it."""
        _check(lib().flb_flush_correlators(self._h))


def _named(arr, names):
    """Named views of a kinds-first array: one kind, or a Re/Im pair packed
    as one complex array; names past the array's kinds are left out."""
    out = {}
    for e in names:
        if e[-1] >= arr.shape[0]:
            continue
        out[e[0]] = arr[e[1]] if len(e) == 2 else arr[e[1]] + 1j * arr[e[2]]
    return out


def _flags(ladd, moments):
    return (FLAG_NO_GHOST_NOISE if ladd else 0) | (FLAG_MOMENT_SPECTRA if moments else 0)


# ---------------------------------------------------------------------------
# Other velocity sets (include/flb_dq.h)
# ---------------------------------------------------------------------------
DQ_MODELS = {"D1Q3": 13, "D2Q9": 29, "D3Q15": 315}


def dq_tables(model):
    """(D, v[Q][3], w[Q], m[Q][Q]) of a velocity set, as the library builds them."""
    D, Q = ctypes.c_int32(), ctypes.c_int32()
    v = np.zeros(45, dtype=np.int32)
    w = np.zeros(15)
    m = np.zeros(225)
    _check(lib().flb_dq_tables(DQ_MODELS[model], ctypes.byref(D), ctypes.byref(Q),
                               v.ctypes.data_as(_i32p), _dptr(w), _dptr(m)))
    q = Q.value
    return D.value, v[:3 * q].reshape(q, 3).copy(), w[:q].copy(), m[:q * q].reshape(q, q).copy()


class DqLattice:
    """One periodic lattice of another velocity set (D1Q3, D2Q9 or D3Q15) on
    the GPU; sides (nx, ny, nz) with the unused ones 1."""

    def __init__(self, model, sides, tau, theta, rho0=1.0, u0=(0.0, 0.0, 0.0), seed=1,
                 stream_id=0, ladd=False):
        L = lib()
        sides = list(sides) + [1] * (3 - len(sides))
        n = np.ascontiguousarray(sides, dtype=np.int32)
        t = np.ascontiguousarray(tau, dtype=np.float64)
        u = np.ascontiguousarray(list(u0) + [0.0] * (3 - len(u0)), dtype=np.float64)
        h = L.flb_dq_create(DQ_MODELS[model], n.ctypes.data_as(_i32p), _dptr(t), float(theta),
                            float(rho0), _dptr(u), int(seed), int(stream_id),
                            FLAG_NO_GHOST_NOISE if ladd else 0)
        if not h:
            raise FlbError(EINVAL, last_error())
        self._h = h
        self.model = model
        self.sides = tuple(int(x) for x in sides)
        D, Q, K = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.flb_dq_info(h, ctypes.byref(D), ctypes.byref(Q), ctypes.byref(K)))
        self.D, self.Q, self.nkinds = D.value, Q.value, K.value

    def close(self):
        if getattr(self, "_h", None):
            lib().flb_dq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self):
        return int(lib().flb_dq_get_step(self._h))

    def set_stream(self, stream):
        ptr = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", 0)
        _check(lib().flb_dq_set_stream(self._h, ctypes.c_void_p(ptr)))

    def synchronize(self):
        _check(lib().flb_dq_synchronize(self._h))

    def step(self, n=1):
        _check(lib().flb_dq_step(self._h, int(n)))

    def run(self, nsteps, sample_every=0):
        _check(lib().flb_dq_run(self._h, int(nsteps), int(sample_every)))

    def thermalize(self):
        _check(lib().flb_dq_thermalize(self._h))

    def accumulate(self):
        _check(lib().flb_dq_accumulate(self._h))

    def reset_correlators(self):
        _check(lib().flb_dq_reset(self._h))

    def read_correlators(self):
        """(raw FP64 sums [nkinds][nz][ny][nx//2+1], number of samples)."""
        nx, ny, nz = self.sides
        out = np.empty((self.nkinds, nz, ny, nx // 2 + 1))
        ns = ctypes.c_int64()
        _check(lib().flb_dq_read(self._h, _dptr(out), out.size, ctypes.byref(ns)))
        return out, ns.value

    def read_normalized(self):
        """The library's normalised structure factors by name: S_rho,
        S_j<a>, S_u<a>, R_uxuy (complex, D >= 2), S_M<a> for the
        non-conserved moments."""
        nx, ny, nz = self.sides
        out = np.empty((self.nkinds, nz, ny, nx // 2 + 1))
        ns = ctypes.c_int64()
        _check(lib().flb_dq_read_normalized(self._h, _dptr(out), out.size, ctypes.byref(ns)))
        return _named(out, dq_kind_names(self.D, self.Q))

    def get_populations(self):
        nx, ny, nz = self.sides
        out = np.empty((self.Q, nz, ny, nx))
        _check(lib().flb_dq_get_populations(self._h, _dptr(out), out.size))
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        nx, ny, nz = self.sides
        assert f.size == self.Q * nx * ny * nz
        _check(lib().flb_dq_set_populations(self._h, _dptr(f), f.size))

    def conservation(self):
        out = np.zeros(4)
        _check(lib().flb_dq_conservation(self._h, _dptr(out)))
        return out


def dq_kind_names(D, Q):
    """Names and kind indices of the flb_dq.h kinds in ``read_normalized``."""
    ax = "xyz"
    names = [("S_rho", 0)]
    k = 1
    for a in range(D):
        names.append(("S_j" + ax[a], k))
        k += 1
    for a in range(D):
        names.append(("S_u" + ax[a], k))
        k += 1
    if D >= 2:
        names.append(("R_uxuy", k, k + 1))
        k += 2
    for a in range(D + 1, Q):
        names.append(("S_M%d" % a, k))
        k += 1
    return tuple(names)
