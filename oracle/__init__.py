"""FP64 CPU oracle for the fluctuating ideal-gas D2Q9 lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_1010_1233_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, libm); this module only
marshals numpy arrays through ctypes.  Each function names the passage of
Kaehler & Wagner (Sec. 2-3, Eqs. 1-12) that it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_DQ = os.path.join(_HERE, "oracle_ddqq.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
             "-Wall", "-Wextra", "-o", tmp, _SRC, _SRC_DQ, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(ctypes.Structure):
    """Mirror of ``oracle_cfg`` in oracle.c."""
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau", ctypes.c_double * 9),
        ("theta", ctypes.c_double), ("rho0", ctypes.c_double),
        ("u0x", ctypes.c_double), ("u0y", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
        ("ladd", ctypes.c_int),
    ]


class DqCfg(ctypes.Structure):
    """Mirror of ``oracle_dq_cfg`` in oracle_ddqq.c."""
    _fields_ = [
        ("model", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("tau", ctypes.c_double * 15),
        ("theta", ctypes.c_double), ("rho0", ctypes.c_double),
        ("u0", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
        ("ladd", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_tables.argtypes = [_dp, _dp, _dp, _ip]
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_noise_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.oracle_normals_from_words.argtypes = [_u32p, _dp]
        L.oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [_dp]
        L.oracle_moments.argtypes = [_dp, _dp]
        L.oracle_equilibrium_moments.argtypes = [ctypes.c_double] * 3 + [_dp]
        L.oracle_noise_amplitudes.argtypes = [_dp, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, _dp]
        L.oracle_collide_site.argtypes = [_dp, _dp, _dp, _dp, _dp]
        cp = ctypes.POINTER(Cfg)
        L.oracle_init.argtypes = [cp, _dp]
        L.oracle_step.argtypes = [cp, _dp, _dp, ctypes.c_uint32]
        L.oracle_conservation.argtypes = [cp, _dp, _dp]
        L.oracle_thermalize.argtypes = [cp, _dp]
        L.oracle_dft2.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int]
        L.oracle_nkx.argtypes = [ctypes.c_int]
        L.oracle_nkx.restype = ctypes.c_int
        L.oracle_sample.argtypes = [cp, _dp, _dp]
        L.oracle_sample_moments.argtypes = [cp, _dp, _dp]
        L.oracle_run.argtypes = [cp, _dp, _dp, ctypes.c_uint32, ctypes.c_int64,
                                 ctypes.c_int, _dp, _dp]
        L.oracle_run.restype = ctypes.c_int64
        dq = ctypes.POINTER(DqCfg)
        L.oracle_dft3.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_dq_tables.argtypes = [ctypes.c_int, _ip, _ip, _ip, _dp, _dp]
        L.oracle_dq_nkinds.argtypes = [ctypes.c_int]
        L.oracle_dq_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.oracle_dq_init.argtypes = [dq, _dp]
        L.oracle_dq_step.argtypes = [dq, _dp, _dp, ctypes.c_uint32]
        L.oracle_dq_conservation.argtypes = [dq, _dp, _dp]
        L.oracle_dq_thermalize.argtypes = [dq, _dp]
        L.oracle_dq_sample.argtypes = [dq, _dp, _dp]
        L.oracle_dq_run.argtypes = [dq, _dp, _dp, ctypes.c_uint32, ctypes.c_int64,
                                    ctypes.c_int, _dp]
        L.oracle_dq_run.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


NKINDS = 15
KINDS = ("rho_rho", "jx_jx", "jy_jy", "ux_ux", "uy_uy",
         "re_ux_uy", "im_ux_uy", "re_rho_jx", "im_rho_jx", "re_rho_jy", "im_rho_jy",
         "re_rho_ux", "im_rho_ux", "re_rho_uy", "im_rho_uy")


def tables():
    """(m[a][i], n[i][a], w[i], v[i][2]) of Eq. (9) and the text after it."""
    m = np.zeros(81); n = np.zeros(81); w = np.zeros(9); v = np.zeros(18, dtype=np.int32)
    lib().oracle_tables(_p(m), _p(n), _p(w), _p(v, _ip))
    return m.reshape(9, 9), n.reshape(9, 9), w, v.reshape(9, 2)


def philox(ctr, key):
    """Philox4x32-10 of one 128-bit counter under one 64-bit key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(o, _u32p))
    return o


def noise_words(seed, stream_id, t, site, d=0):
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_noise_words(seed, stream_id, t, site, d, _p(o, _u32p))
    return o


def normals_from_words(w):
    w = np.ascontiguousarray(w, dtype=np.uint32)
    z = np.zeros(6)
    lib().oracle_normals_from_words(_p(w, _u32p), _p(z))
    return z


def equilibrium(rho, ux, uy):
    """Eq. (2), c = 1."""
    f = np.zeros(9)
    lib().oracle_equilibrium(rho, ux, uy, _p(f))
    return f


def moments(f):
    """Eq. (3)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    M = np.zeros(9)
    lib().oracle_moments(_p(f), _p(M))
    return M


def equilibrium_moments(rho, ux, uy):
    """Eq. (10)."""
    M = np.zeros(9)
    lib().oracle_equilibrium_moments(rho, ux, uy, _p(M))
    return M


def noise_amplitudes(tau, theta, rho0, ladd=False):
    """Eq. (8) with variance scale mu = 3 theta."""
    t = np.ascontiguousarray(tau, dtype=np.float64)
    s = np.zeros(9)
    lib().oracle_noise_amplitudes(_p(t), theta, rho0, int(bool(ladd)), _p(s))
    return s


def collide_site(f, tau, sigma, z):
    """Eq. (5) at one site: post-collision populations."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    o = np.zeros(9)
    lib().oracle_collide_site(_p(f), _p(t), _p(s), _p(zz), _p(o))
    return o


def dft2(x):
    """2-D discrete transform X(k) = sum_x x(x) exp(-i k.x) of an (ny, nx) array."""
    x = np.asarray(x, dtype=np.complex128)
    ny, nx = x.shape
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    lib().oracle_dft2(_p(re), _p(im), nx, ny)
    return re + 1j * im


def nkx(nx):
    return lib().oracle_nkx(nx)


class Lattice:
    """A periodic nx x ny lattice evolved by the oracle in FP64.

    ``f`` is the pre-collision state f[i][y][x]; ``t`` the number of steps
    taken (the noise counter of the next step).
    """

    def __init__(self, nx, ny, tau, theta, rho0=1.0, u0=(0.0, 0.0), seed=1,
                 stream_id=0, ladd=False, thermalize=False, moments=False):
        self.cfg = Cfg()
        self.cfg.nx, self.cfg.ny = int(nx), int(ny)
        for a in range(9):
            self.cfg.tau[a] = float(tau[a])
        self.cfg.theta, self.cfg.rho0 = float(theta), float(rho0)
        self.cfg.u0x, self.cfg.u0y = float(u0[0]), float(u0[1])
        self.cfg.seed, self.cfg.stream_id = int(seed), int(stream_id)
        self.cfg.ladd = int(bool(ladd))
        self.nx, self.ny = int(nx), int(ny)
        self.f = np.zeros((9, self.ny, self.nx))
        self._tmp = np.zeros_like(self.f)
        lib().oracle_init(ctypes.byref(self.cfg), _p(self.f))
        if thermalize:
            lib().oracle_thermalize(ctypes.byref(self.cfg), _p(self.f))
        self.t = 0
        self.acc = np.zeros((NKINDS, self.ny, nkx(self.nx)))
        # |dM^a(k)|^2 of the six non-conserved moments, a = 3..8 (if asked for)
        self.acc_m = np.zeros((6, self.ny, nkx(self.nx))) if moments else None
        self.nsamples = 0

    @property
    def V(self):
        return self.nx * self.ny

    def set_populations(self, f):
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self.f[...] = f

    def step(self, n=1):
        for _ in range(n):
            lib().oracle_step(ctypes.byref(self.cfg), _p(self.f), _p(self._tmp), self.t)
            self.f, self._tmp = self._tmp, self.f
            self.t += 1

    def run(self, nsteps, sample_every=0):
        """nsteps steps, sampling at every t with t % sample_every == 0."""
        ns = lib().oracle_run(ctypes.byref(self.cfg), _p(self.f), _p(self._tmp), self.t,
                              int(nsteps), int(sample_every),
                              _p(self.acc) if sample_every > 0 else None,
                              _p(self.acc_m) if sample_every > 0 and self.acc_m is not None
                              else None)
        self.t += int(nsteps)
        self.nsamples += int(ns)
        return int(ns)

    def sample(self):
        lib().oracle_sample(ctypes.byref(self.cfg), _p(self.f), _p(self.acc))
        if self.acc_m is not None:
            lib().oracle_sample_moments(ctypes.byref(self.cfg), _p(self.f), _p(self.acc_m))
        self.nsamples += 1

    def conservation(self):
        o = np.zeros(5)
        lib().oracle_conservation(ctypes.byref(self.cfg), _p(self.f), _p(o))
        return o

    def thermalize(self):
        lib().oracle_thermalize(ctypes.byref(self.cfg), _p(self.f))


def normalized(acc, nsamples, nx, ny, theta, rho0):
    """Normalised correlators from raw sums, in the oracle's own arithmetic.

    S(rho)  = <|rho_k|^2> / (V mu rho0)        (Eq. 11 with N^rho; mu = 3 theta)
    S(j_a)  = <|j_a,k|^2> / (V rho0 theta)
    S(u_a)  = rho0 <|u_a,k|^2> / (V theta)     (N^{u_a} = 1/(rho0 V kT))
    R(ux,uy) = rho0 <ux uy*> / (V theta)       (Eq. 12)
    R(rho,j_a) = <rho j_a*> / (V mu rho0 c_s),  R(rho,u_a) = <rho u_a*> / (V mu c_s)
    """
    V = nx * ny
    mu = 3.0 * theta
    cs = 1.0 / np.sqrt(3.0)
    m = acc / max(nsamples, 1)
    out = {
        "S_rho": m[0] / (V * mu * rho0),
        "S_jx": m[1] / (V * rho0 * theta),
        "S_jy": m[2] / (V * rho0 * theta),
        "S_ux": rho0 * m[3] / (V * theta),
        "S_uy": rho0 * m[4] / (V * theta),
        "R_uxuy": rho0 * (m[5] + 1j * m[6]) / (V * theta),
        "R_rhojx": (m[7] + 1j * m[8]) / (V * mu * rho0 * cs),
        "R_rhojy": (m[9] + 1j * m[10]) / (V * mu * rho0 * cs),
        "R_rhoux": (m[11] + 1j * m[12]) / (V * mu * cs),
        "R_rhouy": (m[13] + 1j * m[14]) / (V * mu * cs),
    }
    return out


def normalized_moments(acc_m, nsamples, nx, ny, theta, rho0):
    """S(M^a) = <|dM^a_k|^2> / (V mu rho0), a = 3..8 (Eq. 11: every moment of
    the Hermite-normalised basis has per-site variance mu rho0 at rest)."""
    V = nx * ny
    mu = 3.0 * theta
    m = acc_m / max(nsamples, 1)
    return {"S_M%d" % a: m[a - 3] / (V * mu * rho0) for a in range(3, 9)}


# ---------------------------------------------------------------------------
# Other velocity sets (D1Q3, D3Q15; D2Q9 through the same generic code)
# ---------------------------------------------------------------------------
DQ_MODELS = {"D1Q3": 13, "D2Q9": 29, "D3Q15": 315}


def dq_tables(model):
    """(D, v[Q][3], w[Q], m[Q][Q]) of a velocity set: the moments are the
    model's velocity polynomials orthonormalised under the weights (Eq. 4)."""
    D, Q = ctypes.c_int(), ctypes.c_int()
    v = np.zeros(45, dtype=np.int32)
    w = np.zeros(15)
    m = np.zeros(225)
    rc = lib().oracle_dq_tables(DQ_MODELS[model], ctypes.byref(D), ctypes.byref(Q),
                                _p(v, _ip), _p(w), _p(m))
    assert rc == 0
    q = Q.value
    return D.value, v[:3 * q].reshape(q, 3), w[:q].copy(), m[:q * q].reshape(q, q).copy()


def dq_equilibrium(model, rho, u):
    """Eq. (2) (c = 1) on the velocity set of `model`."""
    u = np.ascontiguousarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64)
    f0 = np.zeros(15)
    assert lib().oracle_dq_equilibrium(DQ_MODELS[model], float(rho), _p(u), _p(f0)) == 0
    return f0[:len(dq_tables(model)[2])].copy()


def dq_nkinds(model):
    return int(lib().oracle_dq_nkinds(DQ_MODELS[model]))


def dft3(x):
    """In-place-style 3-D transform of a complex array of shape (nz, ny, nx)."""
    x = np.asarray(x, dtype=complex)
    nz, ny, nx = x.shape
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    lib().oracle_dft3(_p(re), _p(im), nx, ny, nz)
    return re + 1j * im


class DqLattice:
    """A periodic lattice of the generic oracle: sides (nx, ny, nz) with the
    unused ones 1; ``f`` is f[i][z][y][x], pre-collision."""

    def __init__(self, model, sides, tau, theta, rho0=1.0, u0=(0.0, 0.0, 0.0), seed=1,
                 stream_id=0, ladd=False, thermalize=False):
        self.model = model
        self.D, v, w, _ = dq_tables(model)
        self.Q = len(w)
        sides = list(sides) + [1] * (3 - len(sides))
        self.cfg = DqCfg()
        self.cfg.model = DQ_MODELS[model]
        for a in range(3):
            self.cfg.n[a] = int(sides[a])
        for a in range(self.Q):
            self.cfg.tau[a] = float(tau[a])
        self.cfg.theta, self.cfg.rho0 = float(theta), float(rho0)
        u0 = list(u0) + [0.0] * (3 - len(u0))
        for a in range(3):
            self.cfg.u0[a] = float(u0[a])
        self.cfg.seed, self.cfg.stream_id = int(seed), int(stream_id)
        self.cfg.ladd = int(bool(ladd))
        self.sides = tuple(sides)
        nx, ny, nz = self.sides
        self.f = np.zeros((self.Q, nz, ny, nx))
        self._tmp = np.zeros_like(self.f)
        lib().oracle_dq_init(ctypes.byref(self.cfg), _p(self.f))
        if thermalize:
            self.thermalize()
        self.t = 0
        self.nkinds = dq_nkinds(model)
        self.acc = np.zeros((self.nkinds, nz, ny, nx // 2 + 1))
        self.nsamples = 0

    def set_populations(self, f):
        self.f[...] = np.asarray(f, dtype=np.float64).reshape(self.f.shape)

    def step(self, n=1):
        for _ in range(n):
            lib().oracle_dq_step(ctypes.byref(self.cfg), _p(self.f), _p(self._tmp), self.t)
            self.f, self._tmp = self._tmp, self.f
            self.t += 1

    def run(self, nsteps, sample_every=0):
        ns = lib().oracle_dq_run(ctypes.byref(self.cfg), _p(self.f), _p(self._tmp), self.t,
                                 int(nsteps), int(sample_every),
                                 _p(self.acc) if sample_every > 0 else None)
        self.t += int(nsteps)
        self.nsamples += int(ns)
        return int(ns)

    def sample(self):
        lib().oracle_dq_sample(ctypes.byref(self.cfg), _p(self.f), _p(self.acc))
        self.nsamples += 1

    def conservation(self):
        o = np.zeros(4)
        lib().oracle_dq_conservation(ctypes.byref(self.cfg), _p(self.f), _p(o))
        return o

    def thermalize(self):
        lib().oracle_dq_thermalize(ctypes.byref(self.cfg), _p(self.f))


def dq_kind_names(D, Q):
    """Names of the generic oracle's correlator kinds, in order."""
    ax = "xyz"
    names = ["rho_rho"] + [f"j{ax[a]}_j{ax[a]}" for a in range(D)]
    names += [f"u{ax[a]}_u{ax[a]}" for a in range(D)]
    if D >= 2:
        names += ["re_ux_uy", "im_ux_uy"]
    names += [f"M{a}_M{a}" for a in range(D + 1, Q)]
    return names


def dq_normalized(acc, nsamples, D, Q, sides, theta, rho0):
    """Structure factors of the generic kinds: S(rho) = <|rho_k|^2>/(V mu rho0),
    S(j_a) = <|j_a|^2>/(V rho0 theta), S(u_a) = rho0 <|u_a|^2>/(V theta),
    R(u_x,u_y) = rho0 <u_x u_y*>/(V theta), S(M^a) = <|M^a|^2>/(V mu rho0)."""
    V = float(np.prod(sides))
    mu = 3.0 * theta
    m = acc / max(nsamples, 1)
    ax = "xyz"
    out = {"S_rho": m[0] / (V * mu * rho0)}
    k = 1
    for a in range(D):
        out["S_j" + ax[a]] = m[k] / (V * rho0 * theta)
        k += 1
    for a in range(D):
        out["S_u" + ax[a]] = rho0 * m[k] / (V * theta)
        k += 1
    if D >= 2:
        out["R_uxuy"] = rho0 * (m[k] + 1j * m[k + 1]) / (V * theta)
        k += 2
    for a in range(D + 1, Q):
        out["S_M%d" % a] = m[k] / (V * mu * rho0)
        k += 1
    return out
