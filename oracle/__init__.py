"""FP64 CPU oracle of the fluctuating lattice Boltzmann equation: the
two-species model (``Sim``) and its N-species form (``MultiSim``, Apps. C
and D).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path (the HIP
library and its binding) never does.  It shares no code with the GPU path.

The steppers are plain C (``flbe_oracle.c``, ``flbe_multi.c``), called through ctypes.  The
observables that are plain definitions (the structure factor of Sec. VI A and
the mode moments of Eq. (80)) are written here with numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, n) for n in ("flbe_oracle.c", "flbe_multi.c")]
_HDR = os.path.join(_HERE, "flbe_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

D2Q9, D3Q19 = 0, 1
MAX_NORMALS = 128  # ORC_MAX_NORMALS
NOISE_OFF, NOISE_NO_SDF = 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into ``liboracle.so``."""
    newest = max(os.path.getmtime(f) for f in _SRCS + [_HDR])
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("tau", ctypes.c_double * 2), ("tau_d", ctypes.c_double),
                ("G", ctypes.c_double), ("kT", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


MAX_SPECIES = 4


class _MultiParams(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nspecies", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("tau", ctypes.c_double * MAX_SPECIES),
                ("tau_d", ctypes.c_double), ("G", (ctypes.c_double * MAX_SPECIES) * MAX_SPECIES),
                ("kT", ctypes.c_double), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_basis.restype = ctypes.c_int
        L.orc_basis.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int), dp, dp, dp]
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int, dp]
        L.orc_normals.restype = ctypes.c_int
        L.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int, dp]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Params)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_num_sites.restype = ctypes.c_int64
        L.orc_num_sites.argtypes = [ctypes.c_void_p]
        L.orc_current_step.restype = ctypes.c_int64
        L.orc_current_step.argtypes = [ctypes.c_void_p]
        L.orc_init_density.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_set_populations.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64]
        L.orc_get_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_moments.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_collide_site.argtypes = [ctypes.c_void_p, ctypes.c_int64, dp]
        L.orc_health.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_multi_create.restype = ctypes.c_void_p
        L.orc_multi_create.argtypes = [ctypes.POINTER(_MultiParams)]
        L.orc_multi_destroy.argtypes = [ctypes.c_void_p]
        L.orc_multi_current_step.restype = ctypes.c_int64
        L.orc_multi_current_step.argtypes = [ctypes.c_void_p]
        L.orc_multi_init_density.argtypes = [ctypes.c_void_p, dp]
        L.orc_multi_set_populations.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64]
        L.orc_multi_get_populations.argtypes = [ctypes.c_void_p, dp]
        L.orc_multi_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_multi_moments.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_multi_collide_site.argtypes = [ctypes.c_void_p, ctypes.c_int64, dp]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def basis(lattice: int):
    """(c [Q,3] int, w [Q], T [Q,Q] (row = mode), N [Q]) of the oracle's lattice."""
    L = lib()
    D = ctypes.c_int()
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    T = np.zeros(19 * 19)
    N = np.zeros(19)
    Q = L.orc_basis(lattice, ctypes.byref(D), c, _dp(w), _dp(T), _dp(N))
    cc = np.array(c[: 3 * Q], dtype=np.int64).reshape(Q, 3)
    return cc, w[:Q].copy(), T[: Q * Q].reshape(Q, Q).copy(), N[:Q].copy(), D.value


def philox(ctr, key):
    L = lib()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def uniforms(seed: int, site: int, step: int, n: int) -> np.ndarray:
    u = np.zeros(n)
    lib().orc_uniforms(seed, site, step, n, _dp(u))
    return u


def normals(seed: int, site: int, step: int, K: int) -> np.ndarray:
    z = np.zeros(max(K, 1))
    if lib().orc_normals(seed, site, step, K, _dp(z)) != 0:
        raise ValueError(f"orc_normals: K = {K} outside [0, {MAX_NORMALS}]")
    return z[:K]


@dataclass
class Params:
    lattice: int = D2Q9
    nx: int = 64
    ny: int = 64
    nz: int = 1
    tau: tuple = (1.0, 1.0)
    tau_d: float = 1.0
    G: float = 0.0
    kT: float = 0.0
    seed: int = 1
    flags: int = 0


class Sim:
    """The oracle stepper.  Populations are pre-collision f_bar, shaped
    [2, Q, nz, ny, nx] (x fastest)."""

    def __init__(self, p: Params):
        L = lib()
        cp = _Params(p.lattice, p.nx, p.ny, p.nz, (ctypes.c_double * 2)(*p.tau), p.tau_d, p.G,
                     p.kT, p.seed, p.flags)
        h = L.orc_create(ctypes.byref(cp))
        if not h:
            raise ValueError(f"oracle rejected parameters {p}")
        self._h = h
        self.p = p
        self.c, self.w, self.T, self.N, self.D = basis(p.lattice)
        self.Q = len(self.w)
        self.shape = (p.nz, p.ny, p.nx)
        self.nsites = p.nx * p.ny * p.nz

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def step_count(self) -> int:
        return lib().orc_current_step(self._h)

    def init_density(self, rho1, rho2):
        r1 = np.ascontiguousarray(np.broadcast_to(rho1, self.shape), dtype=np.float64)
        r2 = np.ascontiguousarray(np.broadcast_to(rho2, self.shape), dtype=np.float64)
        if lib().orc_init_density(self._h, _dp(r1), _dp(r2)) != 0:
            raise RuntimeError("orc_init_density failed")

    def set_populations(self, f, step: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == 2 * self.Q * self.nsites
        if lib().orc_set_populations(self._h, _dp(f), step) != 0:
            raise RuntimeError("orc_set_populations failed")

    def populations(self) -> np.ndarray:
        f = np.zeros(2 * self.Q * self.nsites)
        lib().orc_get_populations(self._h, _dp(f))
        return f.reshape(2, self.Q, *self.shape)

    def step(self, n: int = 1):
        if lib().orc_step(self._h, n) != 0:
            raise RuntimeError("orc_step failed")

    def moments(self):
        """rho [2, *shape], j_bar [2, D, *shape], F [2, D, *shape] of the stored state."""
        rho = np.zeros(2 * self.nsites)
        j = np.zeros(2 * self.D * self.nsites)
        F = np.zeros(2 * self.D * self.nsites)
        lib().orc_moments(self._h, _dp(rho), _dp(j), _dp(F))
        return (rho.reshape(2, *self.shape), j.reshape(2, self.D, *self.shape),
                F.reshape(2, self.D, *self.shape))

    def collide_site(self, site: int) -> np.ndarray:
        out = np.zeros(2 * self.Q)
        if lib().orc_collide_site(self._h, int(site), _dp(out)) != 0:
            raise RuntimeError("orc_collide_site failed")
        return out.reshape(2, self.Q)

    def health(self):
        c = (ctypes.c_int64 * 2)()
        lib().orc_health(self._h, c)
        return int(c[0]), int(c[1])

    # --- observables that are plain definitions --------------------------------
    def mode_moments(self) -> np.ndarray:
        """m_a = sum_i T_ai f_bar_i (Eq. (80)) of the stored state, [2, Q, *shape]."""
        f = self.populations().reshape(2, self.Q, -1)
        m = np.einsum("ai,sin->san", self.T, f)
        return m.reshape(2, self.Q, *self.shape)


@dataclass
class MultiParams:
    """N species (2..4); G is the symmetric matrix of pair couplings (Eq. (87)
    with one coupling per pair)."""
    lattice: int = D2Q9
    nspecies: int = 3
    nx: int = 16
    ny: int = 16
    nz: int = 1
    tau: tuple = (1.0, 1.0, 1.0)
    tau_d: float = 1.0
    G: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    kT: float = 0.0
    seed: int = 1
    flags: int = 0


class MultiSim:
    """The N-species oracle stepper; populations shaped [N, Q, nz, ny, nx]."""

    def __init__(self, p: MultiParams):
        L = lib()
        n = p.nspecies
        tau = list(p.tau) + [1.0] * (MAX_SPECIES - len(p.tau))
        G = np.zeros((MAX_SPECIES, MAX_SPECIES))
        G[:n, :n] = np.asarray(p.G, dtype=np.float64)
        Gc = ((ctypes.c_double * MAX_SPECIES) * MAX_SPECIES)()
        for a in range(MAX_SPECIES):
            for b in range(MAX_SPECIES):
                Gc[a][b] = G[a, b]
        cp = _MultiParams(p.lattice, n, p.nx, p.ny, p.nz, (ctypes.c_double * MAX_SPECIES)(*tau), p.tau_d, Gc,
                          p.kT, p.seed, p.flags)
        h = L.orc_multi_create(ctypes.byref(cp))
        if not h:
            raise ValueError(f"oracle rejected parameters {p}")
        self._h = h
        self.p = p
        self.N = n
        self.c, self.w, self.T, self.Nn, self.D = basis(p.lattice)
        self.Q = len(self.w)
        self.shape = (p.nz, p.ny, p.nx)
        self.nsites = p.nx * p.ny * p.nz

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_multi_destroy(h)
            self._h = None

    @property
    def step_count(self) -> int:
        return lib().orc_multi_current_step(self._h)

    def init_density(self, rho):
        """rho: N arrays (or scalars) of the lattice shape."""
        r = np.stack([np.broadcast_to(np.asarray(x, dtype=np.float64), self.shape) for x in rho])
        r = np.ascontiguousarray(r)
        assert r.shape[0] == self.N
        lib().orc_multi_init_density(self._h, _dp(r))

    def set_populations(self, f, step: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == self.N * self.Q * self.nsites
        lib().orc_multi_set_populations(self._h, _dp(f), step)

    def populations(self) -> np.ndarray:
        f = np.zeros(self.N * self.Q * self.nsites)
        lib().orc_multi_get_populations(self._h, _dp(f))
        return f.reshape(self.N, self.Q, *self.shape)

    def step(self, n: int = 1):
        if lib().orc_multi_step(self._h, n) != 0:
            raise RuntimeError("orc_multi_step failed")

    def collide_site(self, site: int) -> np.ndarray:
        """Post-collision f*[N, Q] at one site of the stored state."""
        out = np.zeros(self.N * self.Q)
        if lib().orc_multi_collide_site(self._h, int(site), _dp(out)) != 0:
            raise RuntimeError("orc_multi_collide_site failed")
        return out.reshape(self.N, self.Q)

    def moments(self):
        """rho [N, *shape], j_bar [N, D, *shape], F [N, D, *shape]."""
        rho = np.zeros(self.N * self.nsites)
        j = np.zeros(self.N * self.D * self.nsites)
        F = np.zeros(self.N * self.D * self.nsites)
        lib().orc_multi_moments(self._h, _dp(rho), _dp(j), _dp(F))
        return (rho.reshape(self.N, *self.shape), j.reshape(self.N, self.D, *self.shape),
                F.reshape(self.N, self.D, *self.shape))


def structure_factor(X: np.ndarray, Y: np.ndarray | None = None) -> np.ndarray:
    """S_XY(k) = Re <X_hat(k) conj(Y_hat(k))> / N of one snapshot, with
    X_hat(k) = sum_r dX(r) exp(-i k.r), dX = X - spatial mean, k = 2 pi n / L
    (lattice units, Sec. VI A).  Arrays are shaped like the lattice."""
    if Y is None:
        Y = X
    dX = X - X.mean()
    dY = Y - Y.mean()
    Xh = np.fft.fftn(dX)
    Yh = np.fft.fftn(dY)
    return (Xh * np.conj(Yh)).real / X.size
