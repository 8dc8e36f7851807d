"""Python binding of the fmlb C ABI (include/fmlb.h).

Argument marshalling only: every function below forwards to the entry point of
the same name in the in-tree HIP library ``libfmlb.so``; all lattice work runs
in its kernels.  PyTorch provides device memory and the HIP stream.  There is
no fallback: if the library has not been built the import of the entry points
fails with an error that says so.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMLB_LIBRARY names another build of the same library (e.g. a host-sanitizer build).
LIB_PATH = os.environ.get("FMLB_LIBRARY") or os.path.join(_HERE, "libfmlb.so")

FMLB_OK = 0
FMLB_E_INVALID = -1
FMLB_E_SIZE = -2
FMLB_E_HIP = -3
FMLB_E_STATE = -4
FMLB_E_NULL = -5
FMLB_E_UNSUPPORTED = -6

FMLB_D2Q9, FMLB_D3Q19 = 0, 1
FMLB_F64, FMLB_F32, FMLB_BF16_DEV, FMLB_F16_DEV = 0, 1, 2, 3
FMLB_NOISE_OFF, FMLB_NOISE_NO_SDF, FMLB_ROUND_STOCHASTIC = 1, 2, 4
FMLB_BUF_POPS_A, FMLB_BUF_POPS_B, FMLB_BUF_SCRATCH = 0, 1, 2

LATTICES = {"d2q9": FMLB_D2Q9, "d3q19": FMLB_D3Q19}
STORAGES = {"f64": FMLB_F64, "f32": FMLB_F32, "bf16": FMLB_BF16_DEV, "f16": FMLB_F16_DEV}
SK_NAMES = ["rho1rho1", "rho2rho2", "rho1rho2", "j1j1", "j2j2", "j1j2", "vbvb"]


class fmlb_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("tau", ctypes.c_double * 2),
                ("tau_d", ctypes.c_double), ("G", ctypes.c_double), ("kT", ctypes.c_double),
                ("rho_ref", ctypes.c_double * 2), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


FMLB_MAX_SPECIES = 4


class fmlb_multi_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("nspecies", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double * FMLB_MAX_SPECIES), ("tau_d", ctypes.c_double),
                ("G", (ctypes.c_double * FMLB_MAX_SPECIES) * FMLB_MAX_SPECIES), ("kT", ctypes.c_double),
                ("rho_ref", ctypes.c_double * FMLB_MAX_SPECIES), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class FmlbError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = lib().fmlb_status_string(status).decode()
        extra = f" (hip error {lib().fmlb_last_hip_error()})" if status == FMLB_E_HIP else ""
        super().__init__(f"{fn}: {msg}{extra} [status {status}]")
        self.status = status


_lib = None

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_pp = ctypes.POINTER(fmlb_params)
_mpp = ctypes.POINTER(fmlb_multi_params)

_SIGNATURES = {
    "fmlb_required_bytes": (ctypes.c_size_t, [_pp, ctypes.c_int]),
    "fmlb_create": (ctypes.c_int32, [_pp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "fmlb_destroy": (None, [_vp]),
    "fmlb_init_density": (ctypes.c_int32, [_vp, _dp, _dp]),
    "fmlb_step": (ctypes.c_int32, [_vp, ctypes.c_int64]),
    "fmlb_current_step": (ctypes.c_int64, [_vp]),
    "fmlb_moments": (ctypes.c_int32, [_vp, _dp, _dp]),
    "fmlb_global_sums": (ctypes.c_int32, [_vp, _dp]),
    "fmlb_mode_accumulate": (ctypes.c_int32, [_vp]),
    "fmlb_mode_variances": (ctypes.c_int32, [_vp, _dp, _i64p]),
    "fmlb_sk_accumulate": (ctypes.c_int32, [_vp]),
    "fmlb_sk_accumulate_static": (ctypes.c_int32, [_pp, _vp, _vp, _vp]),
    "fmlb_sk_get": (ctypes.c_int32, [_vp, ctypes.c_int, _dp, _i64p]),
    "fmlb_reset_accumulators": (ctypes.c_int32, [_vp]),
    "fmlb_get_populations": (ctypes.c_int32, [_vp, _dp, ctypes.c_size_t]),
    "fmlb_set_populations": (ctypes.c_int32, [_vp, _dp, ctypes.c_size_t, ctypes.c_int64]),
    "fmlb_save_raw": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t, _i64p]),
    "fmlb_load_raw": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t, ctypes.c_int64]),
    "fmlb_health": (ctypes.c_int32, [_vp, _i64p]),
    "fmlb_set_tile": (ctypes.c_int32, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fmlb_set_counter_offset": (ctypes.c_int32, [_vp, ctypes.c_int64]),
    "fmlb_copy_reference": (ctypes.c_int32, [_vp]),
    "fmlb_bandwidth_reference": (ctypes.c_int32, [_vp, ctypes.c_int, _dp]),
    "fmlb_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "fmlb_last_hip_error": (ctypes.c_int32, []),
    "fmlb_batch_required_bytes": (ctypes.c_size_t, [_pp, ctypes.c_int, ctypes.c_int]),
    "fmlb_batch_create": (ctypes.c_int32, [_pp, ctypes.c_int, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "fmlb_batch_destroy": (None, [_vp]),
    "fmlb_batch_init_density": (ctypes.c_int32, [_vp, ctypes.c_int, _dp, _dp]),
    "fmlb_batch_step": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int]),
    "fmlb_batch_get_populations": (ctypes.c_int32, [_vp, ctypes.c_int, _dp, ctypes.c_size_t]),
    "fmlb_batch_global_sums": (ctypes.c_int32, [_vp, ctypes.c_int, _dp]),
    "fmlb_batch_mode_accumulate": (ctypes.c_int32, [_vp]),
    "fmlb_batch_mode_variances": (ctypes.c_int32, [_vp, ctypes.c_int, _dp, _i64p]),
    "fmlb_batch_reset_modes": (ctypes.c_int32, [_vp]),
    "fmlb_batch_autotune": (ctypes.c_int32, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int)]),
    "fmlb_batch_set_tile": (ctypes.c_int32, [_vp, ctypes.c_int, ctypes.c_int]),
    "fmlb_batch_size": (ctypes.c_int, [_vp]),
    "fmlb_batch_total_sites": (ctypes.c_int64, [_vp]),
    "fmlb_batch_current_step": (ctypes.c_int64, [_vp]),
    "fmlb_multi_required_bytes": (ctypes.c_size_t, [_mpp, ctypes.c_int]),
    "fmlb_multi_create": (ctypes.c_int32, [_mpp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "fmlb_multi_destroy": (None, [_vp]),
    "fmlb_multi_init_density": (ctypes.c_int32, [_vp, _dp]),
    "fmlb_multi_step": (ctypes.c_int32, [_vp, ctypes.c_int64]),
    "fmlb_multi_current_step": (ctypes.c_int64, [_vp]),
    "fmlb_multi_set_tile": (ctypes.c_int32, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fmlb_multi_set_form": (ctypes.c_int32, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fmlb_multi_get_populations": (ctypes.c_int32, [_vp, _dp, ctypes.c_size_t]),
    "fmlb_multi_set_populations": (ctypes.c_int32, [_vp, _dp, ctypes.c_size_t, ctypes.c_int64]),
    "fmlb_multi_moments": (ctypes.c_int32, [_vp, _dp, _dp]),
    "fmlb_multi_global_sums": (ctypes.c_int32, [_vp, _dp]),
}


def lib():
    """The loaded HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, status: int):
    if status != FMLB_OK:
        raise FmlbError(fn, status)


def _f64(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _as_field(x, shape) -> np.ndarray:
    """A scalar broadcast to `shape`, or an array of that many values reshaped."""
    x = np.asarray(x, dtype=np.float64)
    n = int(np.prod(shape))
    if x.size == n:
        return np.ascontiguousarray(x.reshape(shape))
    if x.size == 1:
        return np.full(shape, float(x.reshape(-1)[0]))
    raise ValueError(f"field of {x.size} values for a lattice of shape {shape}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# ---- entry points with the C names (marshalling only) ------------------------

def fmlb_required_bytes(p: fmlb_params, which: int) -> int:
    return lib().fmlb_required_bytes(ctypes.byref(p), which)


def fmlb_create(p: fmlb_params, stream: int, bufs) -> int:
    arr = (_vp * 3)(*[_vp(int(b)) for b in bufs])
    out = _vp()
    _check("fmlb_create", lib().fmlb_create(ctypes.byref(p), _vp(stream), arr, ctypes.byref(out)))
    return out.value


def fmlb_destroy(ctx: int):
    lib().fmlb_destroy(_vp(ctx))


def fmlb_init_density(ctx: int, rho1: np.ndarray, rho2: np.ndarray):
    r1, r2 = _f64(rho1), _f64(rho2)
    _check("fmlb_init_density", lib().fmlb_init_density(_vp(ctx), _ptr(r1), _ptr(r2)))


def fmlb_step(ctx: int, n: int):
    _check("fmlb_step", lib().fmlb_step(_vp(ctx), int(n)))


def fmlb_current_step(ctx: int) -> int:
    return lib().fmlb_current_step(_vp(ctx))


def fmlb_moments(ctx: int, rho: np.ndarray | None, j: np.ndarray | None):
    _check("fmlb_moments", lib().fmlb_moments(_vp(ctx), _ptr(rho) if rho is not None else None,
                                              _ptr(j) if j is not None else None))


def fmlb_global_sums(ctx: int, out: np.ndarray):
    _check("fmlb_global_sums", lib().fmlb_global_sums(_vp(ctx), _ptr(out)))


def fmlb_mode_accumulate(ctx: int):
    _check("fmlb_mode_accumulate", lib().fmlb_mode_accumulate(_vp(ctx)))


def fmlb_mode_variances(ctx: int, out: np.ndarray) -> int:
    n = ctypes.c_int64()
    _check("fmlb_mode_variances", lib().fmlb_mode_variances(_vp(ctx), _ptr(out), ctypes.byref(n)))
    return n.value


def fmlb_sk_accumulate(ctx: int):
    _check("fmlb_sk_accumulate", lib().fmlb_sk_accumulate(_vp(ctx)))


SK_STATIC_MAX_SITES = 1 << 20  # FMLB_SK_STATIC_MAX_SITES


def fmlb_sk_accumulate_static(params, pops: int, acc: int, stream: int):
    """params: fmlb_params; pops, acc, stream: device pointers / HIP stream handle."""
    _check("fmlb_sk_accumulate_static",
           lib().fmlb_sk_accumulate_static(ctypes.byref(params), _vp(pops), _vp(acc), _vp(stream)))


def fmlb_sk_get(ctx: int, which: int, out: np.ndarray) -> int:
    n = ctypes.c_int64()
    _check("fmlb_sk_get", lib().fmlb_sk_get(_vp(ctx), which, _ptr(out), ctypes.byref(n)))
    return n.value


def fmlb_reset_accumulators(ctx: int):
    _check("fmlb_reset_accumulators", lib().fmlb_reset_accumulators(_vp(ctx)))


def fmlb_get_populations(ctx: int, out: np.ndarray):
    _check("fmlb_get_populations", lib().fmlb_get_populations(_vp(ctx), _ptr(out), out.nbytes))


def fmlb_set_populations(ctx: int, f: np.ndarray, step: int):
    f = _f64(f)
    _check("fmlb_set_populations", lib().fmlb_set_populations(_vp(ctx), _ptr(f), f.nbytes, int(step)))


def fmlb_save_raw(ctx: int, out: np.ndarray) -> int:
    step = ctypes.c_int64()
    _check("fmlb_save_raw", lib().fmlb_save_raw(_vp(ctx), _vp(out.ctypes.data), out.nbytes, ctypes.byref(step)))
    return step.value


def fmlb_load_raw(ctx: int, raw: np.ndarray, step: int):
    raw = np.ascontiguousarray(raw)
    _check("fmlb_load_raw", lib().fmlb_load_raw(_vp(ctx), _vp(raw.ctypes.data), raw.nbytes, int(step)))


def fmlb_health(ctx: int):
    c = (ctypes.c_int64 * 2)()
    _check("fmlb_health", lib().fmlb_health(_vp(ctx), c))
    return int(c[0]), int(c[1])


def fmlb_set_counter_offset(ctx: int, site_offset: int):
    _check("fmlb_set_counter_offset", lib().fmlb_set_counter_offset(_vp(ctx), int(site_offset)))


def fmlb_set_tile(ctx: int, tile_x: int, tile_y: int, march: int):
    _check("fmlb_set_tile", lib().fmlb_set_tile(_vp(ctx), tile_x, tile_y, march))


def _params_array(ps):
    arr = (fmlb_params * len(ps))(*ps)
    return arr, ctypes.cast(arr, _pp)


def fmlb_batch_required_bytes(ps, which: int) -> int:
    arr, ptr = _params_array(ps)
    return lib().fmlb_batch_required_bytes(ptr, len(ps), which)


def fmlb_batch_create(ps, stream: int, bufs) -> int:
    arr, ptr = _params_array(ps)
    b = (_vp * 3)(*[_vp(int(x)) for x in bufs])
    out = _vp()
    _check("fmlb_batch_create", lib().fmlb_batch_create(ptr, len(ps), _vp(stream), b, ctypes.byref(out)))
    return out.value


def fmlb_batch_destroy(b: int):
    lib().fmlb_batch_destroy(_vp(b))


def fmlb_batch_size(b: int) -> int:
    return lib().fmlb_batch_size(_vp(b))


def fmlb_batch_total_sites(b: int) -> int:
    return lib().fmlb_batch_total_sites(_vp(b))


def fmlb_batch_current_step(b: int) -> int:
    return lib().fmlb_batch_current_step(_vp(b))


def fmlb_batch_init_density(b: int, r: int, rho1: np.ndarray, rho2: np.ndarray):
    r1, r2 = _f64(rho1), _f64(rho2)
    _check("fmlb_batch_init_density", lib().fmlb_batch_init_density(_vp(b), r, _ptr(r1), _ptr(r2)))


def fmlb_batch_step(b: int, n: int, use_graph: bool):
    _check("fmlb_batch_step", lib().fmlb_batch_step(_vp(b), int(n), 1 if use_graph else 0))


def fmlb_batch_set_tile(b: int, tile_x: int, march: int):
    _check("fmlb_batch_set_tile", lib().fmlb_batch_set_tile(_vp(b), tile_x, march))


def fmlb_batch_autotune(b: int, reps: int):
    tx, ch = ctypes.c_int(), ctypes.c_int()
    _check("fmlb_batch_autotune", lib().fmlb_batch_autotune(_vp(b), reps, ctypes.byref(tx), ctypes.byref(ch)))
    return tx.value, ch.value


def fmlb_batch_get_populations(b: int, r: int, out: np.ndarray):
    _check("fmlb_batch_get_populations", lib().fmlb_batch_get_populations(_vp(b), r, _ptr(out), out.nbytes))


def fmlb_batch_global_sums(b: int, r: int, out: np.ndarray):
    _check("fmlb_batch_global_sums", lib().fmlb_batch_global_sums(_vp(b), r, _ptr(out)))


def fmlb_batch_mode_accumulate(b: int):
    _check("fmlb_batch_mode_accumulate", lib().fmlb_batch_mode_accumulate(_vp(b)))


def fmlb_batch_mode_variances(b: int, r: int, out: np.ndarray) -> int:
    n = ctypes.c_int64()
    _check("fmlb_batch_mode_variances", lib().fmlb_batch_mode_variances(_vp(b), r, _ptr(out), ctypes.byref(n)))
    return n.value


def fmlb_batch_reset_modes(b: int):
    _check("fmlb_batch_reset_modes", lib().fmlb_batch_reset_modes(_vp(b)))


def fmlb_copy_reference(ctx: int):
    _check("fmlb_copy_reference", lib().fmlb_copy_reference(_vp(ctx)))


FMLB_BW_PULL_COPY, FMLB_BW_READ, FMLB_BW_WRITE, FMLB_BW_COPY16 = 0, 1, 2, 3


def fmlb_bandwidth_reference(ctx: int, kind: int) -> float:
    """Launch one bandwidth reference kernel; returns the bytes it moves."""
    b = ctypes.c_double()
    _check("fmlb_bandwidth_reference", lib().fmlb_bandwidth_reference(_vp(ctx), kind, ctypes.byref(b)))
    return b.value


# ---- convenience wrapper: torch-owned buffers, numpy host arrays ------------

def fmlb_multi_required_bytes(p: fmlb_multi_params, which: int) -> int:
    return lib().fmlb_multi_required_bytes(ctypes.byref(p), which)


def fmlb_multi_create(p: fmlb_multi_params, stream: int, bufs) -> int:
    arr = (_vp * 3)(*[_vp(int(b)) for b in bufs])
    out = _vp()
    _check("fmlb_multi_create", lib().fmlb_multi_create(ctypes.byref(p), _vp(stream), arr, ctypes.byref(out)))
    return out.value


def fmlb_multi_destroy(m: int):
    lib().fmlb_multi_destroy(_vp(m))


def fmlb_multi_init_density(m: int, rho: np.ndarray):
    r = _f64(rho)
    _check("fmlb_multi_init_density", lib().fmlb_multi_init_density(_vp(m), _ptr(r)))


def fmlb_multi_step(m: int, n: int):
    _check("fmlb_multi_step", lib().fmlb_multi_step(_vp(m), int(n)))


def fmlb_multi_current_step(m: int) -> int:
    return lib().fmlb_multi_current_step(_vp(m))


def fmlb_multi_set_tile(m: int, tile_x: int, tile_y: int, march: int):
    _check("fmlb_multi_set_tile", lib().fmlb_multi_set_tile(_vp(m), tile_x, tile_y, march))


FMLB_BATCH_PACKED, FMLB_BATCH_PACKED_512 = 1, 2
FMLB_MULTI_AUTO, FMLB_MULTI_TWO_PASS, FMLB_MULTI_FUSED, FMLB_MULTI_ASYNC = 0, 1, 2, 3
MULTI_FORMS = {"auto": FMLB_MULTI_AUTO, "two_pass": FMLB_MULTI_TWO_PASS, "fused": FMLB_MULTI_FUSED,
               "async": FMLB_MULTI_ASYNC}


def fmlb_multi_set_form(m: int, form: int, tile_x: int, tile_y: int, march: int):
    _check("fmlb_multi_set_form", lib().fmlb_multi_set_form(_vp(m), form, tile_x, tile_y, march))


def fmlb_multi_get_populations(m: int, out: np.ndarray):
    _check("fmlb_multi_get_populations", lib().fmlb_multi_get_populations(_vp(m), _ptr(out), out.nbytes))


def fmlb_multi_set_populations(m: int, f: np.ndarray, step: int):
    f = _f64(f)
    _check("fmlb_multi_set_populations", lib().fmlb_multi_set_populations(_vp(m), _ptr(f), f.nbytes, int(step)))


def fmlb_multi_moments(m: int, rho: np.ndarray | None, j: np.ndarray | None):
    _check("fmlb_multi_moments", lib().fmlb_multi_moments(_vp(m), _ptr(rho) if rho is not None else None,
                                                          _ptr(j) if j is not None else None))


def fmlb_multi_global_sums(m: int, out: np.ndarray):
    _check("fmlb_multi_global_sums", lib().fmlb_multi_global_sums(_vp(m), _ptr(out)))


@dataclass
class Params:
    lattice: str = "d2q9"
    storage: str = "f64"
    nx: int = 64
    ny: int = 64
    nz: int = 1
    tau: tuple = (1.0, 1.0)
    tau_d: float = 1.0
    G: float = 0.0
    kT: float = 0.0
    rho_ref: tuple = (1.0, 1.0)
    seed: int = 1
    flags: int = 0

    def c(self) -> fmlb_params:
        return fmlb_params(LATTICES[self.lattice], STORAGES[self.storage], self.nx, self.ny, self.nz,
                           (ctypes.c_double * 2)(*self.tau), self.tau_d, self.G, self.kT,
                           (ctypes.c_double * 2)(*self.rho_ref), self.seed, self.flags)


class Lattice:
    """One lattice on the current CUDA/HIP device.  Device buffers are torch
    uint8 tensors owned by this object; the stream is torch's current stream
    at construction."""

    def __init__(self, p: Params, device=None, stream=None):
        import torch
        self.p = p
        cp = p.c()
        sizes = [fmlb_required_bytes(cp, k) for k in range(3)]
        if min(sizes) == 0:
            raise FmlbError("fmlb_required_bytes", FMLB_E_INVALID)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.bufs = [torch.empty(s, dtype=torch.uint8, device=dev) for s in sizes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = fmlb_create(cp, self.stream.cuda_stream, [b.data_ptr() for b in self.bufs])
        self.Q = 9 if p.lattice == "d2q9" else 19
        self.D = 2 if p.lattice == "d2q9" else 3
        self.shape = (p.nz, p.ny, p.nx)
        self.nsites = p.nx * p.ny * p.nz

    def close(self):
        if getattr(self, "ctx", None):
            fmlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass

    @property
    def step_count(self) -> int:
        return fmlb_current_step(self.ctx)

    def init_density(self, rho1, rho2):
        r1 = np.broadcast_to(np.asarray(rho1, dtype=np.float64), self.shape)
        r2 = np.broadcast_to(np.asarray(rho2, dtype=np.float64), self.shape)
        fmlb_init_density(self.ctx, r1, r2)

    def step(self, n: int = 1):
        fmlb_step(self.ctx, n)

    def moments(self):
        rho = np.empty((2,) + self.shape)
        j = np.empty((2, self.D) + self.shape)
        fmlb_moments(self.ctx, rho, j)
        return rho, j

    def global_sums(self):
        out = np.empty(2 + self.D)
        fmlb_global_sums(self.ctx, out)
        return out

    def populations(self):
        out = np.empty((2, self.Q) + self.shape)
        fmlb_get_populations(self.ctx, out)
        return out

    def set_populations(self, f, step: int = 0):
        fmlb_set_populations(self.ctx, np.asarray(f, dtype=np.float64).reshape(2, self.Q, *self.shape), step)

    def mode_accumulate(self):
        fmlb_mode_accumulate(self.ctx)

    def mode_variances(self):
        out = np.empty((2, self.Q))
        n = fmlb_mode_variances(self.ctx, out)
        return out, n

    def sk_accumulate(self):
        fmlb_sk_accumulate(self.ctx)

    def sk(self, which):
        if isinstance(which, str):
            which = SK_NAMES.index(which)
        out = np.empty(self.shape)
        n = fmlb_sk_get(self.ctx, which, out)
        return out, n

    def reset_accumulators(self):
        fmlb_reset_accumulators(self.ctx)

    def save_raw(self):
        elem = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[self.p.storage]
        out = np.empty(2 * self.Q * self.nsites * elem, dtype=np.uint8)
        step = fmlb_save_raw(self.ctx, out)
        return out, step

    def load_raw(self, raw, step: int):
        fmlb_load_raw(self.ctx, raw, step)

    def health(self):
        return fmlb_health(self.ctx)

    def set_tile(self, tile_x: int = 0, tile_y: int = 0, march: int = 0):
        fmlb_set_tile(self.ctx, tile_x, tile_y, march)

    def set_counter_offset(self, site_offset: int):
        """Noise-counter site offset (mod 2^32) for a lattice that is one slab of a larger one."""
        fmlb_set_counter_offset(self.ctx, site_offset)

    def copy_reference(self):
        """One launch of the roofline reference copy (state unchanged)."""
        fmlb_copy_reference(self.ctx)

    def bandwidth_reference(self, kind: int) -> float:
        """One launch of bandwidth reference `kind` (FMLB_BW_*); returns its bytes."""
        return fmlb_bandwidth_reference(self.ctx, kind)

    def synchronize(self):
        self.stream.synchronize()


class Batch:
    """Many independent D2Q9 FP32 lattices stepped by one launch per step.
    params: a list of Params (lattice "d2q9", storage "f32", nz 1)."""

    def __init__(self, params, device=None, stream=None):
        import torch
        self.params = list(params)
        cps = [p.c() for p in self.params]
        sizes = [fmlb_batch_required_bytes(cps, k) for k in range(3)]
        if min(sizes) == 0:
            raise FmlbError("fmlb_batch_required_bytes", FMLB_E_INVALID)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.bufs = [torch.empty(s, dtype=torch.uint8, device=dev) for s in sizes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.b = fmlb_batch_create(cps, self.stream.cuda_stream, [x.data_ptr() for x in self.bufs])

    def close(self):
        if getattr(self, "b", None):
            fmlb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass

    def __len__(self):
        return fmlb_batch_size(self.b)

    @property
    def total_sites(self) -> int:
        return fmlb_batch_total_sites(self.b)

    @property
    def step_count(self) -> int:
        return fmlb_batch_current_step(self.b)

    def shape(self, r: int):
        return (self.params[r].ny, self.params[r].nx)

    def init_density(self, r: int, rho1, rho2):
        sh = self.shape(r)

        fmlb_batch_init_density(self.b, r, _as_field(rho1, sh), _as_field(rho2, sh))

    def step(self, n: int = 1, use_graph: bool = False):
        fmlb_batch_step(self.b, n, use_graph)

    def set_tile(self, tile_x: int = 0, march: int = 0):
        """tile_x: FMLB_BATCH_PACKED / FMLB_BATCH_PACKED_512 (runs of 256 / 512
        consecutive sites per block, replicas up to 128 / 256 wide), 64, 128
        or 256 (one-row tiles); march: blocks or rows per item; 0 =
        defaults."""
        fmlb_batch_set_tile(self.b, tile_x, march)

    def autotune(self, reps: int = 10):
        """Pick the fastest work-list shape; returns (tile_x, march)."""
        return fmlb_batch_autotune(self.b, reps)

    def populations(self, r: int):
        out = np.empty((2, 9, 1) + self.shape(r))
        fmlb_batch_get_populations(self.b, r, out)
        return out

    def global_sums(self, r: int):
        out = np.empty(4)
        fmlb_batch_global_sums(self.b, r, out)
        return out

    def mode_accumulate(self):
        fmlb_batch_mode_accumulate(self.b)

    def mode_variances(self, r: int):
        out = np.empty((2, 9))
        n = fmlb_batch_mode_variances(self.b, r, out)
        return out, n

    def reset_modes(self):
        fmlb_batch_reset_modes(self.b)

    def synchronize(self):
        self.stream.synchronize()


@dataclass
class MultiParams:
    """N species (2..4), the multicomponent model; G: symmetric N x N pair
    couplings."""
    lattice: str = "d2q9"
    storage: str = "f64"
    nspecies: int = 3
    nx: int = 32
    ny: int = 32
    nz: int = 1
    tau: tuple = (1.0, 1.0, 1.0)
    tau_d: float = 1.0
    G: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    kT: float = 0.0
    rho_ref: tuple = (1.0, 1.0, 1.0)
    seed: int = 1
    flags: int = 0

    def c(self) -> fmlb_multi_params:
        n = self.nspecies  # passed as given: the library rejects values outside 2..4
        M = FMLB_MAX_SPECIES
        k = max(0, min(n, M))
        G = ((ctypes.c_double * M) * M)()
        for a in range(k):
            for b in range(k):
                G[a][b] = float(self.G[a][b])
        pad = lambda t, v: (ctypes.c_double * M)(*(list(t)[:k] + [v] * (M - min(len(t), k))))
        return fmlb_multi_params(LATTICES[self.lattice], STORAGES[self.storage], n, self.nx, self.ny, self.nz,
                                 pad(self.tau, 1.0), self.tau_d, G, self.kT, pad(self.rho_ref, 0.0), self.seed,
                                 self.flags)


class Multi:
    """One N-species lattice on the current device (torch-owned buffers,
    torch's current stream)."""

    def __init__(self, p: MultiParams, device=None, stream=None):
        import torch
        self.p = p
        cp = p.c()
        sizes = [fmlb_multi_required_bytes(cp, k) for k in range(3)]
        if min(sizes) == 0:
            raise FmlbError("fmlb_multi_required_bytes", FMLB_E_INVALID)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.bufs = [torch.empty(s, dtype=torch.uint8, device=dev) for s in sizes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.m = fmlb_multi_create(cp, self.stream.cuda_stream, [b.data_ptr() for b in self.bufs])
        self.N = p.nspecies
        self.Q = 9 if p.lattice == "d2q9" else 19
        self.D = 2 if p.lattice == "d2q9" else 3
        self.shape = (p.nz, p.ny, p.nx)
        self.nsites = p.nx * p.ny * p.nz

    def close(self):
        if getattr(self, "m", None):
            fmlb_multi_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass

    @property
    def step_count(self) -> int:
        return fmlb_multi_current_step(self.m)

    def init_density(self, rho):
        """rho: N scalars or arrays of the lattice shape."""
        if len(rho) != self.N:
            raise ValueError(f"{len(rho)} density fields for {self.N} species")
        fmlb_multi_init_density(self.m, np.stack([_as_field(r, self.shape) for r in rho]))

    def step(self, n: int = 1):
        fmlb_multi_step(self.m, n)

    def set_tile(self, tile_x: int = 0, tile_y: int = 0, march: int = 0):
        """(0, 0, 0): the default form; (1, 0, 0): two passes; otherwise the
        register single pass with that tile."""
        fmlb_multi_set_tile(self.m, tile_x, tile_y, march)

    def set_form(self, form: str = "auto", tile_x: int = 0, tile_y: int = 0, march: int = 0):
        """form: "auto", "two_pass", "fused" (register single pass) or "async"
        (single pass with the next plane pulled into LDS; FP32 storage)."""
        fmlb_multi_set_form(self.m, MULTI_FORMS[form], tile_x, tile_y, march)

    def populations(self):
        out = np.empty((self.N, self.Q) + self.shape)
        fmlb_multi_get_populations(self.m, out)
        return out

    def set_populations(self, f, step: int = 0):
        fmlb_multi_set_populations(self.m, np.asarray(f, dtype=np.float64).reshape(self.N, self.Q, *self.shape), step)

    def moments(self):
        rho = np.empty((self.N,) + self.shape)
        j = np.empty((self.N, self.D) + self.shape)
        fmlb_multi_moments(self.m, rho, j)
        return rho, j

    def global_sums(self):
        out = np.empty(self.N + self.D)
        fmlb_multi_global_sums(self.m, out)
        return out

    def synchronize(self):
        self.stream.synchronize()
