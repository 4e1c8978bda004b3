"""ctypes binding of the cmlbm C ABI (include/cmlbm.h).

Argument marshalling only: every function here forwards to the function of
the same name in ``libcmlbm.so`` and raises ``CmlbmError`` on a non-zero
status. Pointers are plain integers (device addresses, e.g.
``tensor.data_ptr()``) unless a host array is expected.

The library links against the HIP runtime; when PyTorch is used, ``torch``
must be imported first so that both share one runtime instance (the loader
binds libcmlbm to the already loaded ``libamdhip64.so.7``).
"""
from __future__ import annotations

import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmlbm.so")

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ESTATE = range(6)
STATUS_NAMES = {0: "CMLBM_OK", 1: "CMLBM_EINVAL", 2: "CMLBM_ENOMEM", 3: "CMLBM_EHIP", 4: "CMLBM_ENONFINITE",
                5: "CMLBM_ESTATE"}
F64, F32, F32_SHIFTED, F16_SHIFTED = range(4)
DT_F64, DT_F32 = 0, 1
FACTORIZED, REDUCED_COMPRESSIBILITY, SGS_FORCE = 1, 2, 4
D3Q27, D2Q9 = 0, 1
STREAM_TWO_BUFFERS, STREAM_IN_PLACE = 0, 1
LATTICE_NAMES = {"d3q27": D3Q27, "d2q9": D2Q9}
ELEM_SIZE = {F64: 8, F32: 4, F32_SHIFTED: 4, F16_SHIFTED: 2}
STORAGE_NAMES = {"f64": F64, "f32": F32, "f32s": F32_SHIFTED, "f16s": F16_SHIFTED}


class CmlbmError(RuntimeError):
    def __init__(self, status, func, message):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("walls", ctypes.c_uint32), ("tuning", ctypes.c_uint32),
                ("wall_u_lo", ctypes.c_double * 3), ("wall_u_hi", ctypes.c_double * 3),
                ("rho0", ctypes.c_double), ("lattice", ctypes.c_int32), ("streaming", ctypes.c_uint32)]


class Relax(ctypes.Structure):
    _fields_ = [("omega_shear", ctypes.c_double), ("omega_bulk", ctypes.c_double),
                ("omega3", ctypes.c_double * 3), ("omega4", ctypes.c_double * 2),
                ("omega5", ctypes.c_double), ("omega6", ctypes.c_double), ("cs_smag", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_P = ctypes.c_void_p
_H = ctypes.c_void_p
SIGNATURES = {
    "cmlbm_create": ([ctypes.POINTER(Desc), _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_H)], ctypes.c_int),
    "cmlbm_destroy": ([_H], ctypes.c_int),
    "cmlbm_set_stream": ([_H, _P], ctypes.c_int),
    "cmlbm_set_relaxation": ([_H, ctypes.POINTER(Relax)], ctypes.c_int),
    "cmlbm_set_force": ([_H, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "cmlbm_init_equilibrium": ([_H, _P, _P, ctypes.c_int], ctypes.c_int),
    "cmlbm_step": ([_H, ctypes.c_int64], ctypes.c_int),
    "cmlbm_step_from": ([_H, _P, _P], ctypes.c_int),
    "cmlbm_state_buffer": ([_H, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cmlbm_read_moments": ([_H, _P, _P, ctypes.c_int], ctypes.c_int),
    "cmlbm_get_populations": ([_H, _P, ctypes.c_int], ctypes.c_int),
    "cmlbm_set_populations": ([_H, _P, ctypes.c_int], ctypes.c_int),
    "cmlbm_reduce": ([_H, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "cmlbm_reduce_noalloc": ([_H, _P], ctypes.c_int),
    "cmlbm_adjoint_step": ([_H, _P, _P, _P, _P], ctypes.c_int),
    "cmlbm_energy_seed": ([_H, _P, _P, _P], ctypes.c_int),
    "cmlbm_set_sgs_buffers": ([_H, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "cmlbm_copy": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "cmlbm_last_error": ([], ctypes.c_char_p),
    "cmlbm_version": ([], ctypes.c_int32),
}

_lib = None


def library_path() -> str:
    return LIB_PATH


def load(path: str | None = None):
    """Load libcmlbm.so (built in-tree by ``build.build()``). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libcmlbm.so not found at {path}; build it with paper_1202_6074_amd.build.build()")
    if "torch" not in sys.modules:
        # share one HIP runtime with PyTorch: load torch's first when it is available
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    lib = ctypes.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status, func):
    if status != OK:
        raise CmlbmError(status, func, load().cmlbm_last_error().decode())


def cmlbm_create(desc: Desc, buf_a: int, buf_b: int, bytes_each: int, stream: int) -> int:
    h = _H()
    _check(load().cmlbm_create(ctypes.byref(desc), buf_a, buf_b, bytes_each, stream, ctypes.byref(h)), "cmlbm_create")
    return h.value


def cmlbm_destroy(h: int):
    _check(load().cmlbm_destroy(h), "cmlbm_destroy")


def cmlbm_set_stream(h: int, stream: int):
    _check(load().cmlbm_set_stream(h, stream), "cmlbm_set_stream")


def cmlbm_set_relaxation(h: int, relax: Relax):
    _check(load().cmlbm_set_relaxation(h, ctypes.byref(relax)), "cmlbm_set_relaxation")


def cmlbm_set_force(h: int, uniform, field_ptr: int | None):
    arr = (ctypes.c_double * 3)(*[float(v) for v in uniform])
    _check(load().cmlbm_set_force(h, arr, field_ptr or None), "cmlbm_set_force")


def cmlbm_init_equilibrium(h: int, rho_ptr: int | None, u_ptr: int, dt: int):
    _check(load().cmlbm_init_equilibrium(h, rho_ptr or None, u_ptr, dt), "cmlbm_init_equilibrium")


def cmlbm_step(h: int, nsteps: int):
    _check(load().cmlbm_step(h, int(nsteps)), "cmlbm_step")


def cmlbm_step_from(h: int, src: int, dst: int):
    _check(load().cmlbm_step_from(h, src, dst), "cmlbm_step_from")


def cmlbm_state_buffer(h: int):
    p = _P()
    n = ctypes.c_size_t()
    _check(load().cmlbm_state_buffer(h, ctypes.byref(p), ctypes.byref(n)), "cmlbm_state_buffer")
    return p.value, n.value


def cmlbm_read_moments(h: int, rho_ptr: int, u_ptr: int, dt: int):
    _check(load().cmlbm_read_moments(h, rho_ptr, u_ptr, dt), "cmlbm_read_moments")


def cmlbm_get_populations(h: int, f_ptr: int, dt: int):
    _check(load().cmlbm_get_populations(h, f_ptr, dt), "cmlbm_get_populations")


def cmlbm_set_populations(h: int, f_ptr: int, dt: int):
    _check(load().cmlbm_set_populations(h, f_ptr, dt), "cmlbm_set_populations")


def cmlbm_reduce(h: int, raise_nonfinite: bool = True):
    out = (ctypes.c_double * 8)()
    st = load().cmlbm_reduce(h, out)
    if st != ENONFINITE or raise_nonfinite:
        _check(st, "cmlbm_reduce")
    return list(out), st


def cmlbm_reduce_noalloc(h: int, out: int):
    """out: device address of 8 doubles (enqueued; no synchronisation)."""
    _check(load().cmlbm_reduce_noalloc(h, out), "cmlbm_reduce_noalloc")


def cmlbm_adjoint_step(h: int, state: int, lam_in: int, lam_out: int, grad_F: int):
    _check(load().cmlbm_adjoint_step(h, state, lam_in, lam_out, grad_F), "cmlbm_adjoint_step")


def cmlbm_energy_seed(h: int, state: int, lam_out: int, grad_F: int):
    _check(load().cmlbm_energy_seed(h, state, lam_out, grad_F), "cmlbm_energy_seed")


def cmlbm_set_sgs_buffers(h: int, stress_a: int, stress_b: int, bytes_each: int):
    _check(load().cmlbm_set_sgs_buffers(h, stress_a, stress_b, bytes_each), "cmlbm_set_sgs_buffers")


def cmlbm_copy(src: int, dst: int, nbytes: int, stream: int):
    _check(load().cmlbm_copy(src, dst, nbytes, stream), "cmlbm_copy")


def cmlbm_last_error() -> str:
    return load().cmlbm_last_error().decode()


def cmlbm_version() -> int:
    return int(load().cmlbm_version())
