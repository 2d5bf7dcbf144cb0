"""ctypes binding of libvdwlb.so (C-ABI in include/vdwlb.h).

Argument marshalling only: every step of the sweep runs in the HIP library.
Device memory comes from torch tensors; streams are torch's current stream.
Importing this module does not touch the GPU; the library is loaded on first
use and a missing build raises immediately (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvdwlb.so")
ABI_VERSION = 2  # VDWLB_ABI_VERSION of include/vdwlb.h

OK, E_INVALID_ARG, E_UNSUPPORTED, E_DEVICE, E_UNPHYSICAL, E_CAPACITY = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
FORCE_LOG, FORCE_NID = 0, 1

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("ncomp", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("force", ctypes.c_int32),
        ("kT", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("gamma_mu", ctypes.c_double),
        ("a", _c_double_p),
        ("b", _c_double_p),
        ("kappa", _c_double_p),
        ("lam", _c_double_p),
    ]


_VP = ctypes.c_void_p
_SIGS = {
    "vdwlb_abi_version": (ctypes.c_int32, []),
    "vdwlb_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "vdwlb_last_device_error": (ctypes.c_char_p, []),
    "vdwlb_plan_create": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.POINTER(_VP)]),
    "vdwlb_plan_destroy": (ctypes.c_int32, [_VP]),
    "vdwlb_plane_elems": (ctypes.c_int64, [_VP]),
    "vdwlb_state_bytes": (ctypes.c_size_t, [_VP]),
    "vdwlb_init": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP]),
    "vdwlb_step": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.POINTER(ctypes.c_int32)]),
    "vdwlb_moments": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "vdwlb_sync_status": (ctypes.c_int32, [_VP, _VP]),
    "vdwlb_schedule_count": (ctypes.c_int32, [_VP]),
    "vdwlb_set_schedule": (ctypes.c_int32, [_VP, ctypes.c_int32]),
    "vdwlb_autotune": (ctypes.c_int32, [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)]),
    "vdwlb_maxwell": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_double_p, _c_double_p]),
    "vdwlb_copy": (ctypes.c_int32, [_VP, _VP, ctypes.c_size_t, _VP]),
    "vdwlb_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(Desc), ctypes.POINTER(_VP)]),
    "vdwlb_batch_destroy": (ctypes.c_int32, [_VP]),
    "vdwlb_batch_state_bytes": (ctypes.c_size_t, [_VP]),
    "vdwlb_batch_offset": (ctypes.c_int64, [_VP, ctypes.c_int32]),
    "vdwlb_batch_density_offset": (ctypes.c_int64, [_VP, ctypes.c_int32]),
    "vdwlb_batch_set_launch": (ctypes.c_int32, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "vdwlb_batch_set_blocking": (ctypes.c_int32, [_VP, ctypes.c_int32]),
    "vdwlb_batch_init": (ctypes.c_int32, [_VP, _VP, _VP, _VP]),
    "vdwlb_batch_density": (ctypes.c_int32, [_VP, _VP, _VP, _VP]),
    "vdwlb_batch_run": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.POINTER(ctypes.c_int32)]),
    "vdwlb_batch_status": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int32), _VP]),
    "vdwlb_adjoint_param_count": (ctypes.c_int32, [_VP]),
    "vdwlb_adjoint_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int32]),
    "vdwlb_moments_adjoint": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP]),
    "vdwlb_adjoint_segment": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP]),
    "vdwlb_adjoint_recompute": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
    "vdwlb_adjoint_reverse": (ctypes.c_int32, [_VP, ctypes.c_int32, _VP, _VP, _VP, _VP]),
    "vdwlb_adjoint_segment_noalloc": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP]),
    "vdwlb_set_adjoint_graphs": (ctypes.c_int32, [_VP, ctypes.c_int32]),
    "vdwlb_adjoint_forward": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP]),
    "vdwlb_pressure_tensor": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "vdwlb_phase_points": (ctypes.c_int32, [ctypes.c_double, _c_double_p, _c_double_p, ctypes.c_int32, _VP, _VP,
                                            ctypes.c_double, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_07251_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.vdwlb_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.vdwlb_abi_version()}, this binding expects "
                               f"{ABI_VERSION}: rebuild it with `python -m paper_1805_07251_amd.build`")
        _lib = L
    return _lib


class VdwlbError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        msg = lib().vdwlb_strerror(status).decode()
        if status == E_DEVICE:
            msg += ": " + lib().vdwlb_last_device_error().decode()
        super().__init__(f"{where}: {msg}" if where else msg)
        self.status = status


def check(status: int, where: str = "") -> int:
    if status != OK:
        raise VdwlbError(status, where)
    return status


def symbols() -> list[str]:
    return list(_SIGS)


def maxwell(a: float, b: float, kT: float) -> tuple[float, float]:
    """Coexisting (rho_gas, rho_liquid) of one van der Waals component."""
    g, l = ctypes.c_double(), ctypes.c_double()
    check(lib().vdwlb_maxwell(a, b, kT, ctypes.byref(g), ctypes.byref(l)), "vdwlb_maxwell")
    return g.value, l.value
