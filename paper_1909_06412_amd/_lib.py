"""ctypes binding of libmgso.so: argument marshalling only, every step of the
propagation runs in the library's HIP kernels.  Function names mirror
include/mgso.h.  Loading fails loudly when the library is missing."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgso.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_EUNSTABLE, MG_ESTATE = 0, -1, -2, -3, -4, -5
MG_C128, MG_C64 = 0, 1
MG_POT_FREE, MG_POT_HARMONIC, MG_POT_MORSE_REP, MG_POT_HENON_HEILES, MG_POT_QUADRATIC = 0, 1, 2, 3, 4
MG_TVT, MG_VTV = 0, 1
MG_COMP_STRANG, MG_COMP_SUZUKI, MG_COMP_TRIPLE_JUMP, MG_COMP_USER = 0, 1, 2, 3
MG_OPT_ENGINE, MG_OPT_GRAPH, MG_OPT_PROFILE, MG_OPT_RENORMALIZE, MG_OPT_GRID = 1, 2, 3, 4, 5
MG_MAX_DIM = 8

_STATUS = {0: "MG_OK", -1: "MG_EINVAL", -2: "MG_ENOMEM", -3: "MG_EDEVICE", -4: "MG_EUNSTABLE",
           -5: "MG_ESTATE"}


class MgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

_vp, _dp, _ip, _i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)

_SIGS = {
    "mg_create": (C.c_int, [C.c_int, _ip, _dp, _dp, C.c_double, C.c_int, _vp, C.POINTER(_vp)]),
    "mg_destroy": (None, [_vp]),
    "mg_state_bytes": (C.c_size_t, [_vp]),
    "mg_workspace_bytes": (C.c_size_t, [_vp]),
    "mg_bind_buffers": (C.c_int, [_vp, _vp, _vp]),
    "mg_state_ptr": (_vp, [_vp]),
    "mg_set_gaussian": (C.c_int, [_vp, _dp, _dp, _dp]),
    "mg_set_state": (C.c_int, [_vp, _dp, _dp, _dp, C.c_double]),
    "mg_get_state": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "mg_set_potential": (C.c_int, [_vp, C.c_int, _dp, C.c_int]),
    "mg_set_scheme": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp, C.c_int]),
    "mg_step": (C.c_int, [_vp, C.c_double, C.c_int64]),
    "mg_observables": (C.c_int, [_vp, _dp]),
    "mg_regrid": (C.c_int, [_vp, _dp]),
    "mg_set_option": (C.c_int, [_vp, C.c_int, C.c_int64]),
    "mg_profile_read": (C.c_int, [_vp, _i64p, _dp, _dp, C.c_int]),
    "mg_profile_class": (C.c_int, [_vp, _ip, _ip, _ip, _ip, _ip]),
    "mg_autocorrelation": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "mg_spectrum": (C.c_int, [_dp, _dp, C.c_int, _dp, C.c_int, C.c_double, C.c_double, _dp]),
    "mg_adjoint": (C.c_int, [_vp, C.c_double, C.c_int64, C.c_int, _dp, _ip, C.c_int, _dp, _dp]),
    "mg_batch_create": (C.c_int, [C.c_int, C.c_int, _ip, _dp, _dp, C.c_double, C.c_int, _vp,
                                  C.POINTER(_vp)]),
    "mg_batch_destroy": (None, [_vp]),
    "mg_batch_set_gaussian": (C.c_int, [_vp, _dp, _dp, _dp]),
    "mg_batch_set_potential": (C.c_int, [_vp, C.c_int, _dp, C.c_int]),
    "mg_batch_set_scheme": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp, C.c_int]),
    "mg_batch_step": (C.c_int, [_vp, C.c_double, C.c_int64]),
    "mg_batch_observables": (C.c_int, [_vp, _dp]),
    "mg_batch_get_state": (C.c_int, [_vp, C.c_int, _dp, _dp, _dp, _dp]),
    "mg_batch_set_state": (C.c_int, [_vp, C.c_int, _dp, _dp, _dp, C.c_double]),
    "mg_batch_adjoint": (C.c_int, [_vp, C.c_double, C.c_int64, C.c_int, _dp, _ip, C.c_int, _dp,
                                   _dp]),
    "mg_batch_set_option": (C.c_int, [_vp, C.c_int, C.c_int64]),
    "mg_batch_config": (C.c_int, [_vp, C.c_int, _ip, _ip]),
    "mg_batch_set_config": (C.c_int, [_vp, C.c_int]),
    "mg_batch_autotune": (C.c_int, [_vp, C.c_double, C.c_int64, _dp, _ip]),
    "mg_batch_points": (C.c_int64, [_vp]),
    "mg_propagate_noalloc": (C.c_int, [C.c_int, _ip, _dp, _dp, C.c_double, C.c_int, C.c_int, _dp, C.c_int,
                                       C.c_int, C.c_int, C.c_int, _dp, C.c_int, _vp, _dp, _dp, C.c_double,
                                       C.c_int64, _vp]),
    "mg_last_error": (C.c_char_p, [_vp]),
    "mg_build_hash": (C.c_char_p, []),
}


def _load_torch_runtime_first():
    """PyTorch ships its own HIP runtime whose SONAME (libamdhip64.so.7) is the one
    libmgso.so needs.  Loading torch first makes the library bind to that runtime,
    so the process has one HIP runtime and torch tensors can back our buffers."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load libmgso.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _load_torch_runtime_first()
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1909_06412_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        from .build import source_hash
        built, want = (L.mg_build_hash() or b"").decode(), source_hash()
        if built != want:
            raise ImportError(f"{LIB_PATH} was built from other sources (embedded {built[:16]}, "
                              f"sources {want[:16]}): rebuild with `python -m paper_1909_06412_amd.build`")
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def f64(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def check(status, handle):
    if status != MG_OK:
        msg = lib().mg_last_error(handle) if handle else b""
        raise MgError(status, (msg or b"").decode(errors="replace"))
