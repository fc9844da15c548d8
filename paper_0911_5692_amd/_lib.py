"""ctypes binding of liblf.so (declarations: include/lf.h).

Argument marshalling only: every step of the evolution runs in the HIP
kernels of liblf.  If the library is not built this module raises; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblf.so")

LF_OK, LF_EINVAL, LF_EHIP, LF_ENONFINITE, LF_ESTATE, LF_ENOMEM = range(6)
LF_F32, LF_F64 = 0, 1
STATUS_NAMES = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_EHIP", 3: "LF_ENONFINITE", 4: "LF_ESTATE",
                5: "LF_ENOMEM"}


class LfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("dtype", ctypes.c_int32), ("L", ctypes.c_double),
                ("dt", ctypes.c_double), ("beta", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("c1", ctypes.c_double), ("G", ctypes.c_double), ("r", ctypes.c_double),
                ("s", ctypes.c_double), ("kappa2", ctypes.c_double), ("tile_y", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("stencil", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("a", ctypes.c_double), ("ad", ctypes.c_double),
                ("hubble", ctypes.c_double), ("K", ctypes.c_double * 2),
                ("Gr", ctypes.c_double * 2), ("P", ctypes.c_double), ("rho", ctypes.c_double),
                ("R", ctypes.c_double), ("status", ctypes.c_uint32), ("pad_", ctypes.c_uint32)]


class Scalars(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("a_half", ctypes.c_double), ("ad", ctypes.c_double),
                ("bg_f", ctypes.c_double * 2), ("bg_v", ctypes.c_double * 2),
                ("pend", ctypes.c_double * 4), ("status", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32)]


class Vacuum(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double * 2), ("u0", ctypes.c_double * 2), ("m2", ctypes.c_double * 2),
                ("eps2", ctypes.c_double), ("cutoff", ctypes.c_double), ("seed", ctypes.c_uint64)]


_lib = None
_vp = ctypes.c_void_p

# name -> (argtypes, restype); every entry point returns an lf_status int
# unless stated.
SIGNATURES = {
    "lf_abi_version": ([], ctypes.c_int),
    "lf_last_error": ([], ctypes.c_char_p),
    "lf_workspace_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_create": ([ctypes.POINTER(Params), _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)], ctypes.c_int),
    "lf_destroy": ([_vp], ctypes.c_int),
    "lf_init": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "lf_init_physical": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double,
                          ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "lf_energies": ([_vp, ctypes.POINTER(Report)], ctypes.c_int),
    "lf_rho_p": ([_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_get_fields": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "lf_get_state": ([_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Scalars)], ctypes.c_int),
    "lf_set_state": ([_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Scalars)], ctypes.c_int),
    "lf_set_coupling": ([_vp, ctypes.c_double], ctypes.c_int),
    "lf_last_step_ms": ([_vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_time_kernels": ([_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "lf_stream_copy": ([_vp] * 8 + [ctypes.c_int64, _vp], ctypes.c_int),
    "lf_slab_rows": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "lf_slab_sweep": ([_vp, ctypes.c_int, ctypes.c_int] + [ctypes.POINTER(_vp)] * 4 + [_vp, ctypes.c_int64],
                      ctypes.c_int),
    "lf_slab_sweep_sums": ([_vp, ctypes.c_int, ctypes.c_int] + [ctypes.POINTER(_vp)] * 4 + [_vp], ctypes.c_int),
    "lf_autotune_workspace_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_ens_autotune_workspace_bytes": ([ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
                                        ctypes.c_int),
    "lf_ens_autotune": ([ctypes.c_int, ctypes.POINTER(Params), _vp, _vp, ctypes.c_size_t, ctypes.c_char_p,
                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_ens_zchunk": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "lf_autotune": ([ctypes.POINTER(Params), _vp, _vp, ctypes.c_size_t, ctypes.c_char_p, ctypes.POINTER(Params),
                     ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_adj_workspace_bytes": ([ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_adj_forward": ([_vp, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp,
                        ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_adj_backward": ([_vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _vp, _vp, _vp, _vp,
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_ens_workspace_bytes": ([ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
                               ctypes.c_int),
    "lf_ens_create": ([ctypes.c_int, ctypes.POINTER(Params), _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)],
                      ctypes.c_int),
    "lf_ens_destroy": ([_vp], ctypes.c_int),
    "lf_ens_size": ([_vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "lf_ens_init": ([_vp, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double],
                    ctypes.c_int),
    "lf_ens_init_physical": ([_vp, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double,
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_ens_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "lf_ens_last_step_ms": ([_vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_ens_energies": ([_vp, ctypes.POINTER(Report)], ctypes.c_int),
    "lf_ens_get_fields": ([_vp, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "lf_vacuum_workspace_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_vacuum_fields": ([ctypes.POINTER(Params), ctypes.POINTER(Vacuum), _vp, _vp, ctypes.c_size_t, _vp, _vp,
                          _vp, _vp], ctypes.c_int),
    "lf_init_vacuum_workspace_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_init_vacuum": ([_vp, ctypes.POINTER(Vacuum), ctypes.c_double, _vp, ctypes.c_size_t,
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lf_spectrum_bins": ([ctypes.c_int], ctypes.c_int),  # returns the count, not a status
    "lf_spectrum_workspace_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lf_spectrum": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                     ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_size_t], ctypes.c_int),
}


def lib() -> ctypes.CDLL:
    """Load liblf.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_0911_5692_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != LF_OK:
        msg = lib().lf_last_error()
        raise LfError(rc, msg.decode() if msg else "")
