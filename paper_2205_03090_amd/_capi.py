"""ctypes binding of the C ABI declared in include/ptflash.h.

Argument marshalling only: every step of the flash runs in the HIP library.
The binding refuses to run without it (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

from . import build as _build

NITERS = 8
IT_NAMES = ["pre", "ss_v", "tr_v", "ss_l", "tr_l", "ss_split", "tr_split", "polish"]
FORM_PERSISTENT, FORM_PLAIN, FORM_FUSED = 0, 1, 2
ST = dict(INVALID=0x0001, SHORTCUT=0x0002, SA_RAN=0x0004, SA_UNCONV=0x0008,
          SPLIT_TR=0x0010, SPLIT_UNCONV=0x0020, SPLIT_TRIVIAL=0x0040,
          SPLIT_FAILED=0x0080, RR_NO_ROOT=0x0100, SWAPPED=0x0200, STEP_CAP=0x0400,
          HINTED=0x0800, SPLIT_RESTART=0x1000)
EXPORTS = ["ptflash_default_options", "ptflash_max_nc", "ptflash_workspace_bytes",
           "ptflash_flash", "ptflash_flash_backward", "ptflash_backward_workspace_bytes",
           "ptflash_eval_phase", "ptflash_strerror", "ptflash_ragged_workspace_bytes",
           "ptflash_flash_ragged", "ptflash_stability", "ptflash_flash_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 << 20   # PTFLASH_NOALLOC_SCRATCH_BYTES

_vp = C.c_void_p


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("nc", C.c_int32), ("props_per_mixture", C.c_int32),
                ("z", _vp), ("T", _vp), ("P", _vp), ("Tc", _vp), ("Pc", _vp),
                ("omega", _vp), ("kij", _vp), ("lnk0", _vp), ("hint", _vp)]


class RaggedProblem(C.Structure):
    _fields_ = [("n", C.c_int64), ("nc_of", _vp), ("off", _vp), ("koff", _vp), ("z", _vp),
                ("T", _vp), ("P", _vp), ("Tc", _vp), ("Pc", _vp), ("omega", _vp),
                ("kij", _vp), ("lnk0", _vp), ("hint", _vp)]


class Options(C.Structure):
    _fields_ = [("max_pre_ss", C.c_int32), ("max_ss", C.c_int32), ("max_tr_sa", C.c_int32),
                ("max_tr_split", C.c_int32), ("max_polish", C.c_int32),
                ("dem_every", C.c_int32), ("tol_sa_ss", C.c_double),
                ("tol_sa_tr", C.c_double), ("tol_split_ss", C.c_double),
                ("tol_split_tr", C.c_double), ("tol_polish", C.c_double),
                ("eps_tm", C.c_double), ("form", C.c_int32), ("keep_factor", C.c_int32),
                ("block", C.c_int32), ("grid", C.c_int32),
                ("lanes_per_mixture", C.c_int32), ("lanes_split", C.c_int32),
                ("lanes_ss", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("label", _vp), ("beta", _vp), ("x", _vp), ("y", _vp), ("iters", _vp),
                ("status", _vp), ("flops", _vp), ("factor", _vp), ("tm", _vp)]


_lib = None


def lib():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"HIP library not built: {_build.LIB} is missing "
                               "(run `python -m paper_2205_03090_amd.build`)")
        L = C.CDLL(_build.LIB)
        L.ptflash_default_options.argtypes = [C.POINTER(Options)]
        L.ptflash_default_options.restype = None
        L.ptflash_max_nc.restype = C.c_int32
        L.ptflash_workspace_bytes.argtypes = [C.POINTER(Problem), C.POINTER(Options)]
        L.ptflash_workspace_bytes.restype = C.c_size_t
        L.ptflash_flash.argtypes = [C.POINTER(Problem), C.POINTER(Options), C.POINTER(Result),
                                    _vp, C.c_size_t, _vp]
        L.ptflash_flash.restype = C.c_int
        L.ptflash_stability.argtypes = L.ptflash_flash.argtypes
        L.ptflash_stability.restype = C.c_int
        L.ptflash_flash_noalloc.argtypes = [C.POINTER(Problem), C.POINTER(Options),
                                            C.POINTER(Result), _vp]
        L.ptflash_flash_noalloc.restype = C.c_int
        L.ptflash_backward_workspace_bytes.argtypes = [C.POINTER(Problem), C.c_int32]
        L.ptflash_backward_workspace_bytes.restype = C.c_size_t
        L.ptflash_flash_backward.argtypes = [C.POINTER(Problem), C.POINTER(Options),
                                             C.POINTER(Result), _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.ptflash_flash_backward.restype = C.c_int
        L.ptflash_eval_phase.argtypes = [C.c_int64, C.c_int32] + [_vp] * 10 + [_vp]
        L.ptflash_eval_phase.restype = C.c_int
        L.ptflash_ragged_workspace_bytes.argtypes = [C.POINTER(RaggedProblem),
                                                     C.POINTER(Options)]
        L.ptflash_ragged_workspace_bytes.restype = C.c_size_t
        L.ptflash_flash_ragged.argtypes = [C.POINTER(RaggedProblem), C.POINTER(Options),
                                           C.POINTER(Result), _vp, C.c_size_t, _vp]
        L.ptflash_flash_ragged.restype = C.c_int
        L.ptflash_strerror.argtypes = [C.c_int]
        L.ptflash_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().ptflash_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def check(rc: int, what: str):
    if rc != 0:
        msg = lib().ptflash_strerror(rc).decode()
        raise RuntimeError(f"{what} failed with code {rc}: {msg}")
