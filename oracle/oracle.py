"""ctypes front end of the C oracle (test infrastructure only).

The C file ``ptflash_oracle.c`` holds all of the arithmetic; this module only
marshals NumPy arrays and splits a batch over host threads.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_lib = None
_lock = threading.Lock()


class OrcOpts(C.Structure):
    _fields_ = [("max_pre_ss", C.c_int32), ("max_ss", C.c_int32),
                ("max_newton", C.c_int32), ("dem_every", C.c_int32),
                ("want_min_tpd", C.c_int32), ("max_newton_split", C.c_int32),
                ("tol_sa_ss", C.c_double), ("tol_sa_tr", C.c_double),
                ("tol_split_ss", C.c_double), ("tol_split", C.c_double),
                ("eps_tm", C.c_double), ("decision_only", C.c_int32)]


INFO_FIELDS = ["case", "pre", "ss_v", "nt_v", "ss_l", "nt_l", "ss_split",
               "nt_split", "flags", "out_v", "out_l", "swap", "split_ss_conv", "unstable"]
FLAG_INVALID, FLAG_SA_UNCONV, FLAG_SPLIT_UNCONV = 1, 2, 4
FLAG_SPLIT_TRIVIAL, FLAG_SPLIT_FAILED, FLAG_RR_NO_ROOT = 8, 16, 32
FLAG_HINTED = 64
FLAG_SPLIT_RESTART = 128

_D = C.POINTER(C.c_double)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB):
                _build.build()
            L = C.CDLL(_build.LIB)
            L.orc_default_opts.argtypes = [C.POINTER(OrcOpts)]
            L.orc_cubic_roots.argtypes = [C.c_double, C.c_double, _D]
            L.orc_cubic_roots.restype = C.c_int
            L.orc_gres.argtypes = [C.c_double, C.c_double, C.c_double]
            L.orc_gres.restype = C.c_double
            L.orc_rr_solve.argtypes = [C.c_int, _D, _D, _D]
            L.orc_rr_solve.restype = C.c_int
            L.orc_lnphi.argtypes = [C.c_int32, _D, _D, _D, _D, C.c_double, C.c_double, _D, _D, _D]
            L.orc_wilson_lnk.argtypes = [C.c_int32, _D, _D, _D, C.c_double, C.c_double, _D]
            L.orc_tpd_probe.argtypes = [C.c_int32, _D, _D, _D, _D, C.c_double, C.c_double, _D, _D]
            L.orc_tpd_probe.restype = C.c_double
            L.orc_split_residual.argtypes = [C.c_int32, _D, _D, _D, _D, C.c_double, C.c_double, _D, _D, _D]
            L.orc_split_residual.restype = C.c_double
            L.orc_ninfo.restype = C.c_int
            L.orc_flash_jacobian.argtypes = [C.c_int32, _D, C.c_double, C.c_double, _D, _D, _D,
                                             _D, C.c_double, _D, C.c_double, _D]
            L.orc_flash_jacobian.restype = C.c_int
            L.orc_flash_batch.argtypes = [C.c_int64, C.c_int32, _D, _D, _D, _D, _D, _D, _D,
                                          C.c_int32, _D, C.c_void_p, C.POINTER(OrcOpts),
                                          C.c_void_p, _D, _D,
                                          _D, C.c_void_p, _D, C.c_void_p, C.c_int64, C.c_int64]
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> OrcOpts:
    o = OrcOpts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def cubic_roots(A: float, B: float) -> np.ndarray:
    r = np.zeros(3)
    n = lib().orc_cubic_roots(A, B, _p(r))
    return r[:n].copy()


def gres(Z: float, A: float, B: float) -> float:
    return lib().orc_gres(Z, A, B)


def rr_solve(z, K):
    z, K = _f64(z), _f64(K)
    th = np.zeros(1)
    rc = lib().orc_rr_solve(len(z), _p(z), _p(K), _p(th))
    return rc, th[0]


def lnphi(Tc, Pc, omega, kij, T, P, c):
    Tc, Pc, omega, kij, c = map(_f64, (Tc, Pc, omega, kij, c))
    out = np.zeros(len(c))
    abz = np.zeros(7)
    lib().orc_lnphi(len(c), _p(Tc), _p(Pc), _p(omega), _p(kij), T, P, _p(c), _p(out), _p(abz))
    return out, dict(A=abz[0], B=abz[1], Z=abz[2], nroots=int(abz[3]), roots=abz[4:4 + int(abz[3])])


def wilson_lnk(Tc, Pc, omega, T, P):
    Tc, Pc, omega = map(_f64, (Tc, Pc, omega))
    out = np.zeros(len(Tc))
    lib().orc_wilson_lnk(len(Tc), _p(Tc), _p(Pc), _p(omega), T, P, _p(out))
    return out


def tpd(Tc, Pc, omega, kij, T, P, z, w):
    Tc, Pc, omega, kij, z, w = map(_f64, (Tc, Pc, omega, kij, z, w))
    return lib().orc_tpd_probe(len(z), _p(Tc), _p(Pc), _p(omega), _p(kij), T, P, _p(z), _p(w))


def split_residual(Tc, Pc, omega, kij, T, P, z, nV):
    Tc, Pc, omega, kij, z, nV = map(_f64, (Tc, Pc, omega, kij, z, nV))
    r = np.zeros(len(z))
    G = lib().orc_split_residual(len(z), _p(Tc), _p(Pc), _p(omega), _p(kij), T, P, _p(z), _p(nV), _p(r))
    return r, G


def flash(w, opts: OrcOpts | None = None, threads: int | None = None, lnk0=None, hint=None,
          **kw):
    """Runs the oracle flash over a workload (``workloads.Workload``).

    lnk0 (n x nc, optional): initial ln K in place of Wilson's (substitutions
    and stability trials); hint (n, int8, optional): 0 = known stable, 1 = known
    unstable (case 4 in info: the split starts at once), other values none.

    Returns a dict of NumPy arrays: label (int8), beta, x, y, min_tpd (NaN
    unless requested), tm (the value that decided stability: the most
    negative triage value of a case-3 mixture, else the smaller final tm of
    the two trials; NaN for invalid input) and info (see INFO_FIELDS)."""
    o = opts if opts is not None else default_opts(**kw)
    L = lib()
    n, nc = w.n, w.nc
    z, T, P = _f64(w.z), _f64(w.T), _f64(w.P)
    Tc, Pc, om, kk = map(_f64, (w.Tc, w.Pc, w.omega, w.kij))
    label = np.zeros(n, np.int8)
    beta = np.zeros(n)
    x = np.zeros((n, nc))
    y = np.zeros((n, nc))
    mtpd = np.full(n, np.nan)
    tmd = np.full(n, np.nan)
    info = np.zeros((n, L.orc_ninfo()), np.int32)
    lk = None if lnk0 is None else _f64(np.asarray(lnk0).reshape(n, nc))
    hn = None if hint is None else np.ascontiguousarray(np.asarray(hint, dtype=np.int8).reshape(n))
    threads = threads or 1
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)

    def run(k):
        L.orc_flash_batch(n, nc, _p(z), _p(T), _p(P), _p(Tc), _p(Pc), _p(om), _p(kk),
                          int(w.per_mixture), _p(lk) if lk is not None else None,
                          hn.ctypes.data if hn is not None else None, C.byref(o),
                          label.ctypes.data, _p(beta),
                          _p(x), _p(y), mtpd.ctypes.data, _p(tmd), info.ctypes.data,
                          int(bounds[k]), int(bounds[k + 1]))

    if threads == 1:
        run(0)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, range(threads)))
    return dict(label=label, beta=beta, x=x, y=y, min_tpd=mtpd, tm=tmd, info=info)


def flash_jacobian(Tc, Pc, omega, kij, z, T, P, beta, y, hrel=1e-3):
    """Jacobian of (beta, x, y) of a converged two-phase result with respect
    to p = (z_raw[nc], T, P, k_ab for a < b), by the implicit function
    theorem on the equal-fugacity system (fourth-order finite-difference
    partials with relative step hrel)."""
    Tc, Pc, omega, kij, z, y = map(_f64, (Tc, Pc, omega, kij, z, y))
    nc = len(z)
    npar = nc + 2 + nc * (nc - 1) // 2
    J = np.zeros((1 + 2 * nc, npar))
    rc = lib().orc_flash_jacobian(nc, _p(z), T, P, _p(Tc), _p(Pc), _p(omega), _p(kij),
                                  float(beta), _p(y), float(hrel), _p(J))
    if rc != 0:
        raise RuntimeError("singular split Jacobian")
    return J
