"""PyTorch front end: device memory and streams from torch, all compute in HIP.

``flash`` runs the SRK PT flash on tensors that live on the current HIP
device and stream; ``eval_phase`` exposes the phase model used inside it.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _capi


@dataclass
class FlashResult:
    label: torch.Tensor     # (n,) int8: 0 single phase, 1 two-phase
    beta: torch.Tensor      # (n,) float64: vapour fraction, -1 for single phase
    x: torch.Tensor         # (n, nc) float64 liquid-like composition
    y: torch.Tensor         # (n, nc) float64 vapour-like composition
    iters: torch.Tensor     # (n, 8) int16 iteration counters (see _capi.IT_NAMES)
    status: torch.Tensor    # (n,) int16 status bits (see _capi.ST)
    flops: torch.Tensor     # (n,) int32 algorithmic flops per mixture
    factor: torch.Tensor | None  # (n, nc(nc+1)/2) Cholesky factor or None
    tm: torch.Tensor | None = None  # (n,) float64 value that decided stability


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f64(t, device):
    return torch.as_tensor(t, dtype=torch.float64, device=device).contiguous()


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_shapes(n, nc, T, P, Tc, Pc, omega, kij):
    """Host-side shape checks before any launch: T, P (n,); a shared
    component set Tc, Pc, omega (nc,) with kij (nc, nc), or one set per
    mixture: (n, nc) with kij (n, nc, nc)."""
    for name, t in (("T", T), ("P", P)):
        if tuple(t.shape) != (n,):
            raise ValueError(f"{name} must have shape ({n},), got {tuple(t.shape)}")
    per = Tc.dim() == 2
    want = (n, nc) if per else (nc,)
    for name, t in (("Tc", Tc), ("Pc", Pc), ("omega", omega)):
        if tuple(t.shape) != want:
            raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    wk = (n, nc, nc) if per else (nc, nc)
    if tuple(kij.shape) != wk:
        raise ValueError(f"kij must have shape {wk}, got {tuple(kij.shape)}")


def make_problem(z, T, P, Tc, Pc, omega, kij, lnk0=None, hint=None):
    if z.dim() != 2:
        raise ValueError(f"z must have shape (n, nc), got {tuple(z.shape)}")
    n, nc = z.shape
    _check_shapes(n, nc, T, P, Tc, Pc, omega, kij)
    per = 1 if Tc.dim() == 2 else 0
    p = _capi.Problem(n=n, nc=nc, props_per_mixture=per, z=_ptr(z).value, T=_ptr(T).value,
                      P=_ptr(P).value, Tc=_ptr(Tc).value, Pc=_ptr(Pc).value,
                      omega=_ptr(omega).value, kij=_ptr(kij).value,
                      lnk0=None if lnk0 is None else _ptr(lnk0).value,
                      hint=None if hint is None else _ptr(hint).value)
    return p


def hint_from_probability(p, p_l: float, p_r: float) -> torch.Tensor:
    """The threshold rule of Sec. 4 for a classifier's probability p that a
    mixture is stable: hint 0 (stable) where p >= p_r, else 1 (unstable)
    where p <= p_l, else -1 (run the stability analysis); p_l <= p_r.  With
    p_l = p_r the classifier alone decides."""
    if not p_l <= p_r:
        raise ValueError("p_l must not exceed p_r")
    p = torch.as_tensor(p)
    h = torch.full(p.shape, -1, dtype=torch.int8, device=p.device)
    h[p <= p_l] = 1
    h[p >= p_r] = 0
    return h


def _warm_start(lnk0, hint, n, nc, dev):
    """The optional per-mixture inputs on the device: lnk0 (n, nc) float64,
    hint (n,) int8."""
    if lnk0 is not None:
        lnk0 = _f64(lnk0, dev)
        if tuple(lnk0.shape) != (n, nc):
            raise ValueError(f"lnk0 must have shape ({n}, {nc})")
    if hint is not None:
        hint = torch.as_tensor(hint, dtype=torch.int8, device=dev).contiguous()
        if tuple(hint.shape) != (n,):
            raise ValueError(f"hint must have shape ({n},)")
    return lnk0, hint


def _workspace(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 1)]


def _new_result(n, nc, dev, keep_factor):
    return FlashResult(
        label=torch.empty(n, dtype=torch.int8, device=dev),
        beta=torch.empty(n, dtype=torch.float64, device=dev),
        x=torch.empty((n, nc), dtype=torch.float64, device=dev),
        y=torch.empty((n, nc), dtype=torch.float64, device=dev),
        iters=torch.empty((n, _capi.NITERS), dtype=torch.int16, device=dev),
        status=torch.empty(n, dtype=torch.int16, device=dev),
        flops=torch.empty(n, dtype=torch.int32, device=dev),
        factor=(torch.full((n, nc * (nc + 1) // 2), float("nan"), dtype=torch.float64,
                           device=dev) if keep_factor else None),
        tm=torch.empty(n, dtype=torch.float64, device=dev))


def _result_struct(out: FlashResult):
    return _capi.Result(label=_ptr(out.label).value, beta=_ptr(out.beta).value,
                        x=_ptr(out.x).value, y=_ptr(out.y).value, iters=_ptr(out.iters).value,
                        status=_ptr(out.status).value, flops=_ptr(out.flops).value,
                        factor=None if out.factor is None else _ptr(out.factor).value,
                        tm=None if out.tm is None else _ptr(out.tm).value)


def flash(z, T, P, Tc, Pc, omega, kij, *, keep_factor: bool = False, stream=None,
          out: FlashResult | None = None, lnk0=None, hint=None, noalloc: bool = False,
          **opts) -> FlashResult:
    """Isothermal two-phase SRK flash of n mixtures on the current GPU.

    z (n, nc), T (n,), P (n,) and the component set Tc, Pc, omega (nc,), kij
    (nc, nc) are float64 tensors (moved to the GPU if needed).  Optional
    lnk0 (n, nc): initial ln K in place of Wilson's; hint (n,)
    int8: 0 known stable, 1 known unstable, else none (ptflash_problem).
    Keyword options override ptflash_default_options (e.g.
    form=_capi.FORM_PLAIN).  noalloc=True calls ptflash_flash_noalloc (the
    library's own device scratch as workspace; at most
    _capi.NOALLOC_SCRATCH_BYTES of it)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    z, T, P = _f64(z, dev), _f64(T, dev), _f64(P, dev)
    Tc, Pc, omega, kij = (_f64(a, dev) for a in (Tc, Pc, omega, kij))
    n, nc = z.shape
    lnk0, hint = _warm_start(lnk0, hint, n, nc, dev)
    o = _capi.default_options(keep_factor=int(keep_factor), **opts)
    prob = make_problem(z, T, P, Tc, Pc, omega, kij, lnk0, hint)
    if out is None:
        out = _new_result(n, nc, dev, keep_factor)
    res = _result_struct(out)
    L = _capi.lib()
    if noalloc:
        rc = L.ptflash_flash_noalloc(C.byref(prob), C.byref(o), C.byref(res),
                                     _stream_handle(stream))
        _capi.check(rc, "ptflash_flash_noalloc")
        out._keepalive = (z, T, P, Tc, Pc, omega, kij, lnk0, hint)
        return out
    ws_bytes = L.ptflash_workspace_bytes(C.byref(prob), C.byref(o))
    ws = _workspace(ws_bytes, dev)
    rc = L.ptflash_flash(C.byref(prob), C.byref(o), C.byref(res), _ptr(ws), ws_bytes,
                         _stream_handle(stream))
    _capi.check(rc, "ptflash_flash")
    out._keepalive = (z, T, P, Tc, Pc, omega, kij, lnk0, hint, ws)  # until the stream is done
    return out


def stability(z, T, P, Tc, Pc, omega, kij, *, stream=None, lnk0=None, hint=None,
              **opts) -> FlashResult:
    """Stability analysis alone (ptflash_stability): label (1 = unstable), tm
    (the value that decided it), iters, status and flops; beta, x, y are None.
    lnk0 and hint as in flash."""
    dev = torch.device("cuda", torch.cuda.current_device())
    z, T, P = _f64(z, dev), _f64(T, dev), _f64(P, dev)
    Tc, Pc, omega, kij = (_f64(a, dev) for a in (Tc, Pc, omega, kij))
    n, nc = z.shape
    lnk0, hint = _warm_start(lnk0, hint, n, nc, dev)
    o = _capi.default_options(**opts)
    prob = make_problem(z, T, P, Tc, Pc, omega, kij, lnk0, hint)
    out = FlashResult(label=torch.empty(n, dtype=torch.int8, device=dev), beta=None, x=None,
                      y=None, iters=torch.empty((n, _capi.NITERS), dtype=torch.int16, device=dev),
                      status=torch.empty(n, dtype=torch.int16, device=dev),
                      flops=torch.empty(n, dtype=torch.int32, device=dev), factor=None,
                      tm=torch.empty(n, dtype=torch.float64, device=dev))
    res = _capi.Result(label=_ptr(out.label).value, beta=None, x=None, y=None,
                       iters=_ptr(out.iters).value, status=_ptr(out.status).value,
                       flops=_ptr(out.flops).value, factor=None, tm=_ptr(out.tm).value)
    L = _capi.lib()
    ws_bytes = L.ptflash_workspace_bytes(C.byref(prob), C.byref(o))
    ws = _workspace(ws_bytes, dev)
    rc = L.ptflash_stability(C.byref(prob), C.byref(o), C.byref(res), _ptr(ws), ws_bytes,
                             _stream_handle(stream))
    _capi.check(rc, "ptflash_stability")
    out._keepalive = (z, T, P, Tc, Pc, omega, kij, lnk0, hint, ws)
    return out


def flash_ragged(z, T, P, nc_of, off, koff, Tc, Pc, omega, kij, *, stream=None, lnk0=None,
                 hint=None, **opts):
    """Flash of a ragged batch (mixtures with their own nc and component set,
    packed as described for ptflash_ragged_problem): z, Tc, Pc, omega hold
    off[n] values, kij the nc_of[m]^2 blocks at koff[m]; the optional lnk0
    (off[n], packed like z) and hint (n,) as in flash.  Returns a
    FlashResult whose x and y are packed like z."""
    dev = torch.device("cuda", torch.cuda.current_device())
    z, T, P, Tc, Pc, omega, kij = (_f64(a, dev) for a in (z, T, P, Tc, Pc, omega, kij))
    nc_of = torch.as_tensor(nc_of, dtype=torch.int32, device=dev).contiguous()
    off = torch.as_tensor(off, dtype=torch.int64, device=dev).contiguous()
    koff = torch.as_tensor(koff, dtype=torch.int64, device=dev).contiguous()
    n = T.shape[0]
    tot = z.shape[0]
    _check_ragged(n, tot, P, nc_of, off, koff, Tc, Pc, omega, kij)
    if lnk0 is not None:
        lnk0 = _f64(lnk0, dev)
        if tuple(lnk0.shape) != (tot,):
            raise ValueError(f"lnk0 must have shape ({tot},), packed like z")
    if hint is not None:
        hint = torch.as_tensor(hint, dtype=torch.int8, device=dev).contiguous()
        if tuple(hint.shape) != (n,):
            raise ValueError(f"hint must have shape ({n},)")
    o = _capi.default_options(**opts)
    prob = _capi.RaggedProblem(n=n, nc_of=_ptr(nc_of).value, off=_ptr(off).value,
                               koff=_ptr(koff).value, z=_ptr(z).value, T=_ptr(T).value,
                               P=_ptr(P).value, Tc=_ptr(Tc).value, Pc=_ptr(Pc).value,
                               omega=_ptr(omega).value, kij=_ptr(kij).value,
                               lnk0=None if lnk0 is None else _ptr(lnk0).value,
                               hint=None if hint is None else _ptr(hint).value)
    out = FlashResult(
        label=torch.empty(n, dtype=torch.int8, device=dev),
        beta=torch.empty(n, dtype=torch.float64, device=dev),
        x=torch.empty(tot, dtype=torch.float64, device=dev),
        y=torch.empty(tot, dtype=torch.float64, device=dev),
        iters=torch.empty((n, _capi.NITERS), dtype=torch.int16, device=dev),
        status=torch.empty(n, dtype=torch.int16, device=dev),
        flops=torch.empty(n, dtype=torch.int32, device=dev),
        factor=None, tm=torch.empty(n, dtype=torch.float64, device=dev))
    res = _capi.Result(label=_ptr(out.label).value, beta=_ptr(out.beta).value,
                       x=_ptr(out.x).value, y=_ptr(out.y).value, iters=_ptr(out.iters).value,
                       status=_ptr(out.status).value, flops=_ptr(out.flops).value, factor=None,
                       tm=_ptr(out.tm).value)
    L = _capi.lib()
    ws_bytes = L.ptflash_ragged_workspace_bytes(C.byref(prob), C.byref(o))
    ws = _workspace(ws_bytes, dev)
    rc = L.ptflash_flash_ragged(C.byref(prob), C.byref(o), C.byref(res), _ptr(ws), ws_bytes,
                                _stream_handle(stream))
    _capi.check(rc, "ptflash_flash_ragged")
    out._keepalive = (z, T, P, nc_of, off, koff, Tc, Pc, omega, kij, lnk0, hint, ws)
    return out


def _check_ragged(n, tot, P, nc_of, off, koff, Tc, Pc, omega, kij):
    """Host-side checks of a ragged batch before any launch: sizes of the
    per-mixture and packed arrays, off[0] = 0, off non-decreasing with
    off[n] = len(z), and every k block inside kij.  (Rows whose off step
    differs from nc_of are not an error here: the library reports them
    INVALID.)"""
    if tuple(P.shape) != (n,) or tuple(nc_of.shape) != (n,) or tuple(koff.shape) != (n,):
        raise ValueError("T, P, nc_of and koff must all have shape (n,)")
    if tuple(off.shape) != (n + 1,):
        raise ValueError(f"off must have shape ({n + 1},)")
    for name, t in (("Tc", Tc), ("Pc", Pc), ("omega", omega)):
        if tuple(t.shape) != (tot,):
            raise ValueError(f"{name} must be packed like z: shape ({tot},)")
    if n == 0:
        return
    # on the arrays' own device, one host read for all of the checks
    nco = nc_of.to(torch.int64)
    bad = torch.stack([off[0] != 0, off[-1] != tot, (off[1:] < off[:-1]).any()])
    if bool(bad.any()):
        raise ValueError("off must start at 0, never decrease and end at len(z)")
    bad = torch.stack([(koff < 0).any(), (nco < 0).any(), (koff + nco * nco).max() > kij.shape[0]])
    if bool(bad.any()):
        raise ValueError("every k block koff[m] + nc_of[m]^2 must lie inside kij")


def eval_phase(c, T, P, Tc, Pc, omega, kij, *, derivs: bool = True, stream=None):
    """ln phi (n, nc), Z (n,) and Phi = n d ln phi/d n (n, nc, nc) of the SRK
    phase model at compositions c (n, nc)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    c, T, P = _f64(c, dev), _f64(T, dev), _f64(P, dev)
    Tc, Pc, omega, kij = (_f64(a, dev) for a in (Tc, Pc, omega, kij))
    if c.dim() != 2:
        raise ValueError(f"c must have shape (n, nc), got {tuple(c.shape)}")
    n, nc = c.shape
    if Tc.dim() != 1:
        raise ValueError("eval_phase takes one shared component set")
    _check_shapes(n, nc, T, P, Tc, Pc, omega, kij)
    lnphi = torch.empty((n, nc), dtype=torch.float64, device=dev)
    Z = torch.empty(n, dtype=torch.float64, device=dev)
    phi = torch.empty((n, nc, nc), dtype=torch.float64, device=dev) if derivs else None
    rc = _capi.lib().ptflash_eval_phase(n, nc, _ptr(c), _ptr(T), _ptr(P), _ptr(Tc), _ptr(Pc),
                                        _ptr(omega), _ptr(kij), _ptr(lnphi), _ptr(Z),
                                        _ptr(phi), _stream_handle(stream))
    _capi.check(rc, "ptflash_eval_phase")
    return lnphi, Z, phi


def flash_backward(z, T, P, Tc, Pc, omega, kij, fwd: FlashResult, g_beta, g_x, g_y, *,
                   kij_reduce: bool = True, stream=None):
    """Vector-Jacobian product of a forward result computed with
    keep_factor=True: returns (g_z, g_T, g_P, g_kij).  g_kij is (nc, nc)
    summed over mixtures when kij_reduce, else (n, nc, nc)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    z, T, P = _f64(z, dev), _f64(T, dev), _f64(P, dev)
    Tc, Pc, omega, kij = (_f64(a, dev) for a in (Tc, Pc, omega, kij))
    g_beta, g_x, g_y = _f64(g_beta, dev), _f64(g_x, dev), _f64(g_y, dev)
    if fwd.factor is None:
        raise ValueError("the forward result holds no factor (run flash with keep_factor=True)")
    n, nc = z.shape
    prob = make_problem(z, T, P, Tc, Pc, omega, kij)
    if tuple(g_beta.shape) != (n,) or tuple(g_x.shape) != (n, nc) or \
            tuple(g_y.shape) != (n, nc):
        raise ValueError(f"cotangents must have shapes ({n},), ({n}, {nc}), ({n}, {nc})")
    if tuple(fwd.x.shape) != (n, nc) or tuple(fwd.factor.shape) != (n, nc * (nc + 1) // 2):
        raise ValueError("the forward result does not match this problem's shape")
    o = _capi.default_options()
    res = _capi.Result(label=_ptr(fwd.label).value, beta=_ptr(fwd.beta).value,
                       x=_ptr(fwd.x).value, y=_ptr(fwd.y).value, iters=_ptr(fwd.iters).value,
                       status=_ptr(fwd.status).value, flops=_ptr(fwd.flops).value,
                       factor=_ptr(fwd.factor).value)
    gz = torch.empty((n, nc), dtype=torch.float64, device=dev)
    gT = torch.empty(n, dtype=torch.float64, device=dev)
    gP = torch.empty(n, dtype=torch.float64, device=dev)
    gk = torch.empty((nc, nc) if kij_reduce else (n, nc, nc), dtype=torch.float64, device=dev)
    L = _capi.lib()
    ws_bytes = L.ptflash_backward_workspace_bytes(C.byref(prob), int(kij_reduce))
    ws = _workspace(ws_bytes, dev)
    rc = L.ptflash_flash_backward(C.byref(prob), C.byref(o), C.byref(res), _ptr(g_beta),
                                  _ptr(g_x), _ptr(g_y), _ptr(gz), _ptr(gT), _ptr(gP), _ptr(gk),
                                  int(kij_reduce), _ptr(ws), ws_bytes, _stream_handle(stream))
    _capi.check(rc, "ptflash_flash_backward")
    gz._keepalive = (ws, z, T, P, Tc, Pc, omega, kij, g_beta, g_x, g_y)
    return gz, gT, gP, gk


class PTFlashFunction(torch.autograd.Function):
    """(z, T, P, kij) -> (beta, x, y, label, status) with the implicit-function
    adjoint in backward; Tc, Pc, omega are constants.  label and status are
    not differentiable."""

    @staticmethod
    def forward(ctx, z, T, P, kij, Tc, Pc, omega):
        r = flash(z, T, P, Tc, Pc, omega, kij, keep_factor=True)
        ctx.save_for_backward(z, T, P, kij, Tc, Pc, omega)
        ctx.fwd = r
        ctx.mark_non_differentiable(r.label, r.status)
        return r.beta, r.x, r.y, r.label, r.status

    @staticmethod
    def backward(ctx, g_beta, g_x, g_y, _gl, _gs):
        z, T, P, kij, Tc, Pc, omega = ctx.saved_tensors
        r = ctx.fwd
        zeros = lambda t, g: torch.zeros_like(t) if g is None else g
        gz, gT, gP, gk = flash_backward(z, T, P, Tc, Pc, omega, kij, r,
                                        zeros(r.beta, g_beta), zeros(r.x, g_x),
                                        zeros(r.y, g_y), kij_reduce=True)
        return gz, gT, gP, gk, None, None, None


def flash_autograd(z, T, P, kij, Tc, Pc, omega):
    """Differentiable flash: returns (beta, x, y, label, status)."""
    return PTFlashFunction.apply(z, T, P, kij, Tc, Pc, omega)
