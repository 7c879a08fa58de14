"""Host-side checks of the C ABI: the library loads, exports every function
that include/ptflash.h declares, and rejects malformed calls before touching
the GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2205_03090_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ptflash.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ptflash_\w+)\s*\(", text)))


def test_header_declarations_are_exported():
    decl = _declared_functions()
    assert set(decl) == set(_capi.EXPORTS)
    L = _capi.lib()
    for name in decl:
        assert hasattr(L, name), name


def test_default_options_are_the_papers():
    o = _capi.default_options()
    assert (o.max_pre_ss, o.max_ss, o.max_tr_sa, o.max_tr_split) == (3, 9, 20, 30)
    assert (o.tol_sa_ss, o.tol_sa_tr, o.tol_split_ss, o.tol_split_tr) == (1e-6, 1e-6, 1e-8, 1e-8)
    assert o.dem_every == 3 and o.eps_tm == 1e-10 and o.form == _capi.FORM_PERSISTENT


def test_rejects_malformed_calls_without_gpu():
    L = _capi.lib()
    o = _capi.default_options()
    r = _capi.Result()
    assert L.ptflash_flash(None, C.byref(o), C.byref(r), None, 0, None) == 1
    p = _capi.Problem(n=-1, nc=3)
    assert L.ptflash_flash(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 1
    p = _capi.Problem(n=5, nc=1, z=8, T=8, P=8, Tc=8, Pc=8, omega=8, kij=8)
    assert L.ptflash_flash(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 2
    p = _capi.Problem(n=5, nc=L.ptflash_max_nc() + 1, z=8, T=8, P=8, Tc=8, Pc=8, omega=8, kij=8)
    assert L.ptflash_flash(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 2
    p = _capi.Problem(n=5, nc=3, z=8, T=8, P=8, Tc=8, Pc=8, omega=8, kij=8)
    r = _capi.Result(label=8, beta=8, x=8, y=8)
    assert L.ptflash_flash(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 3
    bad = _capi.default_options(max_pre_ss=0)
    assert L.ptflash_flash(C.byref(p), C.byref(bad), C.byref(r), None, 0, None) == 1
    p0 = _capi.Problem(n=0, nc=3)
    assert L.ptflash_flash(C.byref(p0), C.byref(o), C.byref(r), None, 0, None) == 0
    assert L.ptflash_workspace_bytes(C.byref(p), C.byref(o)) >= 8
    assert L.ptflash_strerror(3).startswith(b"workspace too small")
    # one component set per mixture is accepted; other values are not
    pm = _capi.Problem(n=5, nc=3, props_per_mixture=2, z=8, T=8, P=8, Tc=8, Pc=8, omega=8,
                       kij=8)
    assert L.ptflash_flash(C.byref(pm), C.byref(o), C.byref(r), None, 0, None) == 1
    pm.props_per_mixture = 1
    assert L.ptflash_flash(C.byref(pm), C.byref(o), C.byref(r), None, 0, None) == 3


def test_ragged_entry_rejects_malformed_calls_without_gpu():
    L = _capi.lib()
    o = _capi.default_options()
    r = _capi.Result(label=8, beta=8, x=8, y=8)
    p = _capi.RaggedProblem(n=0)
    assert L.ptflash_flash_ragged(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 0
    p = _capi.RaggedProblem(n=-1)
    assert L.ptflash_flash_ragged(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 1
    full = dict(n=10, nc_of=8, off=8, koff=8, z=8, T=8, P=8, Tc=8, Pc=8, omega=8, kij=8)
    p = _capi.RaggedProblem(**{**full, "koff": None})
    assert L.ptflash_flash_ragged(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 1
    p = _capi.RaggedProblem(**full)
    ko = _capi.default_options(keep_factor=1)
    assert L.ptflash_flash_ragged(C.byref(p), C.byref(ko), C.byref(r), None, 0, None) == 1
    assert L.ptflash_flash_ragged(C.byref(p), C.byref(o), C.byref(r), None, 0, None) == 3
    need = L.ptflash_ragged_workspace_bytes(C.byref(p), C.byref(o))
    assert need > 10 * 4
    # the workspace does not grow with nc beyond what one chunk needs
    big = _capi.RaggedProblem(**{**full, "n": 1 << 22})
    assert L.ptflash_ragged_workspace_bytes(C.byref(big), C.byref(o)) < 64 * 2 ** 30


def test_hint_from_probability():
    import torch
    from paper_2205_03090_amd import api
    p = torch.tensor([0.0, 0.1, 0.3, 0.5, 0.7, 0.9, 1.0], dtype=torch.float64)
    assert api.hint_from_probability(p, 0.3, 0.7).tolist() == [1, 1, 1, -1, 0, 0, 0]
    # p_l = p_r: the classifier alone decides, stable from the threshold on
    assert api.hint_from_probability(p, 0.5, 0.5).tolist() == [1, 1, 1, 0, 0, 0, 0]
    with pytest.raises(ValueError):
        api.hint_from_probability(p, 0.6, 0.4)


def test_binding_checks_shapes_before_any_launch():
    import numpy as np
    import torch
    from paper_2205_03090_amd import api, workloads
    w = workloads.nc8_workload(n=6, seed=3)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64)
    z, T, P, Tc, Pc, om, k = map(t, (w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij))
    api.make_problem(z, T, P, Tc, Pc, om, k)   # well formed
    bad = [(z, T[:5], P, Tc, Pc, om, k), (z, T, P[:, None], Tc, Pc, om, k),
           (z, T, P, Tc[:7], Pc, om, k), (z, T, P, Tc, Pc, om, k[:7]),
           (z, T, P, Tc[None].repeat(6, 1), Pc, om, k), (z[0], T, P, Tc, Pc, om, k)]
    for args in bad:
        with pytest.raises(ValueError):
            api.make_problem(*args)
    # per-mixture sets need (n, nc) properties and (n, nc, nc) k
    rep = lambda a: a[None].repeat(6, *([1] * a.dim()))
    api.make_problem(z, T, P, rep(Tc), rep(Pc), rep(om), rep(k))
    with pytest.raises(ValueError):
        api.make_problem(z, T, P, rep(Tc), rep(Pc), rep(om), k)
    # ragged offsets
    nc_of = torch.tensor([2, 3], dtype=torch.int32)
    off = torch.tensor([0, 2, 5], dtype=torch.int64)
    koff = torch.tensor([0, 4], dtype=torch.int64)
    zz, kk = torch.ones(5, dtype=torch.float64), torch.zeros(13, dtype=torch.float64)
    T2 = torch.ones(2, dtype=torch.float64)
    api._check_ragged(2, 5, T2, nc_of, off, koff, zz, zz, zz, kk)
    for o2, k2, kij2 in [(torch.tensor([1, 2, 5]), koff, kk), (torch.tensor([0, 3, 2]), koff, kk),
                         (torch.tensor([0, 2, 6]), koff, kk), (off, torch.tensor([0, 5]), kk),
                         (off, koff, kk[:12])]:
        with pytest.raises(ValueError):
            api._check_ragged(2, 5, T2, nc_of, o2.to(torch.int64), k2.to(torch.int64), zz, zz,
                              zz, kij2)
    assert np.isfinite(w.z).all()


def test_noalloc_rejects_problems_beyond_its_scratch_without_gpu():
    # the size check of the allocation-free entry point comes before any HIP
    # call: a problem whose workspace exceeds the library's scratch buffer is
    # refused with PTFLASH_EWORKSPACE (the pointers are never dereferenced)
    L = _capi.lib()
    o = _capi.default_options()
    r = _capi.Result(label=8, beta=8, x=8, y=8)
    assert L.ptflash_flash_noalloc(None, C.byref(o), C.byref(r), None) == 1
    fits = {}
    for nc in (8, 20):
        p = _capi.Problem(n=10_000_000, nc=nc, z=8, T=8, P=8, Tc=8, Pc=8, omega=8, kij=8)
        assert L.ptflash_workspace_bytes(C.byref(p), C.byref(o)) > _capi.NOALLOC_SCRATCH_BYTES
        assert L.ptflash_flash_noalloc(C.byref(p), C.byref(o), C.byref(r), None) == 3
        # largest batch that fits (persistent form), for the limit the header states
        lo, hi = 1, 10_000_000
        while lo < hi:
            mid = (lo + hi + 1) // 2
            p.n = mid
            if L.ptflash_workspace_bytes(C.byref(p), C.byref(o)) <= _capi.NOALLOC_SCRATCH_BYTES:
                lo = mid
            else:
                hi = mid - 1
        fits[nc] = lo
    assert 90_000 < fits[8] < 120_000 and 40_000 < fits[20] < 55_000, fits
    assert b"scratch" in L.ptflash_strerror(3)
