"""The stages with one lane group per mixture (the trust-region stages with
lanes_per_mixture / lanes_split 16 or 32, the substitution stages with
lanes_ss; lane i holds component i) against the CPU oracle, against the
one-mixture-per-lane form, and their option checks.

Sizes: 3,000 mixtures per case (many groups per wavefront and a ragged
tail); nc 12, 16 and 20 with a shared component set, nc 12 and 20 with one
component set per mixture; the adjoint from a group forward's factor.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2205_03090_amd import _capi, api, workloads  # noqa: E402
from parity import assert_parity, compare, gpu_to_numpy, invariants  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(w, **kw):
    r = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, **kw)
    torch.cuda.synchronize()
    return gpu_to_numpy(r)


def _check(w, lanes, tag, split=0, ss=1, min2=0.08):
    print(f"case {tag} nc={w.nc} lanes={lanes}/{split}/{ss} n={w.n}", flush=True)
    g = _run(w, lanes_per_mixture=lanes, lanes_split=split, lanes_ss=ss)
    inv = invariants(w, g)
    print(f"[{tag} invariants] {inv}", flush=True)
    assert inv["mass_balance"] < 1e-13 and inv["sum_x"] < 1e-13 and inv["sum_y"] < 1e-13
    assert inv["single_ok"] and inv["beta_in_range"] and inv["labels_valid"]
    o = oracle.flash(w, threads=8, want_min_tpd=1)
    rep = compare(g, o, w=w)
    print(f"[{tag}] {rep}", flush=True)
    assert_parity(rep, o, path_agree=0.97, min_two_phase_frac=min2)
    # against one mixture per lane: the same decisions; values to rounding
    # wherever both converged
    one = _run(w, lanes_per_mixture=1, lanes_ss=1)
    ok = ((g["status"].astype(np.int64) | one["status"].astype(np.int64)) & 0x20) == 0
    assert np.array_equal(g["label"][ok], one["label"][ok])
    two = ok & (g["label"] == 1)
    assert np.abs(g["beta"][two] - one["beta"][two]).max(initial=0.0) < 1e-10
    assert np.abs(g["x"][two] - one["x"][two]).max(initial=0.0) < 1e-10
    assert np.abs(g["y"][two] - one["y"][two]).max(initial=0.0) < 1e-10
    # stage decisions (substitution counts are computed by the same per-lane
    # stages; the trust-region counts may differ by rounding on a few)
    same_it = np.all(g["iters"] == one["iters"], axis=1)
    print(f"[{tag}] iteration counts equal on {same_it.mean():.4f}", flush=True)
    assert same_it.mean() > 0.97
    return g


@pytest.mark.parametrize("nc,lanes", [(12, 16), (16, 16), (20, 32), (12, 32)])
def test_group_shared_set_parity(nc, lanes):
    w = workloads.uniform_workload(f"nc{nc}", 1000 + nc, 3000, nc, 0.7, (200.0, 600.0),
                                   (1e5, 2e7))
    _check(w, lanes, f"group shared nc{nc}")


@pytest.mark.parametrize("nc,lanes", [(12, 16), (20, 32)])
def test_group_per_mixture_sets_parity(nc, lanes):
    w = workloads.uniform_workload(f"pm{nc}", 2000 + nc, 3000, nc, 0.5, (200.0, 600.0),
                                   (1e5, 2e7), per_mixture=True)
    _check(w, lanes, f"group per-mixture nc{nc}")


@pytest.mark.parametrize("nc,sa,sp", [(20, 32, 1), (20, 1, 32), (14, 16, 1)])
def test_mixed_stage_widths_parity(nc, sa, sp):
    # the two trust-region stages with different lanes per mixture
    w = workloads.uniform_workload(f"mx{nc}", 3000 + nc, 3000, nc, 0.5, (200.0, 600.0),
                                   (1e5, 2e7))
    _check(w, sa, f"mixed nc{nc}", split=sp)


@pytest.mark.parametrize("nc,tr,ss", [(12, 1, 16), (16, 16, 16), (20, 1, 32), (20, 32, 32)])
def test_group_substitution_stages_parity(nc, tr, ss):
    # the two substitution stages (stability trials, split) with lane groups,
    # alone or with group trust-region stages; shared and per-mixture sets
    w = workloads.uniform_workload(f"ss{nc}", 5000 + nc, 3000, nc, 0.5, (200.0, 600.0),
                                   (1e5, 2e7))
    # (these seeded sets hold 5-10 % two-phase mixtures: a few hundred
    # compared splits each)
    _check(w, tr, f"group substitutions nc{nc}", ss=ss, min2=0.05)
    w = workloads.uniform_workload(f"sspm{nc}", 6000 + nc, 3000, nc, 0.5, (200.0, 600.0),
                                   (1e5, 2e7), per_mixture=True)
    _check(w, tr, f"group substitutions per-mixture nc{nc}", ss=ss, min2=0.05)


def test_group_deterministic_across_runs_and_grids():
    w = workloads.uniform_workload("d20", 77, 4000, 20, 0.3, (200.0, 600.0), (1e5, 3e7))
    a = _run(w, lanes_per_mixture=32, lanes_ss=32)
    b = _run(w, lanes_per_mixture=32, lanes_ss=32)
    c = _run(w, lanes_per_mixture=32, lanes_ss=32, grid=7, block=64)
    for k in ("label", "beta", "x", "y", "iters", "status", "flops"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
        assert np.array_equal(a[k], c[k], equal_nan=True), k


def test_group_factor_drives_the_adjoint():
    # the backward reads the factor the split stage keeps; a group forward
    # and a per-lane forward give the same gradients to rounding
    nc = 12
    w = workloads.uniform_workload("adj12", 4242, 2000, nc, 0.5, (200.0, 600.0), (1e5, 2e7))
    gb, gx, gy = workloads.cotangents(9, w.n, nc)
    outs = []
    for lanes in (16, 1):
        r = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, keep_factor=True,
                      lanes_per_mixture=lanes)
        gr = api.flash_backward(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, r, gb, gx, gy)
        torch.cuda.synchronize()
        outs.append((r, gr))
    (ra, ga), (rb, gb_) = outs
    st = (ra.status.cpu().numpy().astype(np.int64) | rb.status.cpu().numpy().astype(np.int64))
    two = (ra.label.cpu().numpy() == 1) & ((st & 0x20) == 0)
    assert two.sum() > 100
    for k in range(3):
        a = ga[k].cpu().numpy()[two]
        b = gb_[k].cpu().numpy()[two]
        scale = np.maximum(1.0, np.abs(b))
        assert np.all(np.isfinite(a))
        assert (np.abs(a - b) / scale).max() < 1e-6, k


def test_lanes_option_checked():
    L = _capi.lib()
    o = _capi.default_options()
    assert o.lanes_per_mixture == 0
    w = workloads.uniform_workload("o", 5, 64, 4, 1.0)
    for lanes in (16, 32):   # nc = 4 is below the group variants' range
        with pytest.raises(RuntimeError):
            _run(w, lanes_per_mixture=lanes)
    w20 = workloads.uniform_workload("o20", 5, 64, 20, 1.0)
    with pytest.raises(RuntimeError):
        _run(w20, lanes_per_mixture=16)   # a group smaller than nc
    with pytest.raises(RuntimeError):
        _run(w20, lanes_per_mixture=8)    # not a supported width
    with pytest.raises(RuntimeError):
        _run(w20, lanes_per_mixture=1, lanes_split=16)   # split group too small
    with pytest.raises(RuntimeError):
        _run(w, lanes_split=32)   # nc = 4
    with pytest.raises(RuntimeError):
        _run(w20, lanes_ss=16)    # substitution group too small
    with pytest.raises(RuntimeError):
        _run(w20, lanes_ss=8)
    assert o.lanes_split == 0 and o.lanes_ss == 0
    _run(w20, lanes_per_mixture=32)
    _run(w20, lanes_per_mixture=1)
    _run(w20, lanes_per_mixture=1, lanes_split=32)
    _run(w20, lanes_ss=32)
    assert L is not None and isinstance(o, C.Structure)
