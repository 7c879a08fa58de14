"""Stability analysis alone (ptflash_stability) and the decisive tangent-plane
value of the flash (result.tm), through the C ABI, against the CPU oracle's
decision and against the full flash."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2205_03090_amd import _capi, api, workloads  # noqa: E402
from parity import gpu_to_numpy  # noqa: E402

pytestmark = pytest.mark.gpu

EPS = 1e-10
ST = _capi.ST


def _stab(w, **kw):
    r = api.stability(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, **kw)
    torch.cuda.synchronize()
    return {k: getattr(r, k).cpu().numpy() for k in ("label", "tm", "iters", "status")}


def _flash(w, **kw):
    r = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, **kw)
    torch.cuda.synchronize()
    return gpu_to_numpy(r)


@pytest.mark.parametrize("maker", [lambda: workloads.nc8_workload(n=20_000),
                                   lambda: workloads.case_study_workload("cs9", 20_000),
                                   lambda: workloads.uniform_workload(
                                       "s20", 44, 3000, 20, 0.3, (200.0, 600.0), (1e5, 3e7))])
def test_stability_matches_oracle_decision(maker):
    w = maker()
    print(f"case stability {w.name} nc={w.nc} n={w.n}", flush=True)
    s = _stab(w)
    o = oracle.flash(w, threads=8, want_min_tpd=1)
    unst = o["info"][:, oracle.INFO_FIELDS.index("unstable")] == 1
    # labels agree wherever the mixture is not within 1e-9 of a boundary
    band = np.abs(o["min_tpd"]) > 1e-9
    bad = np.where(band & ((s["label"] == 1) != unst))[0]
    print(f"[{w.name}] unstable {s['label'].mean():.4f} (oracle {unst.mean():.4f}); "
          f"mismatches outside the band {len(bad)}", flush=True)
    assert len(bad) == 0, bad[:10]
    # the decisive value and the label agree by definition
    assert np.array_equal(s["tm"] < -EPS, s["label"] == 1)
    # the decisive values: identical triage values for case 3 mixtures on both
    # sides to rounding; for stable mixtures both trials end at stationary
    # points of tm (gradient below 1e-6), so the values agree closely
    sc = (s["status"].astype(np.int64) & ST["SHORTCUT"]) != 0
    both = sc & (o["info"][:, 0] == 3)
    assert np.abs(s["tm"][both] - o["tm"][both]).max(initial=0.0) < 1e-8
    stable = band & (s["label"] == 0) & ~unst
    d = np.abs(s["tm"][stable] - o["tm"][stable])
    print(f"[{w.name}] stable |tm - tm_oracle|: median {np.median(d):.2e}, "
          f"99.9 % {np.quantile(d, 0.999):.2e}", flush=True)
    assert np.quantile(d, 0.999) < 1e-8


def test_stability_equals_the_flash_decision():
    w = workloads.nc8_workload(n=50_000, seed=9)
    s = _stab(w)
    f = _flash(w)
    # same stages and arithmetic: the flash's tm and its first counters are
    # the stability call's, bit for bit
    assert np.array_equal(s["tm"], f["tm"])
    assert np.array_equal(s["iters"][:, :5], f["iters"][:, :5])
    # the flash sends exactly the unstable mixtures to the split
    st = f["status"].astype(np.int64)
    to_split = (f["label"] == 1) | ((st & (ST["SPLIT_FAILED"] | ST["SPLIT_TRIVIAL"]
                                           | ST["RR_NO_ROOT"])) != 0)
    assert np.array_equal(s["label"] == 1, to_split)
    # the plain form agrees
    p = _stab(w, form=_capi.FORM_PLAIN)
    for k in ("label", "tm", "iters", "status"):
        assert np.array_equal(s[k], p[k], equal_nan=True), k


def test_stability_invalid_inputs_and_options():
    w = workloads.nc8_workload(n=8, seed=3)
    z = w.z.copy()
    z[1, 3] = 0.0
    r = api.stability(z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij)
    torch.cuda.synchronize()
    assert np.isnan(r.tm[1].item()) and r.label[1].item() == 0
    assert (int(r.status[1].item()) & ST["INVALID"]) != 0
    with pytest.raises(RuntimeError):
        api.stability(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, keep_factor=1)
