"""GPU parity of the ragged-batch flash (mixtures with their own component
counts nc in {2, 4, 6, 8, 12, 16, 20} and their own component sets) against
the CPU oracle, group by group, through the C ABI; the ragged results also
equal, bit for bit, those of the uniform per-mixture-set flash of each
group; unusable rows are reported INVALID."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2205_03090_amd import _capi, api, workloads  # noqa: E402
from parity import assert_parity, compare, gpu_to_numpy  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(w, nc_of=None, **kw):
    r = api.flash_ragged(w.z, w.T, w.P, w.nc_of if nc_of is None else nc_of, w.off, w.koff,
                         w.Tc, w.Pc, w.omega, w.kij, **kw)
    torch.cuda.synchronize()
    return gpu_to_numpy(r)


def _group_view(g, w, idx, nc):
    rows = w.off[idx][:, None] + np.arange(nc)[None, :]
    return dict(label=g["label"][idx], beta=g["beta"][idx], x=g["x"][rows], y=g["y"][rows],
                iters=g["iters"][idx], status=g["status"][idx], flops=g["flops"][idx])


@pytest.mark.parametrize("form", [_capi.FORM_PERSISTENT, _capi.FORM_PLAIN])
def test_ragged_parity_per_group(form):
    w = workloads.ragged_workload("ragged", 31, 7000)
    print(f"case ragged n={w.n} form={form}", flush=True)
    g = _run(w, form=form)
    for nc in (2, 4, 6, 8, 12, 16, 20):
        idx, gw = w.group(nc)
        gg = _group_view(g, w, idx, nc)
        o = oracle.flash(gw, threads=8, want_min_tpd=1)
        rep = compare(gg, o, w=gw)
        print(f"[ragged nc={nc} n={len(idx)}] {rep}", flush=True)
        assert_parity(rep, o, path_agree=0.97, min_two_phase_frac=0.08)
        if form == _capi.FORM_PERSISTENT and nc in (4, 20):
            u = api.flash(gw.z, gw.T, gw.P, gw.Tc, gw.Pc, gw.omega, gw.kij)
            torch.cuda.synchronize()
            u = gpu_to_numpy(u)
            for k in ("label", "beta", "x", "y", "iters", "status"):
                assert np.array_equal(gg[k], u[k], equal_nan=True), (nc, k)


def test_ragged_unusable_rows_are_invalid():
    w = workloads.ragged_workload("ragged_bad", 32, 300)
    nc_of = w.nc_of.copy()
    bad = [3, 77, 150]
    nc_of[3] = 1                      # below the smallest nc
    nc_of[77] = 25                    # above the largest compiled nc
    nc_of[150] = nc_of[150] + 1       # disagrees with its row count
    print("case ragged invalid rows", flush=True)
    g = _run(w, nc_of=nc_of)
    ok = np.setdiff1d(np.arange(w.n), bad)
    st = g["status"].astype(np.int64) & 0xFFFF
    assert np.all(st[bad] & _capi.ST["INVALID"])
    assert np.all(g["label"][bad] == 0) and np.all(g["beta"][bad] == -1.0)
    for m in bad:
        a, b = w.off[m], w.off[m + 1]
        assert np.array_equal(g["x"][a:b], w.z[a:b]) and np.array_equal(g["y"][a:b], w.z[a:b])
    assert not np.any(st[ok] & _capi.ST["INVALID"])
    ref = _run(w)
    for k in ("label", "beta", "status"):
        assert np.array_equal(g[k][ok], ref[k][ok]), k
