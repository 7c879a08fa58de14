"""The seeded input generators: ranges and structure of the random-property
workloads (the case studies are covered by test_case_studies.py)."""
import numpy as np
from scipy import stats

from paper_2205_03090_amd import workloads as W


def _check_ragged(w, nc_set):
    assert set(np.unique(w.nc_of)) <= set(nc_set)
    assert w.off[0] == 0 and np.array_equal(np.diff(w.off), w.nc_of)
    assert np.array_equal(np.diff(w.koff), (w.nc_of[:-1].astype(np.int64)) ** 2)
    for nc in np.unique(w.nc_of):
        _, g = w.group(int(nc))
        assert np.abs(g.z.sum(axis=1) - 1.0).max() < 1e-14 and g.z.min() > 0.0
        assert g.Tc.min() >= 190.0 and g.Tc.max() <= 620.0
        assert g.Pc.min() >= 2e6 and g.Pc.max() <= 5e6
        assert g.omega.min() >= 0.01 and g.omega.max() <= 0.5
        assert np.array_equal(g.kij, g.kij.transpose(0, 2, 1))
        assert np.all(np.diagonal(g.kij, axis1=1, axis2=2) == 0.0)
        assert g.kij.min() >= 0.0 and g.kij.max() <= 0.15
    assert w.T.min() >= 200.0 and w.T.max() <= 600.0


def test_ragged_generators_share_their_distributions():
    nc_set = (2, 4, 6, 8, 12, 16, 20)
    a = W.ragged_workload("a", 5, 4000, nc_set)
    b = W.ragged_workload_vec("b", 6, 40_000, nc_set)
    _check_ragged(a, nc_set)
    _check_ragged(b, nc_set)
    # nc uniform over the set
    counts = np.bincount(b.nc_of, minlength=21)[list(nc_set)]
    assert stats.chisquare(counts).pvalue > 1e-3
    # the per-component marginals of both draws agree (z_0 at nc = 8: Beta(0.5, 3.5))
    _, ga = a.group(8)
    _, gb = b.group(8)
    assert stats.ks_2samp(ga.z[:, 0], gb.z[:, 0]).pvalue > 1e-3
    assert stats.kstest(gb.z[:, 0], stats.beta(0.5, 3.5).cdf).pvalue > 1e-3
    # determinism
    c = W.ragged_workload_vec("c", 6, 40_000, nc_set)
    assert np.array_equal(b.z, c.z) and np.array_equal(b.kij, c.kij)


def test_select_matches_group():
    w = W.ragged_workload_vec("s", 9, 5000)
    idx, g = w.group(12)
    _, h = w.select(idx[::3], 12)
    assert np.array_equal(h.z, g.z[::3]) and np.array_equal(h.kij, g.kij[::3])
