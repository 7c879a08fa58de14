"""The split-convergence diagnostics (host-side post-processing of a flash
result) on a hand-made result whose answers are known."""
import numpy as np

from paper_2205_03090_amd import _capi, diagnostics


def test_critical_distance_closed_form():
    x = np.array([[0.5, 0.5], [0.2, 0.8]])
    y = np.array([[0.5, 0.5], [0.4, 0.6]])
    d = diagnostics.critical_distance(x, y)
    assert d[0] == 0.0
    assert abs(d[1] - np.hypot(np.log(2.0), np.log(0.75))) < 1e-15


def test_split_convergence_counts():
    x = np.array([[0.5, 0.5], [0.6, 0.4], [0.5, 0.5], [0.3, 0.7], [0.4, 0.6]])
    y = np.array([[0.25, 0.75], [0.4, 0.6], [0.5, 0.5], [0.1, 0.9], [0.5, 0.5]])
    it = np.zeros((5, 8), int)
    it[:, 5] = [3, 9, 0, 9, 9]
    it[:, 6] = [0, 2, 0, 5, 30]
    tr, un = _capi.ST["SPLIT_TR"], _capi.ST["SPLIT_UNCONV"]
    st = np.array([0, tr, 0, tr, tr | un])
    d = diagnostics.split_convergence(np.array([1, 1, 0, 1, 1]), x, y, it, st)
    # mixture 4 did not converge and mixture 2 is single phase: three count
    assert d["n_two_phase"] == 3 and d["n_trust_region"] == 2
    assert d["ss_settled_share"][2] == 1 / 3 and len(d["ss_settled_share"]) == 9
    assert d["tr_settled_share"] == [0.0, 0.5, 0.5, 0.5, 1.0]
    assert d["count"] == {"ss": 1, "2": 1, "5": 1}
    assert abs(d["mean_dc"]["2"] - np.hypot(np.log(0.4 / 0.6), np.log(0.6 / 0.4))) < 1e-15
