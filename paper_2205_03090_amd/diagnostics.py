"""Convergence diagnostics of the phase split from a flash result (the
analysis of Sec. 5.1 and Fig. 5): how many splits each iteration settles, and
how close to a critical point the mixtures settled there are.

Everything here is host-side post-processing of the outputs of
``api.flash``; nothing runs on the GPU.
"""
from __future__ import annotations

import numpy as np

from . import _capi

_IT = {k: i for i, k in enumerate(_capi.IT_NAMES)}


def critical_distance(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """d_c = sqrt(sum_i (ln K_i)^2) with K_i = y_i / x_i (eq. dc): small near a
    critical point, where the two phases become alike."""
    return np.sqrt(np.sum(np.log(y / x) ** 2, axis=1))


def split_convergence(label, x, y, iters, status) -> dict:
    """Per iteration of the split: the share of two-phase mixtures settled by
    successive substitution after k updates, the share of the trust-region
    ones settled after k trust-region steps, and the mean critical distance
    of the mixtures settled at each point ("ss" = by substitution, then the
    trust-region step count).  Arrays as returned by the flash (NumPy)."""
    label = np.asarray(label)
    it = np.asarray(iters).astype(np.int64)
    st = np.asarray(status).astype(np.int64) & 0xFFFF
    two = (label == 1) & ((st & _capi.ST["SPLIT_UNCONV"]) == 0)
    tr = two & ((st & _capi.ST["SPLIT_TR"]) != 0)
    ss = two & ~tr
    dc = np.full(len(label), np.nan)
    dc[two] = critical_distance(np.asarray(x)[two], np.asarray(y)[two])
    n_ss = it[:, _IT["ss_split"]]
    n_tr = it[:, _IT["tr_split"]]
    kmax_ss = int(n_ss[two].max(initial=0))
    kmax_tr = int(n_tr[tr].max(initial=0))
    out = {
        "n_two_phase": int(two.sum()),
        "n_trust_region": int(tr.sum()),
        "ss_settled_share": [float(np.sum(ss & (n_ss <= k)) / max(two.sum(), 1))
                             for k in range(1, kmax_ss + 1)],
        "tr_settled_share": [float(np.sum(tr & (n_tr <= k)) / max(tr.sum(), 1))
                             for k in range(1, kmax_tr + 1)],
        "mean_dc": {"ss": float(np.mean(dc[ss])) if ss.any() else float("nan")},
        "count": {"ss": int(ss.sum())},
    }
    for k in range(1, kmax_tr + 1):
        sel = tr & (n_tr == k)
        if sel.any():
            out["mean_dc"][str(k)] = float(np.mean(dc[sel]))
            out["count"][str(k)] = int(sel.sum())
    return out
