"""Reference vector-Jacobian products for the adjoint tests, taken entirely
from the oracle: the oracle's own flash of each mixture, then its dense
implicit-function Jacobian (``oracle.flash_jacobian``) at the oracle's
converged split.  Test infrastructure: it calls the oracle."""
from __future__ import annotations

import numpy as np

import oracle

ORC_UNCONV = oracle.FLAG_SPLIT_UNCONV | oracle.FLAG_SPLIT_FAILED | oracle.FLAG_SPLIT_TRIVIAL


def oracle_vjp(w, ms, ob, hrel=1e-3, spread_h=(3e-3,), tol=1e-10):
    """For the mixtures ms of workload w with cotangents ob (len(ms) rows of
    (g_beta, g_x, g_y)), returns (k, ref, spread) for the rows k whose
    oracle flash is a converged two-phase split: ref = J^T ob with J the
    oracle's Jacobian at the oracle's (beta, y), spread = the largest change
    of ref over the other finite-difference steps (an estimate of the
    reference's own error).  Rows are returned only where the GPU's split
    given in `gpu` matches the oracle's within tol (same split)."""
    ms = np.asarray(ms)
    o = oracle.flash(w.subset(ms), threads=8)
    out = []
    for k, m in enumerate(ms):
        if o["label"][k] != 1 or (o["info"][k, 8] & ORC_UNCONV):
            continue
        sets = (w.Tc[m], w.Pc[m], w.omega[m], w.kij[m]) if w.per_mixture else \
            (w.Tc, w.Pc, w.omega, w.kij)
        args = (*sets, w.z[m], w.T[m], w.P[m], o["beta"][k], o["y"][k])
        ref = oracle.flash_jacobian(*args, hrel=hrel).T @ ob[k]
        spread = max(np.abs(ref - oracle.flash_jacobian(*args, hrel=h).T @ ob[k]).max()
                     for h in spread_h)
        out.append((k, ref, spread, o["beta"][k], o["x"][k], o["y"][k]))
    return out


def check_vjp(w, ms, gpu, grads, ob, spread_h=(3e-3,), rel=1e-7, spread_factor=10.0):
    """Compares the GPU's parameter gradients (gz, gT, gP, gk per mixture,
    k as a full symmetric matrix) with the oracle's VJP on the mixtures ms
    whose GPU split equals the oracle's within 1e-10.  Returns (compared,
    worst error / tolerance, rows skipped as a different split)."""
    gz, gT, gP, gk = grads
    nc = w.nc
    pairs = [(a, b) for a in range(nc) for b in range(a + 1, nc)]
    refs = oracle_vjp(w, ms, ob, spread_h=spread_h)
    worst, n, other = 0.0, 0, 0
    for k, ref, spread, beta, x, y in refs:
        m = ms[k]
        same = max(abs(gpu["beta"][m] - beta), np.abs(gpu["x"][m] - x).max(),
                   np.abs(gpu["y"][m] - y).max()) < 1e-10
        if not same:
            other += 1
            continue
        got = np.concatenate([gz[m], [gT[m], gP[m]], [gk[m, a, b] + gk[m, b, a] for a, b in pairs]])
        tol = rel * np.abs(ref).max() + spread_factor * spread
        err = np.abs(got - ref).max() / tol
        worst = max(worst, err)
        assert err < 1.0, (m, np.abs(got - ref).max(), tol)
        n += 1
    return n, worst, other
