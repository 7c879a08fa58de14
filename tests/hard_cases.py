"""Boundary-hugging flash inputs (the hard-case part of the Nc = 20
workload): mixtures placed, by bisection in pressure on the oracle's
stability label, within 2 % of a phase boundary.

Recipe (seeded, NumPy PCG64): one shared component set as in
``workloads``; per candidate, z ~ Dirichlet(alpha * 1) and T ~ U[T_lo, T_hi];
the oracle's label on a geometric grid of pressures in [P_lo, P_hi] must
change somewhere (else the candidate is dropped); the first change is
bisected (``steps`` halvings in log P) to P_b, and the mixture gets
P = P_b (1 + U[-0.02, 0.02]).  Test infrastructure: it calls the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2205_03090_amd import workloads


def _labels(w: workloads.Workload, P: np.ndarray, threads: int) -> np.ndarray:
    ww = workloads.Workload(w.name, w.n, w.nc, w.z, w.T, P, w.Tc, w.Pc, w.omega, w.kij)
    return oracle.flash(ww, threads=threads)["label"].astype(np.int8)


def boundary_workload(seed: int, n: int, nc: int = 20, alpha: float = 0.3,
                      T_range=(200.0, 600.0), P_range=(1.0e5, 3.0e7), grid: int = 12,
                      steps: int = 30, threads: int = 8) -> workloads.Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    base = workloads.uniform_workload("boundary_props", seed, 1, nc, alpha)
    zs, Ts, Ps = [], [], []
    lp = np.log(np.geomspace(P_range[0], P_range[1], grid))
    while len(Ps) < n:
        k = 4 * (n - len(Ps))
        z = rng.dirichlet(np.full(nc, alpha), size=k)
        T = rng.uniform(T_range[0], T_range[1], k)
        cand = workloads.Workload("cand", k, nc, z, T, np.zeros(k), base.Tc, base.Pc,
                                  base.omega, base.kij)
        labs = np.stack([_labels(cand, np.full(k, np.exp(p)), threads) for p in lp], 1)
        change = np.argmax(labs[:, 1:] != labs[:, :-1], axis=1)
        has = np.any(labs[:, 1:] != labs[:, :-1], axis=1)
        idx = np.where(has)[0][: n - len(Ps)]
        if len(idx) == 0:
            continue
        sub = cand.subset(idx)
        lo, hi = lp[change[idx]], lp[change[idx] + 1]
        llo = labs[idx, change[idx]]
        for _ in range(steps):
            mid = 0.5 * (lo + hi)
            lm = _labels(sub, np.exp(mid), threads)
            same = lm == llo
            lo = np.where(same, mid, lo)
            hi = np.where(same, hi, mid)
        Pb = np.exp(0.5 * (lo + hi))
        zs.append(sub.z)
        Ts.append(sub.T)
        Ps.append(Pb * (1.0 + rng.uniform(-0.02, 0.02, len(idx))))
        Ps = [np.concatenate(Ps)] if len(Ps) > 1 else Ps
        zs = [np.concatenate(zs)] if len(zs) > 1 else zs
        Ts = [np.concatenate(Ts)] if len(Ts) > 1 else Ts
        if len(Ps[0]) >= n:
            break
    z, T, P = zs[0][:n], Ts[0][:n], Ps[0][:n]
    return workloads.Workload(f"boundary_nc{nc}", n, nc, np.ascontiguousarray(z), T, P,
                              base.Tc, base.Pc, base.omega, base.kij)
