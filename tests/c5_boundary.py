"""The boundary-hugging part of the Nc = 20 hard-case workload at its full
size: 30 % of 8,000,000 mixtures placed, by bisection in pressure on the
oracle's stability decision, within 2 % of a phase boundary.  Test
infrastructure: it calls the oracle; the product reads only the file it
writes (``workloads.c5_workload``).

Recipe (NumPy PCG64, seeded per block so that a block can be redrawn alone):
the component set is that of the uniform Nc = 20 workload
(``workloads.nc20_workload``); candidate block b draws, from
Generator(PCG64([C5_SEED, b])), z ~ Dirichlet(0.3 * 1) (BLOCK rows),
T ~ U[200, 600] K and u ~ U[-0.02, 0.02].  A candidate is kept when the
oracle's decision (stable, or sent to the phase split) changes along the
geometric grid of GRID pressures in [1e5, 3e7] Pa; the first change is
bisected STEPS times in ln P (to about 1e-4 relative), the midpoint of the
last bracket is P_b, stored in float32, and the mixture gets
P = P_b (1 + u).  Blocks are processed in order until N_BOUNDARY mixtures
are kept.

Run ``python tests/c5_boundary.py`` to write the cache (tens of minutes on
eight cores); it holds, per kept mixture, the block, the row in the block and
P_b.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2205_03090_amd import workloads  # noqa: E402

C5_SEED = workloads.C5_SEED
BLOCK = workloads.C5_BLOCK
N_BOUNDARY = workloads.C5_N_BOUNDARY
GRID = 12
STEPS = 12
P_RANGE = (1.0e5, 3.0e7)
CACHE = workloads.C5_CACHE


def _decisions(base, z, T, P, threads):
    import oracle
    w = workloads.Workload("c5b", len(T), base.nc, z, T, P, base.Tc, base.Pc, base.omega,
                           base.kij)
    return oracle.flash(w, threads=threads, decision_only=1)["label"].astype(np.int8)


def place_block(base, b: int, threads: int):
    """Kept rows of candidate block b and their boundary pressures P_b."""
    z, T, _ = workloads.c5_candidates(b)
    lp = np.log(np.geomspace(P_RANGE[0], P_RANGE[1], GRID))
    labs = np.stack([_decisions(base, z, T, np.full(len(T), np.exp(p)), threads) for p in lp], 1)
    chg = labs[:, 1:] != labs[:, :-1]
    rows = np.where(chg.any(axis=1))[0]
    first = np.argmax(chg[rows], axis=1)
    lo, hi = lp[first], lp[first + 1]
    l0 = labs[rows, first]
    zs, Ts = z[rows], T[rows]
    for _ in range(STEPS):
        mid = 0.5 * (lo + hi)
        same = _decisions(base, zs, Ts, np.exp(mid), threads) == l0
        lo = np.where(same, mid, lo)
        hi = np.where(same, hi, mid)
    return rows.astype(np.uint16), np.exp(0.5 * (lo + hi)).astype(np.float32)


def build(threads: int = 8, path: str = CACHE, verbose: bool = True) -> str:
    base = workloads.nc20_workload(n=1)
    blocks, rows, pb = [], [], []
    kept, b, t0 = 0, 0, time.perf_counter()
    while kept < N_BOUNDARY:
        r, p = place_block(base, b, threads)
        r, p = r[:N_BOUNDARY - kept], p[:N_BOUNDARY - kept]
        blocks.append(np.full(len(r), b, np.uint16))
        rows.append(r)
        pb.append(p)
        kept += len(r)
        b += 1
        if verbose:
            print(f"block {b}: kept {kept} ({len(r) / BLOCK:.3f} of the block), "
                  f"{time.perf_counter() - t0:.0f} s", flush=True)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, block=np.concatenate(blocks), row=np.concatenate(rows),
             pb=np.concatenate(pb), seed=np.int64(C5_SEED), grid=np.int64(GRID),
             steps=np.int64(STEPS))
    os.replace(tmp, path)
    return path


if __name__ == "__main__":
    th = int(sys.argv[1]) if len(sys.argv) > 1 else min(16, len(os.sched_getaffinity(0)))
    print(build(threads=th))
