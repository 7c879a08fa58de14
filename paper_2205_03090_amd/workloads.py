"""Seeded synthetic flash workloads.

This module only draws random numbers: it holds none of the flash's
arithmetic, so that the GPU path and the CPU oracle can be fed identical
bytes without sharing any thermodynamics.  Every draw uses NumPy's
``Generator(PCG64(seed))`` in a fixed order:

1. one component set (unless ``per_mixture``): Tc ~ U[190, 620] K,
   Pc ~ U[2e6, 5e6] Pa, omega ~ U[0.01, 0.5], then the strict upper triangle
   of k_ij ~ U[0, 0.15] in row-major order (k symmetric, zero diagonal);
2. the feed z ~ Dirichlet(alpha * 1) for all mixtures;
3. T ~ U[T_lo, T_hi] for all mixtures;
4. P ~ U[P_lo, P_hi] for all mixtures.

With ``per_mixture`` the component set of step 1 is drawn per mixture (n
sets, each in the same field order: all Tc, all Pc, all omega, all k).

The paper's own workloads (Sec. 2.3-2.4: Table 1 components, Latin
hypercube + Dirichlet sampling) are replaced by these random-property
workloads; the distributions follow the paper's ranges of T and P and its
Dirichlet feed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Workload:
    name: str
    n: int
    nc: int
    z: np.ndarray       # (n, nc) float64, rows sum to 1
    T: np.ndarray       # (n,) K
    P: np.ndarray       # (n,) Pa
    Tc: np.ndarray      # (nc,) or (n, nc) K
    Pc: np.ndarray      # (nc,) or (n, nc) Pa
    omega: np.ndarray   # (nc,) or (n, nc)
    kij: np.ndarray     # (nc, nc) or (n, nc, nc), symmetric, zero diagonal
    per_mixture: bool = False

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        pick = (lambda a: a[idx]) if self.per_mixture else (lambda a: a)
        return Workload(self.name, len(idx), self.nc, self.z[idx], self.T[idx],
                        self.P[idx], pick(self.Tc), pick(self.Pc), pick(self.omega),
                        pick(self.kij), self.per_mixture)


def _component_set(rng: np.random.Generator, nc: int):
    Tc = rng.uniform(190.0, 620.0, nc)
    Pc = rng.uniform(2.0e6, 5.0e6, nc)
    omega = rng.uniform(0.01, 0.5, nc)
    k = np.zeros((nc, nc))
    iu = np.triu_indices(nc, 1)
    k[iu] = rng.uniform(0.0, 0.15, len(iu[0]))
    k = k + k.T
    return Tc, Pc, omega, k


def uniform_workload(name: str, seed: int, n: int, nc: int, alpha: float,
                     T_range=(200.0, 600.0), P_range=(1.0e5, 2.0e7),
                     per_mixture: bool = False) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    if per_mixture:
        sets = [_component_set(rng, nc) for _ in range(n)]
        Tc = np.stack([s[0] for s in sets])
        Pc = np.stack([s[1] for s in sets])
        omega = np.stack([s[2] for s in sets])
        kij = np.stack([s[3] for s in sets])
    else:
        Tc, Pc, omega, kij = _component_set(rng, nc)
    z = rng.dirichlet(np.full(nc, alpha), size=n)
    T = rng.uniform(T_range[0], T_range[1], n)
    P = rng.uniform(P_range[0], P_range[1], n)
    return Workload(name, n, nc, np.ascontiguousarray(z), T, P, Tc, Pc, omega,
                    kij, per_mixture)


# Named workloads.  Sizes and distributions are those of the flash
# configurations this library is measured on.
SEEDS = {"nc3": 20_250_001, "nc8": 20_250_002, "nc10": 20_250_004, "nc20": 20_250_005}


def nc3_workload(n: int = 10_000, seed: int = SEEDS["nc3"]) -> Workload:
    """Nc = 3, 10,000 mixtures, z ~ Dir(1,1,1), T ~ U[200,600] K,
    P ~ U[1e5, 1e7] Pa, one shared component set."""
    return uniform_workload("nc3_10k", seed, n, 3, 1.0, (200.0, 600.0), (1.0e5, 1.0e7))


def nc8_workload(n: int = 1_000_000, seed: int = SEEDS["nc8"]) -> Workload:
    """Nc = 8, 1,000,000 mixtures, z ~ Dir(0.5 * 1), T ~ U[200,600] K,
    P ~ U[1e5, 2e7] Pa, one shared component set."""
    return uniform_workload("nc8_1m", seed, n, 8, 0.5, (200.0, 600.0), (1.0e5, 2.0e7))


def nc10_workload(n: int = 1_000_000, seed: int = SEEDS["nc10"]) -> Workload:
    """Nc = 10, 1,000,000 mixtures, distributions of the Nc = 8 workload."""
    return uniform_workload("nc10_1m", seed, n, 10, 0.5, (200.0, 600.0), (1.0e5, 2.0e7))


def nc20_workload(n: int = 8_000_000, seed: int = SEEDS["nc20"]) -> Workload:
    """Nc = 20, 8,000,000 mixtures, z ~ Dir(0.3 * 1), T ~ U[200,600] K,
    P ~ U[1e5, 3e7] Pa, one shared component set (the uniform part of the
    hard-case workload; the boundary-hugging part needs the oracle's labels
    and is built by the tests)."""
    return uniform_workload("nc20_8m", seed, n, 20, 0.3, (200.0, 600.0), (1.0e5, 3.0e7))


def cotangents(seed: int, n: int, nc: int):
    """Upstream cotangents on (beta, x, y) ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n), rng.standard_normal((n, nc)), rng.standard_normal((n, nc))


@dataclass
class RaggedWorkload:
    """Mixtures with their own component counts and component sets, packed:
    mixture m's rows are off[m]:off[m+1] of z, Tc, Pc, omega; its k block
    (nc_of[m]^2 values, row-major) starts at koff[m]."""
    name: str
    n: int
    nc_of: np.ndarray   # (n,) int32
    off: np.ndarray     # (n+1,) int64
    koff: np.ndarray    # (n,) int64
    z: np.ndarray
    T: np.ndarray
    P: np.ndarray
    Tc: np.ndarray
    Pc: np.ndarray
    omega: np.ndarray
    kij: np.ndarray

    def group(self, nc: int):
        """(indices, per-mixture-set Workload) of the mixtures with this nc."""
        idx = np.where(self.nc_of == nc)[0]
        rows = (self.off[idx][:, None] + np.arange(nc)[None, :])
        kb = (self.koff[idx][:, None] + np.arange(nc * nc)[None, :])
        w = Workload(f"{self.name}_nc{nc}", len(idx), nc, self.z[rows], self.T[idx],
                     self.P[idx], self.Tc[rows], self.Pc[rows], self.omega[rows],
                     self.kij[kb].reshape(len(idx), nc, nc), True)
        return idx, w


def ragged_workload(name: str, seed: int, n: int, nc_set=(2, 4, 6, 8, 12, 16, 20),
                    alpha: float = 0.5, T_range=(200.0, 600.0),
                    P_range=(1.0e5, 2.0e7)) -> RaggedWorkload:
    """nc ~ U(nc_set) per mixture, then per mixture (in index order) its
    component set (as in step 1 of the module docstring) and its feed
    z ~ Dirichlet(alpha * 1); then T and P for all mixtures."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nc_of = rng.choice(np.asarray(nc_set, dtype=np.int32), size=n).astype(np.int32)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(nc_of)
    ksz = nc_of.astype(np.int64) ** 2
    koff = np.zeros(n, dtype=np.int64)
    koff[1:] = np.cumsum(ksz)[:-1]
    tot, ktot = int(off[-1]), int(ksz.sum())
    z = np.empty(tot); Tc = np.empty(tot); Pc = np.empty(tot); om = np.empty(tot)
    kij = np.empty(ktot)
    for m in range(n):
        nc = int(nc_of[m])
        a, b = off[m], off[m + 1]
        Tc[a:b], Pc[a:b], om[a:b], k = _component_set(rng, nc)
        kij[koff[m]:koff[m] + nc * nc] = k.ravel()
        z[a:b] = rng.dirichlet(np.full(nc, alpha))
    T = rng.uniform(T_range[0], T_range[1], n)
    P = rng.uniform(P_range[0], P_range[1], n)
    return RaggedWorkload(name, n, nc_of, off, koff, z, T, P, Tc, Pc, om, kij)
