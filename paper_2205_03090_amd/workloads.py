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

These random-property workloads follow the paper's ranges of T and P and
its Dirichlet feed.  The paper's own three case studies (Sec. 2.3-2.4:
Table 1 components, Latin hypercube + Dirichlet sampling, Tables 2 and 3
for the nine-component fluids) are built by ``case_study_workload``.
"""
from __future__ import annotations

import os
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
SEEDS = {"nc3": 20_250_001, "nc8": 20_250_002, "ragged": 20_250_003, "nc10": 20_250_004,
         "nc20": 20_250_005}


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


# The hard-case Nc = 20 workload (30 % of its mixtures within 2 % of a phase
# boundary in pressure, the rest the uniform draw above).  The boundary
# pressures come from bisection on the oracle's stability decision, written
# once by tests/c5_boundary.py to a cache file; this module only redraws the
# candidates' random numbers and reads that file.
C5_SEED = 20_250_006
C5_BLOCK = 1 << 16
C5_N = 8_000_000
C5_N_BOUNDARY = 2_400_000
C5_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "tests", "data", "c5_boundary_nc20.npz")


def c5_candidates(b: int):
    """Candidate block b of the boundary part: z ~ Dirichlet(0.3 * 1),
    T ~ U[200, 600] K and the relative offset u ~ U[-0.02, 0.02] of the
    pressure from the boundary, C5_BLOCK rows each."""
    rng = np.random.Generator(np.random.PCG64([C5_SEED, b]))
    z = rng.dirichlet(np.full(20, 0.3), size=C5_BLOCK)
    T = rng.uniform(200.0, 600.0, C5_BLOCK)
    u = rng.uniform(-0.02, 0.02, C5_BLOCK)
    return z, T, u


def c5_workload(path: str = C5_CACHE) -> Workload:
    """Nc = 20, 8,000,000 mixtures, one shared component set (that of
    nc20_workload): 5,600,000 drawn as nc20_workload and 2,400,000 placed
    within 2 % of the oracle's phase boundary (P = P_b (1 + u), P_b from the
    cache file), shuffled together by a seeded permutation."""
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: write it with `python tests/c5_boundary.py`")
    with np.load(path) as f:
        block, row, pb = f["block"].astype(np.int64), f["row"].astype(np.int64), f["pb"]
    if len(pb) != C5_N_BOUNDARY:
        raise ValueError(f"{path} holds {len(pb)} boundary mixtures, not {C5_N_BOUNDARY}")
    uni = nc20_workload(n=C5_N - C5_N_BOUNDARY)
    zb = np.empty((C5_N_BOUNDARY, 20))
    Tb = np.empty(C5_N_BOUNDARY)
    Pb = np.empty(C5_N_BOUNDARY)
    for b in np.unique(block):
        sel = np.where(block == b)[0]
        z, T, u = c5_candidates(int(b))
        zb[sel] = z[row[sel]]
        Tb[sel] = T[row[sel]]
        Pb[sel] = pb[sel].astype(np.float64) * (1.0 + u[row[sel]])
    perm = np.random.Generator(np.random.PCG64(C5_SEED + 1)).permutation(C5_N)
    z = np.concatenate([uni.z, zb])[perm]
    T = np.concatenate([uni.T, Tb])[perm]
    P = np.concatenate([uni.P, Pb])[perm]
    w = Workload("c5_8m", C5_N, 20, np.ascontiguousarray(z), T, P, uni.Tc, uni.Pc, uni.omega,
                 uni.kij)
    w.boundary = perm >= C5_N - C5_N_BOUNDARY   # rows of the boundary part
    return w


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
        return self.select(np.where(self.nc_of == nc)[0], nc)

    def select(self, idx, nc: int):
        """(idx, per-mixture-set Workload) of the given mixtures, all of which
        have this nc."""
        idx = np.asarray(idx)
        rows = (self.off[idx][:, None] + np.arange(nc)[None, :])
        kb = (self.koff[idx][:, None] + np.arange(nc * nc)[None, :])
        w = Workload(f"{self.name}_nc{nc}", len(idx), nc, self.z[rows], self.T[idx],
                     self.P[idx], self.Tc[rows], self.Pc[rows], self.omega[rows],
                     self.kij[kb].reshape(len(idx), nc, nc), True)
        return idx, w


def ragged_workload_vec(name: str, seed: int, n: int, nc_set=(2, 4, 6, 8, 12, 16, 20),
                        alpha: float = 0.5, T_range=(200.0, 600.0),
                        P_range=(1.0e5, 2.0e7)) -> RaggedWorkload:
    """The distributions of ragged_workload, drawn group by group for large n:
    nc ~ U(nc_set) per mixture; then, for each nc of nc_set in increasing
    order, the component sets of all mixtures with that nc (all their Tc, then
    Pc, then omega, then the strict upper k triangles in row-major order) and
    their feeds z ~ Dirichlet(alpha * 1); then T and P for all mixtures."""
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
    for nc in sorted(set(int(v) for v in nc_set)):
        idx = np.where(nc_of == nc)[0]
        cnt = len(idx)
        rows = (off[idx][:, None] + np.arange(nc)[None, :]).ravel()
        Tc[rows] = rng.uniform(190.0, 620.0, (cnt, nc)).ravel()
        Pc[rows] = rng.uniform(2.0e6, 5.0e6, (cnt, nc)).ravel()
        om[rows] = rng.uniform(0.01, 0.5, (cnt, nc)).ravel()
        iu = np.triu_indices(nc, 1)
        k = np.zeros((cnt, nc, nc))
        k[:, iu[0], iu[1]] = rng.uniform(0.0, 0.15, (cnt, len(iu[0])))
        k += k.transpose(0, 2, 1)
        kij[(koff[idx][:, None] + np.arange(nc * nc)[None, :]).ravel()] = k.reshape(-1)
        del k
        z[rows] = rng.dirichlet(np.full(nc, alpha), size=cnt).ravel()
    T = rng.uniform(T_range[0], T_range[1], n)
    P = rng.uniform(P_range[0], P_range[1], n)
    return RaggedWorkload(name, n, nc_of, off, koff, z, T, P, Tc, Pc, om, kij)


def per_mixture_workload_vec(name: str, seed: int, n: int, nc: int, alpha: float,
                             T_range=(200.0, 600.0), P_range=(1.0e5, 2.0e7)) -> Workload:
    """One component set per mixture, as uniform_workload(per_mixture=True), drawn
    vectorised for large n: all Tc, then Pc, then omega (n x nc each), then the
    strict upper k triangles (n x nc(nc-1)/2, row-major), then z, T, P."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Tc = rng.uniform(190.0, 620.0, (n, nc))
    Pc = rng.uniform(2.0e6, 5.0e6, (n, nc))
    om = rng.uniform(0.01, 0.5, (n, nc))
    iu = np.triu_indices(nc, 1)
    k = np.zeros((n, nc, nc))
    k[:, iu[0], iu[1]] = rng.uniform(0.0, 0.15, (n, len(iu[0])))
    k += k.transpose(0, 2, 1)
    z = rng.dirichlet(np.full(nc, alpha), size=n)
    T = rng.uniform(T_range[0], T_range[1], n)
    P = rng.uniform(P_range[0], P_range[1], n)
    return Workload(name, n, nc, np.ascontiguousarray(z), T, P, Tc, Pc, om, k, True)


def ragged_4m_workload(n: int = 4_000_000, seed: int = SEEDS["ragged"]) -> RaggedWorkload:
    """4,000,000 mixtures, nc ~ U{2,4,6,8,12,16,20}, one component set per
    mixture, z ~ Dir(0.5 * 1), T ~ U[200,600] K, P ~ U[1e5, 2e7] Pa."""
    return ragged_workload_vec("ragged_4m", seed, n)


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


# ---------------------------------------------------------------------------
# The paper's case studies (Sec. 2.3 "Case studies", Sec. 2.4 "Data
# generation").
# ---------------------------------------------------------------------------

# Table 1: name, Pc [MPa], Tc [K], acentric factor.
PAPER_COMPONENTS = (
    ("CH4", 4.6, 190.55, 0.0111),
    ("C2H6", 4.875, 305.43, 0.097),
    ("C3H8", 4.268, 369.82, 0.1536),
    ("nC4H10", 3.796, 425.16, 0.2008),
    ("nC5H12", 3.3332, 467.15, 0.2635),
    ("C6H14", 2.9688, 507.4, 0.296),
    ("C7H16+", 2.622, 604.5, 0.3565),
    ("CO2", 7.382, 304.19, 0.225),
    ("N2", 3.3944, 126.25, 0.039),
)
# Sec. 2.3: the only non-zero binary interaction parameter.
KIJ_CH4_CO2 = 0.0882

# Sec. 2.3: the components of the three case studies and their T, P boxes.
CASE_STUDIES = {
    "cs2": (("CH4", "C6H14"), (200.0, 500.0), (1.0e5, 1.0e7)),
    "cs4": (("CH4", "C2H6", "C3H8", "nC4H10"), (200.0, 500.0), (1.0e5, 1.0e7)),
    "cs9": (tuple(c[0] for c in PAPER_COMPONENTS), (200.0, 600.0), (5.0e6, 2.5e7)),
}

FLUIDS = ("wet_gas", "gas_condensate", "volatile_oil", "black_oil")

# Table 2: mole-fraction box of each fluid type, in the order of Table 1.
FLUID_RANGES = {
    "wet_gas": ((0.80, 1.00), (0.02, 0.07), (0.0, 0.03), (0.0, 0.02), (0.0, 0.02),
                (0.0, 0.02), (0.0, 0.01), (0.0, 0.02), (0.0, 0.005)),
    "gas_condensate": ((0.60, 0.80), (0.05, 0.10), (0.0, 0.04), (0.0, 0.03), (0.0, 0.02),
                       (0.0, 0.02), (0.05, 0.10), (0.0, 0.035), (0.0, 0.005)),
    "volatile_oil": ((0.50, 0.70), (0.06, 0.10), (0.0, 0.045), (0.0, 0.03), (0.0, 0.02),
                     (0.0, 0.02), (0.10, 0.30), (0.0, 0.02), (0.0, 0.005)),
    "black_oil": ((0.20, 0.40), (0.03, 0.06), (0.0, 0.015), (0.0, 0.015), (0.0, 0.01),
                  (0.0, 0.02), (0.45, 0.65), (0.0, 0.001), (0.0, 0.005)),
}

# Table 3: Dirichlet concentrations (CH4, C2H6, C7H16+); every other
# component has concentration 1.
FLUID_ALPHA = {
    "wet_gas": (100.0, 5.0, 1.0),
    "gas_condensate": (40.0, 5.0, 5.0),
    "volatile_oil": (55.0, 8.0, 20.0),
    "black_oil": (25.0, 4.0, 40.0),
}

CASE_SEEDS = {"cs2": 20_250_011, "cs4": 20_250_012, "cs9": 20_250_013}


@dataclass
class CaseStudyWorkload(Workload):
    fluid: np.ndarray = None   # (n,) int8 index into FLUIDS (nine components), else None


def case_components(names):
    """Tc, Pc, omega and k of the named Table 1 components (k = 0 except
    for the CH4-CO2 pair)."""
    table = {c[0]: c for c in PAPER_COMPONENTS}
    Tc = np.array([table[n][2] for n in names])
    Pc = np.array([table[n][1] for n in names]) * 1.0e6
    om = np.array([table[n][3] for n in names])
    k = np.zeros((len(names), len(names)))
    for a, na in enumerate(names):
        for b, nb in enumerate(names):
            if {na, nb} == {"CH4", "CO2"}:
                k[a, b] = KIJ_CH4_CO2
    return Tc, Pc, om, k


def latin_hypercube(rng: np.random.Generator, m: int, d: int) -> np.ndarray:
    """m points of a Latin hypercube in [0, 1)^d: in every dimension each of
    the m strata [i/m, (i+1)/m) holds exactly one point, placed uniformly in
    it.  Per dimension: one permutation, then m uniforms."""
    u = np.empty((m, d))
    for j in range(d):
        u[:, j] = (rng.permutation(m) + rng.random(m)) / m
    return u


def fluid_alpha(fluid: str) -> np.ndarray:
    a = np.ones(len(PAPER_COMPONENTS))
    a[0], a[1], a[6] = FLUID_ALPHA[fluid]
    return a


def _lead_component(alpha: np.ndarray, box: np.ndarray) -> int:
    """Among the components with concentration 1, the one whose box has the
    smallest marginal probability (Beta(1, A - 1), CDF 1 - (1 - x)^(A - 1))."""
    b = alpha.sum() - 1.0
    best, arg = 2.0, -1
    for j in range(len(alpha)):
        if alpha[j] != 1.0:
            continue
        p = (1.0 - box[j, 0]) ** b - (1.0 - box[j, 1]) ** b
        if p < best:
            best, arg = p, j
    return arg


def truncated_dirichlet(rng: np.random.Generator, alpha: np.ndarray, box: np.ndarray,
                        m: int, batch: int = 1 << 18) -> np.ndarray:
    """m draws of Dirichlet(alpha) conditioned on lo_i <= z_i <= hi_i for all
    i (box[i] = (lo_i, hi_i)): the feeds the paper keeps after rejecting
    Dirichlet samples outside a fluid type's box.

    Exact rejection sampling, with one shortcut: a lead component j of
    concentration 1 is drawn from its marginal Beta(1, A - 1) (A = sum alpha)
    restricted to its interval, by the closed-form inverse CDF, and the rest
    as (1 - z_j) v with v ~ Dirichlet(alpha without j), which is independent
    of z_j (Dirichlet neutrality).  The density of a draw is then the
    Dirichlet density times the indicator of z_j's interval over a constant,
    so rejecting draws that leave the box of the other components yields the
    box-restricted Dirichlet, with fewer rejections than plain rejection.

    Per batch, in this order: ``batch`` uniforms for z_j, then one
    ``rng.dirichlet`` call for v."""
    nc = len(alpha)
    j = _lead_component(alpha, box)
    rest = np.array([i for i in range(nc) if i != j])
    b = alpha.sum() - 1.0
    F = lambda x: 1.0 - (1.0 - x) ** b
    flo, fhi = F(box[j, 0]), F(box[j, 1])
    out, have = np.empty((m, nc)), 0
    while have < m:
        u = flo + (fhi - flo) * rng.random(batch)
        zj = 1.0 - (1.0 - u) ** (1.0 / b)
        v = rng.dirichlet(alpha[rest], size=batch)
        z = np.empty((batch, nc))
        z[:, j] = zj
        z[:, rest] = (1.0 - zj)[:, None] * v
        ok = np.all((z >= box[:, 0]) & (z <= box[:, 1]), axis=1) & np.all(z > 0.0, axis=1)
        take = z[ok][: m - have]
        out[have:have + len(take)] = take
        have += len(take)
    return out


def case_study_workload(case: str, n: int, seed: int | None = None) -> CaseStudyWorkload:
    """One of the paper's three case studies (Sec. 2.3-2.4), seeded.

    cs2 (CH4, C6H14) and cs4 (CH4, C2H6, C3H8, nC4H10): P in [0.1, 10] MPa,
    T in [200, 500] K, z over the whole simplex.  One Latin hypercube of n
    points in (P, T, u_1 .. u_nc); y_i = Gamma(1, 1) quantile of u_i
    (= -ln(1 - u_i)), z = y / sum y, i.e. z ~ Dirichlet(1).

    cs9 (all Table 1 components, k(CH4, CO2) = 0.0882): P in [5, 25] MPa,
    T in [200, 600] K; the four fluid types equally represented (n // 4 each,
    the first n % 4 types one more), each z ~ Dirichlet(Table 3 alpha)
    restricted to the type's Table 2 box (``truncated_dirichlet``), types in
    the order of FLUIDS; then one permutation shuffles the rows and one Latin
    hypercube of n points in (P, T) gives the conditions.  The paper draws
    z from the same hypercube as P and T and then rejects; at the acceptance
    rates of these boxes (about 0.1 % to 14 %) the kept feeds follow the
    box-restricted Dirichlet, which is drawn here directly."""
    names, (T_lo, T_hi), (P_lo, P_hi) = CASE_STUDIES[case]
    seed = CASE_SEEDS[case] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    Tc, Pc, om, k = case_components(names)
    nc = len(names)
    fluid = None
    if case != "cs9":
        u = latin_hypercube(rng, n, 2 + nc)
        y = -np.log1p(-u[:, 2:])
        z = y / y.sum(axis=1, keepdims=True)
        P = P_lo + (P_hi - P_lo) * u[:, 0]
        T = T_lo + (T_hi - T_lo) * u[:, 1]
    else:
        parts, tags = [], []
        for f, name in enumerate(FLUIDS):
            m = n // 4 + (1 if f < n % 4 else 0)
            parts.append(truncated_dirichlet(rng, fluid_alpha(name),
                                             np.asarray(FLUID_RANGES[name]), m))
            tags.append(np.full(m, f, dtype=np.int8))
        perm = rng.permutation(n)
        z = np.concatenate(parts)[perm]
        fluid = np.concatenate(tags)[perm]
        u = latin_hypercube(rng, n, 2)
        P = P_lo + (P_hi - P_lo) * u[:, 0]
        T = T_lo + (T_hi - T_lo) * u[:, 1]
    return CaseStudyWorkload(f"{case}_{n}", n, nc, np.ascontiguousarray(z), T, P, Tc, Pc,
                             om, k, False, fluid)
