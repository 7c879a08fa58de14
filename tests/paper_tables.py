"""Loads the component table printed in the paper (tests/golden)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def table1():
    rows = [l.strip().split(",") for l in open(os.path.join(HERE, "golden", "table1_components.csv"))
            if l.strip() and not l.startswith("#")][1:]
    names = [r[0] for r in rows]
    Pc = np.array([float(r[1]) for r in rows]) * 1e6
    Tc = np.array([float(r[2]) for r in rows])
    om = np.array([float(r[3]) for r in rows])
    return names, Tc, Pc, om


def components(names_wanted):
    names, Tc, Pc, om = table1()
    idx = [names.index(n) for n in names_wanted]
    k = np.zeros((len(idx), len(idx)))
    for a, ia in enumerate(idx):
        for b, ib in enumerate(idx):
            if {names[ia], names[ib]} == {"CH4", "CO2"}:
                k[a, b] = 0.0882
    return Tc[idx], Pc[idx], om[idx], k


def _rows(name):
    lines = [l.strip() for l in open(os.path.join(HERE, "golden", name))
             if l.strip() and not l.startswith("#")]
    head = lines[0].split(",")
    return head, [l.split(",") for l in lines[1:]]


def table2():
    """{fluid: [(lo, hi) per Table 1 component]} as mole fractions."""
    head, rows = _rows("table2_composition_ranges.csv")
    fluids = [h[:-3] for h in head[1::2]]
    out = {f: [] for f in fluids}
    for r in rows:
        for k, f in enumerate(fluids):
            out[f].append((float(r[1 + 2 * k]) / 100.0, float(r[2 + 2 * k]) / 100.0))
    return [r[0] for r in rows], out


def table3():
    """{fluid: (alpha_CH4, alpha_C2H6, alpha_C7H16+)}."""
    _, rows = _rows("table3_dirichlet_alpha.csv")
    return {r[0]: tuple(float(v) for v in r[1:]) for r in rows}


def table5():
    """{stage: (samples, converged_pct, max_iter)}."""
    _, rows = _rows("table5_profiler_nc9.csv")
    return {r[0]: (int(r[1]), float(r[2]), int(r[3])) for r in rows}
