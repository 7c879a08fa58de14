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
