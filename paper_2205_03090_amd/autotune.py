"""Chooses, per component count and layout of the component sets, the launch
shape of the persistent flash on this GPU: the lanes per mixture of each of
the two trust-region stages and of the two substitution stages (1, or a group
of 16 or 32 lanes) and the threads per block, by timing candidates on seeded
sample workloads: every pair of trust-region choices first (substitution
lanes and block as they stand), then the substitution choice, then the
block, each step keeping the best so far.

  python -m paper_2205_03090_amd.autotune --out DIR [--n 4000000] [--n-pm 1000000]

writes DIR/tuned_gfx950.hpp (the table the library compiles in as its
default, csrc/tuned_gfx950.hpp; component counts outside --nc keep the
current entries) and DIR/autotune_gfx950.md (the timings).

  python -m paper_2205_03090_amd.autotune --out DIR --crossover

times, for small and medium batches, the persistent form at its tuned
launch shape against the fused form (64- and 128-thread blocks) and writes
DIR/fused_crossover_gfx950.md, the measurement behind the batch size up to
which a persistent call with the launch shape left to the library runs
fused (fused_max_n in csrc/flash_launch.hpp).  Sample: uniform_workload(seed
32000 + nc, alpha 0.5, the same T and P ranges).
The sample for nc is uniform_workload(seed 30000 + nc, alpha 0.5,
T in [200, 600] K, P in [1e5, 2e7] Pa) with one shared component set, and
per_mixture_workload_vec(seed 31000 + nc, same distributions) with one set
per mixture.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import _capi, build as _build, workloads

GROUP_MIN_NC = 8   # the group variants are compiled from this nc on
BLOCKS = (64, 128, 256)


def lane_choices(nc: int):
    lanes = [1]
    if nc >= GROUP_MIN_NC and nc <= 16:
        lanes.append(16)
    if nc >= GROUP_MIN_NC:
        lanes.append(32)
    return lanes


def time_one(args, la: int, lb: int, ls: int, block: int, reps: int) -> float:
    import torch
    from . import api
    kw = dict(lanes_per_mixture=la, lanes_split=lb, lanes_ss=ls, block=block)
    out = api.flash(*args, **kw)
    api.flash(*args, out=out, **kw)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.flash(*args, out=out, **kw)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def current_table():
    """The table compiled into the library (csrc/tuned_gfx950.hpp):
    (lanes_sa, lanes_sp, blocks), each [layout][nc]."""
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tuned_gfx950.hpp")
    with open(path) as f:
        text = f.read()

    def table(name):
        body = re.search(name + r"\[2\]\[21\] = \{(.*?)\};", text, re.S).group(1)
        rows = re.findall(r"\{([^{}]*)\}", body)
        return [[int(v) for v in r.split(",")] for r in rows]

    ss = table("kTunedLanesSs") if "kTunedLanesSs" in text else [[1] * 21, [1] * 21]
    return table("kTunedLanesSa"), table("kTunedLanesSp"), ss, table("kTunedBlock")


def header(lanes_sa, lanes_sp, lanes_ss, blocks) -> str:
    """lanes_sa etc.: [layout][nc], layout 0 = shared set, 1 = one per mixture."""
    def row(v):
        return "{" + ", ".join(str(x) for x in v) + "}"
    return f"""// tuned_gfx950.hpp -- launch shape of the persistent flash per component
// count on gfx950: lanes per mixture of the stability and of the split
// trust-region stage and of the two substitution stages (1: one mixture per
// lane; 16 or 32: one group of that many lanes per mixture) and threads per
// block, for a shared component set (row 0) and for one set per mixture
// (row 1).  Written by autotune.py from timed runs (the timings are in the
// autotune summary next to the profiles).
#pragma once

namespace ptf {{

constexpr int kTunedLanesSa[2][21] = {{{row(lanes_sa[0])},
                                       {row(lanes_sa[1])}}};
constexpr int kTunedLanesSp[2][21] = {{{row(lanes_sp[0])},
                                       {row(lanes_sp[1])}}};
constexpr int kTunedLanesSs[2][21] = {{{row(lanes_ss[0])},
                                       {row(lanes_ss[1])}}};
constexpr int kTunedBlock[2][21] = {{{row(blocks[0])},
                                     {row(blocks[1])}}};

constexpr int tuned_lanes_sa(int nc, bool pm)
{{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSa[pm ? 1 : 0][nc] : 1;
}}

constexpr int tuned_lanes_sp(int nc, bool pm)
{{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSp[pm ? 1 : 0][nc] : 1;
}}

constexpr int tuned_lanes_ss(int nc, bool pm)
{{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSs[pm ? 1 : 0][nc] : 1;
}}

constexpr int tuned_block(int nc, bool pm)
{{
    return (nc >= 0 && nc <= 20) ? kTunedBlock[pm ? 1 : 0][nc] : 256;
}}

}}  // namespace ptf
"""


CROSS_NC = (3, 5, 8, 12, 16, 20)
CROSS_N = (1_000, 3_000, 10_000, 30_000, 100_000, 300_000)


def fused_default(nc: int, n: int) -> bool:
    """The library's rule (fused_max_n) for a call that leaves the launch
    shape to it."""
    return n <= (150_000 if nc <= 8 else 400_000 // nc)


def crossover(a):
    import torch
    from . import api
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
    _, _, _, blocks = current_table()
    lines = ["# Fused against persistent form by batch size (gfx950)", "",
             f"Command: `python -m paper_2205_03090_amd.autotune --out <dir> --crossover "
             f"--reps {a.reps}`", "",
             "Sample per (nc, n): uniform_workload(seed 32000 + nc, alpha 0.5, T in [200, 600] K, "
             f"P in [1e5, 2e7] Pa, one shared set); median of {a.reps} timed flashes after two "
             "untimed ones (host clock around each call, launch included). The persistent "
             "form runs at the tuned launch shape; 'default' is the form a call that leaves "
             "the launch shape to the library takes.", "",
             "| nc | n | persistent ms | fused ms (64) | fused ms (128) | default | "
             "default is the faster |", "|---|---|---|---|---|---|---|"]
    for nc in CROSS_NC:
        for n in CROSS_N:
            if n * nc > 2_000_000:
                continue
            w = workloads.uniform_workload(f"cross{nc}", 32_000 + nc, n, nc, 0.5,
                                           (200.0, 600.0), (1.0e5, 2.0e7))
            args = [t(v) for v in (w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij)]
            ms = {}
            for name, kw in (("pers", dict(block=blocks[0][nc])),
                             ("f64", dict(form=_capi.FORM_FUSED, block=64)),
                             ("f128", dict(form=_capi.FORM_FUSED, block=128))):
                out = api.flash(*args, **kw)
                api.flash(*args, out=out, **kw)
                ts = []
                for _ in range(a.reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    api.flash(*args, out=out, **kw)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                ms[name] = 1e3 * float(np.median(ts))
            fused = fused_default(nc, n)
            ok = (ms["f64"] <= ms["pers"]) == fused
            lines.append(f"| {nc} | {n} | {ms['pers']:.3f} | {ms['f64']:.3f} | "
                         f"{ms['f128']:.3f} | {'fused' if fused else 'persistent'} | "
                         f"{'yes' if ok else 'no'} |")
            print(lines[-1], flush=True)
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, "fused_crossover_gfx950.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=4_000_000)
    ap.add_argument("--n-pm", type=int, default=1_000_000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--nc", type=str, default=f"2-{_build.MAX_NC}")
    ap.add_argument("--crossover", action="store_true")
    a = ap.parse_args()
    if a.crossover:
        return crossover(a)
    import torch
    lo, hi = (int(x) for x in a.nc.split("-"))
    dev = torch.device("cuda", 0)
    # component counts outside --nc keep the library's current choice
    lanes_sa, lanes_sp, lanes_ss, blocks = current_table()
    lines = ["# Launch-shape autotune (gfx950)", "",
             f"Command: `python -m paper_2205_03090_amd.autotune --out <dir> --n {a.n} "
             f"--n-pm {a.n_pm} --reps {a.reps} --nc {a.nc}`", "",
             f"Samples per nc: {a.n} mixtures of uniform_workload(seed 30000 + nc, alpha 0.5, "
             "T in [200, 600] K, P in [1e5, 2e7] Pa, one shared set), and "
             f"{a.n_pm} mixtures of per_mixture_workload_vec(seed 31000 + nc, the same "
             f"distributions, one set per mixture); median of {a.reps} timed flashes "
             "after two untimed ones.", "",
             "| sets | nc | lanes (stability TR) | lanes (split TR) | lanes (substitutions) "
             "| block | ms | flashes/s |",
             "|---|---|---|---|---|---|---|---|"]
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
    for pm in (0, 1):
        for nc in range(lo, hi + 1):
            if pm:
                n = a.n_pm
                w = workloads.per_mixture_workload_vec(f"tunepm{nc}", 31_000 + nc, n, nc, 0.5)
            else:
                n = a.n
                w = workloads.uniform_workload(f"tune{nc}", 30_000 + nc, n, nc, 0.5,
                                               (200.0, 600.0), (1.0e5, 2.0e7))
            args = [t(v) for v in (w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij)]
            del w
            tag = "per mixture" if pm else "shared"
            timed = {}

            def timing(cfg):
                if cfg not in timed:
                    dt = time_one(args, *cfg, a.reps)
                    timed[cfg] = dt
                    lines.append(f"| {tag} | {nc} | {cfg[0]} | {cfg[1]} | {cfg[2]} | {cfg[3]} | "
                                 f"{dt * 1e3:.3f} | {n / dt / 1e6:.1f} M |")
                    print(f"{tag} nc {nc} lanes {cfg[0]}/{cfg[1]}/{cfg[2]} block {cfg[3]}: "
                          f"{dt * 1e3:.3f} ms", flush=True)
                return timed[cfg]

            ls = lane_choices(nc)
            cur = (lanes_sa[pm][nc] if lanes_sa[pm][nc] in ls else 1,
                   lanes_sp[pm][nc] if lanes_sp[pm][nc] in ls else 1,
                   lanes_ss[pm][nc] if lanes_ss[pm][nc] in ls else 1, blocks[pm][nc])
            best = min(((la, lb, cur[2], cur[3]) for la in ls for lb in ls), key=timing)
            best = min(((best[0], best[1], lss, best[3]) for lss in ls), key=timing)
            best = min(((best[0], best[1], best[2], k) for k in BLOCKS), key=timing)
            lanes_sa[pm][nc], lanes_sp[pm][nc], lanes_ss[pm][nc], blocks[pm][nc] = best
            lines.append(f"| {tag} | **{nc}** | **{best[0]}** | **{best[1]}** | **{best[2]}** "
                         f"| **{best[3]}** | chosen | |")
            del args
            torch.cuda.empty_cache()
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, "tuned_gfx950.hpp"), "w") as f:
        f.write(header(lanes_sa, lanes_sp, lanes_ss, blocks))
    with open(os.path.join(a.out, "autotune_gfx950.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("lanes", lanes_sa, lanes_sp, lanes_ss, "\nblocks", blocks)


if __name__ == "__main__":
    main()
