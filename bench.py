"""Throughput of the gfx950 SRK PT flash (flashes per second, FP64).

One step = one flash of the whole batch (all stages of the path) with inputs
resident in HBM.  Prints one JSON line (one GPU): `value` is the forward
throughput of the persistent form; `fwd_adjoint` times forward (keeping the
factor) + implicit-function backward; `plain_form` times the plain
one-launch-per-stage-iteration form on the same inputs.

  python bench.py [--steps K] [--warmup W]
                  [--workload nc8_1m|nc3_10k|nc10_1m|nc20_8m|c5_8m|cs2_10m|cs4_5m|cs9_1m|ragged_4m]
                  [--form persistent|plain] [--no-cpu-baseline] [--no-adjoint]
                  [--plain-steps N] [--graph]

Agreement with the CPU oracle is established by the tests (tests/, at the
full sizes and launch configurations timed here), not by this script.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flashes/sec fwd and fwd+adjoint, Nc=8, FP64, ≤1e-10 vs oracle; FP64 roofline %"
FP64_VECTOR_PEAK = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK = 8.0e12


def _kernel_sha() -> str:
    """Hash of the kernel sources and the build script (its flags)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2205_03090_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "paper_2205_03090_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _counters(workload: str) -> dict:
    """Per-launch figures from the committed rocprofv3 counter summary of
    this workload (HBM bytes, issued FP64 VALU flops), or {} when it is
    missing or was taken on a different kernel source or build."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sha") != _kernel_sha():
        return {}
    return t


def _cpu_model() -> str | None:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(run, n: int, threads: int, target_s: float):
    """Oracle flashes/s on the first k mixtures with `threads` threads: one
    warm-up on a short leading sample sizes k so that one run takes about
    target_s, then the median of three timed runs over the same k."""
    k0 = min(n, 2000 * threads)
    t0 = time.perf_counter()
    run(k0, threads)
    rate0 = k0 / max(time.perf_counter() - t0, 1e-6)
    k = int(min(n, max(k0, rate0 * target_s)))
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        run(k, threads)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    return k / dt, k, dt


def _cpu_baseline(name: str, n: int, run, target_s: float = 2.5) -> dict:
    """The oracle, as it stands, on bounded leading samples of the workload:
    on the host cores of this process (at most 16, one GPU's share of the
    host) and on one core (the paper's comparison ran single-core, Sec. 5),
    each the median of three runs after a warm-up."""
    avail = len(os.sched_getaffinity(0))
    threads = max(1, min(16, avail))
    v, k, dt = _oracle_rate(run, n, threads, target_s)
    v1, k1, dt1 = _oracle_rate(run, n, 1, target_s)
    return {"value": v, "unit": "flashes/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} mixtures of {name}, median of 3 runs after a warm-up "
                      f"({dt:.2f} s each)",
            "one_core": {"value": v1, "unit": "flashes/s", "cores": 1,
                         "sample": f"first {k1} mixtures of {name}, median of 3 runs "
                                   f"after a warm-up ({dt1:.2f} s each)"},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": avail}


def cpu_baseline(w) -> dict:
    import oracle

    def run(k, threads):
        oracle.flash(w.subset(np.arange(k)), threads=threads)

    return _cpu_baseline(w.name, w.n, run)


def cpu_baseline_ragged(w) -> dict:
    """As cpu_baseline, one oracle call per nc present in the sample."""
    import oracle

    def run(k, threads):
        idx = np.arange(k)
        for nc in np.unique(w.nc_of[idx]):
            _, sub = w.select(idx[w.nc_of[idx] == nc], int(nc))
            oracle.flash(sub, threads=threads)

    return _cpu_baseline(w.name, w.n, run)


def bench_ragged(args):
    """Mixtures with their own nc and component set in one ptflash_flash_ragged
    call (device-side grouping by nc, then the per-nc pipelines)."""
    import torch
    from paper_2205_03090_amd import _capi, api, workloads
    w = workloads.ragged_4m_workload()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    ti = lambda a, dt: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    args_t = (t(w.z), t(w.T), t(w.P), ti(w.nc_of, torch.int32), ti(w.off, torch.int64),
              ti(w.koff, torch.int64), t(w.Tc), t(w.Pc), t(w.omega), t(w.kij))
    out = api.flash_ragged(*args_t)
    torch.cuda.synchronize()
    for _ in range(max(0, args.warmup - 1)):
        out = api.flash_ragged(*args_t)
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        out = api.flash_ragged(*args_t)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    flops = out.flops.to(torch.int64).sum().item()
    achieved = flops / (avg_ms * 1e-3)
    lab = out.label.cpu().numpy()
    st = out.status.cpu().numpy().astype(np.int64) & 0xffff
    rec = {
        "metric": METRIC, "value": w.n * args.steps / wall, "unit": "flashes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nc": "ragged {2,4,6,8,12,16,20}",
                   "form": "persistent", "props": "per mixture"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK, "traffic": None,
                     "flops_per_flash": flops / w.n, "kernel_ms": avg_ms},
        "two_phase_frac": float((lab == 1).mean()),
        "per_nc": {int(nc): {"n": int((w.nc_of == nc).sum()),
                             "two_phase_frac": float((lab[w.nc_of == nc] == 1).mean())}
                   for nc in np.unique(w.nc_of)},
        "status_counts": {k: int((st & v != 0).sum()) for k, v in _capi.ST.items()},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_ragged(w)
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="nc8_1m")
    ap.add_argument("--form", default="persistent", choices=["persistent", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--flash-only", action="store_true",
                    help="time the flash alone: no adjoint, stability-only, warm-start, "
                         "plain-form or graph legs (for profiler runs)")
    ap.add_argument("--graph", action="store_true",
                    help="also time replays of the persistent flash captured in a HIP graph")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.flash_only:
        args.no_adjoint, args.plain_steps, args.graph = True, 0, False
    if args.calibrate_copy:
        import torch
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(mixtures are independent: a multi-GPU run shards them with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_03090_amd import _capi, api, workloads

    if args.workload == "ragged_4m":
        bench_ragged(args)
        return
    makers = {"nc8_1m": workloads.nc8_workload, "nc3_10k": workloads.nc3_workload,
              "nc10_1m": workloads.nc10_workload, "nc20_8m": workloads.nc20_workload,
              # the hard-case Nc = 20 workload: 30 % within 2 % of the phase
              # boundary (needs the cache written by tests/c5_boundary.py)
              "c5_8m": workloads.c5_workload,
              # the paper's case studies at its largest sizes (Sec. 5.1)
              "cs2_10m": lambda: workloads.case_study_workload("cs2", 10_000_000),
              "cs4_5m": lambda: workloads.case_study_workload("cs4", 5_000_000),
              "cs9_1m": lambda: workloads.case_study_workload("cs9", 1_000_000)}
    w = makers[args.workload]()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    z, T, P, Tc, Pc, om, kij = map(t, (w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij))
    form = _capi.FORM_PERSISTENT if args.form == "persistent" else _capi.FORM_PLAIN
    out = api.flash(z, T, P, Tc, Pc, om, kij, form=form)
    torch.cuda.synchronize()
    for _ in range(max(0, args.warmup - 1)):
        api.flash(z, T, P, Tc, Pc, om, kij, form=form, out=out)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        api.flash(z, T, P, Tc, Pc, om, kij, form=form, out=out)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_ms = float(np.mean(launch_ms))
    value = w.n * args.steps / wall

    flops = out.flops.to(torch.int64).sum().item()
    g = {k: getattr(out, k).cpu().numpy() for k in ("label", "iters", "status")}
    achieved = flops / (avg_ms * 1e-3)
    cnt = _counters(args.workload)
    traffic = cnt.get("bytes_per_launch")

    rec = {
        "metric": METRIC, "value": value, "unit": "flashes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nc": w.nc, "form": args.form},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK,
                     "traffic": traffic, "flops_per_flash": flops / w.n,
                     "kernel_ms": avg_ms},
        "two_phase_frac": float((g["label"] == 1).mean()),
        # the second roofline view: FP64 VALU flops the hardware issued per
        # launch (rocprofv3 FP64 instruction counters, 64 lanes per wave
        # instruction, FMA = 2; transcendental and division sequences
        # included) over this run's launch time; lane_weighted counts only
        # the lanes the exec mask enabled (each stage's issued flops times
        # its SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU))
        "fp64_issued": ({"tflops": cnt["fp64_issued_flops_per_launch"] / (avg_ms * 1e-3) / 1e12,
                         "frac": cnt["fp64_issued_flops_per_launch"] / (avg_ms * 1e-3)
                         / FP64_VECTOR_PEAK,
                         "lane_weighted_frac": (cnt["fp64_lane_weighted_flops_per_launch"]
                                                / (avg_ms * 1e-3) / FP64_VECTOR_PEAK
                                                if "fp64_lane_weighted_flops_per_launch" in cnt
                                                else None)}
                        if "fp64_issued_flops_per_launch" in cnt else None),
        # mean and max iteration counts per slot over the mixtures that ran it
        "iters": {nm: [float(g["iters"][:, k][g["iters"][:, k] > 0].mean())
                       if (g["iters"][:, k] > 0).any() else 0.0, int(g["iters"][:, k].max())]
                  for k, nm in enumerate(_capi.IT_NAMES)},
        "status_counts": {k: int(((g["status"].astype(np.int64) & 0xffff) & v != 0).sum())
                          for k, v in _capi.ST.items()},
    }
    # forward + adjoint: forward keeping the factor, then the implicit-function
    # VJP with seeded N(0,1) cotangents and the batch-reduced k gradient
    if not args.no_adjoint:
        gb, gx, gy = (torch.as_tensor(a, dtype=torch.float64, device=dev)
                      for a in workloads.cotangents(77, w.n, w.nc))
        fo = api.flash(z, T, P, Tc, Pc, om, kij, keep_factor=True)
        api.flash_backward(z, T, P, Tc, Pc, om, kij, fo, gb, gx, gy)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            api.flash(z, T, P, Tc, Pc, om, kij, keep_factor=True, out=fo)
            bw = api.flash_backward(z, T, P, Tc, Pc, om, kij, fo, gb, gx, gy)
        torch.cuda.synchronize()
        wall_a = time.perf_counter() - t1
        rec["fwd_adjoint"] = {"value": w.n * args.steps / wall_a, "unit": "flashes/s",
                              "ms_per_step": wall_a * 1e3 / args.steps,
                              "nan_grad_frac": float(torch.isnan(bw[1]).double().mean().item())}
    if not args.flash_only:
        # stability analysis alone (no phase split), as used to label samples
        st_out = api.stability(z, T, P, Tc, Pc, om, kij)
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        for _ in range(args.steps):
            st_out = api.stability(z, T, P, Tc, Pc, om, kij)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - ts0
        rec["stability_only"] = {"value": w.n * args.steps / wall_s, "unit": "mixtures/s",
                                 "ms_per_step": wall_s * 1e3 / args.steps,
                                 "unstable_frac": float((st_out.label == 1).double().mean().item())}
        # warm start (Sec. 4's integration points) with exact inputs: each mixture
        # hinted with this flash's own label and started from its converged ln K
        # (zeros where single phase: unused behind a stable hint), the bound of
        # the acceleration by a classifier and an initializer
        two = (out.label == 1) & ((out.status.to(torch.int32) & _capi.ST["SPLIT_UNCONV"]) == 0)
        lnk0 = torch.where(two[:, None], torch.log(out.y / out.x), torch.zeros_like(out.x))
        hint = torch.where(two, 1, 0).to(torch.int8)
        wo = api.flash(z, T, P, Tc, Pc, om, kij, lnk0=lnk0, hint=hint)
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        for _ in range(args.steps):
            api.flash(z, T, P, Tc, Pc, om, kij, lnk0=lnk0, hint=hint, out=wo)
        torch.cuda.synchronize()
        wall_w = time.perf_counter() - tw0
        rec["warm_start"] = {"value": w.n * args.steps / wall_w, "unit": "flashes/s",
                             "ms_per_step": wall_w * 1e3 / args.steps,
                             "max_beta_change": float((wo.beta - out.beta)[two].abs().max().item())
                             if bool(two.any()) else 0.0}
    # the same persistent flash captured once into a HIP graph and replayed
    if args.graph:
        g = torch.cuda.CUDAGraph()
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(gs):
            with torch.cuda.graph(g, stream=gs):
                api.flash(z, T, P, Tc, Pc, om, kij, out=out)
        torch.cuda.current_stream().wait_stream(gs)
        g.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        wall_g = time.perf_counter() - tg
        rec["graph_replay"] = {"value": w.n * args.steps / wall_g, "unit": "flashes/s",
                               "ms_per_step": wall_g * 1e3 / args.steps}
    if args.plain_steps > 0:
        api.flash(z, T, P, Tc, Pc, om, kij, form=_capi.FORM_PLAIN, out=out)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.plain_steps):
            api.flash(z, T, P, Tc, Pc, om, kij, form=_capi.FORM_PLAIN, out=out)
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - t2
        rec["plain_form"] = {"value": w.n * args.plain_steps / wall_p, "unit": "flashes/s",
                             "ms_per_step": wall_p * 1e3 / args.plain_steps,
                             "persistent_speedup": (w.n * args.plain_steps / wall_p) and
                             value / (w.n * args.plain_steps / wall_p)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
