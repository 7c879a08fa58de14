"""Builds and runs the host build of the flash's per-mixture work items
(driver.cpp) under the address and undefined-behaviour sanitizers.  The
executables are cached per component count under tests/host_items/build/
(git-ignored), keyed by a hash of the sources they compile."""
from __future__ import annotations

import hashlib
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2205_03090_amd", "csrc")
BUILD = os.path.join(HERE, "build")
SOURCES = [os.path.join(HERE, "driver.cpp"), os.path.join(CSRC, "flash_stages.hpp"),
           os.path.join(CSRC, "srk_device.hpp"), os.path.join(CSRC, "flash_api.hpp"),
           os.path.join(ROOT, "include", "ptflash.h"), os.path.join(HERE, "stub", "lane_value.hpp"),
           os.path.join(HERE, "stub", "hip", "hip_runtime.h"),
           os.path.join(HERE, "stub", "hip", "hip_runtime_api.h")]
# address + undefined behaviour (g++), or uninitialised reads (clang's
# memory sanitizer, which needs every byte it checks to come from
# instrumented code: the run then leaves the records unfilled)
COMPILERS = {"address": "g++", "memory": "/opt/rocm/lib/llvm/bin/clang++"}
FLAGS = {"address": ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
         "memory": ["-std=c++17", "-O1", "-g", "-fsanitize=memory",
                    "-fsanitize-memory-track-origins=2", "-fno-omit-frame-pointer"]}


def _key(nc: int, san: str) -> str:
    h = hashlib.sha256(" ".join(FLAGS[san]).encode())
    for p in SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return f"{san}_{h.hexdigest()[:12]}_nc{nc}"


def build(nc: int, san: str = "address") -> str:
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, f"driver_{_key(nc, san)}")
    if os.path.exists(exe):
        return exe
    cmd = [COMPILERS[san], *FLAGS[san], "-I", os.path.join(HERE, "stub"),
           "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-DPTF_MAX_NC=20", f"-DHOST_NC={nc}", os.path.join(HERE, "driver.cpp"),
           "-o", exe + ".tmp", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(exe + ".tmp", exe)
    return exe


def run(w, opts: dict, threads: int = 4, san: str = "address") -> dict:
    """Flashes workload w (workloads.Workload) with the host build; opts are
    the library's default options (ptflash_options fields)."""
    exe = build(w.nc, san)
    n, nc = w.n, w.nc
    oi = np.array([opts["max_pre_ss"], opts["max_ss"], opts["max_tr_sa"], opts["max_tr_split"],
                   opts["max_polish"], opts["dem_every"], 0, 0], np.int32)
    od = np.array([opts["tol_sa_ss"], opts["tol_sa_tr"], opts["tol_split_ss"],
                   opts["tol_split_tr"], opts["tol_polish"], opts["eps_tm"]], np.float64)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            f.write(np.array([n], np.int64).tobytes())
            f.write(np.array([nc, int(w.per_mixture)], np.int32).tobytes())
            f.write(oi.tobytes())
            f.write(od.tobytes())
            for a in (w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij):
                f.write(np.ascontiguousarray(a, np.float64).tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        args = [exe, fin, fout, str(threads)] if san == "address" else [exe, fin, fout, "1", "nofill"]
        r = subprocess.run(args, capture_output=True, text=True, env=env)
        if r.returncode != 0:
            raise RuntimeError(f"host build of the items failed (rc {r.returncode}):\n"
                               f"{r.stderr[-4000:]}")
        raw = open(fout, "rb").read()
    off = 0
    out = {}
    for name, dt, cnt in (("label", np.int8, n), ("beta", np.float64, n),
                          ("x", np.float64, n * nc), ("y", np.float64, n * nc),
                          ("iters", np.int16, n * 8), ("status", np.uint16, n),
                          ("flops", np.uint32, n), ("tm", np.float64, n)):
        b = np.dtype(dt).itemsize * cnt
        out[name] = np.frombuffer(raw[off:off + b], dtype=dt).copy()
        off += b
    out["x"] = out["x"].reshape(n, nc)
    out["y"] = out["y"].reshape(n, nc)
    out["iters"] = out["iters"].reshape(n, 8)
    return out
