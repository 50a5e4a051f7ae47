"""Throughput of the ASE-DFF compact GKS hot path on one MI355X.

Workload: 2-D compressible Navier-Stokes turbulence on a periodic 2048^2 grid,
9th order (4 Gauss points per face), viscous collision time, CFL 0.5; seeded
solenoidal random-phase velocity with a k^-5/3 shell spectrum (1 <= |k| <= 32),
Mach 0.3, uniform density and pressure.  A step is one full two-stage step of
every cell (reconstruction, interface flux, update of cell averages and
slopes).  The headline value is the FP32-flux variant (reconstruction and flux
moments in FP32, FP64 accumulation); the FP64 path is timed beside it.

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 2048] [--cpu-seconds 20]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_alu": 78.6, "fp32_alu": 157.3, "hbm": 8000.0}  # TFLOP/s, TFLOP/s, GB/s (MI355X)
# Algorithmic FLOPs of one face-kernel launch per cell of the grid (one direction,
# one stage, 9th order, m = 4, Prandtl fix on): Step-2 share 1728 + Step 3 2304 +
# four fluxes 29932 + update 144 (paper_2508_13705_amd/csrc/flop_count.cpp).
FACE_FLOP_PER_CELL = 34108
# Compulsory HBM bytes of one face-kernel launch per cell (FP64 state words,
# m = 4): read the stage input (avg 4 + normal slopes 16 + line values 16),
# read/write the partial averages and accumulator (4 + 4 + 4 + 4) and write the
# normal slopes of the stage state and accumulator (16 + 16): 84 words.
FACE_BYTES_PER_CELL = 84 * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed steps of the FP64 path (default: --steps)")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("cgks.hip", "cgks_device.hpp", "cgks_tables.inc"):
        with open(os.path.join(ROOT, "paper_2508_13705_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "face_kernel_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


def time_path(problem, precision, steps, warmup):
    import torch
    from paper_2508_13705_amd import cgks
    s = cgks.Solver(problem, precision=precision)
    for _ in range(warmup):
        s.step(1)
    torch.cuda.synchronize()
    per = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        for k, (name, ms) in enumerate(s.step_timed()):
            per.setdefault(f"{k:02d}_{name}", []).append(ms)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h = s.health()
    st = s.read(sync_only=True)
    del s
    torch.cuda.empty_cache()
    return el, per, h, st


def cpu_baseline(seconds):
    """The plain FP64 oracle on a bounded sample of the same workload (a
    smaller periodic grid with the same order, viscosity model, spectrum
    shape), timed on this host's cores."""
    if seconds <= 0:
        return None
    import oracle
    from paper_2508_13705_amd import workloads as W
    n = 48
    pb = W.turbulence_2d(seed=4, n=n, order=9, nsteps=1, kmax=8, prandtl=0.72, mu=1e-4, quad=4)
    t0 = time.perf_counter()
    r = oracle.run(pb, nsteps=1)
    one = time.perf_counter() - t0
    k = max(1, int(seconds / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    r = oracle.run(pb, nsteps=k)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n * n * k / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"turbulence {n}x{n} periodic, order 9, viscous, {k} steps ({el:.1f} s), "
                      f"status {r['status']}"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2508_13705_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = a.n
    problem = W.turbulence_2d(seed=4, n=n, order=9, nsteps=a.steps, prandtl=0.72, quad=4)
    cells = n * n

    res = {}
    for precision, steps in (("fp32_flux", a.steps), ("fp64", a.fp64_steps or a.steps)):
        el, per, h, st = time_path(problem, precision, steps, a.warmup)
        avg = {k: sum(v) / len(v) for k, v in per.items()}
        dom = max(avg, key=lambda k: avg[k])
        res[precision] = {"elapsed": el, "steps": steps, "avg_ms": avg, "dominant": dom, "health": h, "t": st["t"]}

    def roof(prec):
        r = res[prec]
        dom = r["dominant"]
        ms = r["avg_ms"][dom]
        if "face" in dom:
            flops = FACE_FLOP_PER_CELL * cells
            peak = PEAK["fp32_alu"] if prec == "fp32_flux" else PEAK["fp64_alu"]
            ach = flops / (ms * 1e-3) / 1e12
            return {"bound": "alu", "kernel": dom, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                    "frac": ach / peak, "traffic": measured_traffic(dom.split("_", 1)[1] + "_" + prec),
                    "avg_ms": ms, "algorithmic_bytes": FACE_BYTES_PER_CELL * cells,
                    "hbm_frac_algorithmic": FACE_BYTES_PER_CELL * cells / (ms * 1e-3) / 1e9 / PEAK["hbm"]}
        return {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK["hbm"], "unit": "GB/s", "frac": None,
                "traffic": None, "avg_ms": ms}

    p = res["fp32_flux"]
    q = res["fp64"]
    value = cells * p["steps"] / p["elapsed"]
    out = {
        "metric": "cell-updates/s 2D 9th-order FP32-flux vs FP64 GPU; served p50/p99 latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": p["steps"],
        "warmup": a.warmup,
        "ms_per_step": 1e3 * p["elapsed"] / p["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 reconstruction/flux, f64 accumulation",
        "data": "synthetic",
        "config": {"workload": f"2-D Navier-Stokes turbulence {n}x{n} periodic, order 9 (m=4), viscous tau "
                               f"mu=1e-4, Pr=0.72, Mach 0.3, k^-5/3 spectrum 1<=|k|<=32, CFL 0.5, seed 4",
                   "cells": cells, "order": 9},
        "roofline": roof("fp32_flux"),
        "fp64": {"value": cells * q["steps"] / q["elapsed"], "ms_per_step": 1e3 * q["elapsed"] / q["steps"],
                 "steps": q["steps"], "roofline": roof("fp64")},
        "kernel_ms": {"fp32_flux": p["avg_ms"], "fp64": q["avg_ms"]},
        "health": {"fp32_flux": p["health"], "fp64": q["health"]},
    }
    out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
