"""Throughput of the ASE-DFF compact GKS hot path on one MI355X.

Workload: 2-D compressible Navier-Stokes turbulence on a periodic 2048^2 grid,
9th order (4 Gauss points per face), viscous collision time, CFL 0.2; seeded
solenoidal random-phase velocity with a k^-5/3 shell spectrum (1 <= |k| <= 32),
Mach 0.3, uniform density and pressure.  A step is one full two-stage step of
every cell (reconstruction, interface flux, update of cell averages and
slopes).  The headline value is the FP32-flux variant (reconstruction and flux
moments in FP32, FP64 accumulation); the FP64 path is timed beside it.

Beside the headline, the same run measures (a) the batched path on the
4096-problem 1-D Riemann batch (200-4000 cells each, 9th order, CFL 0.5),
one persistent launch per phase for the whole batch in a captured hipGraph,
against the same jobs stepped one at a time by the single-grid path, (a')
one 1024^2 order-9 job stepped alone and as the only job of a batch (the
batched kernels' cost over the single-grid ones, with the autotuned tile
shapes), (b) the serving loop on a Poisson trace of 2-D jobs (side 128-2048, orders
5/7/9, smooth or four-quadrant data, 50-500 steps) under an HBM budget:
p50/p99 latency and throughput, (c) the wall and inflow workloads at the
paper's meshes to their end times, and (d) one GPU's share of the 2048^2 grid
cut into 8 slabs (2048 x 256, the shape a multi-GPU run would give each GPU).

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 2048] [--cpu-seconds 20]
                    [--batch-steps 40] [--batch2d-n 1024] [--serve-jobs 200] [--boundaries 1]
                    [--shard-parts 8]
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_alu": 78.6, "fp32_alu": 157.3, "hbm": 8000.0}  # TFLOP/s, TFLOP/s, GB/s (MI355X)
# Algorithmic FLOPs of the 2-D path per face Gauss point: the gas-kinetic flux
# (~2.5k) and the reconstruction and tangential derivatives that feed it
# (~0.6k).  One face launch (one direction, one stage) handles m Gauss points
# per cell, so 3.1k * m FLOP per cell and launch (12.4k at order 9).
ALGO_FLOP_PER_GP = 3100
# Algorithmic HBM bytes per cell-update (one cell through a whole two-stage
# step) of a design where each stage reads and writes the state once, stage 1
# writes an accumulator that stage 2 reads, and the strengths are read and
# written per face: 6 S + 6 words with S = 4 + 8 m state words per cell
# (1776 B at order 9 in FP64).  The FP32-flux variant stores the slopes
# (state, stage state, accumulator) in FP32 and keeps the averages and the
# strengths in FP64: S = 4 x 8 + 32 x 4 = 160 B, 6 S + 6 x 8 = 1008 B.
# 1-D: 6 S + 3 words with S = 6 words (312 B FP64; FP32 slopes 3 x 8 + 3 x 4
# = 36 B, 6 S + 3 x 8 = 240 B).
ALGO_BYTES_2D = {"fp64": 1776, "fp32_flux": 1008}
# Algorithmic FLOPs of the 1-D path per cell-update: per cell and stage one
# reconstruction of both faces (3 components) and one flux, 1630 FLOP by
# source count (paper_2508_13705_amd/csrc/flop_count.cpp), two stages.
ALGO_FLOP_1D = 2 * 1630
ALGO_BYTES_1D = {"fp64": 312, "fp32_flux": 240}
# Compulsory HBM bytes of one face launch of this design per cell (m = 4):
# stage input (avg 4 + normal slopes 16 + line values 16), partial averages
# and accumulator (4 + 4 + 4 + 4), normal slopes of the stage state and
# accumulator (16 + 16): 84 words, 672 B in FP64; with the slopes and line
# values in FP32, 20 FP64 + 64 FP32 words = 416 B.
FACE_BYTES_PER_CELL = {"fp64": 84 * 8, "fp32_flux": 20 * 8 + 64 * 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed steps of the FP64 path (default: --steps)")
    ap.add_argument("--batch-jobs", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=40, help="timed batch steps of the 1-D batch (0: skip)")
    ap.add_argument("--batch2d-n", type=int, default=1024,
                    help="side of the 2-D job timed alone and batched (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=200, help="jobs in the serving trace (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="offered load of the serving trace")
    ap.add_argument("--serve-ref-jobs", type=int, default=48,
                    help="seeded sample of the trace's jobs run alone on the single-grid FP64 path")
    ap.add_argument("--boundaries", type=int, default=1, help="run the wall/inflow workloads to their end times (0: skip)")
    ap.add_argument("--shard-parts", type=int, default=8,
                    help="also time one GPU's slab of the grid split this many ways (0: skip)")
    ap.add_argument("--probe-batch-jobs", type=int, default=1024,
                    help="jobs of the 1-D Riemann batch that --pmc-probe steps (0: none)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for hardware-counter runs: one step of each path, then a device copy of "
                         "COPY_BYTES (the calibration of the byte counters); prints nothing else")
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the kernel sources with their comments and blank lines taken
    out: a change to the code changes it, a change to a comment does not."""
    h = hashlib.sha256()
    for f in ("cgks.hip", "cgks_batch.hip", "cgks_batch.hpp", "cgks_batch_f32.hip", "cgks_internal.hpp", "cgks_device.hpp",
              "cgks_tables.inc"):
        with open(os.path.join(ROOT, "paper_2508_13705_amd", "csrc", f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _profile_entry(field, kernel):
    """A per-launch figure from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "face_kernel_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get(field, {}).get(kernel)


def profile_1d(precision):
    """Counted bytes and FLOPs per cell-stage of the batched 1-D stage kernels
    (mean of the two stages), if the profile matches the current sources."""
    return _profile_entry("batch_1d_per_cell_stage", precision)


def measured_traffic(kernel):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return _profile_entry("bytes_per_launch", kernel)


def counted_flops(kernel):
    """Hardware-counted VALU FLOPs per launch (F32 + F64 add, mul, 2 x fma, trans)."""
    return _profile_entry("valu_flops_per_launch", kernel)


def host_cpu():
    """The host CPU model and the cores the oracle may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"model": model, "nproc": affinity, "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


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


def bench_batch_1d(jobs, steps, precision, graph_steps=10):
    """Batched 1-D Riemann problems: cell-updates/s of the captured batch
    step, and of the same jobs stepped one by one on the single-grid path."""
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    probs = W.riemann_batch(seed=2, count=jobs)
    stream = torch.cuda.Stream()
    B = cgks.Batch(1, precision, max_jobs=jobs, stream=stream)
    sol = [cgks.Solver(pb, precision=precision, stream=stream) for pb in probs]
    cells = {}
    for pb, s in zip(probs, sol):
        cells[B.add(s, max_steps=0, t_end=pb["run"]["t_end"])] = pb["grid"]["nx"]
    B.commit()
    tuning = B.tune(1)
    B.capture(graph_steps)
    B.launch()        # the first replays upload the graph
    B.launch()
    st0 = B.poll()
    reps = max(1, steps // graph_steps)
    # timed: the replays until the stream drains; the progress records are
    # read afterwards (building the per-job dicts can meet a Python GC pause)
    t0 = time.perf_counter()
    for _ in range(reps):
        B.launch()
    stream.synchronize()
    el = time.perf_counter() - t0
    st1 = B.poll()
    upd = sum(cells[k] * (st1[k]["steps"] - st0[k]["steps"]) for k in cells)
    active = sum(1 for k in cells if st1[k]["status"] == 0)
    nonphys = sum(1 for k in cells if st1[k]["status"] == 2)
    # the same jobs one at a time, single-grid path (a sample, same step count)
    sample = sol[: min(256, len(sol))]
    with torch.cuda.stream(stream):
        for s in sample:
            s.step(2, t_end=0.15)
        h0 = [s.health()["steps"] for s in sample]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in sample:
            s.step(graph_steps, t_end=0.15)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t0
        h1 = [s.health()["steps"] for s in sample]
    upd1 = sum(s.plan.gd.nx * (b - a) for s, a, b in zip(sample, h0, h1))
    roof = roofline_1d(precision, upd / el)
    return {"workload": f"{jobs} 1-D Riemann problems, 200-4000 cells, order 9, CFL 0.5, t_end 0.15, seed 2",
            "precision": precision, "value": upd / el, "unit": "cell-updates/s", "roofline": roof,
            "batch_steps": reps * graph_steps,
            "ms_per_batch_step": 1e3 * el / (reps * graph_steps), "jobs_active": active, "jobs_nonphysical": nonphys,
            "tuning": tuning,
            "single_grid_sequential": {"value": upd1 / el1 if el1 > 0 else None, "jobs": len(sample),
                                       "steps_each": graph_steps},
            "speedup_vs_single_grid": (upd / el) / (upd1 / el1) if upd1 > 0 else None}


def roofline_1d(precision, rate):
    """Roofline of the batched 1-D step at `rate` cell-updates/s: the HBM roof
    (algorithmic bytes per cell-update) and the VALU roof (the source count of
    the FLOPs per cell-update), t_roof = max of the two; frac = t_roof / t."""
    t = 1.0 / rate
    b = ALGO_BYTES_1D[precision]
    f = ALGO_FLOP_1D
    t_hbm = b / (PEAK["hbm"] * 1e9)
    peak_alu = PEAK["fp64_alu"]          # FP64, and FP32 without packed instructions
    t_alu = f / (peak_alu * 1e12)
    alu = t_alu >= t_hbm
    out = {"bound": "alu" if alu else "hbm",
           "achieved": f * rate / 1e12 if alu else b * rate / 1e9,
           "peak": peak_alu if alu else PEAK["hbm"], "unit": "TFLOP/s" if alu else "GB/s",
           "frac": (t_alu if alu else t_hbm) / t,
           "algorithmic_bytes_per_cell_update": b, "algorithmic_flops_per_cell_update": f,
           "hbm_frac": t_hbm / t, "alu_frac": t_alu / t, "scope": "whole batch step",
           "traffic": None}
    c = profile_1d(precision)
    if c:
        out["counted"] = c
        if c.get("bytes_per_cell_stage"):
            out["traffic"] = 2 * c["bytes_per_cell_stage"]   # bytes per cell-update, measured
    return out


def bench_batch_2d(n, steps, precision, order=9):
    """One 2-D job (turbulence n x n, order 9) stepped alone on the
    single-grid path and as the only job of a batch (persistent kernels,
    captured graph, autotuned launch and tile shapes): ms per step of each."""
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    pb = W.turbulence_2d(seed=4, n=n, order=order, nsteps=steps, prandtl=1.0, quad=4)
    s = cgks.Solver(pb, precision=precision)
    s.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    single = 1e3 * (time.perf_counter() - t0) / steps
    del s
    stream = torch.cuda.Stream()
    B = cgks.Batch(2, precision, max_jobs=1, stream=stream)
    q = cgks.Solver(pb, precision=precision, stream=stream)
    B.add(q, max_steps=10 ** 6)
    B.commit()
    tuning = B.tune(3)
    gs = 5
    B.capture(gs)
    B.launch()
    stream.synchronize()
    reps = max(1, steps // gs)
    t0 = time.perf_counter()
    for _ in range(reps):
        B.launch()
    stream.synchronize()
    batched = 1e3 * (time.perf_counter() - t0) / (reps * gs)
    del B, q
    torch.cuda.empty_cache()
    return {"workload": f"turbulence {n}x{n}, order {order}, Pr 1, one job", "precision": precision,
            "single_grid_ms_per_step": single, "batched_ms_per_step": batched, "batched_over_single": batched / single,
            "tuning": tuning}


def bench_shard(problem, parts, steps, warmup, full):
    """One GPU's share of the 2-D grid split into `parts` slabs along y, at its
    real shape (n x n/parts cells, periodic in x).  The y ghosts come from the
    transmissive fill, the stand-in for the halo exchange that a multi-GPU
    run would do before each stage; the exchange and the all-reduce of the
    time step are not run.  Reports the slab's step time and its time per
    cell against the whole grid's."""
    n = problem["grid"]["nx"]
    ny = n // parts
    g = dict(problem["grid"], ny=ny, y1=problem["grid"]["y0"] + (problem["grid"]["y1"] - problem["grid"]["y0"]) * ny / n,
             bc=["periodic", "periodic", "transmissive", "transmissive"])
    st = problem["state"]
    pb = dict(problem, name=f"{problem['name']}_slab{ny}", grid=g,
              state={"avg": st["avg"][:, :ny].copy(), "sx": st["sx"][:, :, :ny].copy(), "sy": st["sy"][:, :, :ny].copy()})
    out = {"workload": f"{n}x{ny} slab (1/{parts} of the {n}x{n} grid), periodic in x, transmissive y ghosts "
                       f"standing in for the halo exchange", "parts": parts}
    for precision in ("fp32_flux", "fp64"):
        el, per, h, stt = time_path(pb, precision, steps, warmup)
        ms = 1e3 * el / steps
        out[precision] = {"ms_per_step": ms, "cell_updates_per_s": n * ny * steps / el,
                          "time_per_cell_vs_full_grid": (ms / (n * ny)) / (full[precision] / (n * n)),
                          "status": stt["status"]}
    return out


def serving_reference(trace, precision="fp64"):
    """The serving trace's jobs one at a time on the plain single-grid path:
    each job's initial data is built and uploaded first, then its steps are
    timed (HIP synchronised).  Returns the throughput of running them back to
    back and the per-job device times."""
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    secs, work = [], 0.0
    for job in trace:
        s = cgks.Solver(W.serving_problem(job), precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(job["nsteps"])
        st = s.read(sync_only=True)
        secs.append(time.perf_counter() - t0)
        work += job["n"] * job["n"] * st["steps"]
        del s
        torch.cuda.empty_cache()
    secs = np.array(secs)
    return {"precision": precision, "path": "single-grid, one job at a time", "jobs": len(trace),
            "cell_updates_per_s": work / secs.sum(), "job_seconds_p50": float(np.percentile(secs, 50)),
            "job_seconds_p99": float(np.percentile(secs, 99))}


def bench_serving(jobs, load, ref_rate, precision="fp32_flux", ref_jobs=48):
    """Serving loop on a Poisson trace of 2-D jobs; arrival rate set for an
    offered load `load` of the measured single-grid rate `ref_rate`."""
    from paper_2508_13705_amd import serving
    from paper_2508_13705_amd import workloads as W
    probe = W.serving_trace(seed=5, count=jobs, rate=1.0)
    work = sum(j["n"] * j["n"] * j["nsteps"] for j in probe) / jobs
    rate = load * ref_rate / work
    trace = W.serving_trace(seed=5, count=jobs, rate=rate)
    loop = serving.ServingLoop(2, precision, hbm_budget=64 << 30, max_jobs=32, graph_steps=4, prep_workers=4)
    rep = loop.run(trace, log=lambda m: print("[serve]", m, file=sys.stderr, flush=True))
    rep.pop("records")
    # the plain single-grid FP64 path on a seeded sample of the same jobs, one at a time
    pick = np.random.default_rng(55).choice(len(trace), size=min(ref_jobs, len(trace)), replace=False)
    ref = serving_reference([trace[k] for k in sorted(pick)], "fp64")
    rep["single_grid_fp64"] = ref
    # over the wall time the served throughput is the arrival rate; per busy
    # second it is the rate the loop sustains
    rep["throughput_vs_single_grid_fp64"] = rep["throughput_cell_updates_per_s"] / ref["cell_updates_per_s"]
    busy = rep["device_busy_frac"]
    rep["busy_throughput_vs_single_grid_fp64"] = (rep["throughput_cell_updates_per_s"] / busy / ref["cell_updates_per_s"]
                                                  if busy > 0 else None)
    rep.update({"workload": f"{jobs} 2-D jobs, Poisson arrivals {rate:.3f}/s, side 2^U[7,11], order 5/7/9, "
                            f"smooth or four-quadrant data, 50-500 steps, seed 5, budget 64 GiB",
                "precision": precision, "offered_load": load, "mean_job_cell_updates": work})
    return rep


def bench_small_1d():
    """The 1-D Fourier wave (256 cells, order 5, CFL 0.5, 100 steps, FP64):
    too small to fill the device, so its wall time is launch latency.
    Inputs resident; the timed region is the 100 steps (HIP synchronised)."""
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    pb = W.fourier_1d()
    s = cgks.Solver(pb, precision="fp64")
    s.step(5)
    torch.cuda.synchronize()
    s = cgks.Solver(pb, precision="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(100)
    st = s.read(sync_only=True)
    el = time.perf_counter() - t0
    return {"workload": "1-D Fourier wave, 256 cells on periodic [0,2], order 5, CFL 0.5, 100 steps, FP64, seed 1",
            "wall_ms": 1e3 * el, "us_per_step": 1e4 * el, "launches_per_step": 6, "status": st["status"],
            "steps": st["steps"]}


def bench_boundaries():
    """The paper's wall and inflow workloads at its meshes, run to their end
    times on the single-grid path (FP64): double Mach reflection 960 x 240 to
    t = 0.2 (Sec. 4.8) and the viscous shock tube 500 x 250, Re = 200, to
    t = 1.0 (Sec. 4.9), order 5 (at order 7 the no-slip ghosts make this tube
    go nonphysical near the diaphragm within 21 steps, in the oracle as in
    this library).  Inputs resident in HBM; the timed region is the stepping
    loop (HIP synchronised)."""
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    out = {}
    for key, pb in (("double_mach_960x240_o5", W.double_mach(240, order=5, t_end=0.2)),
                    ("viscous_shock_tube_500x250_o5", W.viscous_shock_tube(500, order=5, t_end=1.0))):
        s = cgks.Solver(pb, precision="fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chunk = 200
        for _ in range(200):        # at most 40,000 steps
            s.step(chunk, t_end=pb["run"]["t_end"])
            st = s.read(sync_only=True)
            if st["status"] != 0 or st["t"] >= pb["run"]["t_end"]:
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g = pb["grid"]
        cells = g["nx"] * g["ny"]
        h = s.health()
        out[key] = {"t": st["t"], "steps": st["steps"], "status": st["status"], "seconds": el,
                    "cell_updates_per_s": cells * st["steps"] / el, "fallbacks": h.get("fallbacks"),
                    "nonphysical": h.get("nonphysical")}
        print("[boundaries]", key, out[key], file=sys.stderr, flush=True)
    return out


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
    cpu = host_cpu()
    threads = int(cpu["omp_num_threads"] or cpu["nproc"] or 1)
    return {"value": n * n * k / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"turbulence {n}x{n} periodic, order 9, viscous, {k} steps ({el:.1f} s), "
                      f"status {r['status']}", "host": cpu}


COPY_BYTES = 1 << 30


def pmc_probe(n, batch_jobs):
    import torch
    from paper_2508_13705_amd import cgks
    from paper_2508_13705_amd import workloads as W
    problem = W.turbulence_2d(seed=4, n=n, order=9, nsteps=1, prandtl=0.72, quad=4)
    for precision in ("fp32_flux", "fp64"):
        s = cgks.Solver(problem, precision=precision)
        s.step(1)
        torch.cuda.synchronize()
        del s
        torch.cuda.empty_cache()
    # the batched 1-D stage kernels: a seeded subset of the 1-D Riemann batch,
    # two batch steps per precision (the second is the one to read)
    if batch_jobs > 0:
        probs = W.riemann_batch(seed=2, count=batch_jobs)
        for precision in ("fp64", "fp32_flux"):
            B = cgks.Batch(1, precision, max_jobs=batch_jobs)
            sol = [cgks.Solver(pb, precision=precision) for pb in probs]
            for pb, q in zip(probs, sol):
                B.add(q, max_steps=0, t_end=pb["run"]["t_end"])
            B.commit()
            B.step(2)
            torch.cuda.synchronize()
            del B, sol
            torch.cuda.empty_cache()
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": True, "copy_bytes": COPY_BYTES, "n": n, "batch_jobs": batch_jobs}))


def main():
    a = parse()
    if a.pmc_probe:
        pmc_probe(a.n, a.probe_batch_jobs)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: the library has no multi-GPU path; run with --gpus 1"}))
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
        step_s = r["elapsed"] / r["steps"]
        # whole step against the HBM roof: algorithmic bytes per cell-update
        hbm_step = {"algorithmic_bytes_per_cell_update": ALGO_BYTES_2D[prec],
                    "achieved_GBps": cells * ALGO_BYTES_2D[prec] / step_s / 1e9,
                    "frac": cells * ALGO_BYTES_2D[prec] / step_s / 1e9 / PEAK["hbm"]}
        if "face" not in dom:
            return {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK["hbm"], "unit": "GB/s",
                    "frac": None, "traffic": None, "avg_ms": ms, "hbm_step": hbm_step}
        m = 4
        flops = ALGO_FLOP_PER_GP * m * cells
        peak = PEAK["fp32_alu"] if prec == "fp32_flux" else PEAK["fp64_alu"]
        ach = flops / (ms * 1e-3) / 1e12
        key = dom.split("_", 1)[1] + "_" + prec
        traffic = measured_traffic(key)
        counted = counted_flops(key)
        out = {"bound": "alu", "kernel": dom, "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
               "algorithmic_flops": flops, "flops_basis": f"{ALGO_FLOP_PER_GP} per face Gauss point x m=4 x cells",
               "avg_ms": ms, "traffic": traffic,
               # the FP32 peak counts packed FP32 instructions, which this
               # library does not emit; unpacked, FP32 issues at the FP64 rate
               "peak_unpacked": PEAK["fp64_alu"], "frac_unpacked": ach / PEAK["fp64_alu"],
               "hbm_launch": {"algorithmic_bytes": FACE_BYTES_PER_CELL[prec] * cells,
                              "frac_algorithmic": FACE_BYTES_PER_CELL[prec] * cells / (ms * 1e-3) / 1e9 / PEAK["hbm"],
                              "frac_measured": (traffic / (ms * 1e-3) / 1e9 / PEAK["hbm"]) if traffic else None},
               "hbm_step": hbm_step}
        if counted:
            out["counted_flops"] = counted
            out["counted_TFLOPs"] = counted / (ms * 1e-3) / 1e12
            out["frac_counted_unpacked"] = out["counted_TFLOPs"] / PEAK["fp64_alu"]
        return out

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
        "dtype": "f32+f64",
        "dtype_detail": "f32 reconstruction and flux moments, f64 accumulation and time coefficients",
        "data": "synthetic",
        "config": {"workload": f"2-D Navier-Stokes turbulence {n}x{n} periodic, order 9 (m=4), viscous tau "
                               f"mu=1e-4, Pr=0.72, Mach 0.3, k^-5/3 spectrum 1<=|k|<=32, CFL 0.2, seed 4",
                   "cells": cells, "order": 9},
        "roofline": roof("fp32_flux"),
        "fp64": {"value": cells * q["steps"] / q["elapsed"], "ms_per_step": 1e3 * q["elapsed"] / q["steps"],
                 "steps": q["steps"], "roofline": roof("fp64")},
        "kernel_ms": {"fp32_flux": p["avg_ms"], "fp64": q["avg_ms"]},
        "health": {"fp32_flux": p["health"], "fp64": q["health"]},
    }
    def section(name, fn):
        # a failure in a secondary measurement is recorded, not fatal: the
        # headline line above is printed regardless
        try:
            out[name] = fn()
        except Exception as e:          # noqa: BLE001
            print(f"[bench] {name} failed: {e!r}", file=sys.stderr, flush=True)
            out[name] = {"error": repr(e)}

    if a.shard_parts > 1:
        full = {k: 1e3 * res[k]["elapsed"] / res[k]["steps"] for k in res}
        section("shard", lambda: bench_shard(problem, a.shard_parts, 10, 2, full))

    def batch_1d():
        r = {prec: bench_batch_1d(a.batch_jobs, a.batch_steps, prec) for prec in ("fp64", "fp32_flux")}
        ref64 = r["fp64"]["single_grid_sequential"]["value"]
        for v in r.values():
            v["speedup_vs_single_grid_fp64"] = v["value"] / ref64 if ref64 else None
        return r

    if a.batch_steps > 0:
        section("batch_1d", batch_1d)
    if a.batch2d_n > 0:
        section("batch_2d", lambda: {p: bench_batch_2d(a.batch2d_n, 10, p) for p in ("fp32_flux", "fp64")})
    if a.serve_jobs > 0:
        section("serving", lambda: bench_serving(a.serve_jobs, a.serve_load, value, ref_jobs=a.serve_ref_jobs))
    if a.boundaries:
        section("boundaries", bench_boundaries)
    section("small_1d", bench_small_1d)
    section("cpu_baseline", lambda: cpu_baseline(a.cpu_seconds))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
