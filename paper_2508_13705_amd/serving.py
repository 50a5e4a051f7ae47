"""Serving loop: simulation jobs arrive over time, are admitted against an HBM
budget, and are advanced together by the library's batched kernels
(continuous batching through a captured hipGraph step).

The loop (one thread) does, in order, until the trace is drained:
  1. arrivals whose time has come join a FIFO queue;
  2. admission: the queue head is admitted when a job slot is free and the
     bytes of its state and work buffers fit the budget, and is handed to a
     preparation worker (initial data on the host, device buffers, upload on
     the worker's own stream); the budget is reserved at admission;
  3. prepared jobs join the batch; the table is committed only when it changed;
  4. the captured graph (``graph_steps`` batch steps) is launched and the
     progress records polled; finished jobs are read back, retired and their
     memory and slot released, so waiting jobs can be admitted at once.
A job whose buffers exceed the whole budget is rejected.  Latency of a job =
completion time - arrival time (queueing, preparation and device time).

All device work of the scheme runs in libcgks (paper_2508_13705_amd.cgks);
this module is host logic only.
"""
import collections
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import cgks
from . import workloads as W


def job_bytes(job, precision, dim=2):
    """State + work bytes of a serving job (grid side n, order), from the
    plan alone: no initial data is built and nothing is allocated."""
    n = job["n"]
    desc = {"grid": {"dim": dim, "nx": n, "ny": n if dim == 2 else 1, "x0": 0.0, "x1": 1.0, "y0": 0.0, "y1": 1.0,
                     "bc": ["periodic"] * 4},
            "scheme": W.default_scheme(job["order"])}
    p = cgks.Plan(desc, precision)
    return p.state_bytes + p.work_bytes


class ServingLoop:
    def __init__(self, dim=2, precision="fp32_flux", hbm_budget=64 << 30, max_jobs=64, graph_steps=4,
                 prep_workers=4, tune=True, keep_results=False, build=None):
        import torch
        self.torch = torch
        self.dim = dim
        self.precision = precision
        self.budget = int(hbm_budget)
        self.max_jobs = max_jobs
        self.graph_steps = graph_steps
        self.tune = tune
        self.keep_results = keep_results
        self.build = build or W.serving_problem
        self.stream = torch.cuda.Stream()
        self.batch = cgks.Batch(dim, precision, max_jobs=max_jobs, hbm_budget=hbm_budget, stream=self.stream)
        self.pool = ThreadPoolExecutor(prep_workers)
        self._tls = threading.local()

    # -- preparation (worker threads) ---------------------------------------
    def _worker_stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self._tls.stream = self.torch.cuda.Stream()
        return s

    def _prepare(self, job):
        t0 = time.perf_counter()
        problem = self.build(job)
        st = self._worker_stream()
        solver = cgks.Solver(problem, precision=self.precision, stream=st)   # uploads and synchronises st
        g = problem["grid"]
        cells = g["nx"] * (g["ny"] if g["dim"] == 2 else 1)
        return solver, cells, time.perf_counter() - t0

    # -- the loop -------------------------------------------------------------
    def run(self, trace, log=None):
        """Serve ``trace`` (dicts with "id", "arrival" [s], "nsteps" and what
        ``build`` needs).  Returns a report with per-job records."""
        B = self.batch
        queue = collections.deque()
        arrivals = collections.deque(sorted(trace, key=lambda j: j["arrival"]))
        preparing = {}      # job id -> (future, job, bytes, admission time)
        running = {}        # slot -> record
        done, rejected = [], []
        blocked = set()
        reserved = 0
        free_slots = self.max_jobs
        captured = False
        tuned = not self.tune
        busy = 0.0
        steps_launched = 0
        max_running = 0
        t_start = time.perf_counter()
        now = lambda: time.perf_counter() - t_start

        while arrivals or queue or preparing or running:
            t = now()
            while arrivals and arrivals[0]["arrival"] <= t:
                queue.append(arrivals.popleft())
            # admission (FIFO)
            while queue and free_slots > 0:
                job = queue[0]
                nbytes = job_bytes(job, self.precision, self.dim)
                if nbytes > self.budget:
                    queue.popleft()
                    rejected.append({"id": job["id"], "bytes": nbytes})
                    continue
                if reserved + nbytes > self.budget:
                    blocked.add(job["id"])     # waits for memory
                    break
                queue.popleft()
                reserved += nbytes
                free_slots -= 1
                fut = self.pool.submit(self._prepare, job)
                preparing[job["id"]] = (fut, job, nbytes, now())
            # prepared jobs join the batch
            changed = False
            for jid in [k for k, v in preparing.items() if v[0].done()]:
                fut, job, nbytes, t_adm = preparing.pop(jid)
                solver, cells, t_prep = fut.result()
                slot = B.add(solver, max_steps=job["nsteps"])
                running[slot] = {"id": job["id"], "job": job, "solver": solver, "bytes": nbytes,
                                 "arrival": job["arrival"], "admitted": t_adm, "started": now(), "prep_s": t_prep,
                                 "cells": cells, "order": job["order"]}
                changed = True
            if changed:
                B.commit()
                if not tuned:
                    B.tune(1)           # real steps under each candidate launch shape
                    tuned = True
                    captured = False
                if not captured:
                    B.capture(self.graph_steps)
                    captured = True
            if not running:
                # idle: wait for a preparation or the next arrival
                if preparing:
                    time.sleep(0.001)
                elif arrivals and not queue:
                    time.sleep(max(0.0, min(0.05, arrivals[0]["arrival"] - now())))
                continue
            max_running = max(max_running, len(running))
            tb = time.perf_counter()
            B.launch()
            steps_launched += self.graph_steps
            st = B.poll()                # synchronises the batch stream
            busy += time.perf_counter() - tb
            finished = [s for s, r in running.items() if st[s]["status"] != 0]
            if finished:
                for s in finished:
                    r = running.pop(s)
                    r["completed"] = now()
                    r["waited_for_memory"] = r["id"] in blocked
                    r["status"] = st[s]["status"]
                    r["steps"] = st[s]["steps"]
                    r["t"] = st[s]["t"]
                    if self.keep_results:
                        r["result"] = r["solver"].read()
                    B.remove(s)
                    reserved -= r["bytes"]
                    free_slots += 1
                    del r["solver"]
                    done.append(r)
                B.commit()
                if log:
                    log(f"t={now():.2f}s done={len(done)} running={len(running)} queue={len(queue)}")
        wall = now()
        self.pool.shutdown(wait=True)
        rep = self._report(done, rejected, wall, busy, steps_launched)
        rep["max_running"] = max_running
        return rep

    def _report(self, done, rejected, wall, busy, steps_launched):
        lat = np.array([r["completed"] - r["arrival"] for r in done]) if done else np.zeros(1)
        work = float(sum(r["cells"] * r["steps"] for r in done))
        return {
            "jobs": len(done), "rejected": len(rejected), "wall_s": wall,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()),
            "queue_p50_s": float(np.percentile([r["admitted"] - r["arrival"] for r in done], 50)) if done else 0.0,
            "prep_p50_s": float(np.percentile([r["prep_s"] for r in done], 50)) if done else 0.0,
            "cell_updates": work, "throughput_cell_updates_per_s": work / wall if wall > 0 else 0.0,
            "device_busy_frac": busy / wall if wall > 0 else 0.0, "batch_steps": steps_launched,
            "nonphysical": sum(1 for r in done if r["status"] == 2),
            "records": done,
        }
