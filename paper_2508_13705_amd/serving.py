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
  4. each lane's captured graph (``graph_steps`` batch steps) is launched
     on the lane's own stream; a lane whose graph has finished (an event
     query, no wait) has its progress records polled, its finished jobs read
     back, retired and their memory and slot released, so waiting jobs can be
     admitted at once, and is launched again.
Jobs are split into lanes by grid side (``lane_sides``): every job of a
batch advances one step per batch step, so a small job batched with a large
one would move at the large job's step rate.  Lanes run concurrently on the
device, each at its own rate.
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


class _Lane:
    """Jobs of one size class: a batch on its own stream and its graph."""

    def __init__(self, loop, max_side):
        torch = loop.torch
        self.max_side = max_side
        self.stream = torch.cuda.Stream()
        self.batch = cgks.Batch(loop.dim, loop.precision, max_jobs=loop.max_jobs, hbm_budget=loop.budget,
                                stream=self.stream)
        self.done_event = torch.cuda.Event()
        self.running = {}       # slot -> record
        self.changed = False    # jobs added or removed since the last commit
        self.captured = False
        self.tuned = not loop.tune
        self.inflight = False


class ServingLoop:
    def __init__(self, dim=2, precision="fp32_flux", hbm_budget=64 << 30, max_jobs=64, graph_steps=4,
                 prep_workers=4, tune=True, keep_results=False, build=None, lane_sides=(512, 1024)):
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
        # lane k takes sides up to lane_sides[k]; the last lane the rest
        self.lanes = [_Lane(self, m) for m in sorted(lane_sides)] + [_Lane(self, None)]
        self.pool = ThreadPoolExecutor(prep_workers)
        self._tls = threading.local()

    def _lane(self, job):
        for lane in self.lanes:
            if lane.max_side is None or job["n"] <= lane.max_side:
                return lane
        return self.lanes[-1]

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
        """Serve ``trace`` (dicts with "id", "arrival" [s], "nsteps", "n" and
        what ``build`` needs).  Returns a report with per-job records."""
        queue = collections.deque()
        arrivals = collections.deque(sorted(trace, key=lambda j: j["arrival"]))
        preparing = {}      # job id -> (future, job, bytes, admission time)
        done, rejected = [], []
        blocked = set()
        reserved = 0
        free_slots = self.max_jobs
        busy = 0.0
        steps_launched = 0
        max_running = 0
        t_start = time.perf_counter()
        now = lambda: time.perf_counter() - t_start
        t_mark = now()

        while arrivals or queue or preparing or any(l.running for l in self.lanes):
            t = now()
            if any(l.inflight for l in self.lanes):
                busy += t - t_mark
            t_mark = t
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
            # prepared jobs join their lane's batch (committed once the lane is idle)
            for jid in [k for k, v in preparing.items() if v[0].done()]:
                fut, job, nbytes, t_adm = preparing.pop(jid)
                solver, cells, t_prep = fut.result()
                lane = self._lane(job)
                slot = lane.batch.add(solver, max_steps=job["nsteps"])
                lane.running[slot] = {"id": job["id"], "job": job, "solver": solver, "bytes": nbytes,
                                      "arrival": job["arrival"], "admitted": t_adm, "started": now(),
                                      "prep_s": t_prep, "cells": cells, "order": job["order"]}
                lane.changed = True
            max_running = max(max_running, sum(len(l.running) for l in self.lanes))
            progressed = False
            for lane in self.lanes:
                # a lane whose graph finished: progress records, retirements
                if lane.inflight and lane.done_event.query():
                    lane.inflight = False
                    progressed = True
                    st = lane.batch.poll()
                    for s in [s for s, r in lane.running.items() if st[s]["status"] != 0]:
                        r = lane.running.pop(s)
                        r["completed"] = now()
                        r["waited_for_memory"] = r["id"] in blocked
                        r["status"] = st[s]["status"]
                        r["steps"] = st[s]["steps"]
                        r["t"] = st[s]["t"]
                        if self.keep_results:
                            r["result"] = r["solver"].read()
                        lane.batch.remove(s)
                        reserved -= r["bytes"]
                        free_slots += 1
                        del r["solver"]
                        done.append(r)
                        lane.changed = True
                        if log:
                            log(f"t={now():.2f}s done={len(done)} "
                                f"running={sum(len(l.running) for l in self.lanes)} queue={len(queue)}")
                if lane.inflight:
                    continue
                # an idle lane: commit its changes, then launch it
                if lane.changed:
                    lane.batch.commit()
                    lane.changed = False
                    if lane.running and not lane.tuned:
                        lane.batch.tune(1)          # real steps under each candidate launch shape
                        lane.tuned = True
                        lane.captured = False
                if lane.running:
                    if not lane.captured:
                        lane.batch.capture(self.graph_steps)
                        lane.captured = True
                    lane.batch.launch()
                    lane.done_event.record(lane.stream)
                    lane.inflight = True
                    steps_launched += self.graph_steps
                    progressed = True
            if not progressed:
                if any(l.inflight for l in self.lanes) or preparing:
                    time.sleep(0.0002)
                elif arrivals and not queue:
                    time.sleep(max(0.0, min(0.05, arrivals[0]["arrival"] - now())))
        wall = now()
        self.pool.shutdown(wait=True)
        rep = self._report(done, rejected, wall, busy, steps_launched)
        rep["max_running"] = max_running
        rep["lanes"] = [l.max_side for l in self.lanes]
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
