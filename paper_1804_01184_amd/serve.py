"""Continuous-batching gradient server.

Requests (a model, its acquisition, its observed data) arrive over time.  A
request is admitted as soon as a slot (a HIP stream) is free and its HBM
footprint — the library's gradient workspace (wavefields, checkpoints,
segment store, partial gradients) plus its model, data and result arrays —
fits in the remaining budget.  Admitted requests run concurrently on their
own streams, so their kernels overlap on the device; requests that arrive
while others run are admitted as slots and memory free up.  Each result is
computed by the same deterministic kernels whatever else runs, so it is the
same alone and in the mix.

A request keeps its whole pressure history when that fits one slot's share
of the budget, else the plan checkpoints every ceil(sqrt(nt)) steps, so one
large request does not hold the memory the others need to run alongside.

Reports per-request latency (completion - arrival), p50/p99, and aggregate
Gcell-updates/s over the makespan.  ``python -m paper_1804_01184_amd.serve``
serves a seeded Poisson stream of mixed-size requests and prints one JSON
line.
"""
from __future__ import annotations

import json
import math
import sys
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .api import Grid, Plan


@dataclass
class Request:
    id: int
    arrival: float                 # seconds after the start of the run
    grid: Grid
    src_xz: np.ndarray
    rec_xz: np.ndarray
    param: str
    m1: np.ndarray
    m2: np.ndarray
    wavelet: np.ndarray
    observed: torch.Tensor         # host (pinned) or device, [S][nrec][nt]
    meta: dict = field(default_factory=dict)

    @property
    def cell_steps(self):
        Nz, Nx = self.grid.padded
        return Nz * Nx * self.grid.nt * self.src_xz.shape[0]


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    done: float
    J: float
    g1: torch.Tensor
    g2: torch.Tensor
    footprint: int
    cell_steps: int

    @property
    def latency(self):
        return self.done - self.arrival


class _Job:
    def __init__(self, req, plan, stream, footprint):
        self.req, self.plan, self.stream, self.footprint = req, plan, stream, footprint
        self.event = torch.cuda.Event()
        self.bufs = None
        self.admitted = None
        self.thread = None
        self.error = None

    def submitted(self):
        return self.thread is not None and not self.thread.is_alive()


def footprint(plan: Plan, req: Request):
    """Device bytes a request holds while it runs."""
    S, nrec, nt = req.observed.shape
    n = req.grid.nz * req.grid.nx
    arrays = 4 * (2 * n + 2 * n + 1 + S * nrec * nt + nt * (S if req.wavelet.ndim == 2 else 1))
    return plan.workspace_bytes(L.FWI_OP_GRADIENT) + arrays


class GradientServer:
    def __init__(self, max_slots=4, hbm_budget=None, device=None, plan_kw=None):
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        total = torch.cuda.get_device_properties(self.device).total_memory
        self.budget = int(hbm_budget if hbm_budget is not None else 0.7 * total)
        self.max_slots = max_slots
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_slots)]
        self.plan_kw = plan_kw or {}
        self.log = []

    def plan_for(self, q):
        """The request's plan: whole history if it fits a slot's share of
        the budget, else sqrt(nt) checkpoints (unless plan_kw fixes it).
        Plans hold host memory only, so making one (and dropping the
        whole-history one) never waits for the device."""
        plan = Plan(q.grid, q.src_xz, q.rec_xz, device=self.device, **self.plan_kw)
        if "ckpt_every" not in self.plan_kw and \
                footprint(plan, q) > self.budget / self.max_slots:
            k = int(math.ceil(math.sqrt(q.grid.nt)))
            plan = Plan(q.grid, q.src_xz, q.rec_xz, device=self.device, ckpt_every=k,
                        **self.plan_kw)
        return plan

    def _start(self, job, now):
        # a gradient enqueues thousands of launches and the enqueue blocks
        # once the device queue is full, so each job is submitted from a
        # thread of its own (the library calls release the GIL): the serving
        # loop keeps admitting and retiring meanwhile
        r = job.req
        dev = self.device

        def submit():
            try:
                torch.cuda.set_device(dev)
                with torch.cuda.stream(job.stream):
                    m1 = torch.as_tensor(r.m1, dtype=torch.float32).to(dev, non_blocking=True)
                    m2 = torch.as_tensor(r.m2, dtype=torch.float32).to(dev, non_blocking=True)
                    f = torch.as_tensor(r.wavelet, dtype=torch.float32).to(dev,
                                                                           non_blocking=True)
                    obs = r.observed.to(dev, non_blocking=True)
                    J = torch.empty(1, dtype=torch.float32, device=dev)
                    g1, g2 = torch.empty_like(m1), torch.empty_like(m1)
                    job.plan.gradient(r.param, m1, m2, f, obs, stream=job.stream,
                                      out=(J, g1, g2))
                    job.event.record(job.stream)
                job.bufs = (m1, m2, f, obs, J, g1, g2)
            except BaseException as e:   # re-raised by the serving loop
                job.error = e

        job.admitted = now
        job.thread = threading.Thread(target=submit, daemon=True)
        job.thread.start()

    def run(self, requests, verbose=False):
        """Serves `requests` in real time (arrival = seconds after the call);
        returns the Results sorted by request id."""
        pending = deque(sorted(requests, key=lambda q: q.arrival))
        waiting = deque()
        running = []
        free_streams = list(self.streams)
        used = 0
        results = []
        t0 = time.perf_counter()
        while pending or waiting or running:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                q = pending.popleft()
                plan = self.plan_for(q)
                fp = footprint(plan, q)
                if fp > self.budget:
                    raise RuntimeError(f"request {q.id} needs {fp} bytes > budget {self.budget}")
                waiting.append((q, plan, fp))
            # admission in arrival order; a later request may pass one that
            # does not fit yet, the head being retried first on every pass
            for item in list(waiting):
                if not free_streams:
                    break
                q, plan, fp = item
                if used + fp <= self.budget:
                    waiting.remove(item)
                    job = _Job(q, plan, free_streams.pop(0), fp)
                    used += fp
                    self._start(job, now)
                    running.append(job)
            progressed = False
            for job in list(running):
                if job.submitted() and job.error is not None:
                    raise job.error
                if job.submitted() and job.event.query():
                    t_done = time.perf_counter() - t0
                    m1, m2, f, obs, J, g1, g2 = job.bufs
                    res = Result(job.req.id, job.req.arrival, job.admitted, t_done,
                                 float(J.item()), g1, g2, job.footprint, job.req.cell_steps)
                    results.append(res)
                    running.remove(job)
                    free_streams.append(job.stream)
                    used -= job.footprint
                    job.bufs = None
                    job.plan.release_workspace()
                    job.plan = None
                    progressed = True
                    if verbose:
                        print(f"  req {res.id:3d} done: latency {res.latency * 1e3:9.1f} ms "
                              f"(queued {(res.admitted - res.arrival) * 1e3:8.1f} ms)", flush=True)
            if not progressed:
                time.sleep(2e-4)
        torch.cuda.synchronize(self.device)
        self.makespan = time.perf_counter() - t0
        return sorted(results, key=lambda r: r.id)


def summary(results, makespan):
    lat = np.array([r.latency for r in results]) * 1e3
    cells = sum(r.cell_steps for r in results)
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "makespan_s": makespan, "aggregate_gcells": cells / makespan / 1e9}


def make_requests(specs, device=None, param="vp-rho", nrec=360, npml=40):
    """Requests for serving_requests()-style specs: a problem shaped like the
    401² Gaussian benchmark per spec (Gaussian anomaly), with observed data modelled from the true
    model on the GPU and kept in pinned host memory."""
    from . import workloads as W
    dev = torch.device(device if device is not None else "cuda")
    out = []
    for s in specs:
        w = W.gauss_problem(s["n"], s["shots"], nrec, s["nt"], npml=npml,
                            contrast=s["contrast"], seed=s["seed"], name=f"req{s['id']}")
        g = Grid.of(w)
        plan = Plan(g, w.src_xz, w.rec_xz, device=dev)
        f = w.wavelet()
        obs = plan.forward("vp-rho", w.vp_true, w.rho_true, f)
        torch.cuda.synchronize(dev)
        obs_h = obs.cpu().pin_memory()
        del plan, obs
        if param == "vp-rho":
            m1, m2 = w.vp_start, w.rho_start
        else:
            raise ValueError(param)
        out.append(Request(s["id"], s["arrival"], g, w.src_xz, w.rec_xz, param, m1, m2, f,
                           obs_h, meta=s))
    return out


def main(argv=None):
    """Serves a seeded Poisson stream of mixed-size gradient requests (sides
    201..1201 + 40 PML, 8-64 shots, 1000-4000 steps) and prints one JSON
    line: latency percentiles, aggregate rate, and the same requests run one
    after another for comparison."""
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.8,
                    help="offered load as a fraction of the measured serial capacity")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    specs = W.serving_requests(a.requests, rate_hz=1.0)
    print(f"preparing {len(specs)} requests", file=sys.stderr, flush=True)
    reqs = make_requests(specs, device=dev)
    server = GradientServer(max_slots=a.slots, device=dev)
    # serial pass: each request alone, back to back (its service time)
    service = {}
    for q in reqs:
        plan = server.plan_for(q)
        m1 = torch.as_tensor(q.m1, dtype=torch.float32, device=dev)
        m2 = torch.as_tensor(q.m2, dtype=torch.float32, device=dev)
        f = torch.as_tensor(q.wavelet, dtype=torch.float32, device=dev)
        obs = q.observed.to(dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.gradient(q.param, m1, m2, f, obs)
        torch.cuda.synchronize()
        service[q.id] = time.perf_counter() - t
        del plan
        print(f"  alone: request {q.id} {q.meta['n']}^2 x {q.meta['shots']} shots x "
              f"{q.meta['nt']} steps: {service[q.id]:.3f} s", file=sys.stderr, flush=True)
    mean_s = float(np.mean(list(service.values())))
    cells = sum(q.cell_steps for q in reqs)
    out = {"slots": a.slots, "mean_service_alone_s": mean_s,
           "serial_gcells": cells / sum(service.values()) / 1e9,
           "requests_spec": [{k: s[k] for k in ("n", "shots", "nt")} for s in specs]}
    # Poisson arrivals rescaled so the offered load is a.load of the serial
    # capacity; then a burst (every request at t = 0) for the capacity
    for name, arrivals in (("poisson", [s["arrival"] * mean_s / a.load for s in specs]),
                           ("burst", [0.0] * len(specs))):
        for q, t in zip(reqs, arrivals):
            q.arrival = t
        res = server.run(reqs)
        rec = summary(res, server.makespan)
        if name == "poisson":
            rec["offered_load"] = a.load
        out[name] = rec
        print(f"{name}: p50 {rec['p50_ms']:.0f} ms, p99 {rec['p99_ms']:.0f} ms, "
              f"{rec['aggregate_gcells']:.1f} Gcell-updates/s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
