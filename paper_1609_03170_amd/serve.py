"""Request loop for continuous batching of gradient evaluations.

Requests (one control array each) arrive over time for several operator
sets (model shapes).  A request is admitted as soon as it has arrived and
the HBM budget (the sum of the device bytes of the requests in flight) has
room for it; every admitted request then advances together with the others
of its shape in the batched launches of og_server_step, so requests that
arrive while others run overlap with them on the device.

Every shape has its own server and stream; one host thread issues all of
them.  A shape's next step is issued as soon as its previous one has
finished on the device (a completion event per step; no device-wide
synchronisation), so the shapes run side by side on the GPU.  Completion
time is taken when the event of the step that retired the request has
fired; latency = completion - arrival.  Controls are uploaded and checked on
a separate admission stream, so admitting a request does not wait for the
steps in flight.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .api import Problem, Server


@dataclass
class Outcome:
    latencies: dict = field(default_factory=dict)   # tag -> seconds
    results: dict = field(default_factory=dict)     # tag -> (phi, grad) on device (keep=True)
    wall: float = 0.0
    peak_bytes: int = 0
    steps: int = 0

    def percentile(self, q):
        v = np.array(sorted(self.latencies.values()))
        return float(np.percentile(v, q)) if len(v) else float("nan")

    def throughput(self):
        return len(self.latencies) / self.wall if self.wall > 0 else float("nan")


class ServingLoop:
    """One Server (and one stream) per model shape; FIFO admission under a
    byte budget."""

    def __init__(self, models: dict, *, prec="f32", budget_bytes=16 << 30, max_slices=8, max_active=4096,
                 resident=False, device=None):
        """resident: every request keeps the packed Hermitian halves of all
        its forward states (no checkpoint recompute in its backward sweep;
        more device bytes per request, counted against the budget)."""
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.budget = int(budget_bytes)
        self.max_slices = int(max_slices)
        self.problems, self.servers, self.streams, self.sigma, self.rho0 = {}, {}, {}, {}, {}
        for key, w in models.items():
            p = Problem.from_workload(w, prec=prec, path="banded", gmode="grape1", device=self.device)
            if resident:
                p.set_resident(1 << 30)  # every slice of every request
            self.problems[key] = p
            self.servers[key] = Server(p, max_active=max_active)
            self.streams[key] = torch.cuda.Stream(device=self.device)
            self.sigma[key] = torch.tensor(w.sigma, device=self.device)
            self.rho0[key] = torch.tensor(w.rho0, device=self.device)
        self.dt = {key: w.dt for key, w in models.items()}
        self.admit_stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)  # operators and states uploaded before any step

    def close(self):
        torch.cuda.synchronize(self.device)
        for s in self.servers.values():
            s.close()
        for p in self.problems.values():
            p.close()

    def _issue(self, key):
        """Enqueue one step of shape `key` on its stream; returns its completion event."""
        with torch.cuda.device(self.device), torch.cuda.stream(self.streams[key]):
            self.servers[key].step(self.max_slices)
            ev = torch.cuda.Event()
            ev.record(self.streams[key])
        return ev

    def run(self, requests, controls, *, time_scale=1.0, keep=False, log=None):
        """requests: list of dicts with keys id, shape, arrival (seconds,
        multiplied by time_scale); controls(req) -> numpy [N_t, K]."""
        pending = sorted(requests, key=lambda r: r["arrival"])
        out = Outcome()
        used = 0
        inflight = {}     # tag -> (shape, bytes, arrival)
        running = {}      # shape -> completion event of its step in flight
        t0 = time.perf_counter()
        i = 0
        n_total = len(pending)
        while len(out.latencies) < n_total:
            now = time.perf_counter() - t0
            # admission: FIFO, arrived, within budget
            while i < n_total and pending[i]["arrival"] * time_scale <= now:
                r = pending[i]
                key = r["shape"]
                srv = self.servers[key]
                need = srv.request_bytes(r["n_t"])
                if used + need > self.budget and inflight:
                    break
                with torch.cuda.device(self.device), torch.cuda.stream(self.admit_stream):
                    u = torch.tensor(controls(r), device=self.device)
                    if not srv.submit(r["id"], u, self.rho0[key], self.sigma[key], self.dt[key]):
                        break
                    # the request's inputs and workspace are complete before its shape's stream uses them
                    self.streams[key].wait_stream(self.admit_stream)
                used += need
                out.peak_bytes = max(out.peak_bytes, used)
                inflight[r["id"]] = (key, need, r["arrival"] * time_scale)
                i += 1
            # retire the steps that have finished
            progressed = False
            for key in list(running):
                if running[key].query():
                    del running[key]
                    progressed = True
                    done_t = time.perf_counter() - t0
                    for tag, res in self.servers[key].completed().items():
                        k2, need, arr = inflight.pop(tag)
                        used -= need
                        out.latencies[tag] = done_t - arr
                        if keep:
                            out.results[tag] = res
            # issue the next step of every shape that has work and no step in flight
            for key, srv in self.servers.items():
                if key not in running and srv.active:
                    running[key] = self._issue(key)
                    out.steps += 1
                    progressed = True
                    if log and out.steps % 500 == 0:
                        log(f"[serve] t={time.perf_counter() - t0:.1f}s done={len(out.latencies)}/{n_total} "
                            f"inflight={len(inflight)} used={used / 2**30:.2f} GiB")
            if progressed:
                continue
            if running:
                # nothing to do on the host until the oldest step ends (or the next arrival)
                ev = next(iter(running.values()))
                if i < n_total:
                    wait = pending[i]["arrival"] * time_scale - (time.perf_counter() - t0)
                    if wait > 0.0005:
                        time.sleep(min(wait, 0.0005))
                        continue
                ev.synchronize()
            elif i < n_total:
                time.sleep(max(0.0, pending[i]["arrival"] * time_scale - (time.perf_counter() - t0)))
        out.wall = time.perf_counter() - t0
        return out
