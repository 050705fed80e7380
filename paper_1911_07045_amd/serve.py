"""Continuous-batching server for many small lattice minimizations.

Requests (box, colloid, anchoring strength, FIRE settings) arrive over time.
The server admits a waiting request as soon as a batch slot and enough HBM
budget are free, builds its lattice and state on the device, and adds it to
one lq_batch; the batch advances every resident request by one kernel launch
per FIRE step, `chunk` steps per call.  Between calls, converged (or capped)
requests are retired, their memory released and new arrivals admitted, so
requests that arrive while others run join the same launches.  Each
request's trajectory is independent of its batch mates (per-request
controller and block-ordered FP64 reductions).

Reported per request: arrival-to-result latency, steps, status, final
max|F| and energy.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import lqfire, synth


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    status: int
    maxF: float
    energy: float
    shape: tuple

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class _Live:
    req: dict
    lat: lqfire.Lattice
    q: object
    v: object
    F: object
    nbytes: int
    admitted: float


def request_bytes(req, prec="f32"):
    """Device bytes one request holds while resident: q, v, F, the FIRE
    workspace (a second q, v, F plus small scratch), the neighbour mask and
    the directors used to build the initial state."""
    nx, ny, nz = req["shape"]
    N = nx * ny * nz
    e = 4 if prec == "f32" else 8
    return 6 * 5 * N * e + N + 3 * N * 8 + (1 << 20)


class Server:
    def __init__(self, max_members=64, hbm_budget=None, chunk=50, prec="f32", keep_states=False):
        import torch
        self.torch = torch
        self.prec = prec
        self.chunk = int(chunk)
        self.max_members = int(max_members)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.used = 0
        self.batch = lqfire.Batch(self.max_members)
        self.live: list[_Live] = []
        self.keep_states = keep_states
        self.states = {}
        self.busy_s = 0.0

    # -- admission -------------------------------------------------------
    def fits(self, req):
        return (len(self.live) < self.max_members
                and self.used + request_bytes(req, self.prec) <= self.budget)

    def admit(self, req, now):
        torch = self.torch
        lat = lqfire.Lattice(req["shape"], req.get("periodic", (True, True, True)), self.prec,
                             L1=req["L1"], L2=req.get("L2", 0.0), L3=req.get("L3", 0.0))
        if req.get("objects"):
            lat.set_boundaries(req["objects"])
        dirs = torch.from_numpy(np.ascontiguousarray(
            synth.random_directors(req["dir_seed"], lat.N))).cuda()
        q = lat.set_uniaxial(dirs, lat.empty())
        v, F = lat.empty(), lat.empty()
        lat.fire_init(lqfire.fire_params_from_config(req), q, v, F)
        del dirs
        nb = request_bytes(req, self.prec)
        self.used += nb
        live = _Live(req, lat, q, v, F, nb, now)
        rep = lat.fire_step(0)
        if rep.status != lqfire.RUNNING:
            return live, rep
        self.batch.add(lat)
        self.live.append(live)
        return live, None

    def _retire(self, live, rep, now, results):
        e = live.lat.energy(live.q)["total"]
        results.append(Result(live.req["id"], live.req["arrival"], live.admitted, now, rep.step, rep.status,
                              rep.maxF, e, tuple(live.req["shape"])))
        if self.keep_states:
            self.states[live.req["id"]] = (live.q.cpu(), live.v.cpu(), live.F.cpu())
        self.used -= live.nbytes
        live.lat.close()

    # -- main loop ---------------------------------------------------------
    def run(self, requests, realtime=True, log=None):
        """Serves requests (dicts with an 'arrival' time in seconds relative
        to the start).  realtime=False admits requests in arrival order as
        soon as they fit, ignoring the clock."""
        pending = sorted(requests, key=lambda r: r["arrival"])
        results = []
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        i = 0
        while i < len(pending) or self.live:
            now = clock()
            while i < len(pending) and pending[i]["arrival"] <= now and self.fits(pending[i]):
                t_adm = time.perf_counter() - t0
                live, rep = self.admit(pending[i], t_adm)
                if rep is not None:  # already converged at the start
                    self._retire(live, rep, time.perf_counter() - t0, results)
                i += 1
            if not self.live:
                if i < len(pending):
                    wait = pending[i]["arrival"] - (time.perf_counter() - t0)
                    if realtime and wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            tb = time.perf_counter()
            reps = self.batch.step(self.chunk)
            self.busy_s += time.perf_counter() - tb
            now = time.perf_counter() - t0
            keep = []
            for live, rep in zip(list(self.live), reps):
                if rep.status != lqfire.RUNNING:
                    self.batch.remove(live.lat)
                    self._retire(live, rep, now, results)
                else:
                    keep.append(live)
            self.live = keep
            if log:
                log(f"t={now:7.2f}s resident={len(self.live)} done={len(results)} "
                    f"admitted={i}/{len(pending)}")
        self.wall_s = time.perf_counter() - t0
        return results


def summarize(results, wall_s, busy_s):
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.finished for r in results)
    site_updates = sum(int(np.prod(r.shape)) * r.steps for r in results)
    return {
        "requests": len(results),
        "solves_per_s": len(results) / (last - first),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "converged": int(sum(r.status == lqfire.CONVERGED for r in results)),
        "capped": int(sum(r.status == lqfire.MAX_STEPS for r in results)),
        "site_updates_per_s": site_updates / (last - first),
        "gpu_busy_frac": busy_s / wall_s,
        "wall_s": wall_s,
    }
