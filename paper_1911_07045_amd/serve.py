"""Continuous-batching server for many small lattice minimizations.

Requests (box, colloid, anchoring strength, FIRE settings) arrive over time.
The server admits a waiting request as soon as a batch slot and enough HBM
budget are free, builds its lattice and state on the device, and adds it to
one lq_batch; the batch advances every resident request by one kernel launch
per FIRE step, `chunk` steps per call.  Between calls, finished requests are
retired, their memory released and new arrivals admitted, so requests that
arrive while others run join the same launches.  Each request's trajectory is
independent of its batch mates (per-request controller and block-ordered
FP64 reductions).

The FP32 form (FP32 state, FP64 reductions and controller) ends with an FP64
polish when FP32 rounding stops it short of the request's tolerance.  One
FP32 force evaluation is off by up to ~30 u |H| max|q| ~ 1e-4 (30 summed
terms, |H| ~ 36 L1 + anchoring the stencil's infinity norm, u = 2^-24), so a
plateau of max|F| below fp32_floor = 1e-4 (no tenth's improvement of its best
for stall_steps steps, or the step limit reached) may be rounding, or just
slow relaxation.  The server then measures which: it evaluates the FP64 force
of the FP32 state and compares it with the FP32 force.  When the FP32 force
is off by at least noise_frac of its own max|F| (rounding dominates), the
request continues from its FP32 state in FP64 (a fresh FIRE start, at most
polish_steps steps) in a second batch; otherwise it keeps relaxing in FP32
(or, at its step limit, is reported as capped).  A request that needs more
device memory than the whole budget is refused at arrival.

Reported per request: arrival-to-result latency, steps (FP32 and polish),
status, final max|F| and energy, and whether it was polished.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import lqfire, synth

REFUSED = -1  # Result.status of a request larger than the whole budget


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
    polish_steps: int = 0
    polished: bool = False

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
    best: float = float("inf")  # best max|F| of the FP32 phase below the floor
    best_step: int = 0          # step at which best last fell by a tenth
    fp32_steps: int = 0         # steps of the FP32 phase (set when the polish starts)


def request_bytes(req, prec="f32"):
    """Device bytes one request holds while resident: q, v, F, the FIRE
    workspace (a second q, v, F plus small scratch), the neighbour mask and
    the directors used to build the initial state."""
    nx, ny, nz = req["shape"]
    N = nx * ny * nz
    e = 4 if prec == "f32" else 8
    return 6 * 5 * N * e + N + 3 * N * 8 + (1 << 20)


def _lattice(req, prec):
    lat = lqfire.Lattice(req["shape"], req.get("periodic", (True, True, True)), prec,
                         L1=req["L1"], L2=req.get("L2", 0.0), L3=req.get("L3", 0.0))
    if req.get("objects"):
        lat.set_boundaries(req["objects"])
    return lat


class Server:
    def __init__(self, max_members=64, hbm_budget=None, chunk=50, prec="f32", keep_states=False,
                 polish_steps=2000, fp32_floor=1e-4, stall_steps=1000, noise_frac=0.3):
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
        # FP64 polish of FP32 requests that stall below the FP32 floor
        self.polish_steps = int(polish_steps) if prec == "f32" else 0
        self.fp32_floor = float(fp32_floor)
        self.stall_steps = stall_steps
        self.noise_frac = float(noise_frac)
        self.noise_checks = 0
        self.batch64 = lqfire.Batch(self.max_members) if self.polish_steps > 0 else None
        self.polishing: list[_Live] = []
        self.keep_states = keep_states
        self.states = {}
        self.busy_s = 0.0

    # -- admission -------------------------------------------------------
    def reserve(self, req):
        """Bytes held for a request from admission to retirement: enough for
        its FP64 polish when the server polishes (the FP64 state is twice the
        FP32 one), so the budget holds in either phase."""
        return request_bytes(req, "f64" if self.polish_steps > 0 else self.prec)

    def fits(self, req):
        return (len(self.live) + len(self.polishing) < self.max_members
                and self.used + self.reserve(req) <= self.budget)

    def admit(self, req, now):
        torch = self.torch
        lat = _lattice(req, self.prec)
        dirs = torch.from_numpy(np.ascontiguousarray(
            synth.random_directors(req["dir_seed"], lat.N))).cuda()
        q = lat.set_uniaxial(dirs, lat.empty())
        v, F = lat.empty(), lat.empty()
        lat.fire_init(lqfire.fire_params_from_config(req), q, v, F)
        del dirs
        nb = self.reserve(req)
        self.used += nb
        live = _Live(req, lat, q, v, F, nb, now)
        rep = lat.fire_step(0)
        if rep.status != lqfire.RUNNING:
            return live, rep
        self.batch.add(lat)
        self.live.append(live)
        return live, None

    def _plateau(self, live, rep):
        """The FP32 phase is below the FP32 floor and has stopped improving:
        at the step limit, or without a tenth's improvement of its best
        max|F| for stall_steps steps."""
        if self.polish_steps <= 0 or rep.status == lqfire.CONVERGED or not rep.maxF < self.fp32_floor:
            return False
        if rep.status == lqfire.MAX_STEPS:
            return True
        if rep.maxF < 0.9 * live.best:
            live.best, live.best_step = rep.maxF, rep.step
        return self.stall_steps is not None and rep.step - live.best_step >= self.stall_steps

    def _rounding_bound(self, live):
        """The FP64 lattice of the request and whether FP32 rounding
        dominates its current force: max|F64(q) - F32(q)| >= noise_frac
        max|F32(q)| at the FP32 state q."""
        self.noise_checks += 1
        lat64 = _lattice(live.req, "f64")
        q64 = live.q.double().contiguous()
        F64 = lat64.compute_forces(q64)
        F32 = live.F.double()
        noise = (F64 - F32).abs().max().item()
        return lat64, q64, noise >= self.noise_frac * F32.abs().max().item()

    def _start_polish(self, live, rep, lat64, q64):
        """Moves a stalled FP32 request to FP64: its state in the FP64
        lattice, a fresh FIRE start with the request's tolerance, at most
        polish_steps steps."""
        req = live.req
        v64, F64 = lat64.empty(), lat64.empty()
        lat64.fire_init(lqfire.fire_params_from_config(req, max_steps=self.polish_steps), q64, v64, F64)
        live.lat.close()
        # the reservation made at admission covers the FP64 state
        p = _Live(req, lat64, q64, v64, F64, live.nbytes, live.admitted, fp32_steps=rep.step)
        r0 = lat64.fire_step(0)
        if r0.status != lqfire.RUNNING:
            return p, r0
        self.batch64.add(lat64)
        self.polishing.append(p)
        return p, None

    def _retire(self, live, rep, now, results, polished=False):
        e = live.lat.energy(live.q)["total"]
        steps = live.fp32_steps if polished else rep.step
        results.append(Result(live.req["id"], live.req["arrival"], live.admitted, now, steps, rep.status,
                              rep.maxF, e, tuple(live.req["shape"]),
                              polish_steps=rep.step if polished else 0, polished=polished))
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
        while i < len(pending) or self.live or self.polishing:
            now = clock()
            while i < len(pending) and pending[i]["arrival"] <= now:
                req = pending[i]
                if self.reserve(req) > self.budget:
                    t = time.perf_counter() - t0
                    results.append(Result(req["id"], req["arrival"], t, t, 0, REFUSED, float("nan"),
                                          float("nan"), tuple(req["shape"])))
                    i += 1
                    continue
                if not self.fits(req):
                    break
                live, rep = self.admit(req, time.perf_counter() - t0)
                if rep is not None:  # already converged at the start
                    self._retire(live, rep, time.perf_counter() - t0, results)
                i += 1
            if not self.live and not self.polishing:
                if i < len(pending):
                    wait = pending[i]["arrival"] - (time.perf_counter() - t0)
                    if realtime and wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            tb = time.perf_counter()
            stepped64 = list(self.polishing)  # members of the FP64 batch during this step
            reps = self.batch.step(self.chunk) if self.live else []
            reps64 = self.batch64.step(self.chunk) if stepped64 else []
            self.busy_s += time.perf_counter() - tb
            now = time.perf_counter() - t0
            keep = []
            for live, rep in zip(list(self.live), reps):
                polish = None
                if self._plateau(live, rep):
                    lat64, q64, rounding = self._rounding_bound(live)
                    if rounding:
                        polish = (lat64, q64)
                    else:
                        lat64.close()
                        live.best_step = rep.step  # slow, not stalled: look again later
                if rep.status == lqfire.RUNNING and polish is None:
                    keep.append(live)
                    continue
                self.batch.remove(live.lat)
                if polish is not None:
                    p, r0 = self._start_polish(live, rep, *polish)
                    if r0 is not None:
                        self._retire(p, r0, now, results, polished=True)
                else:
                    self._retire(live, rep, now, results)
            self.live = keep
            for p, rep in zip(stepped64, reps64):
                if rep.status != lqfire.RUNNING:
                    self.batch64.remove(p.lat)
                    self.polishing.remove(p)
                    self._retire(p, rep, now, results, polished=True)
            if log:
                log(f"t={now:7.2f}s resident={len(self.live)} polishing={len(self.polishing)} "
                    f"done={len(results)} admitted={i}/{len(pending)}")
        self.wall_s = time.perf_counter() - t0
        return results


def _group(rs, span):
    lat = np.array([r.latency for r in rs])
    if len(rs) == 0:
        return {"count": 0}
    return {"count": len(rs), "per_s": len(rs) / span,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean())}


def summarize(results, wall_s, busy_s):
    """Throughput and latency of a served stream, over all requests and split
    by outcome: converged (to the request's tolerance, in FP32 or after the
    FP64 polish) and capped (at the step limit, polish included)."""
    served = [r for r in results if r.status != REFUSED]
    first = min(r.arrival for r in results)
    last = max(r.finished for r in served) if served else first
    span = max(last - first, 1e-9)
    lat = np.array([r.latency for r in served])
    site_updates = sum(int(np.prod(r.shape)) * (r.steps + r.polish_steps) for r in served)
    conv = [r for r in served if r.status == lqfire.CONVERGED]
    capped = [r for r in served if r.status == lqfire.MAX_STEPS]
    pol = [r for r in served if r.polished]
    return {
        "requests": len(results),
        "requests_per_s": len(served) / span,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "converged": _group(conv, span),
        "capped": _group(capped, span),
        "refused": sum(r.status == REFUSED for r in results),
        "nonfinite": sum(r.status == lqfire.NONFINITE for r in served),
        "polished": {"count": len(pol), "converged": sum(r.status == lqfire.CONVERGED for r in pol),
                     "polish_steps_mean": float(np.mean([r.polish_steps for r in pol])) if pol else 0.0},
        "capped_maxF_median": float(np.median([r.maxF for r in capped])) if capped else None,
        "site_updates_per_s": site_updates / span,
        "gpu_busy_frac": busy_s / wall_s,
        "wall_s": wall_s,
    }
