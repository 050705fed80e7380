#!/usr/bin/env python3
"""Benchmark: fused lattice Landau-de Gennes force + FIRE steps on one MI355X.

One step = one pass of the whole path over the lattice: steering, both half
kicks, drift, the bulk + elastic + anchoring force at every site, the FP64
reductions of F.v, |F|^2, |v|^2, max|F| and the FIRE controller.

Default workload: 256^3 periodic box with 8 homeotropic Rapini-Papoular
colloids (radii U[8,16], W U[1,10]), one-constant L1 = 2.32, FP32 q/v/F with
FP64 reductions, random initial directors.  Inputs are resident in HBM before
the timed region; K steps run through lq_fire_step with no host round trip.

Prints one JSON line.  value = lattice sites x steps / wall seconds.
roofline.achieved = algorithmic bytes per step (read + write of q, v, F:
30 values per site) / average step-kernel duration from HIP events on the
library's stream.  cpu_baseline = the FP64 oracle timed on the host cores for
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FIRE site-updates/s & %HBM peak at 256^3; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_1911_07045_amd import synth
    if name == "multi_colloid256":
        return synth.multi_colloid(256)
    if name == "multi_colloid256_f64":
        c = synth.multi_colloid(256)
        c.update(name="multi_colloid256_f64", prec="f64")
        return c
    if name == "colloid_slab128":
        return synth.colloid_slab(128)
    if name == "colloid_slab128_f32":
        c = synth.colloid_slab(128)
        c["prec"] = "f32"
        return c
    if name == "patterned_wall512":
        return synth.patterned_wall(512)
    if name == "bulk32":
        return synth.bulk32()
    if name == "bulk256":
        return synth.bulk(256)
    if name == "bulk256_f64":
        return synth.bulk(256, prec="f64")
    if name == "bulk256_l23":
        c = synth.bulk(256)
        c.update(name="bulk256_l23", L2=1.16, L3=1.16)
        return c
    raise SystemExit(f"unknown workload {name}")


def describe(cfg):
    objs = cfg["objects"]
    kinds = {}
    for o in objs:
        kinds[o["kind"]] = kinds.get(o["kind"], 0) + 1
    return {"workload": cfg["name"], "shape": list(cfg["shape"]), "periodic": list(cfg["periodic"]),
            "objects": kinds, "L1": cfg["L1"], "L2": cfg["L2"], "L3": cfg["L3"],
            "state_dtype": cfg["prec"], "reductions": "f64",
            "fire": {k: cfg["fire"][k] for k in ("dt0", "dt_max", "alpha0")},
            "init": f"random directors, seed {cfg['dir_seed']}, S = S0"}


def gpu_leg(cfg, steps, warmup):
    import numpy as np
    import torch

    from paper_1911_07045_amd import lqfire, synth

    torch.cuda.set_device(0)
    # fresh allocations for the timed lattice: buffers placed in segments that
    # torch's allocator kept from earlier legs measured up to 19% slower (FP64)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    lat = lqfire.lattice_from_config(cfg)
    nx, ny, nz = cfg["shape"]
    N = nx * ny * nz
    dirs = torch.from_numpy(np.ascontiguousarray(synth.random_directors(cfg["dir_seed"], N))).cuda()
    q = lat.set_uniaxial(dirs, lat.empty())
    del dirs
    v, F = lat.empty(), lat.empty()
    # every step is executed: no tolerance stop inside the timed region
    prm = lqfire.fire_params_from_config(cfg, force_tol=0.0, max_steps=1 << 62)
    lat.fire_init(prm, q, v, F)
    e0 = lat.energy(q)
    if warmup:
        lat.fire_step(warmup)
    stream = lat.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    rep = lat.fire_step(steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert rep.status == lqfire.RUNNING and rep.step == warmup + steps, rep.as_dict()
    # the same call with zero steps: everything but the step kernels
    ev[2].record(stream)
    lat.fire_step(0)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_all = ev[0].elapsed_time(ev[1])
    t_fixed = ev[2].elapsed_time(ev[3])
    kernel_ms = max(t_all - t_fixed, 1e-9) / steps
    e1 = lat.energy(q)
    elem = 8 if cfg["prec"] == "f64" else 4
    return dict(wall_s=t1 - t0, kernel_ms=kernel_ms, bytes_per_site=30 * elem, N=N,
                n_sim=e1["n_sim"], report=rep.as_dict(), E0=e0["total"], E1=e1["total"],
                ws_bytes=lat.workspace_bytes())


def _timed_steps(lat, steps):
    """Wall seconds and per-step kernel milliseconds (HIP events on the
    library's stream, minus a zero-step call) of lat.fire_step(steps)."""
    import torch

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(lat.stream)
    rep = lat.fire_step(steps)
    ev[1].record(lat.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev[2].record(lat.stream)
    lat.fire_step(0)
    ev[3].record(lat.stream)
    torch.cuda.synchronize()
    kernel_ms = max(ev[0].elapsed_time(ev[1]) - ev[2].elapsed_time(ev[3]), 1e-9) / steps
    return t1 - t0, kernel_ms, rep


def minimizer_leg(cfg, steps=300, warmup=20):
    """Gradient descent and Nesterov steps on the same workload: the fused
    kernel moves q and F (GD: 20 values per site) or q, m and F (Nesterov:
    30 values per site)."""
    import numpy as np
    import torch

    from paper_1911_07045_amd import lqfire, synth

    nx, ny, nz = cfg["shape"]
    N = nx * ny * nz
    elem = 8 if cfg["prec"] == "f64" else 4
    out = {}
    for method, dt, mu, vals in (("gd", 0.01, 0.0, 20), ("nesterov", 0.01, 0.9, 30)):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()  # fresh allocations, as for the FIRE legs
        lat = lqfire.lattice_from_config(cfg)
        dirs = torch.from_numpy(np.ascontiguousarray(synth.random_directors(cfg["dir_seed"], N))).cuda()
        q = lat.set_uniaxial(dirs, lat.empty())
        del dirs
        v, F = lat.empty(), lat.empty()
        lat.descent_init(lqfire.make_descent_params(method, dt, mu, force_tol=0.0, max_steps=1 << 62), q, v, F)
        lat.fire_step(warmup)
        wall, kernel_ms, rep = _timed_steps(lat, steps)
        assert rep.status == lqfire.RUNNING, rep.as_dict()
        gbs = vals * elem * N / (kernel_ms * 1e-3) / 1e9
        out[method] = {"dt": dt, "momentum": mu, "steps": steps, "ms_per_step": 1e3 * wall / steps,
                       "kernel_ms": kernel_ms, "site_updates_per_s": N * steps / wall,
                       "algorithmic_bytes_per_site": vals * elem, "achieved_GBs": gbs,
                       "frac_hbm_peak": gbs / HBM_PEAK_GBS}
        del q, v, F
        lat.close()
    return out


def _random_start(lat, cfg, seed=None):
    import numpy as np
    import torch

    from paper_1911_07045_amd import synth

    dirs = torch.from_numpy(np.ascontiguousarray(
        synth.random_directors(cfg["dir_seed"] if seed is None else seed, lat.N))).cuda()
    return lat.set_uniaxial(dirs, lat.empty())


def convergence_leg(n=256, prec="f32", budget_s=10.0, chunk=100):
    """FIRE against separately tuned gradient descent (and Nesterov) on the
    n^3 periodic bulk box from the same random start (the paper's FIRE-vs-GD
    comparison of its minimizer section): energy above the uniform nematic
    state and |F|/sqrt(N) against the wall-clock time spent stepping."""
    import math

    import numpy as np
    import torch

    from paper_1911_07045_amd import lqfire, synth

    cfg = synth.bulk(n, prec=prec)
    lat = lqfire.lattice_from_config(cfg)
    N = lat.N
    uni = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    uni[:N] = 1.0
    E_min = lat.energy(lat.set_uniaxial(uni, lat.empty()))["total"]
    del uni

    def run(method, dt=None, mu=0.0, budget=budget_s):
        q = _random_start(lat, cfg)
        v, F = lat.empty(), lat.empty()
        if method == "fire":  # dt: the largest FIRE time step
            lat.fire_init(lqfire.fire_params_from_config(cfg, dt_max=dt, force_tol=0.0, max_steps=1 << 62),
                          q, v, F)
        else:
            lat.descent_init(lqfire.make_descent_params(method, dt, mu, force_tol=0.0, max_steps=1 << 62),
                             q, v, F)
        t, steps, curve = 0.0, 0, []
        E = lat.energy(q)["total"]
        curve.append((0.0, 0, E - E_min, float("nan")))
        while t < budget:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                rep = lat.fire_step(chunk)
            except lqfire.LQError as e:  # a diverging step size in the tuning sweep
                if e.code != lqfire.LQ_ENONFINITE:
                    raise
                curve.append((t, steps, float("inf"), float("inf")))
                break
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            steps += chunk
            E = lat.energy(q)["total"]
            if not math.isfinite(E) or rep.status == lqfire.NONFINITE:
                curve.append((t, steps, float("inf"), float("inf")))
                break
            curve.append((t, steps, E - E_min, rep.normF / math.sqrt(N)))
        del q, v, F
        return curve

    # tuning, separately for each method: the step (FIRE: its largest time
    # step) whose run reaches the lowest energy in the same short time
    tuned = {}
    for method, mu, dts in (("fire", 0.0, (0.01, 0.03, 0.1, 0.2)),
                            ("gd", 0.0, (0.005, 0.01, 0.02, 0.03, 0.04)),
                            ("nesterov", 0.9, (0.002, 0.005, 0.01, 0.02))):
        best = None
        for dt in dts:
            c = run(method, dt, mu, budget=0.5)
            dE = c[-1][2]
            if math.isfinite(dE) and (best is None or dE < best[1]):
                best = (dt, dE)
        tuned[method] = (best[0], mu)
    out = {"workload": f"bulk{n}", "prec": prec, "E_min": E_min, "budget_s": budget_s, "chunk": chunk,
           "tuned": {k: {"dt": v[0], "momentum": v[1]} for k, v in tuned.items()},
           "fire_fixed": {k: cfg["fire"][k] for k in ("dt0", "alpha0")}, "methods": {}}
    runs = [("fire", "fire") + tuned["fire"], ("fire_dtmax_0.01", "fire", 0.01, 0.0),
            ("gd", "gd") + tuned["gd"], ("nesterov", "nesterov") + tuned["nesterov"]]
    for name, method, dt, mu in runs:
        c = run(method, dt, mu)
        reach = {}
        for thr in (1e-1, 1e-2, 1e-3, 1e-4):
            hit = next((r for r in c[1:] if r[3] <= thr), None)
            reach[f"{thr:g}"] = None if hit is None else {"s": hit[0], "steps": hit[1]}
        out["methods"][name] = {"dt": dt, "momentum": mu,
                                "curve": [[round(a, 4), b, d, f] for a, b, d, f in c],
                                "time_to_F_per_sqrtN": reach}
        print(f"[convergence] {name}: {c[-1][1]} steps in {c[-1][0]:.2f} s, "
              f"E-Emin {c[-1][2]:.4g}, |F|/sqrtN {c[-1][3]:.3g}", file=sys.stderr, flush=True)
    lat.close()
    return out


def step_scaling_leg(sizes=(16, 24, 32, 48, 64), seeds=(0, 1, 2), tol=1e-6, max_steps=200000):
    """Steps FIRE needs to reach max|F| < tol from a random start, against the
    box side L: periodic bulk, and one homeotropic colloid of radius L/4 at
    the centre (the paper reports growth about like L and L^(3/2))."""
    import numpy as np

    from paper_1911_07045_amd import lqfire, synth

    out = {"tol": tol, "max_steps": max_steps, "prec": "f64", "geometries": {}}
    for geo in ("bulk", "colloid"):
        rows = []
        for L in sizes:
            cfg = synth.bulk(L, prec="f64")
            if geo == "colloid":
                c = (L - 1) / 2.0
                cfg["objects"] = [dict(kind="sphere", center=(c, c, c), radius=L / 4.0, law="rp", W=5.0,
                                       dir="normal")]
            steps = []
            for sd in seeds:
                lat = lqfire.lattice_from_config(cfg)
                q = _random_start(lat, cfg, seed=1000 * L + sd)
                rep = lat.minimize(lqfire.fire_params_from_config(cfg, force_tol=tol, max_steps=max_steps), q)[0]
                steps.append(int(rep.step) if rep.status == lqfire.CONVERGED else None)
                del q
                lat.close()
            ok = [s for s in steps if s is not None]
            rows.append({"L": L, "steps": steps, "median": float(np.median(ok)) if ok else None})
            print(f"[step-scaling] {geo} L={L}: {steps}", file=sys.stderr, flush=True)
        pts = [(r["L"], r["median"]) for r in rows if r["median"]]
        slope = None
        if len(pts) >= 2:
            x = np.log([p[0] for p in pts])
            y = np.log([p[1] for p in pts])
            slope = float(np.polyfit(x, y, 1)[0])
        out["geometries"][geo] = {"rows": rows, "loglog_slope": slope}
    return out


def cpu_leg(cfg):
    """The FP64 oracle on the same workload: FIRE initialisation untimed,
    then whole FIRE steps over the full lattice until about 10 s have passed."""
    import oracle
    from paper_1911_07045_amd import synth

    p = oracle.Problem(cfg["shape"], cfg["periodic"], L1=cfg["L1"], L2=cfg["L2"], L3=cfg["L3"],
                       objects=cfg["objects"])
    q0 = p.uniaxial(synth.random_directors(cfg["dir_seed"], p.N))
    prm = oracle.fire_params(force_tol=0.0, max_steps=1 << 40, dt0=cfg["fire"]["dt0"],
                             dt_max=cfg["fire"]["dt_max"], alpha0=cfg["fire"]["alpha0"])
    st, q, v, F = p.fire_init(prm, q0)
    del q0
    n = 0
    t0 = time.perf_counter()
    while True:
        p.fire_steps(prm, st, q, v, F, 1)
        n += 1
        if time.perf_counter() - t0 > 10.0:
            break
    dt = time.perf_counter() - t0
    sx, sy, sz = cfg["shape"]
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=p.N * n / dt, unit="site-updates/s", cores=oracle.threads(), kind="oracle",
                cpu_model=cpu, seconds=dt,
                sample=f"{n} whole FIRE step(s) of the FP64 oracle on the full {sx}x{sy}x{sz} "
                       f"workload after an untimed initialisation (literal average over the "
                       f"2^3 difference choices, gcc -O2, OpenMP over z-planes)")


def oracle_steps(name, steps):
    """Times `steps` whole FIRE steps of the FP64 oracle on workload `name`
    after an untimed initialisation, with the threads OpenMP gives it."""
    import oracle
    from paper_1911_07045_amd import synth

    cfg = workload(name)
    p = oracle.Problem(cfg["shape"], cfg["periodic"], L1=cfg["L1"], L2=cfg["L2"], L3=cfg["L3"],
                       objects=cfg["objects"])
    q0 = p.uniaxial(synth.random_directors(cfg["dir_seed"], p.N))
    prm = oracle.fire_params(force_tol=0.0, max_steps=1 << 40)
    st, q, v, F = p.fire_init(prm, q0)
    t0 = time.perf_counter()
    p.fire_steps(prm, st, q, v, F, steps)
    dt = time.perf_counter() - t0
    return {"workload": name, "threads": oracle.threads(), "steps": steps, "seconds": dt,
            "site_updates_per_s": p.N * steps / dt}


def oracle_timing(plan=(("bulk32", 50, 10), ("colloid_slab128", 3, 0), ("multi_colloid256", 2, 0))):
    """The oracle's FIRE step rate on the small, medium and headline
    workloads, on all host cores and on one core (each in a child process,
    since OpenMP fixes its thread count at start-up)."""
    import subprocess

    rows = []
    for name, steps_all, steps_one in plan:
        for threads, steps in ((None, steps_all), (1, steps_one)):
            if steps <= 0:
                continue
            env = dict(os.environ)
            if threads:
                env["OMP_NUM_THREADS"] = str(threads)
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-child", name, str(steps)],
                               env=env, capture_output=True, text=True, check=True)
            rows.append(json.loads(r.stdout.strip().splitlines()[-1]))
            print(f"[bench] oracle {rows[-1]}", file=sys.stderr, flush=True)
    return rows


GOLDEN_SLAB = os.path.join(ROOT, "tests", "golden", "colloid_slab128_fire.json")


def _stage_vs_oracle(gold, lat, q, rep, sites):
    """Errors of one stage's GPU result against the oracle's stored one:
    energy terms (relative to each term), max|F_i| and |F|/sqrt(N_sim)
    (relative), max|dQ| over the stored sites, and whether the controller
    took the same decisions (step, n_pos, restarts)."""
    import numpy as np

    e = lat.energy(q)
    ge = gold["energy"]
    qs = q.double().reshape(5, -1)[:, sites].T.cpu().numpy()
    n_sim = e["n_sim"]
    gs = gold["state"]
    return {
        "rel_energy_err": {k: abs(e[k] - ge[k]) / max(abs(ge[k]), 1e-300)
                           for k in ("bulk", "elastic", "anchoring", "total")},
        "rel_maxF_err": abs(rep.maxF - gold["maxF"]) / gold["maxF"],
        "rel_normF_per_site_err": abs(rep.normF / n_sim ** 0.5 - gold["normF_over_sqrt_nsim"])
                                  / gold["normF_over_sqrt_nsim"],
        "max_abs_dQ_sampled": float(np.abs(qs - np.array(gold["q"])).max()),
        "controller_equal": (rep.step, rep.n_pos, rep.restarts) == (gs["step"], gs["n_pos"], gs["restarts"]),
    }


def precision_vs_oracle(golden=GOLDEN_SLAB):
    """The 128^3 colloid slab (walls, colloid, L2/L3) on the oracle's stored
    FP64 schedule: 2000 FIRE steps from the workload's random start, then a
    fresh FIRE start (v = 0, dt0) for 200 FP64 steps.  Run on the GPU in FP64
    and in the FP32 form (FP32 state and FP64 reductions for the 2000 steps,
    then the 200-step FP64 polish), each stage compared with the oracle's
    stored energy terms, forces and q at its sampled sites."""
    import numpy as np
    import torch

    from paper_1911_07045_amd import lqfire, synth

    if not os.path.exists(golden):
        return {"status": f"no stored oracle result ({os.path.relpath(golden, ROOT)} missing)"}
    with open(golden) as f:
        g = json.load(f)
    cfg = synth.colloid_slab(128)
    sites = np.array(g["sites"], dtype=np.int64)
    steps = dict((st["stage"], st["steps"]) for st in g["schedule"])
    t0 = time.perf_counter()
    lat64 = lqfire.lattice_from_config(cfg, prec="f64")
    dirs = torch.from_numpy(np.ascontiguousarray(synth.random_directors(cfg["dir_seed"], lat64.N))).cuda()

    def fire(lat, q, n):
        v, F = lat.empty(), lat.empty()
        lat.fire_init(lqfire.fire_params_from_config(cfg, force_tol=0.0, max_steps=n), q, v, F)
        return lat.fire_step(n)

    out = {"workload": "colloid_slab128", "reference": "FP64 oracle, stored in " + os.path.relpath(golden, ROOT),
           "schedule": f"{steps['fire2000']} FIRE steps from random directors (seed {cfg['dir_seed']}), then "
                       f"{steps['polish200']} FP64 FIRE steps from a fresh start",
           "sampled_sites": len(sites), "oracle_seconds": g.get("seconds")}
    for form in ("f64", "f32"):
        lat = lat64 if form == "f64" else lqfire.lattice_from_config(cfg, prec="f32")
        q = lat.set_uniaxial(dirs, lat.empty())
        rep = fire(lat, q, steps["fire2000"])
        r = {"fire2000": _stage_vs_oracle(g["stages"]["fire2000"], lat, q, rep, sites)}
        q64 = q if form == "f64" else q.double().contiguous()
        if form == "f32":
            del q
            lat.close()
        rep = fire(lat64, q64, steps["polish200"])
        r["polish200"] = _stage_vs_oracle(g["stages"]["polish200"], lat64, q64, rep, sites)
        out["fp64_gpu" if form == "f64" else "fp32_form"] = r
        del q64
    lat64.close()
    out["seconds"] = time.perf_counter() - t0
    return out


def precision_minima(n=128, tol=1e-9, fp32_tol=1e-5, max_steps=400000, chunk=5000):
    """Converged minima of the two forms on the colloid slab, from a uniform
    x-aligned director (a smooth relaxation into one minimum): FP64 FIRE to
    max|F_i| < tol; the FP32 form (FP32 FIRE to max|F_i| < fp32_tol, above
    its rounding floor, then an FP64 polish from a fresh FIRE start to tol).
    Reports the relative energy difference and max|dQ| over every site,
    against the bars 1e-6 and 1e-5."""
    import torch

    from paper_1911_07045_amd import lqfire, synth

    cfg = synth.colloid_slab(n)
    t0 = time.perf_counter()
    lat64 = lqfire.lattice_from_config(cfg, prec="f64")
    lat32 = lqfire.lattice_from_config(cfg, prec="f32")
    N = lat64.N
    dirs = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    dirs[:N] = 1.0

    def run(lat, q, force_tol, label):
        v, F = lat.empty(), lat.empty()
        lat.fire_init(lqfire.fire_params_from_config(cfg, force_tol=force_tol, max_steps=max_steps), q, v, F)
        rep = lat.fire_step(0)
        while rep.status == lqfire.RUNNING:
            rep = lat.fire_step(chunk)
            print(f"[precision-minima] {label}: step {rep.step} maxF {rep.maxF:.3e}", file=sys.stderr, flush=True)
        return rep

    q64 = lat64.set_uniaxial(dirs, lat64.empty())
    r64 = run(lat64, q64, tol, "fp64")
    q32 = lat32.set_uniaxial(dirs, lat32.empty())
    r32 = run(lat32, q32, fp32_tol, "fp32")
    qp = q32.double().contiguous()
    del q32
    lat32.close()
    rp = run(lat64, qp, tol, "fp32 + fp64 polish")
    e64, ep = lat64.energy(q64)["total"], lat64.energy(qp)["total"]
    dq = (qp - q64).abs().max().item()
    de = abs(ep - e64) / abs(e64)
    lat64.close()
    return {"workload": f"colloid_slab{n}", "start": "uniform director along x, S = S0",
            "fp64": {"steps": r64.step, "status": int(r64.status), "maxF": r64.maxF, "energy": e64},
            "fp32_form": {"fp32_steps": r32.step, "fp32_status": int(r32.status), "fp32_maxF": r32.maxF,
                          "polish_steps": rp.step, "status": int(rp.status), "maxF": rp.maxF, "energy": ep},
            "both_converged": r64.status == lqfire.CONVERGED and rp.status == lqfire.CONVERGED,
            "rel_energy_err": de, "max_abs_dQ": dq,
            "pass_energy_1e-6": de <= 1e-6, "pass_dQ_1e-5": dq < 1e-5,
            "seconds": time.perf_counter() - t0}


def precision_leg(cfg, steps=2000, polish=200):
    """The FP32 form against the FP64 path on the same schedule: `steps` FIRE
    steps, then a fresh FIRE start (v = 0, dt0) for `polish` steps in FP64.
    The FP32 run does its first part with an FP32 state and FP64 reductions;
    the FP64 run does both parts in FP64; so precision is the only
    difference.  Two starts: a uniform director (a smooth relaxation, where
    the difference measures rounding) and the workload's random directors
    (a coarsening defect tangle, where small differences grow and the two
    runs part ways).  The FP64 GPU path stands in for the oracle on the
    whole schedule (the oracle needs seconds per step at this size; the GPU
    path matches its per-step forces to 1e-10 on smaller boxes); at the end
    of each FP64 run the oracle evaluates the force of the reference state
    at sampled sites, which pins the reference at full size."""
    import numpy as np
    import torch

    import oracle
    from paper_1911_07045_amd import lqfire, synth

    p = oracle.Problem(cfg["shape"], cfg["periodic"], L1=cfg["L1"], L2=cfg["L2"], L3=cfg["L3"],
                       objects=cfg["objects"])
    rng = np.random.default_rng(20191115)
    bnd = np.flatnonzero(p.types.reshape(-1) == 1)
    sites = np.unique(np.concatenate([rng.choice(p.N, 1000, replace=False),
                                      rng.choice(bnd, min(1000, len(bnd)), replace=False)]))

    nx, ny, nz = cfg["shape"]
    N = nx * ny * nz
    t0 = time.perf_counter()
    lat32 = lqfire.lattice_from_config(cfg, prec="f32")
    lat64 = lqfire.lattice_from_config(cfg, prec="f64")

    def fire(lat, q, n):
        v, F = lat.empty(), lat.empty()
        lat.fire_init(lqfire.fire_params_from_config(cfg, force_tol=0.0, max_steps=n), q, v, F)
        return lat.fire_step(n)

    out = {"schedule": f"{steps} FIRE steps, then {polish} FP64 steps from a fresh FIRE start",
           "reference": "FP64 GPU path on the same schedule"}
    for start in ("uniform", "random"):
        if start == "uniform":
            dirs = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
            dirs[:N] = 1.0
        else:
            dirs = torch.from_numpy(np.ascontiguousarray(synth.random_directors(cfg["dir_seed"], N))).cuda()
        q32 = lat32.set_uniaxial(dirs, lat32.empty())
        fire(lat32, q32, steps)
        q64 = lat64.set_uniaxial(dirs, lat64.empty())
        fire(lat64, q64, steps)
        d1 = (q32.double() - q64).abs().max().item()
        e1 = abs(lat32.energy(q32)["total"] - lat64.energy(q64)["total"]) / abs(lat64.energy(q64)["total"])
        qp = q32.double().contiguous()
        del q32
        rp = fire(lat64, qp, polish)
        rr = fire(lat64, q64, polish)
        ep, er = lat64.energy(qp)["total"], lat64.energy(q64)["total"]
        F64 = lat64.compute_forces(q64)
        Fo = p.forces_at(q64.cpu().numpy().reshape(p.field_shape), sites)
        Fg = F64.reshape(5, -1)[:, sites].T.cpu().numpy()
        ref_err = float(np.abs(Fg - Fo).max() / np.abs(Fo).max())
        del F64
        out[start] = {"reference_force_vs_oracle": {"sites": len(sites), "max_rel_err": ref_err},
                      "max_abs_dQ_before_polish": d1, "rel_energy_err_before_polish": e1,
                      "max_abs_dQ_polished": (qp - q64).abs().max().item(),
                      "rel_energy_err_polished": abs(ep - er) / abs(er),
                      "maxF_polished": rp.maxF, "maxF_fp64": rr.maxF, "energy_fp64": er}
        del qp, q64, dirs
    lat32.close()
    lat64.close()
    out["seconds"] = time.perf_counter() - t0
    return out


def serving_leg(n_requests=512, rate=20.0):
    """The continuous-batching server on a Poisson stream of small boxes."""
    import torch

    from paper_1911_07045_amd import serve, synth

    reqs = synth.serving_stream(n_requests=n_requests, rate=rate)
    srv = serve.Server(max_members=64, chunk=50, polish_steps=2000, fp32_floor=1e-4, stall_steps=1000,
                       noise_frac=0.3)
    results = srv.run(reqs, realtime=True)
    out = serve.summarize(results, srv.wall_s, srv.busy_s)
    # a solve is a request that reached its force tolerance
    out["solves_per_s"] = out["converged"].get("per_s", 0.0)
    out["stall_checks"] = srv.noise_checks
    out.update({"stream": f"{n_requests} requests, Poisson {rate}/s, side log-U[16,64], one colloid, "
                          f"W_RP log-U[0.1,10], tol 1e-5 or 5000 steps, FP32 with FP64 reductions; a "
                          f"request whose max|F| plateaus below {srv.fp32_floor:g} is checked (FP64 force of "
                          f"its FP32 state) and, when FP32 rounding makes up at least {srv.noise_frac:g} of its "
                          f"force, continues with an FP64 polish of at most {srv.polish_steps} steps",
                "max_members": 64, "chunk_steps": 50,
                "hbm_budget_GB": srv.budget / 1e9})
    torch.cuda.synchronize()
    return out


COPY_BYTES = 1 << 30


def traffic_file(workload_name, dtype):
    """The committed counter summary of the step kernel on one workload."""
    return os.path.join(ROOT, "profiles", f"k_march_fire_{dtype}_{workload_name}_hbm.txt")


TRAFFIC_FILE = traffic_file("multi_colloid256", "f32")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1911_07045_amd", "csrc", f) for f in ("kernels.hip", "lq_internal.h")]


def kernel_source_hash():
    """sha256 of the kernel sources with comments and whitespace removed, so
    that only a change of the code itself invalidates a counter summary."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def read_summary(path):
    """key: value lines of a committed profile summary."""
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals


def measured_traffic(workload_name, dtype="f32"):
    """HBM bytes per step-kernel launch from the committed counter summary
    of this workload and state type (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy's reading), or None when there is none or the kernel source
    has changed since the counters were taken."""
    path = traffic_file(workload_name, dtype)
    if not os.path.exists(path):
        return None
    vals = read_summary(path)
    if vals.get("workload") != workload_name or vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(reps=5):
    """Plain device copies of COPY_BYTES each (the library's streaming copy,
    16 bytes per lane).  Under rocprofv3 --pmc FETCH_SIZE (or WRITE_SIZE) the
    per-dispatch counter of these copies, against the known COPY_BYTES read
    and written, gives the factor that turns the counter into HBM bytes."""
    import torch

    from paper_1911_07045_amd import lqfire

    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        lqfire.stream_copy([src], [dst], width=16)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "reps": reps,
                      "kernel": "k_stream_copy<16>"}), flush=True)


def copy_ceiling(n=256, fields=15, iters=40, prec="f32"):
    """Streaming ceiling for the step's traffic: the library's hand-written
    copy kernel (lq_stream_copy, non-temporal stores like the step kernel's)
    moving 15 SoA fields of n^3 values (in -> out), the 2 x 15 streams a
    FIRE step reads and writes, timed with HIP events.  Three ways:
      - all 15 streams in one kernel, one FP32 value per lane per access:
        the step kernel's own access pattern;
      - all 15 streams in one kernel, 8 or 16 bytes per lane per access;
      - one stream per launch, 16 bytes per lane (the fastest plain copy of
        these bytes found).
    TB/s count read plus written bytes; TB_per_s is the fastest of the three."""
    import torch

    from paper_1911_07045_amd import lqfire

    N = n ** 3
    dtype = torch.float32 if prec == "f32" else torch.float64
    src = [torch.full((N,), float(i + 1), dtype=dtype, device="cuda") for i in range(fields)]
    dst = [torch.empty_like(x) for x in src]
    nbytes = 2.0 * fields * src[0].element_size() * N
    out = {"kernel": "k_stream_copy", "fields": fields, "sites": N, "dtype": prec,
           "store_policy": "non-temporal, as the step kernel's stores"}

    def all_streams(width):
        lqfire.stream_copy(src, dst, width=width)

    def one_by_one(width):
        for a, b in zip(src, dst):
            lqfire.stream_copy([a], [b], width=width)

    for name, fn, width in (("together_width4", all_streams, 4), ("together_width8", all_streams, 8),
                            ("together_width16", all_streams, 16),
                            ("one_stream_per_launch_width16", one_by_one, 16)):
        for x in dst:
            x.zero_()
        for _ in range(3):
            fn(width)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(src, dst))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            fn(width)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / iters
        tbs = nbytes / (ms * 1e-3) / 1e12
        out[name] = {"ms_per_pass": ms, "TB_per_s": tbs, "frac_hbm_peak": tbs * 1e3 / HBM_PEAK_GBS}
    out["TB_per_s"] = max(out[k]["TB_per_s"] for k in ("together_width4", "together_width8", "together_width16",
                                                       "one_stream_per_launch_width16"))
    out["same_pattern_TB_per_s"] = out["together_width4"]["TB_per_s"]
    return out


def dispatch_gaps(trace_csv, kernel="k_march_batch", round_trip_ns=200000):
    """Idle time between consecutive dispatches of the batched step kernel in
    a rocprofv3 kernel trace (CSV).  Dispatches closer than round_trip_ns
    belong to one lq_batch_step call (launches queued back to back); a longer
    gap is the host's admission and retirement between calls.  Returns the
    busy time of the step kernels, the idle time between back-to-back
    dispatches, and their ratio."""
    import csv

    rows = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    steps = [(a, b) for a, b, n in rows if kernel in n]
    busy = sum(b - a for a, b in steps)
    gaps_in, gaps_out, n_in = 0, 0, 0
    prev_end = None
    for a, b, n in rows:
        if prev_end is not None and kernel in n:
            g = max(a - prev_end, 0)
            if g < round_trip_ns:
                gaps_in += g
                n_in += 1
            else:
                gaps_out += g
        prev_end = b if prev_end is None else max(prev_end, b)
    return {"kernel": kernel, "dispatches": len(steps), "busy_ms": busy / 1e6,
            "idle_back_to_back_ms": gaps_in / 1e6, "back_to_back_gaps": n_in,
            "mean_gap_us": gaps_in / max(n_in, 1) / 1e3,
            "idle_frac_of_busy": gaps_in / max(busy, 1),
            "idle_between_calls_ms": gaps_out / 1e6, "round_trip_threshold_us": round_trip_ns / 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="multi_colloid256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of an FP32 workload")
    ap.add_argument("--serving-only", action="store_true", help="only run the serving stream")
    ap.add_argument("--dispatch-gaps", metavar="KERNEL_TRACE_CSV",
                    help="only analyse a rocprofv3 kernel trace: idle time between batched step dispatches")
    ap.add_argument("--precision-minima", action="store_true",
                    help="only compare the converged minima of the FP32 form and FP64 on the 128^3 colloid slab")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--no-minimizers", action="store_true",
                    help="skip the gradient-descent / Nesterov step timings")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle on several workloads, all cores and one core")
    ap.add_argument("--oracle-child", nargs=2, metavar=("WORKLOAD", "STEPS"), help=argparse.SUPPRESS)
    ap.add_argument("--copy-ceiling", action="store_true",
                    help="only time plain device copies of the step's 15 fields (streaming ceiling)")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="print the hash of the kernel sources that a counter summary records")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of a known size (HBM counter scale)")
    ap.add_argument("--convergence", action="store_true",
                    help="only compare FIRE with tuned gradient descent and Nesterov on the 256^3 bulk box")
    ap.add_argument("--step-scaling", action="store_true",
                    help="only count FIRE steps to a force tolerance against the box side (bulk, one colloid)")
    args = ap.parse_args()
    if args.kernel_hash:
        print(kernel_source_hash())
        return
    if args.oracle_child:
        print(json.dumps(oracle_steps(args.oracle_child[0], int(args.oracle_child[1]))), flush=True)
        return
    if args.oracle_timing:
        import platform
        cpu = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        print(json.dumps({"oracle_timing": oracle_timing(), "cpu": cpu, "nproc": os.cpu_count(),
                          "host": platform.node()}), flush=True)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.copy_ceiling:
        print(json.dumps({"copy_ceiling": copy_ceiling()}), flush=True)
        return
    if args.convergence:
        print(json.dumps({"convergence": convergence_leg()}), flush=True)
        return
    if args.dispatch_gaps:
        print(json.dumps({"dispatch_gaps": dispatch_gaps(args.dispatch_gaps)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_leg(args.serving_requests)}), flush=True)
        return
    if args.precision_minima:
        print(json.dumps({"precision_minima": precision_minima()}), flush=True)
        return
    if args.step_scaling:
        print(json.dumps({"step_scaling": step_scaling_leg()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs one GPU only: the hot path here is a single-GPU lattice "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    cfg = workload(args.workload)
    print(f"[bench] {cfg['name']} {cfg['shape']} {cfg['prec']}: {args.warmup} warmup + "
          f"{args.steps} timed steps", file=sys.stderr, flush=True)
    g = gpu_leg(cfg, args.steps, args.warmup)
    value = g["N"] * args.steps / g["wall_s"]
    alg_bytes = g["bytes_per_site"] * g["N"]
    achieved = alg_bytes / (g["kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * g["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfg["prec"],
        "data": "synthetic",
        "config": describe(cfg),
        "simulated_site_updates_per_s": g["n_sim"] * args.steps / g["wall_s"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg["name"], cfg["prec"]),
                     "kernel": "k_march<fused FIRE step>", "kernel_ms": g["kernel_ms"],
                     "algorithmic_bytes_per_launch": alg_bytes},
        "energy_start_end": [g["E0"], g["E1"]],
    }
    if cfg["prec"] == "f32" and cfg["shape"] == (256, 256, 256):
        # context for the roofline: plain copies of the same 15 fields
        cc = copy_ceiling()
        out["roofline"]["copy_ceiling_GBs"] = cc["TB_per_s"] * 1e3
        out["roofline"]["frac_of_copy_ceiling"] = achieved / (cc["TB_per_s"] * 1e3)
        out["roofline"]["copy_same_pattern_GBs"] = cc["same_pattern_TB_per_s"] * 1e3
        out["roofline"]["frac_of_copy_same_pattern"] = achieved / (cc["same_pattern_TB_per_s"] * 1e3)
    if cfg["prec"] == "f32" and not args.no_fp64:
        # the same workload at the paper's precision (FP64 state), same steps
        print("[bench] the same workload in FP64", file=sys.stderr, flush=True)
        c64 = dict(cfg, prec="f64")
        g64 = gpu_leg(c64, args.steps, args.warmup)
        ach64 = g64["bytes_per_site"] * g64["N"] / (g64["kernel_ms"] * 1e-3) / 1e9
        out["fp64"] = {
            "value": g64["N"] * args.steps / g64["wall_s"], "unit": "site-updates/s",
            "ms_per_step": 1e3 * g64["wall_s"] / args.steps, "dtype": "f64",
            "roofline": {"bound": "hbm", "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach64 / HBM_PEAK_GBS, "traffic": measured_traffic(cfg["name"], "f64"),
                         "kernel": "k_march<fused FIRE step>", "kernel_ms": g64["kernel_ms"],
                         "algorithmic_bytes_per_launch": g64["bytes_per_site"] * g64["N"]},
            "energy_start_end": [g64["E0"], g64["E1"]]}
    if not args.no_precision and cfg["prec"] == "f32":
        print("[bench] precision form", file=sys.stderr, flush=True)
        out["precision"] = {cfg["name"]: precision_leg(cfg)}
        if cfg["name"] == "multi_colloid256":
            # the 128^3 colloid slab against the oracle's stored FP64 schedule
            print("[bench] precision form against the stored oracle schedule", file=sys.stderr, flush=True)
            out["precision"]["colloid_slab128"] = precision_vs_oracle()
            print("[bench] precision form at converged minima", file=sys.stderr, flush=True)
            out["precision"]["colloid_slab128_minima"] = precision_minima()
    if not args.no_minimizers:
        print("[bench] gradient descent / Nesterov steps", file=sys.stderr, flush=True)
        out["minimizers"] = minimizer_leg(cfg)
    if not args.no_serving:
        print("[bench] serving stream", file=sys.stderr, flush=True)
        out["serving"] = serving_leg(args.serving_requests)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_leg(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
