"""Serving form: batched FIRE over many small lattices.

Each request's result must be the same alone and in the mix: the batched
launch keeps a controller, block-ordered FP64 partials and a stop test per
member, so the comparison is bit for bit.
"""
import numpy as np
import pytest

from paper_1911_07045_amd import lqfire, serve, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lqfire.lib()


def _bound(req, prec):
    lat = lqfire.Lattice(req["shape"], req.get("periodic", (True,) * 3), prec, L1=req["L1"],
                         L2=req.get("L2", 0.0), L3=req.get("L3", 0.0))
    if req.get("objects"):
        lat.set_boundaries(req["objects"])
    dirs = torch.from_numpy(np.ascontiguousarray(synth.random_directors(req["dir_seed"], lat.N))).cuda()
    q = lat.set_uniaxial(dirs, lat.empty())
    v, F = lat.empty(), lat.empty()
    lat.fire_init(lqfire.fire_params_from_config(req), q, v, F)
    return lat, q, v, F


def _reqs(n, seed, **kw):
    return synth.serving_stream(n_requests=n, seed=seed, side_lo=16, side_hi=26, **kw)


@pytest.mark.parametrize("prec,l23", [("f32", False), ("f64", True)])
def test_batch_equals_alone_bitwise(prec, l23):
    say(f"[batch] alone vs batch {prec} l23={l23}")
    reqs = _reqs(5, 21, force_tol=0.0, max_steps=10 ** 6)
    if l23:
        for r in reqs:
            r["L2"], r["L3"] = 1.16, 0.7
    alone = []
    for r in reqs:
        lat, q, v, F = _bound(r, prec)
        reps = [lat.fire_step(n) for n in (7, 30, 13)]
        alone.append((q.cpu(), v.cpu(), F.cpu(), reps[-1].as_dict()))
        lat.close()
    b = lqfire.Batch(8)
    held = []
    for r in reqs:
        lat, q, v, F = _bound(r, prec)
        b.add(lat)
        held.append((lat, q, v, F))
    reps = None
    for n in (20, 25, 5):
        reps = b.step(n)
    for (lat, q, v, F), (qa, va, Fa, ra), rep in zip(held, alone, reps):
        assert torch.equal(q.cpu(), qa) and torch.equal(v.cpu(), va) and torch.equal(F.cpu(), Fa)
        assert rep.as_dict() == ra


def test_members_join_and_leave_mid_run():
    """A member added after others have run, and one removed early, still
    follow their solo trajectories."""
    say("[batch] join/leave")
    reqs = _reqs(3, 22, force_tol=0.0, max_steps=10 ** 6)
    solo = []
    for r, n in zip(reqs, (40, 25, 30)):
        lat, q, v, F = _bound(r, "f32")
        lat.fire_step(n)
        solo.append((q.cpu(), v.cpu(), F.cpu()))
        lat.close()
    b = lqfire.Batch(4)
    m = [_bound(r, "f32") for r in reqs]
    b.add(m[0][0])
    b.add(m[1][0])
    b.step(15)           # 0: 15, 1: 15
    b.add(m[2][0])
    b.step(10)           # 0: 25, 1: 25, 2: 10
    b.remove(m[1][0])
    b.step(15)           # 0: 40, 2: 25
    m[2][0].fire_step(5)  # alone again: 2: 30
    for (lat, q, v, F), (qs, vs, Fs) in zip(m, solo):
        assert torch.equal(q.cpu(), qs) and torch.equal(v.cpu(), vs) and torch.equal(F.cpu(), Fs)


def test_server_results_equal_alone_and_budget_holds():
    """Requests served by the continuous-batching loop converge to the same
    states, bit for bit, as when minimized one at a time; the HBM budget is
    never exceeded."""
    say("[serve] stream of 8 vs alone")
    reqs = _reqs(8, 23, force_tol=1e-3, max_steps=3000)
    solo = {}
    for r in reqs:
        lat, q, v, F = _bound(r, "f32")
        rep = lat.fire_step(3000)
        solo[r["id"]] = (q.cpu(), rep.step, rep.status)
        lat.close()
    sizes = sorted(serve.request_bytes(r) for r in reqs)
    budget = sizes[-1] + sizes[-2] + 1   # at most two large requests at once
    srv = serve.Server(max_members=3, hbm_budget=budget, chunk=40, keep_states=True, polish_steps=0)
    peak = []
    orig_admit = srv.admit

    def admit(req, now):
        out = orig_admit(req, now)
        peak.append(srv.used)
        return out
    srv.admit = admit
    results = srv.run(reqs, realtime=False)
    assert len(results) == len(reqs)
    assert max(peak) <= budget
    for res in results:
        qs, steps, status = solo[res.id]
        assert res.steps == steps and res.status == status
        assert torch.equal(srv.states[res.id][0], qs)


def test_batch_mixing_narrow_and_wide_tiles_equals_alone():
    """A box narrower than one wide tile runs on narrow tiles, a wide box on
    wide ones; in one batch the two groups go in separate launches and each
    member still follows its solo trajectory bit for bit."""
    say("[batch] narrow + wide members")
    reqs = _reqs(2, 24, force_tol=0.0, max_steps=10 ** 6)
    reqs[1]["shape"] = (136, 20, 18)
    reqs[1]["objects"] = [dict(kind="sphere", center=(60.0, 9.5, 8.5), radius=4.0, law="rp", W=3.0,
                               dir="normal")]
    alone = []
    for r in reqs:
        lat, q, v, F = _bound(r, "f32")
        lat.fire_step(37)
        alone.append((q.cpu(), v.cpu(), F.cpu()))
        lat.close()
    b = lqfire.Batch(4)
    held = [_bound(r, "f32") for r in reqs]
    for h in held[::-1]:
        b.add(h[0])
    b.step(20)
    b.step(17)
    for (lat, q, v, F), (qa, va, Fa) in zip(held, alone):
        assert torch.equal(q.cpu(), qa) and torch.equal(v.cpu(), va) and torch.equal(F.cpu(), Fa)


def test_destroying_a_member_leaves_its_batch():
    """Closing a member lattice removes it from its batch (the batch keeps
    stepping the others, which still follow their solo trajectories); a
    lattice belongs to one batch at a time; closing a batch leaves its
    lattices usable."""
    say("[batch] member destroyed while in a batch")
    reqs = _reqs(3, 25, force_tol=0.0, max_steps=10 ** 6)
    alone = []
    for r in reqs[1:]:
        lat, q, v, F = _bound(r, "f32")
        lat.fire_step(25)
        alone.append((q.cpu(), v.cpu(), F.cpu()))
        lat.close()
    held = [_bound(r, "f32") for r in reqs]
    b = lqfire.Batch(4)
    for h in held:
        b.add(h[0])
    other = lqfire.Batch(2)
    with pytest.raises(lqfire.LQError):
        other.add(held[1][0])
    b.step(10)
    held[0][0].close()
    assert len(b) == 2 and lqfire.lib().lq_batch_size(b.h) == 2
    reps = b.step(15)
    assert len(reps) == 2
    for (lat, q, v, F), (qa, va, Fa) in zip(held[1:], alone):
        assert torch.equal(q.cpu(), qa) and torch.equal(v.cpu(), va) and torch.equal(F.cpu(), Fa)
    b.close()
    other.add(held[1][0])
    assert len(other.step(1)) == 1
    other.close()
    rep = held[2][0].fire_step(1)
    assert rep.step == 26
    for h in held[1:]:
        h[0].close()


def test_server_polishes_stalled_fp32_requests_in_fp64():
    """An FP32 request that reaches its step limit below the FP32 floor, and
    whose force the rounding check attributes to rounding, continues from its
    FP32 state in FP64 (a fresh FIRE start, at most polish_steps steps) in
    the server's second batch: the served result equals that two-stage run
    done alone, bit for bit.  (The floor is raised here so that 200 steps end
    below it, and the check is forced with noise_frac = 0; with the default
    fraction the check finds the force far above FP32 rounding and reports
    the requests as capped.)"""
    say("[serve] FP64 polish of stalled FP32 requests")
    reqs = _reqs(3, 26, force_tol=1e-7, max_steps=200)
    solo = {}
    for r in reqs:
        lat, q, v, F = _bound(r, "f32")
        rep = lat.fire_step(200)
        assert rep.status == lqfire.MAX_STEPS and rep.maxF < 100.0
        lat64 = lqfire.lattice_from_config(r, prec="f64")
        q64 = q.double().contiguous()
        v64, F64 = lat64.empty(), lat64.empty()
        lat64.fire_init(lqfire.fire_params_from_config(r, max_steps=150), q64, v64, F64)
        rep64 = lat64.fire_step(150)
        solo[r["id"]] = (q64.cpu(), rep64.step, rep64.status)
        lat.close()
        lat64.close()
    srv = serve.Server(max_members=2, chunk=40, keep_states=True, polish_steps=150, fp32_floor=100.0,
                       stall_steps=None, noise_frac=0.0)
    results = srv.run(reqs, realtime=False)
    assert len(results) == 3
    for res in results:
        q64, steps, status = solo[res.id]
        assert res.polished and res.steps == 200
        assert res.polish_steps == steps and res.status == status
        assert torch.equal(srv.states[res.id][0], q64)
    s = serve.summarize(results, srv.wall_s, srv.busy_s)
    assert s["polished"]["count"] == 3 and srv.noise_checks == 3
    # after 200 steps from a random start the force is far above FP32
    # rounding: the check finds no stall and the requests are capped
    srv = serve.Server(max_members=2, chunk=40, polish_steps=150, fp32_floor=100.0, stall_steps=None)
    results = srv.run(reqs, realtime=False)
    assert srv.noise_checks == 3
    assert all(not r.polished and r.status == lqfire.MAX_STEPS and r.steps == 200 for r in results)


def test_server_refuses_a_request_beyond_its_budget():
    """A request that needs more device memory than the whole budget is
    refused at arrival (the loop does not wait for it), and the others are
    served."""
    say("[serve] refusal beyond the budget")
    reqs = _reqs(3, 27, force_tol=1e-3, max_steps=100)
    reqs[1]["shape"] = (64, 64, 64)
    budget = max(serve.request_bytes(r, "f64") for i, r in enumerate(reqs) if i != 1)
    srv = serve.Server(max_members=2, hbm_budget=budget, chunk=50)
    results = srv.run(reqs, realtime=False)
    by_id = {r.id: r for r in results}
    assert by_id[1].status == serve.REFUSED
    assert by_id[0].status != serve.REFUSED and by_id[2].status != serve.REFUSED
    s = serve.summarize(results, srv.wall_s, srv.busy_s)
    assert s["refused"] == 1 and s["requests"] == 3
