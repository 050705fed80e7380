"""The FP32 form against the FP64 oracle, on every kernel variant the serving
loop and the large workloads run.

The FP32 form keeps q, v and F in FP32 and the FIRE reductions and
controller in FP64 (Algorithm 1).  The bounds follow from FP32 arithmetic
(unit roundoff u = 2^-24):
  - one step rounds q's update chain (steering, half kick, drift) about
    c = 4 times, so k steps move q by at most k c u max|q|, times the growth
    G >= 1 that the dynamics give such a perturbation over those steps;
  - a force is a linear stencil in q plus the bulk and anchoring terms, whose
    infinity norm is at most |H| = 36 (L1 + L2 + L3) (the metric's row sum 3
    times the Laplacian's 12) + 12 W (the largest Nobili-Durand strength,
    twice for a site touching two objects) + 4 (the bulk curvature near S0),
    so the state difference moves F by at most |H| times it;
  - one evaluation sums about n = 30 terms whose magnitudes add up to at most
    |H| max|q|, so it is off by at most n u |H| max|q|.
Hence max|dq| <= G k c u max|q| and max|dF| <= |H| max|dq|_bound +
n u |H| max|q|.  G is measured on the oracle alone: a second oracle run from
the same state with q and v perturbed by one FP32 rounding per value, over
the same steps, gives G = max(1, final max|dq| / initial max|dq|).  It is
near 1 while the state relaxes smoothly and grows to ~100 over the steps
around a FIRE restart, where the velocity is largest.

The per-step checks run over chunks of k = 10 steps from a common state (the
oracle's q and v rounded to FP32, exact in FP64, with the oracle's
controller; the GPU continues through lq_fire_init's resume path); after
each chunk the controller's decisions also agree exactly (step, n_pos and
restarts, and so dt and alpha, which change only through them).  The served
stream is checked over its whole run of 60 steps, with G the largest growth
from a perturbation at any 10-step mark to the end.

Kernels covered: the narrow FP32 one-constant tiles of small boxes run
through lq_batch_step (the serving kernel) and through the server itself;
the wide FP32 L2/L3 tiles of the patterned-wall workload, through
lq_fire_step and through a batch.
"""
import ctypes

import numpy as np
import pytest

from paper_1911_07045_amd import lqfire, serve, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
CHUNK = 10


def h_inf(cfg, S0=0.5328646154690171):
    """Infinity-norm bound of the force's dependence on q (see the module
    docstring)."""
    w = 0.0
    for o in cfg.get("objects", ()):
        W = abs(o["W"])
        w = max(w, W if o.get("law", "nd") == "nd" else W / (9.0 * S0 * S0))
    return 36.0 * (cfg["L1"] + cfg.get("L2", 0.0) + cfg.get("L3", 0.0)) + 12.0 * w + 4.0


def _clone(ora, st):
    c = ora.FireState()
    ctypes.memmove(ctypes.addressof(c), ctypes.addressof(st), ctypes.sizeof(st))
    return c


def growth(ora, p, prm, st, q, v, k, tag):
    """G over k steps: the oracle from (q, v) and from (q, v) perturbed by one
    FP32 rounding per value, max(1, final max|dq| / initial max|dq|)."""
    xi = synth.uniform(17, tag, 0, 2 * q.size) * 2.0 - 1.0
    qa, va = q.copy(), v.copy()
    qb = q * (1.0 + U32 * xi[:q.size].reshape(q.shape))
    vb = v * (1.0 + U32 * xi[q.size:].reshape(v.shape))
    d0 = np.abs(qb - qa).max()
    sa, sb = _clone(ora, st), _clone(ora, st)
    Fa, Fb = p.forces(qa), p.forces(qb)
    p.fire_steps(prm, sa, qa, va, Fa, k)
    p.fire_steps(prm, sb, qb, vb, Fb, k)
    return max(1.0, np.abs(qb - qa).max() / d0) if d0 > 0 else 1.0


def fp32_bounds(cfg, qmax, k, G=1.0):
    """(max|dq|, max|dF|) bounds after k FP32 steps from a common state."""
    H = h_inf(cfg)
    bq = max(G, 1.0) * k * 4.0 * U32 * max(qmax, 1e-30)
    return bq, H * bq + 30.0 * U32 * H * qmax


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lqfire.lib()


def _problem(ora, cfg):
    return ora.Problem(cfg["shape"], cfg["periodic"], L1=cfg["L1"], L2=cfg.get("L2", 0.0),
                       L3=cfg.get("L3", 0.0), objects=cfg["objects"])


class _Member:
    """One FP32 lattice on the GPU beside its FP64 oracle twin."""

    def __init__(self, ora, cfg):
        self.ora = ora
        self.cfg = cfg
        self.G = 1.0
        self.p = _problem(ora, cfg)
        self.lat = lqfire.lattice_from_config(cfg, prec="f32")
        dirs = synth.random_directors(cfg["dir_seed"], self.p.N)
        q0 = self.p.uniaxial(dirs).astype(np.float32)
        self.q = self.lat.set_uniaxial(torch.from_numpy(np.ascontiguousarray(dirs)).cuda(), self.lat.empty())
        torch.cuda.synchronize()
        assert np.array_equal(self.q.cpu().numpy(), q0)
        self.v, self.F = self.lat.empty(), self.lat.empty()
        self.lat.fire_init(lqfire.fire_params_from_config(cfg, force_tol=0.0, max_steps=10 ** 6),
                           self.q, self.v, self.F)
        self.prm = ora.fire_params(dt0=cfg["fire"]["dt0"], dt_max=cfg["fire"]["dt_max"],
                                   alpha0=cfg["fire"]["alpha0"], force_tol=0.0, max_steps=10 ** 6)
        self.st, self.qo, self.vo, self.Fo = self.p.fire_init(self.prm, q0.astype(np.float64))
        self.worst = 0.0

    def oracle_steps(self, k):
        self.G = growth(self.ora, self.p, self.prm, self.st, self.qo, self.vo, k, self.st.step)
        self.p.fire_steps(self.prm, self.st, self.qo, self.vo, self.Fo, k)

    def resync(self, batch=None):
        """Both sides continue from the oracle's state rounded to FP32."""
        self.qo[...] = self.qo.astype(np.float32)
        self.vo[...] = self.vo.astype(np.float32)
        self.Fo[...] = self.p.forces(self.qo)
        if batch is not None:
            batch.remove(self.lat)
        self.q.copy_(torch.from_numpy(self.qo.astype(np.float32)).reshape(self.q.shape))
        self.v.copy_(torch.from_numpy(self.vo.astype(np.float32)).reshape(self.v.shape))
        st = self.st
        rep = lqfire.FireReport(step=st.step, n_pos=st.n_pos, restarts=st.restarts, dt=st.dt, alpha=st.alpha)
        self.lat.fire_init(lqfire.fire_params_from_config(self.cfg, force_tol=0.0, max_steps=10 ** 6),
                           self.q, self.v, self.F, resume=rep)
        if batch is not None:
            batch.add(self.lat)

    def check(self, rep, k=CHUNK):
        st = self.st
        assert (rep.step, rep.n_pos, rep.restarts) == (st.step, st.n_pos, st.restarts)
        assert rep.dt == st.dt and rep.alpha == st.alpha
        F = self.F.cpu().numpy().astype(np.float64)
        q = self.q.cpu().numpy().astype(np.float64)
        dF = np.abs(F - self.Fo).max()
        dq = np.abs(q - self.qo).max()
        bq, bF = fp32_bounds(self.cfg, np.abs(self.qo).max(), k, self.G)
        say(f"    step {st.step}: |dF| {dF:.2e} (bound {bF:.2e}), |dq| {dq:.2e} (bound {bq:.2e}), "
            f"G {self.G:.1f}, max|F| {np.abs(self.Fo).max():.2e}")
        self.worst = max(self.worst, dF / bF)
        assert dF <= bF, f"step {st.step}: |dF| {dF:.3e} > {bF:.3e}"
        assert dq <= bq, f"step {st.step}: |dq| {dq:.3e} > {bq:.3e}"

def _serving_box(n, radius, W, seed):
    c = (n - 1) / 2.0
    return dict(name=f"box{n}", shape=(n, n, n), periodic=(True, True, True), L1=2.32, L2=0.0, L3=0.0,
                objects=[dict(kind="sphere", center=(c, c, c), radius=radius, law="rp", W=W, dir="normal")],
                dir_seed=seed, prec="f32", fire=dict(synth.FIRE))


def _patterned_box(nx=64, ny=16, nz=40, seed=31):
    """The patterned-wall workload's geometry on a small box: object plane
    z = 0 with a radial in-plane director around a 2 x 1 array of centres
    (Rapini-Papoular W = 2), homeotropic object plane z = nz - 1
    (Rapini-Papoular W = 2), L1 = 2.32, L2 = L3 = 1.16."""
    objs = [dict(kind="patterned_wall", axis=2, plane=0, law="rp", W=2.0, pitch=(32, 16),
                 offset=(15.5, 7.5), count=(2, 1)),
            dict(kind="wall", axis=2, plane=nz - 1, law="rp", W=2.0, dir="normal")]
    return dict(name="patterned_small", shape=(nx, ny, nz), periodic=(True, True, True), L1=2.32,
                L2=1.16, L3=1.16, objects=objs, dir_seed=seed, prec="f32", fire=dict(synth.FIRE))


def test_fp32_batch_narrow_tiles_serving_boxes(ora):
    """Two serving-sized boxes (24^3 with a W = 5 colloid, 18^3 with a
    W = 0.3 colloid) stepped together by lq_batch_step on narrow FP32 tiles
    follow the FP64 oracle over 80 steps (8 chunks from a common state)."""
    say("[fp32] batch of 24^3 + 18^3 serving boxes, 80 steps")
    mem = [_Member(ora, _serving_box(24, 6.0, 5.0, 41)), _Member(ora, _serving_box(18, 3.5, 0.3, 42))]
    assert all(m.lat.N < 64 ** 3 for m in mem)
    b = lqfire.Batch(4)
    for m in mem:
        b.add(m.lat)
    for _ in range(8):
        reps = b.step(10)
        for m, rep in zip(mem, reps):
            m.oracle_steps(10)
            m.check(rep)
        for m in mem:
            m.resync(b)
    say("  worst |dF| / bound " + ", ".join(f"{m.worst:.2e}" for m in mem))
    b.close()


@pytest.mark.parametrize("via", ["fire_step", "batch"])
def test_fp32_wide_l23_patterned_wall(ora, via):
    """The wide FP32 L2/L3 tiles (64 x 8) of the patterned-wall workload, with
    anchored sites on both walls and bulk tiles in between, follow the FP64
    oracle over 100 steps (10 chunks from a common state), through
    lq_fire_step and through a batch."""
    say(f"[fp32] wide L2/L3 patterned wall 64x16x40 via {via}, 100 steps")
    m = _Member(ora, _patterned_box())
    b = None
    if via == "batch":
        b = lqfire.Batch(2)
        b.add(m.lat)
    for _ in range(10):
        rep = b.step(10)[0] if b else m.lat.fire_step(10)
        m.oracle_steps(10)
        m.check(rep)
        m.resync(b)
    say(f"  worst |dF| / bound {m.worst:.2e}")
    if b:
        b.close()


def test_fp32_served_results_match_oracle(ora):
    """Three requests of the serving stream, served by the continuous-batching
    loop for a fixed 60 steps each, end where the oracle's 60-step run ends:
    q and F within the FP32 bounds for 60 steps (with the perturbation growth
    G that a second oracle run from a perturbed start measures), the energy
    within the first-order bound that the measured q difference gives."""
    say("[fp32] served stream of 3 vs the oracle, 60 steps")
    steps = 60
    reqs = synth.serving_stream(n_requests=3, seed=43, side_lo=16, side_hi=22, force_tol=0.0, max_steps=steps)
    srv = serve.Server(max_members=2, chunk=25, keep_states=True, polish_steps=0)
    results = srv.run(reqs, realtime=False)
    assert sorted(r.id for r in results) == [0, 1, 2]
    for res in results:
        req = reqs[res.id]
        p = _problem(ora, req)
        q0 = p.uniaxial(synth.random_directors(req["dir_seed"], p.N)).astype(np.float32).astype(np.float64)
        prm = ora.fire_params(force_tol=0.0, max_steps=steps)
        st, qo, vo, Fo = p.fire_init(prm, q0)
        # growth of a perturbation at every 10-step mark, carried to the end
        G = 1.0
        for t in range(0, steps, CHUNK):
            G = max(G, growth(ora, p, prm, st, qo, vo, steps - t, t))
            p.fire_steps(prm, st, qo, vo, Fo, CHUNK)
        assert res.steps == st.step == steps
        q, v, F = (t.numpy().astype(np.float64) for t in srv.states[res.id])
        dF = np.abs(F - Fo).max()
        dq = np.abs(q - qo).max()
        bq, bF = fp32_bounds(req, np.abs(qo).max(), steps, G)
        say(f"  request {res.id} {req['shape']}: |dF| {dF:.2e} (bound {bF:.2e}), |dq| {dq:.2e} "
            f"(bound {bq:.2e}), G {G:.2f}")
        assert dF <= bF and dq <= bq
        # E(q) - E(q_o) = -F(q_o).dq + O(|H| |dq|^2) (Cauchy-Schwarz on the
        # first-order term), plus the rounding of two FP64 sums
        e_ora = p.energy(qo)
        dq2 = np.linalg.norm(q - qo)
        bound = np.linalg.norm(Fo) * dq2 + h_inf(req) * dq2 * dq2 + 1e-12 * abs(e_ora)
        say(f"    energy difference {abs(res.energy - e_ora):.3e} (bound {bound:.3e})")
        assert abs(res.energy - e_ora) <= bound
