"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
formulas: they use closed forms, invariances, exact finite differences of a
quartic energy, the paper's worked 5CB numbers, the paper's L <-> K mapping
to Frank-Oseen, brute-force counts, and closed-form FIRE trajectories.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1911_07045_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
A, B, C = -0.172, -2.12, 1.73


def rand_q(p, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    q = scale * rng.standard_normal(p.field_shape)
    q[:, (p.types == 2).reshape(p.field_shape[1:])] = 0.0
    return q


def five_point_forces(p, q, h=1e-2):
    """-dE/dq by the 5-point central difference.  E is a polynomial of degree
    at most 4 in every single component, for which this difference is exact,
    so the only error is rounding."""
    qf = q.reshape(-1).copy()
    g = np.zeros_like(qf)
    for i in range(qf.size):
        vals = []
        for s in (-2, -1, 1, 2):
            t = qf.copy()
            t[i] += s * h
            vals.append(p.energy(t))
        g[i] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    return -g.reshape(q.shape)


# ---------------------------------------------------------------- bulk
def test_S0_solves_the_uniaxial_stationarity(ora):
    """Eq. (S0def) is the nonzero root of d/dS of Eq. (fphaseS):
    3/2 A S + 3/4 B S^2 + 9/4 C S^3 = 0."""
    for (a, b, c) in [(A, B, C), (-1.0, -12.33, 10.06), (-0.3, -1.0, 2.0)]:
        s = ora.S0(a, b, c)
        r = 1.5 * a * s + 0.75 * b * s * s + 2.25 * c * s ** 3
        assert abs(r) < 1e-15 * max(1.0, abs(a * s))
        assert s > 0


def test_paper_5cb_worked_numbers(ora):
    """Sec. III.B: with the 5CB coefficients S0 ~ 0.53, and K = 9 S0^2 L1 / 2
    = 1e-11 N with L1 tilde = 2.32 gives dx ~ 4.5 nm; sec. IV.A quotes 74
    spacings as ~ 330 nm."""
    g = json.load(open(os.path.join(GOLD, "units_5cb.json")))
    s0 = ora.S0(g["A"], g["B"], g["C"])
    assert round(s0, g["S0_quoted_digits"]) == g["S0_quoted"]
    L1 = 2.0 * g["K"] / (9.0 * s0 * s0)
    dx = math.sqrt(L1 / (g["L1_tilde"] * abs(g["A"])))
    assert abs(dx - g["dx_quoted_m"]) < 0.1e-9
    assert abs(g["hedgehog_spacings"] * dx - g["hedgehog_quoted_m"]) < 15e-9
    # the S0 of the dimensionless workload constants is the same number
    assert abs(ora.S0(A, B, C) - s0) < 1e-15


def test_bulk_energy_reduces_to_uniaxial_polynomial(ora):
    """Eq. (fphase) at a uniaxial Q equals Eq. (fphaseS)."""
    rng = np.random.default_rng(3)
    p = ora.Problem((3, 3, 3), L1=0.0)
    for _ in range(6):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        S = rng.uniform(-0.5, 1.0)
        dirs = np.repeat(n[:, None], p.N, axis=1)
        q = p.uniaxial(dirs, S)
        e = p.energy(q) / p.N
        ref = 0.75 * A * S ** 2 + 0.25 * B * S ** 3 + 9.0 / 16.0 * C * S ** 4
        assert abs(e - ref) < 1e-15 * max(1.0, abs(ref)) + 1e-16


def test_well_depth_matches_uniaxial_polynomial_at_S0(ora):
    """Eq. (f0): f0 = f_bulk(S0) < 0 in the nematic phase."""
    s0 = ora.S0(A, B, C)
    f0 = 0.75 * A * s0 ** 2 + 0.25 * B * s0 ** 3 + 9.0 / 16.0 * C * s0 ** 4
    p = ora.Problem((3, 3, 3), L1=2.32)
    q = p.uniaxial(np.repeat(np.array([[0.0], [0.6], [0.8]]), p.N, axis=1))
    assert f0 < 0
    assert abs(p.energy(q) - p.N * f0) < 1e-14 * p.N


# ---------------------------------------------------------------- forces
def test_zero_force_on_uniform_bulk_minimum(ora):
    """A uniform uniaxial state at S0 is stationary: the bulk gradient is
    (A + B S/2 + 3 C S^2 / 2) Q plus an isotropic part that the traceless
    parameterization removes, and the prefactor vanishes at S0."""
    rng = np.random.default_rng(5)
    p = ora.Problem((4, 5, 6), L1=2.32, L2=1.16, L3=0.9)
    for _ in range(4):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        q = p.uniaxial(np.repeat(n[:, None], p.N, axis=1))
        assert np.abs(p.forces(q)).max() < 1e-14


def test_zero_force_with_walls_at_preferred_state(ora):
    """With Nobili-Durand walls whose preferred director is n, the uniform
    state Q = Q0(n) is stationary too (no distortion, no anchoring cost)."""
    objs = [dict(kind="wall", axis=2, plane=0, law="nd", W=0.5, dir=(1.0, 0.0, 0.0)),
            dict(kind="wall", axis=2, plane=5, law="rp", W=3.0, dir=(1.0, 0.0, 0.0))]
    p = ora.Problem((4, 4, 6), L1=2.32, L2=1.16, L3=1.16, objects=objs)
    q = p.uniaxial(np.repeat(np.array([[1.0], [0.0], [0.0]]), p.N, axis=1))
    assert np.abs(p.forces(q)).max() < 1e-14


GEOMETRIES = {
    "periodic_L1": dict(shape=(3, 3, 3), L2=0.0, L3=0.0),
    "periodic_L23": dict(shape=(3, 4, 3), L2=1.3, L3=-0.4),
    "open_x_L23": dict(shape=(4, 3, 5), periodic=(False, True, True), L2=1.16, L3=1.16),
    "z_walls": dict(shape=(3, 3, 5), L2=1.16, L3=0.7, objects=[
        dict(kind="wall", axis=2, plane=0, law="nd", W=0.5, dir=(1.0, 0.0, 0.0)),
        dict(kind="wall", axis=2, plane=4, law="rp", W=2.0, dir="normal")]),
    "sphere": dict(shape=(5, 5, 5), L2=0.8, L3=0.3, objects=[
        dict(kind="sphere", center=(2.1, 2.4, 1.8), radius=1.5, law="rp", W=5.0, dir="normal")]),
    "sandwiched_plane": dict(shape=(3, 4, 3), L2=1.0, L3=0.5, objects=[
        dict(kind="wall", axis=2, plane=0, law="nd", W=0.7, dir=(0.0, 1.0, 0.0)),
        dict(kind="wall", axis=2, plane=2, law="nd", W=0.2, dir="normal")]),
    "patterned_and_records": dict(shape=(4, 4, 4), L2=1.16, L3=1.16, objects=[
        dict(kind="patterned_wall", axis=2, plane=0, law="rp", W=2.0, pitch=(2, 2),
             offset=(0.5, 0.5), count=(2, 2))],
        site_records=[dict(site=21, law="nd", W=0.4, n0=(1.0, 2.0, 2.0)),
                      dict(site=21, law="rp", W=1.0, n0=(0.0, 0.0, 1.0))],
        object_sites=[42, 43]),
}


@pytest.mark.parametrize("name", sorted(GEOMETRIES))
def test_forces_are_the_exact_gradient(ora, name):
    """Sec. III.B: forces are -dE/dq of the discrete energy itself."""
    g = dict(GEOMETRIES[name])
    shape = g.pop("shape")
    p = ora.Problem(shape, A=A, B=B, C_=C, L1=2.32, **g)
    q = rand_q(p, seed=len(name))
    F = p.forces(q)
    Ffd = five_point_forces(p, q)
    assert np.abs(F - Ffd).max() <= 1e-10 * np.abs(F).max()
    obj = (p.types == 2).reshape(p.field_shape[1:])
    assert np.all(F[:, obj] == 0.0)


def _forces_at_cases(ora):
    """Every geometry whose full force field is pinned to the exact gradient
    above, plus degenerate planar walls with fields, per-site records, the
    chiral term on an open box, and a 24^3 colloid slab (walls, sphere,
    L2/L3)."""
    for name in sorted(GEOMETRIES):
        g = dict(GEOMETRIES[name])
        shape = g.pop("shape")
        yield name, ora.Problem(shape, A=A, B=B, C_=C, L1=2.32, **g)
    yield "fg_walls_sphere_fields", ora.Problem(
        (4, 3, 5), L1=2.32, L2=0.9, L3=0.4, fields=[((0.2, 0.5, -1.0), 0.7)], objects=[
            dict(kind="wall", axis=2, plane=0, law="fg", W=0.8),
            dict(kind="wall", axis=2, plane=4, law="rp", W=-3.0),
            dict(kind="sphere", center=(1.7, 1.2, 2.0), radius=1.1, law="rp", W=-2.0)])
    yield "fg_records", ora.Problem(
        (3, 4, 3), L1=2.32, fields=[((1.0, 0.0, 0.0), -0.5)],
        site_records=[dict(site=7, law="fg", W=1.3, nu=(0.2, 0.9, 0.3)),
                      dict(site=7, law="nd", W=0.4, n0=(1, 0, 0)),
                      dict(site=20, law="rp", W=-5.0, nu=(0, 0, 1))])
    yield "L4_open", ora.Problem(
        (4, 3, 5), (False, True, False), L1=2.32, L2=0.9, L3=0.4, L4=-0.7, objects=[
            dict(kind="sphere", center=(1.5, 1.0, 2.0), radius=0.9, law="nd", W=0.6, dir="normal")],
        fields=[((0.1, 0.2, 0.3), 0.5)])
    cfg = synth.colloid_slab(24)
    cfg["objects"][2]["radius"] = 5.0
    yield "colloid_slab24", ora.Problem(cfg["shape"], cfg["periodic"], L1=cfg["L1"], L2=cfg["L2"],
                                        L3=cfg["L3"], objects=cfg["objects"])


def test_forces_at_sites_equal_the_full_force_field(ora):
    """The site-list force (used for sampled checks of lattices too large for
    a full pass) is the same gradient of the discrete energy (sec. III.B) as
    the full force field, which the tests above pin to the exact derivative:
    it agrees at every site of every case, up to the summation order of the
    anchoring terms."""
    for i, (name, p) in enumerate(_forces_at_cases(ora)):
        q = rand_q(p, seed=100 + i)
        F = p.forces(q).reshape(5, -1).T
        sites = np.arange(p.N)[::-1].copy()  # every site, in an order unlike the full pass
        Fa = p.forces_at(q, sites)
        assert np.abs(Fa - F[sites]).max() <= 1e-15 * np.abs(F).max(), name
        obj = p.types[sites] == 2
        assert np.all(Fa[obj] == 0.0), name


def test_translation_invariance(ora):
    """Rolling q by a lattice vector on a periodic box rolls F and keeps E."""
    p = ora.Problem((5, 6, 7), L1=2.32, L2=1.16, L3=0.4)
    q = rand_q(p, 11)
    E, F = p.energy(q), p.forces(q)
    for sh in [(1, 2, 3), (4, 0, 1)]:
        q2 = np.roll(q, shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3))
        assert abs(p.energy(q2) - E) <= 1e-12 * abs(E)
        F2 = np.roll(F, shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3))
        assert np.abs(p.forces(q2) - F2).max() <= 1e-12 * np.abs(F).max()


# -- cubic symmetry: a signed axis permutation R maps x -> R x and Q -> R Q R^T
def _full(q):
    q0, q1, q2, q3, q4 = q
    return np.array([[q0, q1, q2], [q1, q3, q4], [q2, q4, -q0 - q3]])


def _five(Q):
    return np.array([Q[0, 0], Q[0, 1], Q[0, 2], Q[1, 1], Q[1, 2]])


def _transform_field(q, shape, perm, sign):
    """new axis a takes old axis perm[a] with sign[a]; returns q' on the new grid."""
    R = np.zeros((3, 3))
    for a in range(3):
        R[a, perm[a]] = sign[a]
    nshape = tuple(shape[perm[a]] for a in range(3))
    Q = _full(q)  # (3,3,nz,ny,nx)
    Zp, Yp, Xp = np.meshgrid(*[np.arange(nshape[2]), np.arange(nshape[1]),
                               np.arange(nshape[0])], indexing="ij")
    newc = (Xp, Yp, Zp)
    old = [None] * 3
    for a in range(3):
        old[perm[a]] = (sign[a] * newc[a]) % shape[perm[a]]
    Qg = Q[:, :, old[2], old[1], old[0]]
    Qn = np.einsum("ab,bcxyz,dc->adxyz", R, Qg, R)
    return _five(Qn), R, nshape


def _transform_objects(objs, shape, perm, sign, R):
    out = []
    inv = {perm[a]: a for a in range(3)}
    for o in objs:
        o = dict(o)
        if o["kind"] == "sphere":
            c = o["center"]
            o["center"] = tuple((sign[a] * c[perm[a]]) % shape[perm[a]] for a in range(3))
        else:
            a = inv[o["axis"]]
            o["axis"] = a
            o["plane"] = (sign[a] * o["plane"]) % shape[perm[a]]
        if not isinstance(o.get("dir", "normal"), str):
            o["dir"] = tuple(R @ np.asarray(o["dir"], dtype=float))
        out.append(o)
    return out


@pytest.mark.parametrize("perm,sign", [((1, 0, 2), (1, 1, 1)), ((0, 2, 1), (1, 1, 1)),
                                       ((0, 1, 2), (-1, 1, 1)), ((2, 0, 1), (1, -1, 1))])
def test_cubic_symmetry(ora, perm, sign):
    """Axis permutations and reflections of lattice and tensor leave E
    invariant and carry F along; the y<->z and cyclic cases exercise the
    elimination Qzz = -Qxx - Qyy."""
    shape = (4, 5, 6)
    objs = [dict(kind="sphere", center=(1.2, 2.3, 3.1), radius=1.4, law="rp", W=4.0),
            dict(kind="wall", axis=0, plane=3, law="nd", W=0.6, dir=(0.3, 0.5, 0.8))]
    p = ora.Problem(shape, L1=2.32, L2=1.1, L3=0.45, objects=objs)
    q = rand_q(p, 21)
    qn, R, nshape = _transform_field(q, shape, perm, sign)
    pn = ora.Problem(nshape, L1=2.32, L2=1.1, L3=0.45,
                     objects=_transform_objects(objs, shape, perm, sign, R))
    E, En = p.energy(q), pn.energy(np.ascontiguousarray(qn))
    assert abs(E - En) <= 1e-12 * abs(E)
    # q' = T q per site with T linear; E(q) = E'(T q)  =>  F = T^T F'
    T = np.zeros((5, 5))
    for b in range(5):
        e = np.zeros(5)
        e[b] = 1.0
        T[:, b] = _five(R @ _full(e) @ R.T)
    Fn = pn.forces(np.ascontiguousarray(qn))
    F = p.forces(q)
    # bring F' back to the old grid: F'(x') at x' = R x
    Zo, Yo, Xo = np.meshgrid(np.arange(shape[2]), np.arange(shape[1]), np.arange(shape[0]),
                             indexing="ij")
    oldc = (Xo, Yo, Zo)
    newc = [(sign[a] * oldc[perm[a]]) % shape[perm[a]] for a in range(3)]
    Fn_old = Fn[:, newc[2], newc[1], newc[0]]
    back = np.einsum("ab,axyz->bxyz", T, Fn_old)
    assert np.abs(back - F).max() <= 1e-12 * np.abs(F).max()


def test_L2_and_L3_agree_on_a_periodic_box(ora):
    """Without boundaries the L2 and L3 terms of Eq. (fdistortionFull) differ
    by a total difference that sums to zero on a periodic lattice."""
    p2 = ora.Problem((5, 4, 6), L1=0.7, L2=1.3, L3=0.0)
    p3 = ora.Problem((5, 4, 6), L1=0.7, L2=0.0, L3=1.3)
    q = rand_q(p2, 31)
    E2, E3 = p2.energy(q), p3.energy(q)
    assert abs(E2 - E3) <= 1e-12 * abs(E2)
    F2, F3 = p2.forces(q), p3.forces(q)
    assert np.abs(F2 - F3).max() <= 1e-12 * np.abs(F2).max()


def _plane_wave(p, m, eps, dQ, Qbar, phi=0.37):
    nx, ny, nz = p.shape
    kap = 2 * np.pi * np.array([m[0] / nx, m[1] / ny, m[2] / nz])
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    th = kap[0] * X + kap[1] * Y + kap[2] * Z + phi
    q = Qbar[:, None, None, None] + eps * dQ[:, None, None, None] * np.cos(th)[None]
    return np.ascontiguousarray(q), kap


def test_L1_plane_wave_closed_form(ora):
    """Averaging the 2^3 one-sided choices on a periodic box makes every bond
    count once: E = L1/2 eps^2 |dQ|^2 N sum_k (1 - cos kappa_k)."""
    p = ora.Problem((6, 5, 7), A=0.0, B=0.0, C_=0.0, L1=2.32)
    rng = np.random.default_rng(7)
    dq, qbar = rng.standard_normal(5), rng.standard_normal(5)
    q, kap = _plane_wave(p, (1, 2, 3), 0.1, dq, qbar)
    dQ = _full(dq)
    ref = 0.5 * 2.32 * 0.01 * (dQ * dQ).sum() * p.N * (1 - np.cos(kap)).sum()
    assert abs(p.energy(q) - ref) <= 1e-12 * ref


def test_L2_L3_plane_wave_closed_form(ora):
    """Same-axis products average to the bond form, cross-axis products to
    the product of the averaged (here central) differences:
    E = (L2+L3) eps^2 N [1/2 sum_j (1-cos k_j)(dQ^2)_jj
                         + 1/2 sum_{j<k} sin k_j sin k_k (dQ^2)_jk]."""
    L2, L3 = 1.16, 0.55
    p = ora.Problem((6, 5, 7), A=0.0, B=0.0, C_=0.0, L1=0.0, L2=L2, L3=L3)
    rng = np.random.default_rng(8)
    dq, qbar = rng.standard_normal(5), rng.standard_normal(5)
    q, kap = _plane_wave(p, (1, 2, 3), 0.1, dq, qbar)
    dQ = _full(dq)
    D2 = dQ @ dQ
    s, c = np.sin(kap), np.cos(kap)
    diag = 0.5 * sum((1 - c[j]) * D2[j, j] for j in range(3))
    cross = 0.5 * sum(s[j] * s[k] * D2[j, k] for j in range(3) for k in range(j + 1, 3))
    ref = (L2 + L3) * 0.01 * p.N * (diag + cross)
    assert abs(p.energy(q) - ref) <= 1e-12 * abs(ref)


def test_wall_ramp_counts_one_sided_bonds_with_weight_three_halves(ora):
    """Reading of the averaging at a boundary: a site with one allowed choice
    along an axis uses it alone, so the bond next to a wall weighs 1 + 1/2.
    For Q linear in z between object planes z = 0 and z = nz-1 the bond
    weights add up to nz - 2 per column."""
    for nz in (4, 5, 8):
        objs = [dict(kind="wall", axis=2, plane=0, law="nd", W=0.0, dir="normal"),
                dict(kind="wall", axis=2, plane=nz - 1, law="nd", W=0.0, dir="normal")]
        p = ora.Problem((3, 4, nz), L1=2.32, objects=objs)
        rng = np.random.default_rng(nz)
        d = rng.standard_normal(5)
        Z = np.arange(nz)[None, :, None, None]
        q = np.ascontiguousarray(np.broadcast_to(d[:, None, None, None] * Z, p.field_shape).copy())
        q[:, (p.types == 2).reshape(p.field_shape[1:])] = 0.0
        dQ = _full(d)
        ref = 0.5 * 2.32 * (dQ * dQ).sum() * 3 * 4 * (nz - 2)
        _, t = p.energy(q, terms=True)
        assert abs(t[1] - ref) <= 1e-12 * ref


def test_axis_without_allowed_difference_contributes_zero(ora):
    """Reading: a site whose two neighbours along an axis are both inside
    objects takes that derivative as zero; the plane z = 1 between object
    planes z = 0, 2 then carries the 2D plane-wave energy."""
    objs = [dict(kind="wall", axis=2, plane=0, law="nd", W=0.0, dir="normal"),
            dict(kind="wall", axis=2, plane=2, law="nd", W=0.0, dir="normal")]
    p = ora.Problem((6, 5, 3), L1=2.32, objects=objs)
    rng = np.random.default_rng(9)
    dq = rng.standard_normal(5)
    q, kap = _plane_wave(p, (1, 2, 0), 0.1, dq, np.zeros(5))
    q[:, (p.types == 2).reshape(p.field_shape[1:])] = 0.0
    dQ = _full(dq)
    ref = 0.5 * 2.32 * 0.01 * (dQ * dQ).sum() * (6 * 5) * ((1 - np.cos(kap[:2])).sum())
    _, t = p.energy(q, terms=True)
    assert abs(t[1] - ref) <= 1e-12 * ref


def test_linear_field_reproduces_frank_oseen_via_paper_mapping(ora):
    """For a field linear in x every allowed one-sided difference is the
    exact derivative, so E / N_sim is the continuum density of Eq.
    (fdistortionFull).  Taking dQ from a uniaxial director field and the
    paper's L <-> K identifications (K3 = K1 so that L6 = 0), the density
    must equal the Frank-Oseen density of Eq. (FOfull) with the saddle-splay
    term written as tr((grad n)^2) - (div n)^2."""
    rng = np.random.default_rng(12)
    S = 0.6
    for _ in range(4):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        D = rng.standard_normal((3, 3))      # D[k, j] = d n_j / d x_k
        D = D - np.outer(D @ n, n)           # keep |n| = 1 to first order
        K1, K2, K24 = rng.uniform(0.5, 2.0, 3)
        K3 = K1
        L1 = 2 / (27 * S * S) * (K3 - K1 + 3 * K2)
        L2 = 4 / (9 * S * S) * (K1 - K24)
        L3 = 4 / (9 * S * S) * (K24 - K2)
        div = np.trace(D)
        curl = np.array([D[1, 2] - D[2, 1], D[2, 0] - D[0, 2], D[0, 1] - D[1, 0]])
        bend = n @ D
        fo = 0.5 * (K1 * div ** 2 + K2 * (n @ curl) ** 2 + K3 * bend @ bend
                    + K24 * (np.einsum("ij,ji->", D, D) - div ** 2))
        # linear Q field on an open 4x4x4 box (every site has a choice on every axis)
        p = ora.Problem((4, 4, 4), periodic=(False, False, False), A=0.0, B=0.0, C_=0.0,
                        L1=L1, L2=L2, L3=L3)
        Q0 = 1.5 * S * (np.outer(n, n) - np.eye(3) / 3)
        dQ = [1.5 * S * (np.outer(D[k], n) + np.outer(n, D[k])) for k in range(3)]
        Z, Y, X = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
        Qf = (Q0[:, :, None, None, None] + dQ[0][:, :, None, None, None] * X
              + dQ[1][:, :, None, None, None] * Y + dQ[2][:, :, None, None, None] * Z)
        q = np.ascontiguousarray(_five(Qf))
        assert abs(p.energy(q) / p.N - fo) <= 1e-12 * abs(fo)


# ---------------------------------------------------------------- anchoring
def test_nobili_durand_reduces_to_rapini_papoular(ora):
    """Sec. II.A.4: for uniaxial Q at S0, W_ND tr((Q - Q0)^2) =
    W_RP/2 (1 - (n.nu)^2) with W_RP = 9 S0^2 W_ND; a Rapini-Papoular
    strength enters through W_ND = W_RP / (9 S0^2)."""
    rng = np.random.default_rng(13)
    for law, W in (("rp", 5.0), ("nd", 0.8)):
        objs = [dict(kind="wall", axis=2, plane=0, law=law, W=W, dir="normal")]
        p = ora.Problem((3, 3, 3), L1=2.32, objects=objs)
        assert len(p.pair_site) == 18  # planes z = 1 and z = 2 (periodic wrap) touch z = 0
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        q = p.uniaxial(np.repeat(n[:, None], p.N, axis=1))
        _, t = p.energy(q, terms=True)
        Wrp = W if law == "rp" else 9 * p.S0 ** 2 * W
        assert abs(t[2] - 18 * 0.5 * Wrp * (1 - n[2] ** 2)) <= 1e-13 * max(1.0, abs(t[2]))


# ---------------------------------------------------------------- geometry
def test_sphere_rasterization_by_brute_force(ora):
    """Sites with |x - c|^2 < R^2 are inside; a simulated site with a face
    neighbour inside is a boundary site (the stencil only reaches face
    neighbours, sec. III.B).  Counted by a plain loop for the 128^3 colloid."""
    c, R, n = 63.5, 12.0, 128
    inside = set()
    for x in range(48, 80):
        for y in range(48, 80):
            for z in range(48, 80):
                if (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 < R * R:
                    inside.add((x, y, z))
    bnd = set()
    for (x, y, z) in inside:
        for d in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            s = (x + d[0], y + d[1], z + d[2])
            if s not in inside:
                bnd.add(s)
    cfg = synth.colloid_slab(n)
    types, ps, pw, pq = ora.rasterize(cfg["shape"], cfg["periodic"], cfg["objects"],
                                      ora.S0(A, B, C))
    assert int((types == 2).sum()) == len(inside) + 2 * n * n
    sphere_pairs = pw > 1.0  # the colloid's W_ND = 5/(9 S0^2) ~ 1.96, walls 0.5
    assert int(sphere_pairs.sum()) == len(bnd)
    assert int((types == 1).sum()) == len(bnd) + 2 * n * n
    assert abs(pw[sphere_pairs][0] - 5.0 / (9 * ora.S0(A, B, C) ** 2)) < 1e-15


def test_patterned_wall_radial_director_by_hand(ora):
    """Radial in-plane director about the nearest centre of the 4 x 4 array
    (centres at 63.5 + 128 i): at (0, 0, 1) the nearest centre is
    (63.5, 63.5), so n0 = (-1, -1, 0)/sqrt(2); at (200, 70, 1) it is
    (191.5, 63.5), so n0 = (8.5, 6.5, 0)/|.|."""
    cfg = synth.patterned_wall(512)
    o = cfg["objects"][0]
    s0 = ora.S0(A, B, C)
    for (x, y), d in [((0, 0), (-1.0, -1.0)), ((200, 70), (8.5, 6.5))]:
        types, ps, pw, pq = ora.rasterize((512, 512, 3), (True, True, False), [o], s0)
        site = x + 512 * (y + 512 * 1)
        i = np.nonzero(ps == site)[0]
        assert len(i) == 1
        v = np.array([d[0], d[1], 0.0])
        v /= np.linalg.norm(v)
        Q0 = 1.5 * s0 * (np.outer(v, v) - np.eye(3) / 3)
        assert np.abs(pq[i[0]] - _five(Q0)).max() < 1e-15


# ---------------------------------------------------------------- FIRE
def test_fire_is_velocity_verlet_until_the_first_restart(ora):
    """Algorithm 1 on F = -k x in one unknown: while P > 0 the steering does
    nothing (v is parallel to F), so x_n = x0 cos(n theta) with
    cos theta = 1 - k dt^2 / 2 (velocity Verlet); the first step with x_n <= 0
    has P <= 0 and restarts: v = 0, dt halves, and the motion starts again from
    rest with the new theta."""
    k, dt0 = 1.0, 0.1
    prm = ora.fire_params(dt0=dt0, dt_max=dt0, alpha0=0.3, f_inc=1.1, f_dec=0.5, f_alpha=0.99,
                          n_min=10 ** 9, force_tol=0.0, max_steps=10 ** 6)
    st, xs, tr, v, F = ora.fire_generic(prm, np.array([1.0]), lambda x: -k * x, 40)
    th = math.acos(1 - k * dt0 ** 2 / 2)
    m = math.ceil(math.pi / (2 * th))
    n = np.arange(m + 1)
    assert np.abs(xs[: m + 1, 0] - np.cos(n * th)).max() < 1e-13
    assert np.all(tr[: m - 1, 0] > 0) and tr[m - 1, 0] <= 0
    assert tr[m - 1, 4] == dt0 * 0.5
    th2 = math.acos(1 - k * (dt0 / 2) ** 2 / 2)
    j = np.arange(0, 10)
    assert np.abs(xs[m: m + 10, 0] - xs[m, 0] * np.cos(j * th2)).max() < 1e-13


def test_fire_timestep_and_steering_schedule(ora):
    """Once P has been positive for more than N_min steps, every further step
    multiplies dt by f_inc (capped at dt_max) and alpha by f_alpha."""
    dt0, dtm, fi, a0, fa, nmin = 0.01, 0.05, 1.1, 0.3, 0.9, 5
    prm = ora.fire_params(dt0=dt0, dt_max=dtm, alpha0=a0, f_inc=fi, f_dec=0.5, f_alpha=fa,
                          n_min=nmin, force_tol=0.0, max_steps=10 ** 6)
    st, xs, tr, v, F = ora.fire_generic(prm, np.array([1.0, -2.0]),
                                        lambda x: -1e-4 * np.array([1.0, 3.0]) * x, 40)
    assert np.all(tr[:, 0] > 0)
    t = np.arange(1, 41)
    e = np.maximum(0, t - nmin)
    assert np.allclose(tr[:, 4], np.minimum(dt0 * fi ** e, dtm), rtol=1e-13, atol=0)
    assert np.allclose(tr[:, 5], a0 * fa ** e, rtol=1e-13, atol=0)


def test_fire_full_steering_aligns_velocity_with_force(ora):
    """With alpha = 1 the mixed velocity is |v| F/|F|: parallel to F with the
    speed the Verlet step produced; after a restart it is zero."""
    prm = ora.fire_params(dt0=0.05, dt_max=0.2, alpha0=1.0, f_inc=1.1, f_dec=0.5, f_alpha=1.0,
                          n_min=3, force_tol=0.0, max_steps=10 ** 6)
    Kd = np.array([1.0, 4.0, 9.0])
    x0 = np.array([1.0, 1.0, -0.5])
    for nsteps in (1, 2, 5, 17, 30):
        st, xs, tr, v, F = ora.fire_generic(prm, x0, lambda x: -Kd * x, nsteps)
        if tr[-1, 0] > 0:
            assert np.abs(np.cross(v, F)).max() < 1e-15 * np.linalg.norm(F) * np.linalg.norm(v) * 10
            assert v @ F > 0
            assert abs(np.linalg.norm(v) - tr[-1, 2]) < 1e-15 * 10
        else:
            assert np.all(v == 0)


@pytest.mark.parametrize("anchor_dir", [(1.0, 0.0, 0.0), "normal"])
def test_fire_reaches_the_exact_wall_minimum(ora, anchor_dir):
    """Between two Nobili-Durand walls preferring the same director n, the
    global minimum is Q = Q0(n) everywhere with E = N_sim f0; FIRE from a
    random start must get there."""
    objs = [dict(kind="wall", axis=2, plane=0, law="nd", W=0.5, dir=anchor_dir),
            dict(kind="wall", axis=2, plane=5, law="nd", W=0.5, dir=anchor_dir)]
    p = ora.Problem((4, 4, 6), L1=2.32, L2=1.16, L3=1.16, objects=objs)
    q = p.uniaxial(synth.random_directors(1, p.N))
    prm = ora.fire_params(dt0=1e-3, dt_max=0.05, alpha0=0.99, force_tol=1e-10, max_steps=20000)
    st, q, v, F = p.minimize(prm, q)
    assert st.status == ora.CONVERGED
    s0 = p.S0
    f0 = 0.75 * A * s0 ** 2 + 0.25 * B * s0 ** 3 + 9.0 / 16.0 * C * s0 ** 4
    E = p.energy(q)
    assert abs(E - p.n_sim * f0) <= 1e-9 * abs(p.n_sim * f0)
    n = np.array([1.0, 0.0, 0.0]) if anchor_dir != "normal" else np.array([0.0, 0.0, 1.0])
    q0 = _five(1.5 * s0 * (np.outer(n, n) - np.eye(3) / 3))
    sim = (p.types != 2).reshape(p.field_shape[1:])
    assert np.abs(q[:, sim] - q0[:, None]).max() < 1e-5


def test_fire_resume_is_bitwise(ora):
    """Stopping after k steps and continuing with the saved state and
    controller gives the same trajectory bit for bit."""
    p = ora.Problem((5, 4, 3), L1=2.32, L2=0.5, L3=0.2,
                    objects=[dict(kind="wall", axis=2, plane=0, law="rp", W=3.0)])
    q0 = p.uniaxial(synth.random_directors(4, p.N))
    prm = ora.fire_params(max_steps=10 ** 6, force_tol=0.0)
    st, q, v, F = p.fire_init(prm, q0)
    p.fire_steps(prm, st, q, v, F, 60)
    st2, q2, v2, F2 = p.fire_init(prm, q0)
    p.fire_steps(prm, st2, q2, v2, F2, 25)
    saved = (st2.dt, st2.alpha, st2.n_pos, st2.step)
    q3, v3 = q2.copy(), v2.copy()
    st3, q3, v3, F3 = p.fire_init(prm, q3, v3, keep_v=True)
    st3.dt, st3.alpha, st3.n_pos, st3.step = saved
    p.fire_steps(prm, st3, q3, v3, F3, 35)
    assert np.array_equal(q3, q) and np.array_equal(v3, v) and np.array_equal(F3, F)


def test_uniform_director_sampling_moments():
    """The generator's directors are unit vectors with <n n> = I/3."""
    n = synth.random_directors(0, 200000)
    assert np.abs((n * n).sum(axis=0) - 1).max() < 1e-12
    M = n @ n.T / n.shape[1]
    assert np.abs(M - np.eye(3) / 3).max() < 5e-3


def test_fire_at_a_stationary_point_restarts(ora):
    """Reading: P = 0 takes the restart branch.  Started at an exact
    stationary point (the isotropic state Q = 0, where every term of the
    gradient vanishes), every step has P = 0: v stays zero, q does not move
    and dt halves each step."""
    p = ora.Problem((3, 4, 5), L1=2.32, L2=1.0, L3=0.3)
    q0 = np.zeros(p.field_shape)
    prm = ora.fire_params(dt0=0.01, force_tol=0.0, max_steps=100)
    st, q, v, F = p.fire_init(prm, q0)
    assert np.all(F == 0.0)
    taken, tr = p.fire_steps(prm, st, q, v, F, 4, trace=True)
    assert taken == 4 and st.restarts == 4
    assert np.all(v == 0.0) and np.array_equal(q, q0)
    assert np.array_equal(tr[:, 4], 0.01 * 0.5 ** np.arange(1, 5))


# ---------------------------------------------------------------- degenerate planar + fields
def test_fournier_galatola_uniaxial_closed_form(ora):
    """Sec. II.A.4, Eq. (planarDegenerate) with the projector P Qt P: for a
    uniaxial Q at S0 with director n and a surface normal nu (c = n.nu),
    Qt - P Qt P = 3/2 S0 [c (n nu + nu n) - c^2 nu nu], so the density is
    W (9/4) S0^2 (2 c^2 - c^4): zero for every n in the surface plane, and
    (9/2) S0^2 W c^2 for small c, i.e. W_RP = 9 S0^2 W_FG (a negative
    Rapini-Papoular strength enters as |W_RP| / (9 S0^2))."""
    rng = np.random.default_rng(31)
    for law, W in (("fg", 0.7), ("rp", -4.0)):
        objs = [dict(kind="wall", axis=2, plane=0, law=law, W=W)]
        p = ora.Problem((3, 3, 3), L1=2.32, objects=objs)
        Wfg = W if law == "fg" else -W / (9 * p.S0 ** 2)
        for _ in range(4):
            n = rng.standard_normal(3)
            n /= np.linalg.norm(n)
            q = p.uniaxial(np.repeat(n[:, None], p.N, axis=1))
            _, t = p.energy(q, terms=True)
            c = n[2]
            ref = 18 * Wfg * 2.25 * p.S0 ** 2 * (2 * c * c - c ** 4)
            assert abs(t[2] - ref) <= 1e-13 * max(1.0, abs(ref))
        # degenerate: any in-plane director costs nothing
        a = rng.uniform(0, 2 * np.pi)
        q = p.uniaxial(np.repeat(np.array([[np.cos(a)], [np.sin(a)], [0.0]]), p.N, axis=1))
        assert abs(p.energy(q, terms=True)[1][2]) < 1e-15


def test_external_field_uniaxial_reduction(ora):
    """Sec. II.A.3: -(1/3) chi h.Q.h at a uniaxial Q equals
    -(1/2) chi S (h.n)^2 up to the n-independent chi S |h|^2 / 6."""
    rng = np.random.default_rng(32)
    h = np.array([0.3, -1.2, 0.5])
    E = np.array([1.0, 0.2, 0.0])
    p = ora.Problem((3, 3, 3), L1=0.0, fields=[(h, 0.8), (E, -0.3)])
    for _ in range(4):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        S = rng.uniform(0.1, 0.9)
        q = p.uniaxial(np.repeat(n[:, None], p.N, axis=1), S)
        _, t = p.energy(q, terms=True)
        ref = 0.0
        for v, chi in ((h, 0.8), (E, -0.3)):
            ref += -0.5 * chi * S * (v @ n) ** 2 + chi * S * (v @ v) / 6.0
        assert abs(t[3] / p.N - ref) <= 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("name", ["fg_walls_sphere_fields", "fg_records"])
def test_forces_exact_gradient_planar_and_fields(ora, name):
    """Forces stay the exact gradient with degenerate planar anchoring and
    external fields switched on."""
    if name == "fg_walls_sphere_fields":
        kw = dict(shape=(4, 3, 5), L2=0.9, L3=0.4, fields=[((0.2, 0.5, -1.0), 0.7)], objects=[
            dict(kind="wall", axis=2, plane=0, law="fg", W=0.8),
            dict(kind="wall", axis=2, plane=4, law="rp", W=-3.0),
            dict(kind="sphere", center=(1.7, 1.2, 2.0), radius=1.1, law="rp", W=-2.0)])
    else:
        kw = dict(shape=(3, 4, 3), L2=0.0, L3=0.0, fields=[((1.0, 0.0, 0.0), -0.5)],
                  site_records=[dict(site=7, law="fg", W=1.3, nu=(0.2, 0.9, 0.3)),
                                dict(site=7, law="nd", W=0.4, n0=(1, 0, 0)),
                                dict(site=20, law="rp", W=-5.0, nu=(0, 0, 1))])
    shape = kw.pop("shape")
    p = ora.Problem(shape, L1=2.32, **kw)
    q = rand_q(p, seed=41)
    F = p.forces(q)
    Ffd = five_point_forces(p, q)
    assert np.abs(F - Ffd).max() <= 1e-10 * np.abs(F).max()


# ---- gradient descent and Nesterov's accelerated gradient (sec. III.B) ----

def _spd(rng, n):
    X = rng.standard_normal((n, n))
    return X @ X.T / n + 0.2 * np.eye(n)


def test_gradient_descent_on_a_quadratic_is_the_matrix_power(ora):
    """For E = 1/2 x^T H x, GD gives x_t = (I - dt H)^t x_0: in the eigenbasis
    of H each coordinate is multiplied by (1 - dt lambda) per step."""
    rng = np.random.default_rng(51)
    H = _spd(rng, 7)
    x0 = rng.standard_normal(7)
    dt = 0.3
    st, xs, tr, m, F = ora.descent_generic(ora.descent_params("gd", dt, force_tol=0.0, max_steps=100),
                                           x0, lambda x: -H @ x, 25)
    lam, U = np.linalg.eigh(H)
    for t in (1, 7, 25):
        ref = U @ ((1.0 - dt * lam) ** t * (U.T @ x0))
        assert np.abs(xs[t] - ref).max() <= 1e-13 * np.abs(x0).max()
    assert np.allclose(F, -H @ xs[-1], rtol=0, atol=1e-15)
    assert st.step == 25 and np.all(m == 0.0)


def test_nesterov_on_a_quadratic_follows_its_two_term_recurrence(ora):
    """For E = 1/2 x^T H x, Nesterov's m' = mu m + dt F(x + mu m), x' = x + m'
    acts on each eigen-coordinate (x, m) of H through the 2x2 matrix
    [[1 - dt l, mu (1 - dt l)], [-dt l, mu (1 - dt l)]]; the t-th iterate is
    its t-th power applied to (x_0, 0)."""
    rng = np.random.default_rng(52)
    H = _spd(rng, 6)
    x0 = rng.standard_normal(6)
    dt, mu = 0.25, 0.8
    st, xs, tr, m, F = ora.descent_generic(
        ora.descent_params("nesterov", dt, mu, force_tol=0.0, max_steps=100), x0, lambda x: -H @ x, 40)
    lam, U = np.linalg.eigh(H)
    c0 = U.T @ x0
    for t in (1, 2, 13, 40):
        xe = np.empty(6)
        for i, l in enumerate(lam):
            a = 1.0 - dt * l
            T = np.array([[a, mu * a], [-dt * l, mu * a]])
            xe[i] = (np.linalg.matrix_power(T, t) @ np.array([c0[i], 0.0]))[0]
        assert np.abs(xs[t] - U @ xe).max() <= 1e-12 * np.abs(x0).max()
    # the kept force is the one at the look-ahead point, and P = F.m
    assert np.allclose(F, -H @ (xs[-1] + mu * m), rtol=0, atol=1e-14)
    assert tr[-1, 0] == pytest.approx(F @ m, rel=1e-12)
    assert tr[-1, 5] == mu and tr[-1, 4] == dt


def test_nesterov_without_momentum_is_gradient_descent_bitwise(ora):
    p = ora.Problem((6, 5, 4), L1=2.32, L2=1.16, L3=0.7, objects=[
        dict(kind="wall", axis=2, plane=0, law="fg", W=0.8),
        dict(kind="sphere", center=(2.5, 2.0, 2.0), radius=1.2, law="nd", W=1.0, dir="normal")],
        fields=[((0.3, 0.4, 0.1), 0.5)])
    q0 = p.uniaxial(synth.random_directors(53, p.N))
    out = []
    for method in ("gd", "nesterov"):
        prm = ora.descent_params(method, 0.02, 0.0, force_tol=0.0, max_steps=100)
        st, q, m, F = p.descent_init(prm, q0)
        p.descent_steps(prm, st, q, m, F, 30)
        out.append((q, F))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_gradient_descent_decreases_the_lattice_energy(ora):
    """A small GD step changes the energy by -dt |F|^2 to first order, and
    the energy decreases monotonically along the descent."""
    p = ora.Problem((7, 6, 5), (True, True, False), L1=2.32, L2=1.16, L3=1.16, objects=[
        dict(kind="wall", axis=2, plane=0, law="rp", W=-2.0),
        dict(kind="wall", axis=2, plane=4, law="nd", W=0.6, dir=(1.0, 0.0, 0.0))],
        fields=[((0.0, 1.0, 0.0), 0.4)])
    q0 = p.uniaxial(synth.random_directors(54, p.N))
    F0 = p.forces(q0)
    err = []
    for dt in (1e-4, 1e-5):
        prm = ora.descent_params("gd", dt, force_tol=0.0, max_steps=10)
        st, q, m, F = p.descent_init(prm, q0)
        p.descent_steps(prm, st, q, m, F, 1)
        err.append(abs((p.energy(q) - p.energy(q0)) / (-dt * (F0 * F0).sum()) - 1.0))
    # the second-order remainder shrinks with dt
    assert err[0] < 0.05 and 0.05 < err[1] / err[0] < 0.2
    prm = ora.descent_params("gd", 0.005, force_tol=0.0, max_steps=1000)
    st, q, m, F = p.descent_init(prm, q0)
    E = [p.energy(q)]
    for _ in range(40):
        p.descent_steps(prm, st, q, m, F, 5)
        E.append(p.energy(q))
    assert all(b < a for a, b in zip(E, E[1:]))


def test_descent_stop_tests(ora):
    """Stops with CONVERGED on the step where max|F| first drops below the
    tolerance, with MAX_STEPS at the step limit, and at once when the
    initial state already satisfies the tolerance."""
    H = np.diag([1.0, 0.5])
    f = lambda x: -H @ x
    st, xs, tr, m, F = ora.descent_generic(ora.descent_params("gd", 0.5, force_tol=1e-3, max_steps=1000),
                                           [1.0, 1.0], f, 1000)
    maxF = np.abs(tr[:, 3])
    assert st.status == ora.CONVERGED and maxF[-1] < 1e-3 and np.all(maxF[:-1] >= 1e-3)
    st, xs, tr, m, F = ora.descent_generic(ora.descent_params("nesterov", 0.5, 0.5, force_tol=0.0,
                                                              max_steps=17), [1.0, 1.0], f, 1000)
    assert st.status == ora.MAX_STEPS and st.step == 17 and len(xs) == 18
    st, xs, tr, m, F = ora.descent_generic(ora.descent_params("gd", 0.5, force_tol=10.0), [1.0, 1.0], f, 5)
    assert st.status == ora.CONVERGED and st.step == 0 and len(xs) == 1


# ---- the chiral L4 term of Eq. (fdistortionFull) ----

def _levi_civita():
    e = np.zeros((3, 3, 3))
    for (a, b, c), sgn in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1,
                           (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
        e[a, b, c] = sgn
    return e


@pytest.mark.parametrize("m", [1, 3])
def test_L4_helix_matches_frank_oseen_twist_through_the_mapping(ora, m):
    """With L4 = -8 q0 K2 / (9 S^2) (the paper's L<->K identification), the
    L4 term of a uniaxial helix n = (cos kz, sin kz, 0) equals the Frank-Oseen
    cross term K2 q0 n.(curl n) = -K2 q0 k.  On the periodic lattice the
    averaged one-sided z-differences are central differences, which scale
    the exact derivative of cos 2kz, sin 2kz by sin(2k)/(2k), so the lattice
    energy per site is exactly -K2 q0 sin(2k)/2."""
    nz = 16
    k = 2 * np.pi * m / nz
    K2, q0 = 1.7, 0.35
    S = 0.53
    L4 = -8.0 * q0 * K2 / (9.0 * S * S)
    p = ora.Problem((3, 4, nz), L1=0.0, L4=L4)
    z = np.arange(nz, dtype=np.float64)
    n = np.zeros((3, nz, 4, 3))
    n[0] = np.cos(k * z)[:, None, None]
    n[1] = np.sin(k * z)[:, None, None]
    q = p.uniaxial(n.reshape(3, -1), S)
    _, t = p.energy(q, terms=True)
    ref = -K2 * q0 * np.sin(2 * k) / 2.0
    assert abs(t[1] / p.N - ref) <= 1e-14 * abs(ref)
    # the opposite handedness costs the opposite
    n[1] *= -1.0
    _, t = p.energy(p.uniaxial(n.reshape(3, -1), S), terms=True)
    assert abs(t[1] / p.N + ref) <= 1e-14 * abs(ref)


def test_L4_linear_field_is_exact_on_an_open_box(ora):
    """For a Q field linear in position every allowed one-sided difference is
    the exact derivative, so with only L4 on, the averaged lattice energy is
    sum over sites of L4/2 eps_lik Q_lj(x) dQ_ij/dx_k, also at the faces of
    an open box."""
    rng = np.random.default_rng(61)
    shape = (4, 3, 5)
    p = ora.Problem(shape, (False, False, False), L1=0.0, L4=0.8)

    def sym_traceless():
        M = rng.standard_normal((3, 3))
        M = M + M.T
        return M - np.trace(M) / 3.0 * np.eye(3)

    Q0 = sym_traceless()
    G = [sym_traceless() for _ in range(3)]
    nx, ny, nz = shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    Q = Q0[None, None, None] + X[..., None, None] * G[0] + Y[..., None, None] * G[1] + Z[..., None, None] * G[2]
    q = np.stack([Q[..., 0, 0], Q[..., 0, 1], Q[..., 0, 2], Q[..., 1, 1], Q[..., 1, 2]])
    _, t = p.energy(q, terms=True)
    eps = _levi_civita()
    dQ = np.stack(G)  # [k, i, j]
    ref = 0.5 * 0.8 * np.einsum("lik,zyxlj,kij->", eps, Q, dQ)
    assert abs(t[1] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("periodic", [(True, True, True), (False, True, False)])
def test_forces_exact_gradient_with_L4(ora, periodic):
    p = ora.Problem((4, 3, 5), periodic, L1=2.32, L2=0.9, L3=0.4, L4=-0.7, objects=[
        dict(kind="sphere", center=(1.5, 1.0, 2.0), radius=0.9, law="nd", W=0.6, dir="normal")],
        fields=[((0.1, 0.2, 0.3), 0.5)])
    q = rand_q(p, seed=62)
    F = p.forces(q)
    Ffd = five_point_forces(p, q)
    assert np.abs(F - Ffd).max() <= 1e-10 * np.abs(F).max()


# ---- director and defect extraction (Eq. Qtensor; the GUI's display) ----

def _rotation(rng):
    A = rng.standard_normal((3, 3))
    R, _ = np.linalg.qr(A)
    return R * np.sign(np.linalg.det(R))


def test_director_of_biaxial_tensors_from_eq_qtensor(ora):
    """For Q = 3/2 S (nn - I/3) + 1/2 S_B (mm - ll) with 3 S > |S_B| the
    largest eigenvalue is S along n (the other two are (-S +- S_B)/2), so the
    extracted director is +-n and lambda_max = S."""
    rng = np.random.default_rng(71)
    N = 200
    ns, Qs, Ss = [], [], []
    for _ in range(N):
        R = _rotation(rng)
        n, m, l = R[:, 0], R[:, 1], R[:, 2]
        S = rng.uniform(0.05, 0.9)
        SB = rng.uniform(-0.9, 0.9) * S
        Q = 1.5 * S * (np.outer(n, n) - np.eye(3) / 3) + 0.5 * SB * (np.outer(m, m) - np.outer(l, l))
        ns.append(n)
        Qs.append(Q)
        Ss.append(S)
    Qs = np.array(Qs)
    q = np.stack([Qs[:, 0, 0], Qs[:, 0, 1], Qs[:, 0, 2], Qs[:, 1, 1], Qs[:, 1, 2]])
    n, lam, w, defect = ora.directors(q, np.zeros(N, np.uint8), 0.3)
    assert np.allclose(lam, Ss, rtol=0, atol=1e-14)
    assert np.allclose(np.abs(np.einsum("in,ni->n", n, np.array(ns))), 1.0, atol=1e-12)
    assert np.array_equal(defect, np.array(Ss) < 0.3)
    # the sign convention: the largest component is positive
    assert np.all(n[np.argmax(np.abs(n), axis=0), np.arange(N)] > 0)


def test_director_special_sites(ora):
    """Q = 0 has no director (n = 0, lambda = 0, a defect for any positive
    threshold); object sites are never defects; an oblate uniaxial Q
    (S < 0) has largest eigenvalue -S/2 and its director lies in the plane
    normal to n."""
    n0 = np.array([0.0, 0.6, 0.8])
    S = -0.4
    Q = 1.5 * S * (np.outer(n0, n0) - np.eye(3) / 3)
    q = np.zeros((5, 3))
    q[:, 2] = [Q[0, 0], Q[0, 1], Q[0, 2], Q[1, 1], Q[1, 2]]
    q[:, 1] = 0.1
    n, lam, w, defect = ora.directors(q, np.array([0, 2, 0], np.uint8), 0.05)
    assert np.all(n[:, 0] == 0.0) and lam[0] == 0.0 and defect[0]
    assert np.all(n[:, 1] == 0.0) and not defect[1]
    assert abs(lam[2] + S / 2) <= 1e-15 and abs(n[:, 2] @ n0) <= 1e-12
