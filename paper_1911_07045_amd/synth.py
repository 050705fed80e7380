"""Seeded synthetic inputs: random directors, object layouts and request streams.

This module holds no Landau-de Gennes arithmetic; it only draws numbers.  Both
the GPU path and the CPU oracle take its outputs as inputs.

Random numbers come from a counter-based SplitMix64 stream (Steele, Lea &
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
i-th draw of stream (seed, tag) is mix(k + (i + 1) * gamma) with
k = mix(seed * gamma + tag), gamma = 0x9E3779B97F4A7C15, and mix the
published finalizer (xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27,
multiply 0x94D049BB133111EB, xor-shift 31).  A uniform in [0, 1) is the top
53 bits times 2^-53.  Draws of one site depend only on (seed, tag, index), so
any window of a large lattice can be regenerated on its own.

The workloads follow the paper's setups: a periodic random-start bulk box
(Fig. 2), colloids between anchoring plates (Fig. 3), many colloids in a
periodic box, a stream of small single-colloid boxes, and a wall patterned by
a square array of +1 in-plane defects (Fig. 6).  No dataset is involved.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, tag: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of stream (seed, tag) as float64 in [0, 1)."""
    with np.errstate(over="ignore"):
        key = _mix(np.uint64(seed) * GAMMA + np.uint64(tag))
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = _mix(key + i * GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


TAG_DIR_Z, TAG_DIR_PHI = 1, 2


def random_directors(seed: int, n_sites: int, start: int = 0) -> np.ndarray:
    """Unit vectors uniform on the sphere, shape (3, n_sites): z = 2u1 - 1, phi = 2 pi u2."""
    z = 2.0 * uniform(seed, TAG_DIR_Z, start, n_sites) - 1.0
    phi = 2.0 * math.pi * uniform(seed, TAG_DIR_PHI, start, n_sites)
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z])


TAG_FIELD = 3


def random_field(seed: int, n_sites: int, scale: float = 0.3, start: int = 0) -> np.ndarray:
    """Generic (not uniaxial) q-components, shape (5, n_sites), uniform in [-scale, scale)."""
    u = uniform(seed, TAG_FIELD, 5 * start, 5 * n_sites).reshape(n_sites, 5).T
    return np.ascontiguousarray(scale * (2.0 * u - 1.0))


class _Stream:
    """Sequential draws from one (seed, tag) stream."""

    def __init__(self, seed, tag):
        self.seed, self.tag, self.i = seed, tag, 0

    def u(self):
        x = float(uniform(self.seed, self.tag, self.i, 1)[0])
        self.i += 1
        return x


def _min_image_dist(a, b, n):
    d = 0.0
    for k in range(3):
        t = a[k] - b[k]
        t -= n[k] * math.floor(t / n[k] + 0.5)
        d += t * t
    return math.sqrt(d)


# Bulk and elastic constants of the workloads: the paper's 5CB coefficients and
# L1 = 2.32 used as dimensionless lattice-unit values.
BULK = dict(A=-0.172, B=-2.12, C_=1.73)
FIRE = dict(dt0=1e-3, dt_max=1e-2, alpha0=0.99)


def bulk32(seed=0):
    """32^3 periodic bulk box, one-constant L1, FP64, no objects."""
    return dict(name="bulk32", shape=(32, 32, 32), periodic=(True, True, True),
                L1=2.32, L2=0.0, L3=0.0, objects=[], dir_seed=seed, prec="f64",
                fire=dict(FIRE, force_tol=1e-9, max_steps=2000))


def bulk(n=256, seed=0, prec="f32"):
    """n^3 periodic bulk box from random directors, one-constant L1 (the
    setting of the paper's FIRE-vs-gradient-descent comparison, a 250^3 bulk
    box)."""
    return dict(name=f"bulk{n}", shape=(n, n, n), periodic=(True, True, True),
                L1=2.32, L2=0.0, L3=0.0, objects=[], dir_seed=seed, prec=prec,
                fire=dict(FIRE, force_tol=1e-9, max_steps=2000))


def colloid_slab(n=128, seed=1, with_colloid=True):
    """n^3 box: object planes z = 0 and z = n-1 with x-aligned Nobili-Durand
    anchoring W = 0.5, one sphere of radius 12 at the box centre with
    homeotropic Rapini-Papoular W = 5; L1 = 2.32, L2 = L3 = 1.16."""
    c = (n - 1) / 2.0
    objs = [dict(kind="wall", axis=2, plane=0, law="nd", W=0.5, dir=(1.0, 0.0, 0.0)),
            dict(kind="wall", axis=2, plane=n - 1, law="nd", W=0.5, dir=(1.0, 0.0, 0.0))]
    if with_colloid:
        objs.append(dict(kind="sphere", center=(c, c, c), radius=12.0, law="rp", W=5.0,
                         dir="normal"))
    return dict(name=f"colloid_slab{n}", shape=(n, n, n), periodic=(True, True, True),
                L1=2.32, L2=1.16, L3=1.16, objects=objs, dir_seed=seed, prec="f64",
                fire=dict(FIRE, force_tol=1e-9, max_steps=2000))


def multi_colloid(n=256, n_spheres=8, geom_seed=1002, seed=2, r_lo=8.0, r_hi=16.0):
    """n^3 periodic box with non-overlapping spheres (radii U[r_lo, r_hi],
    centres U[0, n)^3 by rejection until every pair is more than
    r_i + r_j + 2 apart), homeotropic Rapini-Papoular W ~ U[1, 10]; L1 only."""
    st = _Stream(geom_seed, 7)
    shp = (n, n, n)
    spheres = []
    while len(spheres) < n_spheres:
        r = r_lo + (r_hi - r_lo) * st.u()
        c = (n * st.u(), n * st.u(), n * st.u())
        ok = all(_min_image_dist(c, s["center"], shp) > r + s["radius"] + 2.0 for s in spheres)
        if ok:
            W = 1.0 + 9.0 * st.u()
            spheres.append(dict(kind="sphere", center=c, radius=r, law="rp", W=W, dir="normal"))
    return dict(name=f"multi_colloid{n}", shape=shp, periodic=(True, True, True),
                L1=2.32, L2=0.0, L3=0.0, objects=spheres, dir_seed=seed, prec="f32",
                fire=dict(FIRE, force_tol=1e-9, max_steps=2000), polish_steps=200)


def patterned_wall(n=512, seed=4, pitch=128, count=4):
    """n^3 box periodic in x, y: object plane z = 0 whose boundary layer has a
    radial in-plane preferred director around a count x count square array of
    centres (pitch apart, at half-integer positions), Rapini-Papoular W = 2;
    object plane z = n-1 with homeotropic Rapini-Papoular W = 2;
    L1 = 2.32, L2 = L3 = 1.16; FP32."""
    off = pitch / 2.0 - 0.5
    objs = [dict(kind="patterned_wall", axis=2, plane=0, law="rp", W=2.0,
                 pitch=(pitch, pitch), offset=(off, off), count=(count, count)),
            dict(kind="wall", axis=2, plane=n - 1, law="rp", W=2.0, dir="normal")]
    return dict(name=f"patterned_wall{n}", shape=(n, n, n), periodic=(True, True, True),
                L1=2.32, L2=1.16, L3=1.16, objects=objs, dir_seed=seed, prec="f32",
                fire=dict(FIRE, force_tol=1e-9, max_steps=5000))


def serving_stream(n_requests=512, rate=20.0, seed=3, side_lo=16, side_hi=64,
                   force_tol=1e-5, max_steps=5000):
    """Poisson arrivals (rate per second); cubic periodic box with side
    round(exp(U[ln lo, ln hi])); one sphere at the centre with radius
    U[3, side/4] and homeotropic Rapini-Papoular W log-uniform in [0.1, 10];
    L1 and bulk as the bulk box; FP32."""
    st = _Stream(seed, 11)
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += -math.log(1.0 - st.u()) / rate
        side = int(round(math.exp(math.log(side_lo) + (math.log(side_hi) - math.log(side_lo))
                                  * st.u())))
        R = 3.0 + (side / 4.0 - 3.0) * st.u()
        W = math.exp(math.log(0.1) + (math.log(10.0) - math.log(0.1)) * st.u())
        c = (side - 1) / 2.0
        reqs.append(dict(id=i, arrival=t, shape=(side, side, side), periodic=(True, True, True),
                         L1=2.32, L2=0.0, L3=0.0,
                         objects=[dict(kind="sphere", center=(c, c, c), radius=R, law="rp", W=W,
                                       dir="normal")],
                         dir_seed=100000 + i, prec="f32",
                         fire=dict(FIRE, force_tol=force_tol, max_steps=max_steps)))
    return reqs
