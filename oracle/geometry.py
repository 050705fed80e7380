"""Oracle-side geometry: site types and anchoring pairs, written plainly with numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Shares nothing with the
GPU library's own rasterizer; a CPU test checks that the two agree.

What it encodes (paper sec. III.B, site typing; sec. II.A.4, anchoring):
  * every site is bulk (0), boundary (1) or inside an object (2); only bulk
    and boundary sites are simulated;
  * a wall occupies one lattice plane; a sphere occupies the sites with
    |x - c|^2 < R^2 (minimum-image displacement on periodic axes, each
    component taken in [-n/2, n/2));
  * reading: a simulated site with a face neighbour inside object a forms one
    anchoring pair with a (area weight 1); a site touching two objects has two;
  * surface normal nu: the wall axis, or (x - c)/|x - c| for a sphere;
  * preferred director n0: nu ("normal", homeotropic), a fixed unit vector
    (oriented anchoring), or, for a patterned wall, the in-plane radial unit
    vector away from the nearest centre of a square array;
  * preferred tensor Q0 = 3/2 S0 (n0 n0 - I/3) (sec. II.A.4);
  * the strength used in W tr((Q - Q0)^2) is W for the Nobili-Durand law and
    W / (9 S0^2) for a Rapini-Papoular strength (sec. II.A.4, the relation
    W_RP = 9 S0^2 W_ND);
  * degenerate planar anchoring uses the Fournier-Galatola form
    W |Qt - P Qt P|^2 with the surface normal nu (sec. II.A.4): law "fg" takes
    W as the Fournier-Galatola strength, and a negative Rapini-Papoular
    strength (which the paper assigns to degenerate planar anchoring) enters
    as |W| / (9 S0^2).
"""
from __future__ import annotations

import numpy as np


def _min_image(d, n, periodic):
    if not periodic:
        return d
    return d - n * np.floor(d / n + 0.5)


def _inside(obj, X, Y, Z, shape, periodic):
    nx, ny, nz = shape
    kind = obj["kind"]
    if kind in ("wall", "patterned_wall"):
        c = (X, Y, Z)[obj["axis"]]
        return c == obj["plane"]
    if kind == "sphere":
        cx, cy, cz = obj["center"]
        dx = _min_image(X - cx, nx, periodic[0])
        dy = _min_image(Y - cy, ny, periodic[1])
        dz = _min_image(Z - cz, nz, periodic[2])
        return dx * dx + dy * dy + dz * dz < obj["radius"] ** 2
    raise ValueError(f"unknown object kind {kind!r}")


def _shift(mask, axis_xyz, step, periodic):
    """out[site] = mask[site + step*e_axis]; False off a non-periodic edge."""
    ax = 2 - axis_xyz  # arrays are indexed [z, y, x]
    out = np.roll(mask, -step, axis=ax)
    if not periodic[axis_xyz]:
        idx = [slice(None)] * 3
        idx[ax] = -1 if step > 0 else 0
        out[tuple(idx)] = False
    return out


def q_from_director(n, S):
    """q components of 3/2 S (n n - I/3); n has shape (3, ...)."""
    nx, ny, nz = n
    h = 1.5 * S
    return np.stack([h * (nx * nx - 1.0 / 3.0), h * nx * ny, h * nx * nz,
                     h * (ny * ny - 1.0 / 3.0), h * ny * nz])


KIND_ND, KIND_FG = 0, 1


def _strength(obj_or_rec, S0):
    """(kind, strength) of an object or record."""
    law = obj_or_rec.get("law", "nd")
    W = float(obj_or_rec["W"])
    if law == "nd":
        if W < 0:
            raise ValueError("negative Nobili-Durand strength")
        return KIND_ND, W
    if law == "rp":
        if W < 0:
            return KIND_FG, -W / (9.0 * S0 * S0)
        return KIND_ND, W / (9.0 * S0 * S0)
    if law == "fg":
        if W < 0:
            raise ValueError("negative Fournier-Galatola strength")
        return KIND_FG, W
    raise ValueError(f"unknown anchoring law {law!r}")


def rasterize(shape, periodic, objects, S0, site_records=(), object_sites=(), full=False):
    """Returns (types uint8[N], pair_site int64[P], pair_W float64[P], pair_Q0 float64[P,5]),
    and with full=True also pair_kind uint8[P] and pair_nu float64[P,3].

    shape = (nx, ny, nz); sites are numbered x + nx*(y + ny*z).
    objects: dicts with kind wall / sphere / patterned_wall (see module doc).
    site_records: dicts {site, law, W, n0} adding one pair each at a simulated site.
    object_sites: extra site indices that are inside an (anchoring-free) object.
    """
    nx, ny, nz = shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = X.astype(np.float64)
    Y = Y.astype(np.float64)
    Z = Z.astype(np.float64)
    inside = [_inside(o, X, Y, Z, shape, periodic) for o in objects]
    obj = np.zeros((nz, ny, nx), dtype=bool)
    for m in inside:
        obj |= m
    if len(object_sites):
        obj.reshape(-1)[np.asarray(object_sites, dtype=np.int64)] = True
    sim = ~obj

    sites_l, W_l, Q0_l, K_l, nu_l = [], [], [], [], []
    for o, m in zip(objects, inside):
        touch = np.zeros_like(m)
        for k in range(3):
            for s in (+1, -1):
                touch |= _shift(m, k, s, periodic)
        sel = sim & touch
        flat = np.nonzero(sel.reshape(-1))[0]
        if flat.size == 0:
            continue
        xs = X.reshape(-1)[flat]
        ys = Y.reshape(-1)[flat]
        zs = Z.reshape(-1)[flat]
        if o["kind"] in ("wall", "patterned_wall"):
            nu = np.zeros((3, flat.size))
            nu[o["axis"]] = 1.0
        else:
            cx, cy, cz = o["center"]
            d = np.stack([_min_image(xs - cx, nx, periodic[0]),
                          _min_image(ys - cy, ny, periodic[1]),
                          _min_image(zs - cz, nz, periodic[2])])
            nu = d / np.sqrt((d * d).sum(axis=0))
        if o["kind"] == "patterned_wall":
            n0 = _radial_director(o, xs, ys, zs, shape, periodic)
        else:
            d = o.get("dir", "normal")
            if isinstance(d, str):
                if d != "normal":
                    raise ValueError(f"unknown director mode {d!r}")
                n0 = nu
            else:
                v = np.asarray(d, dtype=np.float64)
                v = v / np.sqrt((v * v).sum())
                n0 = np.repeat(v[:, None], flat.size, axis=1)
        kind, Ws = _strength(o, S0)
        sites_l.append(flat.astype(np.int64))
        W_l.append(np.full(flat.size, Ws))
        Q0_l.append(q_from_director(n0, S0).T)
        K_l.append(np.full(flat.size, kind, dtype=np.uint8))
        nu_l.append(np.ascontiguousarray(nu.T))

    for r in site_records:
        s = int(r["site"])
        if not sim.reshape(-1)[s]:
            raise ValueError(f"anchoring record at non-simulated site {s}")
        kind, Ws = _strength(r, S0)
        key = "nu" if kind == KIND_FG else "n0"
        v = np.asarray(r[key], dtype=np.float64)
        v = v / np.sqrt((v * v).sum())
        sites_l.append(np.array([s], dtype=np.int64))
        W_l.append(np.array([Ws]))
        Q0_l.append(q_from_director(v[:, None], S0).T)
        K_l.append(np.array([kind], dtype=np.uint8))
        nu_l.append(v[None, :])

    if sites_l:
        ps = np.concatenate(sites_l)
        pw = np.concatenate(W_l)
        pq = np.ascontiguousarray(np.concatenate(Q0_l, axis=0))
        pk = np.concatenate(K_l)
        pn = np.ascontiguousarray(np.concatenate(nu_l, axis=0))
    else:
        ps = np.zeros(0, np.int64)
        pw = np.zeros(0)
        pq = np.zeros((0, 5))
        pk = np.zeros(0, np.uint8)
        pn = np.zeros((0, 3))
    types = np.where(obj.reshape(-1), 2, 0).astype(np.uint8)
    types[ps] = 1
    if full:
        return types, ps, pw, pq, pk, pn
    return types, ps, pw, pq


def _radial_director(o, xs, ys, zs, shape, periodic):
    """In-plane unit vector from the nearest centre of a square array, found
    by comparing the squared distance to every centre (first wins a tie)."""
    axis = o["axis"]
    inplane = [k for k in range(3) if k != axis]
    coords = (xs, ys, zs)
    u = coords[inplane[0]]
    w = coords[inplane[1]]
    nu_, nw_ = shape[inplane[0]], shape[inplane[1]]
    pu, pw = o["pitch"]
    ou, ow = o["offset"]
    cu_n, cw_n = o["count"]
    best = np.full(u.shape, np.inf)
    du_best = np.zeros(u.shape)
    dw_best = np.zeros(u.shape)
    for i in range(cu_n):
        for j in range(cw_n):
            du = _min_image(u - (ou + pu * i), nu_, periodic[inplane[0]])
            dw = _min_image(w - (ow + pw * j), nw_, periodic[inplane[1]])
            d2 = du * du + dw * dw
            better = d2 < best
            best = np.where(better, d2, best)
            du_best = np.where(better, du, du_best)
            dw_best = np.where(better, dw, dw_best)
    r = np.sqrt(du_best * du_best + dw_best * dw_best)
    n0 = np.zeros((3, u.size))
    n0[inplane[0]] = du_best / r
    n0[inplane[1]] = dw_best / r
    return n0
