"""Host checks of the step kernels' work plan (lq_step_plan; no GPU).

Every plan must cover each column tile's planes exactly once, keep chunks
within 1 .. 256 planes (at least 4 where the lattice allows), flag as bulk
exactly the chunks whose padded neighbourhood is all full bulk sites, give
every block one or two chunks (listed together), stay within one wave of
resident blocks when the columns fit in one, cut one-constant lattices at
the same planes in every column, balance the cost of L2/L3 blocks (packing
two chunks into a block where whole chunks per column cannot), and give
every XCD (each contiguous eighth of the launch order) its share of the
wall chunks when the lattice takes many waves, the planes next to a
boundary then marching in short chunks of their own.
"""
import numpy as np
import pytest

from paper_1911_07045_amd import lqfire, synth


def full_mask(shape, periodic, objects):
    """Per site (z, y, x): simulated with all six face neighbours simulated."""
    types, *_ = lqfire.rasterize(shape, periodic, objects)
    nx, ny, nz = shape
    sim = np.asarray(types).reshape(nz, ny, nx) != 2
    full = sim.copy()
    for ax, n_per in ((2, periodic[0]), (1, periodic[1]), (0, periodic[2])):
        for s in (1, -1):
            nb = np.roll(sim, s, axis=ax)
            if not n_per:
                idx = [slice(None)] * 3
                idx[ax] = 0 if s == 1 else -1
                nb[tuple(idx)] = False
            full &= nb
    return full


def padded_all_full(full, periodic, x0, y0, z0, zc, tx, ty):
    nz, ny, nx = full.shape

    def idx(a, n, per):
        if 0 <= a < n:
            return a
        return a % n if per else None

    for z in range(z0 - 1, z0 + zc + 1):
        wz = idx(z, nz, periodic[2])
        if wz is None:
            return False
        for y in range(y0 - 1, y0 + ty + 1):
            wy = idx(y, ny, periodic[1])
            if wy is None:
                return False
            xs = [idx(x, nx, periodic[0]) for x in range(x0 - 1, x0 + tx + 1)]
            if any(x is None for x in xs) or not full[wz, wy, xs].all():
                return False
    return True


def check_plan(cfg, prec, resident):
    shape, periodic, objs = cfg["shape"], cfg["periodic"], cfg["objects"]
    chunks, bulk, (tx, ty), block = lqfire.step_plan(shape, periodic, prec, objs, resident, L1=cfg["L1"],
                                                     L2=cfg.get("L2", 0.0), L3=cfg.get("L3", 0.0))
    nx, ny, nz = shape
    # blocks are numbered 0, 1, ... in launch order, each with one or two chunks
    assert block[0] == 0 and (np.diff(block) >= 0).all() and (np.diff(block) <= 1).all()
    assert (np.bincount(block) <= 2).all()
    cols = {}
    for x0, y0, z0, zc in chunks:
        assert x0 % tx == 0 and y0 % ty == 0 and 0 <= x0 < nx and 0 <= y0 < ny
        assert 1 <= zc <= 256 and 0 <= z0 and z0 + zc <= nz
        cols.setdefault((x0, y0), []).append((z0, zc))
    ntx, nty = -(-nx // tx), -(-ny // ty)
    assert len(cols) == ntx * nty
    for runs in cols.values():
        cover = np.zeros(nz, dtype=int)
        for z0, zc in runs:
            cover[z0:z0 + zc] += 1
        assert (cover == 1).all()
        if nz >= 4:
            assert min(zc for _, zc in runs) >= 4
    full = full_mask(shape, periodic, objs)
    for (x0, y0, z0, zc), b in zip(chunks, bulk):
        assert bool(b) == padded_all_full(full, periodic, x0, y0, z0, zc, tx, ty)
    return chunks, bulk, cols, (tx, ty), full, block


def block_costs(chunks, bulk, block, full, periodic, tx, ty, g):
    """The planner's cost model: per chunk its planes (1, or g for a plane
    whose 3 x 3 x 3 neighbourhoods are not all full; the planner takes 3 in
    FP32 and 2.5 in FP64),
    13% more unless the whole padded chunk is full, plus 2; per block
    the sum of its chunks."""
    costs = np.zeros(block.max() + 1)
    for (x0, y0, z0, zc), b, k in zip(chunks, bulk, block):
        c = sum(1.0 if padded_all_full(full, periodic, x0, y0, f, 1, tx, ty) else g for f in range(z0, z0 + zc))
        costs[k] += c * (1.0 if b else 1.13) + 2.0
    return costs


def test_plan_l23_colloid_slab_fills_one_wave_and_balances_cost():
    cfg = synth.colloid_slab(64)
    cfg["objects"][2]["radius"] = 8.0
    resident = 64
    chunks, bulk, cols, (tx, ty), full, block = check_plan(cfg, "f32", resident)
    assert len(chunks) == resident and (np.bincount(block) == 1).all()
    costs = block_costs(chunks, bulk, block, full, cfg["periodic"], tx, ty, 3.0)
    # a cut lands within one plane (cost <= 3.4) of its equal-cost point
    assert costs.max() <= costs.sum() / resident + 2 * 3.4 + 1.0
    assert not bulk.all() and bulk.any()


def test_plan_packs_chunks_where_whole_chunks_cannot_balance():
    # 128^3 colloid slab in FP64: 64 columns for 256 resident blocks
    cfg = synth.colloid_slab(128)
    chunks, bulk, cols, (tx, ty), full, block = check_plan(cfg, "f64", 256)
    n_blocks = block.max() + 1
    assert n_blocks <= 256
    assert (np.bincount(block) == 2).any()
    costs = block_costs(chunks, bulk, block, full, cfg["periodic"], tx, ty, 2.5)
    # whole chunks per column leave the costliest block above 1.25x the mean
    # cost per resident block; packed, it stays within 1.12x
    assert costs.max() <= 1.12 * costs.sum() / 256


def test_plan_l1_cuts_every_column_alike():
    cfg = synth.multi_colloid(64, n_spheres=3, r_lo=4.0, r_hi=7.0)
    chunks, bulk, cols, _, _, block = check_plan(cfg, "f32", 32)
    assert (np.bincount(block) == 1).all()
    cuts = {tuple(sorted(r)) for r in cols.values()}
    assert len(cuts) == 1
    assert len(chunks) <= 32


def test_plan_many_waves_share_walls_among_xcds():
    nz = 512
    objs = [dict(kind="patterned_wall", axis=2, plane=0, law="rp", W=2.0, pitch=(16, 16), offset=(7.5, 7.5),
                 count=(4, 4)),
            dict(kind="wall", axis=2, plane=nz - 1, law="rp", W=2.0, dir="normal")]
    cfg = dict(shape=(64, 64, nz), periodic=(True, True, True), objects=objs, L1=2.32, L2=1.16, L3=1.16)
    resident = 4  # far fewer resident blocks than columns: many waves
    chunks, bulk, cols, _, full, block = check_plan(cfg, "f32", resident)
    assert (np.bincount(block) == 1).all()
    # every column: the planes next to each wall (0 .. 2 and 509 .. 511) in an
    # 8-plane chunk of its own, the bulk between them in two chunks of 248
    for runs in cols.values():
        assert sorted(runs) == [(0, 8), (8, 248), (256, 248), (504, 8)]
    walls = np.array([(z0 == 0) or (z0 + zc == nz) for _, _, z0, zc in chunks])
    assert (bulk == ~walls).all()
    per_xcd = walls.reshape(8, -1).sum(axis=1)
    assert (per_xcd == 2).all()
    # within an eighth: by rank, then column
    first = chunks[: len(chunks) // 8]
    assert list(first[:, 2]) == sorted(first[:, 2])


def test_plan_many_waves_boundary_runs_inside_the_box():
    # a sphere inside a 512-plane L2/L3 box: its planes march in non-bulk
    # chunks of up to 96 planes, every plane outside the runs in bulk chunks
    nz = 512
    objs = [dict(kind="sphere", center=(31.5, 31.5, 200.0), radius=20.0, law="rp", W=2.0, dir="normal")]
    cfg = dict(shape=(64, 64, nz), periodic=(True, True, True), objects=objs, L1=2.32, L2=1.16, L3=1.16)
    chunks, bulk, cols, (tx, ty), full, block = check_plan(cfg, "f32", 4)
    for (x0, y0, z0, zc), b in zip(chunks, bulk):
        assert zc <= (256 if b else 96)
        if not b:
            # a non-bulk chunk holds a plane whose neighbourhood is not all full
            assert any(not padded_all_full(full, cfg["periodic"], x0, y0, f, 1, tx, ty) for f in range(z0, z0 + zc))
    assert bulk.any() and not bulk.all()


@pytest.mark.parametrize("shape,periodic,prec", [((24, 24, 24), (True, True, True), "f32"),
                                                  ((37, 11, 9), (True, False, True), "f64"),
                                                  ((5, 7, 3), (False, False, False), "f32")])
def test_plan_small_and_ragged_boxes(shape, periodic, prec):
    c = [(s - 1) / 2.0 for s in shape]
    objs = [dict(kind="sphere", center=tuple(c), radius=min(shape) / 4.0, law="rp", W=2.0, dir="normal")]
    cfg = dict(shape=shape, periodic=periodic, objects=objs, L1=2.32, L2=0.7, L3=0.3)
    chunks, bulk, cols, _, _, _ = check_plan(cfg, prec, 512)
    cfg["L2"] = cfg["L3"] = 0.0
    check_plan(cfg, prec, 512)


@pytest.mark.parametrize("shape,periodic", [((37, 11, 9), (True, False, True)), ((24, 24, 24), (True, True, True)),
                                            ((5, 7, 3), (False, False, False)), ((70, 20, 300), (True, True, False)),
                                            ((65, 9, 600), (True, True, True))])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_plan_many_waves_small_and_ragged_boxes(shape, periodic, prec):
    # one resident block: every lattice takes many waves, L2/L3 lattices
    # with their boundary runs in chunks of their own
    c = [(s - 1) / 2.0 for s in shape]
    objs = [dict(kind="sphere", center=tuple(c), radius=min(shape) / 4.0, law="rp", W=2.0, dir="normal")]
    cfg = dict(shape=shape, periodic=periodic, objects=objs, L1=2.32, L2=0.7, L3=0.3)
    chunks, bulk, _, _, _, block = check_plan(cfg, prec, 1)
    assert (np.bincount(block) == 1).all()
    cfg["L2"] = cfg["L3"] = 0.0
    check_plan(cfg, prec, 1)


def test_plan_rejects_bad_arguments():
    with pytest.raises(lqfire.LQError):
        lqfire.step_plan((16, 16, 16), resident=0)
