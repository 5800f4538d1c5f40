"""Seeded generators of the voxel structures the capacitance path is exercised on.

Shapes follow the workloads of the paper's numerical-results section (single
conductors, parallel conductors in a dielectric, random multi-conductor
interconnect-like boxes, meander lines on a substrate, a dielectric-coated
sphere).  The paper's own geometries are not fully specified, so these are
synthetic stand-ins of the same kind and size; the recipes are written out in
each docstring.  numpy.random.default_rng(seed) (PCG64) is the only source of
randomness.
"""
from __future__ import annotations

import numpy as np


def _scene(name, cond_id, eps_r, dv, eps_b=1.0, **meta):
    cond_id = np.ascontiguousarray(cond_id, dtype=np.int32)
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    assert cond_id.shape == eps_r.shape and cond_id.ndim == 3
    return {"name": name, "cond_id": cond_id, "eps_r": eps_r, "dv": float(dv),
            "eps_b": float(eps_b), "meta": dict(meta)}


def _empty(shape, eps=1.0):
    return np.full(shape, -1, np.int32), np.full(shape, float(eps), np.float64)


def cube(n=16, edge_m=1.0):
    """A single conductor filling an n^3 grid (the unit cube when edge_m=1)."""
    c, e = _empty((n, n, n))
    c[:] = 0
    return _scene(f"cube{n}", c, e, edge_m / n, m=1)


def parallel_plates(nx=64, ny=64, nz=32, margin=8, thick=2, gap=8, eps_gap=4.0, dv=1e-6):
    """Two square plates (nx-2*margin wide, `thick` voxels thick) stacked along z,
    centred in z, `gap` voxels apart, with a dielectric slab of eps_gap filling
    exactly the space between them."""
    c, e = _empty((nx, ny, nz))
    z0 = (nz - (2 * thick + gap)) // 2
    xs = slice(margin, nx - margin)
    ys = slice(margin, ny - margin)
    c[xs, ys, z0:z0 + thick] = 0
    c[xs, ys, z0 + thick + gap:z0 + 2 * thick + gap] = 1
    e[xs, ys, z0 + thick:z0 + thick + gap] = eps_gap
    return _scene(f"plates{nx}x{ny}x{nz}_gap{gap}", c, e, dv, m=2, z_plates=(z0, z0 + thick + gap),
                  gap=gap, thick=thick, eps_gap=eps_gap)


def _place_boxes(rng, shape, count, lo, hi, gap, region=None, zlo=None, zhi=None, tries=20000):
    """Rejection-place `count` axis-aligned boxes with integer edges U{lo..hi}
    (per axis, lo/hi may be 3-tuples) inside `region` (list of (a, b) per axis),
    keeping at least `gap` empty voxels between any two boxes along some axis."""
    lo = np.broadcast_to(np.asarray(lo), (3,))
    hi = np.broadcast_to(np.asarray(hi), (3,))
    if region is None:
        region = [(0, s) for s in shape]
    boxes = []
    for _ in range(tries):
        if len(boxes) == count:
            break
        ext = [int(rng.integers(lo[a], hi[a] + 1)) for a in range(3)]
        ext = [min(ext[a], region[a][1] - region[a][0]) for a in range(3)]
        org = [int(rng.integers(region[a][0], region[a][1] - ext[a] + 1)) for a in range(3)]
        b = [(org[a], org[a] + ext[a]) for a in range(3)]
        ok = True
        for o in boxes:
            # separated along some axis by >= gap voxels
            sep = any(b[a][0] >= o[a][1] + gap or o[a][0] >= b[a][1] + gap for a in range(3))
            if not sep:
                ok = False
                break
        if ok:
            boxes.append(b)
    if len(boxes) != count:
        raise RuntimeError("could not place boxes")
    return boxes


def random_boxes(n=128, n_cond=8, n_diel=6, seed=3, dv=1e-6, edge=(4, 24), eps_range=(2.0, 10.0)):
    """Random multi-conductor scene: `n_cond` conductor boxes (edges U{edge}) with a
    >=1-voxel gap, and `n_diel` dielectric boxes (eps_r ~ U[eps_range]).  Dielectric
    box d is grown around an assigned conductor subset (boxes 0 and 1 get two
    conductors each, the others one) with a margin U{1..6}, clipped to the grid;
    later dielectric boxes overwrite earlier ones and conductors are painted last."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    c, e = _empty(shape)
    boxes = _place_boxes(rng, shape, n_cond, edge[0], edge[1], 1)
    # conductor subsets for dielectric boxes
    order = list(range(n_cond))
    subsets = []
    k = 0
    for d in range(n_diel):
        take = 2 if d < 2 else 1
        sub = order[k:k + take] if k < n_cond else [order[d % n_cond]]
        k += take
        subsets.append(sub if sub else [order[d % n_cond]])
    for d, sub in enumerate(subsets):
        margin = int(rng.integers(1, 7))
        eps = float(rng.uniform(*eps_range))
        lo = [max(0, min(boxes[i][a][0] for i in sub) - margin) for a in range(3)]
        hi = [min(n, max(boxes[i][a][1] for i in sub) + margin) for a in range(3)]
        e[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = eps
    for i, b in enumerate(boxes):
        c[b[0][0]:b[0][1], b[1][0]:b[1][1], b[2][0]:b[2][1]] = i
    return _scene(f"random{n}_s{seed}", c, e, dv, m=n_cond, boxes=boxes)


def meander(nx=512, ny=512, nz=16, lanes=4, runs=11, width=2, spacing=2, run_pitch=44,
            x0=16, x1=480, y0=16, sub_h=6, cond_h=2, eps_sub=4.4, dv=1e-6):
    """Parallel meander lines: `lanes` conductors, each `width` wide and `cond_h`
    thick, `spacing` apart, running `runs` times along x between x0 and x1 with
    nested U-turns at alternating ends; the lane order reverses on each run.  They
    sit on a substrate (z in [0, sub_h)) of eps_sub; air above."""
    c, e = _empty((nx, ny, nz))
    e[:, :, :sub_h] = eps_sub
    zc = slice(sub_h, sub_h + cond_h)
    pitch = width + spacing
    for lane in range(lanes):
        for r in range(runs):
            pos = lane if r % 2 == 0 else lanes - 1 - lane
            y = y0 + run_pitch * r + pitch * pos
            xa, xb = x0, x1
            # extend the run to the connector on each turning end
            if r < runs - 1:
                if r % 2 == 0:   # turn on the right
                    xb = x1 + pitch * (lanes - 1 - lane) + width
                else:            # turn on the left
                    xa = x0 - width - pitch * lane
            if r > 0:
                if (r - 1) % 2 == 0:   # came from a right turn
                    xb = max(xb, x1 + pitch * (lanes - 1 - lane) + width)
                else:
                    xa = min(xa, x0 - width - pitch * lane)
            c[xa:xb, y:y + width, zc] = lane
            if r < runs - 1:
                pos2 = lanes - 1 - pos
                y2 = y0 + run_pitch * (r + 1) + pitch * pos2
                if r % 2 == 0:
                    cx = x1 + pitch * (lanes - 1 - lane)
                else:
                    cx = x0 - width - pitch * lane
                c[cx:cx + width, y:y2 + width, zc] = lane
    return _scene(f"meander{nx}x{ny}x{nz}", c, e, dv, m=lanes)


def gradient_scene(nx=256, ny=256, nz=64, n_cond=6, seed=5, dv=1e-6, sub=(8, 40), tiles=4,
                   eps_range=(2.0, 10.0)):
    """Substrate z in [sub) tiled into tiles x tiles dielectric blocks (eps_r ~ U[eps_range]),
    each block one gradient parameter; `n_cond` conductor boxes (edges U{8..48} in x, y and
    U{2..8} in z) inside the substrate with >=2-voxel gaps.  meta['block_of_voxel'] maps
    every voxel to its block id (-1 outside the substrate)."""
    rng = np.random.default_rng(seed)
    c, e = _empty((nx, ny, nz))
    blk = np.full((nx, ny, nz), -1, np.int32)
    bx, by = nx // tiles, ny // tiles
    eps = rng.uniform(*eps_range, size=(tiles, tiles))
    for a in range(tiles):
        for b in range(tiles):
            e[a * bx:(a + 1) * bx, b * by:(b + 1) * by, sub[0]:sub[1]] = eps[a, b]
            blk[a * bx:(a + 1) * bx, b * by:(b + 1) * by, sub[0]:sub[1]] = a * tiles + b
    lo = (min(8, nx // 4), min(8, ny // 4), 2)
    hi = (min(48, nx // 3), min(48, ny // 3), min(8, (sub[1] - sub[0]) // 3))
    boxes = _place_boxes(rng, (nx, ny, nz), n_cond, lo, hi, 2,
                         region=[(2, nx - 2), (2, ny - 2), (sub[0] + 2, sub[1] - 2)])
    for i, bb in enumerate(boxes):
        c[bb[0][0]:bb[0][1], bb[1][0]:bb[1][1], bb[2][0]:bb[2][1]] = i
        blk[bb[0][0]:bb[0][1], bb[1][0]:bb[1][1], bb[2][0]:bb[2][1]] = -1
    return _scene(f"grad{nx}x{ny}x{nz}_s{seed}", c, e, dv, m=n_cond, block_of_voxel=blk,
                  nblocks=tiles * tiles, boxes=boxes)


def random_small(seed, shape=None, n_cond=None, n_diel=None, dv=1e-6, eps_b=1.0, edge_max=None):
    """Small random scene for parity tests: grid edges U{6..14} unless given, 1-3
    conductor boxes with a >=1-voxel gap (edges U{1..edge_max}), 0-2 dielectric boxes
    (eps_r ~ U[2, 10]) painted first so conductors sit inside or beside them."""
    rng = np.random.default_rng(seed)
    if shape is None:
        shape = tuple(int(s) for s in rng.integers(6, 15, size=3))
    if n_cond is None:
        n_cond = int(rng.integers(1, 4))
    if n_diel is None:
        n_diel = int(rng.integers(0, 3))
    c, e = _empty(shape, eps_b)
    for _ in range(n_diel):
        lo = [int(rng.integers(0, max(1, s // 2))) for s in shape]
        hi = [int(rng.integers(lo[a] + 1, shape[a] + 1)) for a in range(3)]
        e[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = float(rng.uniform(2.0, 10.0))
    em = edge_max or max(2, min(shape) // 2)
    boxes = _place_boxes(rng, shape, n_cond, 1, em, 1)
    for i, b in enumerate(boxes):
        c[b[0][0]:b[0][1], b[1][0]:b[1][1], b[2][0]:b[2][1]] = i
    return _scene(f"small_s{seed}", c, e, dv, eps_b=eps_b, m=n_cond, boxes=boxes)


def coated_sphere(dv=0.05, r_c=0.25, r_d=0.5, eps_r=2.0, box=1.0):
    """PEC sphere of radius r_c inside a dielectric shell of radius r_d (eps_r), on a
    box of edge `box` centred on the sphere; a voxel takes the material whose region
    holds its centre."""
    n = int(round(box / dv))
    ctr = (np.arange(n) + 0.5) * dv - box / 2
    X, Y, Z = np.meshgrid(ctr, ctr, ctr, indexing="ij")
    rr = np.sqrt(X * X + Y * Y + Z * Z)
    c, e = _empty((n, n, n))
    e[rr <= r_d] = eps_r
    c[rr <= r_c] = 0
    return _scene(f"sphere_dv{dv}", c, e, dv, m=1, r_c=r_c, r_d=r_d, eps_shell=eps_r)


def uneven_batch(count=32, seed0=1000, lo=16, hi=64):
    """`count` independent random scenes (seeds seed0..): grid edges U{lo..hi} per
    axis, 1-4 conductors with edges U{2..max(2, edge/3)}, and with probability 1/2 one
    dielectric box (eps_r ~ U[2, 10]) around the first conductor."""
    out = []
    for s in range(seed0, seed0 + count):
        rng = np.random.default_rng(s)
        shape = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        ncd = int(rng.integers(1, 5))
        c, e = _empty(shape)
        hi_e = [max(2, sh // 3) for sh in shape]
        boxes = _place_boxes(rng, shape, ncd, 2, hi_e, 1)
        if rng.random() < 0.5:
            b = boxes[0]
            mg = int(rng.integers(1, 4))
            l = [max(0, b[a][0] - mg) for a in range(3)]
            h = [min(shape[a], b[a][1] + mg) for a in range(3)]
            e[l[0]:h[0], l[1]:h[1], l[2]:h[2]] = float(rng.uniform(2.0, 10.0))
        for i, b in enumerate(boxes):
            c[b[0][0]:b[0][1], b[1][0]:b[1][1], b[2][0]:b[2][1]] = i
        out.append(_scene(f"batch_s{s}", c, e, 1e-6, m=ncd))
    return out


CONFIG_NAMES = ("cube16", "plates", "random128", "meander", "grad256")


def by_name(name):
    """The five benchmark workloads by name (see each generator for the recipe)."""
    if name == "cube16":
        return cube(16)
    if name == "plates":
        return parallel_plates()
    if name == "random128":
        return random_boxes()
    if name == "meander":
        return meander()
    if name == "grad256":
        return gradient_scene()
    raise KeyError(name)
