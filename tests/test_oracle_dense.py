"""Pins of the oracle's panelizer, dense solve and capacitance against fixed facts.

* panel counts printed for the coated sphere (Sec. III.A) -- exact;
* the unit-cube capacitance (literature) and Thomson monotonicity of Galerkin
  capacitances under nested refinement;
* the parallel-plate limit eps*A/d and the mirror symmetry of two equal plates;
* sign pattern and symmetry of capacitance matrices, C proportional to dv, uniform
  background permittivity scaling;
* the coated-sphere closed form quoted in Sec. III.A (loose: staircase error);
* the adjoint permittivity gradient against central finite differences of C.
"""
import json
import os

import numpy as np
import pytest

import oracle
import scenes
from oracle import dense

K = 4.0 * np.pi * oracle.EPS0


def _panels(s):
    return oracle.panelize(s["cond_id"], s["eps_r"], s["eps_b"])


def test_sphere_panel_counts(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "sphere_panel_counts.json")))
    for dv, nt, n in zip(g["dv"], g["n_voxels"], g["n_panels"]):
        s = scenes.coated_sphere(dv)
        assert s["cond_id"].size == nt
        assert len(_panels(s)["axis"]) == n


def test_plate_counts_and_geometry_errors():
    p = _panels(scenes.parallel_plates())
    assert (p["n_cond"], p["n_diel"]) == (9984, 1536)
    c = np.full((4, 4, 4), -1, np.int32)
    e = np.ones((4, 4, 4))
    with pytest.raises(oracle.GeometryError):
        oracle.panelize(c, e, 1.0)                 # no conductor
    c[1, 1, 1] = 0
    c[1, 1, 2] = 1
    with pytest.raises(oracle.GeometryError):
        oracle.panelize(c, e, 1.0)                 # touching conductors
    c[1, 1, 2] = -1
    e[0, 0, 0] = 0.0
    with pytest.raises(oracle.GeometryError):
        oracle.panelize(c, e, 1.0)                 # eps <= 0
    e[0, 0, 0] = 1.0
    e[2:, :, :] = 1.0                               # same as background: no dielectric panels
    assert _panels({"cond_id": c, "eps_r": e, "eps_b": 1.0})["n_diel"] == 0


def test_unit_cube(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "cube_capacitance.json")))
    vals = [oracle.solve_capacitance(scenes.cube(n))[0, 0] / K for n in (4, 8, 16)]
    assert vals[0] < vals[1] < vals[2] < g["value"]
    assert abs(vals[2] / g["value"] - 1.0) < g["rel_tol_at_16"]


def test_plates_symmetry_and_parallel_plate_limit():
    ratios = []
    for gap in (6, 4, 2):
        s = scenes.parallel_plates(nx=20, ny=20, nz=14, margin=3, thick=2, gap=gap, eps_gap=4.0, dv=1e-6)
        C = oracle.solve_capacitance(s)
        assert abs(C[0, 0] - C[1, 1]) < 1e-10 * C[0, 0]
        assert abs(C[0, 1] - C[1, 0]) < 1e-10 * abs(C[0, 1])
        area = (14e-6) ** 2
        c_pp = 4.0 * oracle.EPS0 * area / (gap * 1e-6)
        assert -C[0, 1] > c_pp                     # fringing only adds
        ratios.append(-C[0, 1] / c_pp)
    assert ratios[0] > ratios[1] > ratios[2] > 1.0


@pytest.mark.parametrize("seed", [1, 4, 11])
def test_sign_pattern_scaling_and_background(seed):
    s = scenes.random_small(seed, n_diel=0)
    C = oracle.solve_capacitance(s)
    m = C.shape[0]
    assert np.all(np.diag(C) > 0)
    if m > 1:
        off = C[~np.eye(m, dtype=bool)]
        assert np.all(off < 0)
        assert np.all(C.sum(axis=1) > -1e-12 * np.abs(C).max())
    assert np.allclose(C, C.T, rtol=1e-9, atol=0)          # no dielectric: A symmetric
    s2 = dict(s, dv=s["dv"] * 3.0)
    assert np.allclose(oracle.solve_capacitance(s2), 3.0 * C, rtol=1e-12, atol=0)
    s3 = dict(s, eps_b=2.5, eps_r=np.full_like(s["eps_r"], 2.5))
    assert np.allclose(oracle.solve_capacitance(s3), 2.5 * C, rtol=1e-10, atol=0)


@pytest.mark.parametrize("seed", [2, 5])
def test_dielectric_scene_sign_pattern(seed):
    s = scenes.random_small(seed, n_diel=2, n_cond=2)
    C = oracle.solve_capacitance(s)
    assert np.all(np.diag(C) > 0) and C[0, 1] < 0 and C[1, 0] < 0
    # with dielectrics the discrete C is only approximately symmetric
    assert abs(C[0, 1] - C[1, 0]) < 0.05 * abs(C[0, 1])


def test_coated_sphere_closed_form():
    s = scenes.coated_sphere(0.05)
    C = oracle.solve_capacitance(s)[0, 0]
    rc, rd, er = 0.25, 0.5, 2.0
    exact = K * er * rd * rc / ((rd - rc) + er * rc)
    assert abs(C / exact - 1.0) < 0.05


def test_gradient_matches_finite_differences():
    s = scenes.random_small(21, shape=(7, 6, 6), n_cond=2, n_diel=0)
    # two dielectric blocks around the conductors
    blk = np.full(s["cond_id"].shape, -1, np.int32)
    eps = s["eps_r"].copy()
    eps[:, :, :3] = 3.0
    blk[:, :, :3] = 0
    eps[:, :3, 3:] = 6.0
    blk[:, :3, 3:] = 1
    cond = s["cond_id"]
    blk[cond >= 0] = -1
    s = dict(s, eps_r=eps)
    g, C = dense.capacitance_gradient(s, blk, 2)
    h = 1e-4
    for b in range(2):
        ep = eps.copy()
        ep[blk == b] += h
        em = eps.copy()
        em[blk == b] -= h
        fd = (oracle.solve_capacitance(dict(s, eps_r=ep)) - oracle.solve_capacitance(dict(s, eps_r=em))) / (2 * h)
        assert np.allclose(g[b], fd, rtol=1e-6, atol=1e-6 * np.abs(C).max()), (b, g[b], fd)


def test_dielectric_orientation_reading():
    """Rows of dielectric panels may be written with the +axis normal and
    I = 2 pi (eps_lo + eps_hi)/(eps_lo - eps_hi) instead of the paper's outward
    normal: that only multiplies each such row by sign = +-1, so the charges agree."""
    s = scenes.random_small(5, n_diel=2, n_cond=2)
    C, st = oracle.solve_capacitance(s, return_all=True)
    p, A = st["panels"], st["A"]
    S = np.where(p["kind"] == 1, p["sign"], 1).astype(float)
    A2 = S[:, None] * A
    lo, hi = p["eps_lo"], p["eps_hi"]
    diel = p["kind"] == 1
    I_plus = np.where(diel, 2 * np.pi * (lo + hi) / (lo - hi), 0.0)
    # the self field integral is 0, so the sign-flipped diagonal is the +axis jump term
    assert np.allclose(np.diag(A2)[diel], I_plus[diel], rtol=1e-14)
    rho2 = np.linalg.solve(A2, oracle.rhs(p))
    assert np.allclose(rho2, st["rho"], rtol=1e-10, atol=1e-14)


def _interface_scene():
    """7x6x5 grid: a conductor on the grid's low x face, two overlapping dielectric boxes
    (eps 3 and 6, so a dielectric-dielectric interface) that reach the grid's high y and
    z faces, and a second conductor inside the eps-6 box."""
    c = np.full((7, 6, 5), -1, np.int32)
    e = np.ones((7, 6, 5))
    e[2:7, 1:6, 1:5] = 3.0
    e[4:7, 2:6, 2:5] = 6.0
    c[0:2, 1:3, 1:3] = 0            # touches the low x face of the grid
    c[5:6, 3:5, 3:4] = 1            # inside the eps-6 box
    return {"cond_id": c, "eps_r": e, "eps_b": 1.0, "dv": 1e-6}


@pytest.mark.parametrize("make", [_interface_scene,
                                  lambda: scenes.random_small(5, n_cond=2, n_diel=2),
                                  lambda: scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1)])
def test_assemble_rows_equals_assemble(make):
    """The sampled-row route (each entry integrated from its own offset) gives the rows
    of the lag-table assembly of eq. (4): conductor rows, dielectric rows of both
    orientation signs with their eq. (7) jump, grid-edge panels and a
    dielectric-dielectric interface; rows asked in any order and repeated."""
    s = make()
    p = _panels(s)
    A = dense.assemble(p)
    n = len(p["axis"])
    diel = p["kind"] == 1
    rng = np.random.default_rng(4)
    rows = rng.permutation(n)[: min(n, 40)]
    # every kind of row the scenes hold: both signs, grid-edge faces, eps on both sides
    edge = np.nonzero((p["idx"][np.arange(n), p["axis"]] == 0) |
                      (p["idx"][np.arange(n), p["axis"]] == np.asarray(s["cond_id"].shape)[p["axis"]]))[0]
    dd = np.nonzero(diel & (p["eps_lo"] != s["eps_b"]) & (p["eps_hi"] != s["eps_b"]))[0]
    want = [np.nonzero(diel & (p["sign"] == 1))[0][:3], np.nonzero(diel & (p["sign"] == -1))[0][:3],
            edge[:3], dd[:3], np.nonzero(~diel)[0][:3]]
    rows = np.concatenate([rows] + want + [rows[:2]]).astype(np.int64)
    if make is _interface_scene:
        assert all(len(w) > 0 for w in want), [len(w) for w in want]
    R = dense.assemble_rows(p, rows)
    ref = A[rows]
    err = np.abs(R - ref).max() / np.abs(A).max()
    assert err <= 1e-15, err
