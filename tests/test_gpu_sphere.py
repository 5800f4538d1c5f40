"""GPU checks on the dielectric-coated PEC sphere of Sec. III.A (sphere radius 0.25 m,
shell radius 0.5 m, voxel centres decide the material).

* Permittivity sweep at dv = 0.05 m (N = 2376 panels): the shell's eps_r from 2 to
  2e7 (the high-contrast range of the section), capacitance against the dense FP64
  oracle and against the closed form of the coated sphere (staircase error only).
  As eps_r grows the dielectric rows approach 2 pi I + E on a closed surface, which is
  singular, so the condition number grows like eps_r and so does the difference of
  two correct implementations whose integrals agree to ~1e-14: the oracle gate is
  1e-12 * max(100, eps_r).  Mixed precision is checked where iterative refinement
  with FP32 products converges (condition number x FP32 rounding < 1, eps_r <= 2e4).
* Preconditioner comparison at dv = 0.01 m (N = 59,016), eps_r = 2, boxes of 10
  voxels, relative residual 1e-8: the section reports 22 (block-diagonal-diagonal),
  27 (block-diagonal over all panels), 41 (diagonal) and 142 (none) iterations
  (`tests/golden/`), and 17.04 MB against 70.26 MB of preconditioner storage.  The ordering is required
  and each count must lie within 15% of the paper's: not exactly, because the paper
  does not state its dielectric-row orientation or whether it preconditions on the
  left or the right (ours is right preconditioning, so the monitored residual is the
  true one)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS0 = 8.8541878128e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _closed_form(eps_r, r_c=0.25, r_d=0.5):
    return 4 * math.pi * EPS0 * eps_r * r_d * r_c / ((r_d - r_c) + eps_r * r_c)


@pytest.mark.parametrize("eps_r", [2.0, 2e2, 2e4, 2e7])
def test_coated_sphere_permittivity_sweep(dev, eps_r):
    from paper_2004_02609_amd import voxcap
    s = scenes.coated_sphere(0.05, eps_r=eps_r)
    P = voxcap.Problem.from_scene(s).setup()
    assert P.N == 2376   # the section's panel count for dv = 0.05 m
    C, st = P.capacitance(prec="fp64", rtol=1e-12)
    C_ref = oracle.solve_capacitance(s)
    rel_oracle = abs(C[0, 0] - C_ref[0, 0]) / abs(C_ref[0, 0])
    rel_formula = abs(C[0, 0] - _closed_form(eps_r)) / _closed_form(eps_r)
    print(f"eps_r {eps_r:g}: C {C[0, 0]:.6e} F, vs oracle {rel_oracle:.2e}, vs closed form {rel_formula:.3f}, "
          f"iterations {st['iters'][0]}", flush=True)
    assert rel_oracle < 1e-12 * max(100.0, eps_r), rel_oracle
    assert rel_formula < 0.1, rel_formula
    if eps_r <= 2e4:
        Cm, stm = P.capacitance(prec="mixed", rtol=1e-10)
        rel_mixed = abs(Cm[0, 0] - C_ref[0, 0]) / abs(C_ref[0, 0])
        print(f"eps_r {eps_r:g}: mixed vs oracle {rel_mixed:.2e}", flush=True)
        assert rel_mixed < 1e-6, rel_mixed


def test_coated_sphere_preconditioner_iterations(dev):
    from paper_2004_02609_amd import voxcap
    s = scenes.coated_sphere(0.01, eps_r=2.0)
    P = voxcap.Problem.from_scene(s).setup(nv=10)
    assert P.N == 59016   # the section's panel count for dv = 0.01 m
    its = {}
    Cs = {}
    for name, pc in (("block-diagonal-diagonal", 1), ("block-diagonal", 3), ("diagonal", 2), ("none", 0)):
        C, st = P.capacitance(prec="fp64", rtol=1e-8, use_precond=pc, max_iter=1000)
        its[name] = st["iters"][0]
        Cs[name] = C[0, 0]
    gold = os.path.join(os.path.dirname(__file__), "golden", "sphere_preconditioner_iterations.json")
    paper = json.load(open(gold))["iterations"]
    for k in its:
        print(f"{k}: {its[k]} iterations (paper {paper[k]}), C {Cs[k]:.6e} F", flush=True)
        assert abs(its[k] - paper[k]) <= 0.15 * paper[k], (k, its[k], paper[k])
    rel_formula = abs(Cs["block-diagonal-diagonal"] - _closed_form(2.0)) / _closed_form(2.0)
    print("vs closed form", rel_formula, flush=True)
    assert its["block-diagonal-diagonal"] < its["diagonal"] < its["none"], its
    # the section's ranking: the proposed preconditioner needs the fewest iterations
    assert its["block-diagonal-diagonal"] < its["block-diagonal"] < its["diagonal"], its
    # storage: the paper's proposed preconditioner needs about a quarter of the
    # conventional one's (17.04 MB vs 70.26 MB): the dielectric shell's panels, about
    # four times the conductor's, get blocks only in the conventional form
    m1, m3 = P.precond_info(1)["bytes"], P.precond_info(3)["bytes"]
    print(f"preconditioner storage: block-diagonal-diagonal {m1 / 1e6:.2f} MB, block-diagonal {m3 / 1e6:.2f} MB",
          flush=True)
    assert m3 > 2 * m1, (m1, m3)
    # the preconditioner changes the iteration count, not the solution
    ref = Cs["block-diagonal-diagonal"]
    for k, v in Cs.items():
        assert abs(v - ref) / ref < 1e-6, (k, v, ref)
    assert rel_formula < 0.05, rel_formula
