"""GPU parity of the FFT product, preconditioner and capacitance with the FP64 oracle.

Tolerances: the FP64 product reaches the dense product up to rounding of the
integrals (~1e-14 relative per entry) and of the FFTs (~1e-15 log2 R); 1e-11 of
max|y| is a loose bound.  The FP32 product: FP32 FFTs of ~log2(R) stages, ~1e-6.
"""
import numpy as np
import pytest

import oracle
import scenes
from helpers import oracle_matrix_library_order

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCENES = [
    ("cube5", lambda: scenes.cube(5, 1.0)),
    ("small_s1", lambda: scenes.random_small(1, n_diel=0)),
    ("small_s5", lambda: scenes.random_small(5, n_cond=2, n_diel=2)),
    ("small_s9", lambda: scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)),
    ("ragged", lambda: scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1)),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _problem(s, **kw):
    from paper_2004_02609_amd import voxcap
    P = voxcap.Problem.from_scene(s)
    P.setup(**kw)
    return P


@pytest.mark.parametrize("name,make", SCENES)
def test_fft_product_matches_dense(dev, name, make):
    s = make()
    P = _problem(s, max_rhs=3)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, P.N))
    xt = torch.tensor(x, device=dev)
    for transpose in (False, True):
        y = P.apply(xt, transpose=transpose, prec="fp64").cpu().numpy()
        ref = (A.T if transpose else A) @ x.T
        err = np.abs(y - ref.T).max() / np.abs(ref).max()
        print(name, "transpose" if transpose else "forward", "fp64 rel err", err, flush=True)
        assert err < 1e-11, (name, transpose, err)
        y32 = P.apply(xt, transpose=transpose, prec="fp32").cpu().numpy()
        err32 = np.abs(y32 - ref.T).max() / np.abs(ref).max()
        print(name, "fp32 rel err", err32, flush=True)
        assert err32 < 2e-5, (name, transpose, err32)


def test_precond_blocks_invert_dense_blocks(dev):
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    P = _problem(s, nv=4)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    pan = P.panels()
    N = P.N
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, N))
    y = P.apply_precond(torch.tensor(x, device=dev)).cpu().numpy()
    # reference: boxes of 4 voxels own the conductor panels of their conductor voxel
    cond = pan["kind"] == 0
    vox = np.stack([pan["i"], pan["j"], pan["k"]], 1).astype(int)
    lo_is_cond = pan["eps_lo"] == 0.0
    vox[np.arange(N), pan["dir"]] -= lo_is_cond.astype(int)
    box = (vox // 4)
    ref = np.zeros_like(x)
    diel = ~cond
    ref[:, diel] = x[:, diel] / np.diag(A)[diel]
    keys = {}
    for p in np.nonzero(cond)[0]:
        keys.setdefault(tuple(box[p]), []).append(p)
    for idx in keys.values():
        idx = np.array(idx)
        B = A[np.ix_(idx, idx)]
        ref[:, idx] = np.linalg.solve(B, x[:, idx].T).T
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 1e-10, err


def test_comparison_preconditioners_match_dense(dev):
    """Kinds 2 and 3 of the preconditioner comparison (Sec. III.A) against the dense
    oracle matrix: the diagonal preconditioner is 1 / diag(A); the conventional
    block-diagonal one solves the full eq. (4) block of every box of 4 voxels, where a
    conductor panel joins the box of its conductor voxel and a dielectric panel the box
    of the voxel on its -axis side (its own voxel on the grid's low face).  The blocks
    are unsymmetric, so the transposed apply is checked against A_box^T as well."""
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    P = _problem(s, nv=4)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    pan = P.panels()
    N = P.N
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, N))
    xt = torch.tensor(x, device=dev)
    y2 = P.apply_precond_kind(2, xt).cpu().numpy()
    ref2 = x / np.diag(A)[None, :]
    e2 = np.abs(y2 - ref2).max() / np.abs(ref2).max()
    print("diagonal preconditioner rel err", e2, flush=True)
    assert e2 < 1e-12, e2
    cond = pan["kind"] == 0
    vox = np.stack([pan["i"], pan["j"], pan["k"]], 1).astype(int)
    rows = np.arange(N)
    shift = np.where(cond, (pan["eps_lo"] == 0.0).astype(int), (vox[rows, pan["dir"]] > 0).astype(int))
    vox[rows, pan["dir"]] -= shift
    box = vox // 4
    groups = {}
    for p in range(N):
        groups.setdefault(tuple(box[p]), []).append(p)
    assert sum(len(g) for g in groups.values()) == N
    assert any(cond[g].any() and (~cond[g]).any() for g in map(np.array, groups.values())), \
        "no box mixes conductor and dielectric panels"
    for transpose in (False, True):
        y3 = P.apply_precond_kind(3, xt, transpose=transpose).cpu().numpy()
        ref3 = np.zeros_like(x)
        for g in groups.values():
            idx = np.array(g)
            B = A[np.ix_(idx, idx)]
            ref3[:, idx] = np.linalg.solve(B.T if transpose else B, x[:, idx].T).T
        e3 = np.abs(y3 - ref3).max() / np.abs(ref3).max()
        print("block-diagonal preconditioner", "transposed" if transpose else "forward", "rel err", e3, flush=True)
        assert e3 < 1e-10, (transpose, e3)
    info1, info3 = P.precond_info(1), P.precond_info(3)
    print("storage kind 1", info1, "kind 3", info3, flush=True)
    assert info3["boxes"] == len(groups)


@pytest.mark.parametrize("name,make", SCENES)
def test_capacitance_fp64(dev, name, make):
    s = make()
    P = _problem(s)
    C, st = P.capacitance(prec="fp64", rtol=1e-13)
    C_ref = oracle.solve_capacitance(s)
    d = np.abs(np.diag(C_ref)).max()
    gate = np.abs(C_ref) >= 1e-3 * d
    rel = np.abs(C - C_ref)[gate] / np.abs(C_ref)[gate]
    norm = np.abs(C - C_ref).max() / d
    print(name, "C fp64 max entry rel err", rel.max(), "normwise", norm, "iters", st["iters"], flush=True)
    assert rel.max() < 1e-10, (name, rel.max())
    assert norm < 1e-10, (name, norm)


@pytest.mark.parametrize("name,make", SCENES[2:4])
@pytest.mark.parametrize("form", ["refinement", "relaxed"])
def test_capacitance_mixed(dev, name, make, form):
    s = make()
    P = _problem(s)
    C, st = P.capacitance(prec="mixed", rtol=1e-10, mixed_form=form)
    assert st["mixed_form"] == form
    C_ref = oracle.solve_capacitance(s)
    d = np.abs(np.diag(C_ref)).max()
    gate = np.abs(C_ref) >= 1e-3 * d
    rel = np.abs(C - C_ref)[gate] / np.abs(C_ref)[gate]
    print(name, form, "C mixed max entry rel err", rel.max(), "ir", st["ir_steps"], st["iters"],
          "fp32 steps", st["steps_fp32"], flush=True)
    assert rel.max() < 1e-6


def test_unit_cube_16(dev):
    s = scenes.cube(16)
    P = _problem(s)
    C, st = P.capacitance(prec="fp64", rtol=1e-13)
    C_ref = oracle.solve_capacitance(s)
    assert abs(C[0, 0] / C_ref[0, 0] - 1) < 1e-10
    assert abs(C[0, 0] / (4 * np.pi * oracle.EPS0) / 0.66068 - 1) < 0.01


# x lengths 6 (one-stage plan), 90 (three stages) and 54 (two stages), with dielectric
# rows so the transposed product takes the six-input variant; and the lengths with
# compiled plans (36, 140, 270, 540, 1050: the fixed-plan kernels run whenever the
# configuration's plan is theirs, the generic kernel otherwise)
XPASS_SCENES = [
    ("x6", lambda: scenes.random_small(21, shape=(2, 6, 5), n_cond=1, n_diel=1)),
    ("x90", lambda: scenes.random_small(23, shape=(44, 5, 4), n_cond=2, n_diel=1)),
    ("x54", lambda: scenes.random_small(29, shape=(25, 4, 6), n_cond=2, n_diel=2)),
    ("x36", lambda: scenes.random_small(31, shape=(16, 5, 3), n_cond=2, n_diel=1)),
    ("x140", lambda: scenes.random_small(31, shape=(64, 5, 3), n_cond=2, n_diel=1)),
    ("x270", lambda: scenes.random_small(31, shape=(128, 5, 3), n_cond=2, n_diel=1)),
    ("x540", lambda: scenes.random_small(31, shape=(256, 5, 3), n_cond=2, n_diel=1)),
    ("x1050", lambda: scenes.random_small(31, shape=(512, 5, 3), n_cond=2, n_diel=1)),
]


# y lengths with compiled register-edge plans (36, 140, 270, 540, 1050)
YPASS_SCENES = [
    ("y36", lambda: scenes.random_small(37, shape=(5, 16, 7), n_cond=2, n_diel=1)),
    ("y140", lambda: scenes.random_small(37, shape=(5, 64, 7), n_cond=2, n_diel=1)),
    ("y270", lambda: scenes.random_small(37, shape=(5, 128, 7), n_cond=2, n_diel=1)),
    ("y540", lambda: scenes.random_small(37, shape=(5, 256, 7), n_cond=2, n_diel=1)),
    ("y1050", lambda: scenes.random_small(37, shape=(5, 512, 6), n_cond=2, n_diel=1)),
]


@pytest.mark.parametrize("name,make", YPASS_SCENES)
def test_ypass_compiled_plans_match_dense(dev, name, make):
    """The register-edge y pass on the lengths whose plans are compiled (the fixed-plan
    kernels), forward and transposed, in both precisions, against the dense product."""
    s = make()
    P = _problem(s, max_rhs=2)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, P.N))
    xt = torch.tensor(x, device=dev)
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        for transpose in (False, True):
            ref = ((A.T if transpose else A) @ x.T).T
            y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
            err = np.abs(y - ref).max() / np.abs(ref).max()
            print(name, prec, "T" if transpose else "F", P.fft_size(), f"{err:.2e}", flush=True)
            assert err < tol, (name, prec, transpose, err)
    rep = [l for l in P.tuning_report().splitlines() if l.startswith("y-pass")]
    print("\n".join(rep), flush=True)
    # at length 1050 an FP64 register-edge tile of two columns exceeds 64 KiB of LDS, so
    # the default there is the LDS-tile kernel (the autotuner may still pick one column)
    need = [l for l in rep if name != "y1050" or "fp32" in l]
    assert need and all("register-edge" in l for l in need), rep
    # pinned tile widths: one column per thread, and (FP32, even widths) two adjacent
    # columns per thread; a width that does not fit falls back to the default tile
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        for transpose in (False, True):
            ref = ((A.T if transpose else A) @ x.T).T
            for cols in (1, 2, 4, 8):
                for inverse in (False, True):
                    P.ypass_set(1, cols, -1, prec=prec, transpose=transpose, inverse=inverse, nrhs=2)
                y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
                err = np.abs(y - ref).max() / np.abs(ref).max()
                assert err < tol, (name, prec, transpose, cols, err)
        print(name, prec, "pinned widths 1, 2, 4, 8 within", tol, flush=True)


def test_ypass_xcd_groups_match_dense(dev):
    """The register-edge y pass with 1, 2, 4 or all column tiles of a row per XCD (a
    permutation of the workgroups over the tiles) and several tile widths, forward and
    transposed, both precisions, against the dense product.  The grid (9 tiles per row
    at 4 columns, 6 planes, 6 components, 2 right-hand sides = 648 workgroups) has both
    the permuted prefix and an unpermuted tail for a group of 4."""
    s = scenes.random_small(41, shape=(5, 20, 30), n_cond=2, n_diel=1)
    P = _problem(s, max_rhs=2)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, P.N))
    xt = torch.tensor(x, device=dev)
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        for transpose in (False, True):
            ref = ((A.T if transpose else A) @ x.T).T
            for cols in (2, 4, 8):
                for g in (1, 2, 4, -1):
                    for inverse in (False, True):
                        P.ypass_set(1, cols, g, prec=prec, transpose=transpose, inverse=inverse, nrhs=2)
                    y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
                    err = np.abs(y - ref).max() / np.abs(ref).max()
                    assert err < tol, (prec, transpose, cols, g, err)
            print(prec, "T" if transpose else "F", P.fft_size(), "all widths and groups within", tol, flush=True)
    from paper_2004_02609_amd import voxcap
    with pytest.raises(voxcap.VoxcapError):
        P.ypass_set(1, 4, 3, prec="fp32", nrhs=2)


@pytest.mark.parametrize("name,make", XPASS_SCENES)
def test_every_xpass_configuration_matches_dense(dev, name, make):
    """Each launch configuration the autotuner may pick (radix plan x column tile, per-RHS
    workgroups or the staged form) gives the dense product of eq. (4), forward and
    transposed, in both precisions."""
    s = make()
    P = _problem(s, max_rhs=2)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, P.N))
    xt = torch.tensor(x, device=dev)
    nplans = set()
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        for transpose in (False, True):
            ref = ((A.T if transpose else A) @ x.T).T
            cands = P.xpass_candidates(prec, transpose)
            assert cands, (name, prec, transpose)
            # stored spectra: the staged form (negative column count) is among them
            assert any(c[7] < 0 for c in cands), (name, prec, transpose, cands)
            for cfg in cands:
                nplans.add(cfg[0])
                P.xpass_set(cfg, prec, transpose, nrhs=2)
                y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
                err = np.abs(y - ref).max() / np.abs(ref).max()
                print(name, prec, "T" if transpose else "F", cfg, f"{err:.2e}", flush=True)
                assert err < tol, (name, prec, transpose, cfg, err)
    print(name, "stage counts covered", sorted(nplans), flush=True)


def test_autotuned_product_matches_dense(dev):
    s = scenes.random_small(29, shape=(25, 4, 6), n_cond=2, n_diel=2)
    P = _problem(s, max_rhs=2, autotune=True)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, P.N))
    xt = torch.tensor(x, device=dev)
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        for transpose in (False, True):
            ref = ((A.T if transpose else A) @ x.T).T
            for rep in range(2):   # first call tunes, second reuses the choice
                y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
                err = np.abs(y - ref).max() / np.abs(ref).max()
                assert err < tol, (prec, transpose, rep, err)
    rep = P.tuning_report()
    print(rep, flush=True)
    xlines = [l for l in rep.splitlines() if l.startswith("x-pass")]
    assert sum("tuned" in l for l in xlines) == 4, rep
    assert any(l.startswith("y-pass") for l in rep.splitlines()), rep
    # the tuning cache file: a second problem of the same shape adopts the four x-pass
    # and eight y-pass choices without timing and computes bitwise the same products
    import os
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tuning.txt")
        assert P.save_tuning(path) == 12
        assert P.save_tuning(path) == 12                     # merge replaces, never duplicates
        assert len(open(path).read().splitlines()) == 12
        Q = _problem(s, max_rhs=2, autotune=True)
        assert Q.load_tuning(path) == 12
        other = _problem(scenes.random_small(21, shape=(2, 6, 5), n_cond=1, n_diel=1), max_rhs=2)
        assert other.load_tuning(path) == 0                  # another shape takes nothing
        assert Q.load_tuning(os.path.join(d, "missing.txt")) == 0
    for prec in ("fp64", "fp32"):
        for transpose in (False, True):
            yq = Q.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
            yp = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
            assert np.array_equal(yq, yp), (prec, transpose)
    rq = Q.tuning_report()
    print(rq, flush=True)
    xq = [l for l in rq.splitlines() if l.startswith("x-pass")]
    yq = [l for l in rq.splitlines() if l.startswith("y-pass")]
    assert sum("cached" in l for l in xq) == 4 and sum("tuned" in l for l in xq) == 0, rq
    assert sum("cached" in l for l in yq) == 8 and sum("tuned" in l for l in yq) == 0, rq


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replayed_cycles_match_eager(dev, prec):
    """Restart cycles replayed from one captured graph (GMRES(5): many replays, host
    reads and eager work between them) give bitwise the eager result, which matches
    the oracle."""
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    P = _problem(s)
    Cg, stg = P.capacitance(prec=prec, rtol=1e-11, restart=5, graph=True)
    Ce, ste = P.capacitance(prec=prec, rtol=1e-11, restart=5, graph=False)
    print(prec, "iters graph", stg["iters"], "eager", ste["iters"], flush=True)
    assert stg["iters"] == ste["iters"]
    assert np.array_equal(Cg, Ce)
    C_ref = oracle.solve_capacitance(s)
    err = np.abs(Cg - C_ref).max() / np.abs(C_ref).max()
    assert err < 1e-9, err
    # a second graph solve reuses the cached graph and reproduces the first
    Cg2, _ = P.capacitance(prec=prec, rtol=1e-11, restart=5, graph=True)
    assert np.array_equal(Cg, Cg2)
