"""GPU parity of the Toeplitz setup path (Sec. II.C, Tab. I) with the oracle.

* The octants the library fills from the panel integrals match the oracle's (the two
  integral routes differ by rounding, ~1e-14 relative; 1e-12 of the largest entry).
* A cache compressed at tol over a largest grid and restored for a smaller one is
  within tol * ||octant over the largest grid|| (Frobenius, per pair) of the oracle's
  octant of the smaller grid, plus the integrals' rounding.
* Saving and loading a cache gives bit-identical restores.
* A problem set up from the cache applies eq. (4) within the error the compression
  allows: a row of the operator holds each offset of a pair once and meets at most
  three pairs, so |dy_i| <= sqrt(3) * tol * max_q ||T_q|| * ||x||_2 on top of the
  direct setup's 1e-11 of max|y|.  Its capacitance matches the oracle's LU solve.
"""
import os

import numpy as np
import pytest

import oracle
import scenes
from helpers import oracle_matrix_library_order
from oracle import toeplitz as otz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NMAX = (18, 16, 14)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def oracle_norms():
    return np.array([np.linalg.norm(otz.octant(q, NMAX)) for q in range(15)])


@pytest.fixture(scope="module")
def caches(dev):
    from paper_2004_02609_amd import voxcap
    out = {tol: voxcap.ToeplitzCache.build(NMAX, tol) for tol in (1e-12, 1e-6)}
    yield out
    for c in out.values():
        c.close()


def test_octant_fill_matches_oracle(dev):
    from paper_2004_02609_amd import voxcap
    for n in [(6, 5, 4), (1, 3, 2)]:
        for q in range(15):
            got = voxcap.toeplitz_octant(q, n).cpu().numpy()
            ref = otz.octant(q, n)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err < 1e-12, (n, q, err)
    print("octant fill: all 15 pairs within 1e-12", flush=True)


def test_cache_restore_matches_oracle(dev, caches, oracle_norms):
    for tol, cache in caches.items():
        info = cache.info()
        assert info["nmax"] == NMAX and info["tol"] == tol
        print("tol", tol, "ranks", info["ranks"], "compression ratio", round(info["compression_ratio"], 1),
              "build s", round(info["seconds"], 3), flush=True)
        for n in [NMAX, (9, 14, 5), (1, 1, 1)]:
            for q in range(15):
                got = cache.restore(q, n).cpu().numpy()
                ref = otz.octant(q, n)
                err = np.linalg.norm(got - ref)
                bound = tol * oracle_norms[q] + 1e-12 * np.abs(ref).max() * np.sqrt(ref.size)
                assert err <= bound, (tol, n, q, err, bound)
        if tol == 1e-6:
            # a real compression: fewer stored numbers than the octants
            assert info["compression_ratio"] > 2


def test_cache_save_load_roundtrip(dev, caches, tmp_path):
    from paper_2004_02609_amd import voxcap
    cache = caches[1e-6]
    path = os.path.join(str(tmp_path), "toeplitz.vct")
    cache.save(path)
    back = voxcap.ToeplitzCache.load(path)
    try:
        a, b = cache.info(), back.info()
        for k in ("nmax", "tol", "ranks", "stored_numbers"):
            assert a[k] == b[k], k
        for q in (0, 4, 9, 14):
            assert torch.equal(cache.restore(q, (7, 3, 9)), back.restore(q, (7, 3, 9)))
    finally:
        back.close()


def test_cache_errors(dev, caches):
    from paper_2004_02609_amd import voxcap
    cache = caches[1e-6]
    with pytest.raises(voxcap.VoxcapError) as e:
        cache.restore(0, (NMAX[0] + 1, 2, 2))
    assert e.value.status == voxcap.VC_ERR_ARG
    with pytest.raises(voxcap.VoxcapError) as e:
        cache.restore(15, (2, 2, 2))
    assert e.value.status == voxcap.VC_ERR_ARG
    big = scenes.random_small(3, shape=(NMAX[0] + 2, 6, 6), n_cond=1, n_diel=0)
    P = voxcap.Problem.from_scene(big)
    with pytest.raises(voxcap.VoxcapError) as e:
        P.set_toeplitz_source(cache)
    assert e.value.status == voxcap.VC_ERR_ARG
    with pytest.raises(voxcap.VoxcapError) as e:
        voxcap.ToeplitzCache.build((0, 4, 4), 1e-6)
    assert e.value.status == voxcap.VC_ERR_ARG


CACHE_SCENES = [
    ("small_s5", lambda: scenes.random_small(5, n_cond=2, n_diel=2)),
    ("ragged", lambda: scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1)),
    ("at_nmax", lambda: scenes.random_small(21, shape=NMAX, n_cond=2, n_diel=1)),
]


@pytest.mark.parametrize("name,make", CACHE_SCENES)
def test_product_from_cache_matches_dense(dev, caches, oracle_norms, name, make):
    from paper_2004_02609_amd import voxcap
    s = make()
    rng = np.random.default_rng(2)
    for tol in (1e-12, 1e-6):
        P = voxcap.Problem.from_scene(s)
        P.set_toeplitz_source(caches[tol])
        P.setup(max_rhs=2)
        A, _, _ = oracle_matrix_library_order(s, P.panels())
        x = rng.standard_normal((2, P.N))
        y = P.apply(torch.tensor(x, device=dev), prec="fp64").cpu().numpy()
        ref = (A @ x.T).T
        err = np.abs(y - ref).max(axis=1)
        bound = np.sqrt(3) * tol * oracle_norms.max() * np.linalg.norm(x, axis=1) + 1e-11 * np.abs(ref).max()
        t = P.setup_time()
        print(name, "tol", tol, "max err", err.max(), "bound", bound.min(), "setup s", round(t["total_s"], 4),
              "toeplitz s", round(t["toeplitz_s"], 4), flush=True)
        assert (err <= bound).all(), (name, tol, err, bound)


@pytest.mark.parametrize("name,make", CACHE_SCENES[:2])
def test_capacitance_from_cache(dev, caches, name, make):
    from paper_2004_02609_amd import voxcap
    s = make()
    C_ref = oracle.solve_capacitance(s)
    d = np.abs(np.diag(C_ref)).max()
    for tol, gate in ((1e-12, 1e-10), (1e-6, 1e-4)):
        P = voxcap.Problem.from_scene(s)
        P.set_toeplitz_source(caches[tol])
        P.setup()
        C, st = P.capacitance(prec="fp64", rtol=1e-13)
        g = np.abs(C_ref) >= 1e-3 * d
        rel = (np.abs(C - C_ref)[g] / np.abs(C_ref)[g]).max()
        err = np.abs(C - C_ref).max() / d
        print(name, "tol", tol, "C max entry rel err", rel, "normwise", err, flush=True)
        assert rel < gate, (name, tol, rel)
        assert err < gate, (name, tol, err)


def _precond_reference(A, pan, x, nv):
    """Eq. (14) from the dense oracle matrix: every box of nv voxels solves the block of
    the conductor panels of its conductor voxels, dielectric panels divide by their
    diagonal entry."""
    N = len(pan)
    cond = pan["kind"] == 0
    vox = np.stack([pan["i"], pan["j"], pan["k"]], 1).astype(int)
    vox[np.arange(N), pan["dir"]] -= (pan["eps_lo"] == 0.0).astype(int)
    box = vox // nv
    ref = np.zeros_like(x)
    ref[:, ~cond] = x[:, ~cond] / np.diag(A)[~cond]
    keys = {}
    for p in np.nonzero(cond)[0]:
        keys.setdefault(tuple(box[p]), []).append(p)
    for idx in keys.values():
        idx = np.array(idx)
        ref[:, idx] = np.linalg.solve(A[np.ix_(idx, idx)], x[:, idx].T).T
    return ref


def test_precond_from_cache_matches_dense(dev, caches):
    """Setup from a cache reads the preconditioner's lag tables from its octants too.
    The blocks are then within tol of the oracle's, so the apply agrees with the dense
    block solves to about tol times the blocks' condition number."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    rng = np.random.default_rng(4)
    for tol, gate in ((1e-12, 1e-9), (1e-6, 1e-3)):
        P = voxcap.Problem.from_scene(s)
        P.set_toeplitz_source(caches[tol])
        P.setup(nv=(4, 4, 4))
        A, _, _ = oracle_matrix_library_order(s, P.panels())
        x = rng.standard_normal((2, P.N))
        y = P.apply_precond(torch.tensor(x, device=dev)).cpu().numpy()
        ref = _precond_reference(A, P.panels(), x, 4)
        err = float(np.abs(y - ref).max() / np.abs(ref).max())
        print("precond from cache, tol", tol, "rel err vs dense blocks", err, flush=True)
        assert err < gate, (tol, err)
