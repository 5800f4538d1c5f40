"""GPU checks of the packed set: problems of uneven size solved as one, each pass of the
product one launch over all members (workgroups split between members by a device
table).  The packed product must equal every member's own product to rounding (same
tiles, plans and arithmetic), and the packed capacitance matrices must match each
member's own solve and the FP64 oracle."""
import numpy as np
import pytest

import oracle
import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _uneven():
    return [scenes.random_small(31, shape=(6, 9, 7), n_cond=1, n_diel=0),
            scenes.random_small(32, shape=(12, 8, 10), n_cond=3, n_diel=2),
            scenes.random_small(33, shape=(9, 13, 6), n_cond=2, n_diel=1),
            scenes.cube(5, 1.0),
            scenes.random_small(34, shape=(14, 11, 9), n_cond=4, n_diel=2)]


def _packed_x(probs, rows, seed):
    rng = np.random.default_rng(seed)
    cols = sum(P.m for P in probs)
    x = np.zeros((cols, rows))
    c = 0
    for P in probs:
        x[c:c + P.m, :P.N] = rng.standard_normal((P.m, P.N))
        c += P.m
    return x


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_packed_product_equals_member_products(dev, prec):
    from paper_2004_02609_amd import voxcap
    ss = _uneven() + scenes.uneven_batch(3, lo=16, hi=28)
    probs = [voxcap.Problem.from_scene(s).setup(autotune=False) for s in ss]
    pk = voxcap.Pack(probs)
    inf = pk.info()
    print(inf, flush=True)
    assert inf["members"] == len(probs) and inf["columns"] == sum(P.m for P in probs)
    assert inf["rows"] == max(P.N for P in probs)
    assert inf["launches_fp64"] >= 5
    x = _packed_x(probs, inf["rows"], 5)
    y = pk.apply(torch.tensor(x, device=dev), prec=prec).cpu().numpy()
    # same tiles, plans and arithmetic per member; the two launches are compiled apart,
    # so the rounding may differ by an ulp or so (an indexing slip would be O(1))
    tol = 1e-14 if prec == "fp64" else 2e-6
    c = 0
    for k, P in enumerate(probs):
        ref = P.apply(torch.tensor(x[c:c + P.m, :P.N], device=dev), prec=prec).cpu().numpy()
        err = np.abs(y[c:c + P.m, :P.N] - ref).max() / np.abs(ref).max()
        print(k, ss[k]["name"], "N", P.N, "m", P.m, "rel diff", err, flush=True)
        assert err <= tol, (k, err)
        assert not np.any(y[c:c + P.m, P.N:]), k   # padding rows untouched (zero)
        c += P.m


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_batch_matches_individual_and_oracle(dev, prec, tol):
    from paper_2004_02609_amd import voxcap
    ss = _uneven()
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    Cb, stb = voxcap.capacitance_batch(probs, prec=prec, rtol=1e-11)
    for k, (s, P) in enumerate(zip(ss, probs)):
        Ci, sti = P.capacitance(prec=prec, rtol=1e-11)
        print(k, prec, "iters packed", stb[k]["iters"], "alone", sti["iters"], flush=True)
        rel = np.abs(Cb[k] - Ci).max() / np.abs(Ci).max()
        assert rel < (1e-10 if prec == "fp64" else 1e-6), (k, rel)
        C_ref = oracle.solve_capacitance(s)
        d = np.abs(np.diag(C_ref)).max()
        gate = np.abs(C_ref) >= 1e-3 * d
        err = (np.abs(Cb[k] - C_ref)[gate] / np.abs(C_ref)[gate]).max()
        print(k, prec, "C rel err vs oracle", err, flush=True)
        assert err < tol, (k, err)
        assert max(stb[k]["final_rre"]) <= 1e-11


def test_pack_replay_is_deterministic_and_matches_one_by_one(dev):
    from paper_2004_02609_amd import voxcap
    ss = scenes.uneven_batch(6, lo=16, hi=40)
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    pk = voxcap.Pack(probs)
    C1, st1 = pk.capacitance(prec="mixed", rtol=1e-9)     # captures the cycle graphs
    C2, st2 = pk.capacitance(prec="mixed", rtol=1e-9)     # replays them
    for k, P in enumerate(probs):
        assert np.array_equal(C1[k], C2[k]), k
        Ci, _ = P.capacitance(prec="mixed", rtol=1e-9)
        rel = np.abs(C1[k] - Ci).max() / np.abs(Ci).max()
        print(k, ss[k]["name"], "m", P.m, "N", P.N, "iters", st1[k]["iters"], "rel", rel, flush=True)
        assert rel < 1e-7, (k, rel)
        # Maxwell capacitance matrix: positive diagonal, non-positive off-diagonal
        assert np.all(np.diag(C1[k]) > 0)
        off = C1[k] - np.diag(np.diag(C1[k]))
        assert np.all(off <= 1e-9 * np.abs(np.diag(C1[k])).max())
