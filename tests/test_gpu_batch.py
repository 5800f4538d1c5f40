"""GPU checks of the batched form: problems of uneven size solved together, one graph
launch per round over every unfinished problem.  Each problem's C must equal its own
solve (the batch replays the same captured cycles) and the FP64 oracle."""
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_batch_matches_individual_and_oracle(dev, prec, tol):
    from paper_2004_02609_amd import voxcap
    ss = _uneven()
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    Cb, stb = voxcap.capacitance_batch(probs, prec=prec, rtol=1e-11)
    for k, (s, P) in enumerate(zip(ss, probs)):
        Ci, sti = P.capacitance(prec=prec, rtol=1e-11)
        print(k, prec, "iters batch", stb[k]["iters"], "alone", sti["iters"], flush=True)
        if prec == "fp64":
            assert np.array_equal(Cb[k], Ci), k
        C_ref = oracle.solve_capacitance(s)
        d = np.abs(np.diag(C_ref)).max()
        gate = np.abs(C_ref) >= 1e-3 * d
        err = (np.abs(Cb[k] - C_ref)[gate] / np.abs(C_ref)[gate]).max()
        print(k, prec, "C rel err vs oracle", err, flush=True)
        assert err < tol, (k, err)
