"""GPU checks of the Tucker form (eq. 13): spectra compressed at setup and rebuilt on the
matrix cores before every product.

The truncation keeps ||X - X_hat|| <= tol ||X|| per stored pair, so the product
differs from the uncompressed one by ~tol relative; the spectra buffers start as NaN,
so a product that skipped the rebuild cannot pass.  Capacitance in mixed precision is
gated at 1e-6 against the FP64 oracle (the spec bar for the compressed, mixed
path); FP64 parity itself is tested uncompressed elsewhere."""
import numpy as np
import pytest

import oracle
import scenes
from helpers import oracle_matrix_library_order

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    ("s5", lambda: scenes.random_small(5, n_cond=2, n_diel=2)),
    ("s9", lambda: scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)),
    ("cube6", lambda: scenes.cube(6, 1.0)),
]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("tol", [1e-10, 1e-6])
def test_tucker_product_matches_dense(dev, name, make, tol):
    from paper_2004_02609_amd import voxcap
    s = make()
    P = voxcap.Problem.from_scene(s).setup(tucker_tol=tol, max_rhs=2)
    A, po, perm = oracle_matrix_library_order(s, P.panels())
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, P.N))
    xt = torch.tensor(x, device=dev)
    info = P.tucker_info()
    print(name, tol, "ranks", info["ranks"], "CR", info["compression_ratio"], flush=True)
    assert info["npairs"] == (15 if P.n_diel else 6)
    for transpose in (False, True):
        ref = ((A.T if transpose else A) @ x.T).T
        for prec, base in (("fp64", 1e-11), ("fp32", 2e-5)):
            y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
            err = np.abs(y - ref).max() / np.abs(ref).max()
            print(name, tol, prec, "T" if transpose else "F", f"{err:.2e}", flush=True)
            assert np.isfinite(err) and err < base + 50 * tol, (name, tol, prec, transpose, err)


def test_tucker_mixed_capacitance_within_1e6(dev):
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    P = voxcap.Problem.from_scene(s).setup(tucker_tol=1e-8)
    C, st = P.capacitance(prec="mixed", rtol=1e-10)
    C_ref = oracle.solve_capacitance(s)
    err = np.abs(C - C_ref).max() / np.abs(C_ref).max()
    info = P.tucker_info()
    print("mixed + Tucker 1e-8: C rel err", err, "CR", info["compression_ratio"], "rank max", st, flush=True)
    assert err < 1e-6
    assert info["compression_ratio"] > 1.0
