"""GPU checks of the Tucker form (eq. 13): spectra compressed at setup and never stored
whole.  Each product rebuilds the strips T1 = S x3 U3 and T2 = T1 x2 U2 on the matrix
cores, and each x-pass workgroup builds its tile's spectra X = U1 T2 into LDS.

The truncation keeps ||X - X_hat|| <= tol ||X|| per stored pair, so the product
differs from the uncompressed one by about tol relative (measured: below 3 tol).
Capacitance in mixed precision is gated at 1e-6 against the FP64 oracle (the
spec bar for the compressed, mixed path); FP64 parity itself is tested
uncompressed elsewhere."""
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
    # nothing of the size of the spectra is resident: exactly the cores and factors (FP64
    # and FP32, U1 in FP64 only), the FP64 copy of U1 with rows padded to r1p = r1
    # rounded up to 4, the FP32 copy transposed with r1 rounded up to 16 and Hx to 64,
    # the strip T1 (r1 r2 x H, FP64 elements) and T2 (Hy x H x r1p) in each precision
    Mx, My, Mz = P.fft_size()
    Hx, Hy, H = Mx // 2 + 1, My // 2 + 1, Mz // 2 + 1
    expect = 0.0
    for r1, r2, r3 in info["ranks"]:
        r1p = (r1 + 3) // 4 * 4
        r1q, hxp = (r1 + 15) // 16 * 16, (Hx + 63) // 64 * 64
        expect += (r1 * r2 * r3 + Hy * r2 + H * r3) * 12.0 + Hx * r1 * 8.0 + Hx * r1p * 8.0 + r1q * hxp * 4.0
        expect += r1 * r2 * H * 8.0 + Hy * H * r1p * 12.0
    resident = P.spectra_bytes()
    print(name, tol, f"resident {resident:.0f} B, uncompressed {info['full_numbers'] * 12:.0f} B", flush=True)
    assert resident == expect
    for transpose in (False, True):
        ref = ((A.T if transpose else A) @ x.T).T
        for prec, base in (("fp64", 1e-11), ("fp32", 2e-5)):
            y = P.apply(xt, transpose=transpose, prec=prec).cpu().numpy()
            err = np.abs(y - ref).max() / np.abs(ref).max()
            print(name, tol, prec, "T" if transpose else "F", f"{err:.2e}", flush=True)
            assert np.isfinite(err) and err < base + 10 * tol, (name, tol, prec, transpose, err)


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
