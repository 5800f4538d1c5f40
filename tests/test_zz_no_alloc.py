"""vc_capacitance_static (no device allocation: the solve's arrays live in the library's
static scratch) against vc_capacitance, through the C ABI.

Both run the same kernels on the same problem; the static call issues the restart
cycles eagerly instead of replaying captured graphs.  Bars: FP64 1e-10 and mixed 1e-6
per gated entry (|C_ij| >= 1e-3 max |C_ii|), the solve's own FP64 / mixed bars; the
charges likewise (relative to max |rho|).  Two calls in a row share the scratch, the
second on a smaller problem, so stale contents of the first must not leak into it.
"""
import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gated_err(C, Cref):
    gate = np.abs(Cref) >= 1e-3 * np.abs(np.diag(Cref)).max()
    return float((np.abs(C - Cref)[gate] / np.abs(Cref)[gate]).max())


def _problem(s):
    from paper_2004_02609_amd import voxcap
    return voxcap.Problem.from_scene(s).setup()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_static_matches_capacitance_two_calls(dev, prec, tol):
    big = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    small = scenes.random_small(5, shape=(8, 7, 6), n_cond=2, n_diel=1)
    probs = [_problem(big), _problem(small)]
    assert probs[1].N < probs[0].N
    for P in probs:
        print(f"static solve {prec}: N={P.N} m={P.m}", flush=True)
        rho_ref = torch.zeros(P.m, P.N, dtype=torch.float64, device=dev)
        rho_st = torch.full((P.m, P.N), float("nan"), dtype=torch.float64, device=dev)
        C_ref, _ = P.capacitance(prec=prec, rtol=1e-12, rho=rho_ref)
        C_st, st = P.capacitance_static(prec=prec, rtol=1e-12, rho=rho_st)
        torch.cuda.synchronize()
        assert np.isfinite(C_st).all()
        e = _gated_err(C_st, C_ref)
        er = float((rho_st - rho_ref).abs().max() / rho_ref.abs().max())
        print(f"  C err {e:.2e}, rho err {er:.2e}, iters {st['iters']}", flush=True)
        assert e <= tol, e
        assert er <= tol, er


def test_static_then_regular_solve_unchanged(dev):
    """A static call leaves the problem's own workspace (and its captured graphs) as it
    was: the regular solve after it gives the regular solve's result bitwise."""
    P = _problem(scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1))
    C1, _ = P.capacitance(prec="fp64", rtol=1e-12)
    C2, _ = P.capacitance_static(prec="fp64", rtol=1e-12)
    C3, _ = P.capacitance(prec="fp64", rtol=1e-12)
    assert np.array_equal(C1, C3)
    assert _gated_err(C2, C1) <= 1e-10


def test_static_rejects_oversized_solve(dev):
    """A solve whose arrays exceed the static scratch is refused before any GPU work."""
    from paper_2004_02609_amd import voxcap
    P = _problem(scenes.random_small(5, shape=(8, 7, 6), n_cond=2, n_diel=1))
    with pytest.raises(voxcap.VoxcapError) as ei:
        P.capacitance_static(prec="fp64", rtol=1e-12, restart=3000)
    assert ei.value.status == voxcap.VC_ERR_ARG
    assert "static array holds" in str(ei.value)
    # the problem stays usable
    C, _ = P.capacitance_static(prec="fp64", rtol=1e-12)
    assert np.isfinite(C).all()
