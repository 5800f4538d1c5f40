"""GPU checks of the differentiation form: dC/d eps by the adjoint method (transposed FFT
product inside GMRES, assembled on the GPU) against the FP64 oracle's adjoint LU
gradient and against central finite differences; dC/d(charges) against the explicit
linear map of eq. (8).

Tolerances: the FP64 solves stop at 1e-12 relative residual, so the adjoint gradient
matches the dense one to ~1e-9 relative; central differences with step 1e-4 carry a
truncation error ~h^2 |C'''| ~ 1e-8 relative, and the spec bar is 1e-5."""
import numpy as np
import pytest

import oracle
import scenes
from oracle import dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _two_block_scene():
    s = scenes.random_small(21, shape=(7, 6, 6), n_cond=2, n_diel=0)
    blk = np.full(s["cond_id"].shape, -1, np.int32)
    eps = s["eps_r"].copy()
    eps[:, :, :3] = 3.0
    blk[:, :, :3] = 0
    eps[:, :3, 3:] = 6.0
    blk[:, :3, 3:] = 1
    blk[s["cond_id"] >= 0] = -1
    return dict(s, eps_r=eps), blk


def test_grad_eps_matches_oracle_adjoint(dev):
    from paper_2004_02609_amd import voxcap
    s, blk = _two_block_scene()
    P = voxcap.Problem.from_scene(s).setup()
    dC, Cm, st = P.capacitance_grad_eps(blk, 2, prec="fp64", rtol=1e-12)
    g_ref, C_ref = dense.capacitance_gradient(s, blk, 2)
    errC = np.abs(Cm - C_ref).max() / np.abs(C_ref).max()
    errg = np.abs(dC - g_ref).max() / np.abs(g_ref).max()
    print("C rel err", errC, "dC/deps rel err", errg, flush=True)
    assert errC < 1e-10
    assert errg < 1e-8


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-5), ("mixed", 1e-5)])
def test_autograd_eps_matches_central_differences(dev, prec, tol):
    from paper_2004_02609_amd.autograd import capacitance_eps
    s, blk = _two_block_scene()
    e0 = torch.tensor([3.0, 6.0], dtype=torch.float64, requires_grad=True)
    m = int(s["cond_id"].max()) + 1
    G = torch.tensor(np.random.default_rng(5).standard_normal((m, m)))
    C = capacitance_eps(s, blk, e0, prec=prec, rtol=1e-12 if prec == "fp64" else 1e-11)
    (C * G).sum().backward()
    g = e0.grad.numpy()
    h = 1e-4
    fd = np.zeros(2)
    for b in range(2):
        ep = e0.detach().clone()
        ep[b] += h
        em = e0.detach().clone()
        em[b] -= h
        cp = capacitance_eps(s, blk, ep, prec="fp64", rtol=1e-13).numpy()
        cm = capacitance_eps(s, blk, em, prec="fp64", rtol=1e-13).numpy()
        fd[b] = ((cp - cm) / (2 * h) * G.numpy()).sum()
    err = np.abs(g - fd) / np.abs(fd).max()
    print(prec, "autograd", g, "central differences", fd, "rel err", err, flush=True)
    assert err.max() < tol, (g, fd)


def test_charges_to_capacitance_and_adjoint(dev):
    from paper_2004_02609_amd import voxcap
    from paper_2004_02609_amd.autograd import charges_to_capacitance
    s = scenes.random_small(5, n_cond=2, n_diel=2)
    P = voxcap.Problem.from_scene(s).setup()
    pan = P.panels()
    N, m = P.N, P.m
    rng = np.random.default_rng(6)
    nrhs = 3
    rho = torch.tensor(rng.standard_normal((nrhs, N)), device=dev, requires_grad=True)
    C = charges_to_capacitance(P, rho)
    # explicit map of eq. (8): W[i, k] = 4 pi eps0 dv eps_adj(k) on the panels of conductor i
    W = np.zeros((m, N))
    cond = pan["kind"] == 0
    W[pan["cond"][cond], np.nonzero(cond)[0]] = pan["eps_adj"][cond]
    W *= 4 * np.pi * oracle.EPS0 * s["dv"]
    ref = W @ rho.detach().cpu().numpy().T
    assert np.allclose(C.detach().cpu().numpy(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    gC = torch.tensor(rng.standard_normal((m, nrhs)), device=dev)
    C.backward(gC)
    gref = (W.T @ gC.cpu().numpy()).T
    assert np.allclose(rho.grad.cpu().numpy(), gref, rtol=1e-13, atol=1e-13 * np.abs(gref).max())
    # the capacitance solve's own charges reproduce its C through the same map
    rho_dev = torch.empty(m, N, dtype=torch.float64, device=dev)
    Cm, st = voxcap.vc_capacitance(P._h, m, rho=rho_dev, prec="fp64", rtol=1e-12)[:2]
    C2 = charges_to_capacitance(P, rho_dev).cpu().numpy()
    assert np.allclose(C2, Cm, rtol=1e-12, atol=1e-14 * np.abs(Cm).max())


def test_update_eps_matches_fresh_setup(dev):
    """New permittivities written into a set-up problem (eq. 7 jump terms, eq. 8 weights,
    the preconditioner's dielectric diagonal) give the product, preconditioner and
    capacitance of a problem set up from scratch with them, and the oracle's C; an
    update that would change the panel list is refused and changes nothing."""
    from paper_2004_02609_amd import voxcap
    s, blk = _two_block_scene()
    e2 = s["eps_r"].copy()
    e2[blk == 0] = 4.5
    e2[blk == 1] = 2.5
    s2 = dict(s, eps_r=e2)
    P = voxcap.Problem.from_scene(s).setup(max_rhs=2)
    C1, _ = P.capacitance(prec="fp64", rtol=1e-13)          # captures graphs on the old values
    P.apply_precond_kind(3, torch.zeros(1, P.N, dtype=torch.float64, device=dev))   # builds kind 3
    P.update_eps(e2)
    Q = voxcap.Problem.from_scene(s2).setup(max_rhs=2)
    x = torch.tensor(np.random.default_rng(8).standard_normal((2, P.N)), device=dev)
    for prec in ("fp64", "fp32"):
        for tr in (False, True):
            a, b = P.apply(x, prec=prec, transpose=tr), Q.apply(x, prec=prec, transpose=tr)
            assert torch.equal(a, b), (prec, tr, float((a - b).abs().max()))
    for kind in (1, 2, 3):
        a, b = P.apply_precond_kind(kind, x), Q.apply_precond_kind(kind, x)
        assert float((a - b).abs().max() / b.abs().max()) < 1e-14, kind
    CP, _ = P.capacitance(prec="fp64", rtol=1e-13)
    CQ, _ = Q.capacitance(prec="fp64", rtol=1e-13)
    C_ref = oracle.solve_capacitance(s2)
    d = np.abs(np.diag(C_ref)).max()
    gate = np.abs(C_ref) >= 1e-3 * d
    print("updated vs fresh", np.abs(CP - CQ).max() / d, "vs oracle",
          (np.abs(CP - C_ref)[gate] / np.abs(C_ref)[gate]).max(), "old C moved", np.abs(CP - C1).max() / d, flush=True)
    assert np.array_equal(CP, CQ)
    assert (np.abs(CP - C_ref)[gate] / np.abs(C_ref)[gate]).max() < 1e-10
    CM, _ = P.capacitance(prec="mixed", rtol=1e-10)
    assert (np.abs(CM - C_ref)[gate] / np.abs(C_ref)[gate]).max() < 1e-6
    # a block set to the background permittivity would remove dielectric panels
    e3 = e2.copy()
    e3[blk == 0] = s["eps_b"]
    with pytest.raises(voxcap.VoxcapError) as ei:
        P.update_eps(e3)
    assert ei.value.status == voxcap.VC_ERR_ARG
    CP2, _ = P.capacitance(prec="fp64", rtol=1e-13)
    assert np.array_equal(CP2, CP)
