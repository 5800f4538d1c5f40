"""GPU checks of the two mixed-precision forms of the capacitance solve.

refinement: FP32-product GMRES inside FP64 iterative refinement.
relaxed: one GMRES on the FP64 system, restarted from FP64 residuals, whose Arnoldi
products switch from FP64 to FP32 once the residual estimate is below rtol / inner_rtol
(the product error a step can afford grows as the residual shrinks).

Both stop on the FP64 true residual, so at a tight rtol both must reach what the FP64
solve reaches: C entrywise within 1e-10 of the FP64 oracle (eq. 8) on the gated entries
(|C_ij| >= 1e-3 max C_ii).
"""
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


def _gated_rel(C, ref):
    gate = np.abs(ref) >= 1e-3 * np.abs(np.diag(ref)).max()
    return (np.abs(C - ref)[gate] / np.abs(ref)[gate]).max()


SCENES = [
    ("s5", lambda: scenes.random_small(5, n_cond=2, n_diel=2)),
    ("s9", lambda: scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)),
]


@pytest.mark.parametrize("name,make", SCENES)
@pytest.mark.parametrize("form", ["refinement", "relaxed"])
def test_tight_rtol_reaches_fp64(dev, name, make, form):
    """At rtol 1e-12 either form's C matches the FP64 oracle to 1e-10 entrywise; the
    relaxed form takes some steps in FP64 (the first ones) and some in FP32."""
    from paper_2004_02609_amd import voxcap
    s = make()
    P = voxcap.Problem.from_scene(s).setup()
    C, st = P.capacitance(prec="mixed", rtol=1e-12, mixed_form=form)
    ref = oracle.solve_capacitance(s)
    err = _gated_rel(C, ref)
    total = max(st["iters"])
    print(name, form, "err", err, "iters", st["iters"], "fp32 steps", st["steps_fp32"], "ir", st["ir_steps"],
          flush=True)
    assert st["mixed_form"] == form
    assert err < 1e-10
    assert all(r <= 1e-12 for r in st["final_rre"])
    assert st["steps_fp32"] > 0
    if form == "relaxed":
        # FP64 products until the estimate reaches rtol / inner_rtol = 1e-6
        assert st["steps_fp32"] < total
        assert st["ir_steps"] == 0


def test_auto_form_follows_the_product_size(dev):
    """mixed_form "auto": a product whose FP64 bytes fit VC_MIXED_RELAXED_MAX_BYTES
    (every small scene) runs the relaxed form; its C equals an explicit relaxed solve's
    bitwise (same steps, same precisions)."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(5, n_cond=2, n_diel=2)
    P = voxcap.Problem.from_scene(s).setup()
    Ca, sta = P.capacitance(prec="mixed", rtol=1e-9)
    Cr, str_ = P.capacitance(prec="mixed", rtol=1e-9, mixed_form="relaxed")
    assert sta["bytes_model"] * 2 <= 256 * 2 ** 20   # FP32 model; FP64 moves twice the bytes
    assert sta["mixed_form"] == "relaxed"
    assert np.array_equal(Ca, Cr)
    assert sta["iters"] == str_["iters"] and sta["steps_fp32"] == str_["steps_fp32"]


def test_relaxed_graph_replay_matches_eager(dev):
    """The relaxed form's segments are captured per precision; the replayed solve gives
    bitwise the eager one's C and iteration counts (the precision choices are the same)."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    P = voxcap.Problem.from_scene(s).setup()
    Ce, ste = P.capacitance(prec="mixed", rtol=1e-11, mixed_form="relaxed", graph=False)
    for _ in range(2):   # the first captures, the second replays
        Cg, stg = P.capacitance(prec="mixed", rtol=1e-11, mixed_form="relaxed")
        assert np.array_equal(Cg, Ce)
        assert stg["iters"] == ste["iters"] and stg["steps_fp32"] == ste["steps_fp32"]


def test_relaxed_packed_batch(dev):
    """The packed solve of uneven scenes in the relaxed form: every member's C matches
    its FP64 oracle to 1e-10 at rtol 1e-12."""
    from paper_2004_02609_amd import voxcap
    ss = [scenes.random_small(5, n_cond=2, n_diel=1), scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1)]
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    Cs, sts = voxcap.capacitance_batch(probs, prec="mixed", rtol=1e-12, mixed_form="relaxed")
    for C, st, s in zip(Cs, sts, ss):
        assert st["mixed_form"] == "relaxed"
        assert _gated_rel(C, oracle.solve_capacitance(s)) < 1e-10


def test_mixed_form_rejects_unknown(dev):
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(5, n_cond=2, n_diel=1)
    P = voxcap.Problem.from_scene(s).setup()
    o = voxcap._solve_opts(prec="mixed", rtol=1e-8)
    o.mixed_form = 3
    import ctypes as C
    Cm = np.zeros((P.m, P.m))
    rc = voxcap._lib.vc_capacitance(P._h, C.byref(o), Cm.ctypes.data_as(C.POINTER(C.c_double)), None, None)
    assert rc == voxcap.VC_ERR_ARG
    assert b"mixed_form" in voxcap._lib.vc_last_error()
