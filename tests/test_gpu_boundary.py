"""GPU checks of the C-ABI calls that follow the problem statement's interface (Sec. II.A):
the tuning cache named in the setup options, the byte model reported with a solve, the
batched call under both of its names, and the one-call Python form.  Results are
compared with the calls they alias, and capacitance with the FP64 oracle."""
import ctypes as C
import os
import tempfile

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


def test_setup_tune_cache_saves_and_loads(dev):
    """tune_cache in the setup options: the first problem's timed x- and y-pass choices
    land in the file; a second problem of the same shape loads them at setup (no timing)
    and computes bitwise the same products."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        P = voxcap.Problem.from_scene(s).setup(max_rhs=2, autotune=True, tune_cache=path)
        x = torch.tensor(np.random.default_rng(3).standard_normal((2, P.N)), device=dev)
        yp = {}
        for prec in ("fp64", "fp32"):
            for transpose in (False, True):
                yp[prec, transpose] = P.apply(x, transpose=transpose, prec=prec).cpu().numpy()
        assert os.path.exists(path)
        lines = open(path).read().splitlines()
        # x: 2 precisions x 2 directions; y: the same x forward / inverse transforms
        assert sum(l.startswith("vc-xpass") for l in lines) == 4, lines
        assert sum(l.startswith("vc-ypass") for l in lines) == 8, lines
        Q = voxcap.Problem.from_scene(s).setup(max_rhs=2, autotune=True, tune_cache=path)
        for (prec, transpose), y in yp.items():
            assert np.array_equal(Q.apply(x, transpose=transpose, prec=prec).cpu().numpy(), y)
        rq = Q.tuning_report()
        xq = [l for l in rq.splitlines() if l.startswith("x-pass")]
        yq = [l for l in rq.splitlines() if l.startswith("y-pass")]
        assert sum("cached" in l for l in xq) == 4 and sum("tuned" in l for l in xq) == 0, rq
        assert sum("cached" in l for l in yq) == 8 and sum("tuned" in l for l in yq) == 0, rq


def test_stats_bytes_model_is_the_pass_model(dev):
    """vc_stats.bytes_model = the algorithmic bytes of one product of the solve's
    right-hand sides, the sum of vc_pass_times' per-pass model."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(5, n_cond=2, n_diel=2)
    P = voxcap.Problem.from_scene(s).setup()
    _, st = P.capacitance(prec="mixed", rtol=1e-10)
    x = torch.zeros(P.m, P.N, dtype=torch.float64, device=dev)
    P.profile(1)
    P.apply(x, prec="fp32")
    P.profile(0)
    _, _, bytes_ = P.pass_times()
    assert st["bytes_model"] > 0
    assert st["bytes_model"] == pytest.approx(sum(bytes_), rel=1e-12)


def test_batch_capacitance_both_names(dev):
    """vc_batch_capacitance and vc_capacitance_batch are one call; both match each
    member's FP64 oracle capacitance."""
    from paper_2004_02609_amd import voxcap
    ss = [scenes.random_small(5, n_cond=2, n_diel=1), scenes.random_small(13, shape=(9, 14, 5), n_cond=2, n_diel=1)]
    probs = [voxcap.Problem.from_scene(s).setup() for s in ss]
    handles = (voxcap._P * len(probs))(*[p._h for p in probs])
    outs = {}
    for name in ("vc_batch_capacitance", "vc_capacitance_batch"):
        Cs = [np.zeros((p.m, p.m)) for p in probs]
        ptrs = (C.c_void_p * len(Cs))(*[c.ctypes.data for c in Cs])
        o = voxcap._solve_opts(prec="fp64", rtol=1e-12)
        st = (voxcap.vc_stats * len(probs))()
        rc = getattr(voxcap._lib, name)(handles, len(probs), C.byref(o), ptrs, st)
        assert rc == voxcap.VC_OK, (name, voxcap._lib.vc_last_error())
        outs[name] = Cs
    for a, b, s in zip(outs["vc_batch_capacitance"], outs["vc_capacitance_batch"], ss):
        assert np.array_equal(a, b)
        ref = oracle.solve_capacitance(s)
        gate = np.abs(ref) >= 1e-3 * np.abs(np.diag(ref)).max()
        assert (np.abs(a - ref)[gate] / np.abs(ref)[gate]).max() < 1e-10


def test_one_call_capacitance(dev):
    """voxcap.capacitance(cond_id, eps_r, dv, precision): the FP64 oracle's C."""
    from paper_2004_02609_amd import voxcap
    s = scenes.random_small(9, shape=(11, 7, 13), n_cond=3, n_diel=2)
    C64, _ = voxcap.capacitance(s["cond_id"], s["eps_r"], s["dv"], precision="fp64", eps_background=s["eps_b"],
                                rtol=1e-12)
    ref = oracle.solve_capacitance(s)
    gate = np.abs(ref) >= 1e-3 * np.abs(np.diag(ref)).max()
    assert (np.abs(C64 - ref)[gate] / np.abs(ref)[gate]).max() < 1e-10
    Cm, st = voxcap.capacitance(s["cond_id"], s["eps_r"], s["dv"], precision="mixed", eps_background=s["eps_b"],
                                rtol=1e-10)
    assert (np.abs(Cm - ref)[gate] / np.abs(ref)[gate]).max() < 1e-6
