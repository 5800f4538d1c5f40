"""Pins of the oracle's Toeplitz octants and their compressed, cropped form (Sec. II.C,
Tab. I), and the library's validation of cache files (no GPU needed).

* Parity reading: the octant and the sign rule reproduce the panel integrals evaluated
  directly at every signed offset of a grid (eq. 5 even in each offset component,
  eq. 6 odd in d_alpha only).  A half shift on the wrong axis, a lost sign or a sign on
  the wrong axis fails it.
* Lag ranges: the signed offsets of App. B are exactly the centre offsets between all
  panel pairs of a grid, found by brute force over the panels, and each maps inside
  the octant of that grid (t_a <= n_a).
* Dense matrix: every entry of the oracle's eq. (4) matrix outside the jump diagonal is
  the octant value of its pair, read at |centre offset| with the parity sign (and the
  row's orientation sign on eq. 6 rows).
* Crop: restoring with the leading factor rows equals restoring the whole tensor and
  cropping it (a property of the Tucker format), and the restored tensor of a smaller
  grid is within the compression bound tol * ||octant over nmax|| of its octant
  computed from the integrals.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import integrals, toeplitz, tucker


def test_pair_numbering():
    assert len(toeplitz.PAIRS) == 15
    assert toeplitz.PAIRS[:6] == [(0, 0, "P"), (1, 1, "P"), (2, 2, "P"), (0, 1, "P"), (0, 2, "P"), (1, 2, "P")]
    for a, b in itertools.product(range(3), range(3)):
        assert toeplitz.PAIRS[6 + 3 * a + b] == (a, b, "E")


@pytest.mark.parametrize("q", range(15))
def test_octant_and_sign_rule_reproduce_direct_integrals(q):
    n = (3, 2, 4)
    alpha, beta, want = toeplitz.PAIRS[q]
    T = toeplitz.octant(q, n)
    d = toeplitz.signed_offsets(q, n)
    direct = integrals.kernel(alpha, beta, d, want)
    via = toeplitz.from_octant(q, T, d)
    scale = np.abs(direct).max()
    assert scale > 0
    assert np.abs(via - direct).max() <= 1e-12 * scale, q
    if want == "E":
        # the odd dependence is real: values at -d_alpha are the negatives, not equal
        flip = d.copy()
        flip[:, alpha] = -flip[:, alpha]
        other = integrals.kernel(alpha, beta, flip, want)
        live = np.abs(direct) > 1e-3 * scale
        assert np.allclose(other[live], -direct[live], rtol=1e-11, atol=0)


def _panel_centres(n, axis):
    """Centres of every axis-normal face of an n0 x n1 x n2 voxel grid."""
    rng = [np.arange(n[a] + 1) if a == axis else np.arange(n[a]) + 0.5 for a in range(3)]
    return np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)


@pytest.mark.parametrize("n", [(2, 3, 1), (3, 1, 2)])
def test_signed_offsets_are_all_panel_pair_offsets(n):
    for q, (alpha, beta, _) in enumerate(toeplitz.PAIRS):
        co, cs = _panel_centres(n, alpha), _panel_centres(n, beta)
        brute = (co[:, None, :] - cs[None, :, :]).reshape(-1, 3)
        brute = {tuple(v) for v in np.round(brute * 2).astype(int)}
        mine = {tuple(v) for v in np.round(toeplitz.signed_offsets(q, n) * 2).astype(int)}
        assert brute == mine, q
        t = np.rint(np.abs(toeplitz.signed_offsets(q, n)) - toeplitz.half_shifts(alpha, beta))
        assert (t >= 0).all() and (t <= np.array(n)).all()


@pytest.mark.parametrize("q", [0, 3, 5, 6, 7, 11])
def test_cropped_restore_within_compression_bound(q):
    nmax, n = (12, 10, 8), (7, 4, 6)
    big = toeplitz.octant(q, nmax)
    small = toeplitz.octant(q, n)
    for tol in (1e-4, 1e-9):
        S, Us = toeplitz.compress(q, nmax, tol)
        crop = toeplitz.restore(S, Us, n)
        whole = tucker.rebuild(S, Us)[: n[0] + 1, : n[1] + 1, : n[2] + 1]
        assert np.abs(crop - whole).max() <= 1e-13 * np.abs(whole).max()
        err = np.linalg.norm(crop - small)
        assert err <= tol * np.linalg.norm(big) * (1 + 1e-9), (q, tol, err)
        if tol == 1e-4:
            # a real compression, so the bound is not met trivially
            assert sum(r for r in S.shape) < sum(big.shape)


def test_dense_matrix_entries_are_octant_values():
    """Every off-diagonal entry of the oracle's eq. (4) matrix, and the conductor rows'
    diagonal, is the octant value of its pair at |centre offset| with the parity sign:
    eq. (5) rows read the pair (min, max) of the two normal axes, eq. (6) rows the pair
    (observer, source) times the row's orientation sign (Sec. II.B note 3)."""
    import oracle
    import scenes
    s = scenes.random_small(5, shape=(5, 4, 6), n_cond=2, n_diel=1)
    po = oracle.panelize(s["cond_id"], s["eps_r"], s["eps_b"])
    A = oracle.assemble(po)
    n = tuple(int(v) for v in s["cond_id"].shape)
    T = [toeplitz.octant(q, n) for q in range(15)]
    ax, ctr, kind = po["axis"], po["center"], po["kind"]
    sign = np.where(kind == 1, po["sign"], 1).astype(float)
    ref = np.zeros_like(A)
    for a in range(3):
        for b in range(3):
            cols = np.nonzero(ax == b)[0]
            for kd in (0, 1):
                rows = np.nonzero((ax == a) & (kind == kd))[0]
                if len(rows) == 0 or len(cols) == 0:
                    continue
                q = toeplitz.PAIRS.index((min(a, b), max(a, b), "P")) if kd == 0 else 6 + 3 * a + b
                d = (ctr[rows][:, None, :] - ctr[cols][None, :, :]).reshape(-1, 3)
                v = toeplitz.from_octant(q, T[q], d).reshape(len(rows), len(cols))
                ref[np.ix_(rows, cols)] = sign[rows][:, None] * v
    off = ~np.eye(len(A), dtype=bool) | (kind == 0)[:, None]
    assert (kind == 1).any() and (kind == 0).any()
    err = np.abs(A - ref)[off].max() / np.abs(A).max()
    assert err < 1e-12, err


def test_cache_file_validation(tmp_path):
    from paper_2004_02609_amd import voxcap
    bad = tmp_path / "junk.vct"
    bad.write_bytes(b"not a cache")
    with pytest.raises(voxcap.VoxcapError) as e:
        voxcap.vc_toeplitz_cache_load(str(bad))
    assert e.value.status == voxcap.VC_ERR_ARG
    # right tag, truncated body
    trunc = tmp_path / "trunc.vct"
    hdr = b"VCTOEP01" + np.array([4, 4, 4, 15], np.int32).tobytes() + np.array([1e-8]).tobytes()
    trunc.write_bytes(hdr + np.array([2, 2, 2], np.int32).tobytes() + b"\0" * 16)
    with pytest.raises(voxcap.VoxcapError) as e:
        voxcap.vc_toeplitz_cache_load(str(trunc))
    assert e.value.status == voxcap.VC_ERR_ARG
    with pytest.raises(voxcap.VoxcapError):
        voxcap.vc_toeplitz_cache_load(os.path.join(str(tmp_path), "missing.vct"))
    # sizes are checked before any device work
    with pytest.raises(voxcap.VoxcapError) as e:
        voxcap.vc_toeplitz_cache_build((1400, 1400, 1400), 1e-8)
    assert e.value.status == voxcap.VC_ERR_ARG
    with pytest.raises(voxcap.VoxcapError) as e:
        voxcap.vc_toeplitz_cache_build((8, 8, 8), 0.0)
    assert e.value.status == voxcap.VC_ERR_ARG

