"""Pins of the oracle's Tucker compression (eq. 13): mode products against explicit
sums, exact recovery of tensors built with known multilinear ranks, the error bound
of the truncation rule, minimality of the chosen ranks, orthonormal factors, and the
rank-1 closed form."""
import numpy as np
import pytest

from oracle import tucker


def _orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def test_mode_products_match_explicit_sums():
    rng = np.random.default_rng(0)
    T = rng.standard_normal((3, 4, 5))
    for mode, n in enumerate(T.shape):
        U = rng.standard_normal((6, n))
        got = tucker.mode_product(T, U, mode)
        ref = np.zeros(T.shape[:mode] + (6,) + T.shape[mode + 1:])
        for idx in np.ndindex(*ref.shape):
            s = 0.0
            for t in range(n):
                src = list(idx)
                src[mode] = t
                s += U[idx[mode], t] * T[tuple(src)]
            ref[idx] = s
        assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_rebuild_matches_quadruple_sum():
    rng = np.random.default_rng(1)
    S = rng.standard_normal((2, 3, 2))
    Us = [rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    got = tucker.rebuild(S, Us)
    ref = np.zeros((4, 3, 5))
    for i, j, k in np.ndindex(4, 3, 5):
        ref[i, j, k] = sum(S[a, b, c] * Us[0][i, a] * Us[1][j, b] * Us[2][k, c]
                           for a in range(2) for b in range(3) for c in range(2))
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_exact_recovery_of_known_ranks():
    rng = np.random.default_rng(2)
    ranks = (3, 4, 2)
    dims = (9, 11, 7)
    S0 = rng.standard_normal(ranks)
    X = tucker.rebuild(S0, [_orth(rng, d, r) for d, r in zip(dims, ranks)])
    S, Us = tucker.st_hosvd(X, 1e-12)
    assert S.shape == ranks
    assert np.abs(tucker.rebuild(S, Us) - X).max() < 1e-13 * np.abs(X).max()
    for U in Us:
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)


def test_rank_one_closed_form():
    a, b, c = np.arange(1.0, 6.0), np.linspace(-1, 2, 4), np.array([3.0, -2.0, 0.5])
    X = np.einsum("i,j,k->ijk", a, b, c)
    S, Us = tucker.st_hosvd(X, 1e-10)
    assert S.shape == (1, 1, 1)
    assert abs(abs(S[0, 0, 0]) - np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c)) < 1e-12 * np.abs(X).max()


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-8])
def test_error_bound_and_minimal_ranks(tol):
    # a smooth, translation-invariant 1/r-like tensor (the structure of the kernels)
    i, j, k = np.meshgrid(np.arange(20.0), np.arange(17.0), np.arange(13.0), indexing="ij")
    X = 1.0 / np.sqrt(1.0 + i * i + 0.7 * j * j + 1.3 * k * k)
    S, Us = tucker.st_hosvd(X, tol)
    nx = np.linalg.norm(X)
    err = np.linalg.norm(tucker.rebuild(S, Us) - X)
    assert err <= tol * nx * (1 + 1e-9)
    assert tucker.stored_size(S, Us) < X.size
    # each rank is the smallest meeting that mode's budget on the tensor it saw
    budget = tol * tol * nx * nx / 3.0
    T = X
    for mode, U in enumerate(Us):
        M = np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1)
        sv = np.linalg.svd(M, compute_uv=False)
        r = U.shape[1]
        assert np.sum(sv[r:] ** 2) <= budget * (1 + 1e-12)
        if r > 1:
            assert np.sum(sv[r - 1:] ** 2) > budget
        T = tucker.mode_product(T, U.T, mode)
