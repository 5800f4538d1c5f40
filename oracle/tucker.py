"""Tucker compression of a 3-way tensor, eq. (13) (Sec. II.C) -- test infrastructure only.

X (D1 x D2 x D3) ~ S x_1 U1 x_2 U2 x_3 U3 with orthonormal factors U_i (D_i x r_i) and
core S (r1 x r2 x r3).  The paper defers the procedure for a given tolerance to its
references; the reading taken here is the sequentially truncated higher-order SVD:
for modes 1, 2, 3 in turn, the left singular vectors of the current tensor's mode-i
unfolding are kept up to the smallest rank whose discarded squared singular values
sum to at most tol^2 ||X||^2 / 3, and the tensor is projected onto them.  The
discarded energies of the three steps add up to the squared reconstruction error, so
||X - X_hat||_F <= tol ||X||_F.

Plain numpy in FP64; numpy.linalg.svd is the only library step.
"""
import numpy as np


def mode_product(T, U, mode):
    """T x_mode U: contracts axis `mode` of T (size U.shape[1]) with the columns of U."""
    T = np.moveaxis(T, mode, 0)
    shp = T.shape
    out = U @ T.reshape(shp[0], -1)
    return np.moveaxis(out.reshape((U.shape[0],) + shp[1:]), 0, mode)


def _rank_for(sv, budget):
    """Smallest r with sum_{j >= r} sv_j^2 <= budget (sv descending)."""
    tail = np.concatenate([np.cumsum((sv ** 2)[::-1])[::-1], [0.0]])   # tail[r] = sum_{j>=r}
    for r in range(len(sv) + 1):
        if tail[r] <= budget:
            return max(r, 1)
    return len(sv)


def st_hosvd(X, tol):
    """(S, [U1, U2, U3]) of the sequentially truncated HOSVD with the per-mode budget
    tol^2 ||X||^2 / 3."""
    X = np.asarray(X, dtype=np.float64)
    budget = tol * tol * float(np.sum(X * X)) / 3.0
    T = X
    Us = []
    for mode in range(3):
        M = np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1)
        U, sv, _ = np.linalg.svd(M, full_matrices=False)
        r = _rank_for(sv, budget)
        Ur = U[:, :r]
        Us.append(Ur)
        T = mode_product(T, Ur.T, mode)
    return T, Us


def rebuild(S, Us):
    """S x_1 U1 x_2 U2 x_3 U3 (eq. 13)."""
    X = S
    for mode, U in enumerate(Us):
        X = mode_product(X, U, mode)
    return X


def stored_size(S, Us):
    """Numbers kept by the compressed form: r1 r2 r3 + sum_i D_i r_i."""
    return S.size + sum(U.size for U in Us)
