"""Toeplitz tensors of App. B kept Tucker-compressed over a largest grid and restored for a
smaller one (Sec. II.C, Tab. I) -- oracle version, test infrastructure only.

The block Toeplitz tensor of a pair (observer normal alpha, source normal beta; eq. 5 or
eq. 6) holds the panel integral at every centre offset d = lag + s between two panels
of the grid, where s_alpha = -1/2 and s_beta = +1/2 when alpha != beta and s = 0
otherwise (the panel centres of App. B).  The integral of eq. (5) does not change when
any offset component changes sign (both squares are symmetric about their centres);
eq. (6) is its derivative along d_alpha, so it changes sign with d_alpha only.  A pair
is therefore fixed by its values at the non-negative offsets

    octant[t0, t1, t2] = K(d),   d_a = t_a + h_a,   t_a = 0..n_a,

with h_a = 1/2 on the two normal axes of an orthogonal pair and 0 otherwise.  That is
the tensor that is compressed: a Tucker factor is indexed by one axis' offset, so the
tensor of a smaller grid is the same core with the leading rows of each factor.

Dimensionless units (voxel edge 1): the values do not depend on the voxel size.
Pairs are numbered 0..5 for eq. (5) xx yy zz xy xz yz and 6 + 3 alpha + beta for eq. (6).
"""
import numpy as np

from . import integrals, tucker

PAIRS = ([(0, 0, "P"), (1, 1, "P"), (2, 2, "P"), (0, 1, "P"), (0, 2, "P"), (1, 2, "P")]
         + [(a, b, "E") for a in range(3) for b in range(3)])


def half_shifts(alpha, beta):
    """h: the half-voxel part of |d| per axis."""
    h = np.zeros(3)
    if alpha != beta:
        h[alpha] = 0.5
        h[beta] = 0.5
    return h


def octant(q, n):
    """Pair q's values at the non-negative offsets of a grid of n voxels per axis:
    array (n0+1, n1+1, n2+1)."""
    alpha, beta, want = PAIRS[q]
    axes = [np.arange(k + 1, dtype=np.float64) for k in n]
    d = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3) + half_shifts(alpha, beta)
    return integrals.kernel(alpha, beta, d, want).reshape(tuple(k + 1 for k in n))


def signed_offsets(q, n):
    """Every centre offset between two panels of pair q on a grid of n voxels per axis
    (lag ranges of App. B: observer and source panel counts n_a + [a == alpha] and
    n_a + [a == beta])."""
    alpha, beta, _ = PAIRS[q]
    s = np.zeros(3)
    if alpha != beta:
        s[alpha], s[beta] = -0.5, 0.5
    rng = []
    for a in range(3):
        no = n[a] + (a == alpha)
        ns = n[a] + (a == beta)
        rng.append(np.arange(-(ns - 1), no, dtype=np.float64) + s[a])
    return np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)


def from_octant(q, T, d):
    """Pair q's value at signed offsets d (K x 3) read from its octant T: |d| gives the
    entry, and for eq. (6) the sign of d_alpha gives the sign."""
    alpha, beta, want = PAIRS[q]
    t = np.rint(np.abs(d) - half_shifts(alpha, beta)).astype(np.int64)
    v = T[t[:, 0], t[:, 1], t[:, 2]]
    if want == "E":
        v = np.where(d[:, alpha] < 0, -v, v)
    return v


def compress(q, nmax, tol):
    """(S, [U1, U2, U3]): pair q's octant over nmax, compressed at relative tolerance tol."""
    return tucker.st_hosvd(octant(q, nmax), tol)


def restore(S, Us, n):
    """Octant of a grid of n voxels from a compressed largest-grid octant: the core with
    the leading n_a + 1 rows of each factor."""
    return tucker.rebuild(S, [U[:k + 1] for U, k in zip(Us, n)])
