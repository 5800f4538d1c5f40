"""Galerkin panel integrals of eq. (5) and eq. (6), oracle version (FP64, numpy).

Dimensionless units (App. C): voxel edge 1, Green's function 1/|r - r'|.

    P(alpha, beta, d) = int_{S_o} int_{S_s} 1/|r - r'| dS' dS                    (eq. 5)
    E(alpha, beta, d) = int_{S_o} d/dr_alpha [ int_{S_s} 1/|r - r'| dS' ] dS     (eq. 6)

S_o is the observer (testing) unit square with normal axis alpha, S_s the source
square with normal axis beta, and d = centre(S_o) - centre(S_s).  The derivative in
(6) is along +alpha, the observer's normal; the paper's sign for -alpha normals
(Sec. II.B note 3) is applied by the caller.  E of two coplanar squares is 0 (the
normal field of a flat sheet vanishes in its plane off the sheet, and on the sheet
its principal value is 0: the jump is the separate term of eq. 7).

Evaluation route (chosen to be independent of the library's):
* the inner integral over S_s is the exact potential (and gradient) of a uniformly
  charged square at a point, written out from the elementary antiderivatives;
* the outer integral over S_o is a tensor tanh-sinh rule for squares that touch
  (edge/corner log singularities sit on the boundary of S_o), a tensor
  Gauss-Legendre rule for separated squares closer than FAR_SEP, and for farther
  pairs a 4-D Gauss-Legendre product rule of 1/|r-r'| itself, the order chosen
  from the separation so the rule error stays below ~1e-15 relative.
"""
from __future__ import annotations

import functools

import numpy as np

FAR_SEP = 5.0


def _inplane(axis):
    return (axis + 1) % 3, (axis + 2) % 3


# ---------------------------------------------------------------- inner closed forms
def _f_corner(a, b, z):
    """Antiderivative with d^2/(da db) f = 1/sqrt(a^2+b^2+z^2)."""
    ra = np.sqrt(a * a + z * z)
    rb = np.sqrt(b * b + z * z)
    r = np.sqrt(a * a + b * b + z * z)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(ra > 0, a * np.arcsinh(b / np.where(ra > 0, ra, 1.0)), 0.0)
        t2 = np.where(rb > 0, b * np.arcsinh(a / np.where(rb > 0, rb, 1.0)), 0.0)
        zr = z * r
        t3 = np.where(zr != 0, z * np.arctan(a * b / np.where(zr != 0, zr, 1.0)), 0.0)
    return t1 + t2 - t3


def square_potential(x, y, z):
    """int over [-1/2,1/2]^2 (plane z=0) of 1/|(x,y,z)-(x',y',0)| dx'dy'."""
    tot = 0.0
    for xe, sx in ((-0.5, -1.0), (0.5, 1.0)):
        for ye, sy in ((-0.5, -1.0), (0.5, 1.0)):
            tot = tot + sx * sy * _f_corner(xe - x, ye - y, z)
    return tot


def square_gradient(x, y, z, comp):
    """d/dx, d/dy or d/dz (comp 0/1/2) of square_potential at the field point."""
    if comp == 2:
        tot = 0.0
        for xe, sx in ((-0.5, -1.0), (0.5, 1.0)):
            for ye, sy in ((-0.5, -1.0), (0.5, 1.0)):
                a = xe - x
                b = ye - y
                r = np.sqrt(a * a + b * b + z * z)
                zr = z * r
                with np.errstate(divide="ignore", invalid="ignore"):
                    t = np.where(zr != 0, np.arctan(a * b / np.where(zr != 0, zr, 1.0)), 0.0)
                tot = tot + sx * sy * t
        return -tot
    if comp == 1:
        return square_gradient(y, x, z, 0)
    # d/dx: -sum_i s_i [asinh(b/rho_i)]_{b1}^{b2}, rho_i = sqrt(a_i^2+z^2), a_i = x_i' - x
    tot = 0.0
    for xe, sx in ((-0.5, -1.0), (0.5, 1.0)):
        a = xe - x
        rho = np.sqrt(a * a + z * z)
        for ye, sy in ((-0.5, -1.0), (0.5, 1.0)):
            b = ye - y
            tot = tot + sx * sy * np.arcsinh(b / rho)
    return -tot


# ---------------------------------------------------------------- quadrature rules
@functools.lru_cache(maxsize=None)
def gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * x, 0.5 * w            # on [-1/2, 1/2]


@functools.lru_cache(maxsize=None)
def tanh_sinh(h=1.0 / 20.0, kmax=75):
    k = np.arange(-kmax, kmax + 1) * h
    s = 0.5 * np.pi * np.sinh(k)
    x = np.tanh(s)
    w = 0.5 * np.pi * h * np.cosh(k) / np.cosh(s) ** 2
    keep = (np.abs(x) < 1.0) & (w > 1e-300)
    return 0.5 * x[keep], 0.5 * w[keep]   # on [-1/2, 1/2]


def _extent(axis):
    e = np.full(3, 0.5)
    e[axis] = 0.0
    return e


def separation(alpha, beta, d):
    """Euclidean distance between the closed observer and source squares."""
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    ext = _extent(alpha) + _extent(beta)
    g = np.maximum(np.abs(d) - ext, 0.0)
    return np.sqrt(np.sum(g * g, axis=1))


def _far_order(sep):
    n = np.full(sep.shape, 6)
    n[sep >= 10.0] = 5
    n[sep >= 20.0] = 4
    n[sep >= 100.0] = 3
    return n


def _near_order(sep):
    return np.where(sep >= 2.0, 10, 14)


def _outer(alpha, beta, d, rule, want):
    """Outer 2-D rule over the observer square of the exact inner integral."""
    u, wu = rule
    po, qo = _inplane(alpha)
    ps, qs = _inplane(beta)
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu).ravel()
    off = np.zeros((U.size, 3))
    off[:, po] = U.ravel()
    off[:, qo] = V.ravel()
    out = np.empty(len(d))
    chunk = max(1, 400000 // U.size)
    for c0 in range(0, len(d), chunk):
        t = d[c0:c0 + chunk, None, :] + off[None, :, :]
        x, y, z = t[..., ps], t[..., qs], t[..., beta]
        if want == "P":
            val = square_potential(x, y, z)
        else:
            comp = 2 if alpha == beta else (0 if alpha == ps else 1)
            val = square_gradient(x, y, z, comp)
        out[c0:c0 + chunk] = val @ W
    return out


def _far4(alpha, beta, d, n, want):
    g, w = gauss_legendre(n)
    po, qo = _inplane(alpha)
    ps, qs = _inplane(beta)
    U, V = np.meshgrid(g, g, indexing="ij")
    W2 = np.outer(w, w).ravel()
    oo = np.zeros((U.size, 3))
    oo[:, po] = U.ravel()
    oo[:, qo] = V.ravel()
    ss = np.zeros((U.size, 3))
    ss[:, ps] = U.ravel()
    ss[:, qs] = V.ravel()
    rel = (oo[:, None, :] - ss[None, :, :]).reshape(-1, 3)   # (Qo*Qs, 3)
    Wp = np.outer(W2, W2).ravel()
    out = np.empty(len(d))
    chunk = max(1, 4000000 // Wp.size)
    for c0 in range(0, len(d), chunk):
        dc = d[c0:c0 + chunk]
        tx = dc[:, 0, None] + rel[None, :, 0]
        ty = dc[:, 1, None] + rel[None, :, 1]
        tz = dc[:, 2, None] + rel[None, :, 2]
        r2 = tx * tx + ty * ty + tz * tz
        if want == "P":
            f = 1.0 / np.sqrt(r2)
        else:
            ta = (tx, ty, tz)[alpha]
            f = -ta / (r2 * np.sqrt(r2))
        out[c0:c0 + chunk] = f @ Wp
    return out


def kernel(alpha, beta, d, want="P"):
    """P (eq. 5) or E (eq. 6) for observer normal alpha, source normal beta, centre
    offsets d (K x 3, observer minus source, voxel units)."""
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    out = np.zeros(len(d))
    sep = separation(alpha, beta, d)
    if want == "E" and alpha == beta:
        live = d[:, alpha] != 0.0
    else:
        live = np.ones(len(d), bool)
    touch = live & (sep == 0.0)
    near = live & (sep > 0.0) & (sep < FAR_SEP)
    far = live & (sep >= FAR_SEP)
    if np.any(touch):
        out[touch] = _outer(alpha, beta, d[touch], tanh_sinh(), want)
    if np.any(near):
        nn = _near_order(sep[near])
        idx = np.nonzero(near)[0]
        for n in np.unique(nn):
            sel = idx[nn == n]
            out[sel] = _outer(alpha, beta, d[sel], gauss_legendre(int(n)), want)
    if np.any(far):
        nf = _far_order(sep[far])
        idx = np.nonzero(far)[0]
        for n in np.unique(nf):
            sel = idx[nf == n]
            out[sel] = _far4(alpha, beta, d[sel], int(n), want)
    return out


def P(alpha, beta, d):
    return kernel(alpha, beta, d, "P")


def E(alpha, beta, d):
    return kernel(alpha, beta, d, "E")


