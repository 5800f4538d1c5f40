"""Pins of the oracle's Galerkin integrals (eq. 5, eq. 6) against things other than itself.

* the self term of a unit square (closed form from the literature);
* the 4-D integrals written as corner sums of antiderivatives (the route the
  paper takes in App. A and its citation for eq. 5), evaluated with 40-digit mpmath
  so cancellation plays no part -- a different route from the oracle's
  inner-closed-form + outer-quadrature;
* brute-force 2-D quadrature of the inner square potential, finite differences of it;
* Gauss's law for the field integrals over a closed surface of voxel faces;
* the far-field multipole expansion;
* reflection and exchange symmetries.
"""
import itertools

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import integrals as I

mp.mp.dps = 40
W3 = (1, -2, 1)


# ---------------------------------------------------------------- 4-D corner-sum forms
def _F(u, v, w):
    """d^2/du^2 d^2/dv^2 F = 1/r (parallel squares)."""
    u, v, w = mp.mpf(u), mp.mpf(v), mp.mpf(w)
    r = mp.sqrt(u * u + v * v + w * w)
    t = mp.mpf(0)
    ruw, rvw = mp.sqrt(u * u + w * w), mp.sqrt(v * v + w * w)
    if ruw > 0:
        t += (u * u - w * w) * v / 2 * mp.asinh(v / ruw)
    if rvw > 0:
        t += (v * v - w * w) * u / 2 * mp.asinh(u / rvw)
    if w != 0:
        t -= u * v * w * mp.atan(u * v / (w * r))
    return t - r * (u * u + v * v - 2 * w * w) / 6


def _Fw(u, v, w):
    u, v, w = mp.mpf(u), mp.mpf(v), mp.mpf(w)
    r = mp.sqrt(u * u + v * v + w * w)
    t = w * r
    ruw, rvw = mp.sqrt(u * u + w * w), mp.sqrt(v * v + w * w)
    if w != 0:
        t -= u * v * mp.atan(u * v / (w * r))
    if rvw > 0:
        t -= u * w * mp.asinh(u / rvw)
    if ruw > 0:
        t -= v * w * mp.asinh(v / ruw)
    return t


def _G(u, v, w):
    """d/du d/dv d^2/dw^2 G = 1/r (orthogonal squares sharing the w direction)."""
    u, v, w = mp.mpf(u), mp.mpf(v), mp.mpf(w)
    r = mp.sqrt(u * u + v * v + w * w)
    rvw, ruw, ruv = mp.sqrt(v * v + w * w), mp.sqrt(u * u + w * w), mp.sqrt(u * u + v * v)
    t = mp.mpf(0)
    if rvw > 0:
        t += (v * w * w / 2 - v ** 3 / 6) * mp.asinh(u / rvw)
    if ruw > 0:
        t += (u * w * w / 2 - u ** 3 / 6) * mp.asinh(v / ruw)
    if ruv > 0:
        t += u * v * w * mp.asinh(w / ruv)
    if w != 0:
        t -= w ** 3 / 6 * mp.atan(u * v / (w * r))
    if v != 0:
        t -= v * v * w / 2 * mp.atan(u * w / (v * r))
    if u != 0:
        t -= u * u * w / 2 * mp.atan(v * w / (u * r))
    return t - u * v * r / 3


def _Gu(u, v, w):
    u, v, w = mp.mpf(u), mp.mpf(v), mp.mpf(w)
    r = mp.sqrt(u * u + v * v + w * w)
    ruw, ruv = mp.sqrt(u * u + w * w), mp.sqrt(u * u + v * v)
    t = -v * r / 2
    if ruw > 0:
        t += (w * w - u * u) / 2 * mp.asinh(v / ruw)
    if ruv > 0:
        t += v * w * mp.asinh(w / ruv)
    if u != 0:
        t -= u * w * mp.atan(v * w / (u * r))
    return t


def ref_kernel(alpha, beta, d, want):
    """Corner-sum evaluation of eq. (5) / eq. (6) in 40-digit arithmetic."""
    d = [mp.mpf(x) for x in d]
    if alpha == beta:
        p, q = (alpha + 1) % 3, (alpha + 2) % 3
        f = _F if want == "P" else _Fw
        if want == "E" and d[alpha] == 0:
            return mp.mpf(0)
        return sum(W3[a + 1] * W3[b + 1] * f(d[p] + a, d[q] + b, d[alpha])
                   for a in (-1, 0, 1) for b in (-1, 0, 1))
    g = 3 - alpha - beta
    f = _G if want == "P" else _Gu
    s = mp.mpf(0)
    for i, si in ((0, -1), (1, 1)):
        for j, sj in ((0, -1), (1, 1)):
            for c in (-1, 0, 1):
                s += si * sj * W3[c + 1] * f(d[alpha] - mp.mpf(1) / 2 + i,
                                             d[beta] - mp.mpf(1) / 2 + j, d[g] + c)
    return s


def grid_offset(alpha, beta, lag):
    """Centre offset of an alpha-panel and a beta-panel whose grid indices differ by lag."""
    d = np.asarray(lag, dtype=float).copy()
    if alpha != beta:
        d[alpha] -= 0.5
        d[beta] += 0.5
    return d


LAGS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 1), (-1, 0, -1),
        (2, 1, 0), (0, -2, 1), (3, 2, 1), (-4, 1, 2), (5, 0, -3), (7, 3, 2), (12, -5, 4),
        (25, 3, -9)]


@pytest.mark.parametrize("alpha,beta", list(itertools.product(range(3), range(3))))
def test_kernels_match_corner_sums(alpha, beta):
    for lag in LAGS:
        d = grid_offset(alpha, beta, lag)
        for want in ("P", "E"):
            ref = float(ref_kernel(alpha, beta, d, want))
            got = I.kernel(alpha, beta, [d], want)[0]
            scale = max(abs(ref), 1e-3 / (1.0 + np.dot(d, d)))
            assert abs(got - ref) <= 2e-14 * scale + 1e-16, (alpha, beta, lag, want, got, ref)


def test_self_term_closed_form():
    # int_{unit square} int_{unit square} 1/|r-r'| = 4 ln(1+sqrt 2) - (4/3)(sqrt 2 - 1)
    exact = 4.0 * np.log(1.0 + np.sqrt(2.0)) - 4.0 / 3.0 * (np.sqrt(2.0) - 1.0)
    assert abs(exact - 2.973209598247379) < 1e-15
    for a in range(3):
        assert abs(I.P(a, a, [[0, 0, 0]])[0] - exact) < 2e-15 * exact
        assert I.E(a, a, [[0, 0, 0]])[0] == 0.0


def test_square_potential_brute_force():
    pts = [(0.3, 1.7, 0.4), (0.1, -0.2, 0.0), (2.5, 0.5, -1.0), (0.5, 0.5, 0.7), (-0.6, 0.2, 0.0)]
    for x, y, z in pts:
        f = lambda yy, xx: 1.0 / np.sqrt((xx - x) ** 2 + (yy - y) ** 2 + z * z)
        pts_x = [x] if -0.5 < x < 0.5 else None
        ref = integrate.dblquad(f, -0.5, 0.5, -0.5, 0.5, epsabs=1e-13, epsrel=1e-13)[0] \
            if z != 0 or not (-0.5 < x < 0.5 and -0.5 < y < 0.5) else None
        got = I.square_potential(np.array(x), np.array(y), np.array(z))
        if ref is not None:
            assert abs(got - ref) < 1e-11 * abs(ref), (x, y, z)
        del pts_x


def test_square_gradient_finite_difference():
    h = 1e-5
    for x, y, z in [(0.3, 1.7, 0.4), (2.5, 0.5, -1.0), (0.2, 0.1, 0.9), (1.3, -0.8, 0.05)]:
        for comp in range(3):
            e = np.zeros(3)
            e[comp] = h
            fd = (I.square_potential(*(np.array([x, y, z]) + e)) -
                  I.square_potential(*(np.array([x, y, z]) - e))) / (2 * h)
            got = I.square_gradient(np.array(x), np.array(y), np.array(z), comp)
            assert abs(got - fd) < 1e-8 * max(1.0, abs(fd)), (x, y, z, comp)


def _box_surface(lo, hi):
    """Faces of the box [lo, hi) of voxels with outward signs: (axis, centre, sign)."""
    out = []
    for a in range(3):
        p, q = (a + 1) % 3, (a + 2) % 3
        for side, pos in ((-1, lo[a]), (1, hi[a])):
            for i in range(lo[p], hi[p]):
                for j in range(lo[q], hi[q]):
                    c = np.zeros(3)
                    c[a] = pos
                    c[p] = i + 0.5
                    c[q] = j + 0.5
                    out.append((a, c, side))
    return out


@pytest.mark.parametrize("src", [
    (0, (1.0, 0.5, 1.5)),     # interior face touching the box surface along its edges
    (2, (1.5, 0.5, 2.0)),     # interior z face
    (1, (0.5, 0.0, 0.5)),     # on the surface itself -> skipped
    (0, (6.0, 0.5, 0.5)),     # outside
    (1, (1.5, -2.0, 1.5)),    # outside, near
])
def test_gauss_law_for_field_integrals(src):
    """sum_k s_k E_kl over a closed surface = -4 pi (area of l) inside, 0 outside."""
    lo, hi = (0, 0, 0), (2, 1, 3)
    beta, cs = src[0], np.asarray(src[1])
    surf = _box_surface(lo, hi)
    on_surface = any(a == beta and np.allclose(c, cs) for a, c, _ in surf)
    if on_surface:
        pytest.skip("source on the surface")
    inside = all(lo[a] <= cs[a] <= hi[a] for a in range(3)) and \
        all(lo[a] < cs[a] < hi[a] for a in range(3) if a != beta)
    tot = 0.0
    for a, c, s in surf:
        tot += s * I.E(a, beta, [c - cs])[0]
    expect = -4.0 * np.pi if inside else 0.0
    assert abs(tot - expect) < 1e-12, (tot, expect)


def _multipole(alpha, beta, d, want):
    """1/R plus the second-moment term of two uniform unit squares; error O(R^-5)."""
    import sympy as sp
    X = sp.symbols("x0:3", real=True)
    R = sp.sqrt(sum(x * x for x in X))
    cov = [0.0, 0.0, 0.0]
    for a in range(3):
        cov[a] += (1.0 / 12.0 if a != alpha else 0.0) + (1.0 / 12.0 if a != beta else 0.0)
    expr = 1 / R + sum(sp.Rational(1, 2) * cov[i] * sp.diff(1 / R, X[i], 2) for i in range(3))
    if want == "E":
        expr = sp.diff(expr, X[alpha])
    return float(expr.subs(dict(zip(X, d))))


def test_far_field_multipole():
    for alpha, beta in [(0, 0), (2, 2), (0, 1), (2, 0)]:
        for lag in [(40, 13, -7), (-9, 33, 21), (60, 0, 5)]:
            d = grid_offset(alpha, beta, lag)
            R = np.linalg.norm(d)
            for want in ("P", "E"):
                ref = _multipole(alpha, beta, d, want)
                got = I.kernel(alpha, beta, [d], want)[0]
                base = 1.0 / R if want == "P" else 1.0 / R ** 2
                assert abs(got - ref) < 2e-7 * base, (alpha, beta, lag, want, got, ref)


def test_symmetries():
    rng = np.random.default_rng(7)
    for _ in range(40):
        alpha, beta = rng.integers(0, 3, 2)
        lag = rng.integers(-6, 7, 3)
        d = grid_offset(alpha, beta, lag)
        P = I.P(alpha, beta, [d])[0]
        # exchange of observer and source
        assert abs(P - I.P(beta, alpha, [-d])[0]) < 1e-14 * abs(P)
        for ax in range(3):
            dr = d.copy()
            dr[ax] = -dr[ax]
            assert abs(P - I.P(alpha, beta, [dr])[0]) < 1e-14 * abs(P)
            E = I.E(alpha, beta, [d])[0]
            Er = I.E(alpha, beta, [dr])[0]
            sgn = -1.0 if ax == alpha else 1.0
            assert abs(E - sgn * Er) < 1e-14 * max(abs(E), 1e-6), (alpha, beta, lag, ax)
