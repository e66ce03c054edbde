"""Pins for the oracle's quadrature tables and panel integrals (Section 3.1).

Each rule is pinned by exactness on monomials of the barycentric coordinates
(closed form 2 a! b! c! / (a+b+c+2)! on the unit-area-normalised triangle)
up to its degree, and by failing at one degree higher, so a wrong digit or a
wrong orbit fails here.  The self integral is pinned by the closed form of
the Laplace single layer over a triangle seen from an interior point and by
brute-force polar integration for the Yukawa kernel.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.integrals import Panels, near_mask, pair_integrals, point_kernels, self_single_layer
from oracle.quadrature import gauss_legendre_01, triangle_rule

DEGREE = {1: 1, 3: 2, 4: 3, 7: 5, 19: 9}


def exact_monomial(a, b, c):
    return 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


@pytest.mark.parametrize("npts", sorted(DEGREE))
def test_rule_exact_to_its_degree(npts):
    bary, w = triangle_rule(npts)
    assert len(w) == npts
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.all(bary >= 0) and np.allclose(bary.sum(1), 1.0, atol=1e-15)
    deg = DEGREE[npts]
    for d in range(deg + 1):
        for a in range(d + 1):
            for b in range(d - a + 1):
                c = d - a - b
                q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
                assert abs(q - exact_monomial(a, b, c)) < 1e-13, (npts, a, b, c)


@pytest.mark.parametrize("npts", sorted(DEGREE))
def test_rule_not_exact_beyond_degree(npts):
    bary, w = triangle_rule(npts)
    d = DEGREE[npts] + 1
    errs = []
    for a in range(d + 1):
        for b in range(d - a + 1):
            c = d - a - b
            q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
            errs.append(abs(q - exact_monomial(a, b, c)) / exact_monomial(a, b, c))
    assert max(errs) > 1e-3


def test_gauss_legendre_edge_rule():
    t, w = gauss_legendre_01(9)
    for k in range(18):
        assert abs(np.sum(w * t ** k) - 1.0 / (k + 1)) < 1e-14
    assert abs(np.sum(w * t ** 18) - 1.0 / 19) > 1e-12


TRI = np.array([[0.0, 0.0, 0.0], [1.3, 0.1, 0.0], [0.4, 0.9, 0.0]])


def _laplace_self_closed_form(v, x):
    """(1/4pi) sum_edges h [asinh(s_b/h) - asinh(s_a/h)], the Laplace single
    layer of a flat triangle at an interior point x of its plane."""
    tot = 0.0
    for i in range(3):
        a, b = v[i], v[(i + 1) % 3]
        e = b - a
        ell = np.linalg.norm(e)
        tvec = e / ell
        sa = np.dot(a - x, tvec)
        sb = np.dot(b - x, tvec)
        h = np.linalg.norm(np.cross(a - x, tvec))
        tot += h * (math.asinh(sb / h) - math.asinh(sa / h))
    return tot / (4 * math.pi)


def _polar_brute(v, x, kappa):
    """Brute-force polar integral of G_Y over the triangle seen from x."""
    def rho_max(th):
        d = np.array([math.cos(th), math.sin(th), 0.0])
        best = np.inf
        for i in range(3):
            a, b = v[i], v[(i + 1) % 3]
            m = np.array([[d[0], a[0] - b[0]], [d[1], a[1] - b[1]]])
            rhs = (a - x)[:2]
            try:
                s, t = np.linalg.solve(m, rhs)
            except np.linalg.LinAlgError:
                continue
            if s > 0 and -1e-12 <= t <= 1 + 1e-12:
                best = min(best, s)
        return best

    def f(th):
        rm = rho_max(th)
        if kappa == 0:
            return rm / (4 * math.pi)
        return -math.expm1(-kappa * rm) / (4 * math.pi * kappa)

    # split at the vertex angles so the integrand is smooth on each piece
    angs = sorted(math.atan2(*(vv - x)[[1, 0]]) % (2 * math.pi) for vv in v)
    pieces = [(angs[i], angs[i + 1]) for i in range(2)] + [(angs[2], angs[0] + 2 * math.pi)]
    return sum(integrate.quad(f, a, b, epsabs=1e-14, epsrel=1e-13)[0] for a, b in pieces)


def test_self_laplace_matches_closed_form_with_fine_edge_rule():
    p = Panels(TRI, np.array([[0, 1, 2]]))
    x = p.centroid
    ref = _laplace_self_closed_form(TRI, x[0])
    vl64, _ = self_single_layer(p, [0], x, 0.125, 64)
    assert abs(vl64[0] - ref) < 1e-12 * ref
    # the paper's 9 points per edge is accurate but not exact
    vl9, _ = self_single_layer(p, [0], x, 0.125, 9)
    assert 1e-8 < abs(vl9[0] - ref) / ref < 1e-4
    assert abs(ref - _polar_brute(TRI, x[0], 0.0)) < 1e-11


def test_self_yukawa_matches_brute_force_and_kappa_limit():
    p = Panels(TRI, np.array([[0, 1, 2]]))
    x = p.centroid
    _, vy64 = self_single_layer(p, [0], x, 0.125, 64)
    brute = _polar_brute(TRI, x[0], 0.125)
    assert abs(vy64[0] - brute) < 1e-11 * brute
    _, vy_small = self_single_layer(p, [0], x, 1e-9, 64)
    _, vy_zero = self_single_layer(p, [0], x, 0.0, 64)
    assert abs(vy_small[0] - vy_zero[0]) < 1e-9 * vy_zero[0]
    assert vy64[0] < vy_zero[0]          # screening lowers the potential


def test_near_rule_against_adaptive_integration():
    """19-point rule at distance ~1.5 L from the panel centroid, compared with
    adaptive 2-D integration over the triangle."""
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.2, 0.9, 0.0]])
    p = Panels(tri, np.array([[0, 1, 2]]))
    L = math.sqrt(2 * p.area[0])
    x = p.centroid[0] + np.array([0.3, 0.2, 1.5 * L])
    assert near_mask(x[None, :], p)[0, 0]
    vl, kl, vy, ky = (a[0] for a in pair_integrals(x[None, :], p, np.array([0]), 19, 0.125))
    v0, v1, v2 = tri

    def integrand(t, s, which):
        y = v0 + s * (v1 - v0) + t * (v2 - v0)
        vals = point_kernels(x, y, p.normal[0], 0.125)
        return vals[which] * 2 * p.area[0]

    for which, got in enumerate((vl, kl, vy, ky)):
        ref = integrate.dblquad(integrand, 0, 1, 0, lambda s: 1 - s, args=(which,),
                                epsabs=1e-13, epsrel=1e-11)[0]
        assert abs(got - ref) < 2e-6 * abs(ref), which


def test_near_predicate_is_two_L():
    tri = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    p = Panels(tri, np.array([[0, 1, 2]]))
    L = math.sqrt(2 * p.area[0])       # = 2
    c = p.centroid[0]
    pts = np.array([c + [0, 0, 2 * L * 0.999], c + [0, 0, 2 * L * 1.001]])
    m = near_mask(pts, p)[:, 0]
    assert m[0] and not m[1]
    # another factor f: the test is |x - c| < f L, in-plane and off-plane
    for f in (1.0, 1.5, 3.0, 7.25):
        for direction in ([0, 0, 1.0], [0.6, 0.8, 0.0]):
            d = np.asarray(direction)
            pts = np.array([c + d * f * L * 0.9999, c + d * f * L * 1.0001])
            m = near_mask(pts, p, near_factor=f)[:, 0]
            assert m[0] and not m[1], (f, direction)
    # exactly on the threshold is not near (strict): f = 2 puts c + 4 e_z
    # at d^4 = 256 = 16 |e1 x e2|^2
    assert not near_mask(np.array([c + [0, 0, 4.0]]), p)[0, 0]


def test_kernels_signs_and_limits():
    x = np.array([0.0, 0.0, 2.0])
    y = np.zeros(3)
    n = np.array([0.0, 0.0, 1.0])
    gl, kl, gy, ky = point_kernels(x, y, n, 0.0)
    assert abs(gl - 1 / (8 * math.pi)) < 1e-15
    assert abs(gy - gl) < 1e-15 and abs(ky - kl) < 1e-15
    # derivative at the source along n: d/dy_z of 1/(4 pi |x-y|) at y = 0
    h = 1e-6
    fd = (1 / (4 * math.pi * np.linalg.norm(x - (y + h * n))) - 1 / (4 * math.pi * np.linalg.norm(x - (y - h * n)))) / (2 * h)
    assert abs(kl - fd) < 1e-9
    _, _, gy, ky = point_kernels(x, y, n, 0.5)
    fd = (math.exp(-0.5 * np.linalg.norm(x - (y + h * n))) / (4 * math.pi * np.linalg.norm(x - (y + h * n)))
          - math.exp(-0.5 * np.linalg.norm(x - (y - h * n))) / (4 * math.pi * np.linalg.norm(x - (y - h * n)))) / (2 * h)
    assert abs(ky - fd) < 1e-9
