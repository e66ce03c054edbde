"""Quadrature rules (Section 3.1, Discretization).

The paper integrates a panel with a "far" rule of 1, 3, 4 or 7 Gauss points,
a fine rule of 19 (or more) points when the panel is closer than 2L to the
collocation point, and, on the panel that holds the collocation point, a
semi-analytical rule with 9 Gauss points along each edge.  It does not print
the rules.  Readings taken here:

* far rules: the classical symmetric rules of degree 1 (centroid), 2
  (barycentric (2/3, 1/6, 1/6) and permutations), 3 (Strang-Fix, centroid
  weight -27/48) and 5 (Radon's 7-point rule);
* near rule: Dunavant's symmetric 19-point rule of degree 9;
* edge rule: Gauss-Legendre on [0, 1].

Triangle rules are returned as barycentric coordinates ``(n, 3)`` and weights
``(n,)`` that sum to 1; the integral of f over a panel of area A is
``A * sum(w * f(bary @ verts))``.
"""
from __future__ import annotations

import math

import numpy as np


def _perm3(a, b, c):
    """Distinct permutations of a barycentric triple."""
    out = []
    for p in ((a, b, c), (b, c, a), (c, a, b), (a, c, b), (c, b, a), (b, a, c)):
        if p not in out:
            out.append(p)
    return out


def _orbit_s21(a, w):
    """Points (1-2a, a, a) and its rotations."""
    return [(p, w) for p in _perm3(1.0 - 2.0 * a, a, a)]


def _orbit_s111(a, b, w):
    return [(p, w) for p in _perm3(a, b, 1.0 - a - b)]


def triangle_rule(npts: int):
    """Symmetric triangle rule with ``npts`` points (1, 3, 4, 7 or 19)."""
    pts = []
    if npts == 1:
        pts = [((1 / 3, 1 / 3, 1 / 3), 1.0)]
    elif npts == 3:
        pts = _orbit_s21(1.0 / 6.0, 1.0 / 3.0)
    elif npts == 4:
        pts = [((1 / 3, 1 / 3, 1 / 3), -27.0 / 48.0)] + _orbit_s21(0.2, 25.0 / 48.0)
    elif npts == 7:
        s15 = math.sqrt(15.0)
        pts = ([((1 / 3, 1 / 3, 1 / 3), 9.0 / 40.0)]
               + _orbit_s21((6.0 - s15) / 21.0, (155.0 - s15) / 1200.0)
               + _orbit_s21((6.0 + s15) / 21.0, (155.0 + s15) / 1200.0))
    elif npts == 19:
        # Dunavant (1985), degree 9.
        pts = ([((1 / 3, 1 / 3, 1 / 3), 0.097135796282799)]
               + _orbit_s21(0.489682519198738, 0.031334700227139)
               + _orbit_s21(0.437089591492937, 0.077827541004774)
               + _orbit_s21(0.188203535619033, 0.079647738927210)
               + _orbit_s21(0.044729513394453, 0.025577675658698)
               + _orbit_s111(0.036838412054736, 0.221962989160766, 0.043283539377289))
    else:
        raise ValueError(f"no {npts}-point triangle rule")
    bary = np.array([p for p, _ in pts], dtype=np.float64)
    w = np.array([x for _, x in pts], dtype=np.float64)
    assert len(w) == npts
    return bary, w


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w
