"""Direct pin of the far field (Section 3.2: Cartesian Taylor expansion of
order P of the Green's functions about a source box's centre).

A small source surface S sits far from a target sphere T, so that every
target group of T accepts S's root box for the far field; with unknowns only
on S, T's solvent rows of the product hold exactly the library's far field
of that box: S as one box (20 panels, 60 Gauss points: P2M + Taylor
recurrence + M2P), or S split into a tree of boxes of at most 6 panels (80
panels: P2M at the leaves, M2M up to the root, M2P).
The reference is the truncated Taylor polynomial in h = y - c of
G(|R - h|), R = x - c, written without any recurrence: the degree-m part of
the expansion is the t^m coefficient of g(t) = G(|R - t h|), and g depends
on h only through a = |R|^2, b = R.h and c = |h|^2, so sympy derives each
coefficient symbolically as a function of (a, b, c); the double layer's
n.grad_h of the polynomial follows from the chain rule through b and c.

Bars: the library's FP64 product equals the reference to 1e-11 of the
largest target value for P = 0..8 (the reference and the library round
differently, nothing else); the truncation error against the exact sums
falls with P as the reference's own does (here |h| / |R| < 0.1: by at least
a factor 0.3 every two orders, and by 1e-6 from P = 0 to 8; from one order
to the next it can rise for a double layer, odd and even orders
alternating).
"""
import numpy as np
import pytest
import sympy as sp

from oracle.integrals import Panels
from oracle.quadrature import triangle_rule
from paper_1506_03745_amd import FP64, from_problem
from workloads.meshes import icosphere
from workloads.problems import CHARGED, MOLECULE, POTENTIAL, Problem, Surface

PMAX = 8
_COEF = {}


def taylor_coefficients(yukawa):
    """Lists (g_m, dg_m/db, dg_m/dc), m = 0..PMAX, of numpy functions of
    (a, b, c, kappa): g_m = t^m coefficient of G(sqrt(a - 2 b t + c t^2))."""
    if yukawa in _COEF:
        return _COEF[yukawa]
    t, a, b, c, k = sp.symbols("t a b c kappa", real=True)
    rho = sp.sqrt(a - 2 * b * t + c * t ** 2)
    g = sp.exp(-k * rho) / (4 * sp.pi * rho) if yukawa else 1 / (4 * sp.pi * rho)
    out, fact = [], 1
    for m in range(PMAX + 1):
        if m:
            g = sp.diff(g, t)
            fact *= m
        e = g.subs(t, 0) / fact
        out.append(tuple(sp.lambdify((a, b, c, k), ex, "numpy") for ex in (e, sp.diff(e, b), sp.diff(e, c))))
    _COEF[yukawa] = out
    return out


def gauss_points(surf):
    """Gauss points (the 3-point rule), weights w_q A_p and normals of a surface, caller order."""
    pan = Panels(surf.verts, surf.tris)
    bary, w = triangle_rule(3)
    y = pan.points(bary).reshape(-1, 3)
    wa = (w[None, :] * pan.area[:, None]).reshape(-1)
    nrm = np.repeat(pan.normal, len(w), axis=0)
    return y, wa, nrm


def reference(P, kappa, x_tgt, y, wa, nrm, dens, double_layer):
    """Truncated Taylor far field of the sources at the targets:
    sum_j wa_j dens_j T_P(h_j) (single layer) or
    -sum_j wa_j dens_j n_j . grad_h T_P(h_j) (double layer, the -K phi term)."""
    c = 0.5 * (y.min(0) + y.max(0))          # expansion centre: bounding-box centre of the Gauss points
    h = y - c
    R = x_tgt - c
    A = np.sum(R * R, 1)[:, None]
    B = R @ h.T
    C = np.sum(h * h, 1)[None, :]
    coef = taylor_coefficients(kappa != 0.0)
    s = np.zeros_like(B)
    for m in range(P + 1):
        g, gb, gc = coef[m]
        if double_layer:
            s += gb(A, B, C, kappa) * (R @ nrm.T) + gc(A, B, C, kappa) * 2 * np.sum(h * nrm, 1)[None, :]
        else:
            s += g(A, B, C, kappa) * np.ones_like(B)
    v = s @ (wa * np.repeat(dens, 3))
    return -v if double_layer else v


def exact(kappa, x_tgt, y, wa, nrm, dens, double_layer):
    d = x_tgt[:, None, :] - y[None, :, :]
    r = np.sqrt(np.sum(d * d, -1))
    e = np.exp(-kappa * r)
    w = wa * np.repeat(dens, 3)
    if double_layer:
        k = np.sum(d * nrm[None], -1) * (1 + kappa * r) * e / (4 * np.pi * r ** 3)
        return -(k @ w)
    return (e / (4 * np.pi * r)) @ w


def two_bodies(kind, src_level=0):
    v, t = icosphere(1, 1.0, (0.0, 0.0, 0.0))
    tgt = Surface(MOLECULE, v, t, eps_in=4.0, q_pos=np.zeros((1, 3)), q=np.array([1.0]))
    sv, st = icosphere(src_level, 0.5, (0.3, -0.2, 7.0))
    src = Surface(kind, sv, st, bc=np.full(len(st), 0.01))
    return tgt, src


def test_taylor_reference_converges():
    """The sympy reference itself tends to the exact sums as P grows, its
    error falling geometrically (|h| / |R| < 0.1 here): over eight seeds of
    densities, single and double layers, by 0.16 or less every two orders."""
    tgt, src = two_bodies(POTENTIAL)
    x = Panels(tgt.verts, tgt.tris).centroid
    y, wa, nrm = gauss_points(src)
    dens = np.random.default_rng(3).standard_normal(src.nt)
    for kappa in (0.125, 0.0):
        for dl in (False, True):
            ex = exact(kappa, x, y, wa, nrm, dens, dl)
            errs = [np.max(np.abs(reference(P, kappa, x, y, wa, nrm, dens, dl) - ex)) for P in range(PMAX + 1)]
            assert errs[PMAX] < 1e-9 * np.max(np.abs(ex)) and errs[PMAX] < 1e-6 * errs[0]
            for P in range(2, PMAX + 1):
                assert errs[P] < 0.3 * errs[P - 2] + 1e-15 * np.max(np.abs(ex))


@pytest.mark.gpu
@pytest.mark.parametrize("kind", [POTENTIAL, CHARGED])
@pytest.mark.parametrize("kappa", [0.125, 0.0])
@pytest.mark.parametrize("tree", ["one_box", "m2m"])
def test_far_field_equals_taylor_polynomial(kind, kappa, tree):
    tgt, src = two_bodies(kind, 0 if tree == "one_box" else 1)
    ncrit = 300 if tree == "one_box" else 6
    x = Panels(tgt.verts, tgt.tris).centroid
    y, wa, nrm = gauss_points(src)
    dens = np.random.default_rng(4).standard_normal(src.nt)
    dl = kind == CHARGED
    ex = exact(kappa, x, y, wa, nrm, dens, dl)
    scale = np.max(np.abs(ex))
    nt = tgt.nt
    xin = np.zeros(2 * nt + src.nt)
    xin[2 * nt:] = dens
    errs = []
    for P in range(PMAX + 1):
        pr = Problem([tgt, src], 80.0, kappa, {}, "taylor_pin")
        s, _ = from_problem(pr, treecode=1, ncrit=ncrit, theta=0.5, taylor_p=P, prec=FP64)
        yv = s.matvec(xin, prec=FP64)
        s.close()
        assert np.all(yv[:nt] == 0.0)                 # T's interior rows do not see S
        lib = yv[nt:2 * nt]
        ref = reference(P, kappa, x, y, wa, nrm, dens, dl)
        assert np.max(np.abs(lib - ref)) <= 1e-11 * scale, (P, np.max(np.abs(lib - ref)) / scale)
        errs.append(np.max(np.abs(lib - ex)))
    assert errs[PMAX] < 1e-6 * errs[0]
    for P in range(2, PMAX + 1):
        assert errs[P] < 0.3 * errs[P - 2] + 1e-12 * scale
