"""Panel geometry and the four panel integrals (Section 3.1).

For a point x and a flat panel j with constant density, the oracle computes

    V_L = int_j G_L(x, y) dy         K_L = int_j dG_L/dn_y(x, y) dy
    V_Y = int_j G_Y(x, y) dy         K_Y = int_j dG_Y/dn_y(x, y) dy

with G_L = 1/(4 pi r), G_Y = exp(-kappa r)/(4 pi r) (eq. free-space; its
arguments are read as G(x, y) with r = |x - y|) and the derivative taken at
the source point y along the panel's outward normal n_j:

    dG_L/dn_y = n_j.(x - y) / (4 pi r^3)
    dG_Y/dn_y = n_j.(x - y) (1 + kappa r) exp(-kappa r) / (4 pi r^3).

Three regimes, as Section 3.1 describes them:

* self (x is the collocation point of panel j): K = 0 because x - y lies in
  the panel's plane; V is integrated in polar coordinates about x, the
  radial integral done in closed form and the angle integral written as a
  sum over edges with Gauss-Legendre points along each edge (Hess & Smith);
* near (|x - c_j| < 2 L_j, L_j = sqrt(2 A_j)): the 19-point rule (the factor
  2 is Section 3.1's; ``near_factor`` takes another);
* far: the K-point rule.

The near test is a decision of floating point over an integer outcome, so it
is written as an exact sequence of correctly rounded FP64 operations without
square roots:  (d2 * d2) < f4 * |e1 x e2|^2  with d2 = (dx*dx + dy*dy) + dz*dz
and f4 = (f * f) * (f * f), which is  |x - c_j| < f sqrt(2 A_j)  since
|e1 x e2| = 2 A_j (f = 2: f4 = 16).
"""
from __future__ import annotations

import numpy as np

from .quadrature import gauss_legendre_01, triangle_rule
from .units import FOUR_PI


class Panels:
    """Geometry of a list of flat triangles (Section 3.1)."""

    def __init__(self, verts: np.ndarray, tris: np.ndarray):
        verts = np.asarray(verts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        self.v0 = verts[tris[:, 0]]
        self.v1 = verts[tris[:, 1]]
        self.v2 = verts[tris[:, 2]]
        e1 = self.v1 - self.v0
        e2 = self.v2 - self.v0
        cx = e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1]
        cy = e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2]
        cz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        self.cross_norm2 = (cx * cx + cy * cy) + cz * cz
        cn = np.sqrt(self.cross_norm2)
        self.area = 0.5 * cn
        self.normal = np.stack([cx / cn, cy / cn, cz / cn], axis=1)
        self.centroid = ((self.v0 + self.v1) + self.v2) * (1.0 / 3.0)
        self.n = len(tris)

    def points(self, bary: np.ndarray) -> np.ndarray:
        """Quadrature points (n_panels, n_pts, 3) for barycentric coordinates."""
        return (bary[None, :, 0, None] * self.v0[:, None, :]
                + bary[None, :, 1, None] * self.v1[:, None, :]
                + bary[None, :, 2, None] * self.v2[:, None, :])


def near_mask(x: np.ndarray, panels: Panels, near_factor: float = 2.0) -> np.ndarray:
    """(M, N) boolean: target x_m is closer than f L_j to centroid c_j (f = 2
    in Section 3.1)."""
    c = panels.centroid
    dx = x[:, None, 0] - c[None, :, 0]
    dy = x[:, None, 1] - c[None, :, 1]
    dz = x[:, None, 2] - c[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    f = float(near_factor)
    f4 = (f * f) * (f * f)
    return (d2 * d2) < f4 * panels.cross_norm2[None, :]


def point_kernels(x, y, n, kappa):
    """G_L, dG_L/dn_y, G_Y, dG_Y/dn_y for broadcastable x, y, n (last axis 3)."""
    d = x - y
    r = np.sqrt(np.sum(d * d, axis=-1))
    nd = np.sum(n * d, axis=-1)
    gl = 1.0 / (FOUR_PI * r)
    kl = nd / (FOUR_PI * r ** 3)
    e = np.exp(-kappa * r)
    gy = gl * e
    ky = kl * (1.0 + kappa * r) * e
    return gl, kl, gy, ky


def rule_integrals(x, panels: Panels, cols, npts, kappa):
    """Integrals of the four kernels over panels ``cols`` seen from points x
    (M, 3) with the ``npts`` triangle rule.  Returns four (M, len(cols))."""
    bary, w = triangle_rule(npts)
    sub = panels.points(bary)[cols]                # (C, Q, 3)
    nrm = panels.normal[cols]                      # (C, 3)
    area = panels.area[cols]                       # (C,)
    # a rule point that coincides with x (the self panel of the rules that
    # contain the centroid) gives inf / nan here; callers replace the self
    # entries by the self integrals, so those values are never used
    with np.errstate(divide="ignore", invalid="ignore"):
        gl, kl, gy, ky = point_kernels(x[:, None, None, :], sub[None, :, :, :],
                                       nrm[None, :, None, :], kappa)
    wa = w[None, None, :] * area[None, :, None]
    return ((gl * wa).sum(-1), (kl * wa).sum(-1), (gy * wa).sum(-1), (ky * wa).sum(-1))


def self_single_layer(panels: Panels, j, x, kappa: float, n_edge: int):
    """V_L and V_Y of panels j at points x inside them (x = their centroids).

    In polar coordinates about x the radial integral of G * rho is
    g_L(rho) = rho / (4 pi) and g_Y(rho) = (1 - exp(-kappa rho)) / (4 pi kappa);
    the angle element along an edge from p to q is h * l * dt / rho(t)^2 with
    h the distance from x to the edge's line and l the edge length.
    ``j`` is an index array and ``x`` is (len(j), 3)."""
    j = np.atleast_1d(np.asarray(j))
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    t, wt = gauss_legendre_01(n_edge)
    verts = (panels.v0[j], panels.v1[j], panels.v2[j])
    vl = np.zeros(len(j))
    vy = np.zeros(len(j))
    for a in range(3):
        p, q = verts[a], verts[(a + 1) % 3]
        e = q - p
        ell = np.linalg.norm(e, axis=1)
        h = np.linalg.norm(np.cross(p - x, e), axis=1) / ell
        pts = p[:, None, :] + t[None, :, None] * e[:, None, :]
        rho = np.linalg.norm(pts - x[:, None, :], axis=2)
        ang = wt[None, :] * (h * ell)[:, None] / rho ** 2
        vl += np.sum(ang * rho, axis=1) / FOUR_PI
        if kappa > 0.0:
            vy += np.sum(ang * (-np.expm1(-kappa * rho)), axis=1) / (FOUR_PI * kappa)
        else:
            vy += np.sum(ang * rho, axis=1) / FOUR_PI
    return vl, vy


def pair_integrals(x, panels: Panels, cols, npts, kappa):
    """Integrals for a list of (point, panel) pairs: x (P, 3), cols (P,)."""
    bary, w = triangle_rule(npts)
    sub = panels.points(bary)[cols]                # (P, Q, 3)
    nrm = panels.normal[cols]
    area = panels.area[cols]
    gl, kl, gy, ky = point_kernels(x[:, None, :], sub, nrm[:, None, :], kappa)
    wa = w[None, :] * area[:, None]
    return ((gl * wa).sum(-1), (kl * wa).sum(-1), (gy * wa).sum(-1), (ky * wa).sum(-1))


def layer_blocks(x, panels: Panels, kappa, k_far=3, k_near=19, k_self_edge=9,
                 self_idx=None, chunk_pairs=2_000_000, near_factor=2.0):
    """Dense (M, N) blocks V_L, K_L, V_Y, K_Y of targets x against all panels.

    ``self_idx[m]`` is the panel that holds target m (or -1): that entry
    uses the self rule.  Every other entry uses the near rule when the near
    test holds and the far rule otherwise."""
    x = np.asarray(x, dtype=np.float64)
    M, N = len(x), panels.n
    out = [np.empty((M, N)) for _ in range(4)]
    allc = np.arange(N)
    rows = max(1, chunk_pairs // max(1, N * max(k_far, 1)))
    for r0 in range(0, M, rows):
        r1 = min(M, r0 + rows)
        blk = rule_integrals(x[r0:r1], panels, allc, k_far, kappa)
        for o, b in zip(out, blk):
            o[r0:r1] = b
        near = near_mask(x[r0:r1], panels, near_factor)
        if self_idx is not None:
            si = np.asarray(self_idx[r0:r1])
            has = si >= 0
            near[np.nonzero(has)[0], si[has]] = False
        mi, ji = np.nonzero(near)
        if len(mi):
            nb = pair_integrals(x[r0 + mi], panels, ji, k_near, kappa)
            for o, b in zip(out, nb):
                o[r0 + mi, ji] = b
    if self_idx is not None:
        si = np.asarray(self_idx)
        m = np.nonzero(si >= 0)[0]
        if len(m):
            vl, vy = self_single_layer(panels, si[m], x[m], kappa, k_self_edge)
            out[0][m, si[m]] = vl
            out[1][m, si[m]] = 0.0
            out[2][m, si[m]] = vy
            out[3][m, si[m]] = 0.0
    return out
