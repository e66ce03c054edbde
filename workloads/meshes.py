"""Triangle surface meshes: icospheres, star-shaped molecules, box plates.

Every mesh is returned as ``(verts, tris)`` with ``verts`` float64 ``(nv, 3)``
and ``tris`` int32 ``(nt, 3)``.  Triangles are counter-clockwise when seen
from the solvent, so ``(v1 - v0) x (v2 - v0)`` points out of the enclosed
body into the solvent.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Icosphere: icosahedron, each triangle split into four per level, vertices
# pushed radially onto the sphere.  20 * 4**level triangles.
# --------------------------------------------------------------------------


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v, f


def _orient_outward(verts, tris, center):
    """Flip any triangle whose normal points toward ``center``."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    bad = np.einsum("ij,ij->i", nrm, cen - center) < 0
    tris = tris.copy()
    tris[bad] = tris[bad][:, [0, 2, 1]]
    return tris


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Sphere of ``20 * 4**level`` flat triangles, vertices on the sphere."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    faces = f
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.add(verts[i], verts[j]) * 0.5
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                k = len(verts) - 1
                cache[key] = k
            return k

        nf = np.empty((4 * len(faces), 3), dtype=np.int64)
        for n, (a, b, c) in enumerate(faces):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * n + 0] = (a, ab, ca)
            nf[4 * n + 1] = (b, bc, ab)
            nf[4 * n + 2] = (c, ca, bc)
            nf[4 * n + 3] = (ab, bc, ca)
        faces = nf
    vv = np.asarray(verts, dtype=np.float64) * float(radius) + np.asarray(center, dtype=np.float64)
    faces = _orient_outward(vv, faces, np.asarray(center, dtype=np.float64))
    return vv, faces.astype(np.int32)


# --------------------------------------------------------------------------
# Octahedron refined by uniform newest-vertex bisection.  The initial
# refinement edges are the four equatorial edges, which makes the marking
# compatible, so every uniform level stays conforming.  8 * 2**levels
# triangles (12 levels -> 32768, 13 -> 65536).
# --------------------------------------------------------------------------


def octa_bisection_sphere(levels: int):
    """Unit-sphere mesh; returns (dirs, tris).  Vertices are unit vectors."""
    v = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (-1.0, 0.0, 0.0), (0.0, -1.0, 0.0),
         (0.0, 0.0, 1.0), (0.0, 0.0, -1.0)]
    # Each triangle is stored as (p, q, apex): edge (p, q) is the refinement
    # edge, apex is the newest vertex.  Equatorial edges (0,1),(1,2),(2,3),(3,0).
    tris = []
    for k in range(4):
        a, b = k, (k + 1) % 4
        tris.append((a, b, 4))
        tris.append((b, a, 5))
    tris = np.asarray(tris, dtype=np.int64)
    verts = [np.asarray(x) for x in v]
    for _ in range(levels):
        cache: dict[tuple[int, int], int] = {}
        out = np.empty((2 * len(tris), 3), dtype=np.int64)
        for n, (p, q, apex) in enumerate(tris):
            key = (p, q) if p < q else (q, p)
            m = cache.get(key)
            if m is None:
                mp = (verts[p] + verts[q]) * 0.5
                mp = mp / np.linalg.norm(mp)
                verts.append(mp)
                m = len(verts) - 1
                cache[key] = m
            # children: refinement edge is the edge opposite the new vertex m
            out[2 * n + 0] = (apex, p, m)
            out[2 * n + 1] = (q, apex, m)
        tris = out
    dirs = np.asarray(verts, dtype=np.float64)
    tris = _orient_outward(dirs, tris, np.zeros(3))
    return dirs, tris.astype(np.int32)


# --------------------------------------------------------------------------
# Star-shaped molecule r(theta, phi) = R0 * (1 + amp * s), s a seeded sum of
# orthonormal real spherical harmonics l = 1..lmax with N(0,1) coefficients,
# rescaled so that max |s| over the mesh vertices is 1.
# --------------------------------------------------------------------------


def _real_sph_harm(l, m, theta, phi):
    """Orthonormal real spherical harmonic; theta polar, phi azimuth."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1) ** m * np.real(y)
    return np.sqrt(2.0) * (-1) ** m * np.imag(y)


def star_directions(dirs, seed: int, lmax: int = 4):
    """Unnormalised shape function s at unit directions ``dirs``."""
    rng = np.random.default_rng(seed)
    theta = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    s = np.zeros(len(dirs))
    coeffs = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            c = rng.standard_normal()
            coeffs.append((l, m, c))
            s += c * _real_sph_harm(l, m, theta, phi)
    return s, coeffs


def star_surface(levels: int, seed: int, r0: float = 15.0, amp: float = 0.15, lmax: int = 4):
    """Star-shaped closed surface, ``8 * 2**levels`` triangles.

    Returns (verts, tris, radius_fn) where ``radius_fn(unit_dirs)`` gives the
    surface radius along arbitrary directions (used to place charges inside).
    """
    dirs, tris = octa_bisection_sphere(levels)
    s, coeffs = star_directions(dirs, seed, lmax)
    scale = 1.0 / np.max(np.abs(s))

    def radius_fn(u):
        u = np.asarray(u, dtype=np.float64)
        theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
        phi = np.arctan2(u[:, 1], u[:, 0])
        ss = np.zeros(len(u))
        for l, m, c in coeffs:
            ss += c * _real_sph_harm(l, m, theta, phi)
        return r0 * (1.0 + amp * scale * ss)

    r = r0 * (1.0 + amp * scale * s)
    verts = dirs * r[:, None]
    tris = _orient_outward(verts, tris, np.zeros(3))
    return verts, tris, radius_fn


# --------------------------------------------------------------------------
# Box plate [x0,x1] x [y0,y1] x [z0,z1]; each face meshed on its own regular
# grid of squares, two triangles per square.  Faces do not share vertices.
# --------------------------------------------------------------------------


def _grid_face(origin, eu, ev, nu, nv):
    """Regular grid on the parallelogram origin + s*eu + t*ev, s,t in [0,1].

    Triangles are CCW around eu x ev."""
    origin, eu, ev = (np.asarray(a, dtype=np.float64) for a in (origin, eu, ev))
    s = np.arange(nu + 1) / nu
    t = np.arange(nv + 1) / nv
    S, T = np.meshgrid(s, t, indexing="ij")
    verts = origin + S.reshape(-1, 1) * eu + T.reshape(-1, 1) * ev
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return verts, tris


def box_plate(x0, x1, y0, y1, z0, z1, n_xy: int, n_side_long: int, n_side_z: int):
    """Closed box, outward normals.  Top/bottom: n_xy x n_xy squares each;
    sides: n_side_long x n_side_z squares each; two triangles per square."""
    lx, ly, lz = x1 - x0, y1 - y0, z1 - z0
    faces = [
        # top (+z): eu x ev = +z
        ((x0, y0, z1), (lx, 0, 0), (0, ly, 0), n_xy, n_xy),
        # bottom (-z)
        ((x0, y0, z0), (0, ly, 0), (lx, 0, 0), n_xy, n_xy),
        # +x side
        ((x1, y0, z0), (0, ly, 0), (0, 0, lz), n_side_long, n_side_z),
        # -x side
        ((x0, y0, z0), (0, 0, lz), (0, ly, 0), n_side_z, n_side_long),
        # +y side
        ((x0, y1, z0), (0, 0, lz), (lx, 0, 0), n_side_z, n_side_long),
        # -y side
        ((x0, y0, z0), (lx, 0, 0), (0, 0, lz), n_side_long, n_side_z),
    ]
    vs, ts, off = [], [], 0
    for o, eu, ev, nu, nv in faces:
        v, t = _grid_face(o, eu, ev, nu, nv)
        vs.append(v)
        ts.append(t + off)
        off += len(v)
    verts = np.concatenate(vs)
    tris = np.concatenate(ts)
    center = np.array([(x0 + x1) / 2, (y0 + y1) / 2, (z0 + z1) / 2])
    tris = _orient_outward(verts, tris, center)
    return verts, tris.astype(np.int32)
