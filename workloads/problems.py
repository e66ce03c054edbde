"""Problem descriptions for the synthetic workloads.

A :class:`Problem` is a list of surfaces in one solvent.  Each surface is a
dielectric molecule boundary (with interior permittivity and point charges),
a surface with imposed charge density, a surface with imposed potential, a
Stern surface (a closed surface around one molecule that bounds a salt-free
layer between the molecule and the ionic solvent), or a cavity (a closed
surface inside one molecule around a salt-free, charge-free region).

Named workloads (sizes are panel counts):

* ``kirkwood``     sphere r = 4 A, 1280 panels, +1 e at the centre.
* ``kirkwood_stern`` the same sphere inside a Stern (ion-exclusion) sphere of
  r = 6 A (1280 panels, salt-free layer of permittivity 20).
* ``stern_plate``  that pair (320 + 320 panels) 14 A above a 40 x 40 x 2 A
  charged plate (1536 panels).
* ``star_plate_stern`` star_plate with a Stern surface 2 A outside the
  molecule (the star mesh pushed out radially, 32768 panels, layer
  permittivity 80).
* ``kirkwood_cavity`` / ``kirkwood_water_cavity`` the Kirkwood sphere with a
  salt-free cavity (r = 1 A, 1280 panels, 2.2 A off the charge) of
  permittivity 4 (the molecule's: a fictitious interface) or 80 (water).
* ``twosphere_charge`` / ``twosphere_potential``  molecule sphere (r = 4 A,
  +1 e centre, 5120 panels) and a second sphere (r = 4 A, 5120 panels) 12 A
  away on z with sigma = 0.05 C/m^2 or phi = 0.05 V.
* ``star_plate``   star molecule (32768 panels, 900 charges) 10 A above an
  80 x 80 x 2 A box plate (20480 panels) with sigma = -0.05 C/m^2.
* ``orient_sweep`` the two-sphere molecule at 64 seeded rotations, 10 A above
  the ``star_plate`` plate.
* ``star_plate_large`` star molecule (65536 panels, 3000 charges) 12 A above a
  120 x 120 x 2 A plate (81920 panels), sigma_j = 0.03 (1 + 0.1 u_j).
* ``star_plate_twin`` the large case at 1/16 resolution (4096 + 5120 panels).
* ``orient_sweep_small`` the orientation sweep at a size the oracle solves in
  seconds: a 1280-panel sphere molecule (r = 4 A, +1 e) 10 A above a
  40 x 40 x 2 A plate of 1536 panels (sigma = -0.05 C/m^2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import box_plate, icosphere, star_surface

MOLECULE, CHARGED, POTENTIAL, STERN, CAVITY = 0, 1, 2, 3, 4
KIND_NAMES = {MOLECULE: "molecule", CHARGED: "charged", POTENTIAL: "potential", STERN: "stern",
              CAVITY: "cavity"}


@dataclass
class Surface:
    kind: int
    verts: np.ndarray            # (nv, 3) float64, Angstrom
    tris: np.ndarray             # (nt, 3) int32, CCW seen from the solvent
    bc: np.ndarray | None = None  # (nt,) sigma [C/m^2] or phi0 [V]
    eps_in: float = 1.0           # molecule interior permittivity (Stern: of the layer)
    q_pos: np.ndarray | None = None  # (nq, 3) Angstrom
    q: np.ndarray | None = None      # (nq,) e
    parent: int = -1              # Stern surface: the molecule it encloses; cavity: the one enclosing it

    @property
    def nt(self) -> int:
        return int(len(self.tris))


@dataclass
class Problem:
    surfaces: list
    eps_out: float = 80.0
    kappa: float = 0.125
    params: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n_panels(self) -> int:
        return sum(s.nt for s in self.surfaces)


def random_rotations(n: int, seed: int) -> np.ndarray:
    """Uniform random rotation matrices from normalised 4-D Gaussian quaternions."""
    rng = np.random.default_rng(seed)
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1)[:, None]
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def interior_charges(radius_fn, rmax: float, n: int, seed: int, margin: float = 1.5):
    """Rejection-sample ``n`` points with |x| <= r(x/|x|) - margin; values
    uniform from {-1, -0.5, 0, 0.5, 1} e."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        cand = rng.uniform(-rmax, rmax, size=(4 * n, 3))
        rr = np.linalg.norm(cand, axis=1)
        cand = cand[(rr <= rmax) & (rr > 1e-9)]
        rr = np.linalg.norm(cand, axis=1)
        ok = rr <= radius_fn(cand / rr[:, None]) - margin
        for p in cand[ok]:
            pts.append(p)
            if len(pts) == n:
                break
    pts = np.asarray(pts)
    vals = rng.choice(np.array([-1.0, -0.5, 0.0, 0.5, 1.0]), size=n)
    return pts, vals


def sphere_molecule(level=4, radius=4.0, center=(0.0, 0.0, 0.0), charge=1.0, eps_in=4.0):
    v, t = icosphere(level, radius, center)
    return Surface(MOLECULE, v, t, eps_in=eps_in,
                   q_pos=np.asarray([center], dtype=np.float64), q=np.array([charge]))


def stern_sphere(parent, level=4, radius=6.0, center=(0.0, 0.0, 0.0), eps_in=80.0):
    """Ion-exclusion (Stern) surface: a sphere around molecule ``parent`` (its
    index in the problem), enclosing a salt-free layer of permittivity eps_in."""
    v, t = icosphere(level, radius, center)
    return Surface(STERN, v, t, eps_in=eps_in, parent=parent)


def cavity_sphere(parent, level=2, radius=1.5, center=(0.0, 0.0, 0.0), eps_in=80.0):
    """Solvent-filled (salt-free) cavity inside molecule ``parent``: a
    sphere of permittivity eps_in without charges."""
    v, t = icosphere(level, radius, center)
    return Surface(CAVITY, v, t, eps_in=eps_in, parent=parent)


def plate(half_x, half_y, thick, n_xy, n_long, n_z, sigma):
    v, t = box_plate(-half_x, half_x, -half_y, half_y, -thick, 0.0, n_xy, n_long, n_z)
    bc = np.full(len(t), sigma, dtype=np.float64) if np.isscalar(sigma) else np.asarray(sigma)
    return Surface(CHARGED, v, t, bc=bc)


def star_molecule(levels, shape_seed, n_charges, charge_seed, gap, eps_in=4.0):
    v, t, rfn = star_surface(levels, shape_seed)
    rmax = float(np.max(np.linalg.norm(v, axis=1)))
    qp, qv = interior_charges(rfn, rmax, n_charges, charge_seed)
    shift = np.array([0.0, 0.0, gap - v[:, 2].min()])
    return Surface(MOLECULE, v + shift, t, eps_in=eps_in, q_pos=qp + shift, q=qv)


def star_stern(levels, shape_seed, gap, thickness=2.0, eps_layer=80.0, parent=0):
    """Stern surface of ``star_molecule(levels, shape_seed, ..., gap)``: the
    same star mesh pushed out radially by ``thickness`` A (a closed surface
    around the molecule; its lowest point is below the molecule's)."""
    v, t, _ = star_surface(levels, shape_seed)
    r = np.linalg.norm(v, axis=1)
    vs = v * ((r + thickness) / r)[:, None]
    shift = np.array([0.0, 0.0, gap - v[:, 2].min()])
    return Surface(STERN, vs + shift, t, eps_in=eps_layer, parent=parent)


CONFIG_NAMES = ("kirkwood", "twosphere_charge", "twosphere_potential", "star_plate",
                "orient_sweep", "star_plate_large", "star_plate_twin", "kirkwood_stern", "stern_plate",
                "kirkwood_cavity", "kirkwood_water_cavity", "star_plate_stern", "orient_sweep_small")

DEFAULT_PARAMS = dict(k_far=3, k_near=19, k_self_edge=9, ncrit=300, taylor_p=6, theta=0.5, tol=1e-6)


def config_problem(name: str, level: int | None = None, rotation: int | None = None) -> Problem:
    """Build a named workload.  ``level`` overrides the sphere refinement of the
    sphere workloads (for convergence studies); ``rotation`` picks one of the
    64 orientations of ``orient_sweep`` (default: unrotated)."""
    p = dict(DEFAULT_PARAMS)
    if name == "kirkwood":
        lv = 3 if level is None else level
        s = sphere_molecule(lv, 4.0)
        return Problem([s], 80.0, 0.125, p, name)
    if name == "kirkwood_stern":
        # sphere r = 4 A (+1 e at the centre) inside a Stern sphere r = 6 A;
        # the layer's permittivity 20 (not 80) makes its every term visible
        # in the solvation energy
        lv = 3 if level is None else level
        return Problem([sphere_molecule(lv, 4.0), stern_sphere(0, lv, 6.0, eps_in=20.0)], 80.0, 0.125, p, name)
    if name in ("kirkwood_cavity", "kirkwood_water_cavity"):
        # the Kirkwood sphere (r = 4 A, +1 e at the centre) with a cavity of
        # r = 1 A centred 2.2 A off the charge; with the cavity's permittivity
        # equal to the molecule's (kirkwood_cavity) the interface is
        # fictitious and the energy is Kirkwood's
        lv = 3 if level is None else level
        eps_c = 4.0 if name == "kirkwood_cavity" else 80.0
        return Problem([sphere_molecule(lv, 4.0), cavity_sphere(0, lv, 1.0, (2.2, 0.0, 0.0), eps_c)],
                       80.0, 0.125, p, name)
    if name == "stern_plate":
        # the Stern-layer sphere pair 14 A above a charged plate
        lv = 2 if level is None else level
        c = (0.0, 0.0, 14.0)
        pl = plate(20.0, 20.0, 2.0, 16, 32, 2, -0.05)
        return Problem([sphere_molecule(lv, 4.0, c), stern_sphere(0, lv, 6.0, c), pl], 80.0, 0.125, p, name)
    if name in ("twosphere_charge", "twosphere_potential"):
        lv = 4 if level is None else level
        mol = sphere_molecule(lv, 4.0)
        v, t = icosphere(lv, 4.0, (0.0, 0.0, 12.0))
        if name == "twosphere_charge":
            surf = Surface(CHARGED, v, t, bc=np.full(len(t), 0.05))
        else:
            surf = Surface(POTENTIAL, v, t, bc=np.full(len(t), 0.05))
        return Problem([mol, surf], 80.0, 0.125, p, name)
    if name == "star_plate":
        mol = star_molecule(12, 1, 900, 2, 10.0)
        pl = plate(40.0, 40.0, 2.0, 64, 128, 4, -0.05)
        return Problem([mol, pl], 80.0, 0.125, p, name)
    if name == "star_plate_stern":
        # star_plate with a 2 A Stern layer (permittivity 80, no ions) around
        # the molecule
        mol = star_molecule(12, 1, 900, 2, 10.0)
        pl = plate(40.0, 40.0, 2.0, 64, 128, 4, -0.05)
        return Problem([mol, star_stern(12, 1, 10.0), pl], 80.0, 0.125, p, name)
    if name in ("orient_sweep", "orient_sweep_small"):
        small = name == "orient_sweep_small"
        lv = (3 if small else 4) if level is None else level
        v, t = icosphere(lv, 4.0, (0.0, 0.0, 0.0))
        if rotation is not None:
            R = random_rotations(64, 3)[rotation]
            v = v @ R.T
        c = np.array([0.0, 0.0, 14.0])
        mol = Surface(MOLECULE, v + c, t, eps_in=4.0, q_pos=c[None, :].copy(), q=np.array([1.0]))
        pl = plate(20.0, 20.0, 2.0, 16, 32, 2, -0.05) if small else plate(40.0, 40.0, 2.0, 64, 128, 4, -0.05)
        return Problem([mol, pl], 80.0, 0.125, p, name)
    if name in ("star_plate_large", "star_plate_twin"):
        big = name == "star_plate_large"
        mol = star_molecule(13 if big else 9, 1, 3000 if big else 3000, 4, 12.0)
        n_xy, n_long, n_z = (128, 256, 8) if big else (32, 64, 2)
        rng = np.random.default_rng(5)
        ntri = 2 * (2 * n_xy * n_xy + 4 * n_long * n_z)
        sig = 0.03 * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, size=ntri))
        pl = plate(60.0, 60.0, 2.0, n_xy, n_long, n_z, sig)
        return Problem([mol, pl], 80.0, 0.125, p, name)
    raise KeyError(name)
