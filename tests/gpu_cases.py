"""Seeded small problems shared by the GPU parity tests (inputs only)."""
import numpy as np

from workloads.meshes import box_plate, icosphere
from workloads.problems import CAVITY, CHARGED, MOLECULE, POTENTIAL, STERN, Problem, Surface, config_problem


def sphere_plate(gap=1.0, kappa=0.125):
    """Molecule sphere close to a small charged box: panels of the two
    surfaces fall within each other's 2L, so cross-surface near corrections
    are exercised; 320 + 448 panels (not multiples of 64)."""
    v, t = icosphere(2, 3.0, (0.0, 0.0, 3.0 + gap))
    rng = np.random.default_rng(11)
    qpos = np.array([[0.0, 0.0, 3.0 + gap], [0.8, -0.5, 3.0 + gap + 0.4]])
    mol = Surface(MOLECULE, v, t, eps_in=2.0, q_pos=qpos, q=np.array([1.0, -0.5]))
    pv, pt = box_plate(-6, 6, -6, 6, -2, 0, 8, 8, 2)
    sig = -0.05 * (1 + 0.2 * rng.uniform(-1, 1, len(pt)))
    pl = Surface(CHARGED, pv, pt, bc=sig)
    return Problem([mol, pl], 80.0, kappa, {}, "sphere_plate")


def three_body(kappa=0.1):
    """Two molecules (different eps_in) and a potential sphere."""
    v1, t1 = icosphere(1, 3.0, (0.0, 0.0, 0.0))
    v2, t2 = icosphere(1, 2.5, (7.0, 0.0, 0.0))
    v3, t3 = icosphere(2, 2.0, (0.0, 6.5, 1.0))
    m1 = Surface(MOLECULE, v1, t1, eps_in=4.0, q_pos=np.array([[0.3, 0.0, 0.0]]), q=np.array([1.0]))
    m2 = Surface(MOLECULE, v2, t2, eps_in=2.0, q_pos=np.array([[7.0, 0.2, 0.0], [6.5, 0, 0]]),
                 q=np.array([-1.0, 0.5]))
    ps = Surface(POTENTIAL, v3, t3, bc=np.full(len(t3), 0.02))
    return Problem([m1, m2, ps], 80.0, kappa, {}, "three_body")


def stern_plate(kappa=0.125):
    """Molecule sphere (r = 3 A, two charges) in a thin Stern shell (r = 3.6
    A, layer permittivity 20) 0.9 A above a charged box: the molecule and its
    Stern surface, and the Stern surface and the box, are within each other's
    2L, so near corrections of every channel are exercised; 320 + 320 + 384
    panels."""
    c = (0.0, 0.0, 4.5)
    v, t = icosphere(2, 3.0, c)
    qpos = np.array([c, [0.8, -0.5, 4.9]])
    mol = Surface(MOLECULE, v, t, eps_in=2.0, q_pos=qpos, q=np.array([1.0, -0.5]))
    sv, st = icosphere(2, 3.6, c)
    stern = Surface(STERN, sv, st, eps_in=20.0, parent=0)
    rng = np.random.default_rng(12)
    pv, pt = box_plate(-6, 6, -6, 6, -2, 0, 8, 8, 2)
    pl = Surface(CHARGED, pv, pt, bc=-0.05 * (1 + 0.2 * rng.uniform(-1, 1, len(pt))))
    return Problem([mol, stern, pl], 80.0, kappa, {}, "stern_plate")


def nested_plate(kappa=0.125):
    """The Stern case with a water cavity (r = 1 A, 80 panels, permittivity
    80) inside the molecule, 0.6 A from its surface and 0.4 A from a charge:
    every nested channel at once (molecule, cavity, Stern layer, solvent,
    plate)."""
    pr = stern_plate(kappa)
    v, t = icosphere(1, 1.0, (-1.2, 0.7, 4.3))
    pr.surfaces.append(Surface(CAVITY, v, t, eps_in=80.0, parent=0))
    pr.name = "nested_plate"
    return pr


def case(name):
    if name == "kirkwood_l1":
        return config_problem("kirkwood", level=1)
    if name == "kirkwood_l2":
        return config_problem("kirkwood", level=2)
    if name == "twosphere_charge_l2":
        return config_problem("twosphere_charge", level=2)
    if name == "twosphere_potential_l2":
        return config_problem("twosphere_potential", level=2)
    if name == "sphere_plate":
        return sphere_plate()
    if name == "sphere_plate_k0":
        return sphere_plate(kappa=0.0)
    if name == "three_body":
        return three_body()
    if name == "three_body_k0":
        return three_body(kappa=0.0)
    if name == "kirkwood_stern_l1":
        return config_problem("kirkwood_stern", level=1)
    if name == "kirkwood_stern_l2":
        return config_problem("kirkwood_stern", level=2)
    if name == "stern_plate":
        return stern_plate()
    if name == "stern_plate_k0":
        return stern_plate(kappa=0.0)
    if name == "kirkwood_water_cavity_l1":
        return config_problem("kirkwood_water_cavity", level=1)
    if name == "nested_plate":
        return nested_plate()
    raise KeyError(name)


SMALL_CASES = ["kirkwood_l1", "kirkwood_l2", "twosphere_charge_l2", "twosphere_potential_l2",
               "sphere_plate", "sphere_plate_k0", "three_body", "three_body_k0",
               "kirkwood_stern_l1", "stern_plate", "stern_plate_k0", "kirkwood_water_cavity_l1", "nested_plate"]
