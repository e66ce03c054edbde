"""Seeded synthetic inputs for the treecode-BEM Poisson-Boltzmann solver.

This package only generates geometry and charges (triangle meshes, point
charges, imposed surface charge or potential, rigid rotations).  It holds
none of the boundary-element arithmetic: no integrals, no operators, no
energies.  Both the independent CPU oracle and the HIP library consume the
arrays it produces, byte for byte.

Units at this level are the ones the C ABI takes: lengths in Angstrom,
charges in e, imposed charge density in C/m^2, imposed potential in V,
Debye parameter kappa in 1/Angstrom.
"""
from .meshes import icosphere, star_directions, star_surface, box_plate, octa_bisection_sphere
from .problems import Surface, Problem, config_problem, CONFIG_NAMES

__all__ = [
    "icosphere", "star_directions", "star_surface", "box_plate", "octa_bisection_sphere",
    "Surface", "Problem", "config_problem", "CONFIG_NAMES",
]
