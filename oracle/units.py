"""Reduced units of the oracle.

The model equations (Section 2, eq. pde and eq. free-space) absorb the vacuum
permittivity: G = 1/(4 pi r) and the source term is q/eps.  The paper never
states units; the oracle reads them as lengths in Angstrom, charges in e,
relative permittivities, so a potential is in e/(eps0 A) and an energy in
e^2/(eps0 A).  The boundary takes sigma in C/m^2 and phi0 in V and reports
energies in kcal/mol; these constants convert.  CODATA-2018 exact values.
"""
import math

E_CHARGE = 1.602176634e-19      # C
EPS0 = 8.8541878128e-12         # F/m
N_AVOGADRO = 6.02214076e23      # 1/mol
CAL = 4.184                     # J
ANGSTROM = 1e-10                # m

#: one reduced potential unit e/(eps0 A) in volts
POTENTIAL_UNIT_V = E_CHARGE / (EPS0 * ANGSTROM)
#: one reduced energy unit e^2/(eps0 A) in kcal/mol
ENERGY_UNIT_KCAL = E_CHARGE ** 2 / (EPS0 * ANGSTROM) * N_AVOGADRO / (CAL * 1000.0)
#: 1 C/m^2 in e/A^2
SIGMA_SI_TO_REDUCED = ANGSTROM ** 2 / E_CHARGE


def sigma_to_reduced(sigma_c_per_m2):
    return sigma_c_per_m2 * SIGMA_SI_TO_REDUCED


def volts_to_reduced(phi_v):
    return phi_v / POTENTIAL_UNIT_V


def energy_to_kcal(e_reduced):
    return e_reduced * ENERGY_UNIT_KCAL


FOUR_PI = 4.0 * math.pi
