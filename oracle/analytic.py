"""Analytical solution for a spherical molecule with a central charge next to a
sphere with imposed charge or potential (Section 4 of the paper), and the
closed forms of the isolated bodies.  Reduced units (see ``units``).

Notation follows Section 4: sphere 1 (the molecule) has radius d1 and
interior permittivity eps1 with charge q at its centre; sphere 2 has radius
d2; R is the centre-to-centre distance; eps2 and kappa are the solvent's.
Outside both spheres

    phi_2 = sum_n a_n k_n(kappa r1) P_n(cos th1) + b_n k_n(kappa r2) P_n(cos th2)

(eq. derivation1), where each polar angle is measured from the axis that
points to the other sphere's centre.  The re-expansion of one sphere's
outgoing functions about the other centre uses the addition formula
(eq. addition_formula) with B_nm of eq. Bnm and the Legendre-product
coefficients A^nu_nm of eq. Anm.  Projecting the interface conditions on
sphere 1 (eq. derivation4) and the boundary condition on sphere 2
(eq. derivation5_phi or eq. derivation5_dphi) onto P_j gives a 2N x 2N linear
system for (a_n, b_n); energies follow from eq. phi_reac_an2 / eq. energy_phi
and eq. G_p_int / eq. G_c_int.

i_n and k_n are the modified spherical Bessel functions (scipy's
normalisation, k_n(x) = sqrt(pi / 2x) K_{n+1/2}(x)); every energy is
independent of the normalisation of k_n.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln, spherical_in, spherical_kn

FOUR_PI = 4.0 * math.pi


def legendre_coeff_A(n: int, m: int, nu: int) -> float:
    """A^nu_nm of eq. Anm (nu = 0..min(n, m))."""
    lg = (gammaln(n - nu + 0.5) + gammaln(m - nu + 0.5) + gammaln(nu + 0.5)
          + gammaln(n + m - nu + 1.0) - gammaln(m + n - nu + 1.5)
          - gammaln(n - nu + 1.0) - gammaln(m - nu + 1.0) - gammaln(nu + 1.0))
    return math.exp(lg) * (n + m - 2 * nu + 0.5) / math.pi


def B_matrix(N: int, kR: float) -> np.ndarray:
    """B_nm = sum_nu A^nu_nm k_{n+m-2nu}(kappa R), n, m < N (eq. Bnm)."""
    B = np.zeros((N, N))
    for n in range(N):
        for m in range(N):
            s = 0.0
            for nu in range(min(n, m) + 1):
                s += legendre_coeff_A(n, m, nu) * spherical_kn(n + m - 2 * nu, kR)
            B[n, m] = s
    return B


def two_sphere(q, d1, eps1, d2, eps2, kappa, R, phi0=None, sigma0=None, N=30):
    """Coefficients and energies of the two-sphere problem.

    Exactly one of ``phi0`` (imposed potential) or ``sigma0`` (imposed charge
    density) is given.  Returns dict with a, b, phi_reac0 (at the charge),
    F_solv = q phi_reac / 2 and F_surf (reduced units)."""
    assert (phi0 is None) != (sigma0 is None)
    k = kappa
    n = np.arange(N)
    B = B_matrix(N, k * R)
    kn1, kn1p = spherical_kn(n, k * d1), spherical_kn(n, k * d1, derivative=True)
    in1, in1p = spherical_in(n, k * d1), spherical_in(n, k * d1, derivative=True)
    kn2, kn2p = spherical_kn(n, k * d2), spherical_kn(n, k * d2, derivative=True)
    in2, in2p = spherical_in(n, k * d2), spherical_in(n, k * d2, derivative=True)
    ratio = eps1 / eps2
    M = np.zeros((2 * N, 2 * N))
    rhs = np.zeros(2 * N)
    # eq. derivation4, row j: interface conditions on sphere 1
    for j in range(N):
        M[j, j] = k * kn1p[j] - ratio * j / d1 * kn1[j]
        for m in range(N):
            M[j, N + m] = (2 * j + 1) * B[m, j] * (k * in1p[j] - ratio * j / d1 * in1[j])
    rhs[0] = -ratio * q / (FOUR_PI * eps1 * d1 ** 2)
    # boundary condition on sphere 2, row N + j
    for j in range(N):
        if phi0 is not None:      # eq. derivation5_phi
            M[N + j, N + j] = kn2[j]
            for m in range(N):
                M[N + j, m] = (2 * j + 1) * B[m, j] * in2[j]
        else:                     # eq. derivation5_dphi
            M[N + j, N + j] = k * kn2p[j]
            for m in range(N):
                M[N + j, m] = (2 * j + 1) * B[m, j] * k * in2p[j]
    rhs[N] = phi0 if phi0 is not None else -sigma0 / eps2
    sol = np.linalg.solve(M, rhs)
    a, b = sol[:N], sol[N:]
    # eq. phi_reac_an2
    phi_reac = a[0] * kn1[0] + np.dot(b, B[:, 0]) * in1[0] - q / (FOUR_PI * eps1 * d1)
    F_solv = 0.5 * q * phi_reac
    if phi0 is not None:          # eq. G_p_int
        F_surf = 2 * math.pi * k * phi0 * d2 ** 2 * eps2 * (b[0] * kn2p[0] + np.dot(a, B[:, 0]) * in2p[0])
    else:                         # eq. G_c_int
        F_surf = 2 * math.pi * sigma0 * d2 ** 2 * (b[0] * kn2[0] + np.dot(a, B[:, 0]) * in2[0])
    return dict(a=a, b=b, phi_reac0=phi_reac, F_solv=F_solv, F_surf=F_surf)


def isolated_molecule_solvation(q, d1, eps1, eps2, kappa):
    """Isolated sphere with a central charge via the series (eq. a0_inf)."""
    k0 = spherical_kn(0, kappa * d1)
    k0p = spherical_kn(0, kappa * d1, derivative=True)
    a0 = -q / d1 ** 2 * (eps1 / eps2) / (FOUR_PI * kappa * k0p * eps1)
    return 0.5 * q * (a0 * k0 - q / (FOUR_PI * eps1 * d1))


def isolated_surface_energy(d2, eps2, kappa, phi0=None, sigma0=None):
    """Isolated sphere with imposed potential or charge via the series
    (eq. energy_isolated_phi / energy_isolated_dphi with b_0 at R -> inf)."""
    k0 = spherical_kn(0, kappa * d2)
    k0p = spherical_kn(0, kappa * d2, derivative=True)
    if phi0 is not None:
        b0 = phi0 / k0
        return 2 * math.pi * kappa * phi0 * d2 ** 2 * b0 * k0p * eps2
    b0 = -sigma0 / (eps2 * kappa * k0p)
    return 2 * math.pi * sigma0 * d2 ** 2 * b0 * k0


# ---- textbook closed forms (independent of the series) -------------------

def born_kirkwood(q, d, eps_in, eps_out, kappa):
    """Solvation energy of a charge at the centre of a sphere of radius d in a
    screened solvent (Debye-Hueckel / Born):
        q^2 / (8 pi d) * (1 / (eps_out (1 + kappa d)) - 1 / eps_in)."""
    return q * q / (8.0 * math.pi * d) * (1.0 / (eps_out * (1.0 + kappa * d)) - 1.0 / eps_in)


def born_kirkwood_stern(q, a, b, eps_in, eps_stern, eps_out, kappa):
    """Solvation energy of a charge at the centre of a sphere of radius a
    (eps_in) inside a concentric salt-free shell a < r < b (eps_stern) in a
    screened solvent (eps_out, kappa).  Outside b the potential is
    A exp(-kappa r) / r, in the shell q / (4 pi eps_stern r) + D, inside
    q / (4 pi eps_in r) + C; continuity of phi and eps dphi/dr at b and a
    gives A, D and C, and F = q C / 2:
        q^2 / (8 pi) * (1 / (eps_stern a) - 1 / (eps_in a)
                        + 1 / (eps_out b (1 + kappa b)) - 1 / (eps_stern b)).
    With b = a it is born_kirkwood."""
    return q * q / (8.0 * math.pi) * (1.0 / (eps_stern * a) - 1.0 / (eps_in * a)
                                      + 1.0 / (eps_out * b * (1.0 + kappa * b)) - 1.0 / (eps_stern * b))


def charged_sphere_energy(sigma, d, eps_out, kappa):
    """Free energy 1/2 Q phi(d) of an isolated sphere carrying Q = 4 pi d^2 sigma
    in a screened solvent, phi(d) = Q / (4 pi eps_out d (1 + kappa d))."""
    Q = FOUR_PI * d * d * sigma
    return Q * Q / (8.0 * math.pi * eps_out * d * (1.0 + kappa * d))


def potential_sphere_energy(phi0, d, eps_out, kappa):
    """-1/2 phi0 Q for an isolated sphere held at phi0; the screened field
    gives Q = 4 pi eps_out d (1 + kappa d) phi0."""
    return -2.0 * math.pi * eps_out * d * (1.0 + kappa * d) * phi0 * phi0
