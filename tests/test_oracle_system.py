"""Pins for the oracle's analytic module, dense BEM system and adjoint.

What fixes each part, independently of the part itself:

* analytic series (Section 4): the Legendre-product identity that eq. Anm
  encodes, the addition theorem pointwise, and the textbook closed forms of
  the isolated bodies at R -> infinity;
* dense BEM (Sections 2-3): O(1/N) convergence to the Kirkwood / Born closed
  form and to the two-sphere series, with observed order near 1 (the paper
  reports 1.007, Section 5.1); the solid-angle sum of the double layer, the
  Gauss-law flux of the interior normal derivative; exact invariance of the
  discrete problem under rigid motions; reciprocity of the reaction field;
* adjoint: central differences, which are exact for a quadratic form.
"""
import copy
import json
import math
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, spherical_in, spherical_kn

from oracle import analytic
from oracle.adjoint import interaction_gradient
from oracle.bem import DenseBEM, interaction_energy, solve_problem
from oracle.integrals import Panels, layer_blocks
from oracle.units import ENERGY_UNIT_KCAL, POTENTIAL_UNIT_V, energy_to_kcal, sigma_to_reduced, volts_to_reduced
from workloads.problems import config_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_unit_constants():
    # Coulomb's constant e^2/(4 pi eps0 A) is 332.0637 kcal/mol (CODATA 2018)
    assert abs(ENERGY_UNIT_KCAL / (4 * math.pi) - 332.0637133) < 1e-6
    assert abs(POTENTIAL_UNIT_V - 180.9512818) < 1e-6
    assert abs(sigma_to_reduced(0.05) - 3.1207545372e-3) < 1e-12


@pytest.mark.parametrize("n,m", [(0, 0), (1, 1), (2, 3), (4, 4), (1, 5), (6, 3)])
def test_legendre_product_identity(n, m):
    x = np.linspace(-1, 1, 41)
    lhs = eval_legendre(n, x) * eval_legendre(m, x)
    rhs = sum(analytic.legendre_coeff_A(n, m, nu) * eval_legendre(n + m - 2 * nu, x)
              for nu in range(min(n, m) + 1))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_addition_theorem_pointwise(n):
    """k_n(kappa r2) P_n(cos th2) = sum_m (2m+1) B_nm i_m(kappa r1) P_m(cos th1),
    polar angles measured toward the other centre."""
    kappa, R, N = 0.125, 12.0, 60
    B = analytic.B_matrix(N, kappa * R)
    rng = np.random.default_rng(7)
    c1, c2 = np.zeros(3), np.array([0.0, 0.0, R])
    for _ in range(5):
        p = rng.normal(size=3)
        p *= rng.uniform(1.0, 6.0) / np.linalg.norm(p)
        r1v, r2v = p - c1, p - c2
        r1, r2 = np.linalg.norm(r1v), np.linalg.norm(r2v)
        cos1 = r1v[2] / r1                 # axis from centre 1 toward centre 2
        cos2 = -r2v[2] / r2                # axis from centre 2 toward centre 1
        lhs = spherical_kn(n, kappa * r2) * eval_legendre(n, cos2)
        m = np.arange(N)
        rhs = np.sum((2 * m + 1) * B[n, :] * spherical_in(m, kappa * r1) * eval_legendre(m, cos1))
        assert abs(lhs - rhs) < 1e-10 * abs(lhs) + 1e-14


def test_series_reduces_to_closed_forms():
    q, d1, e1, d2, e2, k = 1.0, 4.0, 4.0, 4.0, 80.0, 0.125
    sig, phi = sigma_to_reduced(0.05), volts_to_reduced(0.05)
    assert abs(analytic.isolated_molecule_solvation(q, d1, e1, e2, k)
               - analytic.born_kirkwood(q, d1, e1, e2, k)) < 1e-15
    assert abs(analytic.isolated_surface_energy(d2, e2, k, sigma0=sig)
               - analytic.charged_sphere_energy(sig, d2, e2, k)) < 1e-16
    assert abs(analytic.isolated_surface_energy(d2, e2, k, phi0=phi)
               - analytic.potential_sphere_energy(phi, d2, e2, k)) < 1e-16
    # far apart, the two-sphere energies tend to the isolated ones
    r = analytic.two_sphere(q, d1, e1, d2, e2, k, 300.0, sigma0=sig, N=20)
    assert abs(r["F_solv"] - analytic.born_kirkwood(q, d1, e1, e2, k)) < 1e-12
    assert abs(r["F_surf"] - analytic.charged_sphere_energy(sig, d2, e2, k)) < 1e-12


def test_series_converged_and_golden():
    """Energies of the two-sphere case stored by tests/golden/make_golden.py."""
    with open(os.path.join(GOLDEN, "twosphere_analytic.json")) as f:
        gold = json.load(f)
    q, d1, e1, d2, e2, k, R = 1.0, 4.0, 4.0, 4.0, 80.0, 0.125, 12.0
    for case, kw in (("charge", dict(sigma0=sigma_to_reduced(0.05))),
                     ("potential", dict(phi0=volts_to_reduced(0.05)))):
        a = analytic.two_sphere(q, d1, e1, d2, e2, k, R, N=20, **kw)
        b = analytic.two_sphere(q, d1, e1, d2, e2, k, R, N=40, **kw)
        assert abs(a["F_solv"] - b["F_solv"]) < 1e-14
        assert abs(energy_to_kcal(b["F_solv"]) - gold[case]["F_solv_asm"]) < 1e-9
        assert abs(energy_to_kcal(b["F_surf"]) - gold[case]["F_surf_asm"]) < 1e-9


def _order(errs):
    return math.log(abs(errs[-2] / errs[-1])) / math.log(4.0)


def test_kirkwood_convergence():
    exact = energy_to_kcal(analytic.born_kirkwood(1.0, 4.0, 4.0, 80.0, 0.125))
    errs = []
    for lv in (1, 2, 3):
        e, _, _ = solve_problem(config_problem("kirkwood", level=lv))
        errs.append((e.F_solv - exact) / exact)
    assert abs(errs[-1]) < 5e-3
    assert abs(errs[0]) > abs(errs[1]) > abs(errs[2])
    assert 0.85 < _order(errs) < 1.15


def test_kirkwood_stern_closed_form_limits():
    """The Stern-shell closed form reduces to Born/Kirkwood for a shell of
    zero thickness, and for a shell with the solvent's permittivity and no
    screening (the layer then changes nothing)."""
    q, a, e1, e2, k = 1.0, 4.0, 4.0, 80.0, 0.125
    assert abs(analytic.born_kirkwood_stern(q, a, a, e1, 20.0, e2, k)
               - analytic.born_kirkwood(q, a, e1, e2, k)) < 1e-15
    assert abs(analytic.born_kirkwood_stern(q, a, 7.0, e1, e2, e2, 0.0)
               - analytic.born_kirkwood(q, a, e1, e2, 0.0)) < 1e-15


def test_kirkwood_stern_convergence():
    """Dense BEM of a charged sphere inside a Stern sphere (two interfaces,
    four block rows) converges at first order in N to the closed form."""
    exact = energy_to_kcal(analytic.born_kirkwood_stern(1.0, 4.0, 6.0, 4.0, 20.0, 80.0, 0.125))
    errs = []
    for lv in (1, 2, 3):
        e, _, _ = solve_problem(config_problem("kirkwood_stern", level=lv))
        errs.append((e.F_solv - exact) / exact)
    assert abs(errs[-1]) < 5e-3
    assert abs(errs[0]) > abs(errs[1]) > abs(errs[2])
    assert 0.85 < _order(errs) < 1.15


def test_fictitious_cavity_converges_to_kirkwood():
    """A cavity whose permittivity equals the molecule's is no interface at
    all: the dense BEM with it (two more block rows, the cavity's terms in
    the molecule's interior equation and in the reaction potential)
    converges at first order to Kirkwood's closed form, and its difference
    to the system without the cavity falls like 1/N."""
    exact = energy_to_kcal(analytic.born_kirkwood(1.0, 4.0, 4.0, 80.0, 0.125))
    errs, diffs = [], []
    for lv in (1, 2, 3):
        e, _, _ = solve_problem(config_problem("kirkwood_cavity", level=lv))
        e0, _, _ = solve_problem(config_problem("kirkwood", level=lv))
        errs.append((e.F_solv - exact) / exact)
        diffs.append(e.F_solv - e0.F_solv)
    assert abs(errs[-1]) < 5e-3
    assert abs(errs[0]) > abs(errs[1]) > abs(errs[2])
    assert 0.85 < _order(errs) < 1.15
    assert 0.85 < _order(diffs) < 1.15


@pytest.mark.parametrize("case", ["charge", "potential"])
def test_two_sphere_interaction_convergence(case):
    """F_int of the dense BEM against the series, levels 1..3 (80..1280 panels
    per sphere); the paper reports observed order 1.007 (Section 5.1)."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        paper = json.load(f)
    with open(os.path.join(GOLDEN, "twosphere_analytic.json")) as f:
        exact = json.load(f)[case]["F_int"]
    errs = []
    for lv in (1, 2, 3):
        fint, _, _ = interaction_energy(config_problem("twosphere_" + case, level=lv))
        errs.append((fint - exact) / exact)
    assert abs(errs[0]) > abs(errs[1]) > abs(errs[2])
    assert abs(_order(errs) - paper["twosphere_observed_order"]["value"]) < 0.2


def test_double_layer_solid_angle():
    """sum_j K_L[i, j] -> -1/2 on a closed surface (jump relation)."""
    dev = []
    for lv in (2, 3):
        p = config_problem("kirkwood", level=lv)
        pan = Panels(p.surfaces[0].verts, p.surfaces[0].tris)
        _, kl, _, _ = layer_blocks(pan.centroid, pan, 0.125, self_idx=np.arange(pan.n))
        s = kl.sum(1)
        dev.append(np.max(np.abs(s + 0.5)))
    assert dev[1] < 5e-3 and dev[1] < dev[0]


def test_gauss_law_flux():
    """sum_j A_j dphi/dn_j -> -Q / eps_in for the interior normal derivative."""
    devs = []
    for lv in (2, 3):
        e, u, sysm = solve_problem(config_problem("kirkwood", level=lv))
        phi, psi = sysm.split(u)[0]
        flux = np.sum(sysm.panels[0].area * psi)
        devs.append(abs(flux + 1.0 / 4.0))
    assert devs[1] < 1e-2 * 0.25 and devs[1] < devs[0]


def test_rigid_motion_invariance():
    p = config_problem("twosphere_charge", level=2)
    e0, _, _ = solve_problem(p)
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    Rm = Rm @ np.array([[1, 0, 0], [0, math.cos(0.3), -math.sin(0.3)], [0, math.sin(0.3), math.cos(0.3)]])
    sh = np.array([3.0, -2.0, 5.0])
    p2 = copy.deepcopy(p)
    for s in p2.surfaces:
        s.verts = s.verts @ Rm.T + sh
        if s.q_pos is not None:
            s.q_pos = s.q_pos @ Rm.T + sh
    e1, _, _ = solve_problem(p2)
    for a, b in ((e0.F_solv, e1.F_solv), (e0.F_surf, e1.F_surf)):
        assert abs(a - b) < 1e-10 * abs(a)


def test_reaction_field_reciprocity():
    """phi_reac at b from a unit charge at a equals the reverse, up to the
    discretisation error, which falls as the mesh is refined."""
    a, b = np.array([1.0, 0.5, -0.3]), np.array([-0.8, 1.2, 0.6])
    asym = []
    for lv in (1, 2, 3):
        vals = []
        for src, dst in ((a, b), (b, a)):
            p = config_problem("kirkwood", level=lv)
            p.surfaces[0].q_pos = src[None, :]
            sysm = DenseBEM(p)
            u, _, _ = sysm.solve()
            phi, psi = sysm.split(u)[0]
            vl, kl, _, _ = layer_blocks(dst[None, :], sysm.panels[0], 0.125)
            vals.append((-kl @ phi + vl @ psi)[0])
        asym.append(abs(vals[0] - vals[1]) / abs(vals[0]))
    assert asym[2] < asym[0] and asym[2] < 2e-3


def test_adjoint_gradient_is_exact_for_quadratic_form():
    p = config_problem("twosphere_charge", level=1)
    rng = np.random.default_rng(0)
    p.surfaces[1].bc = 0.05 * (1 + 0.3 * rng.uniform(-1, 1, p.surfaces[1].nt))
    p.surfaces[0].q_pos = np.array([[0, 0, 0.0], [1.0, 0.5, 0.3]])
    p.surfaces[0].q = np.array([1.0, -0.5])
    g = interaction_gradient(p)

    def F(pp):
        return interaction_energy(pp)[0]

    for j in (0, 17, 63):
        h = 0.02                          # large step: central differences are exact here
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        pp.surfaces[1].bc[j] += h
        pm.surfaces[1].bc[j] -= h
        fd = (F(pp) - F(pm)) / (2 * h)
        assert abs(fd - g[1][j]) < 1e-8 * abs(g[1][j])
    for k in (0, 1):
        h = 0.3
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        pp.surfaces[0].q[k] += h
        pm.surfaces[0].q[k] -= h
        fd = (F(pp) - F(pm)) / (2 * h)
        assert abs(fd - g[0][k]) < 1e-8 * abs(g[0][k])


def test_adjoint_gradient_with_stern_layer_and_cavity():
    """The same exactness with a Stern layer and a cavity around / inside the
    molecule: the gradient through the dense transpose (cavity terms in the
    reaction potential, the Coulomb sum on the cavity's outside rows, the
    charged surface seen only by the solvent's rows) matches central
    differences of F_int, the molecule isolated with its Stern surface and
    cavity."""
    from workloads.meshes import icosphere
    from workloads.problems import CAVITY, CHARGED, MOLECULE, STERN, Problem, Surface
    rng = np.random.default_rng(1)
    v, t = icosphere(1, 4.0, (0.0, 0.0, 0.0))
    mol = Surface(MOLECULE, v, t, eps_in=4.0, q_pos=np.array([[0, 0, 0.0], [1.0, 0.5, 0.3]]),
                  q=np.array([1.0, -0.5]))
    v, t = icosphere(1, 5.5, (0.0, 0.0, 0.0))
    stern = Surface(STERN, v, t, eps_in=40.0, parent=0)
    v, t = icosphere(1, 1.0, (-1.8, 0.6, 0.0))
    cav = Surface(CAVITY, v, t, eps_in=80.0, parent=0)
    v, t = icosphere(1, 3.0, (0.0, 0.0, 11.0))
    pl = Surface(CHARGED, v, t, bc=0.05 * (1 + 0.3 * rng.uniform(-1, 1, len(t))))
    p = Problem([mol, stern, cav, pl], 80.0, 0.125, {}, "nested_gradient")
    g = interaction_gradient(p)
    assert g[1] is None and g[2] is None

    def F(pp):
        return interaction_energy(pp)[0]

    for j in (0, 41):
        h = 0.02
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        pp.surfaces[3].bc[j] += h
        pm.surfaces[3].bc[j] -= h
        fd = (F(pp) - F(pm)) / (2 * h)
        assert abs(fd - g[3][j]) < 1e-8 * abs(g[3][j])
    for k in (0, 1):
        h = 0.3
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        pp.surfaces[0].q[k] += h
        pm.surfaces[0].q[k] -= h
        fd = (F(pp) - F(pm)) / (2 * h)
        assert abs(fd - g[0][k]) < 1e-8 * abs(g[0][k])


def test_coulomb_energy_hand_computed():
    """F_coul = sum over pairs k < l of q_k q_l / (4 pi eps_in r_kl) (the
    Coulomb term of eq. total_energy), against a value worked out by hand:
    charges 1, -2, 1/2 e at (0,0,0), (3,0,0), (0,4,0) A (a 3-4-5 triangle),
    eps_in = 2: (1 (-2) / 3 + 1 (1/2) / 4 + (-2)(1/2) / 5) / (8 pi)
    = -89 / (960 pi) reduced units.  Each pair counts once, with 1/eps_in."""
    from oracle.bem import coulomb_energy
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [0.0, 4.0, 0.0]])
    q = np.array([1.0, -2.0, 0.5])
    expect = -89.0 / (960.0 * math.pi)
    assert abs(coulomb_energy(pos, q, 2.0) - expect) <= 1e-15 * abs(expect)
    # a lone charge has no Coulomb energy; a zero charge adds none
    assert coulomb_energy(pos[:1], q[:1], 2.0) == 0.0
    pos4 = np.vstack([pos, [[1.0, 1.0, 1.0]]])
    assert abs(coulomb_energy(pos4, np.append(q, 0.0), 2.0) - expect) <= 1e-15 * abs(expect)
    # and the dense system reports it (kcal/mol) for a molecule holding them
    from oracle.bem import MOLECULE
    from workloads.meshes import icosphere
    from workloads.problems import Problem, Surface
    v, t = icosphere(1, 6.0, (0.0, 0.0, 0.0))
    pr = Problem([Surface(MOLECULE, v, t, eps_in=2.0, q_pos=pos, q=q)], 80.0, 0.125, {}, "three_charges")
    e, _, _ = solve_problem(pr)
    assert abs(e.F_coul - expect * ENERGY_UNIT_KCAL) <= 1e-12 * abs(expect * ENERGY_UNIT_KCAL)


@pytest.mark.parametrize("name", ["stern_plate", "nested_plate", "three_body"])
def test_operator_rows_match_assembly(name):
    """The row-at-a-time form the full-size parity tests use equals the
    assembled operator and right-hand side on the same rows (molecule,
    Stern, cavity and imposed-BC row blocks, every block's first and last
    row included)."""
    from tests.gpu_cases import case
    sysm = DenseBEM(case(name))
    A, b = sysm.assemble()
    edges = []
    for t, st in enumerate(sysm.surfs):
        w = 2 * st.nt if st.kind in (0, 3, 4) else st.nt
        r0 = sysm.row_off[t]
        edges += [r0, r0 + w - 1] + ([r0 + st.nt - 1, r0 + st.nt] if w == 2 * st.nt else [])
    rng = np.random.default_rng(21)
    rows = np.unique(np.concatenate([edges, rng.choice(sysm.n, 40, replace=False)]))
    rng.shuffle(rows)
    Ar, br = sysm.operator_rows(rows)
    scale = np.max(np.abs(A))
    assert np.max(np.abs(Ar - A[rows])) <= 1e-15 * scale
    assert np.max(np.abs(br - b[rows])) <= 1e-15 * np.max(np.abs(b))
