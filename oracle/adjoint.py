"""Gradient of the free energy through the dense transpose.

For a fixed geometry the discrete system is A u = B p + b0, where p holds the
point charges q (e) and the imposed charge densities sigma (reduced units),
and b0 collects imposed potentials.  Every energy of Section 2 is a bilinear
form in (p, u): F = 1/2 g(p)^T u + F_coul(q) with g(p) = C p + g0:

* solvation   F_solv = 1/2 q^T (R u), R the phi_reac evaluator
              (eq. phi_reac_bem), so C_q = R^T;
* set charge  F_surf = 1/2 sum_j phi_j sigma_j A_j, so C_sigma = diag(A)
              on the phi unknowns of the surface;
* set potential  F_surf = 1/2 eps_out sum_j phi0_j psi_j A_j, a constant g0.

Hence  dF/dp = 1/2 (C^T u + B^T lambda) + dF_coul/dp  with  A^T lambda = g.
The interaction energy's gradient is the assembly's minus that of each
isolated component that holds the parameter (the Coulomb part cancels).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .bem import CHARGED, MOLECULE, POTENTIAL, DenseBEM
from .integrals import layer_blocks
from .units import FOUR_PI, SIGMA_SI_TO_REDUCED, energy_to_kcal


def _system_gradient(sysm: DenseBEM):
    """dF_total/dq per molecule and dF_total/dsigma per charged surface, in
    reduced units (per e and per e/A^2), for one system."""
    A, b = sysm.assemble()
    lu = scipy.linalg.lu_factor(A)
    u = scipy.linalg.lu_solve(lu, b)
    g = np.zeros(sysm.n)
    R_ops = {}
    for s, ss in enumerate(sysm.surfs):
        c = sysm.col_off[s]
        if ss.kind == MOLECULE:
            vl, kl, _, _ = layer_blocks(ss.q_pos, sysm.panels[s], sysm.kappa, sysm.k_far,
                                        sysm.k_near, sysm.k_self_edge)
            R = np.concatenate([-kl, vl], axis=1)          # (nq, 2 nt)
            R_ops[s] = R
            g[c:c + 2 * ss.nt] += R.T @ ss.q
        elif ss.kind == CHARGED:
            g[c:c + ss.nt] += sysm.sigma[s] * sysm.panels[s].area
        else:
            g[c:c + ss.nt] += sysm.eps_out * sysm.phi0[s] * sysm.panels[s].area
    lam = scipy.linalg.lu_solve(lu, g, trans=1)
    grads = {}
    for s, ss in enumerate(sysm.surfs):
        c = sysm.col_off[s]
        if ss.kind == MOLECULE:
            r = sysm.row_off[s]
            x = sysm.panels[s].centroid
            d = x[:, None, :] - ss.q_pos[None, :, :]
            Bq = 1.0 / (FOUR_PI * ss.eps_in * np.sqrt(np.sum(d * d, axis=-1)))   # (nt, nq)
            dq = 0.5 * (R_ops[s] @ u[c:c + 2 * ss.nt] + Bq.T @ lam[r:r + ss.nt])
            # Coulomb part: dF_coul/dq_k = sum_{l != k} q_l / (4 pi eps r_kl)
            dd = ss.q_pos[:, None, :] - ss.q_pos[None, :, :]
            rr = np.sqrt(np.sum(dd * dd, axis=-1))
            np.fill_diagonal(rr, np.inf)
            dq = dq + (1.0 / (FOUR_PI * ss.eps_in * rr)) @ ss.q
            grads[id(ss)] = ("q", dq)
        elif ss.kind == CHARGED:
            # b_sol(t) += V_Y^{ts} sigma_s / eps_out for every solvent row t
            bt_lam = np.zeros(ss.nt)
            for t, st in enumerate(sysm.surfs):
                r = sysm.row_off[t] + (st.nt if st.kind == MOLECULE else 0)
                _, _, vy, _ = sysm._blocks(t, s)
                bt_lam += vy.T @ lam[r:r + st.nt] / sysm.eps_out
            dsig = 0.5 * (sysm.panels[s].area * u[c:c + ss.nt] + bt_lam)
            grads[id(ss)] = ("sigma", dsig)
    return grads


def interaction_gradient(problem, k_far=3, k_near=19, k_self_edge=9):
    """Gradient of F_int: returns list aligned with problem.surfaces holding
    dF_int/dq [kcal/mol per e] for molecules, dF_int/dsigma
    [kcal/mol per C/m^2] for charged surfaces, None otherwise."""
    surfs = problem.surfaces
    g_all = _system_gradient(DenseBEM(problem, k_far, k_near, k_self_edge))
    out = []
    for i, ss in enumerate(surfs):
        en = [j == i for j in range(len(surfs))]
        g_iso = _system_gradient(DenseBEM(problem, k_far, k_near, k_self_edge, enabled=en))
        if id(ss) not in g_all:
            out.append(None)
            continue
        kind, ga = g_all[id(ss)]
        _, gi = g_iso[id(ss)]
        d = energy_to_kcal(ga - gi)
        if kind == "sigma":
            d = d * SIGMA_SI_TO_REDUCED
        out.append(d)
    return out
