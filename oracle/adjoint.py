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
isolated component that holds the parameter (the Coulomb part cancels); a
molecule's component includes its Stern surface and cavities, whose terms
enter R (cavities: seen from outside) and whose outside rows carry the
molecule's Coulomb sum (cavities).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .bem import CAVITY, CHARGED, MOLECULE, POTENTIAL, SOLVENT, STERN, TWO_ROWS, DenseBEM, components
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
            # phi_reac = R u: the molecule seen from inside, each of its
            # cavities from outside (eq. phi_reac_bem over the region's boundary)
            R = np.zeros((len(ss.q), sysm.n))
            vl, kl, _, _ = layer_blocks(ss.q_pos, sysm.panels[s], sysm.kappa, sysm.k_far,
                                        sysm.k_near, sysm.k_self_edge, near_factor=sysm.near_factor)
            R[:, c:c + ss.nt] = -kl
            R[:, c + ss.nt:c + 2 * ss.nt] = vl
            for cv, sc in enumerate(sysm.surfs):
                if sc.kind == CAVITY and sysm.outer[cv] == s:
                    vc, kc, _, _ = layer_blocks(ss.q_pos, sysm.panels[cv], sysm.kappa, sysm.k_far,
                                                sysm.k_near, sysm.k_self_edge, near_factor=sysm.near_factor)
                    cc = sysm.col_off[cv]
                    R[:, cc:cc + sc.nt] = kc
                    R[:, cc + sc.nt:cc + 2 * sc.nt] = -(sc.eps_in / ss.eps_in) * vc
            R_ops[s] = R
            g += R.T @ ss.q
        elif ss.kind == CHARGED:
            g[c:c + ss.nt] += sysm.sigma[s] * sysm.panels[s].area
        elif ss.kind == POTENTIAL:
            g[c:c + ss.nt] += sysm.eps_out * sysm.phi0[s] * sysm.panels[s].area
    lam = scipy.linalg.lu_solve(lu, g, trans=1)
    grads = {}
    for s, ss in enumerate(sysm.surfs):
        c = sysm.col_off[s]
        if ss.kind == MOLECULE:
            # the Coulomb sum sits on every row of the molecule's interior:
            # its own interior rows and its cavities' outside rows
            bt = np.zeros(len(ss.q))
            for t, st in enumerate(sysm.surfs):
                if t == s:
                    r = sysm.row_off[t]
                elif st.kind == CAVITY and sysm.outer[t] == s:
                    r = sysm.row_off[t] + st.nt
                else:
                    continue
                d = sysm.panels[t].centroid[:, None, :] - ss.q_pos[None, :, :]
                Bq = 1.0 / (FOUR_PI * ss.eps_in * np.sqrt(np.sum(d * d, axis=-1)))   # (nt, nq)
                bt += Bq.T @ lam[r:r + st.nt]
            dq = 0.5 * (R_ops[s] @ u + bt)
            # Coulomb part: dF_coul/dq_k = sum_{l != k} q_l / (4 pi eps r_kl)
            dd = ss.q_pos[:, None, :] - ss.q_pos[None, :, :]
            rr = np.sqrt(np.sum(dd * dd, axis=-1))
            np.fill_diagonal(rr, np.inf)
            dq = dq + (1.0 / (FOUR_PI * ss.eps_in * rr)) @ ss.q
            grads[id(ss)] = ("q", dq)
        elif ss.kind == CHARGED:
            # b_sol(t) += V_Y^{ts} sigma_s / eps_out for every solvent row t
            # only the solvent's rows see the charged surface (from outside)
            bt_lam = np.zeros(ss.nt)
            for t, st in enumerate(sysm.surfs):
                if sysm.outer[t] != SOLVENT:
                    continue
                r = sysm.row_off[t] + (st.nt if st.kind in TWO_ROWS else 0)
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
    comp = {next(i for i, on in enumerate(en) if on and surfs[i].kind not in (STERN, CAVITY)): en
            for en in components(problem)}
    out = []
    for i, ss in enumerate(surfs):
        if i not in comp:
            out.append(None)
            continue
        g_iso = _system_gradient(DenseBEM(problem, k_far, k_near, k_self_edge, enabled=comp[i]))
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
