"""Dense collocation BEM for molecules and charged / potential surfaces.

Sections 2 and 3 of the paper, written out for any number of surfaces in one
solvent (the paper's eq. matrix_phi and eq. matrix_dphi are the case of one
molecule and one surface; its conclusion notes that an imposed-BC surface
adds one block row and a molecule boundary two).

Unknowns per surface, in problem order:
    molecule   [phi (N), dphi/dn inside (N)]
    charged    [phi (N)]          (dphi/dn = -sigma / eps_out is known)
    potential  [dphi/dn (N)]      (phi = phi0 is known)
Rows per surface, in problem order:
    molecule   [interior row (N), solvent row (N)]
    charged / potential   [solvent row (N)]

Interior row of molecule t at collocation point x_i (eq. integral_eq, first
line, with the 1/eps_1 of eq. green_identity kept on the right):
    phi_i / 2 + sum_j K_L[i,j] phi_j - V_L[i,j] psi_j
        = (1 / eps_t) sum_k q_k / (4 pi |x_i - r_k|)
Solvent row of surface t (eq. integral_eq, second and third lines):
    u_i / 2 + sum_s sum_j ( -K_Y[i,j] phi_out_j + V_Y[i,j] psi_out_j ) = 0
with u = phi (molecule, charged) or phi0 (potential), phi_out = phi or phi0,
psi_out = (eps_s / eps_out) psi (molecule), -sigma / eps_out (charged) or
the unknown psi (potential).  Known terms move to the right-hand side.

Energies (Section 2, Energy calculation), in reduced units then kcal/mol:
    F_solv = 1/2 sum_k q_k phi_reac(r_k),            (eq. solv_energy, first line)
    phi_reac(r_k) = -K_L^{r_k}(phi) + V_L^{r_k}(psi)  (eq. phi_reac_bem)
    F_surf = 1/2 sum_j phi_j sigma_j A_j             (set charge)
           = 1/2 eps_out sum_j phi0_j psi_j A_j      (set potential, with
             sigma = -eps_out dphi/dn so that F = -1/2 sum phi0 sigma A)
    F_coul = sum_{k<l} q_k q_l / (4 pi eps_t r_kl)
    F_total = F_coul + F_surf + F_solv,  F_int = F_total(all) - sum F_total(each)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from .integrals import Panels, layer_blocks
from .units import FOUR_PI, energy_to_kcal, sigma_to_reduced, volts_to_reduced

MOLECULE, CHARGED, POTENTIAL = 0, 1, 2


@dataclass
class Energies:
    F_coul: float
    F_solv: float
    F_surf: float

    @property
    def F_total(self):
        return self.F_coul + self.F_solv + self.F_surf


class DenseBEM:
    """Dense BEM system of a problem (``workloads.Problem``-like object)."""

    def __init__(self, problem, k_far=3, k_near=19, k_self_edge=9, enabled=None):
        surfs = list(problem.surfaces)
        if enabled is not None:
            surfs = [s for s, on in zip(surfs, enabled) if on]
        self.surfs = surfs
        self.eps_out = float(problem.eps_out)
        self.kappa = float(problem.kappa)
        self.k_far, self.k_near, self.k_self_edge = k_far, k_near, k_self_edge
        self.panels = [Panels(s.verts, s.tris) for s in surfs]
        # unknown and row offsets
        self.col_off, self.row_off = [], []
        c = r = 0
        for s in surfs:
            self.col_off.append(c)
            self.row_off.append(r)
            w = 2 * s.nt if s.kind == MOLECULE else s.nt
            c += w
            r += w
        self.n = c
        # boundary data in reduced units
        self.sigma = [sigma_to_reduced(np.asarray(s.bc)) if s.kind == CHARGED else None for s in surfs]
        self.phi0 = [volts_to_reduced(np.asarray(s.bc)) if s.kind == POTENTIAL else None for s in surfs]

    # -- blocks ------------------------------------------------------------
    def _blocks(self, t, s, rows=None):
        """V_L, K_L, V_Y, K_Y of target surface t (rows) vs source surface s."""
        pt, ps = self.panels[t], self.panels[s]
        idx = np.arange(pt.n) if rows is None else np.asarray(rows)
        x = pt.centroid[idx]
        self_idx = idx if t == s else None
        return layer_blocks(x, ps, self.kappa, self.k_far, self.k_near, self.k_self_edge,
                            self_idx=self_idx)

    def row_block(self, t, rows=None):
        """Rows of the operator and right-hand side for target surface t.

        Returns (A_int, b_int, A_sol, b_sol); the interior pair is None unless
        t is a molecule.  ``rows`` selects panels of surface t."""
        st = self.surfs[t]
        nt = st.nt
        idx = np.arange(nt) if rows is None else np.asarray(rows)
        m = len(idx)
        A_sol = np.zeros((m, self.n))
        b_sol = np.zeros(m)
        A_int = b_int = None
        for s, ss in enumerate(self.surfs):
            vl, kl, vy, ky = self._blocks(t, s, idx)
            cs = self.col_off[s]
            ns = ss.nt
            if s == t and st.kind == MOLECULE:
                A_int = np.zeros((m, self.n))
                A_int[:, cs:cs + ns] = kl
                A_int[np.arange(m), cs + idx] += 0.5
                A_int[:, cs + ns:cs + 2 * ns] = -vl
                b_int = self._coulomb_rhs(st, self.panels[t].centroid[idx])
            if ss.kind == MOLECULE:
                A_sol[:, cs:cs + ns] += -ky
                A_sol[:, cs + ns:cs + 2 * ns] += (ss.eps_in / self.eps_out) * vy
            elif ss.kind == CHARGED:
                A_sol[:, cs:cs + ns] += -ky
                b_sol += vy @ (self.sigma[s] / self.eps_out)
            else:
                A_sol[:, cs:cs + ns] += vy
                b_sol += ky @ self.phi0[s]
        ct = self.col_off[t]
        if st.kind in (MOLECULE, CHARGED):
            A_sol[np.arange(m), ct + idx] += 0.5
        else:
            b_sol -= 0.5 * self.phi0[t][idx]
        return A_int, b_int, A_sol, b_sol

    def _coulomb_rhs(self, s, x):
        d = x[:, None, :] - s.q_pos[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=-1))
        return (s.q[None, :] / (FOUR_PI * r)).sum(1) / s.eps_in

    def assemble(self):
        A = np.zeros((self.n, self.n))
        b = np.zeros(self.n)
        for t, st in enumerate(self.surfs):
            A_int, b_int, A_sol, b_sol = self.row_block(t)
            r = self.row_off[t]
            if st.kind == MOLECULE:
                A[r:r + st.nt] = A_int
                b[r:r + st.nt] = b_int
                r += st.nt
            A[r:r + st.nt] = A_sol
            b[r:r + st.nt] = b_sol
        return A, b

    def operator_rows(self, rows):
        """Rows (global row indices) of A and b, computed one block at a time."""
        rows = np.asarray(rows)
        A = np.zeros((len(rows), self.n))
        b = np.zeros(len(rows))
        for t, st in enumerate(self.surfs):
            r0 = self.row_off[t]
            w = 2 * st.nt if st.kind == MOLECULE else st.nt
            sel = np.nonzero((rows >= r0) & (rows < r0 + w))[0]
            if len(sel) == 0:
                continue
            loc = rows[sel] - r0
            if st.kind == MOLECULE:
                ii = sel[loc < st.nt]
                if len(ii):
                    A_int, b_int, _, _ = self.row_block(t, loc[loc < st.nt])
                    A[ii], b[ii] = A_int, b_int
                ss = sel[loc >= st.nt]
                if len(ss):
                    _, _, A_sol, b_sol = self.row_block(t, loc[loc >= st.nt] - st.nt)
                    A[ss], b[ss] = A_sol, b_sol
            else:
                _, _, A_sol, b_sol = self.row_block(t, loc)
                A[sel], b[sel] = A_sol, b_sol
        return A, b

    def solve(self):
        A, b = self.assemble()
        return scipy.linalg.solve(A, b), A, b

    # -- energies -----------------------------------------------------------
    def split(self, u):
        """Per surface (phi, psi) with knowns filled in (psi = interior
        derivative for molecules, solvent-side derivative otherwise)."""
        out = []
        for s, ss in enumerate(self.surfs):
            c = self.col_off[s]
            if ss.kind == MOLECULE:
                out.append((u[c:c + ss.nt], u[c + ss.nt:c + 2 * ss.nt]))
            elif ss.kind == CHARGED:
                out.append((u[c:c + ss.nt], -self.sigma[s] / self.eps_out))
            else:
                out.append((self.phi0[s], u[c:c + ss.nt]))
        return out

    def reaction_potential(self, s, phi, psi):
        """phi_reac at the charges of molecule s (eq. phi_reac_bem)."""
        ss = self.surfs[s]
        vl, kl, _, _ = layer_blocks(ss.q_pos, self.panels[s], self.kappa, self.k_far,
                                    self.k_near, self.k_self_edge, self_idx=None)
        return -kl @ phi + vl @ psi

    def energies(self, u) -> Energies:
        fc = fs = fsurf = 0.0
        for s, (ss, (phi, psi)) in enumerate(zip(self.surfs, self.split(u))):
            if ss.kind == MOLECULE:
                fs += 0.5 * np.dot(ss.q, self.reaction_potential(s, phi, psi))
                fc += coulomb_energy(ss.q_pos, ss.q, ss.eps_in)
            elif ss.kind == CHARGED:
                fsurf += 0.5 * np.sum(phi * self.sigma[s] * self.panels[s].area)
            else:
                fsurf += 0.5 * self.eps_out * np.sum(self.phi0[s] * psi * self.panels[s].area)
        return Energies(energy_to_kcal(fc), energy_to_kcal(fs), energy_to_kcal(fsurf))


def coulomb_energy(pos, q, eps):
    """sum_{k<l} q_k q_l / (4 pi eps r_kl), reduced units."""
    pos = np.asarray(pos)
    n = len(q)
    e = 0.0
    for k in range(n - 1):
        d = pos[k + 1:] - pos[k]
        r = np.sqrt(np.sum(d * d, axis=1))
        e += np.sum(q[k] * q[k + 1:] / r)
    return e / (FOUR_PI * eps)


def solve_problem(problem, k_far=3, k_near=19, k_self_edge=9, enabled=None):
    """Dense LU solve and energies (kcal/mol).  Returns (Energies, u, system)."""
    sysm = DenseBEM(problem, k_far, k_near, k_self_edge, enabled)
    u, _, _ = sysm.solve()
    return sysm.energies(u), u, sysm


def interaction_energy(problem, **kw):
    """F_int = F_total(assembly) - sum over components F_total(isolated)
    (eq. interaction_energy).  Components are the surfaces."""
    e_all, _, _ = solve_problem(problem, **kw)
    parts = []
    for i in range(len(problem.surfaces)):
        en = [j == i for j in range(len(problem.surfaces))]
        e_i, _, _ = solve_problem(problem, enabled=en, **kw)
        parts.append(e_i)
    return e_all.F_total - sum(p.F_total for p in parts), e_all, parts
