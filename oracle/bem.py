"""Dense collocation BEM for molecules, Stern layers and charged / potential
surfaces.

Sections 2 and 3 of the paper, written out for any number of surfaces in one
solvent (the paper's eq. matrix_phi and eq. matrix_dphi are the case of one
molecule and one surface; its conclusion notes that an imposed-BC surface
adds one block row and a molecule boundary two).  A Stern surface (the extra
interfaces of Section 2's closing remarks: an ion-exclusion layer) encloses
one molecule and bounds a salt-free region of its own permittivity between
that molecule and the ionic solvent; it carries two unknowns and two rows
like a molecule.

Every surface separates two regions.  A region is the solvent (Yukawa,
eps_out, kappa), the interior of a molecule (Laplace, eps_in, with the point
charges) or the layer inside a Stern surface (Laplace, that surface's eps_in,
no charges).  A molecule enclosed by a Stern surface has that layer outside
it; every other surface has the solvent outside.

Unknowns per surface, in problem order:
    molecule, stern   [phi (N), dphi/dn inside (N)]
    charged    [phi (N)]          (dphi/dn = -sigma / eps_out is known)
    potential  [dphi/dn (N)]      (phi = phi0 is known)
Rows per surface, in problem order:
    molecule, stern   [row of the inside region (N), row of the outside region (N)]
    charged / potential   [solvent row (N)]

The row of region R at collocation point x_i of surface t is Green's
representation of R (eq. green_identity) taken to the boundary (eq.
integral_eq): u_i / 2, plus for the surface whose inside is R (seen from
inside, Laplace)
    + K_L[i,j] phi_j - V_L[i,j] psi_j,
plus for every surface s with R outside it (seen from outside, with R's
kernel G_R: Yukawa in the solvent, Laplace in a Stern layer)
    - K_R[i,j] phi_out_j + V_R[i,j] psi_out_j,
equal to (1 / eps_t) sum_k q_k / (4 pi |x_i - r_k|) when R is the interior
of molecule t and to 0 otherwise.  Here u = phi (molecule, stern, charged)
or phi0 (potential), phi_out = phi or phi0, psi_out = (eps_s / eps_R) psi
(molecule, stern), -sigma / eps_out (charged) or the unknown psi
(potential).  Known terms move to the right-hand side.  Without Stern
surfaces these are the interior and solvent rows of eq. integral_eq.

Energies (Section 2, Energy calculation), in reduced units then kcal/mol:
    F_solv = 1/2 sum_k q_k phi_reac(r_k),            (eq. solv_energy, first line)
    phi_reac(r_k) = -K_L^{r_k}(phi) + V_L^{r_k}(psi)  (eq. phi_reac_bem)
    F_surf = 1/2 sum_j phi_j sigma_j A_j             (set charge)
           = 1/2 eps_out sum_j phi0_j psi_j A_j      (set potential, with
             sigma = -eps_out dphi/dn so that F = -1/2 sum phi0 sigma A)
    F_coul = sum_{k<l} q_k q_l / (4 pi eps_t r_kl)
    F_total = F_coul + F_surf + F_solv,  F_int = F_total(all) - sum F_total(each),
    a molecule and its Stern surface forming one component.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from .integrals import Panels, layer_blocks
from .units import FOUR_PI, energy_to_kcal, sigma_to_reduced, volts_to_reduced

MOLECULE, CHARGED, POTENTIAL, STERN, CAVITY = 0, 1, 2, 3, 4
TWO_ROWS = (MOLECULE, STERN, CAVITY)
SOLVENT = -1


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

    def __init__(self, problem, k_far=3, k_near=19, k_self_edge=9, enabled=None, near_factor=2.0):
        allsurfs = list(problem.surfaces)
        on = [True] * len(allsurfs) if enabled is None else list(enabled)
        keep = [i for i, o in enumerate(on) if o]
        new_index = {i: k for k, i in enumerate(keep)}
        surfs = [allsurfs[i] for i in keep]
        self.surfs = surfs
        self.eps_out = float(problem.eps_out)
        self.kappa = float(problem.kappa)
        self.k_far, self.k_near, self.k_self_edge = k_far, k_near, k_self_edge
        self.near_factor = float(near_factor)
        self.panels = [Panels(s.verts, s.tris) for s in surfs]
        # the region outside each surface: the solvent, or the layer of the
        # Stern surface that encloses it (the region inside surface k is k)
        self.outer = [SOLVENT] * len(surfs)
        for k, s in enumerate(surfs):
            if s.kind in (STERN, CAVITY):
                par = getattr(s, "parent", -1)
                if par not in new_index or surfs[new_index[par]].kind != MOLECULE:
                    raise ValueError("a Stern surface or cavity needs its molecule in the same system")
                if s.kind == CAVITY:
                    self.outer[k] = new_index[par]
                    continue
                if self.outer[new_index[par]] != SOLVENT:
                    raise ValueError("one Stern surface per molecule")
                self.outer[new_index[par]] = k
        # unknown and row offsets
        self.col_off, self.row_off = [], []
        c = r = 0
        for s in surfs:
            self.col_off.append(c)
            self.row_off.append(r)
            w = 2 * s.nt if s.kind in TWO_ROWS else s.nt
            c += w
            r += w
        self.n = c
        # boundary data in reduced units
        self.sigma = [sigma_to_reduced(np.asarray(s.bc)) if s.kind == CHARGED else None for s in surfs]
        self.phi0 = [volts_to_reduced(np.asarray(s.bc)) if s.kind == POTENTIAL else None for s in surfs]

    def region_eps(self, R):
        return self.eps_out if R == SOLVENT else float(self.surfs[R].eps_in)

    def region_kappa(self, R):
        return self.kappa if R == SOLVENT else 0.0

    # -- blocks ------------------------------------------------------------
    def _blocks(self, t, s, rows=None):
        """V_L, K_L, V_Y, K_Y of target surface t (rows) vs source surface s."""
        pt, ps = self.panels[t], self.panels[s]
        idx = np.arange(pt.n) if rows is None else np.asarray(rows)
        x = pt.centroid[idx]
        self_idx = idx if t == s else None
        return layer_blocks(x, ps, self.kappa, self.k_far, self.k_near, self.k_self_edge,
                            self_idx=self_idx, near_factor=self.near_factor)

    def region_row(self, t, R, rows=None):
        """Rows (panels ``rows`` of surface t) of the equation of region R,
        which must be one of the two regions surface t separates."""
        st = self.surfs[t]
        idx = np.arange(st.nt) if rows is None else np.asarray(rows)
        m = len(idx)
        A = np.zeros((m, self.n))
        b = np.zeros(m)
        ct = self.col_off[t]
        if st.kind == POTENTIAL:
            b -= 0.5 * self.phi0[t][idx]
        else:
            A[np.arange(m), ct + idx] += 0.5
        eps_R = self.region_eps(R)
        for s, ss in enumerate(self.surfs):
            inside = R == s
            outside = self.outer[s] == R
            if not (inside or outside):
                continue
            vl, kl, vy, ky = self._blocks(t, s, idx)
            cs = self.col_off[s]
            ns = ss.nt
            if inside:
                A[:, cs:cs + ns] += kl
                A[:, cs + ns:cs + 2 * ns] += -vl
                continue
            v, k = (vy, ky) if self.region_kappa(R) != 0.0 else (vl, kl)
            if ss.kind in TWO_ROWS:
                A[:, cs:cs + ns] += -k
                A[:, cs + ns:cs + 2 * ns] += (ss.eps_in / eps_R) * v
            elif ss.kind == CHARGED:
                A[:, cs:cs + ns] += -k
                b += v @ (self.sigma[s] / self.eps_out)
            else:
                A[:, cs:cs + ns] += v
                b += k @ self.phi0[s]
        if R != SOLVENT and self.surfs[R].kind == MOLECULE:
            # the molecule's charges lie in its region, whichever of the
            # region's boundaries (the molecule's or a cavity's) t is
            b += self._coulomb_rhs(self.surfs[R], self.panels[t].centroid[idx])
        return A, b

    def row_block(self, t, rows=None):
        """Rows of the operator and right-hand side for target surface t.

        Returns (A_int, b_int, A_sol, b_sol): the rows of the region inside t
        (None unless t is a molecule or a Stern surface) and of the region
        outside it.  ``rows`` selects panels of surface t."""
        A_int = b_int = None
        if self.surfs[t].kind in TWO_ROWS:
            A_int, b_int = self.region_row(t, t, rows)
        A_sol, b_sol = self.region_row(t, self.outer[t], rows)
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
            if st.kind in TWO_ROWS:
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
            w = 2 * st.nt if st.kind in TWO_ROWS else st.nt
            sel = np.nonzero((rows >= r0) & (rows < r0 + w))[0]
            if len(sel) == 0:
                continue
            loc = rows[sel] - r0
            if st.kind in TWO_ROWS:
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
            if ss.kind in TWO_ROWS:
                out.append((u[c:c + ss.nt], u[c + ss.nt:c + 2 * ss.nt]))
            elif ss.kind == CHARGED:
                out.append((u[c:c + ss.nt], -self.sigma[s] / self.eps_out))
            else:
                out.append((self.phi0[s], u[c:c + ss.nt]))
        return out

    def reaction_potential(self, s, phi, psi, parts=None):
        """phi_reac at the charges of molecule s (eq. phi_reac_bem): the
        molecule's boundary seen from inside, and each cavity of it seen
        from outside (Laplace kernel, psi scaled by eps_cavity / eps_in)."""
        ss = self.surfs[s]
        vl, kl, _, _ = layer_blocks(ss.q_pos, self.panels[s], self.kappa, self.k_far,
                                    self.k_near, self.k_self_edge, self_idx=None, near_factor=self.near_factor)
        out = -kl @ phi + vl @ psi
        cavities = [c for c, sc in enumerate(self.surfs) if sc.kind == CAVITY and self.outer[c] == s]
        if cavities and parts is None:
            raise ValueError("the cavities' densities are needed")
        for c in cavities:
            sc = self.surfs[c]
            vc, kc, _, _ = layer_blocks(ss.q_pos, self.panels[c], self.kappa, self.k_far,
                                        self.k_near, self.k_self_edge, self_idx=None,
                                        near_factor=self.near_factor)
            pc, qc = parts[c]
            out += kc @ pc - (sc.eps_in / ss.eps_in) * (vc @ qc)
        return out

    def energies(self, u) -> Energies:
        fc = fs = fsurf = 0.0
        parts = self.split(u)
        for s, (ss, (phi, psi)) in enumerate(zip(self.surfs, parts)):
            if ss.kind == MOLECULE:
                fs += 0.5 * np.dot(ss.q, self.reaction_potential(s, phi, psi, parts))
                fc += coulomb_energy(ss.q_pos, ss.q, ss.eps_in)
            elif ss.kind == CHARGED:
                fsurf += 0.5 * np.sum(phi * self.sigma[s] * self.panels[s].area)
            elif ss.kind == POTENTIAL:
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


def solve_problem(problem, k_far=3, k_near=19, k_self_edge=9, enabled=None, near_factor=2.0):
    """Dense LU solve and energies (kcal/mol).  Returns (Energies, u, system)."""
    sysm = DenseBEM(problem, k_far, k_near, k_self_edge, enabled, near_factor)
    u, _, _ = sysm.solve()
    return sysm.energies(u), u, sysm


def components(problem):
    """Enabled-surface masks of the isolated components: each molecule with
    its Stern surface, and each charged or potential surface alone."""
    surfs = list(problem.surfaces)
    out = []
    for i, s in enumerate(surfs):
        if s.kind in (STERN, CAVITY):
            continue
        out.append([j == i or (t.kind in (STERN, CAVITY) and getattr(t, "parent", -1) == i)
                    for j, t in enumerate(surfs)])
    return out


def interaction_energy(problem, **kw):
    """F_int = F_total(assembly) - sum over components F_total(isolated)
    (eq. interaction_energy)."""
    e_all, _, _ = solve_problem(problem, **kw)
    parts = []
    for en in components(problem):
        e_i, _, _ = solve_problem(problem, enabled=en, **kw)
        parts.append(e_i)
    return e_all.F_total - sum(p.F_total for p in parts), e_all, parts
