"""torch.autograd.Function for the interaction free energy.

``InteractionEnergy.apply(q, sigma, handle)`` returns F_int (kcal/mol) of the
problem held by ``handle`` (a :class:`PBProblem`) with the molecule's charges
``q`` [e] and the charged surface's densities ``sigma`` [C/m^2]; its backward
pass calls the library's adjoint gradient (pbt_gradient: transpose treecode
product and adjoint GMRES).  Tensors are copied to host buffers for the C ABI;
all computation runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from .pbt import Solver


class PBProblem:
    """A solver plus the ids of one molecule and one charged surface."""

    def __init__(self, solver: Solver, mol_id: int, eps_in: float, q_xyz, sigma_id: int, n_sigma: int):
        self.solver = solver
        self.mol_id = mol_id
        self.eps_in = float(eps_in)
        self.q_xyz = np.ascontiguousarray(np.asarray(q_xyz, dtype=np.float64))
        self.sigma_id = sigma_id
        self.n_sigma = n_sigma
        self.n_surfaces = None

    def set_parameters(self, q, sigma):
        self.solver.set_charges(self.mol_id, self.eps_in, self.q_xyz, np.asarray(q, dtype=np.float64))
        self.solver.set_bc(self.sigma_id, np.asarray(sigma, dtype=np.float64))


class InteractionEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, sigma, handle: PBProblem, n_surfaces: int):
        handle.set_parameters(q.detach().cpu().numpy(), sigma.detach().cpu().numpy())
        f, _ = handle.solver.interaction_energy(n_surfaces)
        ctx.handle = handle
        ctx.shapes = (q.shape, sigma.shape, q.dtype, sigma.dtype, q.device, sigma.device)
        return torch.tensor(f, dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, grad_out):
        h = ctx.handle
        qs, ss, qd, sd, qdev, sdev = ctx.shapes
        ds, dq = h.solver.gradient(h.sigma_id, h.n_sigma, h.mol_id, int(np.prod(qs)))
        g = float(grad_out)
        gq = torch.tensor(g * dq, dtype=qd, device=qdev).reshape(qs)
        gs = torch.tensor(g * ds, dtype=sd, device=sdev).reshape(ss)
        return gq, gs, None, None
