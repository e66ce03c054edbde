"""torch.autograd.Function for the interaction free energy.

``InteractionEnergy.apply(q, sigma, handle, n_surfaces)`` returns F_int
(kcal/mol, eq. interaction_energy) of the problem held by ``handle`` (a
:class:`PBProblem`) with the molecule's charges ``q`` [e] and the charged
surface's densities ``sigma`` [C/m^2]; its backward pass calls the library's
adjoint gradient (pbt_gradient: transpose treecode product and adjoint
GMRES).  Tensors on the GPU go through the library's device entry points
(pbt_set_charges_dev, pbt_set_bc_dev, pbt_gradient_dev) on the current
stream; CPU tensors through the host ones.  All computation runs in the HIP
library.

Each application saves its own (q, sigma) and the backward pass sets them
again before the gradient, so several applications in one graph, or
parameters changed between forward and backward, give each application the
gradient at its own point.
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
        """q, sigma: numpy arrays or torch tensors (GPU tensors stay on the GPU)."""
        if isinstance(q, torch.Tensor) and q.is_cuda:
            self.solver.set_charges_dev(self.mol_id, self.eps_in, q.detach().to(torch.float64).contiguous())
        else:
            qh = q.detach().cpu().numpy() if isinstance(q, torch.Tensor) else q
            self.solver.set_charges(self.mol_id, self.eps_in, self.q_xyz, np.asarray(qh, dtype=np.float64))
        if isinstance(sigma, torch.Tensor) and sigma.is_cuda:
            self.solver.set_bc_dev(self.sigma_id, sigma.detach().to(torch.float64).contiguous())
        else:
            sh = sigma.detach().cpu().numpy() if isinstance(sigma, torch.Tensor) else sigma
            self.solver.set_bc(self.sigma_id, np.asarray(sh, dtype=np.float64))

    def gradient(self, nq, device):
        """(dF/dsigma, dF/dq) as float64 tensors on `device`."""
        if device.type == "cuda":
            ds = torch.empty(self.n_sigma, dtype=torch.float64, device=device)
            dq = torch.empty(nq, dtype=torch.float64, device=device)
            self.solver.gradient_dev(self.sigma_id, ds, self.mol_id, dq)
            return ds, dq
        ds, dq = self.solver.gradient(self.sigma_id, self.n_sigma, self.mol_id, nq)
        return torch.from_numpy(ds), torch.from_numpy(dq)


class InteractionEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, sigma, handle: PBProblem, n_surfaces: int):
        handle.set_parameters(q, sigma)
        f, _ = handle.solver.interaction_energy(n_surfaces)
        ctx.handle = handle
        ctx.save_for_backward(q, sigma)
        return torch.tensor(f, dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, grad_out):
        h = ctx.handle
        q, sigma = ctx.saved_tensors
        # the gradient at this application's own (q, sigma), whatever the
        # library holds now
        h.set_parameters(q, sigma)
        ds, dq = h.gradient(q.numel(), q.device)
        g = grad_out.to(torch.float64)
        gq = (g.to(dq.device) * dq).to(dtype=q.dtype, device=q.device).reshape(q.shape)
        gs = (g.to(ds.device) * ds).to(dtype=sigma.dtype, device=sigma.device).reshape(sigma.shape)
        return gq, gs, None, None
