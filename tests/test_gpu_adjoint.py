"""GPU parity of the adjoint: exact transpose of the treecode operator,
gradients of F_int against the oracle's dense-transpose gradient, central
differences of the GPU's own F_int, and the autograd wrapper.

Bars: the transpose identity <A x, l> = <x, A^T l> to 1e-12 (FP64) for the
treecode operator (same lists and expansions, summed in another order);
direct FP64 A^T element-wise within 1e-11 of the oracle's dense A^T;
gradients within 1e-6 (relative to the largest entry) of the oracle's dense
gradient (FP64 direct form, GMRES tol 1e-11); central differences of the
treecode F_int (exactly quadratic in the parameters) within 1e-5.
"""
import copy

import numpy as np
import pytest

from oracle.adjoint import interaction_gradient
from oracle.bem import DenseBEM
from paper_1506_03745_amd import FP64, MIXED, from_problem
from tests.gpu_cases import case

pytestmark = pytest.mark.gpu


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name", ["sphere_plate", "three_body", "twosphere_potential_l2", "stern_plate",
                                  "nested_plate"])
@pytest.mark.parametrize("treecode", [0, 1])
def test_transpose_identity(name, treecode):
    s, _ = from_problem(case(name), treecode=treecode, ncrit=24, theta=0.5, taylor_p=6)
    n = s.num_unknowns()
    rng = np.random.default_rng(3)
    for _ in range(2):
        x, l = rng.standard_normal(n), rng.standard_normal(n)
        ax = s.matvec(x)
        atl = s.matvec(l, transpose=True)
        lhs, rhs = np.dot(ax, l), np.dot(x, atl)
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax) * np.linalg.norm(l)
        atl32 = s.matvec(l, transpose=True, prec=MIXED)
        assert rel_inf(atl32, atl) < 5e-5


@pytest.mark.parametrize("name", ["kirkwood_l1", "sphere_plate", "three_body", "stern_plate_k0", "nested_plate"])
def test_direct_transpose_matches_oracle(name):
    A, _ = DenseBEM(case(name)).assemble()
    s, _ = from_problem(case(name), treecode=0)
    l = np.random.default_rng(4).standard_normal(A.shape[0])
    assert rel_inf(s.matvec(l, transpose=True), A.T @ l) < 1e-11


def _sphere_plate_params():
    pr = case("sphere_plate")
    return pr


def test_gradient_matches_oracle_dense_transpose():
    pr = _sphere_plate_params()
    g_or = interaction_gradient(pr)
    s, ids = from_problem(pr, treecode=0, tol=1e-11)
    ds, dq = s.gradient(ids[1], pr.surfaces[1].nt, ids[0], len(pr.surfaces[0].q))
    assert rel_inf(dq, g_or[0]) < 1e-6
    assert rel_inf(ds, g_or[1]) < 1e-6


def test_gradient_with_stern_layer_and_cavity():
    """Nested interfaces on the adjoint path: the gradient of F_int with a
    Stern layer and a cavity (the molecule isolated with both) against the
    oracle's dense transpose, FP64 direct; and the treecode's against central
    differences of its own F_int (exactly quadratic in q and sigma)."""
    pr = case("nested_plate")
    g_or = interaction_gradient(pr)
    s, ids = from_problem(pr, treecode=0, tol=1e-11)
    ds, dq = s.gradient(ids[2], pr.surfaces[2].nt, ids[0], len(pr.surfaces[0].q))
    assert rel_inf(dq, g_or[0]) < 1e-6
    assert rel_inf(ds, g_or[2]) < 1e-6
    s.close()
    s, ids = from_problem(pr, treecode=1, ncrit=24, theta=0.5, taylor_p=6, tol=1e-11)
    ds, dq = s.gradient(ids[2], pr.surfaces[2].nt, ids[0], len(pr.surfaces[0].q))
    q0, s0 = pr.surfaces[0].q.copy(), pr.surfaces[2].bc.copy()

    def fint(q, sig):
        s.set_charges(ids[0], pr.surfaces[0].eps_in, pr.surfaces[0].q_pos, q)
        s.set_bc(ids[2], sig)
        return s.interaction_energy(len(pr.surfaces))[0]

    for j in (3, 200):
        h = 0.05
        sp, sm = s0.copy(), s0.copy()
        sp[j] += h
        sm[j] -= h
        fd = (fint(q0, sp) - fint(q0, sm)) / (2 * h)
        assert abs(fd - ds[j]) <= 2e-5 * np.max(np.abs(ds)), (j, fd, ds[j])
    for k in range(len(q0)):
        h = 0.5
        qp, qm = q0.copy(), q0.copy()
        qp[k] += h
        qm[k] -= h
        fd = (fint(qp, s0) - fint(qm, s0)) / (2 * h)
        assert abs(fd - dq[k]) <= 2e-5 * np.max(np.abs(dq)), (k, fd, dq[k])
    s.close()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_treecode_gradient_central_differences(prec):
    """F_int of the treecode system is exactly quadratic in (q, sigma):
    central differences with a large step reproduce the adjoint gradient."""
    pr = _sphere_plate_params()
    kw = dict(treecode=1, ncrit=24, theta=0.5, taylor_p=6, tol=1e-11, prec=prec)
    s, ids = from_problem(pr, **kw)
    nq, ns = len(pr.surfaces[0].q), pr.surfaces[1].nt
    ds, dq = s.gradient(ids[1], ns, ids[0], nq)

    def fint(q, sig):
        s.set_charges(ids[0], pr.surfaces[0].eps_in, pr.surfaces[0].q_pos, q)
        s.set_bc(ids[1], sig)
        return s.interaction_energy(2)[0]

    q0, s0 = pr.surfaces[0].q.copy(), pr.surfaces[1].bc.copy()
    tol = 2e-5 if prec == FP64 else 2e-3
    for j in np.random.default_rng(6).choice(ns, 4, replace=False):
        h = 0.05
        sp, sm = s0.copy(), s0.copy()
        sp[j] += h
        sm[j] -= h
        fd = (fint(q0, sp) - fint(q0, sm)) / (2 * h)
        assert abs(fd - ds[j]) <= tol * np.max(np.abs(ds)), (j, fd, ds[j])
    for k in range(nq):
        h = 0.5
        qp, qm = q0.copy(), q0.copy()
        qp[k] += h
        qm[k] -= h
        fd = (fint(qp, s0) - fint(qm, s0)) / (2 * h)
        assert abs(fd - dq[k]) <= tol * np.max(np.abs(dq)), (k, fd, dq[k])


def test_autograd_function():
    import torch
    from paper_1506_03745_amd.autograd import InteractionEnergy, PBProblem
    pr = _sphere_plate_params()
    s, ids = from_problem(pr, treecode=0, tol=1e-11)
    h = PBProblem(s, ids[0], pr.surfaces[0].eps_in, pr.surfaces[0].q_pos, ids[1], pr.surfaces[1].nt)
    q = torch.tensor(pr.surfaces[0].q, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(pr.surfaces[1].bc, dtype=torch.float64, requires_grad=True)
    f = InteractionEnergy.apply(q, sig, h, 2)
    (2.0 * f).backward()
    g_or = interaction_gradient(pr)
    assert rel_inf(q.grad.numpy() / 2.0, g_or[0]) < 1e-6
    assert rel_inf(sig.grad.numpy() / 2.0, g_or[1]) < 1e-6
