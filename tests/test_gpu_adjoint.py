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


def _at(pr, q=None, sig=None):
    """A copy of the problem with other charges / densities."""
    pr2 = copy.deepcopy(pr)
    if q is not None:
        pr2.surfaces[0].q = np.asarray(q, dtype=np.float64)
    if sig is not None:
        pr2.surfaces[1].bc = np.asarray(sig, dtype=np.float64)
    return pr2


def test_autograd_on_device_two_applications_in_one_graph():
    """Device tensors through the _dev entry points; two applications at
    different charges in one graph each get the gradient at their own point
    (the library holds the second point when backward runs)."""
    import torch
    from paper_1506_03745_amd.autograd import InteractionEnergy, PBProblem
    pr = _sphere_plate_params()
    s, ids = from_problem(pr, treecode=0, tol=1e-11)
    h = PBProblem(s, ids[0], pr.surfaces[0].eps_in, pr.surfaces[0].q_pos, ids[1], pr.surfaces[1].nt)
    dev = torch.device("cuda:0")
    q1 = torch.tensor(pr.surfaces[0].q, dtype=torch.float64, device=dev, requires_grad=True)
    q2v = pr.surfaces[0].q * np.array([-0.5, 2.0])
    q2 = torch.tensor(q2v, dtype=torch.float64, device=dev, requires_grad=True)
    sig = torch.tensor(pr.surfaces[1].bc, dtype=torch.float64, device=dev, requires_grad=True)
    f = InteractionEnergy.apply(q1, sig, h, 2) + 3.0 * InteractionEnergy.apply(q2, sig, h, 2)
    f.backward()
    g1 = interaction_gradient(pr)
    g2 = interaction_gradient(_at(pr, q=q2v))
    assert q1.grad.device.type == "cuda" and sig.grad.device.type == "cuda"
    assert rel_inf(q1.grad.cpu().numpy(), g1[0]) < 1e-6
    assert rel_inf(q2.grad.cpu().numpy() / 3.0, g2[0]) < 1e-6
    assert rel_inf(sig.grad.cpu().numpy(), g1[1] + 3.0 * g2[1]) < 1e-6


def test_device_entry_points_match_host_ones():
    """pbt_set_charges_dev / pbt_set_bc_dev / pbt_get_solution_dev /
    pbt_gradient_dev against the host entry points and the oracle."""
    import torch
    from paper_1506_03745_amd import PbtError
    pr = _sphere_plate_params()
    mol, plate = pr.surfaces
    dev = torch.device("cuda:0")
    s, ids = from_problem(pr, treecode=0, tol=1e-11)
    q2 = mol.q * np.array([1.5, -1.0])
    sig2 = plate.bc * 0.7
    s.set_charges_dev(ids[0], mol.eps_in, torch.tensor(q2, device=dev))
    s.set_bc_dev(ids[1], torch.tensor(sig2, device=dev))
    r = s.solve()
    phi = torch.empty(mol.nt, dtype=torch.float64, device=dev)
    dphi = torch.empty(mol.nt, dtype=torch.float64, device=dev)
    s.get_solution_dev(ids[0], phi, dphi)
    ph, dh = s.get_solution(ids[0], mol.nt)
    assert np.array_equal(phi.cpu().numpy(), ph) and np.array_equal(dphi.cpu().numpy(), dh)
    ds = torch.empty(plate.nt, dtype=torch.float64, device=dev)
    dq = torch.empty(len(q2), dtype=torch.float64, device=dev)
    s.gradient_dev(ids[1], ds, ids[0], dq)
    g = interaction_gradient(_at(pr, q=q2, sig=sig2))
    assert rel_inf(dq.cpu().numpy(), g[0]) < 1e-6
    assert rel_inf(ds.cpu().numpy(), g[1]) < 1e-6
    # new positions through xyz_dev, and the energies against the oracle
    from oracle.bem import solve_problem
    e, _, _ = solve_problem(_at(pr, q=q2, sig=sig2))
    assert abs(r.F_solv - e.F_solv) <= 1e-8 * abs(e.F_solv)
    xyz = mol.q_pos + np.array([0.1, -0.1, 0.05])
    s.set_charges_dev(ids[0], mol.eps_in, torch.tensor(q2, device=dev), torch.tensor(xyz, device=dev))
    r2 = s.solve()
    pr3 = _at(pr, q=q2, sig=sig2)
    pr3.surfaces[0].q_pos = xyz
    e3, _, _ = solve_problem(pr3)
    assert abs(r2.F_solv - e3.F_solv) <= 1e-8 * abs(e3.F_solv)
    # host memory is not a device pointer
    with pytest.raises(PbtError, match="INVALID"):
        import ctypes
        from paper_1506_03745_amd.pbt import lib
        buf = np.zeros(plate.nt)
        st = lib().pbt_set_bc_dev(s._h, ids[1], buf.ctypes.data_as(ctypes.c_void_p), None)
        s._check(st)
