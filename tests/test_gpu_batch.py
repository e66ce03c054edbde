"""Batched rigid placements (pbt_solve_batch) against one-at-a-time solves
and the oracle.

Each placement's F_int from the block-diagonal batch must equal the F_int of
a separate context holding the moved molecule (same discretisation; FP64
direct form, GMRES tol 1e-10: agreement to 1e-7 of |F_solv| + |F_surf|), and
one placement is checked against the dense oracle.  The batch is also run
with the treecode in mixed precision against FP64 one-at-a-time solves.
"""
import copy

import numpy as np
import pytest

from oracle.bem import interaction_energy
from paper_1506_03745_amd import MIXED, from_problem
from workloads.meshes import box_plate, icosphere
from workloads.problems import CAVITY, CHARGED, MOLECULE, POTENTIAL, STERN, Problem, Surface, random_rotations

pytestmark = pytest.mark.gpu


def body_problem():
    v, t = icosphere(2, 3.0, (0.0, 0.0, 0.0))
    qpos = np.array([[0.4, -0.3, 0.2], [-0.5, 0.2, -0.1]])
    mol = Surface(MOLECULE, v, t, eps_in=2.0, q_pos=qpos, q=np.array([1.0, -0.5]))
    pv, pt = box_plate(-6, 6, -6, 6, -2, 0, 8, 8, 2)
    pl = Surface(CHARGED, pv, pt, bc=np.full(len(pt), -0.05))
    return Problem([mol, pl], 80.0, 0.125, {}, "batch_body")


def placed(pr, R, t):
    p = copy.deepcopy(pr)
    for k, m in enumerate(p.surfaces):
        if k == 0 or m.parent == 0:   # the molecule and its nested surfaces move
            m.verts = m.verts @ R.T + t
            if m.q_pos is not None:
                m.q_pos = m.q_pos @ R.T + t
    return p


def placements(nb):
    R = random_rotations(nb, 21)
    t = np.tile(np.array([0.0, 0.0, 4.5]), (nb, 1))
    t[:, 0] = np.linspace(-1.0, 1.0, nb)
    return R, t


def test_batch_matches_individual_and_oracle():
    pr = body_problem()
    nb = 5
    R, t = placements(nb)
    s, ids = from_problem(pr, treecode=0, tol=1e-10)
    f_batch = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    for b in range(nb):
        pb = placed(pr, R[b], t[b])
        sb, _ = from_problem(pb, treecode=0, tol=1e-10)
        f, res = sb.interaction_energy(2)
        scale = abs(res[0].F_solv) + abs(res[0].F_surf)
        assert abs(f_batch[b] - f) <= 1e-7 * scale, (b, f_batch[b], f)
        sb.close()
    f_or, e_all, _ = interaction_energy(placed(pr, R[2], t[2]))
    assert abs(f_batch[2] - f_or) <= 1e-6 * (abs(e_all.F_solv) + abs(e_all.F_surf))


def test_batch_mixed_treecode():
    pr = body_problem()
    nb = 8
    R, t = placements(nb)
    s, ids = from_problem(pr, treecode=1, ncrit=32, theta=0.4, taylor_p=8, prec=MIXED, tol=1e-8)
    f_batch = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    s64, ids64 = from_problem(pr, treecode=0, tol=1e-10)
    f_ref = s64.solve_batch(ids64[0], R.reshape(nb, 9), t)
    e = s64.solve()
    scale = abs(e.F_solv) + abs(e.F_surf)
    assert np.max(np.abs(f_batch - f_ref)) <= 2e-4 * scale
    assert len(set(np.round(f_ref, 8))) > 1   # placements differ


@pytest.mark.parametrize("kappa,k_far", [(0.125, 3), (0.0, 7), (0.125, 1)])
def test_batch_shared_surfaces_treecode(kappa, k_far, monkeypatch):
    """The plate is the same in every placement, so its P2P and M2P pairs
    with itself are evaluated once for 16 placements at a time.  With 18
    placements (a block of 16 and a block of 2), FP64 treecode: the batched
    F_int equals that of the same batch with those pairs in per-placement
    tasks (PBT_NO_SHARED) to the solver's tolerance, and a separate solve of
    a moved pair to the treecode's accuracy (its isolated energies come from
    the moved molecule's own tree).  Salt-free and Yukawa solvent; rules with
    and without the barycentre, whose self pair is skipped."""
    pr = body_problem()
    pr.kappa = kappa
    prm = dict(treecode=1, ncrit=24, theta=0.5, taylor_p=6, k_far=k_far, tol=1e-10)
    nb = 18
    R, t = placements(nb)
    s, ids = from_problem(pr, **prm)
    f_batch = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    monkeypatch.setenv("PBT_NO_SHARED", "1")
    f_plain = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    monkeypatch.delenv("PBT_NO_SHARED")
    e = s.solve()
    scale = abs(e.F_solv) + abs(e.F_surf)
    assert np.max(np.abs(f_batch - f_plain)) <= 1e-8 * scale
    assert np.any(f_batch != f_plain)   # the two paths did differ (summation order)
    for b in (0, 17):
        pb = placed(pr, R[b], t[b])
        sb, _ = from_problem(pb, **prm)
        f, res = sb.interaction_energy(2)
        assert abs(f_batch[b] - f) <= 1e-5 * scale, (b, f_batch[b], f)
        sb.close()


def test_batch_two_shared_surfaces(monkeypatch):
    """Two unmoved surfaces (the plate and a second, potential-carrying
    plate beside it): the pairs within each and between the two go to the
    shared-surface tasks (two box-offset rows); 18 placements, mixed
    precision, against the same batch in per-placement tasks."""
    pr = body_problem()
    pv, pt = box_plate(8, 14, -6, 6, -2, 0, 4, 8, 2)
    pr.surfaces.append(Surface(POTENTIAL, pv, pt, bc=np.full(len(pt), 0.02)))
    prm = dict(treecode=1, ncrit=24, theta=0.5, taylor_p=6, prec=MIXED, tol=1e-8)
    nb = 18
    R, t = placements(nb)
    s, ids = from_problem(pr, **prm)
    f_batch = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    monkeypatch.setenv("PBT_NO_SHARED", "1")
    f_plain = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    monkeypatch.delenv("PBT_NO_SHARED")
    e = s.solve()
    scale = abs(e.F_solv) + abs(e.F_surf)
    assert np.max(np.abs(f_batch - f_plain)) <= 1e-5 * scale
    assert np.any(f_batch != f_plain)   # the two paths did differ (summation order)
    assert len(set(np.round(f_batch, 8))) > 1


def nested_body_problem():
    """The batch body with a Stern layer (r = 3.6 A, permittivity 20) and an
    off-centre water cavity that move with the molecule."""
    pr = body_problem()
    v, t = icosphere(2, 3.6, (0.0, 0.0, 0.0))
    pr.surfaces.append(Surface(STERN, v, t, eps_in=20.0, parent=0))
    v, t = icosphere(1, 0.8, (1.2, 0.8, -0.6))
    pr.surfaces.append(Surface(CAVITY, v, t, eps_in=80.0, parent=0))
    return pr


def test_batch_with_stern_layer_and_cavity():
    """Placements of a molecule with its Stern surface and cavity: each
    batched F_int equals a separate solve of the moved assembly (FP64
    direct), and one placement the oracle's."""
    pr = nested_body_problem()
    nb = 3
    R, t = placements(nb)
    t[:, 2] = 5.2      # the Stern surface clears the plate
    s, ids = from_problem(pr, treecode=0, tol=1e-10)
    f_batch = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    for b in range(nb):
        pb = placed(pr, R[b], t[b])
        sb, _ = from_problem(pb, treecode=0, tol=1e-10)
        f, res = sb.interaction_energy(len(pb.surfaces))
        scale = abs(res[0].F_solv) + abs(res[0].F_surf)
        assert abs(f_batch[b] - f) <= 1e-7 * scale, (b, f_batch[b], f)
        sb.close()
    f_or, e_all, _ = interaction_energy(placed(pr, R[1], t[1]))
    assert abs(f_batch[1] - f_or) <= 1e-6 * (abs(e_all.F_solv) + abs(e_all.F_surf))


def test_orientation_sweep_file_matches_one_batch(tmp_path):
    """The sweep driver (chunks of 2, one JSON line per placement, then a
    resumed call with nothing left) against one pbt_solve_batch of all five
    placements: each placement is its own system solved to tol 1e-10, so the
    chunking changes F_int only at the solver's tolerance (1e-7 of
    |F_solv| + |F_surf| of one placement)."""
    import json

    from paper_1506_03745_amd.sweep import orientation_sweep
    pr = body_problem()
    nb = 5
    R, t = placements(nb)
    s, ids = from_problem(pr, treecode=0, tol=1e-10)
    f_all = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    path = tmp_path / "sweep.jsonl"
    f_sw = orientation_sweep(s, ids[0], R.reshape(nb, 9), t, str(path), chunk=2)
    s0, _ = from_problem(placed(pr, R[0], t[0]), treecode=0, tol=1e-10)
    _, res = s0.interaction_energy(2)
    s0.close()
    scale = abs(res[0].F_solv) + abs(res[0].F_surf)
    assert np.max(np.abs(f_sw - f_all)) <= 1e-7 * scale
    recs = [json.loads(x) for x in path.read_text().splitlines()]
    assert sorted(r["index"] for r in recs) == list(range(nb))
    assert all(r["chunk_rel_resid"] <= 1e-10 for r in recs)
    np.testing.assert_array_equal(orientation_sweep(s, ids[0], R.reshape(nb, 9), t, str(path)), f_sw)
    s.close()
