"""Set-up geometry formed on the host.

The host forms the panels' centroids, areas and Gauss points itself (for the
octree, the target groups, the near-candidate search and the energies)
instead of reading back the device's; both sides use the same sequence of
correctly rounded operations.  With PBT_CHECK_HOST_GEOMETRY set, the library
reads the device's values back and fails the set-up unless they agree bit for
bit: checked here for every far-field rule (the 1- and 7-point rules contain
the barycentre, which takes the collocation point's formula), on a system of
several surfaces and on a batched system of rotated placements.
"""
import numpy as np
import pytest

from paper_1506_03745_amd import from_problem
from workloads.problems import config_problem, random_rotations

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k_far", [1, 3, 4, 7])
def test_host_geometry_matches_device(k_far, monkeypatch):
    monkeypatch.setenv("PBT_CHECK_HOST_GEOMETRY", "1")
    s, _ = from_problem(config_problem("stern_plate"), treecode=1, k_far=k_far)
    s.prepare()


def test_host_geometry_matches_device_batched(monkeypatch):
    monkeypatch.setenv("PBT_CHECK_HOST_GEOMETRY", "1")
    pr = config_problem("orient_sweep_small")
    s, ids = from_problem(pr, treecode=1)
    nb = 3
    R = random_rotations(nb, 5)
    c = pr.surfaces[0].q_pos[0]
    t = c[None, :] - R @ c   # rotations about the molecule's centre
    f = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    assert np.all(np.isfinite(f))


def test_batched_near_rows_copied_match_searched(monkeypatch):
    """In a batch the plate's copies take the near rows of group 0's copy
    (shifted to their own panels) where nothing else comes near them; with
    PBT_CHECK_NEAR set the library searches and evaluates every row again
    and fails the set-up unless the copies agree bit for bit.  One placement
    brings the molecule within the near distance of the plate, so that some
    of its plate copy's rows are searched instead of copied."""
    monkeypatch.setenv("PBT_CHECK_NEAR", "1")
    pr = config_problem("orient_sweep_small")
    s, ids = from_problem(pr, treecode=1)
    nb = 3
    R = random_rotations(nb, 7)
    c = pr.surfaces[0].q_pos[0]
    t = c[None, :] - R @ c
    t[2, 2] -= 8.5   # the last placement's sphere ends 1.5 A above the plate
    f = s.solve_batch(ids[0], R.reshape(nb, 9), t)
    assert np.all(np.isfinite(f))
