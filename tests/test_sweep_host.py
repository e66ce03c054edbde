"""Host logic of the orientation-sweep driver (paper_1506_03745_amd.sweep):
one JSON line per placement, written chunk by chunk, and a resumed sweep
solving only the placements its file does not hold yet.  A stand-in solver
(no GPU) returns a value computed from each placement's rotation and shift."""
import json

import numpy as np
import pytest

from paper_1506_03745_amd.sweep import orientation_sweep


class Stats:
    iters = 7
    rel_resid = 3e-7


class FakeSolver:
    def __init__(self):
        self.calls = []

    def solve_batch(self, mol_id, rot, shift):
        rot = np.asarray(rot).reshape(-1, 9)
        shift = np.asarray(shift).reshape(-1, 3)
        self.calls.append(len(rot))
        return rot.sum(axis=1) + 10.0 * shift[:, 2]

    def last_stats(self):
        return Stats()


def placements(n):
    rng = np.random.default_rng(11)
    return rng.standard_normal((n, 9)), rng.standard_normal((n, 3))


def test_one_line_per_placement_in_chunks(tmp_path):
    rot, shift = placements(10)
    path = tmp_path / "sweep.jsonl"
    s = FakeSolver()
    f = orientation_sweep(s, 0, rot, shift, str(path), chunk=4)
    assert s.calls == [4, 4, 2]
    np.testing.assert_array_equal(f, rot.sum(axis=1) + 10.0 * shift[:, 2])
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [r["index"] for r in lines] == list(range(10))
    assert [r["chunk"] for r in lines] == [0] * 4 + [1] * 4 + [2] * 2
    for r in lines:
        assert r["F_int_kcal"] == f[r["index"]]
        assert r["rotation"] == rot[r["index"]].tolist() and r["shift"] == shift[r["index"]].tolist()
        assert r["chunk_iters"] == 7 and r["chunk_rel_resid"] == 3e-7


def test_resume_skips_done_placements_and_cut_lines(tmp_path):
    rot, shift = placements(9)
    path = tmp_path / "sweep.jsonl"
    full = rot.sum(axis=1) + 10.0 * shift[:, 2]
    # a sweep stopped after placements 0, 1, 5, with a line cut short
    with open(path, "w") as fh:
        for i in (0, 1, 5):
            fh.write(json.dumps({"index": i, "F_int_kcal": float(full[i])}) + "\n")
        fh.write('{"index": 2, "F_int_ka')
    s = FakeSolver()
    f = orientation_sweep(s, 0, rot, shift, str(path), chunk=4)
    assert s.calls == [4, 2]          # 2, 3, 4, 6 then 7, 8
    np.testing.assert_array_equal(f, full)
    # a second resume has nothing left to do
    s2 = FakeSolver()
    np.testing.assert_array_equal(orientation_sweep(s2, 0, rot, shift, str(path)), full)
    assert s2.calls == []


def test_mismatched_inputs_raise(tmp_path):
    rot, shift = placements(3)
    with pytest.raises(ValueError):
        orientation_sweep(FakeSolver(), 0, rot, shift[:2], str(tmp_path / "a.jsonl"))
    with pytest.raises(ValueError):
        orientation_sweep(FakeSolver(), 0, rot, shift, str(tmp_path / "b.jsonl"), chunk=0)
