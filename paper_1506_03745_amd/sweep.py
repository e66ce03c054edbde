"""Orientation sweep over rigid placements of one molecule, written as it goes.

``orientation_sweep(solver, mol_id, rot, shift, path)`` solves the interaction
free energy (eq. interaction_energy) of every placement x -> R x + t of the
molecule `mol_id` (row-major 3x3 rotations `rot`, shifts `shift` in A) with
the library's batched solve (pbt_solve_batch), a chunk of placements at a
time, and appends one JSON object per placement to the text file `path` as
soon as its chunk is done:

    {"index": i, "rotation": [9 floats], "shift": [3 floats],
     "F_int_kcal": F, "chunk": c, "chunk_iters": n, "chunk_rel_resid": r}

(`chunk_iters` and `chunk_rel_resid` are the chunk's largest GMRES iteration
count and FP64 relative residual).  Each chunk's lines are flushed and synced
before the next chunk starts, so a sweep that is stopped loses at most the
chunk in flight: called again with the same path, it skips every index the
file already holds (lines that do not parse, such as a line cut short, are
ignored) and solves only the rest.  Returns F_int of every placement, in
index order.  All computation runs in the library.
"""
from __future__ import annotations

import json
import os

import numpy as np


def _done(path):
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            try:
                rec = json.loads(line)
                out[int(rec["index"])] = float(rec["F_int_kcal"])
            except (ValueError, KeyError, TypeError):
                continue
    return out


def orientation_sweep(solver, mol_id, rot, shift, path, chunk=16):
    rot = np.ascontiguousarray(np.asarray(rot, dtype=np.float64).reshape(-1, 9))
    shift = np.ascontiguousarray(np.asarray(shift, dtype=np.float64).reshape(-1, 3))
    if len(rot) != len(shift):
        raise ValueError(f"{len(rot)} rotations but {len(shift)} shifts")
    if chunk < 1:
        raise ValueError("chunk must be at least 1")
    have = _done(path)
    todo = [i for i in range(len(rot)) if i not in have]
    # a line cut short by a stopped sweep gets its newline, so that the
    # next record starts a line of its own
    if todo and os.path.exists(path) and os.path.getsize(path) > 0:
        with open(path, "rb") as fh:
            fh.seek(-1, os.SEEK_END)
            cut = fh.read(1) != b"\n"
        if cut:
            with open(path, "a") as fh:
                fh.write("\n")
    for c0 in range(0, len(todo), chunk):
        idx = todo[c0:c0 + chunk]
        f = solver.solve_batch(mol_id, rot[idx], shift[idx])
        st = solver.last_stats()
        with open(path, "a") as fh:
            for k, i in enumerate(idx):
                rec = {"index": i, "rotation": rot[i].tolist(), "shift": shift[i].tolist(),
                       "F_int_kcal": float(f[k]), "chunk": c0 // chunk, "chunk_iters": int(st.iters),
                       "chunk_rel_resid": float(st.rel_resid)}
                fh.write(json.dumps(rec) + "\n")
                have[i] = float(f[k])
            fh.flush()
            os.fsync(fh.fileno())
    return np.array([have[i] for i in range(len(rot))])
