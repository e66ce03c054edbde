"""Grid-convergence study with Richardson extrapolation (Section 5.1: the
two-sphere verification reports the observed order of convergence of the
interaction free energy over the three finest meshes; Section 5.2 uses the
same extrapolation on the protein-surface runs).

Each level refines the mesh once, multiplying the number of panels N by 4;
orders are with respect to N, as the paper states them (error ~ N^-p, p ~ 1
for flat panels with constant unknowns).  For three consecutive values f1,
f2, f3 (coarse to fine) the observed order is p = log((f1 - f2) / (f2 - f3))
/ log 4 and the extrapolated value f3 + (f3 - f2) / (4^p - 1).

    python -m paper_1506_03745_amd.convergence            # two-sphere, charge
"""
from __future__ import annotations

import argparse
import json
import math
import time

from .pbt import MIXED, from_problem


def observed_order(f1: float, f2: float, f3: float, ratio: float = 4.0) -> float:
    """Order p from three values on meshes whose panel counts grow by `ratio`."""
    return math.log(abs((f1 - f2) / (f2 - f3))) / math.log(ratio)


def richardson(f2: float, f3: float, p: float, ratio: float = 4.0) -> float:
    """Extrapolated value from the two finest values and the order p."""
    return f3 + (f3 - f2) / (ratio ** p - 1.0)


def study(make_problem, levels, n_surfaces: int, **params) -> dict:
    """F_int of make_problem(level) at each level (GPU solves through the
    library), with the observed order and the extrapolated value from the
    three finest levels."""
    rows = []
    for lv in levels:
        pr = make_problem(lv)
        s, _ = from_problem(pr, **params)
        t0 = time.perf_counter()
        f, parts = s.interaction_energy(n_surfaces)
        rows.append({"level": lv, "panels": sum(su.nt for su in pr.surfaces), "F_int": f,
                     "F_solv": parts[0].F_solv, "F_surf": parts[0].F_surf,
                     "seconds": time.perf_counter() - t0})
        s.close()
    out = {"levels": rows}
    if len(rows) >= 3:
        f1, f2, f3 = (r["F_int"] for r in rows[-3:])
        p = observed_order(f1, f2, f3)
        out["observed_order"] = p
        out["extrapolated_F_int"] = richardson(f2, f3, p)
    return out


def main():
    from workloads.problems import config_problem
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="twosphere_charge", choices=["twosphere_charge", "twosphere_potential"])
    ap.add_argument("--levels", default="2,3,4,5")
    a = ap.parse_args()
    levels = [int(v) for v in a.levels.split(",")]
    res = study(lambda lv: config_problem(a.case, level=lv), levels, 2, prec=MIXED, theta=0.5, taylor_p=6,
                ncrit=300, k_far=3, k_near=19, k_self_edge=9, tol=1e-8)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
