"""Write the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py            # analytic values (seconds)
    python tests/golden/make_golden.py --dense    # + dense oracle solves of the
                                                  #   two-sphere workload (minutes)
    python tests/golden/make_golden.py --twin     # + dense oracle energies and
                                                  #   gradient of the 1/16-resolution
                                                  #   star/plate twin (minutes)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import analytic  # noqa: E402
from oracle.units import energy_to_kcal, sigma_to_reduced, volts_to_reduced  # noqa: E402


def analytic_values():
    q, d1, e1, d2, e2, k, R = 1.0, 4.0, 4.0, 4.0, 80.0, 0.125, 12.0
    out = {"source": "oracle.analytic (two-sphere series of Section 4, N = 40); "
                     "molecule r = 4 A, +1 e centre, eps 4/80, kappa 0.125, R = 12 A",
           "units": "kcal/mol"}
    iso_solv = energy_to_kcal(analytic.born_kirkwood(q, d1, e1, e2, k))
    for case, kw, iso in (
            ("charge", dict(sigma0=sigma_to_reduced(0.05)),
             analytic.charged_sphere_energy(sigma_to_reduced(0.05), d2, e2, k)),
            ("potential", dict(phi0=volts_to_reduced(0.05)),
             analytic.potential_sphere_energy(volts_to_reduced(0.05), d2, e2, k))):
        r = analytic.two_sphere(q, d1, e1, d2, e2, k, R, N=40, **kw)
        fs, fsu = energy_to_kcal(r["F_solv"]), energy_to_kcal(r["F_surf"])
        out[case] = dict(F_solv_asm=fs, F_surf_asm=fsu, F_solv_iso=iso_solv,
                         F_surf_iso=energy_to_kcal(iso),
                         F_int=fs + fsu - iso_solv - energy_to_kcal(iso))
    out["kirkwood_F_solv"] = iso_solv
    return out


def dense_values():
    from oracle.bem import interaction_energy
    from workloads.problems import config_problem
    out = {"source": "oracle.bem dense LU, k_far 3, k_near 19, 9 per edge", "units": "kcal/mol"}
    for name in ("kirkwood", "twosphere_charge", "twosphere_potential"):
        p = config_problem(name)
        if name == "kirkwood":
            from oracle.bem import solve_problem
            e, _, _ = solve_problem(p)
            out[name] = dict(F_solv=e.F_solv, F_coul=e.F_coul, F_surf=e.F_surf)
            continue
        fint, e_all, parts = interaction_energy(p)
        out[name] = dict(F_int=fint, F_solv_asm=e_all.F_solv, F_surf_asm=e_all.F_surf,
                         F_solv_iso=parts[0].F_solv, F_surf_iso=parts[1].F_surf)
        print(name, out[name], flush=True)
    return out


def twin_values():
    """Dense LU energies and the dense-transpose gradient of F_int for the
    1/16-resolution twin of the large star/plate workload (4096 + 5120
    panels, the same charges and plate densities law): the gradient at 64
    seeded plate panels and 32 seeded charges, and its largest magnitudes."""
    import numpy as np
    from oracle.adjoint import interaction_gradient
    from oracle.bem import interaction_energy
    from workloads.problems import config_problem
    p = config_problem("star_plate_twin")
    fint, e_all, parts = interaction_energy(p)
    out = {"source": "oracle.bem dense LU and oracle.adjoint dense transpose, k_far 3, k_near 19, 9 per edge",
           "units": "kcal/mol; gradients in kcal/mol per C/m^2 (sigma) and per e (q)",
           "F_int": fint, "F_solv_asm": e_all.F_solv, "F_surf_asm": e_all.F_surf, "F_coul_asm": e_all.F_coul,
           "F_total_iso": [q.F_total for q in parts]}
    print("twin energies", out, flush=True)
    dq, ds = interaction_gradient(p)
    mol, plate = p.surfaces
    js = np.sort(np.random.default_rng(7).choice(plate.nt, 64, replace=False))
    ks = np.sort(np.random.default_rng(8).choice(len(mol.q), 32, replace=False))
    out["grad_sigma_idx"] = js.tolist()
    out["grad_sigma"] = ds[js].tolist()
    out["grad_sigma_maxabs"] = float(np.abs(ds).max())
    out["grad_q_idx"] = ks.tolist()
    out["grad_q"] = dq[ks].tolist()
    out["grad_q_maxabs"] = float(np.abs(dq).max())
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "twosphere_analytic.json"), "w") as f:
        json.dump(analytic_values(), f, indent=1)
    if "--twin" in sys.argv:
        vals = twin_values()
        with open(os.path.join(HERE, "twin_oracle.json.tmp"), "w") as f:
            json.dump(vals, f, indent=1)
        os.replace(os.path.join(HERE, "twin_oracle.json.tmp"), os.path.join(HERE, "twin_oracle.json"))
    if "--dense" in sys.argv:
        with open(os.path.join(HERE, "dense_oracle_energies.json"), "w") as f:
            json.dump(dense_values(), f, indent=1)
