#!/usr/bin/env python
"""Benchmark: treecode BEM matvec throughput and GMRES time to 1e-6, FP32 vs FP64.

Workload: the two-sphere case (molecule sphere r = 4 A with +1 e at its
centre and a sphere with sigma = 0.05 C/m^2, 5120 flat triangles each, centres
12 A apart, eps 4/80, kappa 0.125 / A), treecode theta 0.5, Taylor order 6,
300 panels per leaf, 3 Gauss points per panel, near rule 19 points, self rule
9 points per edge.  Synthetic meshes; inputs resident on the GPU before the
timed region (the system is prepared once, outside it).

One step = one solve of the assembled system: right-hand side (one FP64
operator pass with the imposed charge density), GMRES with FP32 interactions
and FP64 Krylov vectors inside FP64 iterative refinement to a relative
residual of 1e-6, and the energies.  value = dense-equivalent target x
Gauss-point interactions per second over the step (pairs a dense product
needs, times the operator applications the step makes, over the step time).

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3          # published MI355X FP32 vector peak (packed FP32 FMA)
FP32_NONPACKED_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, one FP32 op per lane
FLOPS_FUSED_PAIR = 29    # Laplace + Yukawa, single + double layer (op list in the design doc)
FLOPS_YUKAWA_PAIR = 26
P2P_PROFILE = os.path.join(ROOT, "profiles", "k_p2p_twosphere_charge.json")
P2P_SOURCES = (os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "p2p.hip"),
               os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "near_field.h"))


PROFILED_WORKLOAD = "twosphere_charge"   # the workload of the committed counter summary


def profiled_traffic(workload, grid):
    """HBM bytes per P2P launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken, the
    counters were taken on another workload, or this run's P2P launch has
    another shape (grid work-items) than the profiled one."""
    import hashlib
    if workload != PROFILED_WORKLOAD:
        return None
    try:
        prof = json.load(open(P2P_PROFILE))
        sha = [hashlib.sha256(open(f, "rb").read()).hexdigest() for f in P2P_SOURCES]
    except (OSError, ValueError):
        return None
    same = prof.get("source_sha256") == sha[0] and prof.get("header_sha256") == sha[1]
    if not same:
        return None
    for shape in [prof] + prof.get("other_shapes", []):
        if shape.get("grid_size") == grid:
            return shape.get("traffic_bytes_per_launch")
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="twosphere_charge")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the mixed-precision steps (for profiler runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-fd", action="store_true",
                    help="star_plate_large: skip the central-difference check of the gradient")
    ap.add_argument("--autotune-cache", default=None,
                    help="text cache of tuned launch shapes (read if present, appended otherwise)")
    return ap.parse_args()


def cpu_baseline(problem, budget_s=15.0):
    """Oracle (dense FP64 CPU BEM) on a bounded sample of target panels of the
    same workload: every target against every panel (far, near and self
    rules) exactly as the oracle assembles its rows."""
    import numpy as np
    from oracle.bem import DenseBEM
    sysm = DenseBEM(problem)
    ns = sum(s.nt for s in problem.surfaces) * 3
    rng = np.random.default_rng(0)
    done_pairs, t_used, n = 0, 0.0, 16
    while t_used < budget_s:
        idx = rng.choice(problem.surfaces[0].nt, n, replace=False)
        t0 = time.perf_counter()
        sysm.row_block(0, idx)
        dt = time.perf_counter() - t0
        done_pairs += n * ns
        t_used += dt
        n = min(problem.surfaces[0].nt, max(16, int(n * 2)))
        if t_used + 2 * dt > budget_s:
            break
    return {"value": done_pairs / t_used / 1e9, "unit": "Ginteractions/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{done_pairs // ns} target panels of the molecule x all {ns} Gauss points "
                      f"(rows of the dense FP64 operator), {t_used:.1f} s"}


WORKLOADS = {
    "twosphere_charge": "two spheres r=4 A, 2x5120 panels, R=12 A, sigma 0.05 C/m^2, eps 4/80, kappa 0.125",
    "twosphere_potential": "two spheres r=4 A, 2x5120 panels, R=12 A, phi0 0.05 V, eps 4/80, kappa 0.125",
    "kirkwood": "sphere r=4 A, 1280 panels, +1 e at the centre, eps 4/80, kappa 0.125",
    "star_plate": "star molecule 32768 panels + 900 charges, 10 A above a 80x80x2 A plate of 20480 panels "
                  "(sigma -0.05 C/m^2), eps 4/80, kappa 0.125",
    "star_plate_stern": "star_plate with a Stern (ion-exclusion) surface 2 A outside the molecule, 32768 "
                        "panels, salt-free layer of permittivity 80",
    "orient_sweep": "64 rigid rotations of a 5120-panel sphere molecule (+1 e) 10 A above the 20480-panel "
                    "plate, solved together (one Krylov space each)",
    "star_plate_large": "star molecule 65536 panels + 3000 charges, 12 A above a 120x120x2 A plate of 81920 "
                        "panels; gradient of F_int w.r.t. the plate's sigma and the charges",
}
PRM = dict(theta=0.5, taylor_p=6, ncrit=300, k_far=3, k_near=19, k_self_edge=9, tol=1e-6)


def common_fields(a, ms_step):
    return {"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 interactions + f64 Krylov/refinement", "data": "synthetic"}


def bench_batch(a):
    """Orientation sweep: one step = pbt_solve_batch of 64 placements (the
    isolated energies included), FP32 interactions in FP64 refinement."""
    import numpy as np
    from paper_1506_03745_amd import MIXED, from_problem
    from workloads.problems import config_problem, random_rotations
    pr = config_problem("orient_sweep")
    s, ids = from_problem(pr, prec=MIXED, **PRM)
    s.prepare()
    R = random_rotations(64, 3)
    c = pr.surfaces[0].q_pos[0]
    T = c[None, :] - R @ c            # rotations about the molecule's centre
    for _ in range(max(a.warmup, 1)):
        s.solve_batch(ids[0], R.reshape(64, 9), T)
    t0 = time.perf_counter()
    stats, f = [], None
    for _ in range(a.steps):
        f = s.solve_batch(ids[0], R.reshape(64, 9), T)
        stats.append(s.last_stats())
    dt = (time.perf_counter() - t0) / a.steps
    pairs = sum(x.dense_pairs for x in stats) / len(stats)
    st = stats[-1]
    out = {"metric": "treecode BEM matvec Ginteractions/s + GMRES time to 1e-6 resid, FP32 vs FP64",
           "value": round(pairs / dt / 1e9, 3), "unit": "Ginteractions/s", **common_fields(a, 1e3 * dt),
           "config": {"workload": f"orient_sweep: {WORKLOADS['orient_sweep']}", "placements": 64,
                      "unknowns_per_placement": s.num_unknowns(), **{k: v for k, v in PRM.items()},
                      "precision": "mixed"},
           "roofline": None,
           "batch": {"ms_per_placement": round(1e3 * dt / 64, 3), "iters_max": st.iters,
                     "operator_applications": st.matvecs, "setup_s": round(st.t_setup_s, 4),
                     "F_int_kcal": {"min": float(f.min()), "max": float(f.max()), "mean": float(f.mean())}}}
    print(json.dumps(out), flush=True)


def bench_gradient(a):
    """Adjoint gradient at large size: one step = pbt_gradient (three forward
    and three transposed solves); then central differences of F_int on 20
    random plate panels and 5 charges (F_int is exactly quadratic in them)."""
    import numpy as np
    from paper_1506_03745_amd import MIXED, from_problem
    from workloads.problems import config_problem
    pr = config_problem("star_plate_large")
    mol, plate = pr.surfaces
    s, ids = from_problem(pr, prec=MIXED, **PRM)
    s.prepare()
    if not a.no_autotune:
        s.autotune(a.autotune_cache)
    s.gradient(ids[1], plate.nt, ids[0], len(mol.q))
    t0 = time.perf_counter()
    stats = []
    for _ in range(a.steps):
        ds, dq = s.gradient(ids[1], plate.nt, ids[0], len(mol.q))
        stats.append(s.last_stats())
    dt = (time.perf_counter() - t0) / a.steps
    pairs = sum(x.dense_pairs for x in stats) / len(stats)
    out = {"metric": "treecode BEM matvec Ginteractions/s + GMRES time to 1e-6 resid, FP32 vs FP64",
           "value": round(pairs / dt / 1e9, 3), "unit": "Ginteractions/s", **common_fields(a, 1e3 * dt),
           "config": {"workload": f"star_plate_large: {WORKLOADS['star_plate_large']}",
                      "unknowns": s.num_unknowns(), **PRM, "precision": "mixed"},
           "roofline": None,
           "gradient": {"ms": round(1e3 * dt, 2), "operator_applications": stats[-1].matvecs,
                        "max_abs_dF_dsigma": float(np.abs(ds).max()), "max_abs_dF_dq": float(np.abs(dq).max())}}
    if not a.no_fd:
        tight = dict(PRM, tol=1e-10)
        f, fids = from_problem(pr, prec=MIXED, **tight)
        gs, gq = f.gradient(fids[1], plate.nt, fids[0], len(mol.q))

        def fint(q, sig):
            f.set_charges(fids[0], mol.eps_in, mol.q_pos, q)
            f.set_bc(fids[1], sig)
            return f.interaction_energy(2)[0]

        rng = np.random.default_rng(6)
        q0, s0 = mol.q.copy(), plate.bc.copy()
        err_s, err_q = 0.0, 0.0
        for j in rng.choice(plate.nt, 20, replace=False):
            sp, sm = s0.copy(), s0.copy()
            sp[j] += 0.05
            sm[j] -= 0.05
            fd = (fint(q0, sp) - fint(q0, sm)) / 0.1
            err_s = max(err_s, abs(fd - gs[j]))
            print(f"fd panel {j}: {fd:.6e} adjoint {gs[j]:.6e}", file=sys.stderr, flush=True)
        for k in rng.choice(len(q0), 5, replace=False):
            qp, qm = q0.copy(), q0.copy()
            qp[k] += 0.5
            qm[k] -= 0.5
            fd = (fint(qp, s0) - fint(qm, s0)) / 1.0
            err_q = max(err_q, abs(fd - gq[k]))
            print(f"fd charge {k}: {fd:.6e} adjoint {gq[k]:.6e}", file=sys.stderr, flush=True)
        out["gradient"]["central_differences"] = {
            "panels": 20, "charges": 5, "tol": 1e-10, "seed": 6,
            "max_err_rel_dF_dsigma": err_s / float(np.abs(gs).max()),
            "max_err_rel_dF_dq": err_q / float(np.abs(gq).max()),
            "mixed_vs_tight_rel_dF_dsigma": float(np.abs(ds - gs).max() / np.abs(gs).max()),
            "mixed_vs_tight_rel_dF_dq": float(np.abs(dq - gq).max() / np.abs(gq).max())}
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              f"(the multi-GPU design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if a.workload == "orient_sweep":
        return bench_batch(a)
    if a.workload == "star_plate_large":
        return bench_gradient(a)
    import numpy as np
    import torch

    from paper_1506_03745_amd import FP64, MIXED, from_problem
    from workloads.problems import config_problem

    if a.copy_calib:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    problem = config_problem(a.workload)
    prm = PRM

    # ---- mixed precision (the benchmarked path) -----------------------------
    s32, _ = from_problem(problem, prec=MIXED, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s32.prepare()
    setup_wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    if not a.no_autotune:
        s32.autotune(a.autotune_cache)
    autotune_s = time.perf_counter() - t0
    s32.solve()
    for _ in range(a.warmup):
        s32.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [s32.solve() for _ in range(a.steps)]
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_step = 1e3 * t_steps / a.steps
    r = rs[-1]
    applications = sum(x.matvecs for x in rs) / len(rs)
    value = r.dense_pairs * applications / (ms_step / 1e3) / 1e9

    # ---- operator timing on the context's stream (HIP events) ----------------
    # First with the tuned schedule (the solve's), then the FP32 operator once
    # more on the serial schedule, where P2P is a launch of its own: the
    # roofline is that kernel's.
    n = s32.num_unknowns()
    x = torch.tensor(np.random.default_rng(0).standard_normal(n), device="cuda:0")
    y = torch.empty_like(x)
    keys = ("total_ms", "p2p_ms", "m2p_ms", "moments_ms", "rest_ms")
    nrep = 20

    def op_timing(prec):
        store = dict.fromkeys(keys, 0.0)
        s32.matvec_dev(x, y, prec=prec)
        s32.last_matvec_timing()
        for _ in range(nrep):
            s32.matvec_dev(x, y, prec=prec)
            t = s32.last_matvec_timing()
            for k in store:
                store[k] += t[k] / nrep
        return store

    schedule = s32.schedule()
    shape = s32.launch_shape()
    acc, acc64 = op_timing(MIXED), op_timing(FP64)
    s32.set_schedule(0)
    acc_serial = op_timing(MIXED)
    s32.set_schedule(schedule)
    p2p_flops = FLOPS_FUSED_PAIR * r.p2p_fused_pairs + FLOPS_YUKAWA_PAIR * (r.p2p_pairs - r.p2p_fused_pairs)
    achieved = p2p_flops / (acc_serial["p2p_ms"] / 1e3) / 1e12
    out = {
        "metric": "treecode BEM matvec Ginteractions/s + GMRES time to 1e-6 resid, FP32 vs FP64",
        "value": round(value, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 interactions + f64 Krylov/refinement",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS.get(a.workload, a.workload)}",
                   "panels": sum(s.nt for s in problem.surfaces), "unknowns": n,
                   "theta": 0.5, "taylor_p": 6, "ncrit": 300, "k_far": 3, "k_near": 19,
                   "self_per_edge": 9, "tol": 1e-6, "precision": "mixed"},
        "roofline": {"bound": "alu", "kernel": "k_p2p<float>", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": profiled_traffic(a.workload, shape[2]), "p2p_grid": shape[2],
                     "frac_of_nonpacked_fp32": round(achieved / FP32_NONPACKED_TFLOPS, 4),
                     "flops_per_launch": int(p2p_flops), "avg_launch_ms": round(acc_serial["p2p_ms"], 5)},
        "gmres": {"iters": r.iters, "outer": r.outer, "rel_resid": r.rel_resid,
                  "applications_per_step": applications, "setup_s": round(setup_wall, 4),
                  "autotune_s": round(autotune_s, 3)},
        "far_field_schedule": {0: "serial", 1: "two streams", 2: "joint M2P + P2P launch",
                               3: "moments inside the P2P launch",
                               4: "moments with 7/8 of P2P, then M2P with 1/8 of P2P",
                               5: "moments with 3/4 of P2P, then M2P with 1/4 of P2P",
                               6: "moments with 1/2 of P2P, then M2P with 1/2 of P2P"}[schedule],
        "matvec_ms": {"fp32": {k: round(v, 4) for k, v in acc.items()},
                      "fp64": {k: round(v, 4) for k, v in acc64.items()},
                      "fp32_serial_schedule": {k: round(v, 4) for k, v in acc_serial.items()}},
        "matvec_gint_s": {"fp32": round(r.dense_pairs / acc["total_ms"] / 1e6, 2),
                          "fp64": round(r.dense_pairs / acc64["total_ms"] / 1e6, 2)},
        "p2p_gpairs_s": round(r.p2p_pairs / acc_serial["p2p_ms"] / 1e6, 2),
        "pairs": {"dense": r.dense_pairs, "p2p": r.p2p_pairs, "p2p_fused": r.p2p_fused_pairs,
                  "m2p": r.m2p_pairs},
        "energies_kcal": {"F_solv": r.F_solv, "F_surf": r.F_surf},
    }
    if not a.profile_only:
        # FP64 treecode at the same (theta, P) and the plain FP64 direct form
        s64, _ = from_problem(problem, prec=FP64, **prm)
        s64.solve()
        t0 = time.perf_counter()
        r64 = s64.solve()
        r64b = s64.solve()
        t64 = (time.perf_counter() - t0) / 2
        sd, _ = from_problem(problem, prec=FP64, treecode=0, **{k: v for k, v in prm.items()})
        sd.solve()
        t0 = time.perf_counter()
        rd = sd.solve()
        td = time.perf_counter() - t0
        out["fp64"] = {"treecode_ms_per_solve": round(1e3 * t64, 3), "iters": r64b.iters,
                       "direct_ms_per_solve": round(1e3 * td, 3), "direct_iters": rd.iters,
                       "speedup_mixed_vs_fp64_treecode": round(t64 / (ms_step / 1e3), 3),
                       "speedup_mixed_vs_fp64_direct": round(td / (ms_step / 1e3), 3),
                       "F_solv_fp64_treecode": r64.F_solv, "F_solv_fp64_direct": rd.F_solv,
                       "rel_diff_F_solv_mixed_vs_fp64": abs(r.F_solv - r64.F_solv) / abs(r64.F_solv)}
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
