#!/usr/bin/env python
"""Benchmark: treecode BEM matvec throughput and GMRES time to 1e-6, FP32 vs FP64.

Default workload: the large star/plate system (a star-shaped molecule of
65536 flat triangles with 3000 interior point charges, 12 A above a
120 x 120 x 2 A plate of 81920 triangles with per-panel sigma =
0.03 (1 + 0.1 u) C/m^2; 212992 unknowns), eps 4/80, kappa 0.125 / A, treecode
theta 0.5, Taylor order 6, 300 panels per leaf, 3 Gauss points per panel,
near rule 19 points, self rule 9 points per edge.  Synthetic meshes; the
system is prepared (geometry, near corrections, tree, work lists, launch
shapes) before the timed region, so every input is resident in HBM.

One step = one solve of the assembled system: the right-hand side (an FP64
pass over the plate's known densities plus the Coulomb sums), GMRES with
FP32 interactions and FP64 Krylov vectors inside FP64 iterative refinement
to a relative residual of 1e-6 (the FP64 residual is checked at exit), and
the energies.  value = dense-equivalent target x Gauss-point interactions
per second over the step (targets x sources of every operator application
the step makes; the right-hand side's pass counts only the plate's sources).

Roofline: the launch that holds the P2P tasks (whichever far-field schedule
the autotuner chose) is timed with HIP events on its own stream over every
product of the timed steps.  Its algorithmic work uses the flop convention
FMA = 2, any other operation = 1, transcendental = 1: a pair whose target
and source lie on one molecule (single and double layer of both the Laplace
and the Yukawa kernel) is 34 flops (difference 3, r^2 5, 1/r^3 2, r 1,
n.(x-y) 5, -kappa r log2(e) 2, dG_L 1, G_Y 1, dG_Y 4, four accumulating FMAs
8, rsqrt 1, exp 1), a Yukawa-only pair 30.  An M2P (target, box) pair is
counted from the Taylor recurrences as written (m2p_pair_flops below): 1,344
flops at P = 6 for a Yukawa-only pair and 1,975 when the Laplace expansion of
a molecule's interior row is formed too.  The line's roofline is that of
the kernel that takes the most time in the timed solve (P2P or M2P); both
are reported.  Peaks: FP32 157.3 TFLOP/s (the published MI355X vector
figure, which counts packed FP32), FP64 78.6.

Other modes: --workload twosphere_charge | star_plate | star_plate_stern |
... (a solve of that workload), orient_sweep (pbt_solve_batch of 64 rigid
placements), gradient (pbt_gradient of the large workload with a central
difference check).

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "treecode BEM matvec Ginteractions/s + GMRES time to 1e-6 resid, FP32 vs FP64"
FP32_PEAK_TFLOPS = 157.3          # published MI355X FP32 vector peak (packed FP32 FMA)
FP64_PEAK_TFLOPS = 78.6           # published MI355X FP64 vector peak
FLOPS_FUSED_PAIR = 34
FLOPS_YUKAWA_PAIR = 30
PROFILES = os.path.join(ROOT, "profiles")
P2P_SOURCES = (os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "p2p.hip"),
               os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "near_field.h"),
               os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "taylor.hip"))

WORKLOADS = {
    "star_plate_large": "star molecule 65536 panels + 3000 charges, 12 A above a 120x120x2 A plate of 81920 "
                        "panels, sigma 0.03(1 + 0.1u) C/m^2, eps 4/80, kappa 0.125",
    "twosphere_charge": "two spheres r=4 A, 2x5120 panels, R=12 A, sigma 0.05 C/m^2, eps 4/80, kappa 0.125",
    "twosphere_potential": "two spheres r=4 A, 2x5120 panels, R=12 A, phi0 0.05 V, eps 4/80, kappa 0.125",
    "kirkwood": "sphere r=4 A, 1280 panels, +1 e at the centre, eps 4/80, kappa 0.125",
    "star_plate": "star molecule 32768 panels + 900 charges, 10 A above a 80x80x2 A plate of 20480 panels "
                  "(sigma -0.05 C/m^2), eps 4/80, kappa 0.125",
    "star_plate_stern": "star_plate with a Stern (ion-exclusion) surface 2 A outside the molecule, 32768 "
                        "panels, salt-free layer of permittivity 80",
    "orient_sweep": "64 rigid rotations of a 5120-panel sphere molecule (+1 e) 10 A above the 20480-panel "
                    "plate, solved together (one Krylov space each)",
    "gradient": "star_plate_large; gradient of F_int w.r.t. the plate's sigma and the charges",
}
# the stored oracle values that check each workload's energies (a twin at
# lower resolution where the oracle cannot solve the workload itself)
ORACLE_CHECK = {"star_plate_large": ("star_plate_twin", "twin_oracle.json"),
                "twosphere_charge": ("twosphere_charge", "dense_oracle_energies.json"),
                "twosphere_potential": ("twosphere_potential", "dense_oracle_energies.json")}
PRM = dict(theta=0.5, taylor_p=6, ncrit=300, k_far=3, k_near=19, k_self_edge=9, tol=1e-6)
SCHEDULES = {0: "serial", 1: "two streams", 2: "joint M2P + P2P launch", 3: "moments inside the P2P launch",
             4: "moments with 7/8 of P2P, then M2P with 1/8 of P2P",
             5: "moments with 3/4 of P2P, then M2P with 1/4 of P2P",
             6: "moments with 1/2 of P2P, then M2P with 1/2 of P2P"}


def m2p_kernel_name(schedule, prec="float", P=6):
    if schedule == 2:
        return f"k_m2p_p2p<{prec}, {P}, false, false>"
    return f"k_m2p<{prec}, {P}, false>"


def p2p_kernel_name(schedule, prec="float", P=6):
    """The kernel (as the profiler names it) that holds the P2P tasks."""
    if schedule in (0, 1):
        return f"k_p2p<{prec}, false>"
    if schedule == 2:
        return f"k_m2p_p2p<{prec}, {P}, false, false>"
    return f"k_p2p_mom<{prec}, {P}, false>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="star_plate_large")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work per CPU-baseline leg (one core, then all cores)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the mixed-precision steps (for profiler runs)")
    ap.add_argument("--no-direct", action="store_true", help="skip the plain FP64 direct solve")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-fd", action="store_true", help="gradient: skip the central-difference check")
    ap.add_argument("--autotune-cache", default=None,
                    help="text cache of tuned launch shapes (read if present, appended otherwise)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="no GPU work: reduce two rocprofv3 --pmc counter_collection CSVs (FETCH_SIZE, "
                         "WRITE_SIZE of runs with --copy-calib) to HBM bytes per launch of each kernel "
                         "and write them as JSON")
    return ap.parse_args()


# ---- CPU baseline: the oracle's dense FP64 rows on the host cores ------------------
_ORACLE = None


def _oracle_rows(args):
    """Worker: oracle rows (a target panel's interior and solvent rows against
    every Gauss point) for `budget` seconds.  Returns (target panels, seconds)."""
    import numpy as np
    seed, budget = args
    sysm = _ORACLE
    rng = np.random.default_rng(seed)
    nt = sysm.surfs[0].nt
    done, t_used, n = 0, 0.0, 8
    while True:
        idx = rng.choice(nt, n, replace=False)
        t0 = time.perf_counter()
        sysm.row_block(0, idx)
        dt = time.perf_counter() - t0
        done += n
        t_used += dt
        if t_used + dt > budget:
            return done, t_used


def cpu_baseline(problem, budget_s):
    """The oracle (dense FP64 CPU BEM, unchanged) on a bounded sample of the
    same workload: rows of seeded random molecule panels against every
    Gauss point of every surface (far, near and self rules), first on one
    core, then in one process per core (fork, before the GPU is touched)."""
    import multiprocessing as mp
    from oracle.bem import DenseBEM
    global _ORACLE
    _ORACLE = DenseBEM(problem)
    ns = sum(s.nt for s in problem.surfaces) * 3
    rows1, t1 = _oracle_rows((0, budget_s))
    one = rows1 * ns / t1 / 1e9
    ncores = min(16, len(os.sched_getaffinity(0)))   # the host share of one GPU is at most 16 cores
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(ncores) as pool:
        res = pool.map(_oracle_rows, [(100 + k, budget_s) for k in range(ncores)])
    wall = time.perf_counter() - t0
    rows_all = sum(r for r, _ in res)
    return {"value": rows_all * ns / wall / 1e9, "unit": "Ginteractions/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"dense FP64 operator rows (interior + solvent row) of seeded random molecule panels "
                      f"against all {ns} Gauss points: {rows_all} target panels on {ncores} processes in "
                      f"{wall:.1f} s wall; one core: {rows1} target panels in {t1:.1f} s",
            "single_core_value": one, "nproc": os.cpu_count(),
            "host_cpus_available": len(os.sched_getaffinity(0))}


# ---- helpers --------------------------------------------------------------------------
def common_fields(a, ms_step, dtype="f32 interactions + f64 Krylov/refinement"):
    return {"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic"}


def profiled_traffic(workload, kernel, grid):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (profiles/counters_<workload>.json), or None
    when there is none, the interaction kernels' sources changed since the
    counters were taken, or this run's launch has another shape (grid
    work-items) than the profiled one."""
    path = os.path.join(PROFILES, f"counters_{workload}.json")
    try:
        prof = json.load(open(path))
        sha = [hashlib.sha256(open(f, "rb").read()).hexdigest() for f in P2P_SOURCES]
    except (OSError, ValueError):
        return None
    if prof.get("sources_sha256") != sha or grid is None:
        return None
    for k in prof.get("kernels", []):
        if k.get("kernel") == kernel and k.get("grid_size") == grid:
            return k.get("traffic_bytes_per_launch")
    return None


def p2p_flops(r):
    return FLOPS_FUSED_PAIR * r.p2p_fused_pairs + FLOPS_YUKAWA_PAIR * (r.p2p_pairs - r.p2p_fused_pairs)


def m2p_pair_flops(P, laplace_too):
    """Flops of one M2P (target, box) pair, the Taylor coefficients of
    e^(-kappa rho)/rho (coefficients a and the auxiliary b of e^(-kappa rho))
    up to degree P by their recurrences and their dot with the box's moments;
    with laplace_too also those of 1/rho and a second dot.  Per coefficient
    k of degree n with f nonzero and s >= 2 entries: the first-neighbour sums
    2f - 1 each, the second-neighbour sums s - 1 each, the combination, the
    dot (FMA 2); per degree the scaled vectors; once the difference, r^2,
    rsqrt and exp."""
    f = 3 + 5 + 1 + 1 + 1 + 2 + 1 + 1 + 1      # R, R^2, rsqrt, 1/R^2, kappa R^2, -kappa r, exp, a_0, dot
    lap = 1                                    # dot of a_0
    for n in range(1, P + 1):
        f += 10                                # c1, c2, c3, e4, u (3), v (3)
        lap += 5                               # c1, c2, u (3)
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                k = (a, b, n - a - b)
                nf = sum(1 for q in k if q >= 1)
                ns = sum(1 for q in k if q >= 2)
                f += 2 * (2 * nf - 1) + (2 * (ns - 1) + 4 if ns else 0) + 1 + 2
                if n < P:
                    f += 1 + (2 if ns else 0)
                lap += (2 * nf - 1) + ((ns - 1) + 2 if ns else 0) + 2
    return f + (lap if laplace_too else 0)


def m2p_flops(r, P=6):
    return (m2p_pair_flops(P, True) * r.m2p_fused_pairs
            + m2p_pair_flops(P, False) * (r.m2p_pairs - r.m2p_fused_pairs))


def timed_solves(s, a, sync):
    """Warm-up, then a.steps timed solves with per-kernel profiling."""
    for _ in range(a.warmup):
        s.solve()
    sync()
    s.profile(True)
    t0 = time.perf_counter()
    rs, pairs = [], 0
    for _ in range(a.steps):
        rs.append(s.solve())
        pairs += s.last_stats().dense_pairs
    sync()
    dt = time.perf_counter() - t0
    kt = s.kernel_times()
    s.profile(False)
    return rs, pairs, dt, kt


def oracle_check(workload, prec):
    """Energies of the workload's oracle-checked twin (or itself) at the
    benchmark parameters, against the stored dense oracle values."""
    from paper_1506_03745_amd import from_problem
    from workloads.problems import config_problem
    if workload not in ORACLE_CHECK:
        return None
    name, fname = ORACLE_CHECK[workload]
    path = os.path.join(ROOT, "tests", "golden", fname)
    if not os.path.exists(path):
        return None
    try:
        gold = json.load(open(path))
    except (OSError, ValueError):
        return None
    gold = gold.get(name, gold)
    pr = config_problem(name)
    s, _ = from_problem(pr, prec=prec, **PRM)
    f, parts = s.interaction_energy(len(pr.surfaces))
    asm = parts[0]
    scale = abs(gold["F_solv_asm"]) + abs(gold["F_surf_asm"])
    out = {"workload": name, "F_solv_rel": abs(asm.F_solv - gold["F_solv_asm"]) / abs(gold["F_solv_asm"]),
           "F_surf_rel": abs(asm.F_surf - gold["F_surf_asm"]) / abs(gold["F_surf_asm"]),
           "F_int_abs_kcal": abs(f - gold["F_int"]), "F_int_rel_to_asm": abs(f - gold["F_int"]) / scale,
           "F_int_kcal": f, "F_int_oracle_kcal": gold["F_int"]}
    if "F_coul_asm" in gold and gold["F_coul_asm"] != 0:
        out["F_coul_rel"] = abs(asm.F_coul - gold["F_coul_asm"]) / abs(gold["F_coul_asm"])
    s.close()
    return {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in out.items()}


# ---- modes ------------------------------------------------------------------------------
def bench_solve(a, cpu):
    import numpy as np
    import torch

    from paper_1506_03745_amd import FP64, MIXED, from_problem
    from workloads.problems import config_problem

    sync = torch.cuda.synchronize
    if a.copy_calib:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        del src, dst
    problem = config_problem(a.workload)

    # ---- mixed precision (the benchmarked path) -----------------------------
    s32, _ = from_problem(problem, prec=MIXED, **PRM)
    sync()
    t0 = time.perf_counter()
    s32.prepare()
    setup_wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    if not a.no_autotune:
        s32.autotune(a.autotune_cache)
    autotune_s = time.perf_counter() - t0
    s32.solve()
    print(f"[bench] {a.workload}: prepared in {setup_wall:.2f} s, autotuned in {autotune_s:.2f} s",
          file=sys.stderr, flush=True)
    rs, pairs, t_steps, kt = timed_solves(s32, a, sync)
    ms_step = 1e3 * t_steps / a.steps
    r = rs[-1]
    value = pairs / t_steps / 1e9
    schedule = s32.schedule()
    shape = s32.launch_shape()
    print(f"[bench] timed {a.steps} solves: {ms_step:.2f} ms each", file=sys.stderr, flush=True)

    def per_kernel(kt, prec):
        out = {}
        for kind in ("p2p", "m2p", "moments", "combine"):
            ms, n = kt[(prec, kind)]
            if n:
                out[kind] = {"launches_per_step": n / a.steps, "avg_ms": round(ms / n, 5),
                             "ms_per_step": round(ms / a.steps, 4)}
        return out

    k32 = per_kernel(kt, "fp32")

    def roofline(kind, prec, flops, peak, sched, shape_grid=None):
        ms, n = kt_sel[prec][(prec, kind)]
        avg = ms / max(n, 1)
        ach = flops / (avg / 1e3) / 1e12
        name = (p2p_kernel_name if kind == "p2p" else m2p_kernel_name)(sched, "float" if prec == "fp32" else "double")
        return {"bound": "alu", "kernel": name, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": profiled_traffic(a.workload, name, shape_grid)
                if prec == "fp32" else None,
                "flops_per_launch": int(flops), "avg_launch_ms": round(avg, 5), "launches": n}

    kt_sel = {"fp32": kt}
    fl_p2p, fl_m2p = p2p_flops(r), m2p_flops(r)
    rf_p2p = roofline("p2p", "fp32", fl_p2p, FP32_PEAK_TFLOPS, schedule, shape[2])
    rf_m2p = roofline("m2p", "fp32", fl_m2p, FP32_PEAK_TFLOPS, schedule, shape[3])
    for rf, fl in ((rf_p2p, "34 per Laplace+Yukawa pair, 30 per Yukawa-only pair"),
                   (rf_m2p, f"{m2p_pair_flops(6, True)} per (target, box) with the Laplace expansion too, "
                            f"{m2p_pair_flops(6, False)} Yukawa only")):
        rf["flop_convention"] = "FMA 2, other op 1, transcendental 1; " + fl
    dom = max(("p2p", "m2p", "moments", "combine"), key=lambda k: kt[("fp32", k)][0])
    main_rf = dict(rf_m2p if dom == "m2p" else rf_p2p)
    main_rf["dominant_in_solve"] = dom
    p2p_ms, p2p_n = kt[("fp32", "p2p")]
    m2p_ms, m2p_n = kt[("fp32", "m2p")]
    avg_p2p = p2p_ms / max(p2p_n, 1)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Ginteractions/s",
        **common_fields(a, ms_step),
        "config": {"workload": f"{a.workload}: {WORKLOADS.get(a.workload, a.workload)}",
                   "panels": sum(s.nt for s in problem.surfaces), "unknowns": s32.num_unknowns(),
                   **PRM, "precision": "mixed"},
        "roofline": main_rf,
        "roofline_p2p": rf_p2p, "roofline_m2p": rf_m2p,
        "gmres": {"iters": r.iters, "outer": r.outer, "rel_resid": r.rel_resid,
                  "applications_per_step": sum(x.matvecs for x in rs) / len(rs),
                  "setup_s": round(setup_wall, 3), "autotune_s": round(autotune_s, 3)},
        "far_field_schedule": SCHEDULES[schedule],
        "launch_shape": {"p2p_segment": shape[0], "m2p_boxes_per_task": shape[1], "p2p_grid_work_items": shape[2],
                         "m2p_grid_work_items": shape[3]},
        "kernels_fp32": k32,
        "p2p_gpairs_s": round(r.p2p_pairs / (avg_p2p / 1e3) / 1e9, 2),
        "m2p_g_target_box_s": round(r.m2p_pairs / (m2p_ms / max(m2p_n, 1) / 1e3) / 1e9, 3) if m2p_n else None,
        "pairs_per_product": {"dense": r.dense_pairs, "p2p": r.p2p_pairs, "p2p_fused": r.p2p_fused_pairs,
                              "m2p": r.m2p_pairs, "m2p_fused": r.m2p_fused_pairs},
        "energies_kcal": {"F_solv": r.F_solv, "F_surf": r.F_surf, "F_coul": r.F_coul},
    }
    if not a.profile_only:
        # operator timing on the context's stream (HIP events), tuned schedule
        n = s32.num_unknowns()
        x = torch.tensor(np.random.default_rng(0).standard_normal(n), device="cuda:0")
        y = torch.empty_like(x)

        def op_timing(prec, nrep=10):
            keys = ("total_ms", "p2p_ms", "m2p_ms", "moments_ms", "rest_ms")
            store = dict.fromkeys(keys, 0.0)
            s32.matvec_dev(x, y, prec=prec)
            for _ in range(nrep):
                s32.matvec_dev(x, y, prec=prec)
                t = s32.last_matvec_timing()
                for k in store:
                    store[k] += t[k] / nrep
            return {k: round(v, 4) for k, v in store.items()}

        m32, m64 = op_timing(MIXED), op_timing(FP64)
        s32.set_schedule(0)              # serial: each kernel with the machine to itself
        m32s = op_timing(MIXED)
        s32.set_schedule(schedule)
        out["matvec_ms"] = {"fp32": m32, "fp64": m64, "fp32_serial_schedule": m32s}
        out["matvec_gint_s"] = {"fp32": round(r.dense_pairs / m32["total_ms"] / 1e6, 2),
                                "fp64": round(r.dense_pairs / m64["total_ms"] / 1e6, 2)}
        del x, y
        s32.close()
        # FP64 treecode at the same (theta, P), autotuned in FP64, profiled
        s64, _ = from_problem(problem, prec=FP64, **PRM)
        s64.prepare()
        if not a.no_autotune:
            s64.autotune(a.autotune_cache)
        s64.solve()
        n64 = max(2, a.steps // 4)
        s64.profile(True)
        sync()
        t0 = time.perf_counter()
        r64 = [s64.solve() for _ in range(n64)][-1]
        sync()
        t64 = (time.perf_counter() - t0) / n64
        kt64 = s64.kernel_times()
        sched64 = s64.schedule()
        s64.close()
        kt_sel["fp64"] = kt64
        r64_p2p = roofline("p2p", "fp64", fl_p2p, FP64_PEAK_TFLOPS, sched64)
        r64_m2p = roofline("m2p", "fp64", fl_m2p, FP64_PEAK_TFLOPS, sched64)
        dom64 = "m2p" if kt64[("fp64", "m2p")][0] > kt64[("fp64", "p2p")][0] else "p2p"
        out["roofline_fp64"] = dict(r64_m2p if dom64 == "m2p" else r64_p2p, dominant_in_solve=dom64,
                                    far_field_schedule=SCHEDULES[sched64])
        out["roofline_fp64_p2p"], out["roofline_fp64_m2p"] = r64_p2p, r64_m2p
        mm64, nm64 = kt64[("fp64", "m2p")]
        out["m2p_g_target_box_s_fp64"] = (round(r.m2p_pairs / (mm64 / max(nm64, 1) / 1e3) / 1e9, 3)
                                          if nm64 else None)
        out["fp64"] = {"treecode_ms_per_solve": round(1e3 * t64, 3), "iters": r64.iters,
                       "speedup_mixed_vs_fp64_treecode": round(t64 / (ms_step / 1e3), 3),
                       "kernels": per_kernel(kt64, "fp64"),
                       "F_solv_fp64_treecode": r64.F_solv, "F_surf_fp64_treecode": r64.F_surf,
                       "rel_diff_F_solv_mixed_vs_fp64": abs(r.F_solv - r64.F_solv) / abs(r64.F_solv),
                       "rel_diff_F_surf_mixed_vs_fp64": abs(r.F_surf - r64.F_surf) / abs(r64.F_surf)}
        print(f"[bench] FP64 treecode solve {1e3 * t64:.1f} ms", file=sys.stderr, flush=True)
        if not a.no_direct:
            sd, _ = from_problem(problem, prec=FP64, treecode=0, **PRM)
            sd.prepare()
            sync()
            t0 = time.perf_counter()
            rd = sd.solve()
            sync()
            td = time.perf_counter() - t0
            sd.close()
            out["fp64"].update({"direct_ms_per_solve": round(1e3 * td, 3), "direct_iters": rd.iters,
                                "speedup_mixed_vs_fp64_direct": round(td / (ms_step / 1e3), 3),
                                "F_solv_fp64_direct": rd.F_solv, "F_surf_fp64_direct": rd.F_surf,
                                "rel_diff_F_solv_mixed_vs_fp64_direct": abs(r.F_solv - rd.F_solv) / abs(rd.F_solv),
                                "rel_diff_F_surf_mixed_vs_fp64_direct": abs(r.F_surf - rd.F_surf) / abs(rd.F_surf)})
            print(f"[bench] FP64 direct solve {1e3 * td:.1f} ms", file=sys.stderr, flush=True)
        chk = {p: oracle_check(a.workload, v) for p, v in (("mixed", MIXED), ("fp64", FP64))}
        if chk["mixed"] is not None:
            out["energy_error_vs_oracle"] = chk
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_batch(a):
    """Orientation sweep: one step = pbt_solve_batch of 64 placements (the
    isolated energies included), FP32 interactions in FP64 refinement."""
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
    s.profile(True)
    t0 = time.perf_counter()
    stats, f = [], None
    for _ in range(a.steps):
        f = s.solve_batch(ids[0], R.reshape(64, 9), T)
        stats.append(s.last_stats())
    dt = (time.perf_counter() - t0) / a.steps
    kt = s.kernel_times()
    s.profile(False)
    pairs = sum(x.dense_pairs for x in stats) / len(stats)
    st = stats[-1]
    out = {"metric": METRIC, "value": round(pairs / dt / 1e9, 3), "unit": "Ginteractions/s",
           **common_fields(a, 1e3 * dt),
           "config": {"workload": f"orient_sweep: {WORKLOADS['orient_sweep']}", "placements": 64,
                      "unknowns_per_placement": s.num_unknowns(), **PRM, "precision": "mixed"},
           "roofline": None,
           "kernels_fp32_ms_per_step": {k: round(kt[("fp32", k)][0] / a.steps, 3)
                                        for k in ("p2p", "m2p", "moments", "combine")},
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
    out = {"metric": METRIC, "value": round(pairs / dt / 1e9, 3), "unit": "Ginteractions/s",
           **common_fields(a, 1e3 * dt),
           "config": {"workload": f"gradient: {WORKLOADS['gradient']}",
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


def summarize_counters(fetch_csv, write_csv, out_json):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
    counter reads for the plain 256 MiB device-to-device copy that
    --copy-calib runs (256 MiB read and 256 MiB written).  Averages over the
    dispatches of each (kernel, grid size)."""
    import collections
    import csv

    def load(path, counter):
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]) * 1024.0)
        return per

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    copy_bytes = 256.0 * 2 ** 20

    def calib(per, name):
        # the copy: the runtime's copy kernel with the most bytes moved
        cands = [(max(v), k) for k, v in per.items() if "copyBuffer" in k[0]]
        if not cands:
            raise SystemExit(f"no copy kernel in the {name} run (was it made with --copy-calib?)")
        return copy_bytes / max(cands)[0]

    ff, fw = calib(fetch, "FETCH_SIZE"), calib(write, "WRITE_SIZE")
    kernels = []
    for key in sorted(set(fetch) & set(write)):
        name, grid = key
        if "copyBuffer" in name or "fillBuffer" in name:
            continue
        f = sum(fetch[key]) / len(fetch[key]) * ff
        w = sum(write[key]) / len(write[key]) * fw
        m = re.search(r"::(k_\w+(?:<[^()]*>)?)\(", name)
        if not m:
            continue   # not a kernel of this library
        short = m.group(1)
        kernels.append({"kernel": short, "grid_size": grid, "dispatches": len(fetch[key]),
                        "fetch_bytes_per_launch": round(f), "write_bytes_per_launch": round(w),
                        "traffic_bytes_per_launch": round(f + w)})
    sha = [hashlib.sha256(open(p, "rb").read()).hexdigest() for p in P2P_SOURCES]
    out = {"fetch_scale": ff, "write_scale": fw, "calibration": "256 MiB device-to-device copy",
           "sources": [os.path.relpath(p, ROOT) for p in P2P_SOURCES], "sources_sha256": sha,
           "kernels": kernels}
    with open(out_json, "w") as fh:   # one kernel a line
        fh.write("{\n" + "".join(f" {json.dumps(k)}: {json.dumps(v)},\n" for k, v in out.items() if k != "kernels")
                 + ' "kernels": [\n' + ",\n".join("  " + json.dumps(k) for k in kernels) + "\n ]\n}\n")
    print(json.dumps({"written": out_json, "fetch_scale": ff, "write_scale": fw, "kernels": len(kernels)}))


def main():
    a = parse()
    if a.summarize_counters:
        return summarize_counters(*a.summarize_counters)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported (the sharded multi-GPU path "
              f"is not built)", file=sys.stderr)
        sys.exit(2)
    if a.workload == "orient_sweep":
        return bench_batch(a)
    if a.workload == "gradient":
        return bench_gradient(a)
    cpu = None
    if not (a.no_cpu_baseline or a.profile_only):
        # before anything touches the GPU: the oracle's worker processes are forked
        from workloads.problems import config_problem
        t0 = time.perf_counter()
        cpu = cpu_baseline(config_problem(a.workload), a.cpu_budget)
        print(f"[bench] CPU baseline (oracle) {time.perf_counter() - t0:.1f} s: "
              f"{cpu['value']:.4g} Gint/s on {cpu['cores']} cores", file=sys.stderr, flush=True)
    return bench_solve(a, cpu)


if __name__ == "__main__":
    main()
