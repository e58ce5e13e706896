"""Benchmark of the matrix-free Laplace hot path on one MI355X.

Timed step (the JSON `value`): one FP64 operator application dst = A src of the
continuous Q4 Laplacian on 64^3 curved cells (257^3 = 16,974,593 DoFs; deformation
x + 0.1 sin(pi x) sin(pi y) sin(pi z) per coordinate; 5 Gauss points per direction;
seeded U[-1,1] input already in HBM).  value = DoFs per second of that step.

Also reported, outside the timed region:
  roofline      the dominant kernel (curved-cell operator kernel) timed with HIP events on
                its stream, against the HBM roofline with the algorithmic bytes of one
                application; `traffic` from the committed rocprofv3 counter summary when it
                was taken on the current kernel source;
  timing_protocol  min and median ms per application over 20 repetitions of 10 back-to-back
                applications (events on the library's stream);
  fp32_apply    the same operator in FP32 (FP32 vectors and geometry factors);
  small_q2      CG Q2 on 8^3 cells: apply latency and the FP64 GMG-PCG solve;
  sipg          SIPG Q3 and Q5 on 32^3 cells and, for steady state, 64^3 cells (FP64 apply),
                with HBM and FP64-ALU fractions;
  paper_example time to solution of the paper's smooth-solution example (CG and DG-SIP),
                next to the paper's own timings
  gmg_pcg       GMG-PCG time to solution, V-cycle in FP32 and in FP64 inside the FP64 outer
                CG, Cartesian 64^3 fine level, levels down to 2^3, Chebyshev(5)-Jacobi,
                tolerance 1e-10 relative residual, sine right-hand side, degrees 2..6;
  adjoint       forward solve + adjoint solve + gradient kernel, CG Q3 on 32^3 cells,
                FP32 V-cycle;
  cpu_baseline  the CPU oracle (element-by-element dense element matrices) on a bounded
                sample of rows of the timed workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--solve-degrees 2,3,4,5,6]
       python bench.py --sipg-only [--steps K]     (the SIPG applies alone, for profiling)
       python bench.py --solve-only [--solve-degrees 4]   (the GMG-PCG solves alone, for profiling)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "matrix-free Laplace apply DoFs/s (FP64) + GMG-PCG time-to-solution FP32-MG vs FP64"
KERNEL_SOURCES = ["paper_1611_03029_amd/csrc/kernels_cg.hip", "paper_1611_03029_amd/csrc/ct_tables.h",
                  "paper_1611_03029_amd/csrc/device_common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_apply_q4_64cubed_curved_traffic.json")


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter summary, or
    None when the summary is missing or was taken on another version of the kernel."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def apply_bytes(n_dofs, n_cells, q_per_cell, real_bytes, curved=True):
    """Algorithmic bytes of one CG application: read src, write dst once, one kappa per
    cell, and on curved cells the 6-entry metric per quadrature point."""
    b = 2 * real_bytes * n_dofs + real_bytes * n_cells
    if curved:
        b += 6 * real_bytes * q_per_cell * n_cells
    return b


def time_applies(prob, src, dst, steps, warmup):
    import torch
    for _ in range(warmup):
        prob.apply(src, dst)
    torch.cuda.synchronize()
    prob.profile_start()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.apply(src, dst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kern_ms = prob.profile_stop()
    return (t1 - t0) * 1e3 / steps, kern_ms / max(launches, 1), launches


def repetitions(prob, src, dst, reps=20, per_rep=10):
    """Apply timed in `reps` repetitions of `per_rep` back-to-back applications with events
    on the stream the library launches on (torch's current stream); ms per application."""
    import torch
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(per_rep):
            prob.apply(src, dst)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / per_rep)
    times.sort()
    return {"reps": reps, "applies_per_rep": per_rep, "min_ms": times[0], "median_ms": times[reps // 2]}


def calibration_copy(n):
    """A plain device copy of n doubles (the reference kernel for counter scaling)."""
    import torch
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": 8 * n, "bytes_written": 8 * n}


def small_config(steps):
    import torch
    import paper_1611_03029_amd as mfl
    from seeded_inputs import SEED_CG_Q2_SMALL, uniform_vector
    prob = mfl.Problem(2, 8, build_mg=True)
    u = torch.tensor(uniform_vector(prob.n_dofs, SEED_CG_Q2_SMALL), device="cuda")
    y = torch.empty_like(u)
    ms, kms, _ = time_applies(prob, u, y, steps, 10)
    b = prob.rhs_sine()
    best, its, res = None, 0, 0.0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, its, res = prob.solve(b, rtol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return {"n_dofs": prob.n_dofs, "apply_us": ms * 1e3, "kernel_us": kms * 1e3,
            "pcg_fp64_mg_s": best, "iterations": its, "final_rel_residual": res}


FP64_VECTOR_PEAK_TFLOPS = 78.6


def sipg_configs(steps):
    """SIPG Q3 and Q5 applies on 32^3 cells (the workload) and on 64^3 cells (steady state).
    Fractions of both bounds: HBM with 16 B/DoF (src read and dst written once), FP64 ALU
    with the element-centric flop model 2 (6 n^4 + 45 n^3) per cell (n = k+1)."""
    import torch
    import paper_1611_03029_amd as mfl
    from seeded_inputs import SEED_SIPG_Q3, SEED_SIPG_Q5, uniform_vector
    out = {}
    for nc in (32, 64):
        for k, seed in ((3, SEED_SIPG_Q3), (5, SEED_SIPG_Q5)):
            prob = mfl.Problem(k, nc, disc=mfl.SIPG)
            u = torch.tensor(uniform_vector(prob.n_dofs, seed), device="cuda")
            y = torch.empty_like(u)
            ms, kms, _ = time_applies(prob, u, y, steps if nc == 32 else max(steps // 4, 10), 10)
            n = k + 1
            byts = 16 * prob.n_dofs
            flops = 2.0 * (6 * n ** 4 + 45 * n ** 3) * prob.n_cells
            out["Q%d_%d^3" % (k, nc)] = {
                "n_dofs": prob.n_dofs, "ms_per_apply": ms, "kernel_ms": kms,
                "dofs_per_s": prob.n_dofs / (ms * 1e-3),
                "equiv_dofs_per_s": prob.n_cells * k ** 3 / (ms * 1e-3),
                "hbm_frac_16B_per_dof": byts / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "fp64_alu_frac": flops / (kms * 1e-3) / (FP64_VECTOR_PEAK_TFLOPS * 1e12)}
            del prob, u, y
            torch.cuda.empty_cache()
    return out


def solve_comparison(degree, cells, repeats=2):
    import torch
    import paper_1611_03029_amd as mfl
    out = {}
    xs = {}
    for name, prec in (("fp64_mg", mfl.F64), ("fp32_mg", mfl.F32)):
        t0 = time.perf_counter()
        prob = mfl.Problem(degree, cells, build_mg=True, mg_precision=prec)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        b = prob.rhs_sine()
        best = None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, its, res = prob.solve(b, rtol=1e-10, maxit=100)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        xs[name] = x
        out[name] = {"time_s": best, "iterations": its, "final_rel_residual": res,
                     "setup_s": setup_s, "dofs_per_s": prob.n_dofs / best}
        del prob
    diff = (xs["fp32_mg"] - xs["fp64_mg"]).abs().max().item() / xs["fp64_mg"].abs().max().item()
    out["n_dofs"] = int(xs["fp64_mg"].numel())
    out["speedup_fp32_mg"] = out["fp64_mg"]["time_s"] / out["fp32_mg"]["time_s"]
    out["max_rel_diff_fp32_vs_fp64_solution"] = diff
    return out


# The paper's solver timings for its smooth-solution example (Sec. 4.3, data tables of Fig.
# accuracy_3d_cube: columns qTime/qIt for the matrix-free CG solver and dgTim/dgIt for
# DG-SIP), full 28-core Broadwell node, FP64, tolerance 1e-9: {(k, Nc): (s, its, s, its)}.
PAPER_EXAMPLE_TIMES = {(2, 64): (0.1269, 5, 1.2825, 12), (3, 64): (0.4598, 5, 2.6152, 10),
                       (4, 64): (1.0753, 5, 5.2967, 10), (5, 48): (0.9218, 5, 4.4418, 11)}


def paper_example(repeats=2):
    """Time to solution of the smooth-solution example (three Gaussians on (-1,1)^3, Neumann
    at x_e = -1, Dirichlet at x_e = +1) with GMG-PCG at the paper's tolerance 1e-9, CG and
    DG-SIP (penalty (k+1)^2 3/h, GLL-basis Jacobi smoother), FP32 and FP64 V-cycles."""
    import torch
    import paper_1611_03029_amd as mfl
    out = {}
    for (k, nc), (cg_s, cg_it, dg_s, dg_it) in PAPER_EXAMPLE_TIMES.items():
        rec = {"cells": nc ** 3}
        for disc, name in ((mfl.CG, "cg"), (mfl.SIPG, "dg_sip")):
            for prec, pname in ((mfl.F32, "fp32_mg"), (mfl.F64, "fp64_mg")):
                # the paper's hierarchy: uniform refinement of the coarse mesh, i.e. down to
                # one cell for 2^m cells per direction and to 3^3 cells for 48^3
                prob = mfl.Problem(k, nc, disc=disc, bc=mfl.MIXED, build_mg=True, mg_precision=prec,
                                   penalty_factor=3.0, domain_lo=-1.0, domain_len=2.0,
                                   min_level_cells=3 if nc % 3 == 0 else 1)
                b = prob.rhs_gaussians()
                best = None
                for _ in range(repeats):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, its, res = prob.solve(b, rtol=1e-9, maxit=200)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    best = dt if best is None else min(best, dt)
                rec["%s_%s" % (name, pname)] = {"time_s": best, "iterations": its, "n_dofs": prob.n_dofs,
                                                "dofs_per_s": prob.n_dofs / best}
                del prob, b
                torch.cuda.empty_cache()
        rec["paper_28_cores"] = {"cg_time_s": cg_s, "cg_iterations": cg_it, "dg_sip_time_s": dg_s,
                                 "dg_sip_iterations": dg_it}
        out["Q%d_%d^3" % (k, nc)] = rec
    return out


def adjoint_config():
    import numpy as np
    import torch
    import paper_1611_03029_amd as mfl
    from seeded_inputs import SEED_KAPPA_FIELD, SEED_KAPPA_PERTURB, gaussian_field
    Nc, k = 32, 3
    g = gaussian_field(Nc ** 3, SEED_KAPPA_FIELD, 0.5)
    prob = mfl.Problem(k, Nc, build_mg=True, mg_precision=mfl.F32, kappa=np.exp(g))
    b = prob.rhs_sine()
    prob.set_kappa(np.exp(g + gaussian_field(Nc ** 3, SEED_KAPPA_PERTURB, 0.1)))
    u_t, _, _ = prob.solve(b, rtol=1e-10)
    best = None
    for _ in range(3):
        kt = torch.tensor(np.exp(g), device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = mfl.PoissonSolve.apply(kt, prob, b, 1e-10, 100)
        (0.5 * ((u - u_t) ** 2).sum()).backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return {"n_dofs": prob.n_dofs, "n_cells": prob.n_cells,
            "forward_adjoint_gradient_s": best,
            "note": "includes two set_kappa rebuilds (diagonals, eigenvalue estimates)"}


def cpu_baseline(budget_s=15.0):
    """The oracle's element-by-element apply (dense element matrices from per-point
    integrals) on sampled rows of the 64^3 curved Q4 workload, one host thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cg as o_cg
    from oracle.mesh import Box
    from seeded_inputs import SEED_CG_Q4_CURVED, uniform_vector

    box = Box(64, 4, 0.1)
    u = uniform_vector(box.n_dofs, SEED_CG_Q4_CURVED)
    rng = np.random.default_rng(99)
    done, t_used = 0, 0.0
    with threadpool_limits(1):
        while t_used < budget_s:
            rows = rng.choice(box.n_dofs, 64, replace=False)
            t0 = time.perf_counter()
            o_cg.apply_rows(box, u, rows)
            t_used += time.perf_counter() - t0
            done += len(rows)
    return {"value": done / t_used, "unit": "DoFs/s", "cores": 1, "kind": "oracle",
            "sample": "%d sampled rows of CG Q4 64^3 curved (dense element matrices per "
                      "cell, element-by-element), %.1f s on 1 host thread" % (done, t_used)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--solve-degrees", default="2,3,4,5,6")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed step and FP32 apply")
    ap.add_argument("--sipg-only", action="store_true",
                    help="only the SIPG applies (a profiling target; prints their JSON, not the bench line)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the GMG-PCG solves of --solve-degrees (a profiling target; prints their JSON)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path is single-GPU (multi-GPU sharding is a "
              "design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1611_03029_amd as mfl
    from seeded_inputs import SEED_CG_Q4_CURVED, uniform_vector

    torch.cuda.set_device(0)
    if args.sipg_only:
        print(json.dumps({"sipg": sipg_configs(args.steps)}), flush=True)
        return
    if args.solve_only:
        for d in [int(s) for s in args.solve_degrees.split(",") if s.strip()]:
            print(json.dumps({"gmg_pcg": {"Q%d_64^3" % d: solve_comparison(d, 64)}}), flush=True)
            torch.cuda.empty_cache()
        return
    k, Nc = 4, 64
    prob = mfl.Problem(k, Nc, geometry=mfl.CURVED, curve_amp=0.1)
    n, cells, q = prob.n_dofs, prob.n_cells, (k + 1) ** 3
    u64 = torch.tensor(uniform_vector(n, SEED_CG_Q4_CURVED), dtype=torch.float64, device="cuda")
    y64 = torch.empty_like(u64)
    ms_step, kern_ms, launches = time_applies(prob, u64, y64, args.steps, args.warmup)
    protocol = repetitions(prob, u64, y64)
    progress("timed FP64 applies done")
    traffic = measured_traffic()
    bytes64 = apply_bytes(n, cells, q, 8)
    achieved = bytes64 / (kern_ms * 1e-3) / 1e9

    u32 = u64.float()
    y32 = torch.empty_like(u32)
    ms32, kern32, _ = time_applies(prob, u32, y32, max(args.steps // 2, 10), args.warmup)
    bytes32 = apply_bytes(n, cells, q, 4)
    del prob, u32, y32, y64
    calib = calibration_copy(n)
    del u64
    torch.cuda.empty_cache()

    result = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "CG Q4 operator apply, 64^3 curved cells (257^3 DoFs), FP64",
                   "degree": k, "cells_per_dim": Nc, "n_dofs": n, "geometry": "x+0.1 sin sin sin",
                   "quadrature": "Gauss %d^3" % (k + 1), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "measured_GBs": None if traffic is None else traffic / (kern_ms * 1e-3) / 1e9,
                     "kernel": "apply_brick_kernel<4,double,curved>", "kernel_ms": kern_ms,
                     "algorithmic_bytes": bytes64, "timed_launches": launches,
                     "kernel_source_hash": kernel_source_hash()},
        "equiv_dofs_per_s": cells * k ** 3 / (ms_step * 1e-3),
        "fp32_apply": {"ms_per_step": ms32, "dofs_per_s": n / (ms32 * 1e-3), "kernel_ms": kern32,
                       "achieved_GBs": bytes32 / (kern32 * 1e-3) / 1e9,
                       "frac": bytes32 / (kern32 * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "timing_protocol": protocol,
        "calibration_copy": calib,
        "paper_context": {"cg_curved_q4_dofs_per_s": 4.58e8,
                          "hardware": "2x14-core Xeon E5-2690 v4 (Broadwell), FP64, 393216-cell shell"},
    }
    progress("FP32 applies done")
    if not args.no_extras:
        result["small_q2"] = small_config(args.steps)
        result["sipg"] = sipg_configs(args.steps)
        progress("small Q2 and SIPG applies done")
        solves = {}
        for d in [int(s) for s in args.solve_degrees.split(",") if s.strip()]:
            solves["Q%d_64^3" % d] = solve_comparison(d, 64)
            torch.cuda.empty_cache()
            progress("GMG-PCG Q%d solves done" % d)
        result["gmg_pcg"] = solves
        result["adjoint"] = adjoint_config()
        progress("adjoint workload done")
        result["paper_example"] = paper_example()
        progress("paper example solves done")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_budget)
        progress("CPU oracle baseline done")
    print(json.dumps(result))


if __name__ == "__main__":
    main()
