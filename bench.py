"""Benchmark of the matrix-free Laplace hot path on one MI355X.

Timed step (the JSON `value`): one FP64 operator application dst = A src of the
continuous Q4 Laplacian on 64^3 curved cells (257^3 = 16,974,593 DoFs; deformation
x + 0.1 sin(pi x) sin(pi y) sin(pi z) per coordinate; 5 Gauss points per direction;
seeded U[-1,1] input already in HBM), with the library's default for this mesh, the metric
formed on the fly from the node displacements.  value = DoFs per second of that step.

Also reported, outside the timed region:
  roofline      the dominant kernel (curved-cell operator kernel) timed with HIP events on
                its stream (recorded by each launch's dispatch, in a second pass of the same
                number of applications right after the timed steps), against the FP64
                vector peak with the algorithmic flops of one application (plain
                sum-factorization count; the model intensity is above the FP64 ridge), its
                HBM fraction beside; `traffic` from the committed rocprofv3 counter summary
                when it was taken on the current kernel source;
  stored_metric_apply  the same operator with the metric stored per quadrature point (the
                kernel read-bound by that metric stream), against the HBM roofline;
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
  gmg_pcg_curved_q4_64^3  the same solver (FP32 V-cycle) on the curved mesh of the timed
                apply, metric on the fly and stored;
  adjoint       forward solve + adjoint solve + gradient kernel, CG Q3 on 32^3 cells,
                FP32 V-cycle;
  kappa_field_apply  the same apply with the variable coefficient of Sec. 4.3 folded into the
                stored metric (the stored-metric kernel);
  cpu_baseline  the CPU oracle on the host: its assembled CSR matrix of the timed operator
                (16^3 curved cells) applied over all host threads, and its GMG-PCG solve of
                CG Q2 on 32^3 cells.

  roofline.frac is the operator cell kernel's (HIP events around its launches); step_frac is
  the whole application (cell kernel plus halo addition) at the timed step's rate.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--solve-degrees 2,3,4,5,6]
       python bench.py --reduce NAME DIR [DIR]   (rocprofv3 CSV output -> summary under profiles/)
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


def measured_traffic(kernel=None):
    """HBM bytes per launch of the dominant kernel (or of `kernel`, a label of the summary)
    from the committed counter summary, or None when the summary is missing or was taken on
    another version of the kernels."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    if kernel is not None:
        return rec.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")
    return rec.get("hbm_bytes_per_launch")


def apply_bytes(n_dofs, n_cells, q_per_cell, real_bytes, geometry="stored"):
    """Algorithmic bytes of one CG application: read src, write dst once, one kappa per
    cell; on curved cells either the stored 6-entry metric per quadrature point
    (geometry "stored") or the node displacement field, one value per DoF ("otf")."""
    b = 2 * real_bytes * n_dofs + real_bytes * n_cells
    if geometry == "stored":
        b += 6 * real_bytes * q_per_cell * n_cells
    elif geometry == "otf":
        b += real_bytes * n_dofs
    return b


def apply_flops(n, n_cells, geometry="stored"):
    """Algorithmic flops of one curved CG application in the plain sum-factorization count
    (each one-dimensional application n^2 multiply-adds per line, no even-odd saving):
    values and gradients at the Gauss points and the test with gradients, 12 applications
    of n^4 multiply-adds per cell, plus 9 multiply-adds per point for q = G grad u.  With the
    metric on the fly add the gradient of the displacement field (6 applications) and the
    closed-form metric, 31 flops per point."""
    f = 24 * n ** 4 + 18 * n ** 3
    if geometry == "otf":
        f += 12 * n ** 4 + 31 * n ** 3
    return f * n_cells


def time_applies(prob, src, dst, steps, warmup):
    """ms per application over `steps` timed applications (after `warmup`), then the cell
    kernel's average duration over a second pass of `steps` applications in which every
    cell-kernel launch carries its own start and stop events (the per-launch events add about
    0.03 ms to each application, so they stay out of the first pass)."""
    import torch
    for _ in range(warmup):
        prob.apply(src, dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.apply(src, dst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.profile_start()
    for _ in range(steps):
        prob.apply(src, dst)
    launches, kern_ms = prob.profile_stop()
    return (t1 - t0) * 1e3 / steps, kern_ms / max(launches, 1), launches


def repetitions(prob, src, dst, reps=20, per_rep=100):
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


HBM_CEILING_BYTES = 1 << 30


def hbm_ceilings(nbytes=HBM_CEILING_BYTES, reps=10):
    """Practical HBM rates on this GPU with library kernels: a streaming read (sum of a
    float64 tensor of nbytes) and a device copy of nbytes; best of `reps`, GB/s."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, moved in (("read_GBs", lambda: a.sum(), nbytes), ("copy_GBs", lambda: b.copy_(a), 2 * nbytes)):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        out[name] = moved / (best * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


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


def curved_solves(degree=4, cells=64, repeats=2):
    """GMG-PCG on the curved mesh of the timed apply (sine problem, tolerance 1e-10, FP32
    V-cycle), with the metric formed on the fly (the default) and stored: time to solution,
    iterations, setup time and workspace, and the difference of the two solutions."""
    import torch
    import paper_1611_03029_amd as mfl
    out = {}
    xs = {}
    for name, mode in (("on_the_fly", mfl.METRIC_ON_THE_FLY), ("stored", mfl.METRIC_STORED)):
        t0 = time.perf_counter()
        prob = mfl.Problem(degree, cells, geometry=mfl.CURVED, curve_amp=0.1, build_mg=True,
                           mg_precision=mfl.F32, metric_mode=mode)
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
        out[name] = {"time_s": best, "iterations": its, "final_rel_residual": res, "setup_s": setup_s,
                     "workspace_bytes": int(prob.workspace.numel())}
        del prob
        torch.cuda.empty_cache()
    out["max_rel_diff_of_the_solutions"] = ((xs["on_the_fly"] - xs["stored"]).abs().max().item() /
                                            xs["stored"].abs().max().item())
    return out


# The paper's solver timings for its smooth-solution example (Sec. 4.3, data tables of Fig.
# accuracy_3d_cube: columns qTime/qIt for the matrix-free CG solver and dgTim/dgIt for
# DG-SIP), full 28-core Broadwell node, FP64, tolerance 1e-9: {(k, Nc): (s, its, s, its)}.
PAPER_EXAMPLE_TIMES = {(2, 64): (0.1269, 5, 1.2825, 12), (3, 64): (0.4598, 5, 2.6152, 10),
                       (4, 64): (1.0753, 5, 5.2967, 10), (5, 48): (0.9218, 5, 4.4418, 11)}


def paper_example(repeats=2, degrees=None):
    """Time to solution of the smooth-solution example (three Gaussians on (-1,1)^3, Neumann
    at x_e = -1, Dirichlet at x_e = +1) with GMG-PCG at the paper's tolerance 1e-9, CG and
    DG-SIP (penalty (k+1)^2 3/h, GLL-basis Jacobi smoother), FP32 and FP64 V-cycles."""
    import torch
    import paper_1611_03029_amd as mfl
    out = {}
    for (k, nc), (cg_s, cg_it, dg_s, dg_it) in PAPER_EXAMPLE_TIMES.items():
        if degrees is not None and k not in degrees:
            continue
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
    for rep in range(3):
        # a new kappa in every repetition (as in an optimization loop), so that the forward
        # solve's set_kappa rebuilds; the adjoint's call with the same kappa returns at once
        kt = torch.tensor(np.exp(g) * (1.0 + 0.01 * rep), device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = mfl.PoissonSolve.apply(kt, prob, b, 1e-10, 100)
        (0.5 * ((u - u_t) ** 2).sum()).backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return {"n_dofs": prob.n_dofs, "n_cells": prob.n_cells,
            "forward_adjoint_gradient_s": best,
            "note": "includes the forward solve's set_kappa rebuild (diagonals, eigenvalue estimates); "
                    "the adjoint's set_kappa with the same kappa is recognized and skipped"}


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cells=16, reps=5, products=20):
    """The CPU oracle on the host cores of this machine.

    apply: the oracle's assembled CSR matrix of the timed operator (CG Q4, curved cells,
    assembled from dense element matrices) applied with torch's CSR product over all host
    threads; `cells`^3 cells instead of 64^3 (the 64^3 matrix would hold about 3.7e9 nonzeros,
    44 GB), which leaves the CSR product out of cache, so its DoFs/s carries over.  Min and
    median over `reps` runs of `products` products; assembly is not timed.
    solve: the oracle's textbook GMG-PCG (scipy CSR, one thread) on CG Q2 with 32^3 cells,
    sine right-hand side, tolerance 1e-10: setup (assembly of every level, eigenvalue
    estimates) and solve wall times."""
    import numpy as np
    import torch

    from oracle import cg as o_cg
    from oracle import mg as o_mg
    from oracle.mesh import Box
    from seeded_inputs import SEED_CG_Q4_CURVED, uniform_vector

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    torch.set_num_threads(threads)
    t0 = time.perf_counter()
    box = Box(cells, 4, 0.1)
    A = o_cg.assemble(box)
    assemble_s = time.perf_counter() - t0
    nnz = int(A.nnz)
    At = torch.sparse_csr_tensor(torch.from_numpy(A.indptr.astype(np.int64)),
                                 torch.from_numpy(A.indices.astype(np.int64)),
                                 torch.from_numpy(A.data), size=A.shape)
    u = torch.from_numpy(uniform_vector(box.n_dofs, SEED_CG_Q4_CURVED))
    y = At @ u
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for _ in range(products):
            y = At @ u
        times.append((time.perf_counter() - t0) / products)
    times.sort()
    del At, A, y
    t0 = time.perf_counter()
    mg = o_mg.Multigrid(32, 2)
    setup_s = time.perf_counter() - t0
    fine = mg.levels[-1]
    b = o_cg.rhs(fine["box"])
    t0 = time.perf_counter()
    _, its, res, _ = o_mg.pcg(fine["A"], b, mg.vcycle, tol=1e-10)
    solve_s = time.perf_counter() - t0
    return {"value": box.n_dofs / times[0], "unit": "DoFs/s", "cores": threads, "kind": "oracle",
            "sample": "CSR product of the oracle's assembled CG Q4 operator on %d^3 curved cells "
                      "(%d DoFs, %d nonzeros; torch CSR over %d host threads), min of %d runs of %d "
                      "products" % (cells, box.n_dofs, nnz, threads, reps, products),
            "median_dofs_per_s": box.n_dofs / times[len(times) // 2],
            "ms_per_product_min": times[0] * 1e3,
            "assembly_s": assemble_s,
            "nproc": os.cpu_count(), "cpu_model": host_cpu_model(),
            "gmg_pcg_q2_32cubed": {"n_dofs": fine["box"].n_dofs, "setup_s": setup_s, "solve_s": solve_s,
                                   "iterations": its, "final_rel_residual": res,
                                   "threads": "1 (scipy CSR products)"}}


# ---- reduction of rocprofv3 output (CSV) into the summaries kept under profiles/ ----------

def _find_csv(path, suffix):
    """`path` itself, or the one file under the directory `path` whose name ends in `suffix`."""
    import glob
    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit("no *%s under %s" % (suffix, path))
    return hits[-1]


def _col(row, name):
    for k in row:
        if k.lower() == name:
            return row[k]
    raise KeyError(name)


def counter_dispatches(path, counter=None, resources=None):
    """Per-dispatch counter values of a rocprofv3 --pmc CSV (counter_collection.csv):
    {(dispatch id, counter): [kernel name, grid size, value summed over the rows]}.
    resources (a dict) receives {kernel name: (VGPRs, AGPRs, SGPRs, LDS bytes, work-group size)}."""
    import csv
    out = {}
    with open(_find_csv(path, "counter_collection.csv"), newline="") as f:
        for r in csv.DictReader(f):
            name = _col(r, "counter_name")
            if counter is not None and name != counter:
                continue
            key = (int(_col(r, "dispatch_id")), name)
            rec = out.setdefault(key, [_col(r, "kernel_name"), int(float(_col(r, "grid_size"))), 0.0])
            rec[2] += float(_col(r, "counter_value"))
            if resources is not None:
                resources[rec[0]] = tuple(int(float(_col(r, c))) for c in (
                    "vgpr_count", "accum_vgpr_count", "sgpr_count", "lds_block_size", "workgroup_size"))
    return out


def waves_per_simd(vgprs, agprs, lds, wg):
    """Resident waves per SIMD from the register and LDS use (512 registers per lane of a
    SIMD shared by VGPRs and AGPRs in granules of 8; 160 KiB of LDS per CU; 4 SIMDs per CU;
    at most 8 waves per SIMD)."""
    regs = max(8, -(-(vgprs + agprs) // 8) * 8)
    by_regs = 512 // regs
    waves_wg = -(-wg // 64)
    by_lds = (160 * 1024 // lds) * waves_wg / 4.0 if lds else 8
    return min(8, by_regs, by_lds)


def short_kernel_name(name):
    """Kernel name without namespaces and argument list: apply_brick_kernel<4, double, true, 0>."""
    n = name
    for pre in ("(anonymous namespace)::", "void ", "mfl::"):
        n = n.replace(pre, "")
    return n.split("(")[0].strip()


def reduce_traffic(fetch, write, calib_bytes, kernels, algorithmic, workload, commands, out_path):
    """HBM bytes per dispatch of each kernel whose name contains one of `kernels` (dict
    substring -> {"algorithmic_bytes": ...}, optionally "grid": the launch's grid size), from a
    FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch).  Each counter is scaled by what it
    reads for the largest plain device copy in the same run (__amd_rocclr_copyBuffer of
    `calib_bytes` bytes each way, the size of the largest copy that run makes).  WRITE_SIZE
    counts a copy's written bytes exactly (scale 1.0 on copies of 136 MB, 453 MB and 1 GiB), so
    a write scale away from 1 means that `calib_bytes` is not the size of that copy: refused."""
    import statistics
    f = counter_dispatches(fetch, "FETCH_SIZE")
    w = counter_dispatches(write, "WRITE_SIZE")

    def calib(recs):
        vals = [v for (name, _g, v) in recs.values() if "copyBuffer" in name]
        if not vals:
            raise SystemExit("no copyBuffer dispatch for the calibration")
        return max(vals)

    fk, wk = calib(f), calib(w)
    fs, ws = calib_bytes / (fk * 1024.0), calib_bytes / (wk * 1024.0)
    if not 0.95 <= ws <= 1.05:
        raise SystemExit("calibration copy of %d bytes does not match the largest copy of the run "
                         "(WRITE_SIZE %.0f KiB)" % (calib_bytes, wk))
    res = {"workload": workload, "kernel_source_hash": kernel_source_hash(), "commands": commands,
           "calibration": {"kernel": "__amd_rocclr_copyBuffer (largest device copy of the run)",
                           "bytes_each_way": calib_bytes, "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk,
                           "fetch_scale": fs, "write_scale": ws},
           "kernels": {}}
    for label, spec in kernels.items():
        def pick(recs):
            return [v for (name, g, v) in recs.values()
                    if spec["match"] in short_kernel_name(name) and ("grid" not in spec or g == spec["grid"])]
        fv, wv = pick(f), pick(w)
        if not fv or not wv:
            raise SystemExit("kernel %s not found" % spec["match"])
        rd = statistics.median(fv) * 1024.0 * fs
        wr = statistics.median(wv) * 1024.0 * ws
        rec = {"match": spec["match"], "dispatches": [len(fv), len(wv)],
               "FETCH_SIZE_KiB_per_dispatch": statistics.median(fv),
               "WRITE_SIZE_KiB_per_dispatch": statistics.median(wv),
               "hbm_read_bytes": rd, "hbm_write_bytes": wr, "hbm_bytes_per_launch": rd + wr}
        if "algorithmic_bytes" in spec:
            rec["algorithmic_bytes"] = spec["algorithmic_bytes"]
            rec["hbm_over_algorithmic"] = (rd + wr) / spec["algorithmic_bytes"]
        res["kernels"][label] = rec
    if algorithmic is not None:
        res["algorithmic_bytes_per_launch"] = algorithmic
        first = next(iter(res["kernels"].values()))
        res["hbm_bytes_per_launch"] = first["hbm_bytes_per_launch"]
    with open(out_path, "w") as fo:
        json.dump(res, fo, indent=1)
    print("wrote", out_path)


def summarize_sq(path, groups, title, command, out_path):
    """Median over dispatches of SQ (and TA/TD/TCP/TCC) counters per kernel group
    (substring, label[, grid size]), with the ratios used in the design notes and the
    register/LDS use and resident waves per SIMD, as a text summary."""
    import statistics
    res = {}
    recs = counter_dispatches(path, resources=res)
    lines = ["# rocprofv3 SQ counters: " + title, "# command: " + command,
             "# kernel source hash (bench.kernel_source_hash): " + kernel_source_hash(),
             "# median over dispatches of the per-dispatch sums; ratios are between counters of the same unit", ""]
    for grp in groups:
        match, label = grp[0], grp[1]
        grid = grp[2] if len(grp) > 2 else None
        vals, kn = {}, None
        for (_d, cname), (kname, g, v) in recs.items():
            if match in short_kernel_name(kname) and (grid is None or g == grid):
                vals.setdefault(cname, []).append(v)
                kn = kname
        if not vals:
            continue
        med = {c: statistics.median(v) for c, v in vals.items()}
        lines.append("## %s (%d dispatches%s)" % (label, max(len(v) for v in vals.values()),
                                                   "" if grid is None else ", grid %d" % grid))
        if kn in res:
            vg, ag, sg, lds, wg = res[kn]
            lines.append("resources: %d VGPRs, %d AGPRs, %d SGPRs, %d B LDS per work-group of %d; "
                         "%.2g waves per SIMD resident" % (vg, ag, sg, lds, wg, waves_per_simd(vg, ag, lds, wg)))
        for c in sorted(med):
            lines.append("%-30s %14.6g" % (c, med[c]))
        cyc = med.get("SQ_WAVE_CYCLES")
        for c in ("SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_ANY",
                  "SQ_WAIT_INST_LDS", "SQ_INST_CYCLES_VMEM_RD", "SQ_INST_CYCLES_VMEM_WR"):
            if cyc and c in med:
                lines.append("%-40s %8.3f" % (c + " / SQ_WAVE_CYCLES", med[c] / cyc))
        if "TCC_HIT_sum" in med and med.get("TCC_HIT_sum", 0) + med.get("TCC_MISS_sum", 0) > 0:
            lines.append("%-40s %8.3f" % ("L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS)",
                                          med["TCC_HIT_sum"] / (med["TCC_HIT_sum"] + med["TCC_MISS_sum"])))
        if "SQ_LDS_BANK_CONFLICT" in med and med.get("SQ_INSTS_LDS"):
            lines.append("%-40s %8.3f" % ("SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS",
                                          med["SQ_LDS_BANK_CONFLICT"] / med["SQ_INSTS_LDS"]))
        lines.append("")
    open(out_path, "w").write("\n".join(lines))
    print("wrote", out_path)


def summarize_stats(path, title, command, out_path, top=25):
    """Kernel statistics of a rocprofv3 --kernel-trace --stats run as a text table."""
    import csv
    rows = []
    with open(_find_csv(path, "kernel_stats.csv"), newline="") as f:
        for r in csv.DictReader(f):
            rows.append((short_kernel_name(_col(r, "name")), int(_col(r, "calls")),
                         float(_col(r, "averagens")), float(_col(r, "totaldurationns")),
                         float(_col(r, "percentage"))))
    rows.sort(key=lambda x: -x[3])
    lines = ["# rocprofv3 kernel statistics: " + title, "# command: " + command,
             "# kernel source hash (bench.kernel_source_hash): " + kernel_source_hash(),
             "%-58s %8s %12s %14s %8s" % ("kernel", "calls", "average_ns", "total_ns", "percent")]
    for n, c, a, t, pc in rows[:top]:
        lines.append("%-58s %8d %12.0f %14.0f %8.2f" % (n[:58], c, a, t, pc))
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("wrote", out_path)


# How each committed summary under profiles/ is made: the rocprofv3 runs (R = repository
# root on the GPU machine, OUT = a directory for their output) and the reduction that turns
# their CSV output into the summary (`python bench.py --reduce NAME DIR [DIR]`).
_BENCH_Q4 = "python3 $R/bench.py --steps 5 --warmup 1 --no-extras --no-cpu-baseline"
_SQ = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
       "SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT")
_SOLVE_Q4 = "python3 $R/bench.py --solve-only --solve-degrees 4"
_SIPG = "python3 $R/bench.py --sipg-only --steps 5"
_SQ2 = "SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_LDS SQ_INST_CYCLES_VMEM_RD SQ_INSTS_VMEM_RD TA_BUSY_avr TD_TD_BUSY_sum"
_TCC = "TCC_HIT_sum TCC_MISS_sum"
REDUCTIONS = {
    "cg_apply_traffic": {
        "out": "profiles/cg_apply_q4_64cubed_curved_traffic.json",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
                 "-d $OUT/pmc_fetch -o run -- " + _BENCH_Q4,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
                 "-d $OUT/pmc_write -o run -- " + _BENCH_Q4]},
    "cg_apply_sq": {
        "out": "profiles/cg_apply_q4_64cubed_curved_sq_counters.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _SQ + " --output-format csv "
                 "-d $OUT/pmc_sq -o run -- " + _BENCH_Q4]},
    "cg_solve_sq": {
        "out": "profiles/gmg_pcg_q4_64cubed_sq_counters.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _SQ + " --output-format csv "
                 "-d $OUT/solve_sq -o run -- " + _SOLVE_Q4,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _SQ2 + " --output-format csv "
                 "-d $OUT/solve_sq2 -o run -- " + _SOLVE_Q4]},
    "cg_solve_traffic": {
        "out": "profiles/gmg_pcg_q4_64cubed_traffic.json",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
                 "-d $OUT/solve_fetch -o run -- " + _SOLVE_Q4,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
                 "-d $OUT/solve_write -o run -- " + _SOLVE_Q4]},
    "cg_solve_stats": {
        "out": "profiles/gmg_pcg_q4_64cubed_kernel_stats.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
                 "-d $OUT/solve_ktrace -o run -- " + _SOLVE_Q4]},
    "sipg_sq": {
        "out": "profiles/sipg_apply_q3_q5_sq_counters.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _SQ + " --output-format csv "
                 "-d $OUT/sipg_sq -o run -- " + _SIPG,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _SQ2 + " --output-format csv "
                 "-d $OUT/sipg_sq2 -o run -- " + _SIPG,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + _TCC + " --output-format csv "
                 "-d $OUT/sipg_tcc -o run -- " + _SIPG]},
    "sipg_stats": {
        "out": "profiles/sipg_apply_q3_q5_kernel_stats.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
                 "-d $OUT/sipg_ktrace -o run -- python3 $R/bench.py --sipg-only --steps 20"]},
    "sipg_traffic": {
        "out": "profiles/sipg_apply_q3_q5_traffic.json",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
                 "-d $OUT/sipg_fetch -o run -- " + _SIPG,
                 "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
                 "-d $OUT/sipg_write -o run -- " + _SIPG]},
    "cg_apply_stats": {
        "out": "profiles/cg_apply_q4_64cubed_curved_kernel_stats.txt",
        "runs": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
                 "-d $OUT/prof_ktrace -o run -- python3 $R/bench.py --steps 20 --warmup 2 "
                 "--no-extras --no-cpu-baseline"]},
}


def run_reduction(name, dirs):
    spec = REDUCTIONS[name]
    cmd = " ; ".join(spec["runs"]) + "  (R = repository root, OUT = output directory)"
    out = os.path.join(ROOT, spec["out"])
    if name == "cg_apply_traffic":
        n, cells, q = 257 ** 3, 64 ** 3, 125
        alg = apply_bytes(n, cells, q, 8, "otf")
        # the run's largest device copy: the copy of the measured HBM ceilings
        reduce_traffic(dirs[0], dirs[1], HBM_CEILING_BYTES,
                       {"apply_brick_kernel<4,double,curved,on-the-fly>": {
                            "match": "apply_brick_kernel<4, double, true, 0, true>", "algorithmic_bytes": alg},
                        "apply_brick_kernel<4,double,curved,stored>": {
                            "match": "apply_brick_kernel<4, double, true, 0, false>",
                            "algorithmic_bytes": apply_bytes(n, cells, q, 8, "stored")},
                        "halo_add_kernel<4,double>": {"match": "halo_add_kernel<4, double>"}},
                       alg, "CG Q4 operator apply, 64^3 curved cells (257^3 DoFs), FP64 (metric on the fly; "
                       "the stored-metric apply of the same run beside it)", spec["runs"], out)
    elif name == "cg_apply_sq":
        summarize_sq(dirs[0], [("apply_brick_kernel<4, double, true, 0, true>", "FP64, metric on the fly"),
                               ("apply_brick_kernel<4, float, true, 0, true>", "FP32, metric on the fly"),
                               ("apply_brick_kernel<4, double, true, 0, false>", "FP64, stored metric"),
                               ("halo_add_kernel<4, double>", "halo addition, FP64")],
                     "CG Q4 operator kernel, 64^3 curved cells (257^3 DoFs)", cmd, out)
    elif name == "cg_solve_sq":
        fine = 8192 * 256   # work-items of the 64^3 level's operator launch (8192 bricks)
        groups = [("apply_brick_kernel<4, double, false", "Cartesian operator, FP64, 64^3 level", fine),
                  ("apply_brick_kernel<4, float, false", "Cartesian operator, FP32, 64^3 level", fine),
                  ("cheb_halo_quad_kernel<4, double>", "Chebyshev update + halo, FP64, 64^3 level", fine),
                  ("cheb_halo_quad_kernel<4, float>", "Chebyshev update + halo, FP32, 64^3 level", fine),
                  ("restrict_cell_kernel<4, double, 2>", "restriction, rows of 2 cells, FP64, 64^3 level"),
                  ("restrict_cell_kernel<4, float, 4>", "restriction, rows of 4 cells, FP32, 64^3 level"),
                  ("prolongate_kernel<4, double, double, 6>", "prolongation, rows of 6 cells, FP64, 64^3 level"),
                  ("prolongate_kernel<4, float, float, 8>", "prolongation, rows of 8 cells, FP32, 64^3 level")]
        summarize_sq(dirs[0], groups, "GMG-PCG solve kernels, CG Q4 on 64^3 Cartesian cells "
                     "(FP64 and FP32 V-cycles)", cmd, out)
        if len(dirs) > 1:
            summarize_sq(dirs[1], groups, "GMG-PCG solve kernels, CG Q4 on 64^3 Cartesian cells, waits, "
                         "vector-memory cycles, texture units", cmd, out.replace(".txt", "_2.txt"))
    elif name == "cg_solve_traffic":
        n = 257 ** 3
        kern = {"apply_brick_kernel<4,double,cartesian>": {"match": "apply_brick_kernel<4, double, false",
                                                           "grid": 8192 * 256, "algorithmic_bytes": 16 * n},
                "apply_brick_kernel<4,float,cartesian>": {"match": "apply_brick_kernel<4, float, false",
                                                          "grid": 8192 * 256, "algorithmic_bytes": 8 * n},
                # four DoFs per lane only on the 64^3 level (the 32^3 level's one-DoF-per-lane
                # form has the same grid size and another name)
                "cheb_halo_quad_kernel<4,float>": {"match": "cheb_halo_quad_kernel<4, float>", "grid": 8192 * 256,
                                                   "algorithmic_bytes": 28 * n},
                "cheb_halo_quad_kernel<4,double>": {"match": "cheb_halo_quad_kernel<4, double>", "grid": 8192 * 256,
                                                    "algorithmic_bytes": 56 * n}}
        reduce_traffic(dirs[0], dirs[1], 8 * n, kern, None,
                       "GMG-PCG solve, CG Q4 on 64^3 Cartesian cells, FP64 and FP32 V-cycles",
                       spec["runs"], out)
    elif name == "cg_solve_stats":
        summarize_stats(dirs[0], "GMG-PCG solves of the sine problem, CG Q4 on 64^3 Cartesian cells, "
                        "FP64 and FP32 V-cycles, two solves each", cmd, out, top=40)
    elif name == "sipg_sq":
        groups = [("sipg_kernel<3, double, false>", "SIPG Q3, FP64"), ("sipg_kernel<5, double, false>", "SIPG Q5, FP64")]
        summarize_sq(dirs[0], groups, "SIPG operator kernel, Q3 and Q5 on 32^3 and 64^3 cells", cmd, out)
        for i, d in enumerate(dirs[1:]):
            summarize_sq(d, groups, "SIPG operator kernel, Q3 and Q5 on 32^3 and 64^3 cells", cmd,
                         out.replace(".txt", "_%d.txt" % (i + 2)))
    elif name == "sipg_stats":
        summarize_stats(dirs[0], "SIPG applies, Q3 and Q5 on 32^3 and 64^3 Cartesian cells, FP64", cmd, out)
    elif name == "sipg_traffic":
        kern = {}
        for k, nc, n in ((3, 32, 32 ** 3 * 64), (3, 64, 64 ** 3 * 64), (5, 32, 32 ** 3 * 216), (5, 64, 64 ** 3 * 216)):
            cpb = (256 // 64) * (64 // (k + 1) ** 2) if k <= 3 else 256 // (k + 1) ** 2
            grid = 8 * (((nc // 2) * (nc // 4) * nc + cpb - 1) // cpb) * 256
            kern["Q%d_%d^3" % (k, nc)] = {"match": "sipg_kernel<%d, double, false>" % k, "grid": grid,
                                          "algorithmic_bytes": 16 * n}
        reduce_traffic(dirs[0], dirs[1], 8 * 64 ** 3 * 216, kern, None,
                       "SIPG applies, Q3 and Q5 on 32^3 and 64^3 Cartesian cells, FP64 (16 B/DoF algorithmic)",
                       spec["runs"], out)
    elif name == "cg_apply_stats":
        summarize_stats(dirs[0], "CG Q4 operator, 64^3 curved cells (257^3 DoFs), FP64 and FP32 applies "
                        "(warm-up, timed and repetition-protocol applies; setup kernels once)", cmd, out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--solve-degrees", default="2,3,4,5,6")
    ap.add_argument("--cpu-cells", type=int, default=16,
                    help="cells per direction of the oracle's CSR matrix timed on the host")
    ap.add_argument("--reduce", nargs="+", metavar=("NAME", "DIR"),
                    help="turn rocprofv3 CSV output into the summary NAME under profiles/ "
                         "(names: %s); no GPU needed" % ", ".join(sorted(REDUCTIONS)))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed step and FP32 apply")
    ap.add_argument("--sipg-only", action="store_true",
                    help="only the SIPG applies (a profiling target; prints their JSON, not the bench line)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the GMG-PCG solves of --solve-degrees (a profiling target; prints their JSON)")
    ap.add_argument("--example-only", action="store_true",
                    help="only the paper's smooth-solution example at --solve-degrees (a profiling target)")
    args = ap.parse_args()
    if args.reduce:
        run_reduction(args.reduce[0], args.reduce[1:])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path is single-GPU (multi-GPU sharding is a "
              "design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1611_03029_amd as mfl
    from seeded_inputs import SEED_CG_Q4_CURVED, uniform_vector

    torch.cuda.set_device(0)
    if args.sipg_only:
        res = {"sipg": sipg_configs(args.steps)}
        res["calibration_copy"] = calibration_copy(64 ** 3 * 216)
        print(json.dumps(res), flush=True)
        return
    if args.example_only:
        degs = [int(x) for x in args.solve_degrees.split(",") if x.strip()]
        print(json.dumps({"paper_example": paper_example(degrees=degs)}), flush=True)
        return
    if args.solve_only:
        for d in [int(s) for s in args.solve_degrees.split(",") if s.strip()]:
            print(json.dumps({"gmg_pcg": {"Q%d_64^3" % d: solve_comparison(d, 64)}}), flush=True)
            torch.cuda.empty_cache()
        return
    k, Nc = 4, 64
    # the library's default for this mesh: the metric formed on the fly in every apply
    prob = mfl.Problem(k, Nc, geometry=mfl.CURVED, curve_amp=0.1)
    n, cells, q = prob.n_dofs, prob.n_cells, (k + 1) ** 3
    u64 = torch.tensor(uniform_vector(n, SEED_CG_Q4_CURVED), dtype=torch.float64, device="cuda")
    y64 = torch.empty_like(u64)
    # the repetition protocol first: the timed steps then start on a GPU that has been busy
    protocol = repetitions(prob, u64, y64)
    ms_step, kern_ms, launches = time_applies(prob, u64, y64, args.steps, args.warmup)
    progress("timed FP64 applies done")
    traffic = measured_traffic()
    bytes64 = apply_bytes(n, cells, q, 8, "otf")
    flops = apply_flops(k + 1, cells, "otf")
    achieved_tf = flops / (kern_ms * 1e-3) / 1e12

    u32 = u64.float()
    y32 = torch.empty_like(u32)
    ms32, kern32, _ = time_applies(prob, u32, y32, max(args.steps // 2, 10), args.warmup)
    del prob, u32, y32
    torch.cuda.empty_cache()
    # the same operator with the metric stored per quadrature point (read by every apply)
    probs = mfl.Problem(k, Nc, geometry=mfl.CURVED, curve_amp=0.1, metric_mode=mfl.METRIC_STORED)
    mss, kerns, _ = time_applies(probs, u64, y64, max(args.steps // 2, 10), args.warmup)
    stored_bytes = apply_bytes(n, cells, q, 8, "stored")
    stored = {"ms_per_step": mss, "dofs_per_s": n / (mss * 1e-3), "kernel_ms": kerns,
              "algorithmic_bytes": stored_bytes,
              "achieved_GBs": stored_bytes / (kerns * 1e-3) / 1e9,
              "frac": stored_bytes / (kerns * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "step_frac": stored_bytes / (mss * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "traffic": measured_traffic("apply_brick_kernel<4,double,curved,stored>")}
    u32 = u64.float()
    y32 = torch.empty_like(u32)
    ms32s, kern32s, _ = time_applies(probs, u32, y32, max(args.steps // 2, 10), args.warmup)
    bytes32s = apply_bytes(n, cells, q, 4, "stored")
    stored["fp32"] = {"ms_per_step": ms32s, "kernel_ms": kern32s,
                      "frac": bytes32s / (kern32s * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del probs, u32, y32
    torch.cuda.empty_cache()
    progress("stored-metric applies done")
    # the variable-coefficient curved case: the coefficient of Sec. 4.3 folded into the stored
    # metric, so the kernel and bytes of the stored-metric apply
    probk = mfl.Problem(k, Nc, geometry=mfl.CURVED, curve_amp=0.1, kappa_field=mfl.KAPPA_COSINE,
                        kappa_field_amp=1e6)
    msk, kernk, _ = time_applies(probk, u64, y64, max(args.steps // 2, 10), args.warmup)
    kfield = {"ms_per_step": msk, "dofs_per_s": n / (msk * 1e-3), "kernel_ms": kernk,
              "achieved_GBs": stored_bytes / (kernk * 1e-3) / 1e9,
              "frac": stored_bytes / (kernk * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "coefficient": "1 + 1e6 prod_e cos^2(2 pi x_e + 0.1 e) at every Gauss point, folded into the metric"}
    del probk, y64
    progress("variable-coefficient applies done")
    calib = calibration_copy(n)
    del u64
    torch.cuda.empty_cache()
    ceilings = hbm_ceilings()

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
        # the metric on the fly: model intensity flops / bytes above the FP64 ridge (9.8), so
        # the vector FP64 peak bounds it; its HBM fraction is given beside
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "apply_brick_kernel<4,double,curved,on-the-fly metric>", "kernel_ms": kern_ms,
                     "algorithmic_flops": flops, "algorithmic_bytes": bytes64,
                     "intensity_flop_per_byte": flops / bytes64,
                     "hbm_frac": bytes64 / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "timed_launches": launches, "kernel_source_hash": kernel_source_hash(),
                     "step_frac": flops / (ms_step * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "step_frac_protocol_min": flops / (protocol["min_ms"] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "hbm_ceilings_measured": ceilings},
        "equiv_dofs_per_s": cells * k ** 3 / (ms_step * 1e-3),
        "fp32_apply": {"ms_per_step": ms32, "dofs_per_s": n / (ms32 * 1e-3), "kernel_ms": kern32},
        "timing_protocol": protocol,
        "stored_metric_apply": stored,
        "kappa_field_apply": kfield,
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
        result["gmg_pcg_curved_q4_64^3"] = curved_solves()
        progress("curved GMG-PCG solves done")
        result["adjoint"] = adjoint_config()
        progress("adjoint workload done")
        result["paper_example"] = paper_example()
        progress("paper example solves done")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_cells)
        progress("CPU oracle baseline done")
    print(json.dumps(result))


if __name__ == "__main__":
    main()
