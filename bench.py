"""Benchmark of the finite element hot path on one MI355X.

A step is one pass of the whole path over the synthetic workload: element
integration (K3) + deterministic CSR scatter (K5, with the Jacobi diagonal)
+ Jacobi-PCG to rtol 1e-10 (SpMV K7 and vector kernels K8).  The set-up
(mesh upload, DOF numbering, CSR pattern) is done once before timing, as the
pattern is reused by every assembly.  Default workload: 3D Poisson on the
unit cube, 128^3 Q1 hexahedra with interior vertices jittered by +-0.2h,
lognormal per-cell coefficients, f = 1, u = 0 on the boundary, FP64.

Prints one JSON line.  Run ``python bench.py`` (1 GPU, 10 timed steps).
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q1–Q4 hex elements assembled/s, % HBM/MFMA peak; solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    "c2": dict(dim=3, n=128, k=1, problem="poisson", precision="fp64", rtol=1e-10,
               text="3D Poisson -div(k grad u) = 1 on the unit cube, 128^3 Q1 hexes, interior vertices jittered "
                    "+-0.2h (seed 17080), lognormal per-cell k (seed 17081), u = 0 on the boundary, FP64 assembly "
                    "+ Jacobi-PCG to rtol 1e-10"),
    "c3q2": dict(dim=3, n=48, k=2, problem="elasticity", precision="fp64", rtol=1e-10, lognormal=False,
                 text="3D linear elasticity (E = 1, nu = 0.3), 48^3 Q2 hexes, jittered +-0.2h, f = (0,0,-1), clamped"),
    "c3q3": dict(dim=3, n=32, k=3, problem="elasticity", precision="fp64", rtol=1e-10, lognormal=False,
                 text="3D linear elasticity (E = 1, nu = 0.3), 32^3 Q3 hexes, jittered +-0.2h, f = (0,0,-1), clamped"),
    "c3q4": dict(dim=3, n=24, k=4, problem="elasticity", precision="fp64", rtol=1e-10, lognormal=False,
                 text="3D linear elasticity (E = 1, nu = 0.3), 24^3 Q4 hexes, jittered +-0.2h, f = (0,0,-1), clamped"),
    "c1": dict(dim=2, n=32, k=1, problem="poisson", precision="fp64", rtol=1e-10, jitter=0.0, lognormal=False,
               source_kind=2,
               text="2D Poisson on the unit square, 32^2 Q1 quads, k = 1, f = 2 pi^2 sin(pi x) sin(pi y), u = 0, "
                    "FP64 + Jacobi-PCG to rtol 1e-10"),
}


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def spmv_bytes(n, nnz, mode="csr"):
    """Algorithmic HBM bytes of one SpMV.  csr: values + column indices, row
    pointers, the input vector once and the output vector.  mesh (pattern
    evaluated from the mesh): values, the input vector once and the output
    vector.  sym (symmetric storage): the upper triangle's values (diagonal
    included) once, the input vector once and the output vector."""
    if mode == "sym":
        return (nnz + n) // 2 * 8 + 16 * n
    if mode == "mesh":
        return nnz * 8 + 16 * n
    return nnz * 12 + (n + 1) * 8 + 16 * n


def traffic_for(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counters of this kernel on
    this workload, or None when there are none or the kernel source changed
    since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("bench_workload") != workload:
        return None
    src = os.path.join(ROOT, e["source"])
    if not os.path.exists(src) or source_sha(src) != e["source_sha"]:
        return None
    return e["bytes_per_launch"]


def cpu_model():
    """The host CPU's model name (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(wl, gpu_iters, ncells_full, nnz_full, n=64, cg_its=60):
    """The oracle timed on this host on a bounded sample of the same workload
    (an n^d mesh of the same recipe), single-threaded (the parity build) and on
    all cores (its OpenMP build: element matrices per cell in parallel, then
    row-parallel accumulation in the serial order; row-parallel SpMV, dot
    products over fixed chunks).  Symbolic assembly (CSR pattern), numeric
    assembly and CG iterations are timed separately.  The step of the full
    workload is scaled from the sample as cells x numeric time per cell +
    the GPU's iteration count x CG time per iteration x nnz ratio; the symbolic
    phase is set-up on both sides and excluded from the step, as on the GPU."""
    import numpy as np
    import oracle as O
    from fe_inputs import lognormal_coefficients, structured_vertices

    dim, k = wl["dim"], wl["k"]
    P = O.Problem(dim, [n] * dim, k, source_kind=wl.get("source_kind", 1), source=(1.0,))
    v = structured_vertices(dim, n, jitter=wl.get("jitter", 0.2))
    coef = lognormal_coefficients(P.ncells) if wl.get("lognormal", True) else None
    code, nf, _ = O.number_nodes(dim, P.n, k, P.faces)
    cd = O.cell_dofs(P, code)
    nfree = nf * P.ncomp
    legs = {}
    for name, pat, asm, cg in (("single_thread", O.csr_pattern, O.assemble,
                                lambda rp, ci, va, b: O.pcg(rp, ci, va, b, 0.0, cg_its)),
                               ("all_cores", O.omp_csr_pattern, O.omp_assemble,
                                lambda rp, ci, va, b: O.omp_pcg(rp, ci, va, b, 0.0, cg_its))):
        t0 = time.perf_counter()
        rp, ci = pat(cd, nfree)
        t_sym = time.perf_counter() - t0
        t0 = time.perf_counter()
        vals, rhs, _ = asm(P, v, coef, cd, nfree, rp, ci)
        t_num = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = cg(rp, ci, vals, rhs)
        t_it = (time.perf_counter() - t0) / max(res["iters"], 1)
        nnz = int(rp[-1])
        step = t_num / P.ncells * ncells_full + t_it * (nnz_full / nnz) * gpu_iters
        legs[name] = {"value": ncells_full / step, "unit": "elements/s",
                      "cores": 1 if name == "single_thread" else O.omp_threads(),
                      "symbolic_s": t_sym, "numeric_s": t_num, "cg_ms_per_iteration": t_it * 1e3,
                      "cg_iterations_timed": res["iters"], "step_s_scaled": step}
    omp = legs["all_cores"]
    return {
        "value": omp["value"], "unit": "elements/s", "cores": omp["cores"], "kind": "oracle",
        "sample": f"oracle (C, FP64) on the same recipe at {n}^{dim} cells ({P.ncells} cells, {nfree} unknowns, "
                  f"nnz {int(rp[-1])}): symbolic, numeric and {cg_its} CG iterations timed; the full step scaled as "
                  f"cells x numeric time per cell + {gpu_iters:.0f} iterations x per-iteration time x nnz ratio "
                  f"({nnz_full}/{int(rp[-1])}); value from the all-cores (OpenMP) build",
        "cpu_model": cpu_model(), "affinity_cores": len(os.sched_getaffinity(0)),
        "single_thread": legs["single_thread"], "all_cores": omp,
    }


PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0}
E_BYTES = {"fp64": 8, "fp32": 4, "fp16": 4, "bf16": 4}  # element-matrix storage (FP32 for the reduced GEMMs)


def ne_ff(dim, n, k, ncomp):
    """Free-free element entries of a brick with every face clamped: the sum
    over cells of (free local DOFs)^2, which factors per axis into the sum over
    the cells along the axis of (free local nodes along it)^2."""
    tot = 1
    for _ in range(dim):
        tot *= sum(((k + 1) - (i == 0) - (i == n - 1)) ** 2 for i in range(n))
    return tot * ncomp * ncomp


def timed_launches(fn, stream, torch, reps):
    """Average duration of fn() from HIP events recorded on `stream` around
    `reps` back-to-back launches (after 3 warm-up launches)."""
    for _ in range(3):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def csr_roofline(A, F, torch, stream, reps=30):
    """The CSR SpMV (row pointers, column indices and values read; the K7 of the
    method's accounting: 12 nnz + 8 (n + 1) + 16 n bytes) of the assembled
    system, timed alone on the step's stream."""
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand(A.n_rows, dtype=torch.float64, device="cuda", generator=g)
    y = torch.empty_like(x)
    t = timed_launches(lambda: F.spmv(A.csr, x, y, stream), stream, torch, reps)
    sb = spmv_bytes(A.n_rows, A.nnz, "csr")
    mode, rpw, _ = F.spmv_plan_of(A.n_rows, A.nnz)
    return {"kernel": "spmv_kernel/csr", "plan": {"mode": mode, "rows_per_wave": rpw}, "bound": "hbm",
            "achieved": sb / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sb / t / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": sb, "avg_launch_us": t * 1e6, "timed_launches": reps,
            "traffic": traffic_for("spmv_kernel/csr", "c2"),
            "timing": f"HIP events around {reps} back-to-back launches on the step's stream"}


def c3_assembly(F, torch, reps=5, precisions=("fp64", "bf16", "fp16")):
    """3D elasticity on Q2 48^3, Q3 32^3, Q4 24^3 (jittered, f = (0,0,-1),
    clamped): assembly (K3 + K5) per precision with event-timed kernels, the
    K3 fraction of the matrix-core peak on 18 nn^2 nq flops per cell and of HBM
    on its element-matrix bytes, the K5 fraction of HBM on NE_ff (8 + 4) + 8 nnz
    + 8 n bytes (element entries and their positions read, values and rhs
    written); then the SpMV of the FP64 system through the block-staged
    traversal and through the CSR."""
    from fe_inputs import structured_vertices

    out = {}
    stream = torch.cuda.current_stream()
    for key in ("c3q2", "c3q3", "c3q4"):
        wl = WORKLOADS[key]
        dim, n, k = wl["dim"], wl["n"], wl["k"]
        ncells, nn = n ** dim, (k + 1) ** dim
        v = structured_vertices(dim, n, jitter=0.2)
        mesh = F.create_mesh(dim, [n] * dim, v, None)
        res = {"workload": wl["text"], "cells": ncells}
        for prec in precisions:
            coeff = F.make_coeff("elasticity", prec, source_kind=1, source=(0.0, 0.0, -1.0), dim=dim)
            A = F.Assembly(mesh, k, coeff)
            A.pattern()
            A.assemble()
            torch.cuda.synchronize()
            F.set_timing(True)
            F.get_timing(reset=True)
            for _ in range(reps):
                A.assemble(stream)
            torch.cuda.synchronize()
            tm = F.get_timing(reset=True)
            F.set_timing(False)
            k3 = tm["integrate_ms"] / max(tm["integrate_calls"], 1) * 1e-3
            k5 = tm["scatter_ms"] / max(tm["scatter_calls"], 1) * 1e-3
            nloc = 3 * nn
            fl = k3_flops(wl, ncells)
            e_bytes = ncells * (8 + nloc * nloc * E_BYTES[prec]) + (n + 1) ** dim * dim * 8
            k5_bytes = ne_ff(dim, n, k, 3) * (E_BYTES[prec] + 4) + 8 * A.nnz + 8 * A.n_rows
            r = {"elements_per_s": ncells / (k3 + k5), "k3_ms": k3 * 1e3, "k5_ms": k5 * 1e3,
                 "k3_algorithmic_tflops": fl / k3 / 1e12, "k3_mfma_frac": fl / k3 / 1e12 / PEAK_TFLOPS[prec],
                 "k3_hbm_frac": e_bytes / k3 / 1e9 / HBM_PEAK_GBS, "k5_hbm_frac": k5_bytes / k5 / 1e9 / HBM_PEAK_GBS,
                 "k3_bytes": e_bytes, "k5_bytes": k5_bytes}
            if prec == "fp64":
                res["dofs"], res["nnz"] = A.n_rows, A.nnz
                g = torch.Generator(device="cuda").manual_seed(6)
                x = torch.rand(A.n_rows, dtype=torch.float64, device="cuda", generator=g)
                y = torch.empty_like(x)
                tb = timed_launches(lambda: F.spmv_mesh(mesh, k, coeff, A.csr, x, y, stream), stream, torch, 10)
                tc = timed_launches(lambda: F.spmv(A.csr, x, y, stream), stream, torch, 10)
                k7 = spmv_bytes(A.n_rows, A.nnz, "csr")
                own = spmv_bytes(A.n_rows, A.nnz, "mesh")
                res["spmv"] = {
                    "block_staged_us": tb * 1e6, "block_staged_frac_own_bytes": own / tb / 1e9 / HBM_PEAK_GBS,
                    "csr_us": tc * 1e6, "csr_frac": k7 / tc / 1e9 / HBM_PEAK_GBS, "csr_bytes": k7,
                    "own_bytes": own, "csr_plan": list(F.spmv_plan_of(A.n_rows, A.nnz)[:2])}
                del x, y
            res[prec] = r
            print(f"[bench] {key} {prec}: K3 {k3 * 1e3:.2f} ms ({r['k3_mfma_frac']:.2f} of MFMA, "
                  f"{r['k3_hbm_frac']:.2f} of HBM), K5 {k5 * 1e3:.2f} ms ({r['k5_hbm_frac']:.2f} of HBM)",
                  file=sys.stderr, flush=True)
            del A
            torch.cuda.empty_cache()
        out[key] = res
        del mesh
    return out


def k3_flops(wl, ncells):
    """Algorithmic flops of element integration: Poisson 2 nn^2 d nq, elasticity
    18 nn^2 nq per cell (geometry excluded)."""
    d, k = wl["dim"], wl["k"]
    nn = nq = (k + 1) ** d
    per = 18 * nn * nn * nq if wl["problem"] == "elasticity" else 2 * nn * nn * d * nq
    return per * ncells


def assemble_only(args, wl, A, ncells, F, torch):
    for _ in range(args.warmup):
        A.assemble()
    torch.cuda.synchronize()
    F.set_timing(True)
    F.get_timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        A.assemble()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    tm = F.get_timing(reset=True)
    F.set_timing(False)
    k3 = tm["integrate_ms"] / max(tm["integrate_calls"], 1) * 1e-3
    k5 = tm["scatter_ms"] / max(tm["scatter_calls"], 1) * 1e-3
    fl = k3_flops(wl, ncells)
    peak = PEAK_TFLOPS[wl["precision"]]
    out = {"metric": "hex elements assembled/s (assembly only)", "value": ncells * args.steps / total,
           "unit": "elements/s", "steps": args.steps, "ms_per_step": total / args.steps * 1e3,
           "dtype": wl["precision"], "config": {"workload": wl["text"], "cells": ncells, "order": wl["k"],
                                                "dofs": A.n_rows, "nnz": A.nnz},
           "k3": {"ms": k3 * 1e3, "algorithmic_tflops": fl / k3 / 1e12, "peak_tflops": peak,
                  "frac": fl / k3 / 1e12 / peak},
           "k5": {"ms": k5 * 1e3}}
    print(json.dumps(out), flush=True)


def mixed_form(args, wl, mesh, A, x_fp64, F, torch, stream, ncells, lo="fp32"):
    """Same workload solved by iterative refinement: A_hi assembled in FP64
    (outer residual), A_lo with FP32 element integration and FP32-stored values
    (inner Jacobi-PCG; Q1 scalar systems in FP32 symmetric storage, 4 B per
    upper-triangle entry, else FP32 CSR at 8 B per nonzero).  Reports the step
    time and the solution's distance to the plain FP64 solve on this GPU."""
    src = (0.0, 0.0, -1.0) if wl["problem"] == "elasticity" else (1.0,)
    coeff_lo = F.make_coeff(wl["problem"], lo, source_kind=wl.get("source_kind", 1), source=src, dim=wl["dim"])
    A_lo = F.Assembly(mesh, wl["k"], coeff_lo)
    A_lo.pattern()
    # Q1 scalar systems: the inner operator in FP32 symmetric storage; else FP32 CSR values
    sym = wl["k"] == 1 and wl["problem"] == "poisson"
    if sym:
        v32 = torch.empty(F.sym_query(mesh, wl["k"], coeff_lo) // 8, dtype=torch.float32, device="cuda")
    else:
        v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
    ws = torch.empty(F.refine_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")

    def step():
        A.assemble(stream)
        A_lo.assemble(stream)
        x.zero_()
        if sym:
            F.sym_fp32_from_csr(mesh, wl["k"], coeff_lo, A_lo.csr, v32, stream)
            return F.refine_solve_sym(mesh, wl["k"], coeff_lo, A.csr, A_lo.csr, v32, A.rhs, x, wl["rtol"], 1e-5, 50,
                                      100000, ws, stream=stream)
        F.csr_to_fp32(A_lo.csr, v32, stream)
        return F.refine_solve(A.csr, A_lo.csr, A.rhs, x, wl["rtol"], 1e-5, 50, 100000, ws, values32=v32, stream=stream)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = step()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    err = (torch.linalg.vector_norm(x - x_fp64) / torch.linalg.vector_norm(x_fp64)).item()
    return {"elements_per_s": ncells * args.steps / total, "ms_per_step": total / args.steps * 1e3,
            "lo_precision": lo, "value_storage_lo": "fp32 symmetric (upper triangle)" if sym else "fp32 CSR",
            "inner_rtol": 1e-5,
            "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"], "relres": info["relres"],
            "rel_error_vs_fp64_solution": err}


def c3_precision(F, torch, orders=("c3q2", "c3q3", "c3q4"), precisions=("fp32", "fp16", "bf16")):
    """The precision form on 3D elasticity Q2 48^3 / Q3 32^3 / Q4 24^3: the plain
    FP64 solve (evaluated pattern, rtol 1e-10) against, per element-GEMM
    precision, (a) the matrix assembled with that precision solved in FP64 (the
    workload's configuration; its distance to the FP64 solution is the
    integration error, stated) and (b) iterative refinement to 1e-10: FP64
    residual with the FP64 matrix, inner Jacobi-PCG on the low-precision matrix
    stored in FP32 with the pattern evaluated from the mesh (4 B per entry),
    inner rtol 1e-4.  One solve each, wall clock."""
    from fe_inputs import structured_vertices

    out = {}
    for key in orders:
        wl = WORKLOADS[key]
        dim, n, k = wl["dim"], wl["n"], wl["k"]
        v = structured_vertices(dim, n, jitter=0.2)
        mesh = F.create_mesh(dim, [n] * dim, v, None)

        def assemble(prec):
            c = F.make_coeff("elasticity", prec, source_kind=1, source=(0.0, 0.0, -1.0), dim=dim)
            A = F.Assembly(mesh, k, c)
            A.pattern()
            A.assemble()
            return A

        A_hi = assemble("fp64")
        ws = torch.empty(F.refine_query(A_hi.n_rows), dtype=torch.uint8, device="cuda")
        x64 = torch.zeros(A_hi.n_rows, dtype=torch.float64, device="cuda")
        A_hi.solve(x64, wl["rtol"], 100000, ws)  # warm-up
        x64.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = A_hi.solve(x64, wl["rtol"], 100000, ws)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        nx = torch.linalg.vector_norm(x64)
        res = {"workload": wl["text"], "fp64": {"s": t64, "iters": info["iters"], "relres": info["relres"]}}
        for prec in precisions:
            A_lo = assemble(prec)
            dA = (torch.linalg.vector_norm(A_lo.values[:A_lo.nnz] - A_hi.values[:A_hi.nnz]) /
                  torch.linalg.vector_norm(A_hi.values[:A_hi.nnz])).item()
            xl = torch.zeros_like(x64)
            il = A_lo.solve(xl, wl["rtol"], 100000, ws)
            e_plain = (torch.linalg.vector_norm(xl - x64) / nx).item()
            del xl
            v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
            F.csr_to_fp32(A_lo.csr, v32)
            xr = torch.zeros_like(x64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ri = F.refine_solve_mesh(mesh, k, A_hi.coeff, A_hi.csr, A_lo.csr, A_hi.rhs, xr, wl["rtol"], 1e-4, 50,
                                     100000, ws, values32=v32)
            torch.cuda.synchronize()
            tr = time.perf_counter() - t0
            e_ref = (torch.linalg.vector_norm(xr - x64) / nx).item()
            res[prec] = {"matrix_rel_error": dA, "plain_fp64_solve_of_it": {"iters": il["iters"],
                                                                             "rel_error_vs_fp64": e_plain},
                         "refined": {"s": tr, "speedup_vs_fp64": t64 / tr, "outer_iters": ri["outer_iters"],
                                     "inner_iters": ri["inner_iters"], "status_ok": ri["status"] == F.FE_OK,
                                     "relres": ri["relres"], "rel_error_vs_fp64": e_ref}}
            print(f"[bench] {key} {prec}: |dA|/|A| {dA:.1e}, its FP64 solve {e_plain:.1e} from FP64; refined "
                  f"{tr:.2f} s vs {t64:.2f} s ({ri['outer_iters']} outer, {ri['inner_iters']} inner), "
                  f"{e_ref:.1e} from FP64", file=sys.stderr, flush=True)
            del A_lo, v32, xr
            torch.cuda.empty_cache()
        out[key] = res
        del A_hi, ws, x64, mesh
        torch.cuda.empty_cache()
    return out


DG_WORKLOAD = dict(dim=3, n=48, k=2, gamma=36.0, tau=1.0, rtol=1e-8,
                   text="interior-penalty DG (symmetric, tau = 1, gamma = 4 (k+1)^2 = 36) for -Laplace(u) = f on "
                        "the unit cube, 48^3 Q2 hexes jittered +-0.2h (seed 17080), f = 3 pi^2 prod sin(pi x_r), "
                        "u = 0 imposed weakly on the boundary, FP64 assembly + Jacobi-PCG to rtol 1e-8")


def dg_facet_bytes(n_rows, nnz, ncells, nn):
    """Algorithmic bytes of one launch of the DG cell kernel: the values of
    every row written once (8 nnz), the volume element matrices and loads read
    (8 ncells nn^2 + 8 n), rhs and dinv written (16 n), one row pointer per
    cell read (8 ncells).  The diagonal block's facet updates re-touch bytes
    the same workgroup has just written (an L2 hit), not counted."""
    return 8 * nnz + 8 * ncells * nn * nn + 8 * n_rows + 16 * n_rows + 8 * ncells


def dg_cpu_baseline(wl, gpu_iters, ncells_full, nnz_full, n=16, cg_its=100):
    """The oracle's DG assembly (single thread, the parity build) and its
    all-cores CG on the DG system of an n^3 mesh of the same recipe, scaled to
    the full workload like the main baseline: cells x assembly time per cell
    + the GPU's iterations x CG time per iteration x nnz ratio."""
    import oracle as O
    from fe_inputs import structured_vertices
    dim, k = wl["dim"], wl["k"]
    P = O.Problem(dim, [n] * dim, k, source_kind=2, source=(1.0,))
    v = structured_vertices(dim, n, jitter=0.2)
    t0 = time.perf_counter()
    D = O.DGSystem(P, v, gamma=wl["gamma"], tau=wl["tau"])
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = O.omp_pcg(D.rowptr, D.colind, D.values, D.rhs, 0.0, cg_its)
    t_it = (time.perf_counter() - t0) / max(res["iters"], 1)
    step = t_asm / P.ncells * ncells_full + t_it * (nnz_full / D.nnz) * gpu_iters
    return {"value": 1.0 / step, "unit": "solves/s", "cores": O.omp_threads(), "kind": "oracle",
            "sample": f"oracle (C, FP64) DG system at {n}^3 Q{k} ({P.ncells} cells, nnz {D.nnz}): pattern + "
                      f"assembly single-threaded ({t_asm:.2f} s, the pattern included), {res['iters']} CG "
                      f"iterations on all cores ({t_it * 1e3:.2f} ms each); the full solve scaled as cells x "
                      f"assembly time per cell + {gpu_iters:.0f} iterations x per-iteration time x nnz ratio",
            "step_s_scaled": step}


def dg_form(args, F, torch, steps=3, warmup=1):
    """The DG workload: a step is the DG assembly (volume integration + the
    cell kernel with the facet terms) + Jacobi-PCG through the cell-block
    SpMV (pattern evaluated), the pattern built once before timing.  Kernel
    times from HIP events on the step's stream; the CSR SpMV of the same
    system is timed alone for comparison."""
    from fe_inputs import structured_vertices
    wl = DG_WORKLOAD
    dim, n, k = wl["dim"], wl["n"], wl["k"]
    v = structured_vertices(dim, n, jitter=0.2)
    mesh = F.create_mesh(dim, [n] * dim, v)
    coeff = F.make_coeff("poisson", "fp64", source_kind=2, source=(1.0,), dim=dim)
    A = F.DGAssembly(mesh, k, coeff, wl["gamma"], wl["tau"])
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ncells, nn = n ** dim, (k + 1) ** dim
    torch.cuda.synchronize()
    print(f"[bench] DG form: cells={ncells} rows={A.n_rows} nnz={A.nnz}", file=sys.stderr, flush=True)

    def step():
        A.assemble(stream)
        x.zero_()
        return A.solve(x, wl["rtol"], 100000, ws, stream)

    for _ in range(warmup):
        info = step()
    F.set_timing(True)
    F.get_timing(reset=True)
    torch.cuda.synchronize()
    lat, iters = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        iters.append(info["iters"])
        print(f"[bench] DG step {i}: {lat[-1] * 1e3:.1f} ms, {info['iters']} iterations", file=sys.stderr,
              flush=True)
    total = time.perf_counter() - t0
    tm = F.get_timing(reset=True)
    F.set_timing(False)
    assert F.get_status(mesh) == F.FE_OK
    facet_s = tm["scatter_ms"] / max(tm["scatter_calls"], 1) * 1e-3
    k3_s = tm["integrate_ms"] / max(tm["integrate_calls"], 1) * 1e-3
    spmv_s = tm["spmv_ms"] / max(tm["spmv_calls"], 1) * 1e-3
    fb = dg_facet_bytes(A.n_rows, A.nnz, ncells, nn)
    sb = 8 * A.nnz + 16 * A.n_rows  # values read once, x read once, y written
    # the CSR traversal of the same system (row pointers and column indices read), for comparison
    g = torch.Generator(device="cuda").manual_seed(5)
    xr = torch.rand(A.n_rows, dtype=torch.float64, device="cuda", generator=g)
    yr = torch.empty_like(xr)
    t_csr = timed_launches(lambda: F.spmv(A.csr, xr, yr, stream), stream, torch, 10)
    t_blk = timed_launches(lambda: A.spmv(xr, yr, stream), stream, torch, 10)
    sb_csr = spmv_bytes(A.n_rows, A.nnz, "csr")
    mode, rpw, _ = F.spmv_plan_of(A.n_rows, A.nnz)
    out = {
        "workload": wl["text"], "cells": ncells, "dofs": A.n_rows, "nnz": A.nnz, "steps": steps,
        "solves_per_s": steps / total, "ms_per_step": total / steps * 1e3,
        "p50_ms": statistics.median(lat) * 1e3, "pcg_iters": statistics.mean(iters),
        "relres": info["relres"], "true_relres": info["true_relres"],
        "assembly": {"integrate_ms": k3_s * 1e3, "dg_cell_kernel_ms": facet_s * 1e3,
                     "elements_per_s": ncells / (k3_s + facet_s)},
        "roofline_dg_cell_kernel": {"kernel": "dg_cell_kernel<3,2>", "bound": "hbm", "achieved": fb / facet_s / 1e9,
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": fb / facet_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": fb,
                                    "avg_launch_us": facet_s * 1e6, "timed_launches": tm["scatter_calls"],
                                    "traffic": traffic_for("dg_cell_kernel", "dg_q2_48")},
        "roofline_spmv": {"kernel": "pcg_spmv_kernel/dg cell blocks", "bound": "hbm",
                          "achieved": sb / spmv_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": sb / spmv_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": sb,
                          "avg_launch_us": spmv_s * 1e6, "timed_launches": tm["spmv_calls"],
                          "traffic": traffic_for("pcg_spmv_kernel/dg", "dg_q2_48"),
                          "bytes": "8 nnz + 16 n: the values and x read once, y written (the pattern is evaluated)"},
        "spmv_alone": {"cell_blocks_us": t_blk * 1e6, "cell_blocks_frac": sb / t_blk / 1e9 / HBM_PEAK_GBS,
                       "csr_us": t_csr * 1e6, "csr_plan": {"mode": mode, "rows_per_wave": rpw},
                       "csr_frac_on_csr_bytes": sb_csr / t_csr / 1e9 / HBM_PEAK_GBS, "csr_bytes": sb_csr,
                       "timing": "HIP events around 10 back-to-back launches on the step's stream"},
    }
    del A, ws, x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle's DG system on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = dg_cpu_baseline(wl, statistics.mean(iters), ncells, out["nnz"])
    return out


SIMPLEX_WORKLOAD = dict(dim=3, n=64, k=2, rtol=1e-10,
                        text="P2 Lagrange on tetrahedra: the Kuhn subdivision of the 64^3 unit-cube brick "
                             "(1,572,864 tetrahedra as general connectivity), interior vertices jittered +-0.2h "
                             "(seed 17080), lognormal per-cell coefficient (seed 17081), f = 1, u = 0 on the "
                             "boundary; FP64 assembly + Jacobi-PCG (CSR SpMV) to rtol 1e-10")


NEDELEC_WORKLOAD = dict(dim=3, n=64, kappa=1.0, rtol=1e-8,
                        text="lowest-order Nedelec edge elements on tetrahedra: the Kuhn subdivision of the 64^3 "
                             "unit-cube brick (1,572,864 tetrahedra as general connectivity, jittered +-0.2h, seed "
                             "17080), curl(k curl u) + u = f with lognormal k per cell (seed 17081), f = (2 pi^2 + 1) "
                             "(sin pi y sin pi z, sin pi z sin pi x, sin pi x sin pi y), zero tangential trace; FP64 "
                             "assembly + Jacobi-PCG (CSR SpMV) to rtol 1e-8")


NEDELEC2_WORKLOAD = dict(dim=3, n=24, kappa=1.0, rtol=1e-8,
                         text="second-order Nedelec elements on tetrahedra (two DOFs per edge and per face): the "
                              "Kuhn subdivision of the 24^3 unit-cube brick (82,944 tetrahedra, jittered +-0.2h, seed "
                              "17080), curl(k curl u) + u = f with lognormal k per cell (seed 17081), f = (2 pi^2 + 1) "
                              "(sin pi y sin pi z, sin pi z sin pi x, sin pi x sin pi y), zero tangential trace; FP64 "
                              "assembly + Jacobi-PCG (CSR SpMV) to rtol 1e-8")


RT2_WORKLOAD = dict(dim=3, n=24, kappa=1.0, rtol=1e-8,
                    text="second-order Raviart-Thomas elements on tetrahedra (three fluxes per face, three interior "
                         "moments): the Kuhn subdivision of the 24^3 unit-cube brick (82,944 tetrahedra, jittered "
                         "+-0.2h, seed 17080), -grad(k div u) + u = f with lognormal k per cell (seed 17081), "
                         "f = (pi^2 + 1) (sin pi x_r)_r, zero normal trace; FP64 assembly + Jacobi-PCG (CSR SpMV) to "
                         "rtol 1e-8")


def vector_source(family, kappa):
    """The manufactured field's load factor: curl curl of the Nedelec field is
    2 pi^2 times it, -grad div of the Raviart-Thomas field pi^2 times it."""
    return ((math.pi ** 2 if family.startswith("raviart") else 2 * math.pi ** 2) + kappa,) * 3


def simplex_element_bytes(ncells, ntri, nloc, nverts, dim):
    """Algorithmic bytes of the element kernel: the element matrices' upper
    triangles and the loads written, connectivity, coefficients and vertex
    coordinates read once."""
    return 8 * ncells * (ntri + nloc) + 4 * (dim + 1) * ncells + 8 * ncells + 8 * dim * nverts


def simplex_gather_bytes(nnz, ncontrib):
    """Algorithmic bytes of the value gather: the contribution list (4 B per
    entry) and the element entry it names (8 B) in list order, the entry
    offsets and the values written."""
    return 12 * ncontrib + 8 * (nnz + 1) + 8 * nnz


def simplex_cpu_baseline(wl, gpu_iters, ncells_full, nnz_full, n=12, cg_its=100):
    """The oracle's P_k system on the Kuhn mesh of an n^3 brick of the same
    recipe (numbering, pattern and assembly single-threaded) and its
    all-cores CG, scaled to the full workload like the other baselines."""
    import oracle as O
    from fe_inputs import lognormal_coefficients, simplex_mesh
    v, c = simplex_mesh(wl["dim"], n, jitter=0.2)
    coef = lognormal_coefficients(c.shape[0])
    S = O.SimplexSystem(wl["dim"], wl["k"], v, c, coef=coef, source_kind=1, source=(1.0,))
    t_asm = S.t_assemble
    t0 = time.perf_counter()
    res = O.omp_pcg(S.rowptr, S.colind, S.values, S.rhs, 0.0, cg_its)
    t_it = (time.perf_counter() - t0) / max(res["iters"], 1)
    step = t_asm / c.shape[0] * ncells_full + t_it * (nnz_full / S.nnz) * gpu_iters
    return {"value": ncells_full / step, "unit": "elements/s", "cores": O.omp_threads(), "kind": "oracle",
            "sample": f"oracle (C, FP64) P{wl['k']} system on the Kuhn mesh of {n}^3 ({c.shape[0]} tetrahedra, "
                      f"nnz {S.nnz}): numeric assembly single-threaded ({t_asm:.2f} s; numbering and pattern "
                      f"{S.t_setup:.2f} s, outside the step as on the GPU), "
                      f"{res['iters']} CG iterations on all cores ({t_it * 1e3:.2f} ms each); the full step scaled "
                      f"as cells x assembly time per cell + {gpu_iters:.0f} iterations x per-iteration "
                      f"time x nnz ratio",
            "step_s_scaled": step}


def simplex_form(args, F, torch, steps=3, warmup=1, family=None):
    """The simplicial workload (Lagrange P2, or with family "nedelec" /
    "nedelec2" the first- / second-order edge elements, "raviart_thomas2" the
    second-order facet elements): a step is the
    assembly (element kernel + gathers through the stored map) + Jacobi-PCG
    on the CSR, the numbering, pattern and gather map built once before
    timing (Sect. 11.1)."""
    from fe_inputs import lognormal_coefficients, simplex_mesh
    wl = {None: SIMPLEX_WORKLOAD, "nedelec": NEDELEC_WORKLOAD, "nedelec2": NEDELEC2_WORKLOAD,
          "raviart_thomas2": RT2_WORKLOAD}[family]
    dim, n = wl["dim"], wl["n"]
    v, c = simplex_mesh(dim, n, jitter=0.2)
    coef = lognormal_coefficients(c.shape[0])
    t0 = time.perf_counter()
    if family is None:
        coeff = F.make_coeff("poisson", "fp64", source_kind=1, source=(1.0,), dim=dim)
        G = F.Simplex(dim, v, c, wl["k"], coeff, cell_coeff=coef)
    else:
        src = vector_source(family, wl["kappa"])
        coeff = F.make_coeff("poisson", "fp64", source_kind=2, source=src, dim=dim)
        G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=coef, family=family, kappa=wl["kappa"])
    t_setup = time.perf_counter() - t0
    ncells = c.shape[0]
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    print(f"[bench] simplex form ({family or 'lagrange'}): cells={ncells} rows={G.n_rows} nnz={G.nnz} "
          f"contributions={G.n_contrib} "
          f"set-up {t_setup:.1f} s", file=sys.stderr, flush=True)

    def step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        G.assemble(stream)
        e1.record(stream)
        x.zero_()
        return F.pcg_solve(G.csr, G.rhs, x, wl["rtol"], 200000, ws, stream), e0, e1

    for _ in range(warmup):
        step()
    F.set_timing(True)
    F.get_timing(reset=True)
    torch.cuda.synchronize()
    lat, iters, asm = [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        info, e0, e1 = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        iters.append(info["iters"])
        asm.append(e0.elapsed_time(e1) * 1e-3)
        print(f"[bench] simplex step {i}: {lat[-1] * 1e3:.1f} ms, {info['iters']} iterations", file=sys.stderr,
              flush=True)
    total = time.perf_counter() - t0
    tm = F.get_timing(reset=True)
    F.set_timing(False)
    spmv_s = tm["spmv_ms"] / max(tm["spmv_calls"], 1) * 1e-3
    sb = spmv_bytes(G.n_rows, G.nnz, "csr")
    mode, rpw, _ = F.spmv_plan_of(G.n_rows, G.nnz)
    t_asm = statistics.mean(asm)
    eb = simplex_element_bytes(ncells, G.ntri, G.nloc, len(v), dim)
    gb = simplex_gather_bytes(G.nnz, G.n_contrib)
    out = {
        "workload": wl["text"], "cells": ncells, "dofs": G.n_rows, "nnz": G.nnz, "contributions": G.n_contrib,
        "steps": steps, "elements_per_s": ncells * steps / total, "ms_per_step": total / steps * 1e3,
        "p50_ms": statistics.median(lat) * 1e3, "pcg_iters": statistics.mean(iters), "relres": info["relres"],
        "true_relres": info["true_relres"], "setup_s": t_setup,
        "assembly": {"ms": t_asm * 1e3, "elements_per_s": ncells / t_asm,
                     "algorithmic_bytes": {"element_kernel": eb, "value_gather": gb},
                     "hbm_frac_of_assembly_bytes": (eb + gb) / t_asm / 1e9 / HBM_PEAK_GBS,
                     "timing": "HIP events around fe_simplex_assemble (element kernel, value gather, rhs/dinv)"},
        "roofline_spmv": {"kernel": f"pcg_spmv_kernel/csr (plan mode {mode}, {rpw} rows per tile)", "bound": "hbm",
                          "achieved": sb / spmv_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": sb / spmv_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": sb,
                          "avg_launch_us": spmv_s * 1e6, "timed_launches": tm["spmv_calls"],
                          "bytes": "12 nnz + 8 (n + 1) + 16 n: values, column indices, row pointers, x once, y"},
    }
    del G, ws, x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle's simplex system on the host", file=sys.stderr, flush=True)
        if family is None:
            out["cpu_baseline"] = simplex_cpu_baseline(wl, statistics.mean(iters), ncells, out["nnz"])
        else:
            out["cpu_baseline"] = vector_cpu_baseline(wl, family, statistics.mean(iters), ncells, out["nnz"])
    return out


def vector_cpu_baseline(wl, family, gpu_iters, ncells_full, nnz_full, n=16, cg_its=100):
    """The oracle's vector-element system on the Kuhn mesh of an n^3 brick of
    the same recipe (numeric assembly single-threaded) and its all-cores CG,
    scaled to the full workload like the other baselines."""
    import oracle as O
    from fe_inputs import lognormal_coefficients, simplex_mesh
    v, c = simplex_mesh(wl["dim"], n, jitter=0.2)
    coef = lognormal_coefficients(c.shape[0])
    src = vector_source(family, wl["kappa"])
    S = O.VectorSystem(family, wl["dim"], v, c, coef=coef, kappa=wl["kappa"], source_kind=2, source=src)
    t_asm = S.t_assemble
    t0 = time.perf_counter()
    res = O.omp_pcg(S.rowptr, S.colind, S.values, S.rhs, 0.0, cg_its)
    t_it = (time.perf_counter() - t0) / max(res["iters"], 1)
    step = t_asm / c.shape[0] * ncells_full + t_it * (nnz_full / S.nnz) * gpu_iters
    return {"value": ncells_full / step, "unit": "elements/s", "cores": O.omp_threads(), "kind": "oracle",
            "sample": f"oracle (C, FP64) {family} system on the Kuhn mesh of {n}^3 ({c.shape[0]} tetrahedra, "
                      f"nnz {S.nnz}): numeric assembly single-threaded ({t_asm:.2f} s), {res['iters']} CG "
                      f"iterations on all cores ({t_it * 1e3:.2f} ms each); the full step scaled as cells x "
                      f"assembly time per cell + {gpu_iters:.0f} iterations x per-iteration time x nnz ratio",
            "step_s_scaled": step}


STOKES_WORKLOAD = dict(dim=3, n=24, k=1, mu=1.0, rtol=1e-8,
                       text="Taylor-Hood Stokes (Q2^3 velocity x Q1 pressure) on the unit cube, 24^3 hexes jittered "
                            "+-0.2h (seed 17080), mu = 1, f = 3 pi^2 prod sin(pi x_r) (1, -0.5, 0.25), u = 0 on the "
                            "boundary, FP64 assembly + block-Jacobi-preconditioned MINRES to rtol 1e-8")


def stokes_iteration_bytes(nu, np_, nnz_a, nnz_b):
    """Algorithmic bytes of one MINRES iteration: the A SpMV (pattern
    evaluated: 8 nnz + 16 n_u), the B^T and B SpMVs (CSR: 12 nnz + row
    pointers + x + y each), the B^T product added to A x (24 n_u), the dot
    product (16 n), the Lanczos update (48 n), the solution update (48 n) and
    the rescaling (32 n), n = n_u + n_p."""
    n = nu + np_
    spmv_b = 12 * nnz_b + 8 * (nu + 1) + 8 * np_ + 8 * nu + 12 * nnz_b + 8 * (np_ + 1) + 8 * nu + 8 * np_
    return 8 * nnz_a + 16 * nu + spmv_b + 24 * nu + (16 + 48 + 48 + 32) * n


def stokes_cpu_baseline(wl, gpu_iters, ncells_full, nnz_full, n=8, its=100):
    """The oracle's Stokes system on an n^3 mesh of the same recipe (its
    assembly, single-threaded) and MINRES on it (scipy's, the library
    routine, with the same block-diagonal preconditioner; a fixed number of
    iterations), scaled to the full workload like the other baselines."""
    import numpy as np
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import oracle as O
    from fe_inputs import structured_vertices
    v = structured_vertices(3, n, jitter=0.2)
    t0 = time.perf_counter()
    S = O.StokesSystem(3, [n] * 3, wl["k"], v, mu=wl["mu"], source_kind=2, source=(1.0, -0.5, 0.25))
    t_asm = time.perf_counter() - t0
    K = S.matrix()
    d = np.concatenate([1.0 / S.A.scipy().diagonal(), wl["mu"] / S.md])
    M = sp.diags(d)
    t0 = time.perf_counter()
    spla.minres(K, S.rhs(), M=M, maxiter=its, rtol=0.0)
    t_it = (time.perf_counter() - t0) / its
    step = t_asm / S.Pp.ncells * ncells_full + t_it * (nnz_full / K.nnz) * gpu_iters
    return {"value": 1.0 / step, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle Stokes system at {n}^3 Q{wl['k'] + 1}-Q{wl['k']} ({S.Pp.ncells} cells, nnz {K.nnz}): "
                      f"assembly single-threaded ({t_asm:.2f} s), {its} iterations of scipy's MINRES with the same "
                      f"preconditioner ({t_it * 1e3:.2f} ms each); the full solve scaled as cells x assembly time "
                      f"per cell + {gpu_iters:.0f} iterations x per-iteration time x nnz ratio",
            "step_s_scaled": step}


def stokes_form(args, F, torch, steps=3, warmup=1):
    """The Stokes workload: a step is the block assembly (velocity block,
    divergence blocks, gathers) + MINRES, set-up (spaces, patterns, gather
    maps) once before timing.  The MINRES iteration's roofline counts the
    bytes of all its kernels over its wall-clock time."""
    from fe_inputs import structured_vertices
    wl = STOKES_WORKLOAD
    dim, n, k = wl["dim"], wl["n"], wl["k"]
    v = structured_vertices(dim, n, jitter=0.2)
    mesh = F.create_mesh(dim, [n] * dim, v)
    t0 = time.perf_counter()
    S = F.Stokes(mesh, k, mu=wl["mu"], source_kind=2, source=(1.0, -0.5, 0.25))
    t_setup = time.perf_counter() - t0
    u = torch.zeros(S.n_u, dtype=torch.float64, device="cuda")
    p = torch.zeros(S.n_p, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    print(f"[bench] Stokes form: cells={n ** dim} velocity={S.n_u} pressure={S.n_p} nnz A={S.nnz_a} B={S.nnz_b}",
          file=sys.stderr, flush=True)

    def step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.assemble(stream)
        e1.record(stream)
        u.zero_()
        p.zero_()
        ts = time.perf_counter()
        info = S.solve(u, p, wl["rtol"], 20000, stream)
        return info, e0, e1, time.perf_counter() - ts

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, asm, solve_s, iters = [], [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        info, e0, e1, ds = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        asm.append(e0.elapsed_time(e1))
        solve_s.append(ds)
        iters.append(info["iters"])
        print(f"[bench] Stokes step {i}: {lat[-1] * 1e3:.1f} ms, {info['iters']} MINRES iterations", file=sys.stderr,
              flush=True)
    total = time.perf_counter() - t0
    assert F.get_status(mesh) == F.FE_OK
    it_s = statistics.mean(solve_s) / max(statistics.mean(iters), 1)
    ib = stokes_iteration_bytes(S.n_u, S.n_p, S.nnz_a, S.nnz_b)
    out = {
        "workload": wl["text"], "cells": n ** dim, "velocity_dofs": S.n_u, "pressure_dofs": S.n_p,
        "nnz_a": S.nnz_a, "nnz_b": S.nnz_b, "steps": steps, "solves_per_s": steps / total,
        "ms_per_step": total / steps * 1e3, "minres_iters": statistics.mean(iters), "relres": info["relres"],
        "true_relres": info["true_relres"], "setup_s": t_setup,
        "assembly_ms": statistics.mean(asm),
        "roofline_minres_iteration": {"kernels": "A SpMV (evaluated pattern), B and B^T SpMVs (CSR), vector kernels",
                                      "bound": "hbm", "achieved": ib / it_s / 1e9, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": ib / it_s / 1e9 / HBM_PEAK_GBS,
                                      "algorithmic_bytes_per_iteration": ib, "avg_iteration_us": it_s * 1e6,
                                      "timing": "wall clock of the solve over its iterations (scalars on the "
                                                "device; the host reads a control word per 8 iterations)"},
    }
    del S, u, p
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle's Stokes system on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = stokes_cpu_baseline(wl, statistics.mean(iters), n ** dim, out["nnz_a"] + 2 * out["nnz_b"])
    return out


def peak_probe(torch):
    """Achievable rates of this GPU, measured, to set the published peaks the
    roofline uses in context: a 1 GiB device copy and a 4 GiB read (a sum) in
    GB/s, and library GEMMs (torch.matmul, 8192^3 in FP64 and FP32, 16384^3 in
    BF16) in TFLOP/s.  Median of 5 timed runs after 2 warm-ups, HIP events."""
    def timed(fn, reps=5):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return sorted(ts)[len(ts) // 2]
    out = {}
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out["copy_GBps"] = 2 * a.numel() * 8 / timed(lambda: b.copy_(a)) / 1e9
    del a, b
    r = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
    out["read_GBps"] = r.numel() * 8 / timed(lambda: r.sum()) / 1e9
    del r
    for name, dt, m in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192), ("bf16", torch.bfloat16, 16384)):
        x = torch.rand(m, m, dtype=dt, device="cuda")
        y = torch.rand(m, m, dtype=dt, device="cuda")
        out[f"gemm_{name}_TFLOPs"] = 2 * m ** 3 / timed(lambda: torch.matmul(x, y)) / 1e12
        del x, y
    torch.cuda.empty_cache()
    out["published"] = {"hbm_GBps": 8000, "fp64_matrix_TFLOPs": 78.6, "fp32_TFLOPs": 157.3, "bf16_matrix_TFLOPs": 2500}
    return out


def batch_form(args, F, torch):
    """Batching form: a sample of the 512-problem batch (3D Poisson, n uniform
    in [8, 64], order uniform in {1, 2, 3}) with FP32 element integration and
    FP64 solves by iterative refinement (FP64 residuals with each problem's
    FP64 system, inner Jacobi-PCG on the FP32-integrated one), run as batched
    waves, against the same problems refined one by one (results must be
    bitwise equal) and against the plain FP64 path one by one (the distance of
    the refined solutions to the FP64 ones)."""
    from fe_inputs import batch_specs
    from paper_1708_01773_amd import batch as BT

    rtol, maxit = 1e-10, 100000
    specs = batch_specs(512)
    sample = specs[: args.batch_sample]
    run = BT.BatchRun(sample, precision="fp32", budget=int(args.batch_budget_gb * (1 << 30)))
    print(f"[bench] batch form: {len(sample)} problems, {len(run.waves)} wave(s), "
          f"{sum(run.nnz) / 1e9:.2f} G nnz", file=sys.stderr, flush=True)
    tuned = run.autotune()
    print("[bench] batch form: autotuned " + ", ".join(
        f"class {c}: mode {t['chosen']['mode']} rpw {t['chosen']['rows_per_wave']}" for c, t in tuned.items()),
        file=sys.stderr, flush=True)
    ref64, ref32 = {}, {}
    if args.batch_no_sequential:
        seq64 = seq32 = None
    else:
        seq64 = BT.run_sequential([BT.make_problem(i, n, k, "fp64") for i, (n, k) in enumerate(sample)], rtol, maxit,
                                  keep=lambda i, x: ref64.__setitem__(i, x.clone()))
        print(f"[bench] batch form: sequential FP64 {seq64['assemble_s'] + seq64['solve_s']:.2f} s", file=sys.stderr,
              flush=True)
        seq32 = BT.run_sequential(run.problems, rtol, maxit, keep=lambda i, x: ref32.__setitem__(i, x.clone()),
                                  coeffs_hi=run.coeffs_hi)
        print(f"[bench] batch form: sequential refined {seq32['assemble_s'] + seq32['solve_s']:.2f} s",
              file=sys.stderr, flush=True)
    same = [True]
    err = [0.0]

    def keep(i, x):
        if seq32 is None:
            return
        same[0] = same[0] and torch.equal(x, ref32[i])
        r = ref64[i]
        if r.numel():
            err[0] = max(err[0], (torch.linalg.vector_norm(x - r) / torch.linalg.vector_norm(r)).item())

    res = run.run(rtol, maxit, keep=keep, progress=lambda w, nw, ta, ts: print(
        f"[bench] batch form: wave {w + 1}/{nw} assembled in {ta:.2f} s, solved in {ts:.2f} s", file=sys.stderr,
        flush=True))
    t_b = res["assemble_s"] + res["solve_s"]
    t_s = seq32["assemble_s"] + seq32["solve_s"] if seq32 else None
    print(f"[bench] batch form: batched {t_b:.2f} s (set-up {res['setup_s']:.2f} s)", file=sys.stderr, flush=True)
    iters = [i["inner_iters"] for i in res["infos"]]
    outer = [i["outer_iters"] for i in res["infos"]]
    return {
        "sample": f"first {len(sample)} of the 512 problems drawn with seed 17082 (n uniform in [8, 64], order "
                  f"uniform in 1..3); per-problem seeds 17080/17081 + 1000 (i + 1)",
        "problems": len(sample), "cells": run.cells, "dofs": sum(run.n_rows), "nnz": sum(run.nnz),
        "waves": len(run.waves), "budget_gb": args.batch_budget_gb, "integration": "fp32",
        "solve": "fp64 iterative refinement (FP64 residual with the FP64-integrated system, inner Jacobi-PCG on the "
                 "FP32-integrated one to 1e-4)",
        "rtol": rtol, "status_ok": res["status"] == F.FE_OK, "inner_iters_min": min(iters),
        "inner_iters_max": max(iters), "outer_iters_max": max(outer),
        "batched": {"s": t_b, "assemble_s": res["assemble_s"], "solve_s": res["solve_s"],
                    "setup_s": res["setup_s"], "problems_per_s": len(sample) / t_b,
                    "elements_per_s": run.cells / t_b},
        "sequential_same_precision": {"s": t_s, "assemble_s": seq32["assemble_s"], "solve_s": seq32["solve_s"],
                                      "problems_per_s": len(sample) / t_s} if seq32 else None,
        "sequential_plain_fp64": {"s": seq64["assemble_s"] + seq64["solve_s"]} if seq64 else None,
        "speedup_vs_sequential": t_s / t_b if t_s else None,
        "bitwise_equal_to_sequential": bool(same[0]) if seq32 else None,
        "max_rel_error_vs_plain_fp64_solution": err[0] if seq64 else None,
        "waves_detail": [{"problems": len(w), "bytes": sum(run.sizes[i] for i in w)} for w in run.waves],
        "autotuned_spmv": {f"order {t['matrix']['order']}": {
            "mode": t["chosen"]["mode"], "rows_per_wave": t["chosen"]["rows_per_wave"], "us": t["chosen"]["us"],
            "tried_us": [round(x["us"], 2) for x in t["tried"]]} for c, t in tuned.items()},
    }


def serve_form(args, F, torch):
    """Serving form: the first --serve-requests requests of the seeded
    Poisson-process stream (3D Poisson, n log-uniform in [8, 96], order uniform
    in 1..4, rtol 1e-8), every drawn request submitted to the library's server
    (a budget near the HBM size; only the server's own admission refuses a
    request, at submission, if it needs more than the whole budget).  Rate 0:
    every request arrives at once (the saturated throughput is the capacity).
    --serve-max-dofs thins the stream to requests of at most that many
    unknowns (not by default).  Three requests are re-run alone through the
    plain path and compared bitwise with their result in the mix."""
    from fe_inputs import serving_requests
    from paper_1708_01773_amd import serve as SV

    rtol, maxit = 1e-8, 200000
    drawn = serving_requests(2000, args.serve_rate if args.serve_rate > 0 else 1.0)
    cap = args.serve_max_dofs
    kept = [(t if args.serve_rate > 0 else 0.0, n, k, i) for i, (t, n, k) in enumerate(drawn)
            if cap is None or (n * k - 1) ** 3 <= cap]
    kept = kept[: args.serve_requests]
    torch.cuda.empty_cache()
    t_first = kept[0][0]
    span = kept[-1][0] - t_first
    stream = [(t - t_first, n, k, i) for (t, n, k, i) in kept]
    print(f"[bench] serving form: {len(stream)} requests over {span:.2f} s of arrivals", file=sys.stderr, flush=True)
    srv = F.Server(int(args.serve_budget_gb * (1 << 30)), max_active=args.serve_slots)
    probes = {}
    # probes: the smallest, the median and the largest request of at most 5e6 unknowns
    order = sorted((j for j in range(len(stream)) if (stream[j][1] * stream[j][2] - 1) ** 3 <= 5e6),
                   key=lambda j: (stream[j][1] * stream[j][2]) ** 3)
    for j in (order[0], order[len(order) // 2], order[-1]):
        probes[j] = None

    def keep(j, ticket, r):
        if j in probes and r["state"] == F.FE_REQ_DONE:
            x = torch.empty(r["n_rows"], dtype=torch.float64, device="cuda")
            srv.solution(ticket, x)
            probes[j] = x

    results, makespan = SV.run_stream(srv, stream, rtol=rtol, maxit=maxit, on_done=keep, progress=1,
                                      timeout=3000.0)
    stats = srv.stats()
    srv.close()
    summary = SV.summarize(results, makespan)
    failed = [{"request": stream[j][3], "n": stream[j][1], "k": stream[j][2], "state": r["state"],
               "status": r.get("status"), "iters": r.get("iters"), "relres": r.get("relres"), "error": r["error"]}
              for j, r in enumerate(results) if not (r["state"] == F.FE_REQ_DONE and r["status"] == F.FE_OK)]
    same = True
    for j, x_mix in probes.items():
        _, n, k, i = stream[j]
        a = SV.request_inputs(i, n, k)
        mesh = F.create_mesh(3, a["n"], a["vertices"], a["cell_coeff"])
        A = F.Assembly(mesh, k, a["coeff"])
        A.pattern()
        A.assemble()
        x = torch.zeros(max(A.n_rows, 1), dtype=torch.float64, device="cuda")
        ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
        A.solve(x, rtol, maxit, ws)
        torch.cuda.synchronize()
        same = same and x_mix is not None and torch.equal(x[: A.n_rows], x_mix)
        del A, mesh, x, ws
    print(f"[bench] serving form: {summary['solves_per_s']:.1f} solves/s, p50 {summary['p50_ms']:.1f} ms, "
          f"p99 {summary['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    return {
        "sample": (f"first {len(stream)} requests of the stream drawn with seed 17083 " +
                   (f"at {args.serve_rate}/s" if args.serve_rate > 0 else "arriving at once") +
                   " (n log-uniform in [8, 96], order uniform in 1..4), every request submitted" +
                   ("" if cap is None else f"; thinned to at most {cap} unknowns ({len(stream)} of "
                                           f"{kept[-1][3] + 1} drawn)")),
        "largest_request_dofs": max((n * k - 1) ** 3 for _, n, k, _ in stream),
        "arrival_rate_per_s": (len(stream) - 1) / span if span > 0 else None,
        "rtol": rtol, "budget_gb": args.serve_budget_gb, "max_active": args.serve_slots, **summary,
        "peak_in_flight": stats["peak_solving"], "peak_bytes": stats["peak_in_use"],
        "admission_waits": stats["admission_waits"], "chunks": stats["chunks"],
        "bitwise_equal_alone_vs_mix": bool(same), "checked_alone": len(probes),
        "not_converged": failed[:20],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=None, help="override cells per axis (development)")
    ap.add_argument("--k", type=int, default=None, help="override the order (development)")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "fp16", "bf16"],
                    help="element-GEMM precision (the solve stays FP64)")
    ap.add_argument("--no-forms", action="store_true", help="skip the mixed-precision form measurement")
    ap.add_argument("--phase", default="step", choices=["step", "assemble"],
                    help="step = assemble + PCG (default); assemble = assembly only, K3 against the matrix-core peak")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3D elasticity Q2-Q4 assembly figures")
    ap.add_argument("--spmv", default="sym", choices=["sym", "mesh", "csr"],
                    help="sym: Q1 scalar systems in symmetric storage, filled from the assembled CSR inside the "
                         "step (fe_sym_from_csr + fe_pcg_solve_sym; other spaces fall back to mesh); mesh: pattern "
                         "evaluated from the mesh (fe_pcg_solve_mesh); csr: row pointers and column indices read "
                         "(fe_pcg_solve)")
    ap.add_argument("--batch-sample", type=int, default=16,
                    help="problems of the 512-problem batch run by the batching form (0 = skip)")
    ap.add_argument("--batch-budget-gb", type=float, default=160.0, help="device memory per batch wave")
    ap.add_argument("--batch-no-sequential", action="store_true",
                    help="batching form: skip the one-by-one comparison runs (for the full 512-problem batch)")
    ap.add_argument("--serve-requests", type=int, default=12, help="requests of the serving form (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=0.15,
                    help="arrival rate of the drawn stream (1/s); 0 = every request at once")
    ap.add_argument("--serve-max-dofs", type=int, default=None,
                    help="thin the stream to requests of at most this many unknowns (default: every request)")
    ap.add_argument("--serve-budget-gb", type=float, default=256.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--form", default=None,
                    choices=["batch", "serve", "precision", "dg", "stokes", "simplex", "nedelec", "nedelec2",
                             "raviart_thomas2"],
                    help="run only this form and print its JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device 3 times (calibrates the HBM byte counters)")
    ap.add_argument("--peak-probe", action="store_true",
                    help="only measure this GPU's achievable rates (copy, read, library GEMMs) for context")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path would shard by "
              f"cells, each GPU owning its rows with one layer of ghost cells, and exchange a halo of p and two "
              f"scalars per CG iteration)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_launch": a.numel() * 8, "launches": 3}))
        return

    if args.peak_probe:
        print(json.dumps(peak_probe(torch)), flush=True)
        return

    from fe_inputs import lognormal_coefficients, structured_vertices
    from paper_1708_01773_amd import fe as F

    if args.form == "batch":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "batch", **batch_form(args, F, torch)}), flush=True)
        return
    if args.form == "serve":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "serve", **serve_form(args, F, torch)}), flush=True)
        return
    if args.form == "simplex":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "simplex", **simplex_form(args, F, torch)}), flush=True)
        return
    if args.form == "nedelec":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "nedelec", **simplex_form(args, F, torch, family="nedelec")}), flush=True)
        return
    if args.form == "raviart_thomas2":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "raviart_thomas2",
                          **simplex_form(args, F, torch, steps=2, warmup=1, family="raviart_thomas2")}), flush=True)
        return
    if args.form == "nedelec2":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "nedelec2", **simplex_form(args, F, torch, steps=2, warmup=1, family="nedelec2")}),
              flush=True)
        return
    if args.form == "stokes":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "stokes", **stokes_form(args, F, torch)}), flush=True)
        return
    if args.form == "dg":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "dg", **dg_form(args, F, torch)}), flush=True)
        return
    if args.form == "precision":
        torch.cuda.set_device(0)
        print(json.dumps({"form": "precision_c3", **c3_precision(F, torch)}), flush=True)
        return

    wl = dict(WORKLOADS[args.workload])
    if args.n:
        wl["n"] = args.n
    if args.k:
        wl["k"] = args.k
    if args.precision:
        wl["precision"] = args.precision
    dim, n, k = wl["dim"], wl["n"], wl["k"]
    torch.cuda.set_device(0)
    v = structured_vertices(dim, n, jitter=wl.get("jitter", 0.2))
    ncells = n ** dim
    coef = lognormal_coefficients(ncells) if wl.get("lognormal", True) else None
    mesh = F.create_mesh(dim, [n] * dim, v, coef)
    src = (0.0, 0.0, -1.0) if wl["problem"] == "elasticity" else (1.0,)
    coeff = F.make_coeff(wl["problem"], wl["precision"], source_kind=wl.get("source_kind", 1), source=src, dim=dim)
    A = F.Assembly(mesh, k, coeff)
    A.pattern()
    if args.spmv == "sym" and not (k == 1 and wl["problem"] == "poisson"):
        args.spmv = "mesh"
    sym = None
    if args.spmv == "sym" and args.phase == "step":
        sym = torch.empty(F.sym_query(mesh, k, coeff) // 8, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    print(f"[bench] set-up done: cells={ncells} rows={A.n_rows} nnz={A.nnz}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    if args.phase == "assemble":
        return assemble_only(args, wl, A, ncells, F, torch)

    def step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        A.assemble(stream)
        e1.record(stream)
        if sym is not None:
            F.sym_from_csr(mesh, k, coeff, A.csr, sym, stream)
        e2.record(stream)
        x.zero_()
        if sym is not None:
            info = F.pcg_solve_sym(mesh, k, coeff, A.csr, sym, A.rhs, x, wl["rtol"], 100000, ws, stream)
        elif args.spmv == "mesh":
            info = A.solve(x, wl["rtol"], 100000, ws, stream)
        else:
            info = F.pcg_solve(A.csr, A.rhs, x, wl["rtol"], 100000, ws, stream)
        return info, e0, e1, e2

    for i in range(args.warmup):
        info, _, _, _ = step()
        print(f"[bench] warmup {i}: iters={info['iters']} relres={info['relres']:.2e}", file=sys.stderr, flush=True)
    F.set_timing(True)
    F.get_timing(reset=True)
    torch.cuda.synchronize()
    lat, asm_ms, fill_ms, iters = [], [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        info, e0, e1, e2 = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        asm_ms.append(e0.elapsed_time(e1))
        fill_ms.append(e1.elapsed_time(e2))
        iters.append(info["iters"])
        if info["status"] != F.FE_OK:
            print(f"[bench] step {i}: solver status {info['status']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    tm = F.get_timing(reset=True)
    F.set_timing(False)
    print(f"[bench] timed {args.steps} steps in {total:.3f} s", file=sys.stderr, flush=True)

    ms_step = total / args.steps * 1e3
    spmv_avg_s = tm["spmv_ms"] / max(tm["spmv_calls"], 1) * 1e-3
    sb = spmv_bytes(A.n_rows, A.nnz, args.spmv)
    achieved = sb / spmv_avg_s / 1e9 if spmv_avg_s > 0 else 0.0
    kname = "pcg_spmv_kernel/" + args.spmv
    traffic = traffic_for(kname, args.workload)
    lat_sorted = sorted(lat)
    p99 = lat_sorted[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]
    out = {
        "metric": METRIC,
        "value": ncells * args.steps / total,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["text"], "cells": ncells, "order": k, "dofs": A.n_rows, "nnz": A.nnz,
                   "operator_storage": {"sym": "symmetric (upper triangle)", "mesh": "CSR values",
                                        "csr": "CSR"}[args.spmv]},
        "assembly": {"ms_mean": statistics.mean(asm_ms), "ms_median": statistics.median(asm_ms),
                     "ms_min": min(asm_ms),
                     "elements_per_s": ncells / (statistics.mean(asm_ms) * 1e-3),
                     "integrate_ms": tm["integrate_ms"] / max(tm["integrate_calls"], 1),
                     "scatter_ms": tm["scatter_ms"] / max(tm["scatter_calls"], 1),
                     "sym_fill_ms": statistics.mean(fill_ms) if sym is not None else None},
        "solve": {"pcg_iters": statistics.mean(iters), "relres": info["relres"],
                  "true_relres": info["true_relres"], "solves_per_s": args.steps / total,
                  "p50_ms": statistics.median(lat) * 1e3, "p99_ms": p99 * 1e3, "min_ms": min(lat) * 1e3,
                  "kappa_est": info["lambda_max_est"] / info["lambda_min_est"] if info["lambda_min_est"] else None},
        "roofline": {"kernel": kname, "traversal": {
                         "sym": "symmetric storage (upper triangle, slot-major), pattern evaluated from the mesh",
                         "mesh": "CSR values, pattern evaluated from the mesh",
                         "csr": "CSR row pointers and column indices read"}[args.spmv], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": sb, "avg_launch_us": spmv_avg_s * 1e6,
                     "timed_launches": tm["spmv_calls"],
                     "timing": "HIP events around the SpMV launch of every 16th CG iteration of the timed steps"},
    }
    if args.workload == "c2" and wl["precision"] == "fp64":
        out["roofline_csr"] = csr_roofline(A, F, torch, stream)
        print(f"[bench] CSR SpMV {out['roofline_csr']['avg_launch_us']:.1f} us "
              f"({out['roofline_csr']['frac']:.3f} of HBM)", file=sys.stderr, flush=True)
    forms = not args.no_forms and wl["precision"] == "fp64"
    if forms:
        print("[bench] mixed-precision form", file=sys.stderr, flush=True)
        out["forms"] = {"mixed_refine": mixed_form(args, wl, mesh, A, x, F, torch, stream, ncells)}
    del A, ws, x, sym
    torch.cuda.empty_cache()
    if args.workload == "c2" and not args.no_c3:
        out["c3_assembly"] = c3_assembly(F, torch)
        if forms:
            out["forms"]["precision_c3"] = c3_precision(F, torch, orders=("c3q2", "c3q4"))
    if forms and args.workload == "c2":
        if args.batch_sample > 0:
            out["forms"]["batch"] = batch_form(args, F, torch)
        if args.serve_requests > 0:
            out["forms"]["serve"] = serve_form(args, F, torch)
        print("[bench] DG form", file=sys.stderr, flush=True)
        out["forms"]["dg"] = dg_form(args, F, torch)
        print("[bench] Stokes form", file=sys.stderr, flush=True)
        out["forms"]["stokes"] = stokes_form(args, F, torch)
        print("[bench] simplex form", file=sys.stderr, flush=True)
        out["forms"]["simplex"] = simplex_form(args, F, torch)
        print("[bench] Nedelec form", file=sys.stderr, flush=True)
        out["forms"]["nedelec"] = simplex_form(args, F, torch, family="nedelec")
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, statistics.mean(iters), ncells, out["config"]["nnz"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
