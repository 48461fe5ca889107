"""Benchmark of the matrix-free finite-strain tangent on one MI355X.

Headline workload: 3-D unit cube, 32^3 Q2 cells (823,875 DoFs), (p+1)^3 Gauss
points, compressible Neo-Hookean matrix (mu = 1, nu = 0.3) with 20 seeded
spheres 100x stiffer, seeded smooth displacement of amplitude 0.1, x ~ N(0,1).
A step is one tangent vmult (gather -> sum factorisation -> quadrature-point
stage -> transposed sum factorisation -> scatter in the mode the tuned table
picks: for this workload the cell kernel writes an element buffer and a
node-sum kernel adds it into y) with the inputs resident in HBM.  Every
quadrature-point policy is timed in FP64 and FP32; the best FP64 one is the
headline value.  The roofline object covers the kernels of one vmult of the
headline variant (both kernels of the ELEMENT scatter), timed with HIP events
on the library's stream around the timed steps, plus per-call warm and cold
(cache-flushed) timings.  Further parts: the 64^3 Q2 Newton benchmark (mixed
against all-FP64 GMG-CG), the 256-problem batch, the matrix-based (CSR)
comparison, the Q4 48^3 level vmults and Newton loadings (with a wall-time
budget each), and cpu_baseline, the oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-q4] ...
"""
import argparse
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tangent vmult DoFs/s (FP64/FP32, Q2 3D); GMG-CG Newton-step time at 1e-8"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
POLICIES = {0: "recompute", 1: "cache_F", 2: "cache_T2", 3: "cache_T4"}

# Algorithmic flop counts: minimal sum factorisation of one d-component field,
# 4 d^2 n^(d+1), plus the per-quadrature-point algebra.  Measured HBM bytes per
# vmult of the 32^3 Q2 workload (cell kernel + node-sum kernel of the ELEMENT scatter) from
# rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a 256 MiB device copy (reads
# x2.0, writes x1.0; profiles/tangent_vmult_q2_32cube_hbm_counters.md); valid
# only for the kernel source they were taken on.
TRAFFIC_SOURCE_SHA = "100930e8fd80cb5a"
TRAFFIC = {"recompute/f64/element": 58784664, "cache_F/f64/element": 116125656,
           "cache_T2/f64/element": 123012254, "cache_T4/f64/element": 348807387,
           "recompute/f32/element": 32022950, "cache_F/f32/element": 60365742,
           "cache_T2/f32/element": 63739593, "cache_T4/f32/element": 173464575}

QP_FLOPS_3D = {0: 261, 1: 255, 2: 170, 3: 246}
QP_FLOPS_2D = {0: 100, 1: 98, 2: 55, 3: 71}
CACHE_WORDS = {3: {0: 0, 1: 9, 2: 10, 3: 36}, 2: {0: 0, 1: 4, 2: 5, 3: 13}}


def algorithmic_cost(dim, degree, n_cells, n_dofs, policy, word):
    n = degree + 1
    ncells = n_cells ** dim
    nq = n ** dim
    fields = 3 if policy == 0 else 2      # forward x (+ forward u), backward
    sf = 4 * dim * dim * n ** (dim + 1)
    qpf = (QP_FLOPS_3D if dim == 3 else QP_FLOPS_2D)[policy]
    flops = ncells * (fields * sf + nq * qpf)
    nbytes = 2 * word * n_dofs                        # x read once, y written once
    if policy == 0:
        nbytes += 8 * n_dofs if word == 8 else 4 * n_dofs   # displacement
    nbytes += CACHE_WORDS[dim][policy] * nq * ncells * word
    nbytes += 4 * ncells * ((nq + 31) // 32)          # material bits
    return flops, nbytes


def measured_traffic(policy, dtype, scatter):
    import hashlib
    src = os.path.join(ROOT, "paper_1904_13131_amd", "csrc", "cellops.hpp")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if sha != TRAFFIC_SOURCE_SHA:
        return None
    return TRAFFIC.get(f"{POLICIES[policy]}/{dtype}/{scatter}")


def roofline(dim, degree, n_cells, n_dofs, policy, dtype, kernel_ms, scatter):
    word = 8 if dtype == "f64" else 4
    traffic = measured_traffic(policy, dtype, scatter)
    flops, nbytes = algorithmic_cost(dim, degree, n_cells, n_dofs, policy, word)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (PEAK_TFLOPS[dtype] * 1e12)
    s = kernel_ms * 1e-3
    timed = {"element": "cell kernel k_tangent + node-sum kernel k_elem_gather of each vmult (ELEMENT scatter)",
             "atomic": "output fill + cell kernel k_tangent of each vmult (atomic scatter)",
             "tile": "output fill + tile kernel k_tangent_tile of each vmult",
             "color": "output fill + the 2^d colour launches of k_tangent of each vmult"}[scatter]
    timed += ": HIP events on the library's stream around the timed steps, divided by the steps"
    if t_hbm >= t_alu:
        ach = nbytes / s / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": traffic, "alg_bytes": nbytes, "alg_flops": flops, "timed": timed}
    ach = flops / s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": ach / PEAK_TFLOPS[dtype], "traffic": traffic, "alg_bytes": nbytes, "alg_flops": flops,
            "timed": timed}


def time_vmult(P, x, y, steps, warmup, cold=False, flush=None):
    """(ms per step, per-call ms list).  The steps run back to back with one
    HIP event pair on the library's stream around all of them (the step time);
    a second pass brackets every call with its own event pair (per-call
    durations for the median and minimum; a pair costs a few microseconds, so
    it stays out of the step time).  cold: a 512 MB buffer is read (summed)
    before every call, which evicts the working set from the caches; a
    rewritten buffer would also leave dirty lines whose write-back the timed
    call would pay."""
    import torch
    for _ in range(warmup):
        P.tangent_vmult(x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(P.stream)
    for _ in range(steps):
        if cold:
            flush.sum()
        P.tangent_vmult(x, y)
    e1.record(P.stream)
    torch.cuda.synchronize()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for b, e in pairs:
        if cold:
            flush.sum()
        b.record(P.stream)
        P.tangent_vmult(x, y)
        e.record(P.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, [b.elapsed_time(e) for b, e in pairs]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed(fn, seconds):
    fn()
    n, t0 = 0, time.perf_counter()
    while True:
        fn()
        n += 1
        wall = time.perf_counter() - t0
        if wall >= seconds:
            return wall / n


def cpu_baseline(w, sample_cells=16, spmv_seconds=4.0, ebe_cells=4096):
    """The oracle on the host cores: its assembled FP64 tangent (CSR) of the
    same recipe at 16^3 Q2 cells (the largest size it assembles in seconds),
    applied by SciPy on one core and by the oracle's OpenMP CSR SpMV on all
    cores; the assembly time; and, for reference, the oracle's
    element-by-element apply (element matrices re-formed on every apply)."""
    import workloads as W
    from oracle import fe
    from oracle import spmv as ospmv
    ws = W.cube_spheres_q2(sample_cells)
    mesh = fe.Mesh(ws["dim"], ws["n_cells"], ws["degree"])
    mat = fe.Material(ws["mu"], ws["lam"], ws["inclusions"])
    t0 = time.perf_counter()
    K = fe.tangent_matrix(mesh, mat, ws["u"])
    t_asm = time.perf_counter() - t0
    x = ws["x"]
    t_scipy = _timed(lambda: K @ x, spmv_seconds)
    csr = ospmv.prepare(K)
    y = np.empty(mesh.n_dofs)
    t_omp = _timed(lambda: ospmv.spmv(csr, x, y), spmv_seconds)
    threads = ospmv.threads()
    # element-by-element apply over a sample of the full-size cells
    full = fe.Mesh(w["dim"], w["n_cells"], w["degree"])
    fmat = fe.Material(w["mu"], w["lam"], w["inclusions"])
    cells = np.sort(np.random.default_rng(0).choice(full.n_cells, ebe_cells, replace=False))
    t0 = time.perf_counter()
    fe.vmult_ebe(full, fmat, w["u"], w["x"], cells=cells)
    t_ebe = time.perf_counter() - t0
    n = mesh.n_dofs
    return {"value": n / t_omp, "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle FP64 tangent of the same recipe at {sample_cells}^3 Q2 ({n:,} DoFs, {K.nnz:,} nnz) "
                      f"assembled in {t_asm:.1f} s, applied as CSR SpMV by the oracle's OpenMP kernel on "
                      f"{threads} threads ({t_omp * 1e3:.2f} ms per product, {spmv_seconds:.0f} s timed)",
            "scipy_csr_1core_dofs_per_s": n / t_scipy,
            "assembly_s": round(t_asm, 2),
            "element_by_element_1core_dofs_per_s": full.n_dofs * ebe_cells / full.n_cells / t_ebe,
            "element_by_element_note": f"oracle element-by-element apply (element matrices formed on every "
                                       f"apply) on {ebe_cells} of {full.n_cells} cells of the full mesh, "
                                       f"scaled to its DoFs",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def law_bench(w, steps, warmup):
    """The tensor4 policy with the Mooney-Rivlin law on the headline workload
    (same mesh, inclusions and fields; moduli with the same small-strain Lame
    pair): the operator does not evaluate the law, so the vmult costs what the
    Neo-Hookean cache_T4 variant costs."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import LAW_MOONEY_RIVLIN, QP_CACHE_T4, Problem
    from paper_1904_13131_amd.mfh import SCATTER_NAMES
    mu, lam, mu2 = W.two_phase_mooney_rivlin()
    P = Problem(w["dim"], w["n_cells"], w["degree"], mu=tuple(mu), lam=tuple(lam), mu2=tuple(mu2),
                law=LAW_MOONEY_RIVLIN, qp_policy=QP_CACHE_T4, inclusions=w["inclusions"])
    P.set_deformation(torch.as_tensor(w["u"], device="cuda"))
    out = {}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        x = torch.as_tensor(w["x"], device="cuda").to(tdt)
        y = torch.empty_like(x)
        ms, calls = time_vmult(P, x, y, steps, warmup)
        out[dt] = {"ms_per_step": ms, "call_ms_median": float(np.median(calls)), "dofs_per_s": P.n_dofs() / (ms * 1e-3),
                   "scatter": SCATTER_NAMES[P.scatter_mode(-1, 0 if dt == "f64" else 1)]}
        print(f"[bench] cache_T4 Mooney-Rivlin {dt}: {ms * 1e3:8.1f} us/vmult", file=sys.stderr, flush=True)
    return out


MB_CASES = ((1, 64), (2, 32), (3, 21), (4, 16))   # (degree, cells per direction): 0.79-0.82 M DoFs


def _time_ms(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def matrix_based_bench(steps=20, warmup=3, library_spmv=True):
    """Matrix-free vmult against the matrix-based operator (K_c assembled in
    CSR, one SpMV per step) for Q1-Q4 at about 0.8 M DoFs, with the memory
    each needs per DoF."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import Problem
    out = []
    for deg, nc in MB_CASES:
        w = W.problem(3, nc, deg, n_spheres=20, sphere_seed=3, u_seed=4, u_amp=0.1, u_kmax=1, x_seed=5)
        u = torch.as_tensor(w["u"], device="cuda")
        x = torch.as_tensor(w["x"], device="cuda")
        y = torch.empty_like(x)
        row = {"degree": deg, "cells": nc ** 3}
        for pol in (0, 2, 3):
            P = Problem(3, nc, deg, mu=tuple(w["mu"]), lam=tuple(w["lam"]), inclusions=w["inclusions"],
                        qp_policy=pol)
            P.set_deformation(u)
            n = P.n_dofs()
            ms = _time_ms(lambda: P.tangent_vmult(x, y), steps, warmup)
            nq = (deg + 1) ** 3
            mem = 8 * n + CACHE_WORDS[3][pol] * nq * nc ** 3 * 8 + 4 * nc ** 3 * ((nq + 31) // 32)
            row[f"mf_{POLICIES[pol]}"] = {"ms": ms, "dofs_per_s": n / (ms * 1e-3), "bytes_per_dof": mem / n}
            if pol == 0:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                csr = P.csr_assemble()
                t_asm = time.perf_counter() - t0
                rows, nnz = P.csr_size()
                yc = torch.empty_like(x)
                ms_c = _time_ms(lambda: P.csr_spmv(csr, x, yc), steps, warmup)
                ref = P.tangent_vmult(x)
                err = float((yc - ref).norm() / ref.norm())
                nbytes = 12 * nnz + 8 * (rows + 1) + 16 * rows
                row["n_dofs"] = n
                row["csr"] = {"ms": ms_c, "dofs_per_s": n / (ms_c * 1e-3), "nnz": nnz,
                              "nnz_per_row": nnz / rows, "bytes_per_dof": (12 * nnz + 8 * (rows + 1)) / n,
                              "assembly_s": t_asm, "alg_bytes": nbytes,
                              "achieved_gbs": nbytes / (ms_c * 1e-3) / 1e9,
                              "frac_hbm": nbytes / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "hbm_bound_ms": nbytes / (HBM_PEAK_GBS * 1e9) * 1e3, "rel_err_vs_mf": err}
                if library_spmv:
                    try:
                        A = torch.sparse_csr_tensor(csr[0], csr[1].long(), csr[2], (rows, rows))
                        ms_l = _time_ms(lambda: torch.mv(A, x), steps, warmup)
                        err_l = float((torch.mv(A, x) - ref).norm() / ref.norm())
                        row["csr_torch_sparse"] = {"ms": ms_l, "rel_err_vs_mf": err_l}
                        del A
                    except RuntimeError as e:
                        row["csr_torch_sparse"] = {"error": str(e)[:200]}
                del csr
            del P
            torch.cuda.empty_cache()
        mf_best = min(row["mf_recompute"]["ms"], row["mf_cache_T2"]["ms"])
        row["mf_speedup_vs_csr"] = row["csr"]["ms"] / mf_best
        row["mf_speedup_vs_csr_at_hbm_peak"] = row["csr"]["hbm_bound_ms"] / mf_best
        print(f"[bench] matrix-based Q{deg} {nc}^3: CSR {row['csr']['ms'] * 1e3:.1f} us "
              f"({row['csr']['bytes_per_dof']:.0f} B/DoF, {row['csr']['achieved_gbs']:.0f} GB/s), MF recompute "
              f"{row['mf_recompute']['ms'] * 1e3:.1f} us, MF cache_T2 {row['mf_cache_T2']['ms'] * 1e3:.1f} us "
              f"({row['mf_cache_T2']['bytes_per_dof']:.0f} B/DoF), MF cache_T4 {row['mf_cache_T4']['ms'] * 1e3:.1f} us "
              f"({row['mf_cache_T4']['bytes_per_dof']:.0f} B/DoF)", file=sys.stderr, flush=True)
        out.append(row)
    return out


def cpu_newton_baseline(w, n_cells=8, n_levels=3, stretch=0.025):
    """The oracle's Newton solve with its GMG-CG (same solver settings and
    material) on a small mesh of the Newton benchmark's recipe, one load step, timed on
    the host cores: the oracle beside the device Newton step."""
    from oracle import fe, gmg, newton
    import workloads as W
    H = gmg.Hierarchy(3, n_cells >> (n_levels - 1), 2, n_levels, fe.Material(w["mu"], w["lam"], w["inclusions"]),
                      W.clamp_bottom_top(3))
    fv = np.zeros((6, 3))
    fv[5][2] = stretch
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    u, recs = newton.solve(H, fv, n_steps=1)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    n = H.meshes[-1].n_dofs
    return {"value": wall / max(len(recs), 1) * 1e3, "unit": "ms per Newton step", "cores": round(cpu / wall, 1),
            "kind": "oracle", "newton_steps": len(recs), "cg_iters": [r["cg_iters"] for r in recs],
            "sample": f"oracle Newton + GMG-CG (V(2,2) Chebyshev(4), direct coarse solve, CG to 1e-8) on 3-D Q2 "
                      f"{n_cells}^3 ({n:,} DoFs, levels {n_cells >> (n_levels - 1)}^3..{n_cells}^3), one load step of "
                      f"{stretch:.1%} stretch, {wall:.1f} s wall"}


def newton_bench(w, n_cells=64, n_levels=5, stretch=0.1, n_steps=4, shear_traction=0.1, only=None):
    """Newton load stepping with GMG-CG (1e-8) on the two-phase material,
    64^3 Q2 (6.44M DoFs), levels 4^3..64^3, clamped bottom/top, 10 % stretch in
    4 steps; mixed-precision (FP32 V-cycle) and all-FP64 forms.  `only`: the
    names of the runs to make ("shear_traction" for the traction load path),
    all when None."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import F32, F64, Problem
    out = {"workload": f"3-D Q2 {n_cells}^3 ({(2 * n_cells + 1) ** 3 * 3:,} DoFs), levels "
                       f"{n_cells >> (n_levels - 1)}^3..{n_cells}^3, two-phase material, clamped bottom/top, "
                       f"{stretch:.0%} stretch in {n_steps} load steps, FP64 CG to 1e-8 with a V(2,2) "
                       f"Chebyshev(4) GMG preconditioner, cached F^-1 and c1 on every level, FP64 dense coarse "
                       f"solve (variants: recompute / cached-F level operators, V(1,1), the "
                       f"Chebyshev coarse solver to 1e-3, eigenvalue estimates of the first linearisation "
                       f"reused)"}
    # level operators with cached F^-1 and c1 (Algorithm 2's trade-off); the
    # other policies and the paper's solver alternatives (Sec. 7) as variants
    runs = (("mixed", dict(vcycle_dtype=F32, qp_policy=2)), ("fp64", dict(vcycle_dtype=F64, qp_policy=2)),
            ("mixed_recompute", dict(vcycle_dtype=F32, qp_policy=0)),
            ("fp64_recompute", dict(vcycle_dtype=F64, qp_policy=0)),
            ("mixed_cache_F", dict(vcycle_dtype=F32, qp_policy=1)),
            # V-cycles replayed from HIP graphs (on a stream of the problem's own)
            ("mixed_graphs", dict(vcycle_dtype=F32, qp_policy=2, graphs=True)),
            ("mixed_V11", dict(vcycle_dtype=F32, qp_policy=2, n_smooth=1)),
            ("mixed_chebyshev_coarse", dict(vcycle_dtype=F32, qp_policy=2, coarse_solver=1)),
            ("mixed_eig_reuse", dict(vcycle_dtype=F32, qp_policy=2, eig_refresh=0)))
    for name, kw in runs:
        if only is not None and name not in only:
            continue
        kw = dict(kw)
        graphs = kw.pop("graphs", False)
        if graphs:
            kw["stream"] = torch.cuda.Stream()
        P = Problem(3, n_cells, 2, n_levels=n_levels, mu=tuple(w["mu"]), lam=tuple(w["lam"]),
                    inclusions=w["inclusions"], dirichlet_mask=W.clamp_bottom_top(3), **kw)
        if graphs:
            P.enable_graphs(True)
        u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
        fv = np.zeros((6, 3))
        fv[5][2] = stretch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, st = P.newton_solve(u, fv, n_steps=n_steps, raise_on_error=False)
        total = time.perf_counter() - t0
        steps = [r["setup_ms"] + r["residual_ms"] + r["solve_ms"] for r in recs]
        out[name] = {
            "status": int(st), "newton_steps": len(recs), "total_s": round(total, 3),
            "median_step_ms": float(np.median(steps)), "mean_step_ms": float(np.mean(steps)),
            "median_setup_ms": float(np.median([r["setup_ms"] for r in recs])),
            "median_residual_ms": float(np.median([r["residual_ms"] for r in recs])),
            "median_solve_ms": float(np.median([r["solve_ms"] for r in recs])),
            "cg_iters": [r["cg_iters"] for r in recs],
            "max_cg_relres": max(r["cg_relres"] for r in recs),
            "final_residual": recs[-1]["residual_after"] if recs else None,
            "coarse_negative_eigs": max(r["coarse_negative"] for r in recs) if recs else None,
        }
        print(f"[bench] newton {name}: {len(recs)} steps, median {out[name]['median_step_ms']:.1f} ms, "
              f"total {total:.2f} s, status {st}", file=sys.stderr, flush=True)
        del P
        torch.cuda.empty_cache()
    if "fp64" in out and "mixed" in out:
        out["speedup_mixed_vs_fp64"] = out["fp64"]["median_step_ms"] / out["mixed"]["median_step_ms"]
    if only is not None and "shear_traction" not in only:
        return out
    # the paper's load path (Sec. 7): bottom clamped, dead shear traction on the top face in 5 steps
    P = Problem(3, n_cells, 2, n_levels=n_levels, mu=tuple(w["mu"]), lam=tuple(w["lam"]),
                inclusions=w["inclusions"], dirichlet_mask=W.face_bits(3, 2, 0), vcycle_dtype=F32, qp_policy=2)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    ft = np.zeros((6, 3))
    ft[5][0] = shear_traction
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, st = P.newton_solve(u, np.zeros((6, 3)), n_steps=5, face_traction=ft, raise_on_error=False)
    total = time.perf_counter() - t0
    steps = [r["setup_ms"] + r["residual_ms"] + r["solve_ms"] for r in recs]
    out["mixed_shear_traction"] = {
        "loading": f"bottom clamped, dead shear traction {shear_traction} (x) on the top face, 5 load steps",
        "status": int(st), "newton_steps": len(recs), "total_s": round(total, 3),
        "median_step_ms": float(np.median(steps)), "cg_iters": [r["cg_iters"] for r in recs],
        "max_cg_relres": max(r["cg_relres"] for r in recs), "final_residual": recs[-1]["residual_after"],
        "max_top_displacement": float(u.abs().max().item())}
    print(f"[bench] newton mixed shear traction: {len(recs)} steps, median {np.median(steps):.1f} ms, "
          f"total {total:.2f} s, status {st}", file=sys.stderr, flush=True)
    del P
    torch.cuda.empty_cache()
    return out


def _q4_problem(n_cells, n_levels, level_field):
    import workloads as W
    from paper_1904_13131_amd import F32, Problem
    mu, lam = W.two_phase_material()
    return Problem(3, n_cells, 4, n_levels=n_levels, mu=tuple(mu), lam=tuple(lam), inclusions=W.spheres(200, 7),
                   dirichlet_mask=W.clamp_bottom_top(3), qp_policy=2, vcycle_dtype=F32, level_field=level_field)


def _q4_reach(n_cells, n_levels, cg_max_it, coarse_solver=0, fp64_vcycle=False, budget_s=30.0, strain=-0.2):
    """The config-5 body at another resolution: one Newton solve over the five
    load steps towards `strain`, within a wall-time budget; how far it gets
    and why it stops."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import F32, F64, Problem, lib
    mu, lam = W.two_phase_material()
    P = Problem(3, n_cells, 4, n_levels=n_levels, mu=tuple(mu), lam=tuple(lam), inclusions=W.spheres(200, 7),
                dirichlet_mask=W.clamp_bottom_top(3), qp_policy=2, vcycle_dtype=F64 if fp64_vcycle else F32,
                coarse_solver=coarse_solver)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    fv = np.zeros((6, 3))
    fv[5][2] = strain
    t0 = time.perf_counter()
    recs, st = P.newton_solve(u, fv, n_steps=5, cg_max_it=cg_max_it, raise_on_error=False, max_seconds=budget_s)
    why = lib().mfh_last_error(P.handle).decode() if st != 0 else ""
    out = {"mesh": f"{n_cells}^3 Q4", "levels": n_levels,
           "preconditioner": "Chebyshev solver on the one level" if coarse_solver else "GMG, direct coarse solve",
           "vcycle": "f64" if fp64_vcycle else "f32", "cg_max_it": cg_max_it, "status": int(st), "stop_reason": why,
           "strain_reached": _converged_fraction(recs) * strain, "newton_steps": len(recs),
           "max_cg_iters": max([r["cg_iters"] for r in recs] or [0]),
           "max_coarse_negative": max([r["coarse_negative"] for r in recs] or [0]),
           "wall_s": round(time.perf_counter() - t0, 2)}
    print(f"[bench] q4 body {out['mesh']}, {n_levels} level(s), {out['preconditioner']}, CG cap {cg_max_it}: "
          f"{out['strain_reached']:.2%} of -20 %, status {st} ({why[:80]})", file=sys.stderr, flush=True)
    P.close()
    del P
    torch.cuda.empty_cache()
    return out


def _converged_fraction(recs, du_tol=1e-5, r_tol=1e-8):
    """Largest load fraction whose increment converged, from the Newton records
    (an increment's records share its load fraction, with rising step numbers)."""
    best, i = 0.0, 0
    while i < len(recs):
        j = i
        while (j + 1 < len(recs) and recs[j + 1]["load_fraction"] == recs[i]["load_fraction"]
               and recs[j + 1]["newton_iter"] == recs[j]["newton_iter"] + 1):
            j += 1
        last, r0 = recs[j], recs[i]["residual_norm"]
        ra = last["residual_after"]
        if np.isfinite(ra) and last["du_norm"] <= du_tol and (ra <= r_tol or ra <= r_tol * r0):
            best = max(best, last["load_fraction"])
        i = j + 1
    return best


def _q4_newton(n_cells, n_levels, strain, n_steps, level_field, cg_max_it=500, budget_s=60.0):
    """Newton load stepping to `strain` (negative: compression) in n_steps
    increments, within a wall-time budget (the library's max_seconds)."""
    import torch
    P = _q4_problem(n_cells, n_levels, level_field)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    fv = np.zeros((6, 3))
    fv[5][2] = strain
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, st, done, why = [], 0, 0.0, ""
    name = f"{'compression' if strain < 0 else 'tension'} {abs(strain):.0%}, {['nodal', 'vertex'][level_field]}"
    for k in range(1, n_steps + 1):   # one call per load step (progress lines between them)
        left = budget_s - (time.perf_counter() - t0)
        if left <= 0:
            st, why = -5, "time budget"
            break
        rk, st = P.newton_solve(u, fv * (k / n_steps), n_steps=1, cg_max_it=cg_max_it, raise_on_error=False,
                                max_seconds=left)
        frac = _converged_fraction(rk)
        for r in rk:
            r["load_fraction"] = (k - 1 + r["load_fraction"]) / n_steps
        recs += rk
        print(f"[bench] q4_48cube {name} load step {k}: {len(rk)} Newton steps, CG iterations "
              f"{[r['cg_iters'] for r in rk][-12:]}, status {st}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        if st != 0:
            done = (k - 1 + frac) / n_steps
            from paper_1904_13131_amd import lib
            why = lib().mfh_last_error(P.handle).decode()
            break
        done = k / n_steps
    total = time.perf_counter() - t0
    ok = [r for r in recs if np.isfinite(r["residual_after"]) and r["cg_relres"] <= 1e-8]
    P.close()
    del P
    torch.cuda.empty_cache()
    return {"loading": name, "level_field": ["nodal", "vertex"][level_field], "status": int(st),
            "stop_reason": why, "budget_s": budget_s,
            "wall_s": round(total, 2), "newton_steps": len(recs), "strain_reached": done * strain,
            "cutbacks": max([r["cutbacks"] for r in recs] or [0]),
            "min_J_last": recs[-1]["min_J"] if recs else None,
            "max_coarse_negative": max([r["coarse_negative"] for r in recs] or [0]),
            "median_newton_step_ms": float(np.median([r["setup_ms"] + r["residual_ms"] + r["solve_ms"]
                                                      for r in ok])) if ok else None,
            "cg_iters_converged_steps": [r["cg_iters"] for r in ok][-40:],
            "step_lengths_below_1": sum(1 for r in recs if np.isfinite(r["step_length"]) and r["step_length"] < 1)}


def q4_48cube_bench(n_cells=48, n_levels=5, n_steps=5, steps=10, newton=True, budget_s=60.0):
    """3-D Q4 48^3 (21.6 M DoFs), 5^3 Gauss points, 200 spheres (seed 7),
    two-phase Neo-Hookean material, bottom/top clamped, levels 3^3..48^3, FP32 V(2,2)
    Chebyshev(4) GMG under FP64 CG.  Level vmults (FP32 on three levels, FP64 on
    the finest) and the FP64 residual at a smooth start state; then Newton to
    20 % compression (paper-literal nodal level fields) and to 20 % tension with
    vertex level fields."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import F32, F64
    from paper_1904_13131_amd.mfh import SCATTER_NAMES
    P = _q4_problem(n_cells, n_levels, 0)
    n = P.n_dofs()
    out = {"workload": f"3-D Q4 {n_cells}^3 ({n:,} DoFs), 125 Gauss points per cell, 200 spheres (seed 7), "
                       f"two-phase material, clamped bottom/top, {n_steps} load steps, levels "
                       f"{n_cells >> (n_levels - 1)}^3..{n_cells}^3, FP32 V(2,2) Chebyshev(4) GMG under FP64 CG "
                       f"to 1e-8 (at most 500 iterations), FP64 dense coarse solve", "qp_policy": "cache_T2"}
    u0 = torch.as_tensor(W.sine_field(3, 4 * n_cells + 1, 4, 0.01, kmax=1, coords=P.node_coords_1d()),
                         device="cuda")
    P.set_deformation(u0)
    lv = {}
    for level in range(n_levels - 1, max(-1, n_levels - 4), -1):
        nl = P.n_dofs(level)
        x = torch.as_tensor(W.normal_vector(nl, 5), device="cuda")
        for dt, tdt, code in (("f32", torch.float32, F32), ("f64", torch.float64, F64)):
            if dt == "f64" and level != n_levels - 1:
                continue
            xx = x.to(tdt)
            y = torch.empty_like(xx)
            for _ in range(3):
                P.tangent_vmult(xx, y, level=level)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(P.stream)
            for _ in range(steps):
                P.tangent_vmult(xx, y, level=level)
            e1.record(P.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            lv[f"level{level}_{dt}"] = {"n_dofs": nl, "ms": ms, "dofs_per_s": nl / (ms * 1e-3),
                                        "scatter": SCATTER_NAMES[P.scatter_mode(level, code)]}
            print(f"[bench] q4_48cube vmult level {level} {dt}: {ms:.3f} ms, {nl / (ms * 1e-3):.3e} DoF/s",
                  file=sys.stderr, flush=True)
    r = torch.empty_like(u0)
    for _ in range(2):
        P.residual(u0, r)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(P.stream)
    for _ in range(steps):
        P.residual(u0, r)
    e1.record(P.stream)
    torch.cuda.synchronize()
    out["level_vmults"] = lv
    out["residual_fp64_ms"] = e0.elapsed_time(e1) / steps
    P.close()
    del P
    torch.cuda.empty_cache()
    if newton:
        out["newton"] = [_q4_newton(n_cells, n_levels, -0.2, n_steps, 0, budget_s=budget_s),
                         _q4_newton(n_cells, n_levels, +0.2, n_steps, 1, budget_s=budget_s)]
        # the same body and compression at coarser resolutions: where the load
        # path ends with the multigrid preconditioner, and where the body's
        # own tangent gives out (one level, no coarse displacements)
        out["resolution_study"] = [_q4_reach(4, 2, 3000, fp64_vcycle=True),
                                   _q4_reach(12, 3, 3000),
                                   _q4_reach(12, 1, 2000, coarse_solver=1, fp64_vcycle=True)]
    return out


def batch_bench(policy=2, steps=20, warmup=3, n=256, solve=True):
    """A batch of 256 independent 3-D problems (N in {8, 12, 16, 24}, p in {1, 2, 3},
    1-10 spheres, loaded linearisation point).  Aggregate batched vmult DoFs/s in
    FP64 and FP32 against one launch per problem, and one Newton correction per
    problem (K du = -R) by mixed-precision GMG-CG to 1e-8, all problems in
    lockstep from one host thread, with graph-captured V-cycles."""
    import torch

    import workloads as W
    from paper_1904_13131_amd import F32, Batch, Problem
    mu, lam = W.two_phase_material()
    descs = W.batch_of_cubes(n=n)
    probs, us, x64 = [], [], []
    t0 = time.perf_counter()
    for d in descs:
        incl = W.spheres(d["n_spheres"], d["sphere_seed"], 3)
        P = Problem(3, d["n_cells"], d["degree"], n_levels=d["n_levels"], mu=tuple(mu), lam=tuple(lam),
                    inclusions=incl, dirichlet_mask=d["mask"], qp_policy=policy, vcycle_dtype=F32,
                    stream=torch.cuda.Stream())
        _, u, x = W.batch_fields(d, coords=P.node_coords_1d())
        probs.append(P)
        us.append(torch.as_tensor(u, device="cuda"))
        x64.append(torch.as_tensor(x, device="cuda"))
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    dofs = [P.n_dofs() for P in probs]
    total = int(sum(dofs))
    ws_gb = sum(P.workspace.numel() for P in probs) / 1e9
    B = Batch(probs)
    t0 = time.perf_counter()
    mj = B.set_deformation(us)
    t_setdef = time.perf_counter() - t0
    out = {"workload": f"{n} independent 3-D problems (seed 6): N in {{8,12,16,24}}, p in {{1,2,3}}, 1-10 spheres, "
                       f"uniaxial stretch 2-8 % plus a smooth perturbation of 1/20 of it; {total:,} DoFs in total "
                       f"({min(dofs):,}..{max(dofs):,})",
           "n_problems": n, "total_dofs": total, "qp_policy": POLICIES[policy], "workspace_gb": round(ws_gb, 2),
           "create_s": round(t_create, 2), "set_deformation_s": round(t_setdef, 3), "min_J": min(mj),
           "degree_bins": len({d["degree"] for d in descs})}
    stream = torch.cuda.current_stream()
    for name, xs in (("f64", x64), ("f32", [x.float() for x in x64])):
        ys = [torch.empty_like(x) for x in xs]
        for _ in range(warmup):
            B.tangent_vmult(xs, ys)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            B.tangent_vmult(xs, ys)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
        for _ in range(warmup):
            for P, x, y in zip(probs, xs, ys):
                P.tangent_vmult(x, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for P, x, y in zip(probs, xs, ys):
                P.tangent_vmult(x, y)
        torch.cuda.synchronize()
        ms_l = (time.perf_counter() - t0) * 1e3 / steps
        out[f"vmult_{name}"] = {"batched_ms": ms_b, "batched_dofs_per_s": total / (ms_b * 1e-3),
                                "per_problem_launches_ms": ms_l, "per_problem_dofs_per_s": total / (ms_l * 1e-3),
                                "speedup_batched_vs_per_problem": ms_l / ms_b}
        print(f"[bench] batch vmult {name}: {ms_b:.3f} ms ({total / (ms_b * 1e-3):.3e} DoF/s), "
              f"one launch per problem {ms_l:.3f} ms", file=sys.stderr, flush=True)
        del ys
    # the same batch linearised about random smooth deformations (amplitude
    # 0.025-0.1, read literally; tangents may be indefinite: vmult only)
    ul = [torch.as_tensor(W.batch_literal_field(d, coords=P.node_coords_1d()), device="cuda")
          for d, P in zip(descs, probs)]
    mjl = B.set_deformation(ul)
    lit = {"min_J": min(mjl)}
    for name, xs in (("f64", x64), ("f32", [x.float() for x in x64])):
        ys = [torch.empty_like(x) for x in xs]
        for _ in range(warmup):
            B.tangent_vmult(xs, ys)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            B.tangent_vmult(xs, ys)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
        lit[f"vmult_{name}"] = {"batched_ms": ms_b, "batched_dofs_per_s": total / (ms_b * 1e-3)}
        print(f"[bench] batch vmult {name}, random smooth deformations: {ms_b:.3f} ms "
              f"({total / (ms_b * 1e-3):.3e} DoF/s), min J {min(mjl):.3f}", file=sys.stderr, flush=True)
        del ys
    out["random_smooth_linearisation"] = lit
    del ul
    B.set_deformation(us)
    if not solve:
        B.close()
        for P in probs:
            P.close()
        torch.cuda.empty_cache()
        return out
    # one Newton correction per problem: K du = -R(u), mixed-precision GMG-CG to 1e-8
    bs = [P.residual(u) for P, u in zip(probs, us)]      # on the problems' streams
    torch.cuda.synchronize()
    for b in bs:
        b.neg_()
    xs = [torch.empty_like(b) for b in bs]
    torch.cuda.synchronize()
    for P in probs:
        P.enable_graphs(True)
    runs = {}
    for label in ("first", "graphs", "eager"):
        if label == "eager":
            for P in probs:
                P.enable_graphs(False)
        t0 = time.perf_counter()
        it, rel, ms = B.cg_solve(bs, xs, rtol=1e-8, max_it=300)
        wall = time.perf_counter() - t0
        runs[label] = {"wall_s": round(wall, 4), "dofs_per_s": total / wall,
                       "per_problem_ms": {"median": float(np.median(ms)), "p90": float(np.percentile(ms, 90)),
                                          "max": float(np.max(ms))},
                       "cg_iters": {"min": int(min(it)), "median": float(np.median(it)), "max": int(max(it))},
                       "max_relres": float(max(rel))}
        print(f"[bench] batch solve ({label}): {wall:.3f} s wall, per-problem median {np.median(ms):.1f} ms, "
              f"iters {min(it)}..{max(it)}, max relres {max(rel):.2e}", file=sys.stderr, flush=True)
    # per-problem cost: every problem solved alone (set-up done, graphs on), so
    # that its own GPU time is measured instead of its lockstep finish time
    for P in probs:
        P.enable_graphs(True)
    alone = []
    for P, b, x in zip(probs, bs, xs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.cg_solve(b, x, rtol=1e-8, max_it=300)
        alone.append((time.perf_counter() - t0) * 1e3)
    by_deg = {}
    for d, ms in zip(descs, alone):
        by_deg.setdefault(d["degree"], []).append(ms)
    runs["alone"] = {"sum_s": round(sum(alone) / 1e3, 4),
                     "per_problem_ms": {"median": float(np.median(alone)), "p90": float(np.percentile(alone, 90)),
                                        "max": float(np.max(alone))},
                     "median_ms_by_degree": {str(k): float(np.median(v)) for k, v in sorted(by_deg.items())}}
    print(f"[bench] batch solve (alone): {sum(alone) / 1e3:.3f} s summed, per-problem median {np.median(alone):.1f} ms",
          file=sys.stderr, flush=True)
    out["solve"] = {"note": "first: includes the preconditioner set-up (diagonals, eigenvalue estimates, coarse "
                            "inverse) and the graph capture; graphs: replayed V-cycle graphs; eager: no graphs; "
                            "per_problem_ms of these three is the time from the call's start at which a problem "
                            "finished (lockstep); alone: each problem's own solve time, one problem at a time "
                            "(set-up done, graphs on), and their sum",
                    **runs}
    B.close()
    for P in probs:
        P.close()
    del probs, us, x64, bs, xs
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--policies", default="0,1,2,3")
    ap.add_argument("--dtypes", default="f64,f32")
    ap.add_argument("--no-cold", action="store_true")
    ap.add_argument("--scatter", type=int, default=-1, help="-1 auto (tuned table), 0 atomic, 1 colour, 2 tile, 3 element")
    ap.add_argument("--no-newton", action="store_true", help="skip the 64^3 Q2 Newton-step measurement")
    ap.add_argument("--newton-runs", default="", help="comma-separated Newton runs to make (mixed, fp64, "
                    "mixed_recompute, ..., shear_traction); all when empty")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-problem batched measurement")
    ap.add_argument("--no-batch-solve", action="store_true", help="256-problem batch: time the batched vmult only")
    ap.add_argument("--no-q4", action="store_true", help="skip the Q4 48^3 level vmults and Newton runs")
    ap.add_argument("--q4-48cube", action="store_true", help="with a partial policy/dtype run: add the Q4 48^3 part")
    ap.add_argument("--q4-48cube-vmult-only", action="store_true", help="Q4 48^3: level vmults only, no Newton")
    ap.add_argument("--q4-budget", type=float, default=60.0,
                    help="wall-time budget in seconds of each Q4 48^3 Newton loading (compression, tension)")
    ap.add_argument("--no-matrix-based", action="store_true", help="skip the CSR matrix-based comparison")
    ap.add_argument("--matrix-based-only", action="store_true", help="only the CSR matrix-based comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        return 2

    import torch

    import workloads as W
    from paper_1904_13131_amd import F32, F64, Problem
    from paper_1904_13131_amd.mfh import SCATTER_NAMES

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.matrix_based_only:
        print(json.dumps({"partial": True, "matrix_based": matrix_based_bench()}), flush=True)
        return 0
    w = W.cube_spheres_q2()
    dim, nc, deg = w["dim"], w["n_cells"], w["degree"]
    u = torch.as_tensor(w["u"], device="cuda")
    x64 = torch.as_tensor(w["x"], device="cuda")
    x32 = x64.float()
    flush = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")   # 512 MB > MALL, read to flush
    if a.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written", file=sys.stderr)
        del src, dst
    dtypes = a.dtypes.split(",")
    res = {}
    n_dofs = None
    for pol in [int(p) for p in a.policies.split(",")]:
        P = Problem(dim, nc, deg, mu=tuple(w["mu"]), lam=tuple(w["lam"]), inclusions=w["inclusions"], qp_policy=pol,
                    scatter=a.scatter)
        P.set_deformation(u)
        n_dofs = P.n_dofs()
        for dt, x in (("f64", x64), ("f32", x32)):
            if dt not in dtypes:
                continue
            y = torch.empty_like(x)
            ms, calls = time_vmult(P, x, y, a.steps, a.warmup)
            cold = [float("nan")]
            if not a.no_cold:
                _, cold = time_vmult(P, x, y, max(10, a.steps // 5), 1, cold=True, flush=flush)
            mode = SCATTER_NAMES[P.scatter_mode(-1, F64 if dt == "f64" else F32)]
            res[(pol, dt)] = dict(ms_per_step=ms, call_ms_median=float(np.median(calls)), call_ms_min=min(calls),
                                  cold_ms_median=float(np.median(cold)), cold_ms_min=min(cold),
                                  dofs_per_s=n_dofs / (ms * 1e-3), scatter=mode)
            print(f"[bench] {POLICIES[pol]:9s} {dt} ({mode}): {ms * 1e3:8.1f} us/vmult, per call median "
                  f"{np.median(calls) * 1e3:8.1f} min {min(calls) * 1e3:8.1f} us, cold median "
                  f"{np.median(cold) * 1e3:8.1f} us, {n_dofs / (ms * 1e-3):.3e} DoF/s", file=sys.stderr, flush=True)
        del P
        torch.cuda.empty_cache()
    if not any(k[1] == "f64" for k in res) or not any(k[1] == "f32" for k in res):
        part = {"partial": True, "variants": {f"{POLICIES[k[0]]}/{k[1]}": res[k] for k in res}}
        if a.q4_48cube or a.q4_48cube_vmult_only:
            part["q4_48cube"] = q4_48cube_bench(newton=not a.q4_48cube_vmult_only, budget_s=a.q4_budget)
        print(json.dumps(part))
        return 0
    best = max((k for k in res if k[1] == "f64"), key=lambda k: res[k]["dofs_per_s"])
    best32 = max((k for k in res if k[1] == "f32"), key=lambda k: res[k]["dofs_per_s"])
    r = res[best]
    out = {
        "metric": METRIC,
        "value": r["dofs_per_s"],
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D unit cube 32^3 Q2 (823,875 DoFs), 27 Gauss points per cell, Neo-Hookean "
                               "matrix mu=1 nu=0.3 with 20 seeded spheres (r 0.05-0.12, 100x stiffer), smooth "
                               "seeded displacement amplitude 0.1; one FP64 tangent vmult per step",
                   "n_dofs": n_dofs, "cells": nc ** dim, "degree": deg, "qp_policy": POLICIES[best[0]],
                   "scatter": ("auto: " if a.scatter < 0 else "") + r["scatter"]},
        "roofline": roofline(dim, deg, nc, n_dofs, best[0], "f64", r["ms_per_step"], r["scatter"]),
        "fp32": {"value": res[best32]["dofs_per_s"], "unit": "DoF/s", "qp_policy": POLICIES[best32[0]],
                 "scatter": res[best32]["scatter"],
                 "roofline": roofline(dim, deg, nc, n_dofs, best32[0], "f32", res[best32]["ms_per_step"],
                                      res[best32]["scatter"])},
        "variants": {f"{POLICIES[k[0]]}/{k[1]}": {kk: (round(v, 6) if isinstance(v, float) else v)
                                                 for kk, v in res[k].items()} for k in res},
    }
    # per-call timings (an event pair around each call adds a few us): warm
    # median and minimum, and cold (after a 512 MB cache flush) median, with
    # the fraction of the HBM roofline the cold median reaches
    rl = out["roofline"]
    rl.update(call_ms_median=r["call_ms_median"], call_ms_min=r["call_ms_min"], cold_ms_median=r["cold_ms_median"],
              cold_ms_min=r["cold_ms_min"])
    if rl["bound"] == "hbm" and np.isfinite(r["cold_ms_median"]):
        rl["achieved_cold"] = rl["alg_bytes"] / (r["cold_ms_median"] * 1e-3) / 1e9
        rl["frac_cold"] = rl["achieved_cold"] / rl["peak"]
    if 3 in [int(p) for p in a.policies.split(",")]:
        out["mooney_rivlin_cache_T4"] = law_bench(w, a.steps, a.warmup)
    if not a.no_matrix_based:
        out["matrix_based"] = matrix_based_bench()
    if not a.no_newton:
        out["newton_step"] = newton_bench(w, only=a.newton_runs.split(",") if a.newton_runs else None)
        if not a.no_cpu:
            out["newton_step"]["cpu_oracle"] = cpu_newton_baseline(w)
    if not a.no_batch:
        out["batched"] = batch_bench(solve=not a.no_batch_solve)
    if not a.no_q4:
        out["q4_48cube"] = q4_48cube_bench(newton=not a.q4_48cube_vmult_only, budget_s=a.q4_budget)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
