"""Autotuner of the tangent vmult's launch shapes (run on the GPU).

Scatter mode, tile shape and cells per block: for every (dim, degree,
precision, qp policy, size class) it times one whole tangent vmult (output
fill or node sums included) on a representative mesh with each scatter mode,
the TILE mode with each of its two compiled tile shapes and the pencil-kernel
modes (ATOMIC, ELEMENT, COLOR) with each of their two compiled cell-block
lengths, and records the fastest mode with its cell-block length, and the
faster tile shape (used whenever TILE runs).  Batch
launch: on the 256-problem batch of independent 3-D problems (degrees 1 to
3) it times the batched vmult as one launch per degree bin and as one
persistent launch over every degree, in both precisions, and records the
faster.  Contraction stage: the sum factorisation's 1-D contractions at
degrees 3 and 4 in FP32, VALU against MFMA (recorded in the table; the
tangent kernels implement the VALU form, which the measurement favours).  Both go to ``tuning/gfx950.json``; ``csrc/tuned.hpp`` is generated
from that table and compiled into the library, where MFH_SCATTER_AUTO and
MFH_BATCH_LAUNCH_AUTO look them up.

    python -m paper_1904_13131_amd.autotune [--quick] [--out tuning/gfx950.json]
    python -m paper_1904_13131_amd.autotune --emit-header     # JSON -> csrc/tuned.hpp only
    python -m paper_1904_13131_amd.autotune --policies cache_T4 --out new.json
        # re-measure some policies; the other entries are kept from the table
    python -m paper_1904_13131_amd.autotune --batch-only
        # re-measure the batch launch and the contraction stage only; the
        # scatter entries are kept
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
JSON_PATH = os.path.join(HERE, "tuning", "gfx950.json")
HEADER_PATH = os.path.join(HERE, "csrc", "tuned.hpp")

MODES = {"atomic": 0, "color": 1, "tile": 2, "element": 3}
POLICIES = {"recompute": 0, "cache_F": 1, "cache_T2": 2, "cache_T4": 3}
DTYPES = {"f64": 0, "f32": 1}
# size classes by cells of the level: small < 4096 <= medium < 65536 <= large
CLASS_BOUNDS = (4096, 65536)
CLASSES = ("small", "medium", "large")
# representative cells per direction for each (dim, class); large 3-D meshes
# of degree >= 3 use 48^3 cells to bound the memory
MESH = {(2, "small"): 32, (2, "medium"): 128, (2, "large"): 512,
        (3, "small"): 12, (3, "medium"): 32, (3, "large"): 64}


def size_class(cells):
    return 0 if cells < CLASS_BOUNDS[0] else 1 if cells < CLASS_BOUNDS[1] else 2


def _time_vmult(P, x, reps, warmup):
    import torch
    y = torch.empty_like(x)
    for _ in range(warmup):
        P.tangent_vmult(x, y)
    s = P.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        P.tangent_vmult(x, y)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps   # microseconds per vmult


def measure(dims=(2, 3), degrees=(1, 2, 3, 4), quick=False, log=print, policies=None):
    import torch

    import workloads as W
    from .mfh import Problem
    mu, lam = W.two_phase_material()
    entries = []
    reps, warmup = (10, 2) if quick else (30, 5)
    for dim in dims:
        for degree in degrees:
            for cls in CLASSES:
                N = MESH[(dim, cls)]
                if dim == 3 and cls == "large" and degree >= 3:
                    N = 48
                if dim == 2 and cls == "large" and degree == 4:
                    N = 384   # lattice of at most 1600 nodes per direction
                incl = W.spheres(8, 3, dim)
                for pname, pol in POLICIES.items():
                    if policies is not None and pname not in policies:
                        continue
                    times = {dt: {} for dt in DTYPES}
                    pencil = ["atomic", "element"] + (["color"] if cls == "large" else [])
                    modes = [m + b for m in pencil for b in ("", "/b1")] + ["tile0", "tile1"]
                    for mname in modes:
                        tile = int(mname[4]) if mname.startswith("tile") else -1
                        cb = 1 if mname.endswith("/b1") else 0
                        base = "tile" if tile >= 0 else mname.split("/")[0]
                        P = Problem(dim, N, degree, mu=tuple(mu), lam=tuple(lam), inclusions=incl, qp_policy=pol,
                                    scatter=MODES[base], tile_shape=tile, cell_block=cb)
                        L = degree * N + 1
                        u = W.sine_field(dim, L, 4, 0.02, kmax=1, coords=P.node_coords_1d())
                        P.set_deformation(torch.as_tensor(u, device="cuda"))
                        x = torch.as_tensor(W.normal_vector(P.n_dofs(), 5), device="cuda")
                        for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
                            times[dt][mname] = _time_vmult(P, x.to(tdt), reps, warmup)
                        del P, x
                        torch.cuda.empty_cache()
                    for dt in DTYPES:
                        best = min(times[dt], key=times[dt].get)
                        tile = 0 if times[dt]["tile0"] <= times[dt]["tile1"] else 1
                        scatter = "tile" if best.startswith("tile") else best.split("/")[0]
                        entries.append(dict(dim=dim, degree=degree, dtype=dt, policy=pname, size_class=cls,
                                            cells=N ** dim, scatter=scatter, tile=tile,
                                            cell_block=1 if best.endswith("/b1") else 0,
                                            us={k: round(v, 2) for k, v in times[dt].items()}))
                        log(f"[autotune] d{dim} p{degree} {cls:6s} N={N:3d} {pname:9s} {dt}: "
                            + " ".join(f"{k}={v:7.1f}" for k, v in times[dt].items()) + f" -> {best}")
    return entries


def measure_batch(log=print, reps=20, warmup=3):
    """The batched vmult of the 256-problem batch (cache_T2), per-degree
    launches against the fused persistent launch, FP64 and FP32 (ms)."""
    import numpy as np
    import torch

    import workloads as W
    from .mfh import Batch, Problem
    from . import mfh
    mu, lam = W.two_phase_material()
    probs, us = [], []
    for d in W.batch_of_cubes():
        incl = W.spheres(d["n_spheres"], d["sphere_seed"], 3)
        P = Problem(3, d["n_cells"], d["degree"], n_levels=d["n_levels"], mu=tuple(mu), lam=tuple(lam),
                    inclusions=incl, dirichlet_mask=d["mask"], qp_policy=2, stream=torch.cuda.current_stream())
        L = d["degree"] * d["n_cells"] + 1
        us.append(torch.as_tensor(W.stretched_field(3, L, d["stretch"], d["u_seed"], d["amp"],
                                                    coords=P.node_coords_1d()), device="cuda"))
        probs.append(P)
    B = Batch(probs)
    B.set_deformation(us)
    out = {}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        xs = [torch.as_tensor(W.normal_vector(P.n_dofs(), 5), device="cuda").to(tdt) for P in probs]
        ys = [torch.empty_like(x) for x in xs]
        for mode, code in (("per_degree", mfh.BATCH_LAUNCH_PER_DEGREE), ("fused", mfh.BATCH_LAUNCH_FUSED)):
            B.set_launch(code)
            for _ in range(warmup):
                B.tangent_vmult(xs, ys)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(B.stream)
            for _ in range(reps):
                B.tangent_vmult(xs, ys)
            e1.record(B.stream)
            torch.cuda.synchronize()
            out.setdefault(dt, {})[mode] = round(e0.elapsed_time(e1) / reps, 4)
        log(f"[autotune] batch {dt}: " + " ".join(f"{k}={v:.3f} ms" for k, v in out[dt].items()))
    total = {m: sum(out[dt][m] for dt in out) for m in ("per_degree", "fused")}
    B.close()
    del B, probs, us
    torch.cuda.empty_cache()
    return {"policy": "cache_T2", "ms": out, "launch": min(total, key=total.get)}


def measure_contraction(log=print, sweeps=200, blocks=4096, reps=10):
    """The sum factorisation's 1-D contraction stage (Sec. 5) at degrees 3 and
    4 in FP32, VALU against MFMA (mfh_contraction_stage): time of `reps`
    launches of `blocks` x 256 lines x `sweeps` dependent applications of a
    table pair, as table-FLOP rates (4 n^2 per line and sweep), and the
    largest difference of the two forms' results."""
    import torch

    from .mfh import contraction_stage
    out = {}
    for degree in (3, 4):
        n = degree + 1
        res, bufs = {}, {}
        for form, m in (("valu", 0), ("mfma", 1)):
            buf = torch.empty(blocks * n * 256, dtype=torch.float32, device="cuda")
            contraction_stage(degree, m, sweeps, blocks, buf)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                contraction_stage(degree, m, sweeps, blocks, buf)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[form] = {"ms": round(ms, 4), "table_tflops": round(4 * n * n * blocks * 256 * sweeps / ms / 1e9, 2)}
            bufs[form] = buf
        diff = float(((bufs["valu"] - bufs["mfma"]).abs().max() / bufs["valu"].abs().max()).item())
        choice = min(res, key=lambda f: res[f]["ms"])
        out[str(degree)] = dict(res, max_rel_diff=diff, faster=choice)
        log(f"[autotune] contraction p{degree} fp32: valu {res['valu']['ms']:.3f} ms "
            f"({res['valu']['table_tflops']} TFLOP/s), mfma {res['mfma']['ms']:.3f} ms "
            f"({res['mfma']['table_tflops']} TFLOP/s), max rel diff {diff:.1e} -> {choice}")
    return out


def emit_header(table, path=HEADER_PATH):
    rows = []
    for e in table["entries"]:
        rows.append(f"    {{{e['dim']}, {e['degree']}, {DTYPES[e['dtype']]}, {POLICIES[e['policy']]}, "
                    f"{CLASSES.index(e['size_class'])}, {MODES[e['scatter']]}, {e.get('tile', 0)}, "
                    f"{e.get('cell_block', 0)}}},")
    if not rows:
        rows = ["    {0, 0, 0, 0, 0, 0, 0, 0},   // no measurements: every lookup falls back to ATOMIC, shapes 0"]
    batch = table.get("batch_launch")
    batch_fused = "true" if batch and batch["launch"] == "fused" else "false"
    batch_note = (" (" + ", ".join(f"{dt}: " + " / ".join(f"{k} {v} ms" for k, v in ms.items())
                                   for dt, ms in batch["ms"].items()) + ")") if batch else " (not measured)"
    text = f"""// Generated by paper_1904_13131_amd/autotune.py from tuning/gfx950.json
// ({table.get('note', '')}).  Do not edit: rerun the autotuner.
// Scatter mode measured fastest for one whole tangent vmult, per (dim, degree,
// precision 0 = FP64 / 1 = FP32, qp policy, size class of the level's cells)
// with the cell-block variant of the pencil kernels it was fastest with, and
// the faster of the TILE mode's two tile shapes.
#pragma once

namespace mfh {{

struct TunedScatter {{
  signed char dim, degree, dtype, policy, size_class, scatter, tile, cell_block;
}};

constexpr TunedScatter kTunedScatter[] = {{
{chr(10).join(rows)}
}};

inline int tuned_size_class(long long cells) {{ return cells < {CLASS_BOUNDS[0]} ? 0 : cells < {CLASS_BOUNDS[1]} ? 1 : 2; }}

// Batched vmult: one persistent launch over every degree (true) or one launch
// per degree bin (false), as measured on the 256-problem batch{batch_note}.
constexpr bool kTunedBatchFused = {batch_fused};

// Table entry of a level (nullptr when the table has none).
inline const TunedScatter* tuned_entry(int dim, int degree, int dtype, int policy, long long cells) {{
  const int c = tuned_size_class(cells);
  for (const TunedScatter& e : kTunedScatter)
    if (e.dim == dim && e.degree == degree && e.dtype == dtype && e.policy == policy && e.size_class == c)
      return &e;
  return nullptr;
}}

// Scatter mode for a level (0 = ATOMIC when the table has no entry).
inline int tuned_scatter(int dim, int degree, int dtype, int policy, long long cells) {{
  const TunedScatter* e = tuned_entry(dim, degree, dtype, policy, cells);
  return e ? e->scatter : 0;
}}

// Tile shape of the TILE mode for a level (0 when the table has no entry).
inline int tuned_tile(int dim, int degree, int dtype, int policy, long long cells) {{
  const TunedScatter* e = tuned_entry(dim, degree, dtype, policy, cells);
  return e ? e->tile : 0;
}}

// Cell-block variant of the pencil kernels for a level (0 when the table has no entry).
inline int tuned_cell_block(int dim, int degree, int dtype, int policy, long long cells) {{
  const TunedScatter* e = tuned_entry(dim, degree, dtype, policy, cells);
  return e ? e->cell_block : 0;
}}

}}  // namespace mfh
"""
    with open(path, "w") as f:
        f.write(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=JSON_PATH)
    ap.add_argument("--emit-header", action="store_true", help="only regenerate csrc/tuned.hpp from the JSON")
    ap.add_argument("--dims", default="2,3")
    ap.add_argument("--policies", default=None, help="comma list of policy names to re-measure (default: all)")
    ap.add_argument("--batch-only", action="store_true", help="re-measure the batch launch only")
    a = ap.parse_args(argv)
    if a.emit_header:
        emit_header(json.load(open(a.out)))
        return 0
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    if a.batch_only:
        table = json.load(open(JSON_PATH))
        table["batch_launch"] = measure_batch()
        table["contraction"] = measure_contraction()
        with open(a.out, "w") as f:
            json.dump(table, f, indent=1)
        emit_header(table)
        return 0
    t0 = time.time()
    pols = a.policies.split(",") if a.policies else None
    entries = measure(dims=tuple(int(d) for d in a.dims.split(",")), quick=a.quick, policies=pols)
    note = f"whole-vmult time, {'quick' if a.quick else 'full'} sweep, {time.time() - t0:.0f} s"
    if pols is not None:   # keep the other policies' entries of the current table
        old = json.load(open(JSON_PATH))
        entries = [e for e in old["entries"] if e["policy"] not in pols] + entries
        note = old.get("note", "") + f"; {','.join(pols)}: {note}"
    table = {"arch": "gfx950", "device": torch.cuda.get_device_name(0), "note": note,
             "size_class_bounds_cells": list(CLASS_BOUNDS), "entries": entries, "batch_launch": measure_batch(),
             "contraction": measure_contraction()}
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    emit_header(table)
    return 0


if __name__ == "__main__":
    sys.exit(main())
