#!/usr/bin/env python3
"""Benchmark: DoF-solves per second of the deflated block-Jacobi CG on one MI355X.

A step is one pass of the whole method over one synthetic cracked-body system:
setup (block-Jacobi inverses, K Z, E = Z^T K Z and E^-1, device layout) followed by
one solve of K u = f to relative residual 1e-8 and the release of the handle.  The
inputs (K, Z, blocks, f as device arrays) are resident in HBM before timing starts.

The headline workload is the 80^3 configuration (1.66M DoFs), the largest that the
method's configurations put on one GPU; its matrix (1.38 GB of block values) is far
larger than the 256 MB last-level cache, so the SpMV roofline there is an HBM figure.
Prints one JSON line with the throughput, the SpMV kernel's HBM roofline fraction
(algorithmic bytes / average launch duration measured with HIP events on the
library's stream during the timed steps), the mixed-precision comparison and both
paths' errors against the CPU oracle, the oracle itself timed on this host, and the
40^3 lines (FP64, 32 right-hand sides, uneven systems, subdomain blocks) as extras.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DoF-solves/sec to rel. residual 1e-8 + SpMV HBM GB/s fraction; FP64 vs mixed/batched"
WORKLOADS = {
    "penny80": "80^3 hex8 unit cube (1.66M DoFs), curved penny crack (R=0.25, z=0.5+0.3 rho^2), Heaviside + "
               "branch enrichment within r_e=0.05, 8^3 subdomains, clamped bottom, unit top traction, FP64, "
               "tol 1e-8",
    "penny40": "40^3 hex8 unit cube, curved penny crack (R=0.25, z=0.5+0.3 rho^2), Heaviside + branch "
               "enrichment within r_e=0.05, 4^3 subdomains, clamped bottom, unit top traction, FP64, tol 1e-8",
    "edge10": "10^3 hex8 unit cube, planar edge crack x=0.5 z<0.45, Heaviside + branch enrichment within "
              "r_e=0.15, 2^3 subdomains, clamped bottom, unit top traction, FP64, tol 1e-8",
}

# HBM bytes moved by one k_spmv_p launch on the headline workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the launches of
# iterations that did work), each scaled by what the same counter reads for a 512 MiB
# device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources
# with these digests: after any change to them the figure is reported as null until
# re-measured.
SPMV_TRAFFIC = {
    "workload": "penny80",
    "sources": {
        "paper_2111_09294_amd/csrc/kernels.hip": "9184e2300ba6de0e7e9657e77a8c4bb8355af437fa3be6de05a3e341df1b7577",
        "paper_2111_09294_amd/csrc/dpcg_internal.h": "09b37faadb31f46c783ea09d232a204d9f7c117366662471a83d34623f83b69c"
    },
    "fetch_bytes": 1444818874,
    "write_bytes": 16007888,
}
SPMV_SOURCES = ("paper_2111_09294_amd/csrc/kernels.hip", "paper_2111_09294_amd/csrc/dpcg_internal.h")

# The roofline's kernel duration comes from start/stop events recorded by every
# TIMING_EVERY-th SpMV launch of the timed steps: events on each launch add about 8 us to
# every iteration, sampling keeps the timed run close to an untimed one.
TIMING_EVERY = 8


def _source_digests():
    import hashlib
    out = {}
    for rel in SPMV_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            out[rel] = hashlib.sha256(fh.read()).hexdigest()
    return out


def spmv_traffic(workload):
    """Counter-measured HBM bytes per k_spmv_p launch, or None when the kernel sources
    changed since the counters were taken (or for another workload)."""
    t = SPMV_TRAFFIC
    if workload != t["workload"] or t["fetch_bytes"] is None or _source_digests() != t["sources"]:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def spmv_bytes(nnzb, n, value_bytes=8, col_bytes=4):
    """Algorithmic bytes of one q = K p launch: each 3x3 block (9 values and its block
    column: a 2 B offset from its row, or a 4 B index) once, the block-row pointers, p
    read once and q written once."""
    return nnzb * (9 * value_bytes + col_bytes) + 4 * (n // 3 + 1) + 2 * 8 * n


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, literal_iters=20, budget_s=10.0, max_steps=3):
    """The oracle (plain C FP64, OpenMP over rows and blocks, sequential dot products)
    on the same workload: full steps of its fast mode (setup, then K Z, E^-1 and a solve
    to 1e-8; the rewrites the GPU uses, one merged coarse solve and a precomputed K Z,
    which take the literal mode's iterates, as the CPU tests pin), repeated until
    budget_s or max_steps.  The literal mode (two coarse Cholesky solves and an explicit
    K y per iteration) is timed on its first literal_iters iterations and scaled to the
    fast mode's iteration count.  Returns (line, oracle solution)."""
    import oracle

    steps, total, parts, r = 0, 0.0, [0.0, 0.0, 0.0], None
    while steps < max_steps and (steps == 0 or total < budget_s):
        t0 = time.perf_counter()
        o = oracle.Oracle.from_problem(p)
        t1 = time.perf_counter()
        o.prepare_fast()
        t2 = time.perf_counter()
        r = o.solve(p.f, tol=1e-8, fast=True)
        t3 = time.perf_counter()
        for i, d in enumerate((t1 - t0, t2 - t1, t3 - t2)):
            parts[i] += d
        total += t3 - t0
        steps += 1
        if steps < max_steps and total < budget_s:
            del o
    t3 = time.perf_counter()
    lit = o.solve(p.f, tol=1e-8, max_iter=literal_iters)
    t4 = time.perf_counter()
    del o
    setup_s, prep_s, solve_s = (x / steps for x in parts)
    lit_iter_s = (t4 - t3) / max(1, lit["iterations"])
    lit_step_s = setup_s + lit_iter_s * r["iterations"]
    line = {"value": p.n * steps / total, "unit": "DoF-solves/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} full steps of the workload with the oracle's fast mode, {total:.1f} s; per step: "
                      f"setup {setup_s:.1f} s, K Z and E^-1 {prep_s:.1f} s, solve to 1e-8 {solve_s:.1f} s "
                      f"({r['iterations']} iterations)",
            "cpu_model": cpu_model(), "iterations": r["iterations"], "status": r["status"],
            "solve_only_dof_solves_per_s": p.n / solve_s,
            "literal_mode": {"value": p.n / lit_step_s, "unit": "DoF-solves/s",
                             "sample": f"setup plus {lit['iterations']} literal iterations ({t4 - t3:.1f} s), "
                                       f"scaled to {r['iterations']} iterations"}}
    return line, r["u"]


def upload(p, dev):
    import numpy as np
    import torch
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    K = (t(p.k_rowptr, torch.int64), t(p.k_col, torch.int32), t(p.k_val, torch.float64))
    Z = (t(p.z_rowptr, torch.int64), t(p.z_col, torch.int32), t(p.z_val, torch.float64))
    return K, Z, t(p.block_ptr, torch.int32), t(p.f, torch.float64)


def run_steps(p, tensors, steps, warmup, stream, precision="fp64"):
    """warmup untimed then `steps` timed full steps (setup, solve to 1e-8, release),
    SpMV events on every TIMING_EVERY-th launch.  Returns a dict of the results and the
    last solution (device tensor)."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg
    K, Z, bp, f = tensors
    u = torch.empty_like(f)

    def step(timing):
        s = dpcg.Solver(p.n, *K, p.k, *Z, bp, stream=stream)
        if timing:
            s.set_timing(True, every=TIMING_EVERY)
        _, info = s.solve(f, u, tol=1e-8, precision=precision)
        tm = s.timing() if timing else None
        st = s.stats()
        s.close()
        return info, tm, st

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, spmv_ms, spmv_n, st = [], 0.0, 0, None
    for _ in range(steps):
        info, tm, st = step(True)
        infos.append(info)
        spmv_ms += tm["spmv_ms"]
        spmv_n += tm["spmv_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_launch_s = spmv_ms / 1e3 / max(spmv_n, 1)
    nbytes = spmv_bytes(st["nnzb"], p.n, value_bytes=8 if precision == "fp64" else 4,
                        col_bytes=st["spmv_col_bytes"])
    achieved = nbytes / per_launch_s / 1e9
    out = {"value": p.n * steps / dt, "unit": "DoF-solves/s", "ms_per_step": dt * 1e3 / steps,
           "ok": all(i["status"] == 0 and i["rel_res_true"] <= 1.5e-8 for i in infos),
           "iterations": infos[-1]["iterations"], "rel_res_true": infos[-1]["rel_res_true"],
           "setup_ms": float(np.mean([i["setup_ms"] for i in infos])),
           "solve_ms": float(np.mean([i["solve_ms"] for i in infos])),
           "spmv": {"kernel": "k_spmv_p<32, %s%s>" % ("double" if precision == "fp64" else "float",
                                                      ", short" if st["spmv_col_bytes"] == 2 else ""),
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "bytes_per_launch": nbytes, "launches": spmv_n, "avg_launch_us": per_launch_s * 1e6},
           "stats": st}
    if precision != "fp64":
        out["refinements"] = infos[-1]["refinements"]
        out["iterations_fp64"] = infos[-1]["iterations_fp64"]
    out["solve_only_dof_solves_per_s"] = p.n / (out["solve_ms"] / 1e3)
    return out, u


def run_batched(name, p, args, K, Z, bp, f, stream, nrhs=32):
    """The same steps with nrhs right-hand sides solved together (Case A of the batching
    workload: seeded random top-face tractions, N(0, 1) components per face node),
    every column to 1e-8."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg

    from fixtures import box
    F = box(name).random_top_tractions(nrhs, seed=2024)
    Fd = torch.as_tensor(F, device=f.device)
    U = torch.empty_like(Fd)

    def step(timing):
        s = dpcg.Solver(p.n, *K, p.k, *Z, bp, stream=stream)
        if timing:
            s.set_timing(True, every=TIMING_EVERY)
        _, infos = s.solve_batch(Fd, U, tol=1e-8)
        tm = s.timing() if timing else None
        s.close()
        return infos, tm

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    spmm_ms, spmm_n, last = 0.0, 0, None
    ok = True
    for _ in range(args.steps):
        infos, tm = step(True)
        last = infos
        spmm_ms += tm["spmv_ms"]
        spmm_n += tm["spmv_launches"]
        ok = ok and all(i["status"] == 0 and i["rel_res_true"] <= 1.5e-8 for i in infos)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nb = p.n // 3
    nnzb = None
    with dpcg.Solver(p.n, *K, p.k, *Z, bp, stream=stream) as s:
        nnzb = s.stats()["nnzb"]
    nbytes = nnzb * 76 + 4 * (nb + 1) + 2 * 8 * p.n * nrhs
    per_launch_s = spmm_ms / 1e3 / max(spmm_n, 1)
    achieved = nbytes / per_launch_s / 1e9
    return {"value": p.n * nrhs * args.steps / dt, "unit": "DoF-solves/s", "nrhs": nrhs,
            "ms_per_step": dt * 1e3 / args.steps, "ok": ok,
            "iterations_max": max(i["iterations"] for i in last),
            "iterations_col0": last[0]["iterations"], "solve_ms": last[0]["solve_ms"],
            "spmm": {"kernel": "k_bspmm<0>", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": nbytes, "launches": spmm_n,
                     "avg_launch_us": per_launch_s * 1e6}}


def run_many(args, count=16):
    """Case B of the batching workload: count independent systems (ne^3 meshes, ne uniform
    in [20, 48], penny cracks at random centres in [0.3, 0.7]^3), solved together by
    dpcg_solve_many (one launch per iteration phase for all) against the same systems
    solved one after another.  Solve time only: the systems are set up (and the SpMV
    lane groups tuned) once before timing."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg
    from fixtures import uneven_systems

    t_gen = time.perf_counter()
    ps = uneven_systems(count, seed=16, ne_range=(20, 48))
    t_gen = time.perf_counter() - t_gen
    solvers = [dpcg.Solver.from_problem(p, "cuda:0") for p in ps]
    fs = [torch.as_tensor(p.f, device="cuda:0") for p in ps]
    us = [torch.empty_like(f) for f in fs]
    for s in solvers:
        s.autotune(5)
    for _ in range(max(1, args.warmup)):
        dpcg.solve_many(solvers, fs, us)
        for s, f, u in zip(solvers, fs, us):
            s.solve(f, u)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos = dpcg.solve_many(solvers, fs, us)
    torch.cuda.synchronize()
    t_many = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        singles = [s.solve(f, u)[1] for s, f, u in zip(solvers, fs, us)]
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    for s in solvers:
        s.close()
    n_tot = sum(p.n for p in ps)
    same_its = all(a["iterations"] == b["iterations"] for a, b in zip(infos, singles))
    return {"value": n_tot / t_many, "unit": "DoF-solves/s", "systems": count, "dofs_total": n_tot,
            "dofs_min": min(p.n for p in ps), "dofs_max": max(p.n for p in ps),
            "ms_together": t_many * 1e3, "ms_sequential": t_seq * 1e3,
            "sequential_dof_solves_per_s": n_tot / t_seq, "speedup": t_seq / t_many,
            "ok": all(i["status"] == 0 for i in infos), "same_iterations_as_single": same_its,
            "iterations_max": max(i["iterations"] for i in infos), "generation_s": t_gen}


def run_subdomain(name, args, p, nsds=(8, 4)):
    """The paper's subdomain-sized block-Jacobi blocks (Sec. 3.4): the same system
    renumbered subdomain by subdomain with one block per subdomain of an nsd^3 box
    partition (explicit inverses from batched Gauss-Jordan sweeps at setup, a dense
    matrix-vector apply each iteration).  Full steps (setup + solve to 1e-8) as in the
    headline; the larger blocks take fewer steps."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg
    from fixtures import with_subdomain_blocks

    out = {}
    dev = torch.device("cuda:0")
    for nsd in nsds:
        q, _ = with_subdomain_blocks(name, nsd, p)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
        K = (t(q.k_rowptr, torch.int64), t(q.k_col, torch.int32), t(q.k_val, torch.float64))
        Z = (t(q.z_rowptr, torch.int64), t(q.z_col, torch.int32), t(q.z_val, torch.float64))
        bp = t(q.block_ptr, torch.int32)
        f = t(q.f, torch.float64)
        u = torch.empty_like(f)

        def step():
            s = dpcg.Solver(q.n, *K, q.k, *Z, bp)
            _, info = s.solve(f, u, tol=1e-8)
            st = s.stats()
            s.close()
            return info, st

        steps = max(1, args.steps // (1 if nsd > 4 else 5))
        for _ in range(max(1, args.warmup // 2)):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(steps):
            info, st = step()
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sizes = np.diff(q.block_ptr)
        out[f"{nsd}^3"] = {
            "value": q.n * steps / dt, "unit": "DoF-solves/s", "steps": steps, "ms_per_step": dt * 1e3 / steps,
            "ok": all(i["status"] == 0 and i["rel_res_true"] <= 1.5e-8 for i in infos),
            "iterations": infos[-1]["iterations"], "blocks": int(len(sizes)),
            "block_dofs": [int(sizes.min()), int(sizes.max())],
            "setup_ms": float(np.mean([i["setup_ms"] for i in infos])),
            "solve_ms": float(np.mean([i["solve_ms"] for i in infos])),
            "inverse_bytes_per_iteration": 8 * int(st["dense_values"]),
        }
        del K, Z, bp, f, u, q
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="penny80", choices=sorted(WORKLOADS))
    ap.add_argument("--extra-workload", default="penny40", choices=sorted(WORKLOADS),
                    help="workload of the 32-RHS, uneven-systems and subdomain-block lines")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison line")
    ap.add_argument("--no-extra", action="store_true", help="skip every line on the extra workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-right-hand-side and uneven-systems lines")
    ap.add_argument("--no-many", action="store_true", help="skip the uneven-systems line only")
    ap.add_argument("--no-subdomain", action="store_true", help="skip the subdomain-block comparison lines")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run N plain 512 MiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this method is built and measured on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg
    from fixtures import load

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    print(f"[bench] {args.workload}: generating the system", file=sys.stderr, flush=True)
    p = load(args.workload)
    tensors = upload(p, dev)

    if args.calibrate_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.calibrate_copy):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    print(f"[bench] {args.workload}: FP64 steps", file=sys.stderr, flush=True)
    fp64, u64 = run_steps(p, tensors, args.steps, args.warmup, stream)
    if not fp64["ok"]:
        print(f"solve failed: {fp64}", file=sys.stderr)
        return 1
    stats = fp64.pop("stats")
    rf = fp64["spmv"]
    out = {
        "metric": METRIC,
        "value": fp64["value"],
        "unit": "DoF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n_dofs": p.n,
                   "n_std": p.meta["n_std"], "n_enr": p.meta["n_enr"], "k": p.k, "nnzb": stats["nnzb"],
                   "nblocks": p.nblocks, "parallelism": "single GPU"},
        "iterations": fp64["iterations"],
        "setup_ms": fp64["setup_ms"],
        "solve_ms": fp64["solve_ms"],
        "solve_only_dof_solves_per_s": fp64["solve_only_dof_solves_per_s"],
        "rel_res_true": fp64["rel_res_true"],
        "roofline": {"bound": "hbm", "achieved": rf["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": rf["frac"], "traffic": spmv_traffic(args.workload), "kernel": rf["kernel"],
                     "bytes_per_launch": rf["bytes_per_launch"], "launches": rf["launches"],
                     "avg_launch_us": rf["avg_launch_us"]},
    }
    um = None
    if not args.no_mixed:
        print(f"[bench] {args.workload}: mixed-precision steps", file=sys.stderr, flush=True)
        mixed, um = run_steps(p, tensors, args.steps, args.warmup, stream, precision="mixed")
        mixed.pop("stats")
        mixed["spmv_fp32_values"] = mixed.pop("spmv")
        mixed["speedup_vs_fp64"] = mixed["value"] / fp64["value"]
        out["mixed"] = mixed
    if not args.no_cpu_baseline:
        print(f"[bench] {args.workload}: CPU oracle", file=sys.stderr, flush=True)
        line, uo = cpu_baseline(p)
        out["cpu_baseline"] = line
        nref = np.linalg.norm(uo)
        out["error_vs_oracle"] = {"fp64": float(np.linalg.norm(u64.cpu().numpy() - uo) / nref)}
        if um is not None:
            out["error_vs_oracle"]["mixed"] = float(np.linalg.norm(um.cpu().numpy() - uo) / nref)
    # distance of both answers from the solution of K u = f, taken as the FP64 solve to a
    # residual of 1e-12 (four decades below the stopping test): the two paths stop at
    # different iterates of residual <= 1e-8, so their distance to each other is not
    # their accuracy
    with dpcg.Solver(p.n, *tensors[0], p.k, *tensors[1], tensors[2], stream=stream) as s:
        ut, it = s.solve(tensors[3], tol=1e-12)
    ut = ut.cpu().numpy()
    nt = np.linalg.norm(ut)
    out["error_vs_tight_solve"] = {"tol": 1e-12, "iterations": it["iterations"],
                                   "fp64": float(np.linalg.norm(u64.cpu().numpy() - ut) / nt)}
    if um is not None:
        out["error_vs_tight_solve"]["mixed"] = float(np.linalg.norm(um.cpu().numpy() - ut) / nt)
    del tensors, u64, um
    torch.cuda.empty_cache()

    if not args.no_extra:
        name = args.extra_workload
        print(f"[bench] {name}: extra lines", file=sys.stderr, flush=True)
        q = load(name)
        tq = upload(q, dev)
        line, _ = run_steps(q, tq, args.steps, args.warmup, stream)
        line.pop("stats")
        line["workload"] = name
        line["n_dofs"] = q.n
        out["fp64_" + name] = line
        if not args.no_batched:
            out["batched"] = run_batched(name, q, args, tq[0], tq[1], tq[2], tq[3], stream)
            if not args.no_many:
                out["many_systems"] = run_many(args)
        if not args.no_subdomain:
            out["subdomain_blocks"] = run_subdomain(name, args, q)
        del tq
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
