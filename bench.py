#!/usr/bin/env python3
"""Benchmark: DoF-solves per second of the deflated block-Jacobi CG on one MI355X.

A step is one pass of the whole method over one synthetic cracked-body system:
setup (block-Jacobi inverses, K Z, E = Z^T K Z and E^-1, device layout) followed by
one solve of K u = f to relative residual 1e-8 and the release of the handle.  The
inputs (K, Z, blocks, f as device arrays) are resident in HBM before timing starts.

Prints one JSON line with the throughput, the SpMV kernel's HBM roofline fraction
(algorithmic bytes / average launch duration measured with HIP events on the
library's stream during the timed steps) and the CPU oracle timed on this host.
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

# HBM bytes moved by one k_spmv_p launch on penny40, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the launches of iterations
# that did work), each scaled by what the same counter reads for a 512 MiB device copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources with these
# digests: after any change to them the figure is reported as null until re-measured.
SPMV_TRAFFIC = {
    "workload": "penny40",
    "sources": {
        "paper_2111_09294_amd/csrc/kernels.hip": "60fe0a48b57125dca7338279e4cbb335fc9bc8626137cc3e6124bb84713b9bc3",
        "paper_2111_09294_amd/csrc/dpcg_internal.h": "c0ba109d4262e5c5c843b0b0f6bd48ea92e9f470dca8de0f2b5f3d72bdf9d8c6"
    },
    "fetch_bytes": 171350110,
    "write_bytes": 2029550,
}


def _source_digests():
    import hashlib
    out = {}
    for rel in ("paper_2111_09294_amd/csrc/kernels.hip", "paper_2111_09294_amd/csrc/dpcg_internal.h"):
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
METRIC = "DoF-solves/sec to rel. residual 1e-8 + SpMV HBM GB/s fraction; FP64 vs mixed/batched"
WORKLOADS = {
    "penny40": "40^3 hex8 unit cube, curved penny crack (R=0.25, z=0.5+0.3 rho^2), Heaviside + branch "
               "enrichment within r_e=0.05, 4^3 subdomains, clamped bottom, unit top traction, FP64, tol 1e-8",
    "edge10": "10^3 hex8 unit cube, planar edge crack x=0.5 z<0.45, Heaviside + branch enrichment within "
              "r_e=0.15, 2^3 subdomains, clamped bottom, unit top traction, FP64, tol 1e-8",
    "penny80": "80^3 hex8 unit cube, curved penny crack, r_e=0.05, 8^3 subdomains, FP64, tol 1e-8",
}


# The roofline's kernel duration comes from start/stop events recorded by every
# TIMING_EVERY-th SpMV launch of the timed steps: events on each launch add about 8 us to
# every iteration (0.8 ms per solve), sampling keeps the timed run close to an untimed one.
TIMING_EVERY = 8


def spmv_bytes(nnzb, n, value_bytes=8):
    """Algorithmic bytes of one q = K p launch: each 3x3 block (9 values + a 4 B column
    index) once, the block-row pointers, p read once and q written once."""
    return nnzb * (9 * value_bytes + 4) + 4 * (n // 3 + 1) + 2 * 8 * n


def cpu_baseline(p, budget_s=12.0):
    """The oracle (plain C FP64, OpenMP row loops) on the same workload, full steps."""
    import oracle

    t0 = time.perf_counter()
    reps = 0
    its = None
    while True:
        o = oracle.Oracle.from_problem(p)
        r = o.solve(p.f, tol=1e-8)
        del o
        its = r["iterations"]
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 20:
            break
    dt = time.perf_counter() - t0
    return {"value": p.n * reps / dt, "unit": "DoF-solves/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{reps} full steps (setup + solve to 1e-8, {its} iterations) of the same workload, "
                      f"{dt:.1f} s"}


def run_mixed(step, p, args, stats):
    """The same steps with precision "mixed" (FP64 refinement around inner solves on
    binary32 copies of K and of the block inverses), to the same true FP64 residual."""
    import numpy as np
    import torch

    for _ in range(args.warmup):
        step(False, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, spmv_ms, spmv_n = [], 0.0, 0
    for _ in range(args.steps):
        info, tm, _ = step(True, "mixed")
        infos.append(info)
        spmv_ms += tm["spmv_ms"]
        spmv_n += tm["spmv_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bad = [i for i in infos if i["status"] != 0 or i["rel_res_true"] > 1e-8]
    per_launch_s = spmv_ms / 1e3 / max(spmv_n, 1)
    nbytes = spmv_bytes(stats["nnzb"], p.n, value_bytes=4)
    achieved = nbytes / per_launch_s / 1e9
    return {"value": p.n * args.steps / dt, "unit": "DoF-solves/s", "ms_per_step": dt * 1e3 / args.steps,
            "ok": not bad, "iterations": infos[-1]["iterations"], "refinements": infos[-1]["refinements"],
            "rel_res_true": infos[-1]["rel_res_true"],
            "setup_ms": float(np.mean([i["setup_ms"] for i in infos])),
            "solve_ms": float(np.mean([i["solve_ms"] for i in infos])),
            "spmv_fp32_values": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": nbytes,
                                 "launches": spmv_n, "avg_launch_us": per_launch_s * 1e6}}


def run_batched(p, args, K, Z, bp, f, stream, nrhs=32):
    """The same steps with nrhs right-hand sides solved together (Case A of the batching
    workload: seeded random top-face tractions, N(0, 1) components per face node),
    every column to 1e-8."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg

    from fixtures import box
    F = box(args.workload).random_top_tractions(nrhs, seed=2024)
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


def run_large(name="penny80", steps=2):
    """The FP64 path on the 80^3 configuration (1.66M DoFs): its matrix (1.38 GB of block
    values) is far larger than the 256 MB last-level cache, so the SpMV figure there is
    an HBM figure; at 40^3 an iteration's data (about 250 MB) can partly stay in that
    cache.  Full steps (setup + solve to 1e-8), SpMV events on every 8th launch."""
    import numpy as np
    import torch

    import paper_2111_09294_amd as dpcg
    from fixtures import load

    t_gen = time.perf_counter()
    q = load(name)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    K = (t(q.k_rowptr, torch.int64), t(q.k_col, torch.int32), t(q.k_val, torch.float64))
    Z = (t(q.z_rowptr, torch.int64), t(q.z_col, torch.int32), t(q.z_val, torch.float64))
    bp = t(q.block_ptr, torch.int32)
    f = t(q.f, torch.float64)
    u = torch.empty_like(f)

    def step(timing):
        s = dpcg.Solver(q.n, *K, q.k, *Z, bp)
        if timing:
            s.set_timing(True, every=TIMING_EVERY)
        _, info = s.solve(f, u, tol=1e-8)
        tm = s.timing() if timing else None
        st = s.stats()
        s.close()
        return info, tm, st

    step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, spmv_ms, spmv_n = [], 0.0, 0
    for _ in range(steps):
        info, tm, st = step(True)
        infos.append(info)
        spmv_ms += tm["spmv_ms"]
        spmv_n += tm["spmv_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_launch_s = spmv_ms / 1e3 / max(spmv_n, 1)
    nbytes = spmv_bytes(st["nnzb"], q.n)
    achieved = nbytes / per_launch_s / 1e9
    out = {"value": q.n * steps / dt, "unit": "DoF-solves/s", "workload": name, "n_dofs": q.n, "k": q.k,
           "nnzb": st["nnzb"], "steps": steps, "ms_per_step": dt * 1e3 / steps,
           "ok": all(i["status"] == 0 and i["rel_res_true"] <= 1.5e-8 for i in infos),
           "iterations": infos[-1]["iterations"],
           "setup_ms": float(np.mean([i["setup_ms"] for i in infos])),
           "solve_ms": float(np.mean([i["solve_ms"] for i in infos])),
           "spmv": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "bytes_per_launch": nbytes, "launches": spmv_n, "avg_launch_us": per_launch_s * 1e6},
           "generation_s": t_gen}
    del K, Z, bp, f, u, q
    torch.cuda.empty_cache()
    return out


def run_subdomain(args, p, nsds=(8, 4)):
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
        q, _ = with_subdomain_blocks(args.workload, nsd, p)
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
    ap.add_argument("--workload", default="penny40", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison line")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-right-hand-side comparison line")
    ap.add_argument("--no-subdomain", action="store_true", help="skip the subdomain-block comparison lines")
    ap.add_argument("--no-large", action="store_true", help="skip the 80^3 FP64 line")
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
    p = load(args.workload)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    K = (t(p.k_rowptr, torch.int64), t(p.k_col, torch.int32), t(p.k_val, torch.float64))
    Z = (t(p.z_rowptr, torch.int64), t(p.z_col, torch.int32), t(p.z_val, torch.float64))
    bp = t(p.block_ptr, torch.int32)
    f = t(p.f, torch.float64)
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream()

    def step(timing, precision="fp64"):
        s = dpcg.Solver(p.n, *K, p.k, *Z, bp, stream=stream)
        if timing:
            s.set_timing(True, every=TIMING_EVERY)
        _, info = s.solve(f, u, tol=1e-8, precision=precision)
        tm = s.timing() if timing else None
        st = s.stats()
        s.close()
        return info, tm, st

    if args.calibrate_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.calibrate_copy):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, spmv_ms, spmv_n = [], 0.0, 0
    stats = None
    for _ in range(args.steps):
        info, tm, stats = step(True)
        infos.append(info)
        spmv_ms += tm["spmv_ms"]
        spmv_n += tm["spmv_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for info in infos:
        if info["status"] != 0 or info["rel_res_true"] > 1.5e-8:
            print(f"solve failed: {info}", file=sys.stderr)
            return 1
    ms_step = dt * 1e3 / args.steps
    solve_ms = float(np.mean([i["solve_ms"] for i in infos]))
    setup_ms = float(np.mean([i["setup_ms"] for i in infos]))
    per_launch_s = spmv_ms / 1e3 / max(spmv_n, 1)
    nbytes = spmv_bytes(stats["nnzb"], p.n)
    achieved = nbytes / per_launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": p.n * args.steps / dt,
        "unit": "DoF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n_dofs": p.n,
                   "n_std": p.meta["n_std"], "n_enr": p.meta["n_enr"], "k": p.k, "nnzb": stats["nnzb"],
                   "nblocks": p.nblocks, "parallelism": "single GPU"},
        "iterations": infos[-1]["iterations"],
        "setup_ms": setup_ms,
        "solve_ms": solve_ms,
        "solve_only_dof_solves_per_s": p.n / (solve_ms / 1e3),
        "rel_res_true": infos[-1]["rel_res_true"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": spmv_traffic(args.workload),
                     "kernel": "k_spmv_p", "bytes_per_launch": nbytes, "launches": spmv_n,
                     "avg_launch_us": per_launch_s * 1e6},
    }
    if not args.no_mixed:
        out["mixed"] = run_mixed(step, p, args, stats)
    if not args.no_batched:
        out["batched"] = run_batched(p, args, K, Z, bp, f, stream)
        out["many_systems"] = run_many(args)
    if not args.no_subdomain:
        out["subdomain_blocks"] = run_subdomain(args, p)
    if not args.no_large:
        out["large_80"] = run_large()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
