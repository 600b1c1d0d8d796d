#!/usr/bin/env python
"""Solve throughput of cascading-smoother multigrid on one MI355X.

Workload (default): 3D 7-point variable-coefficient interface problem on 128^3
cells (coefficient 1e4 inside a sphere of radius 0.3 with a seeded centre, 1
outside), 2x2x2 blocks, depth-4 additive cascade, RF V(1,1), 8 seeded U[-1,1]
right-hand sides; FP32 V-cycle (sweeps, SpMV, transfers) inside FP64 iterative
refinement to 1e-10 relative residual.

A step is one pass of the whole hot path on inputs resident in HBM: the GPU
setup (prescaling, symbolic fill, Frobenius fit of every level, bottom
factorisation) followed by the solve.  `value` is the solve throughput
(fine-level unknowns x right-hand sides / solve time); setup time is reported
beside it.  The plain FP64 V-cycle solve on the same setup gives the speedup.

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solve DOF/s to 1e-10 rel. residual, mixed/learned vs plain FP64 V-cycle"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(n: int, nrhs: int, depth: int):
    """The FP64 oracle, single-threaded, on a smaller instance of the same
    problem family (setup untimed, solve to 1e-10 timed)."""
    from threadpoolctl import threadpool_limits

    import oracle
    from synth import fd
    with threadpool_limits(limits=1):
        p = fd.interface3d(n, nrhs=nrhs)
        t0 = time.perf_counter()
        sm = oracle.setup_hierarchy(p.levels, depth)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, hist = oracle.solve(p.levels, sm, p.rhs, 1e-10, 200, "RF", 1, 1)
        t_solve = time.perf_counter() - t0
    return dict(value=p.n * nrhs / t_solve, unit="DOF/s", cores=1, kind="oracle",
                sample=(f"3D interface problem {n}^3 (same generator and contrast), {nrhs} RHS, depth-{depth} "
                        f"additive RF V(1,1), FP64 stationary solve to 1e-10 in {len(hist) - 1} V-cycles; "
                        f"solve {t_solve:.2f} s timed, setup {t_setup:.2f} s not timed"))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_interface3d_128_traffic.md")


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("solve.hip", "cs_internal.h"):
        with open(os.path.join(ROOT, "paper_2606_12577_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(args):
    """HBM bytes per launch of the sweep kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration),
    or None when the summary is missing, for another workload, or older than
    the kernel source."""
    if args.n != 128 or args.nrhs != 8 or args.precision != "fp32" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("source") != kernel_source_digest():
        return None
    return int(float(vals["bytes_per_launch"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--depth", type=int, default=4)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=200)
    ap.add_argument("--cpu-n", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true", help="do not time the sweep kernel with events")
    ap.add_argument("--trace-period", type=int, default=8,
                    help="time every n-th launch of the sweep kernel with HIP events")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_12577_amd import cascade
    from synth import fd

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    prob = fd.interface3d(args.n, nrhs=args.nrhs)
    log(f"generated {prob.name}: {prob.n} unknowns x {prob.nrhs} RHS, {len(prob.levels)} levels "
        f"in {time.perf_counter() - t0:.1f} s")
    s = cascade.Solver(prob.levels, device=0)
    b = torch.as_tensor(prob.rhs, device=dev).contiguous()
    opts = dict(depth=args.depth, mode="additive", order="RF", n_pre=1, n_post=1, precision=args.precision)

    def step():
        s.setup(**opts)
        x, info = s.solve(b, rtol=args.rtol, maxit=args.maxit)
        return info

    for w in range(args.warmup):
        info = step()
        log(f"warmup {w}: setup {info['setup_ms']:.1f} ms, solve {info['solve_ms']:.1f} ms, "
            f"{info['iterations']} it, rho {info['rho']:.4f}")
    torch.cuda.synchronize()
    if not args.no_trace:
        s.trace(("sweep",), period=args.trace_period)
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr = s.trace_read()
    s.trace(())
    for k, info in enumerate(infos):
        log(f"step {k}: setup {info['setup_ms']:.1f} ms, solve {info['solve_ms']:.1f} ms, "
            f"{info['iterations']} it, rel_res {info['rel_res']:.2e}")
    solve_ms = float(np.mean([i["solve_ms"] for i in infos]))
    setup_ms = float(np.mean([i["setup_ms"] for i in infos]))
    dof = prob.n * prob.nrhs
    value = dof / (solve_ms * 1e-3)
    last = infos[-1]

    sw = tr["sweep"]
    avg_ms = sw["ms"] / max(sw["launches"], 1)
    bytes_per_launch = sw["bytes"] / max(sw["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = None if args.no_trace else dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(args),
                    kernel=(f"k_sweep<{'float' if args.precision == 'fp32' else 'double'}, 8, {args.nrhs}, "
                            "false, false, false, 256> (cascade sweep reading A, large levels)"),
                    launches=sw["launches"], avg_us=round(avg_ms * 1e3, 2),
                    algorithmic_bytes_per_launch=int(bytes_per_launch))

    extra = {}
    if not args.no_fp64_baseline:
        s.set_precision("fp64")
        _, i64 = s.solve(b, rtol=args.rtol, maxit=args.maxit)
        ms64 = []
        for _ in range(2):
            _, i64 = s.solve(b, rtol=args.rtol, maxit=args.maxit)
            ms64.append(i64["solve_ms"])
        ms64 = float(np.mean(ms64))
        extra["fp64_vcycle"] = dict(solve_ms=round(ms64, 2), iterations=i64["iterations"],
                                    rho=round(i64["rho"], 4), dof_per_s=dof / (ms64 * 1e-3))
        extra["speedup_vs_fp64_vcycle"] = round(ms64 / solve_ms, 3)
        extra["rho_ratio_vs_fp64"] = round(last["rho"] / i64["rho"], 4)
        s.set_precision(args.precision)
    if args.copy_mib:
        nel = args.copy_mib * 1024 * 1024 // 4
        src = torch.ones(nel, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_mib"] = args.copy_mib

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(args.cpu_n, args.nrhs, args.depth)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point interface problem {args.n}^3, contrast 1e4 sphere r=0.3, "
                        f"{args.nrhs} RHS, 2x2x2 blocks, depth-{args.depth} additive cascade, RF V(1,1), "
                        f"{args.precision.upper()} V-cycle in FP64 iterative refinement to {args.rtol:g}",
            "dof": prob.n, "nrhs": prob.nrhs, "levels": len(prob.levels), "parallelism": "single GPU",
        },
        "solve_ms": round(solve_ms, 3),
        "setup_ms": round(setup_ms, 3),
        "setup_plus_solve_dof_per_s": dof / ((solve_ms + setup_ms) * 1e-3),
        "iterations": last["iterations"],
        "rho": round(last["rho"], 4),
        "rel_res": last["rel_res"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
