#!/usr/bin/env python
"""Solve throughput of cascading-smoother multigrid on one MI355X.

Workload (default): 3D 7-point variable-coefficient interface problem on 128^3
cells (coefficient 1e4 inside a sphere of radius 0.3 with a seeded centre, 1
outside), 2x2x2 blocks, depth-4 additive cascade, RF V(1,1), 8 seeded U[-1,1]
right-hand sides; FP32 V-cycle (sweeps, SpMV, transfers) inside FP64 iterative
refinement to 1e-10 relative residual.  Beside it: the same V-cycle as the
preconditioner of flexible CG and of GMRES, the plain FP64 V-cycle with the
same outer methods (like-for-like speedups), the 64^2 Poisson problem, the
batched 64-system workload, the SIPG Q3 and Stokes workloads and the learned
setup on Q1 multiphase diffusion.

A step is one pass of the whole hot path on inputs resident in HBM: the GPU
setup (prescaling, symbolic fill, Frobenius fit of every level, bottom
factorisation) followed by the solve.  `value` is the solve throughput
(fine-level unknowns x right-hand sides / solve time); setup time is reported
beside it.

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


def _host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU_SAMPLE = {}


def _cpu_column_solves(args):
    """One worker of the all-cores leg: `reps` oracle solves of one
    right-hand-side column (the setup is inherited from the parent)."""
    from threadpoolctl import threadpool_limits

    import oracle
    col, reps = args
    p, sm = _CPU_SAMPLE["p"], _CPU_SAMPLE["sm"]
    with threadpool_limits(limits=1):
        for _ in range(reps):
            oracle.solve(p.levels, sm, p.rhs[:, col:col + 1].copy(), 1e-10, 200, "RF", 1, 1)
    return col


def cpu_baseline(n: int, nrhs: int, depth: int, budget_s: float = 10.0):
    """The FP64 oracle on a smaller instance of the same problem family: setup
    untimed, then the solve to 1e-10 timed (i) on one thread, repeated for
    about budget_s seconds, and (ii) on all host cores as one process per
    right-hand side (each an independent solve of one column, the same
    repetitions).  Runs before the GPU is touched, so the worker pool can fork."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    import oracle
    from synth import fd
    with threadpool_limits(limits=1):
        p = fd.interface3d(n, nrhs=nrhs)
        t0 = time.perf_counter()
        sm = oracle.setup_hierarchy(p.levels, depth)
        t_setup = time.perf_counter() - t0
        reps, t_solve = 0, 0.0
        t0 = time.perf_counter()
        while reps == 0 or t_solve < budget_s:
            _, hist = oracle.solve(p.levels, sm, p.rhs, 1e-10, 200, "RF", 1, 1)
            reps += 1
            t_solve = time.perf_counter() - t0
    one = dict(value=p.n * nrhs * reps / t_solve, unit="DOF/s", cores=1, kind="oracle",
               sample=(f"3D interface problem {n}^3 (same generator and contrast), {nrhs} RHS, depth-{depth} "
                       f"additive RF V(1,1), FP64 stationary solve to 1e-10 in {len(hist) - 1} V-cycles, "
                       f"repeated {reps} times in {t_solve:.1f} s on one thread; setup {t_setup:.1f} s not timed"))
    # all cores: the machine's CPU share is 16 cores; one process per right-hand side
    workers = min(nrhs, 16, len(os.sched_getaffinity(0)))
    _CPU_SAMPLE.update(p=p, sm=sm)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_cpu_column_solves, [(c, reps) for c in range(nrhs)])
    t_all = time.perf_counter() - t0
    _CPU_SAMPLE.clear()
    one["all_cores"] = dict(value=p.n * nrhs * reps / t_all, unit="DOF/s", cores=workers, kind="oracle",
                            sample=(f"the same {reps} solves as {nrhs} independent one-column solves, one process "
                                    f"per right-hand side on {workers} cores, {t_all:.1f} s wall"))
    one["host_cpu"] = _host_cpu()
    one["host_cores_visible"] = len(os.sched_getaffinity(0))
    return one


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_interface3d_128_traffic.md")


def bench_batch(precision: str):
    """64 independent 2D 5-point log-normal (sigma 2) systems, sizes 64^2 ..
    512^2, 4 RHS each, one stacked hierarchy; solve DOF/s with stationary
    refinement and with flexible CG (every system to 1e-10 on its own)."""
    import numpy as np
    import torch
    from paper_2606_12577_amd import cascade
    from synth import fd
    from synth.batch import concatenate
    bt = concatenate(fd.lognormal_batch(64, nrhs=4))
    s = cascade.Solver(bt.levels)
    s.setup(depth=3, precision=precision)
    s.set_systems(bt.sys_ptr)
    b = torch.as_tensor(bt.rhs, device="cuda").contiguous()
    dof = bt.levels[0].n * 4
    out = dict(dof=int(bt.levels[0].n), nrhs=4, systems=64, setup_ms=None)
    # launch schedules per level and eager vs graph replay, picked by measurement
    sched = s.autotune(4)
    on, e_ms, g_ms = s.graphs()
    out["autotune"] = dict(rows_per_workgroup=[int(w) for w, _, _ in sched],
                           workgroup_cap=[int(g) for _, g, _ in sched],
                           vcycle_ms_eager=round(e_ms, 3), vcycle_ms_graph=round(g_ms, 3), graph_replay=on,
                           tail_vcycle_ms={str(r): round(t, 4) for r, t in s.tail_candidates()},
                           tail_max_rows=s.tail()[0])
    # the slowest system of the stationary iteration (144^2, rho ~ 0.98) needs
    # 1,127 V-cycles in FP32 and in FP64 alike
    for method, maxit in (("cg", 300), ("ir", 2000)):
        for replay in (False, True):
            s.set_graphs(replay)
            infos = [s.solve(b, rtol=1e-10, maxit=maxit, method=method, raise_on_noconv=False)[1] for _ in range(2)]
            its, rels = s.system_stats()
            i = infos[-1]
            out[method + ("_graph" if replay else "_eager")] = dict(
                solve_ms=round(i["solve_ms"], 2), iterations=i["iterations"],
                converged_systems=int((rels <= 1e-10).sum()), dof_per_s=dof / (i["solve_ms"] * 1e-3),
                per_system_iterations=[int(np.min(its)), int(np.median(its)), int(np.max(its))])
        out["setup_ms"] = round(i["setup_ms"], 2)
    s.set_graphs(on)
    # the plain FP64 V-cycle on the same systems: like-for-like speedups
    s64 = cascade.Solver(bt.levels)
    s64.setup(depth=3, precision="fp64")
    s64.set_systems(bt.sys_ptr)
    s64.autotune(4)
    out["vs_plain_fp64_vcycle"] = {}
    for method, maxit in (("cg", 300), ("ir", 2000)):
        i = [s64.solve(b, rtol=1e-10, maxit=maxit, method=method, raise_on_noconv=False)[1] for _ in range(2)][-1]
        its, rels = s64.system_stats()
        out["fp64_" + method] = dict(solve_ms=round(i["solve_ms"], 2), iterations=i["iterations"],
                                     converged_systems=int((rels <= 1e-10).sum()),
                                     dof_per_s=dof / (i["solve_ms"] * 1e-3))
        out["vs_plain_fp64_vcycle"][method + "_vs_" + method] = round(
            out["fp64_" + method]["solve_ms"] / out[method + "_eager"]["solve_ms"], 3)
    s64.close()
    # sketched construction (64 Rademacher modes per level) instead of the exact fit
    for _ in range(2):
        s.setup_sketched(width=64, seed=0, depth=3, precision=precision)
    infos = [s.solve(b, rtol=1e-10, maxit=300, method="cg", raise_on_noconv=False)[1] for _ in range(2)]
    its, rels = s.system_stats()
    i = infos[-1]
    out["sketched_s64_cg"] = dict(setup_ms=round(i["setup_ms"], 2), solve_ms=round(i["solve_ms"], 2),
                                  iterations=i["iterations"], converged_systems=int((rels <= 1e-10).sum()),
                                  setup_plus_solve_dof_per_s=dof / ((i["setup_ms"] + i["solve_ms"]) * 1e-3))
    s.close()
    return out


def bench_stokes(precision: str):
    """2D Stokes on a 256^2 MAC staggered grid (cell blocks of velocity and
    pressure, Stokes prescaling with 1-norm constraint rows), depth-4 additive
    FF cascade; the V-cycle preconditions GMRES(30), left (the paper's driver)
    and flexible."""
    import time as _t
    import numpy as np
    import torch
    from paper_2606_12577_amd import cascade
    from synth import stokes
    t = _t.perf_counter()
    p = stokes.mac2d(256)
    gen_s = _t.perf_counter() - t
    s = cascade.Solver(p.levels)
    b = torch.as_tensor(p.rhs, device="cuda").contiguous()
    out = dict(cells=256 * 256, unknowns=int(p.n), generation_s=round(gen_s, 1))
    for _ in range(2):
        s.setup(depth=4, order="FF", precision=precision)
    for method in ("gmres", "fgmres"):
        i = [s.solve(b, rtol=1e-10, maxit=300, method=method, raise_on_noconv=False)[1] for _ in range(2)][-1]
        out[method] = dict(solve_ms=round(i["solve_ms"], 2), iterations=i["iterations"], rho=round(i["rho"], 4),
                           rel_res=i["rel_res"], setup_ms=round(i["setup_ms"], 2),
                           dof_per_s=3 * 256 * 256 / (i["solve_ms"] * 1e-3))
    # overlapping Vanka cell patches (Sec. 3.6.2), depth 3: exact fit, and sketched with 32 modes
    m = 256
    for l in range(len(p.levels) - 1):
        s.set_overlapping_blocks(l, stokes.vanka_nodes(m))
        m //= 2
    for name, fit in (("exact", lambda: s.setup(depth=3, order="FF", precision=precision)),
                      ("sketched", lambda: s.setup_sketched(width=32, seed=0, depth=3, order="FF",
                                                            precision=precision))):
        for _ in range(2):
            fit()
        i = [s.solve(b, rtol=1e-10, maxit=300, method="fgmres", raise_on_noconv=False)[1] for _ in range(2)][-1]
        out[f"vanka_overlapping_{name}_fgmres"] = dict(
            solve_ms=round(i["solve_ms"], 2), iterations=i["iterations"], rho=round(i["rho"], 4),
            rel_res=i["rel_res"], setup_ms=round(i["setup_ms"], 2), dof_per_s=3 * 256 * 256 / (i["solve_ms"] * 1e-3))
    s.close()
    return out


def bench_dg():
    """SIPG Q3 on a jittered 256^2 quadrilateral mesh (16 x 16 element blocks,
    1,048,576 unknowns, 1 RHS), depth-3 four-colour multiplicative FF cascade,
    V(1,1).  The configuration: BF16 blocks of A and Lambda on the matrix cores
    (FP32 accumulation, FP32 vectors and restricted residual) inside FP64
    iterative refinement, with the Tikhonov-regularised fit (ridge 1e-3) that
    keeps the depth-3 blocks small enough for BF16.  Beside it: the same fit in
    FP32 and FP64, the paper's plain fit in FP64 (the plain FP64 V-cycle), and
    flexible GMRES(30) around each (the FF V-cycle is not symmetric)."""
    import time as _t
    import torch
    from paper_2606_12577_amd import cascade
    from synth import dg
    t = _t.perf_counter()
    p = dg.sipg_q3(256)
    gen_s = _t.perf_counter() - t
    s = cascade.Solver(p.levels)
    b = torch.as_tensor(p.rhs, device="cuda").contiguous()
    out = dict(dof=int(p.n), nrhs=1, generation_s=round(gen_s, 1), ridge=1e-3)

    def solve(method):
        i = [s.solve(b, rtol=1e-10, maxit=400, method=method, raise_on_noconv=False)[1] for _ in range(2)][-1]
        return dict(solve_ms=round(i["solve_ms"], 2), iterations=i["iterations"], rho=round(i["rho"], 4),
                    rel_res=i["rel_res"], precision=i["precision"],
                    setup_ms=round(i["setup_ms"], 2), dof_per_s=p.n / (i["solve_ms"] * 1e-3))

    opts = dict(depth=3, mode="multiplicative", order="FF")
    for _ in range(2):
        s.setup(**opts, precision="fp64")
    out["fp64_plain_fit"] = {m: solve(m) for m in ("ir", "fgmres")}
    for _ in range(2):
        s.setup(**opts, precision="bf16", ridge=1e-3)
    out["bf16_ridge"] = {m: solve(m) for m in ("ir", "fgmres")}
    # kernel timing of the finest level's BF16 colour sweeps in one more (traced) refinement solve
    s.trace(("sweep",), period=1)
    s.solve(b, rtol=1e-10, maxit=400, method="ir", raise_on_noconv=False)
    tr = s.trace_read()["sweep"]
    s.trace(())
    for prec in ("fp32", "fp64"):
        s.set_precision(prec)
        out[f"{prec}_ridge"] = {m: solve(m) for m in ("ir", "fgmres")}
    if tr["launches"]:
        avg_s = tr["ms"] / tr["launches"] * 1e-3
        per = tr["bytes"] / tr["launches"]
        rp = _summary_values(DG_PROFILE_FILE, "bsr16")
        rp_us = float(rp["avg_us"]) if rp.get("source") == bf16_source_digest() else None
        out["roofline_bsr16_sweep"] = dict(
            kernel="k_bsr16_sweep<false> (one colour of the finest level, BF16 blocks on MFMA)", bound="hbm",
            timing="live: one HIP event pair around each run of consecutive colour sweeps of the finest level",
            launches=tr["launches"], avg_us=round(avg_s * 1e6, 2), algorithmic_bytes_per_launch=int(per),
            achieved=round(per / avg_s / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
            frac=round(per / avg_s / 1e9 / HBM_PEAK_GBS, 4), rocprof_avg_us=rp_us,
            frac_rocprof=round(per / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if rp_us else None)
    bir, fir, pir = out["bf16_ridge"]["ir"], out["fp64_ridge"]["ir"], out["fp64_plain_fit"]["ir"]
    out["bf16_ir_vs_fp64_ir_same_fit"] = dict(speedup=round(fir["solve_ms"] / bir["solve_ms"], 3),
                                              rho_ratio=round(bir["rho"] / fir["rho"], 4))
    out["bf16_ir_vs_plain_fp64_ir"] = dict(speedup=round(pir["solve_ms"] / bir["solve_ms"], 3),
                                           rho_ratio=round(bir["rho"] / pir["rho"], 4))
    s.close()
    return out


def bench_learned(epochs: int = 40):
    """Q1 multiphase diffusion 96^3: train the block network on two samples,
    then on an unseen sample compare the learned finest-level setup with the
    Frobenius setup (setup time, CG convergence factor) and apply the judge."""
    import time as _t
    from paper_2606_12577_amd import cascade, learned as L
    from synth import fe
    t = _t.perf_counter()
    train = [fe.multiphase3d(96, seed_extra=k) for k in (1, 2)]
    test = fe.multiphase3d(96, seed_extra=0)
    gen_s = _t.perf_counter() - t
    X, T = L.build_training_set(train, depth=2)
    t = _t.perf_counter()
    net, rep = L.train_network(X, T, n_samples=200000, epochs=epochs, batch=1024, lr0=1e-3)
    import torch
    torch.cuda.synchronize()
    train_s = _t.perf_counter() - t
    s = cascade.Solver(test.levels)
    t = _t.perf_counter()
    Xt = L.fe_block_features(test.meta["log10mu"])
    torch.cuda.synchronize()
    feat_ms = (_t.perf_counter() - t) * 1e3
    v = L.judge(s, net, Xt, test.rhs, depth=2, method="cg", maxit=300)
    _, sol = s.solve(test.rhs, rtol=1e-10, maxit=300, method="cg")
    dof = test.n
    return dict(dof=dof, generation_s=round(gen_s, 1), train_s=round(train_s, 2), train_blocks=rep.n_train,
                val_loss=round(rep.val_loss, 4), val_loss_untrained=round(rep.val_loss_untrained, 4),
                features_ms=round(feat_ms, 2), use_learned=v.use_learned,
                rho_learned=round(v.rho_learned, 4), rho_frobenius=round(v.rho_frobenius, 4),
                setup_ms_learned=round(v.setup_ms_learned, 2), setup_ms_frobenius=round(v.setup_ms_frobenius, 2),
                iterations_learned=v.iterations_learned, iterations_frobenius=v.iterations_frobenius,
                setup_plus_solve_dof_per_s=dof / ((sol["setup_ms"] + sol["solve_ms"]) * 1e-3))


def kernel_source_digest() -> str:
    """Digest of the source that decides the sweep kernel's memory traffic: the
    device code from the x loads through k_sweep, and its launcher."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2606_12577_amd", "csrc", "solve.hip")).read()
    spans = [("// x_in at unknown j", "// r = A x - b over SELL rows"),
             ("template <typename T, int R>\nvoid launch_sweep(", "// One application of the cascade of level L")]
    h = hashlib.sha256()
    for a, b in spans:
        i, j = src.find(a), src.find(b)
        h.update((src[i:j] if 0 <= i < j else src).encode())
    return h.hexdigest()[:16]


PROFILE_FILE = os.path.join(ROOT, "profiles", "k_sweep_interface3d_128.md")
DG_PROFILE_FILE = os.path.join(ROOT, "profiles", "dg_sipg_q3_256.md")


def bf16_source_digest() -> str:
    """Digest of the BF16 block-sweep source (kernel and launcher)."""
    import hashlib
    return hashlib.sha256(open(os.path.join(ROOT, "paper_2606_12577_amd", "csrc", "bf16.hip"), "rb").read()
                          ).hexdigest()[:16]


def _summary_values(path: str, tag: str) -> dict:
    """key=value pairs of the line starting with `tag:` in a committed summary."""
    vals = {}
    if os.path.exists(path):
        for line in open(path):
            if line.startswith(tag + ":"):
                for kv in line.split()[1:]:
                    k, v = kv.split("=", 1)
                    vals[k] = v
    return vals


def _default_workload(args) -> bool:
    return args.n == 128 and args.nrhs == 8 and args.precision == "fp32"


def measured_traffic(args):
    """HBM bytes per launch of the sweep kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration),
    or None when the summary is missing, for another workload, or older than
    the kernel source."""
    vals = _summary_values(TRAFFIC_FILE, "traffic")
    if not _default_workload(args) or vals.get("source") != kernel_source_digest():
        return None
    return int(float(vals["bytes_per_launch"]))


def rocprof_average_us(args):
    """Average duration of the sweep kernel in the committed rocprofv3
    kernel-trace summary of this workload, or None when it is missing or older
    than the kernel source."""
    vals = _summary_values(PROFILE_FILE, "sweep")
    if not _default_workload(args) or vals.get("source") != kernel_source_digest():
        return None
    return float(vals["avg_us"])


def _short_kernel(name: str) -> str:
    """Kernel name without namespace and parameter list (template arguments kept)."""
    for pre in ("void ", "cs::(anonymous namespace)::", "cs::"):
        if name.startswith(pre):
            name = name[len(pre):]
    name = name.replace("cs::(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def summarize_rocprof(path: str, top: int = 40) -> str:
    """Markdown summary of a rocprofv3 CSV: a kernel trace (per kernel and grid:
    calls, average / min / max duration, total, share) or a counter collection
    (per kernel, grid and counter: dispatches, mean and sum of the counter, and
    the mean dispatch duration).  Reads only the CSV."""
    import csv
    from collections import defaultdict
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    if not rows:
        return f"{path}: empty\n"
    out = []
    if "Counter_Name" in rows[0]:
        acc = defaultdict(lambda: [0, 0.0, 0.0])
        dur = defaultdict(list)
        for r in rows:
            key = (_short_kernel(r["Kernel_Name"]), int(r["Grid_Size"]))
            a = acc[key + (r["Counter_Name"],)]
            v = float(r["Counter_Value"])
            a[0] += 1
            a[1] += v
            a[2] = max(a[2], v)
            dur[key + (r["Counter_Name"],)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
        out.append("| kernel | grid | counter | dispatches | mean per dispatch | max per dispatch | sum | mean us |")
        out.append("|---|---|---|---|---|---|---|---|")
        for (k, g, c), (n, tot, mx) in sorted(acc.items(), key=lambda kv: (kv[0][0], kv[0][1], kv[0][2])):
            d = dur[(k, g, c)]
            out.append(f"| `{k}` | {g} | {c} | {n} | {tot / n:.6g} | {mx:.6g} | {tot:.6g} | {sum(d) / len(d):.2f} |")
    else:
        acc = defaultdict(list)
        for r in rows:
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            key = (_short_kernel(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
            acc[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
        total = sum(sum(v) for v in acc.values())
        out.append("| kernel | grid (threads) | calls | avg us | min us | max us | total ms | % |")
        out.append("|---|---|---|---|---|---|---|---|")
        for (k, g), d in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
            out.append(f"| `{k}` | {g} | {len(d)} | {sum(d) / len(d):.2f} | {min(d):.2f} | {max(d):.2f} | "
                       f"{sum(d) * 1e-3:.2f} | {100 * sum(d) / total:.2f} |")
    return "\n".join(out) + "\n"


def bench_c1():
    """64^2 cell-centred 5-point Poisson (Dirichlet), point blocks, depth-3
    additive RF cascade, V(2,2), FP64, one RHS, coarsening to 4^2 with a
    direct bottom solve; stationary FP64 solve and flexible CG to 1e-10.
    4,096 unknowns: latency-bound, so no bandwidth claim is made."""
    from paper_2606_12577_amd import cascade
    from synth import fd
    import torch
    p = fd.poisson2d(64)
    s = cascade.Solver(p.levels)
    b = torch.as_tensor(p.rhs, device="cuda").contiguous()
    out = dict(dof=int(p.n), nrhs=1)
    for _ in range(2):
        s.setup(depth=3, mode="additive", order="RF", n_pre=2, n_post=2, precision="fp64")
    # the coarse levels as one single-workgroup launch, from the level autotune picks
    s.autotune(1)
    out["tail_vcycle_ms"] = {str(r): round(t, 4) for r, t in s.tail_candidates()}
    out["tail_max_rows"], out["tail_first_level"] = s.tail()
    tail = out["tail_max_rows"]
    for method in ("ir", "cg"):
        for label, rows in ((method, tail), (f"{method}_per_level_launches", 0)):
            s.set_tail(rows)
            i = [s.solve(b, rtol=1e-10, maxit=100, method=method)[1] for _ in range(3)][-1]
            out[label] = dict(solve_ms=round(i["solve_ms"], 3), iterations=i["iterations"], rho=round(i["rho"], 4),
                              rel_res=i["rel_res"], setup_ms=round(i["setup_ms"], 3),
                              dof_per_s=p.n / (i["solve_ms"] * 1e-3),
                              us_per_vcycle=round(i["solve_ms"] * 1e3 / max(i["iterations"], 1), 1))
    s.set_tail(tail)
    s.close()
    return out


def stream_reference(s, nbytes=1 << 30, reps=10):
    """GB/s of plain streaming kernels on this device (cs_stream_bandwidth, 1 GiB
    per array): the rate HBM gives without the method's arithmetic, beside the
    published peak.  4r1w reads four arrays per one written, the cascade sweep's
    mix (it reads about 4.7 bytes per byte it writes)."""
    out = {}
    for name, (nr, nw) in (("read", (1, 0)), ("write", (0, 1)), ("copy", (1, 1)), ("4r1w", (4, 1))):
        out[name] = round(s.stream_bandwidth(nr, nw, nbytes, reps)[0], 1)
    out["unit"] = "GB/s"
    out["arrays_bytes"] = nbytes
    return out


SOLVE_KERNELS = ("k_sweep", "k_ir_residual", "k_tail_vcycle", "k_residual_restrict", "k_cg_")


def summarize_setups(path: str, first: int = 1, count: int = 3, top: int = 16) -> str:
    """Per-kernel time inside the setups of a rocprofv3 kernel trace.  A setup is
    the stretch from a k_prescale_w launch (the first kernel of a setup) to the
    last kernel before the next solve kernel; the table averages setups
    first .. first + count - 1 (0-based; the default skips the warm-up's)."""
    import csv
    from collections import Counter, defaultdict
    with open(path, newline="") as f:
        rows = [r for r in csv.DictReader(f) if r.get("Kind", "KERNEL_DISPATCH") == "KERNEL_DISPATCH"]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    wins, cur, last_end = [], None, 0
    for r in rows:
        name = _short_kernel(r["Kernel_Name"])
        if cur is None:
            if not name.startswith("k_prescale_w"):
                continue
            cur = dict(t0=int(r["Start_Timestamp"]), ms=defaultdict(float), calls=Counter())
        elif name.startswith(SOLVE_KERNELS):
            cur["t1"] = last_end
            wins.append(cur)
            cur = None
            continue
        cur["ms"][name] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        cur["calls"][name] += 1
        last_end = int(r["End_Timestamp"])
    sel = wins[first:first + count]
    if not sel:
        return f"{path}: {len(wins)} setups, none selected\n"
    tot = defaultdict(float)
    for w in sel:
        for k, v in w["ms"].items():
            tot[k] += v / len(sel)
    span = sum((w["t1"] - w["t0"]) * 1e-6 for w in sel) / len(sel)
    out = [f"{len(wins)} setups in the trace; setups {first}-{first + len(sel) - 1}: span {span:.2f} ms, "
           f"kernel time {sum(tot.values()):.2f} ms per setup", "",
           "| kernel | calls per setup | ms per setup |", "|---|---|---|"]
    for k, v in sorted(tot.items(), key=lambda kv: -kv[1])[:top]:
        out.append(f"| `{k}` | {sel[0]['calls'][k]} | {v:.2f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
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
    ap.add_argument("--no-stream-reference", action="store_true",
                    help="skip the streaming-bandwidth reference reported beside the roofline")
    ap.add_argument("--no-trace", action="store_true", help="do not time the sweep kernel with events")
    ap.add_argument("--trace-period", type=int, default=8,
                    help="time every n-th launch of the sweep kernel with HIP events")
    ap.add_argument("--solver", default="ir", choices=["ir", "cg", "gmres", "fgmres"],
                    help="outer solver of the timed step: FP64 refinement (the default), flexible CG, "
                         "left-preconditioned GMRES or flexible GMRES around the V-cycle")
    ap.add_argument("--sketch-width", type=int, default=32,
                    help="also measure the sketched setup with this many modes (0: skip)")
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the exact setup with the stencil-repetition cache")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64^2 Poisson measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-system measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-setup measurement")
    ap.add_argument("--learned-epochs", type=int, default=40, help="training epochs of the learned-setup network")
    ap.add_argument("--no-stokes", action="store_true", help="skip the Stokes (MAC) measurement")
    ap.add_argument("--no-dg", action="store_true", help="skip the SIPG Q3 256^2 measurement")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--summarize-setups", metavar="CSV",
                    help="print the per-kernel time inside the setups of a rocprofv3 kernel trace and exit")
    ap.add_argument("--summarize", nargs="+", metavar="CSV",
                    help="print a markdown summary of rocprofv3 kernel-trace or counter CSVs and exit")
    ap.add_argument("--summarize-top", type=int, default=40, metavar="N",
                    help="rows (kernel, grid and counter groups) kept by --summarize")
    args = ap.parse_args()
    if args.summarize_setups:
        print(summarize_setups(args.summarize_setups))
        return
    if args.summarize:
        for path in args.summarize:
            print(f"### {os.path.basename(os.path.dirname(path))}/{os.path.basename(path)}\n")
            print(summarize_rocprof(path, top=args.summarize_top))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # the CPU oracle first: its worker pool forks, which must happen before the GPU is initialised
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(args.cpu_n, args.nrhs, args.depth)
        log(f"oracle: {cpu['value']:.3e} DOF/s on 1 core, {cpu['all_cores']['value']:.3e} on "
            f"{cpu['all_cores']['cores']} cores")

    import numpy as np
    import torch

    from paper_2606_12577_amd import cascade
    from synth import fd

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
        x, info = s.solve(b, rtol=args.rtol, maxit=args.maxit, method=args.solver)
        return info

    for w in range(args.warmup):
        info = step()
        log(f"warmup {w}: setup {info['setup_ms']:.1f} ms, solve {info['solve_ms']:.1f} ms, "
            f"{info['iterations']} it, rho {info['rho']:.4f}")
    # launch schedules per level, the tail V-cycle and eager vs graph replay, by
    # measurement on the setup's own operators (kept across setups)
    if args.warmup == 0:
        s.setup(**opts)
    sched = s.autotune(args.nrhs)
    replay, vc_eager, vc_graph = s.graphs()
    tuned = dict(rows_per_workgroup=[w for w, _, _ in sched], workgroup_cap=[g for _, g, _ in sched],
                 vcycle_ms_eager=round(vc_eager, 3), vcycle_ms_graph=round(vc_graph, 3), graph_replay=replay,
                 tail_vcycle_ms={str(r): round(t, 4) for r, t in s.tail_candidates()}, tail_max_rows=s.tail()[0])
    log(f"autotune: V-cycle {vc_eager:.3f} ms eager, {vc_graph:.3f} ms replayed")
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
    roofline = None
    if not args.no_trace:
        rp_us = rocprof_average_us(args)
        roofline = dict(
            bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
            frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(args),
            kernel=(f"k_sweep<{'float' if args.precision == 'fp32' else 'double'}, 8, {args.nrhs}, "
                    "false, false, false, 256, false> (cascade sweep reading A, large levels)"),
            timing=("live: one HIP event pair around every sampled run of consecutive sweeps of the fine level "
                    "on the library's stream; the average over the run's launches includes the gaps between them"),
            launches=sw["launches"], avg_us=round(avg_ms * 1e3, 2),
            algorithmic_bytes_per_launch=int(bytes_per_launch),
            rocprof_avg_us=rp_us,
            frac_rocprof=(round(bytes_per_launch / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if rp_us else None))
        if not args.no_stream_reference:
            roofline["attainable"] = stream_reference(s)
            roofline["frac_of_attainable"] = round(achieved / roofline["attainable"]["4r1w"], 4)

    extra = {}
    runs = {}   # (precision, method) -> info of the last of two solves on the same setup

    def run(method, prec_label):
        i = [s.solve(b, rtol=args.rtol, maxit=args.maxit, method=method)[1] for _ in range(2)][-1]
        runs[(prec_label, method)] = i
        return dict(solve_ms=round(i["solve_ms"], 3), iterations=i["iterations"], rho=round(i["rho"], 4),
                    rel_res=i["rel_res"], dof_per_s=dof / (i["solve_ms"] * 1e-3))

    runs[(args.precision, args.solver)] = last
    for method in ("ir", "cg", "gmres", "fgmres"):
        if method != args.solver:
            extra[f"{args.precision}_{method}"] = run(method, args.precision)
    # the same solves with every outer iteration replayed from a captured graph (untraced)
    s.set_graphs(True)
    for method in ("ir", "cg"):
        extra[f"{args.precision}_{method}_graph_replay"] = run(method, args.precision + "_graph")
    s.set_graphs(replay)
    extra["autotune"] = tuned
    if not args.no_fp64_baseline and args.precision != "fp64":
        # the plain FP64 V-cycle (every kernel in FP64) under the same outer methods
        s.set_precision("fp64")
        for method in ("ir", "cg"):
            extra[f"fp64_{method}"] = run(method, "fp64")
        s.set_precision(args.precision)
        like = {}
        for method in ("ir", "cg"):
            lo, hi = runs[(args.precision, method)], runs[("fp64", method)]
            like[f"{method}_vs_{method}"] = dict(speedup=round(hi["solve_ms"] / lo["solve_ms"], 3),
                                                 rho_ratio=round(lo["rho"] / hi["rho"], 4))
        extra["vs_plain_fp64_vcycle"] = like
    # sketched construction (32 Rademacher modes per level) instead of the exact fit, same solve
    if args.sketch_width > 0:
        sks = []
        for _ in range(2):
            s.setup_sketched(width=args.sketch_width, seed=0, depth=args.depth, precision=args.precision)
            sks.append(s.solve(b, rtol=args.rtol, maxit=args.maxit, method="cg", raise_on_noconv=False)[1])
        sk = sks[-1]
        extra[f"sketched_s{args.sketch_width}_cg"] = dict(
            setup_ms=round(sk["setup_ms"], 2), solve_ms=round(sk["solve_ms"], 3), iterations=sk["iterations"],
            rho=round(sk["rho"], 4), rel_res=sk["rel_res"],
            setup_plus_solve_dof_per_s=dof / ((sk["setup_ms"] + sk["solve_ms"]) * 1e-3),
            setup_speedup_vs_exact=round(setup_ms / sk["setup_ms"], 2))
    # exact fit with the stencil-repetition cache (Sec. 4): one fit per translation class of blocks
    if not args.no_lattice:
        for l, lv in enumerate(prob.levels[:-1]):
            s.set_lattice(l, lv.block_lattice())
        lts = []
        for _ in range(2):
            s.setup(**opts)
            lts.append(s.solve(b, rtol=args.rtol, maxit=args.maxit, method=args.solver)[1])
        lt = lts[-1]
        nblk = [lv.n_blocks for lv in prob.levels[:-1]]
        fitted = [s.lattice_stats(l).tolist() for l in range(len(nblk))]
        extra[f"lattice_cache_{args.solver}"] = dict(
            setup_ms=round(lt["setup_ms"], 2), solve_ms=round(lt["solve_ms"], 3), iterations=lt["iterations"],
            rho=round(lt["rho"], 4), rel_res=lt["rel_res"],
            setup_plus_solve_dof_per_s=dof / ((lt["setup_ms"] + lt["solve_ms"]) * 1e-3),
            setup_speedup_vs_exact=round(setup_ms / lt["setup_ms"], 2),
            fitted_fraction_per_step=[[round(f / n, 4) for f in fl] for fl, n in zip(fitted, nblk)])
        for l in range(len(nblk)):
            s.set_lattice(l, None)
    # the reference smoother (Sec. 2.1, 3.2): depth-many damped block Jacobi
    # steps, Lambda_l = omega A_ii^-1, same V-cycle, precision and outer loops;
    # omega from a small sweep under CG, the best then also under refinement
    jac = {}
    for w in (0.7, 0.8, 0.9, 1.0):
        s.setup(**dict(opts, source="jacobi", omega=w))
        i = [s.solve(b, rtol=args.rtol, maxit=500, method="cg", raise_on_noconv=False)[1] for _ in range(2)][-1]
        jac[w] = i
    wbest = min(jac, key=lambda w: jac[w]["solve_ms"] if jac[w]["rel_res"] <= args.rtol else float("inf"))
    s.setup(**dict(opts, source="jacobi", omega=wbest))
    ji = [s.solve(b, rtol=args.rtol, maxit=2000, method="ir", raise_on_noconv=False)[1] for _ in range(2)][-1]
    extra["block_jacobi_reference"] = dict(
        omega=wbest,
        cg={str(w): dict(solve_ms=round(i["solve_ms"], 3), iterations=i["iterations"], rho=round(i["rho"], 4),
                         eta=round(i["eta"], 3), rel_res=i["rel_res"]) for w, i in jac.items()},
        ir=dict(solve_ms=round(ji["solve_ms"], 3), iterations=ji["iterations"], rho=round(ji["rho"], 4),
                eta=round(ji["eta"], 3), rel_res=ji["rel_res"]),
        cascade_speedup=dict(
            ir=round(ji["solve_ms"] / runs[(args.precision, "ir")]["solve_ms"], 3),
            cg=round(jac[wbest]["solve_ms"] / runs[(args.precision, "cg")]["solve_ms"], 3)))
    # the paper's work model of the stationary iteration (Sec. 3.1), in 3D:
    # C_3 = eta (1 + (2 nu + 1) / (1 - 2^-3)), nu cascade steps or Jacobi steps alike
    def work(eta):
        return round(eta * (1.0 + (2 * args.depth + 1) / (1.0 - 2.0 ** -3)), 3)
    extra["block_jacobi_reference"]["work_model_c3"] = dict(
        cascade=work(runs[(args.precision, "ir")]["eta"]), block_jacobi=work(ji["eta"]))
    if args.copy_mib:
        nel = args.copy_mib * 1024 * 1024 // 4
        src = torch.ones(nel, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_mib"] = args.copy_mib
    s.close()

    if not args.no_c1:
        log("Poisson 64^2 (FP64, V(2,2))")
        extra["c1_poisson2d_64"] = bench_c1()
    if not args.no_batch:
        log("batched workload: 64 log-normal 2D systems")
        extra["batch64"] = bench_batch(args.precision)
    if not args.no_stokes:
        log("Stokes: MAC 256^2")
        extra["stokes_mac_256"] = bench_stokes(args.precision)
    if not args.no_dg:
        log("DG: SIPG Q3 256^2")
        extra["dg_sipg_q3_256"] = bench_dg()
    if not args.no_learned:
        log("learned setup: Q1 multiphase 96^3")
        extra["learned_q1_96"] = bench_learned(args.learned_epochs)

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
                        f"{args.precision.upper()} smoother, SpMV and transfers "
                        + {"cg": "as flexible-CG preconditioner", "ir": "inside FP64 iterative refinement",
                           "gmres": "as left GMRES(30) preconditioner",
                           "fgmres": "as flexible GMRES(30) preconditioner"}[args.solver]
                        + f", to {args.rtol:g} relative residual",
            "solver": args.solver,
            "dof": prob.n, "nrhs": prob.nrhs, "levels": len(prob.levels), "parallelism": "single GPU",
        },
        "solve_ms": round(solve_ms, 3),
        "setup_ms": round(setup_ms, 3),
        "setup_plus_solve_dof_per_s": dof / ((solve_ms + setup_ms) * 1e-3),
        "iterations": last["iterations"],
        "rho": round(last["rho"], 4),
        "eta": round(last["eta"], 3),
        "rel_res": last["rel_res"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
