"""Parity at full size for the batched workload: 64 independent 2D log-normal
systems (64^2 .. 512^2 cells, 4 RHS each) in one stacked hierarchy, depth-3
additive RF cascade, FP32 V-cycle in flexible CG - bench.py's batch leg.

  * the smoothers of the smallest and the median system (every level) against
    the oracle's setup of that system alone, and sampled blocks of the largest
    system's finest level against the oracle's patch fit (per-block bounds
    from the oracle's condition numbers, tests/parity.py);
  * the solve: every system reaches 1e-10 on its own residual, and the
    smallest system needs the iterations of the oracle's FP64 flexible CG on
    that system alone (within one: the V-cycle runs in FP32 here).
"""
import numpy as np
import pytest

import oracle as O
from parity import check_level_smoothers, record, scalar_bound
from synth import fd
from synth.batch import concatenate
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu

DEPTH = 3


@pytest.fixture(scope="module")
def full(gpu_lib):
    probs = fd.lognormal_batch(64, nrhs=4)
    bt = concatenate(probs)
    print(f"[fullsize-batch] {len(probs)} systems, {bt.levels[0].n} unknowns", flush=True)
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=DEPTH, precision="fp32")
    s.set_systems(bt.sys_ptr)
    return probs, bt, s


def block_offset(bt, q, l):
    """First block of system q on batch level l (systems stacked in bt.order)."""
    off = 0
    for t in bt.order:
        p = bt.problems[t]
        if len(p.levels) <= l:
            continue
        if t == q:
            return off
        off += p.levels[l].n_blocks
    raise ValueError("system not on this level")


def test_batch_fullsize_system_smoothers(full):
    probs, bt, s = full
    sizes = np.array([p.n for p in probs])
    order = np.argsort(sizes, kind="stable")
    for q in (int(order[0]), int(order[len(order) // 2])):
        sm = O.setup_hierarchy(probs[q].levels, DEPTH)
        for l in range(len(probs[q].levels) - 1):
            off = block_offset(bt, q, l)
            nblk = probs[q].levels[l].n_blocks
            check_level_smoothers(s, sm[l], l, DEPTH, f"batch64 system {q}", rows=slice(off, off + nblk))
    q = int(order[-1])
    A0 = probs[q].levels[0].A
    rng = stream(7, TEST)
    centres = sorted({0, A0.shape[0] - 1, *rng.integers(0, A0.shape[0], size=3).tolist()})
    loc, cond = O.fit_local(A0, 1, DEPTH, centres, with_cond=True)
    off = block_offset(bt, q, 0)
    for ell in range(1, DEPTH + 1):
        g = s.get_smoother(0, ell)
        for c in centres:
            o = loc[c][ell - 1]
            e = np.linalg.norm(g[off + c] - o) / np.linalg.norm(o)
            bound = scalar_bound(cond[c][:ell])
            assert record(f"batch64 largest system block {c} Lambda_{ell}", e, bound) <= 1.0, (c, ell, e)


def test_batch_fullsize_solve(full):
    probs, bt, s = full
    x, info = s.solve(bt.rhs, rtol=1e-10, maxit=300, method="cg")
    its, rels = s.system_stats()
    print(f"[fullsize-batch] CG: {info['iterations']} it (max), per system {its.min()}..{its.max()}, "
          f"{info['solve_ms']:.1f} ms", flush=True)
    assert np.all(rels <= 1e-10)
    xs = bt.split(x.cpu().numpy())
    for q, p in enumerate(probs):
        r = p.rhs - p.levels[0].A @ xs[q]
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1.5e-10, q
    q = int(np.argmin([p.n for p in probs]))
    sm = O.setup_hierarchy(probs[q].levels, DEPTH)
    p = probs[q]
    _, hist = O.fcg(p.levels[0].A, lambda r: O.vcycle(p.levels, sm, r, "RF", 1, 1), p.rhs, 1e-10, 300)
    pos = int(np.flatnonzero(np.asarray(bt.order) == q)[0])   # stats are in the stacked order
    assert abs(int(its[pos]) - (len(hist) - 1)) <= 1, (its[pos], len(hist) - 1)


def test_batch_fullsize_refinement_fp32_vs_fp64(full, gpu_lib):
    """The configured outer loop: FP64 refinement around the FP32 V-cycle brings
    every system to 1e-10, in the V-cycles the plain FP64 V-cycle needs on the
    same systems (the stationary iteration's rate is the V-cycle's convergence
    factor, so equal counts mean equal factors up to the last step; the
    slowest system, rho ~ 0.98, needs about 1,100)."""
    probs, bt, s = full
    _, info = s.solve(bt.rhs, rtol=1e-10, maxit=2000, method="ir")
    its32, rels32 = s.system_stats()
    s64 = gpu_lib.Solver(bt.levels)
    s64.setup(depth=DEPTH, precision="fp64")
    s64.set_systems(bt.sys_ptr)
    _, info64 = s64.solve(bt.rhs, rtol=1e-10, maxit=2000, method="ir")
    its64, rels64 = s64.system_stats()
    s64.close()
    print(f"[fullsize-batch] refinement: FP32 V-cycle {info['iterations']} (max), {info['solve_ms']:.1f} ms; "
          f"FP64 V-cycle {info64['iterations']}, {info64['solve_ms']:.1f} ms", flush=True)
    assert np.all(rels32 <= 1e-10) and np.all(rels64 <= 1e-10)
    for q in range(len(probs)):
        d = abs(int(its32[q]) - int(its64[q]))
        bound = 1 + 0.02 * int(its64[q])
        assert record(f"batch64 system {q} refinement V-cycles FP32 vs FP64", d, bound) <= 1.0, (q, its32[q], its64[q])
