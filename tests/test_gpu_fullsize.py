"""Parity at the benchmark's full size: the 128^3 interface problem with 8
right-hand sides, 2x2x2 blocks, depth-4 additive cascade, FP32 V-cycle in
FP64 refinement - the configuration bench.py times.

The oracle cannot fit all 262,144 blocks of this level in reasonable time, so
  * sampled smoother blocks are compared with the oracle's fit of the same
    blocks on their radius-nu neighbourhood (exact: Lambda_{l,i} depends on A
    only within l block layers of i);
  * the V-cycle is compared with the oracle's V-cycle at full size with the
    same injected smoothers (block Jacobi weights, every level);
  * the solve is checked by properties: 1e-10 reached, monotone residuals, and
    the FP32 convergence factor within 5% of the FP64 V-cycle's.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from parity import VCYCLE_TOL, check_vec, record, scalar_bound
from synth import fd
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu

N = 128
DEPTH = 4


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def blockdiag_inverse(A, nb):
    C = sp.coo_matrix(A)
    m = (C.row // nb) == (C.col // nb)
    B = A.shape[0] // nb
    D = np.zeros((B, nb, nb))
    D[C.row[m] // nb, C.row[m] % nb, C.col[m] % nb] = C.data[m]
    return np.linalg.inv(D)


@pytest.fixture(scope="module")
def full(gpu_lib):
    p = fd.interface3d(N, nrhs=8)
    print(f"[fullsize] problem {p.name}: {p.n} unknowns, {len(p.levels)} levels", flush=True)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=DEPTH, mode="additive", order="RF", precision="fp32")
    return p, s


def test_fullsize_sampled_smoother_blocks(full):
    p, s = full
    A0 = p.levels[0].A
    mu = fd.sphere_mu(N, np.array(p.meta["centre"]), 0.3, 1e4)
    blk = (p.levels[0].cells // 8).ravel()
    lo = np.full(blk.max() + 1, np.inf)
    hi = np.zeros(blk.max() + 1)
    np.minimum.at(lo, blk, mu.ravel())
    np.maximum.at(hi, blk, mu.ravel())
    mixed = np.flatnonzero(lo != hi)
    inside = np.flatnonzero(lo == 1e4)
    B = len(lo)
    rng = stream(2, TEST)
    centres = sorted({0, B - 1, 63, int(mixed[0]), int(mixed[len(mixed) // 2]), int(inside[len(inside) // 2]),
                      *rng.integers(0, B, size=3).tolist()})
    loc, cond = O.fit_local(A0, 8, DEPTH, centres, with_cond=True)
    for ell in range(1, DEPTH + 1):
        g = s.get_smoother(0, ell)
        for c in centres:
            o = loc[c][ell - 1]
            e = np.linalg.norm(g[c] - o) / np.linalg.norm(o)
            bound = scalar_bound(cond[c][:ell])   # from the conditioning met in the block's patch
            assert record(f"interface3d_128 block {c} Lambda_{ell}", e, bound) <= 1.0, (c, ell, e, bound)


def test_fullsize_solve_fp32_ir(full):
    p, s = full
    s.set_precision("fp32")
    x32, i32 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    h = i32["history"]
    print(f"[fullsize] fp32+IR: {i32['iterations']} it, rho {i32['rho']:.4f}, {i32['solve_ms']:.1f} ms")
    assert i32["rel_res"] <= 1e-10
    assert all(b < a for a, b in zip(h, h[1:]))
    s.set_precision("fp64")
    x64, i64 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    print(f"[fullsize] fp64: {i64['iterations']} it, rho {i64['rho']:.4f}, {i64['solve_ms']:.1f} ms")
    assert i32["rho"] <= 1.05 * i64["rho"]
    assert rel(x32.cpu().numpy(), x64.cpu().numpy()) <= 1e-8
    r = p.rhs - p.levels[0].A @ x32.cpu().numpy()
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-10


def test_fullsize_vcycle_injected_smoothers(full):
    """Runs last: replaces the fitted smoothers."""
    p, s = full
    weights = (0.55, 0.7, 0.85, 1.0)
    sm = []
    for l, lv in enumerate(p.levels[:-1]):
        D = blockdiag_inverse(lv.A, lv.block_size)
        lams = [w * D for w in weights]
        for ell in range(DEPTH):
            s.set_smoother(l, ell + 1, lams[ell])
        sm.append(dict(lam=lams, colours=None))
    s.set_precision("fp64")
    g = s.vcycle(p.rhs).cpu().numpy()
    o = O.vcycle(p.levels, sm, p.rhs, "RF")
    e = check_vec(g, o, VCYCLE_TOL, "interface3d_128 FP64 V-cycle, injected smoothers")
    print(f"[fullsize] FP64 V-cycle vs oracle: {e:.2e}")
    s.set_precision("fp32")
    g32 = s.vcycle(p.rhs).cpu().numpy()
    e32 = check_vec(g32, o, 1e-5, "interface3d_128 FP32 V-cycle vs FP64 oracle, injected smoothers")
    print(f"[fullsize] FP32 V-cycle vs FP64 oracle: {e32:.2e}")


def test_fullsize_lattice_cache(gpu_lib, full):
    """The stencil-repetition cache at full size: every block's smoother equals
    the uncached fit (blockwise 1e-10: no oracle fit of all blocks exists at
    this size), and sampled members of the bulk class and their
    representatives equal the oracle's patch fit (per-block bounds from the
    patch's conditioning)."""
    p, _ = full   # the shared solver holds injected smoothers by now: fit a fresh uncached one
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=DEPTH, mode="additive", order="RF", precision="fp32")
    t = gpu_lib.Solver(p.levels)
    for l, lv in enumerate(p.levels[:-1]):
        t.set_lattice(l, lv.block_lattice())
    t.setup(depth=DEPTH, mode="additive", order="RF", precision="fp32")
    fitted, rep = t.lattice_stats(0, classes=True)
    B = p.levels[0].n_blocks
    print(f"[fullsize] lattice cache: fitted per step {fitted.tolist()} of {B}", flush=True)
    assert fitted[0] < B // 10 and np.all(np.diff(fitted) >= 0)
    for ell in range(1, DEPTH + 1):
        g, o = t.get_smoother(0, ell), s.get_smoother(0, ell)
        num = np.linalg.norm((g - o).reshape(B, -1), axis=1)
        den = np.linalg.norm(o.reshape(B, -1), axis=1)
        assert record(f"interface3d_128 lattice-cached vs uncached Lambda_{ell}", (num / den).max(), 1e-10) <= 1.0
    members = np.flatnonzero(rep[DEPTH - 1] != np.arange(B))
    rng = stream(3, TEST)
    pick = rng.choice(members, size=3, replace=False)
    centres = sorted({*pick.tolist(), *rep[DEPTH - 1][pick].tolist()})
    loc, cond = O.fit_local(p.levels[0].A, 8, DEPTH, centres, with_cond=True)
    for ell in range(1, DEPTH + 1):
        g = t.get_smoother(0, ell)
        for c in centres:
            o = loc[c][ell - 1]
            e = np.linalg.norm(g[c] - o) / np.linalg.norm(o)
            bound = scalar_bound(cond[c][:ell])
            assert record(f"interface3d_128 lattice-cached block {c} Lambda_{ell}", e, bound) <= 1.0, (c, ell, e)
