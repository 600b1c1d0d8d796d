"""Parity at full size for the SIPG Q3 workload: 256^2 jittered quadrilaterals,
16x16 element blocks (1,048,576 unknowns), depth-3 four-colour multiplicative
FF cascade, FP64 V-cycle - the configuration bench.py's DG leg times.

  * sampled smoother blocks (a corner, a boundary and two interior elements)
    against the oracle's fit of the same blocks on their radius nu * chi
    patch (exact: a multiplicative step reads A within nu * chi layers), to
    16384 u cond, cond the worst normal-equation condition number met in the
    patch up to that cascade level (tests/parity.py);
  * the FP64 V-cycle against the oracle's at full size with injected block
    Jacobi weights on every level (1e-12, 2-norm and per entry);
  * the solve by properties: 1e-10 reached by flexible CG, and its convergence
    factor below the stationary iteration's.
"""
import numpy as np
import pytest

import oracle as O
from parity import VCYCLE_TOL, check_vec, record, scalar_bound
from synth import dg
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu

N = 256
DEPTH = 3


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def full(gpu_lib):
    p = dg.sipg_q3(N)
    print(f"[fullsize-dg] {p.n} unknowns, {len(p.levels)} levels", flush=True)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=DEPTH, mode="multiplicative", order="FF", precision="fp64")
    return p, s


def test_dg_fullsize_sampled_smoother_blocks(full):
    p, s = full
    lv = p.levels[0]
    rng = stream(6, TEST)
    centres = [0, 100, int(N * (N // 2) + N // 2), int(rng.integers(N, N * N - N))]
    loc, cond = O.fit_local(lv.A, 16, DEPTH, centres, mode="multiplicative", colours=lv.colour, with_cond=True)
    for ell in range(1, DEPTH + 1):
        g = s.get_smoother(0, ell)
        for c in centres:
            o = loc[c][ell - 1]
            bound = scalar_bound(cond[c][:ell])
            e = np.linalg.norm(g[c] - o) / np.linalg.norm(o)
            assert record(f"sipg_q3_256 block {c} Lambda_{ell}", e, bound) <= 1.0, (c, ell, e, bound)


def test_dg_fullsize_solve(full):
    p, s = full
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=200, method="cg")
    print(f"[fullsize-dg] FP64 CG: {info['iterations']} it, rho {info['rho']:.4f}, {info['solve_ms']:.1f} ms",
          flush=True)
    assert info["rel_res"] <= 1e-10 and info["precision"] == "fp64"
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.linalg.norm(r) / np.linalg.norm(p.rhs) <= 1.5e-10
    _, ir = s.solve(p.rhs, rtol=1e-10, maxit=200, method="ir", raise_on_noconv=False)
    assert info["rho"] < ir["rho"] < 1.0


def test_dg_fullsize_bf16_ridge_refinement(gpu_lib, full):
    """The configuration bench.py times: the regularised fit (ridge 1e-3), BF16
    blocks on the matrix cores inside FP64 refinement, to 1e-10, at most 5%
    above the FP64 V-cycle's convergence factor on the same fit."""
    p, _ = full
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=DEPTH, mode="multiplicative", order="FF", precision="fp64", ridge=1e-3)
    _, f64 = s.solve(p.rhs, rtol=1e-10, maxit=400)
    s.set_precision("bf16")
    x, b16 = s.solve(p.rhs, rtol=1e-10, maxit=400)
    print(f"[fullsize-dg] ridge 1e-3 refinement: fp64 {f64['iterations']} it rho {f64['rho']:.4f}, "
          f"bf16 {b16['iterations']} it rho {b16['rho']:.4f}", flush=True)
    assert b16["precision"] == "bf16" and b16["rel_res"] <= 1e-10
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.linalg.norm(r) / np.linalg.norm(p.rhs) <= 1.5e-10
    assert b16["rho"] <= 1.05 * f64["rho"]
    s.close()


def test_dg_fullsize_vcycle_injected_smoothers(full):
    """Runs last: replaces the fitted smoothers."""
    p, s = full
    weights = (0.6, 0.8, 1.0)
    sm = []
    for l, lv in enumerate(p.levels[:-1]):
        D = O.jacobi_smoother(lv.A, lv.block_size, 1)["lam"][0]
        lams = [w * D for w in weights]
        for ell in range(DEPTH):
            s.set_smoother(l, ell + 1, lams[ell])
        sm.append(dict(lam=lams, colours=np.asarray(lv.colour)))
    g = s.vcycle(p.rhs).cpu().numpy()
    o = O.vcycle(p.levels, sm, p.rhs, "FF")
    e = check_vec(g, o, VCYCLE_TOL, "sipg_q3_256 FP64 V-cycle, injected smoothers")
    print(f"[fullsize-dg] FP64 V-cycle vs oracle: {e:.2e}", flush=True)
