"""SIPG Q3 (16x16 element blocks) with the 4-colour multiplicative cascade:
FP64 parity against the oracle, and the BF16 matrix-core path.

FP64 smoother blocks: per block 16384 u cond (tests/parity.py), cond the worst
condition number of the normal equations met up to that cascade level (the
oracle reports it; up to ~3e7 for DG blocks at the third level).  FP64
V-cycle: 1e-12 with the oracle's smoothers injected; with the GPU's own
setup the V-cycle inherits the smoother differences, bounded by 16384 u times
the worst condition number of the hierarchy.

BF16 tolerances: the sweep is compared with the oracle run on A and Lambda
rounded to BF16 (round to nearest even), so only the FP32 accumulation and the
hi/lo BF16 split of the vectors (about 2^-17 relative) differ: 5e-5 on a
well-conditioned cascade.  With the Frobenius cascade the BF16 solve must reach
1e-10 (FP64 outer iteration) within a few iterations of the FP64 V-cycle.
"""
import numpy as np
import pytest

import oracle as O
from parity import C_SUM, U, VCYCLE_TOL, check_level_smoothers, check_vec
from synth import dg
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def bf16(a):
    """Round FP64 values to BF16 (through FP32, nearest even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def dg16():
    p = dg.sipg_q3(16)
    return p, O.setup_hierarchy(p.levels, 3, "multiplicative")


def inject(s, sm):
    for l, d in enumerate(sm):
        for ell, L in enumerate(d["lam"]):
            s.set_smoother(l, ell + 1, L)


def test_dg_setup_and_vcycle_parity_fp64(gpu_lib, dg16):
    p, sm = dg16
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, mode="multiplicative", order="FF")
    for l in range(len(p.levels) - 1):
        np.testing.assert_array_equal(s.get_colours(l), p.levels[l].colour)
        check_level_smoothers(s, sm[l], l, 3, "sipg_q3_16")
    expect = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    worst = max(float(np.max(c)) for d in sm for c in d["gram_cond"])
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, max(VCYCLE_TOL, C_SUM * U * worst),
              "sipg_q3_16 FF FP64 V-cycle, own setup")
    inject(s, sm)
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, VCYCLE_TOL, "sipg_q3_16 FF FP64 V-cycle, oracle smoothers")


def test_bf16_sweep_matches_rounded_oracle(gpu_lib, dg16):
    """The matrix-core sweep against the oracle on BF16-rounded A and Lambda.
    A block Gauss-Seidel-type cascade (Lambda_l = 0.8 D^-1 on every colour) is
    injected: it is well conditioned (FP32 and FP64 runs of it agree to ~1e-6),
    so the comparison isolates the kernel (operand layout, packing, colour
    order, the hi/lo split of the vectors).  The Frobenius DG cascade itself
    amplifies rounding by orders of magnitude (its blocks have condition
    numbers up to ~3e7), which the solve test below covers."""
    p, _ = dg16
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, mode="multiplicative", order="FF", precision="bf16")
    rng = stream(3, TEST, 1)
    for l in range(len(p.levels) - 1):
        lv = p.levels[l]
        jac = O.jacobi_smoother(lv.A, 16, 3, 0.8)
        jac["colours"] = lv.colour
        for ell in range(3):
            s.set_smoother(l, ell + 1, jac["lam"][ell])
        b = rng.uniform(-1, 1, size=(lv.n, 1))
        x0 = rng.uniform(-1, 1, size=(lv.n, 1))
        A16 = lv.A.copy()
        A16.data = bf16(A16.data)
        sm16 = dict(jac)
        sm16["lam"] = [bf16(L) for L in jac["lam"]]
        for rev in (False, True):
            g = s.smooth(l, b, x0, reverse=rev).cpu().numpy()
            o = O.smooth(A16, sm16, x0, b, reverse=rev)
            assert rel(g, o) <= 5e-5, (l, rev, rel(g, o))


def test_bf16_solve_depth1_and_escalation(gpu_lib, dg16):
    """A depth-1 multicoloured cascade (block Gauss-Seidel type) tolerates
    BF16 A and Lambda: the BF16 solve converges as the FP64 one does.  The
    depth-3 plain Frobenius cascade does not (tests/test_oracle_precision.py:
    its large, cancelling blocks amplify BF16 rounding): the solve detects the
    divergence and finishes in FP32."""
    p, _ = dg16
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=1, mode="multiplicative", order="FF", precision="fp64")
    _, f64 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    s.set_precision("bf16")
    x, b16 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    assert b16["precision"] == "bf16"
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(p.rhs)
    print(f"depth 1: rho fp64 {f64['rho']:.4f} ({f64['iterations']} it), bf16 {b16['rho']:.4f} ({b16['iterations']} it)")
    assert b16["rho"] <= 1.05 * f64["rho"]
    s.setup(depth=3, mode="multiplicative", order="FF", precision="bf16")
    x, e = s.solve(p.rhs, rtol=1e-10, maxit=200)
    assert e["precision"] == "fp32" and e["rel_res"] <= 1e-10


@pytest.fixture(scope="module")
def dg16_ridge():
    p = dg.sipg_q3(16)
    return p, O.setup_hierarchy(p.levels, 3, "multiplicative", ridge=1e-3)


def test_ridge_fit_parity_fp64(gpu_lib, dg16_ridge):
    """The Tikhonov-regularised fit (ridge 1e-3) against the oracle's: the
    regularised normal equations are far better conditioned, so the per-block
    bounds from their condition numbers are tight."""
    p, sm = dg16_ridge
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, mode="multiplicative", order="FF", ridge=1e-3)
    for l in range(len(p.levels) - 1):
        check_level_smoothers(s, sm[l], l, 3, "sipg_q3_16 ridge 1e-3")
    expect = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, VCYCLE_TOL, "sipg_q3_16 ridge FF FP64 V-cycle, own setup")


def test_bf16_blocks_with_ridge_fit_converge_at_depth_3(gpu_lib, dg16_ridge):
    """BF16 blocks on the matrix cores (FP32 restricted residual) with the
    regularised depth-3 fit: the FP64 refinement reaches 1e-10 in BF16, with
    the convergence factor within 5% of the FP64 V-cycle's on the same fit."""
    p, sm = dg16_ridge
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, mode="multiplicative", order="FF", precision="fp64", ridge=1e-3)
    _, f64 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    s.set_precision("bf16")
    x, b16 = s.solve(p.rhs, rtol=1e-10, maxit=200)
    print(f"depth 3 ridge: rho fp64 {f64['rho']:.4f} ({f64['iterations']} it), "
          f"bf16 {b16['rho']:.4f} ({b16['iterations']} it)")
    assert b16["precision"] == "bf16"
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(p.rhs)
    assert b16["rho"] <= 1.05 * f64["rho"]
    # the oracle's FP64 refinement with the same fit converges at the FP64 rate
    _, hist = O.solve(p.levels, sm, p.rhs, 1e-10, 200, "FF", 1, 1)
    assert abs(f64["iterations"] - (len(hist) - 1)) <= 1
