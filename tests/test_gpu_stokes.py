"""Stokes (saddle-point) levels: Stokes prescaling on the GPU, cascade fit,
V-cycle and GMRES on the MAC staggered grid, against the oracle.

Lambda blocks: 16384 u cond(G_i) per block as for the elliptic fits (the
normal equations are the same; only W differs; tests/parity.py).  V-cycle with
the oracle's smoothers injected: 1e-12 (2-norm and per entry); with the GPU's
own exact overlapping fit: 16384 u times the worst condition number met.  GMRES histories: 1e-6 relative, 1e-13 absolute
(recomputed residuals at restarts), iterates 1e-8.
"""
import numpy as np
import pytest

import oracle as O
from parity import C_SUM, U, VCYCLE_TOL, check_level_smoothers, check_vec
from synth import stokes

pytestmark = pytest.mark.gpu


def check(s, sm, depth, label="mac2d_16"):
    for l, d in enumerate(sm):
        check_level_smoothers(s, d, l, depth, label)


@pytest.fixture(scope="module")
def mac16():
    return stokes.mac2d(16, nrhs=2)


@pytest.mark.parametrize("l1", [True, False])
def test_stokes_setup_parity(gpu_lib, mac16, l1):
    p = mac16
    s = gpu_lib.Solver(p.levels)
    for i, lv in enumerate(p.levels):
        s.set_saddle_point(i, lv.kind, l1=l1)
    s.setup(depth=3)
    sm = O.setup_hierarchy(p.levels, 3, norm="l1" if l1 else "max")
    check(s, sm, 3)


def test_stokes_vcycle_and_gmres_parity(gpu_lib, mac16):
    p = mac16
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=4, order="FF")
    sm = O.setup_hierarchy(p.levels, 4, norm="l1")
    for l, d in enumerate(sm):
        for ell, L in enumerate(d["lam"]):
            s.set_smoother(l, ell + 1, L)
    expect = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, VCYCLE_TOL, "mac2d_16 FF V-cycle, oracle smoothers")
    pre = lambda r: O.vcycle(p.levels, sm, r, "FF")
    for flexible in (False, True):
        xo, ho = O.gmres(p.levels[0].A, pre, p.rhs, restart=30, rtol=1e-10, maxit=100, flexible=flexible)
        x, info = s.solve(p.rhs, rtol=1e-10, maxit=100, method="fgmres" if flexible else "gmres")
        assert info["iterations"] == len(ho) - 1
        np.testing.assert_allclose(info["history"], ho, rtol=1e-6, atol=1e-13)
        check_vec(x.cpu().numpy(), xo, 1e-8, f"mac2d_16 GMRES flexible={flexible} iterate vs oracle")


def test_stokes_fp32_gmres_and_sketch(gpu_lib):
    p = stokes.mac2d(64, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=4, order="FF", precision="fp32")
    for method in ("gmres", "fgmres"):
        x, info = s.solve(p.rhs, rtol=1e-10, maxit=200, method=method)
        assert info["precision"] == "fp32" and info["rel_res"] <= 1e-10
        r = p.rhs - p.levels[0].A @ x.cpu().numpy()
        true = np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0))
        assert true <= (1e-10 if method == "fgmres" else 1e-7), (method, true)
        print(f"mac64 {method}: {info['iterations']} it, rho {info['rho']:.3f}")
    S = s.setup_sketched(width=32, seed=4, depth=3, order="FF").cpu().numpy()
    off, sm = 0, []
    for lv in p.levels[:-1]:
        sm.append(O.fit_sketched(lv.A, 4, 3, S[off:off + lv.n], kind=lv.kind, norm="l1"))
        off += lv.n
    check(s, sm, 3)


def test_saddle_point_needs_its_kinds(gpu_lib, mac16):
    s = gpu_lib.Solver(mac16.levels)
    s.set_saddle_point(0, None)            # level 0 back to elliptic: zero pressure diagonal
    with pytest.raises(gpu_lib.CascadeError):
        s.setup(depth=2)
    bad = mac16.levels[0].kind.copy()
    bad[5] = 7
    with pytest.raises(gpu_lib.CascadeError):
        s.set_saddle_point(0, bad)


# ---------------------------------------------------------------------------
# Overlapping blocks (Vanka cell patches), exact and sketched fits
# ---------------------------------------------------------------------------

def vanka_solver(gpu_lib, p):
    s = gpu_lib.Solver(p.levels)
    m = p.meta["n"]
    for l in range(len(p.levels) - 1):
        s.set_overlapping_blocks(l, stokes.vanka_nodes(m))
        m //= 2
    return s


def oracle_vanka(p, depth, S=None, width=None):
    sm, m, off = [], p.meta["n"], 0
    for lv in p.levels[:-1]:
        Sl = None if S is None else S[off:off + lv.n]
        off += lv.n
        sm.append(O.fit_overlapping(lv.A, stokes.vanka_nodes(m), depth, S=Sl, kind=lv.kind, norm="l1"))
        m //= 2
    return sm


def test_overlapping_sketched_setup_parity(gpu_lib, mac16):
    p = mac16
    s = vanka_solver(gpu_lib, p)
    S = s.setup_sketched(width=32, seed=6, depth=2, order="FF").cpu().numpy()
    check(s, oracle_vanka(p, 2, S), 2)


@pytest.mark.parametrize("depth", [1, 3])
def test_overlapping_exact_setup_parity(gpu_lib, mac16, depth):
    """The exact overlapping-block fit (scalar residual rows, blockwise normal
    equations over the replicated slots) against the oracle's."""
    p = mac16
    s = vanka_solver(gpu_lib, p)
    s.setup(depth=depth, order="FF")
    sm = oracle_vanka(p, depth)
    check(s, sm, depth, f"mac2d_16 Vanka depth {depth}")
    expect = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    worst = max(float(np.max(c)) for d in sm for c in d["gram_cond"])
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, max(VCYCLE_TOL, C_SUM * U * worst),
              f"mac2d_16 Vanka depth {depth} FF V-cycle, own exact setup")


def test_overlapping_vcycle_parity_with_exact_smoothers(gpu_lib, mac16):
    p = mac16
    s = vanka_solver(gpu_lib, p)
    s.setup_sketched(width=32, seed=6, depth=2, order="FF")
    sm = oracle_vanka(p, 2)
    for l, d in enumerate(sm):
        for ell, L in enumerate(d["lam"]):
            s.set_smoother(l, ell + 1, L)
    expect = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    check_vec(s.vcycle(p.rhs).cpu().numpy(), expect, VCYCLE_TOL, "mac2d_16 Vanka FF V-cycle, oracle smoothers")
    rng = np.random.default_rng(3)
    x0 = rng.uniform(-1, 1, size=p.rhs.shape)
    got = s.smooth(0, p.rhs, x0).cpu().numpy()
    check_vec(got, O.smooth_overlapping(p.levels[0].A, sm[0], x0, p.rhs), VCYCLE_TOL,
              "mac2d_16 Vanka cascade apply, oracle smoothers")


def test_overlapping_partition_equals_plain_blocks(gpu_lib, mac16):
    p = mac16
    s = gpu_lib.Solver(p.levels)
    S = s.setup_sketched(width=32, seed=8, depth=2, order="FF")
    plain = [[s.get_smoother(l, e) for e in (1, 2)] for l in range(len(p.levels) - 1)]
    for l, lv in enumerate(p.levels[:-1]):
        s.set_overlapping_blocks(l, np.arange(lv.n).reshape(-1, 4))
    s.setup_sketched(width=32, sketch=S, depth=2, order="FF")
    for l in range(len(p.levels) - 1):
        for e in (1, 2):
            np.testing.assert_allclose(s.get_smoother(l, e), plain[l][e - 1], rtol=1e-10, atol=1e-13)


def test_overlapping_fp32_gmres(gpu_lib):
    p = stokes.mac2d(64, nrhs=2)
    s = vanka_solver(gpu_lib, p)
    s.setup_sketched(width=32, seed=1, depth=3, order="FF", precision="fp32")
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=200, method="fgmres")
    assert info["rel_res"] <= 1e-10
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-10
    print(f"mac64 Vanka sketched: {info['iterations']} it, rho {info['rho']:.3f}")
    with pytest.raises(gpu_lib.CascadeError):
        s.setup_sketched(width=32, seed=1, depth=3, order="RF")
    with pytest.raises(gpu_lib.CascadeError):
        s.setup(depth=2, order="RF")
    s.setup(depth=3, order="FF", precision="fp32")
    x, ex = s.solve(p.rhs, rtol=1e-10, maxit=200, method="fgmres")
    assert ex["rel_res"] <= 1e-10
    print(f"mac64 Vanka exact: {ex['iterations']} it, rho {ex['rho']:.3f}")
