"""GPU <-> oracle parity through the C ABI (MI355X).

Every expected value comes from the FP64 CPU oracle on the same seeded inputs.
Tolerances (the bounds and their derivation are in tests/parity.py):
  * integer artefacts (patterns, colours): bit-exact;
  * FP64 smoother blocks: per block, 16384 u max(cond(G_i), the worst
    condition met at earlier cascade levels), u = 2^-53, cond from the
    oracle's normal equations.  Blocks whose G_i is exactly singular (from
    the second cascade level on) compare through the minimum-norm solution,
    both sides cutting eigenvalues below 1e-13 of the largest;
  * FP64 V-cycle, with the GPU's own setup and with the oracle's smoothers
    injected: 1e-12 relative, in the 2-norm and per entry;
  * FP32 V-cycle: 1e-5 against the FP64 oracle (about 100 x the FP32 unit
    round-off for the ~40 dependent sweeps of a V-cycle).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from parity import VCYCLE_TOL, check_level_smoothers, check_vec, rel2
from synth import fd
from synth.problem import Level, Problem
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu

APPLY_TOL = VCYCLE_TOL
FP32_TOL = 1e-5


def rel(a, b):
    return rel2(a, b)


def gpu_solver(cascade, prob, **opts):
    s = cascade.Solver(prob.levels)
    s.setup(**opts)
    return s


def oracle_setup(prob, depth, mode="additive", alpha=None):
    return O.setup_hierarchy(prob.levels, depth, mode, alpha)


def check_smoothers(s, sm, prob, depth, label=None):
    label = label or prob.name
    for l in range(len(prob.levels) - 1):
        check_level_smoothers(s, sm[l], l, depth, label)


def inject(s, sm):
    """Replace the GPU's smoothers by the oracle's (every level and ell)."""
    for l, d in enumerate(sm):
        for ell, L in enumerate(d["lam"]):
            s.set_smoother(l, ell + 1, L)


def check_vcycle(s, sm, prob, order="RF", npre=1, npost=1, b=None):
    """V b against the oracle: with the GPU's own setup, then with the oracle's
    smoothers injected (the apply path alone)."""
    b = prob.rhs if b is None else b
    o = O.vcycle(prob.levels, sm, b, order, npre, npost)
    g = s.vcycle(b).cpu().numpy()
    check_vec(g, o, VCYCLE_TOL, f"{prob.name} {order} V({npre},{npost}) FP64 V-cycle, own setup")
    inject(s, sm)
    g = s.vcycle(b).cpu().numpy()
    check_vec(g, o, VCYCLE_TOL, f"{prob.name} {order} V({npre},{npost}) FP64 V-cycle, oracle smoothers")
    return o


def check_patterns(s, sm, prob):
    for l in range(len(prob.levels) - 1):
        pats = sm[l]["patterns"]
        for step, pat in enumerate(pats):
            ptr, col = s.get_pattern(l, step)
            pat = pat.tocsr()
            pat.sort_indices()
            np.testing.assert_array_equal(ptr, pat.indptr.astype(np.int64))
            np.testing.assert_array_equal(col, pat.indices.astype(np.int32))


# ---------------------------------------------------------------------------
# 64^2 Dirichlet Poisson, point blocks, depth-3 additive, V(2,2) RF, FP64
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def poisson64():
    p = fd.poisson2d(64)
    return p, oracle_setup(p, 3)


def test_poisson64_setup_parity(gpu_lib, poisson64):
    p, sm = poisson64
    s = gpu_solver(gpu_lib, p, depth=3, n_pre=2, n_post=2)
    check_smoothers(s, sm, p, 3)
    check_patterns(s, sm, p)


def test_poisson64_apply_and_vcycle_parity(gpu_lib, poisson64):
    p, sm = poisson64
    s = gpu_solver(gpu_lib, p, depth=3, n_pre=2, n_post=2)
    rng = stream(1, TEST, 0)
    x0 = rng.uniform(-1, 1, size=p.rhs.shape)
    inject(s, sm)
    for rev in (False, True):
        g = s.smooth(0, p.rhs, x0, reverse=rev).cpu().numpy()
        o = O.smooth(p.levels[0].A, sm[0], x0, p.rhs, reverse=rev)
        check_vec(g, o, APPLY_TOL, f"poisson64 cascade apply reverse={rev}")
    check_vcycle(s, sm, p, "RF", 2, 2)


def test_poisson64_solve(gpu_lib, poisson64):
    p, sm = poisson64
    s = gpu_solver(gpu_lib, p, depth=3, n_pre=2, n_post=2)
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=50)
    xo, ho = O.solve(p.levels, sm, p.rhs, 1e-10, 50, "RF", 2, 2)
    assert info["rel_res"] <= 1e-10
    assert info["iterations"] == len(ho) - 1
    # each history entry is ||b - A x|| / ||b||: its absolute error is ~ eps * ||A|| ||x|| / ||b||
    np.testing.assert_allclose(info["history"], ho, rtol=1e-6, atol=1e-14)
    check_vec(x.cpu().numpy(), xo, 1e-11, "poisson64 FP64 IR solution")


# ---------------------------------------------------------------------------
# 3D interface problem, 2x2x2 blocks, depth-4 additive, 8 RHS (reduced sizes)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def iface32():
    p = fd.interface3d(32, nrhs=8)
    return p, oracle_setup(p, 4)


def test_interface_setup_parity(gpu_lib, iface32):
    p, sm = iface32
    s = gpu_solver(gpu_lib, p, depth=4)
    check_smoothers(s, sm, p, 4)
    check_patterns(s, sm, p)


def test_deep_cascade_long_rows(gpu_lib):
    """A depth-6 cascade on 16^3 cells (8^3 blocks of 2x2x2): the deepest
    steps' rows hold up to 302 blocks, more than the 8x8 normal equations keep
    positions for in LDS (256) and more matches than the row product caches
    (302 x 7 > 2048), so both search as they go."""
    p = fd.interface3d(16, nrhs=1)
    sm = oracle_setup(p, 6)
    s = gpu_solver(gpu_lib, p, depth=6)
    check_smoothers(s, sm, p, 6)
    s.close()


@pytest.mark.parametrize("order", ["RF", "FF"])
def test_interface_vcycle_fp64_and_fp32(gpu_lib, iface32, order):
    p, sm = iface32
    s = gpu_solver(gpu_lib, p, depth=4, order=order)
    o = check_vcycle(s, sm, p, order)
    s.set_precision("fp32")
    g32 = s.vcycle(p.rhs).cpu().numpy()
    check_vec(g32, o, FP32_TOL, f"iface32 {order} FP32 V-cycle vs FP64 oracle")


def test_interface_solve_fp32_ir_matches_oracle_rate(gpu_lib, iface32):
    p, sm = iface32
    xo, ho = O.solve(p.levels, sm, p.rhs, 1e-10, 60)
    rho_o = O.rho_regression(ho)
    s = gpu_solver(gpu_lib, p, depth=4, precision="fp32")
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=60)
    assert info["rel_res"] <= 1e-10
    h = info["history"]
    assert all(b < a for a, b in zip(h, h[1:]))
    print(f"rho fp32+IR {info['rho']:.4f} vs oracle {rho_o:.4f}; x error {rel(x.cpu().numpy(), xo):.2e}")
    assert info["rho"] <= 1.05 * rho_o
    check_vec(x.cpu().numpy(), xo, 1e-8, "iface32 FP32+IR solution vs FP64 oracle")


def test_ragged_sizes(gpu_lib):
    """18^3 unknowns: 5832 rows, not a multiple of the 64-row slice; odd
    bottom level (9^3) with point blocks."""
    p = fd.interface3d(18, nrhs=2)
    sm = oracle_setup(p, 3)
    s = gpu_solver(gpu_lib, p, depth=3)
    check_smoothers(s, sm, p, 3)
    check_vcycle(s, sm, p)


@pytest.mark.parametrize("bs", [2, 4])
def test_block_sizes_2d(gpu_lib, bs):
    """2D log-normal coefficients with 2x2 (nb = 4) and 4x4 (nb = 16) blocks."""
    z = stream(7, 1).standard_normal((32, 32))
    levels = fd.fv_hierarchy(np.exp(2.0 * z), bs=bs, n_stop=4)
    p = Problem(f"ln2d-{bs}x{bs}", levels, stream(7, 0).uniform(-1, 1, size=(32 * 32, 4)))
    sm = oracle_setup(p, 2)
    s = gpu_solver(gpu_lib, p, depth=2)
    check_smoothers(s, sm, p, 2)
    check_patterns(s, sm, p)
    check_vcycle(s, sm, p)


# ---------------------------------------------------------------------------
# Multiplicative (multicoloured) cascades
# ---------------------------------------------------------------------------

def test_multiplicative_red_black_2d(gpu_lib):
    p = fd.lognormal2d(32, nrhs=2, n_stop=4)
    for lv in p.levels:
        m = int(round(np.sqrt(lv.n)))
        lv.colour = fd.parity_colour(m, 2, 1, lv.cells)
    sm = oracle_setup(p, 3, "multiplicative")
    for order in ("FF", "RF"):
        s = gpu_solver(gpu_lib, p, depth=3, mode="multiplicative", order=order)
        check_smoothers(s, sm, p, 3)
        check_patterns(s, sm, p)
        check_vcycle(s, sm, p, order)
        x0 = stream(2, TEST).uniform(-1, 1, size=p.rhs.shape)
        for rev in (False, True):
            g = s.smooth(0, p.rhs, x0, reverse=rev).cpu().numpy()
            check_vec(g, O.smooth(p.levels[0].A, sm[0], x0, p.rhs, rev), APPLY_TOL,
                      f"red-black {order} cascade apply reverse={rev}")


def test_multiplicative_greedy_colouring_blocks(gpu_lib):
    """No colours supplied: the library colours greedily in block order; the
    colouring must equal the sequential greedy colouring bit for bit."""
    p = fd.interface3d(16, nrhs=1)
    sm = oracle_setup(p, 2, "multiplicative")
    s = gpu_solver(gpu_lib, p, depth=2, mode="multiplicative", order="FF")
    for l in range(len(p.levels) - 1):
        np.testing.assert_array_equal(s.get_colours(l), sm[l]["colours"])
    check_smoothers(s, sm, p, 2)
    check_patterns(s, sm, p)
    check_vcycle(s, sm, p, "FF")


def test_improper_colouring_is_rejected(gpu_lib):
    p = fd.lognormal2d(16, nrhs=1, n_stop=4)
    for lv in p.levels:
        lv.colour = np.zeros(lv.n, dtype=np.int32)
    s = gpu_lib.Solver(p.levels)
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.setup(depth=2, mode="multiplicative")
    assert e.value.status == -5


# ---------------------------------------------------------------------------
# Truncation, options, state and persistence
# ---------------------------------------------------------------------------

def test_truncation_parity(gpu_lib):
    p = fd.lognormal2d(24, nrhs=1, n_stop=6)
    sm = oracle_setup(p, 3, alpha=4)
    s = gpu_solver(gpu_lib, p, depth=3, alpha=4)
    check_smoothers(s, sm, p, 3)
    check_patterns(s, sm, p)


def test_depth_one_and_single_level(gpu_lib):
    p = fd.lognormal2d(16, nrhs=1, n_stop=4)
    sm = oracle_setup(p, 1)
    s = gpu_solver(gpu_lib, p, depth=1, n_pre=2, n_post=3)
    check_vcycle(s, sm, p, "RF", 2, 3)
    one = Problem("bottom", [Level(A=p.levels[-1].A)], stream(3, 0).uniform(-1, 1, size=(p.levels[-1].n, 1)))
    s1 = gpu_solver(gpu_lib, one, depth=1)
    g = s1.vcycle(one.rhs).cpu().numpy()
    check_vec(g, np.linalg.solve(one.levels[0].A.toarray(), one.rhs), 1e-12, "single-level direct solve")


def test_state_and_argument_errors(gpu_lib):
    p = fd.lognormal2d(16, nrhs=1, n_stop=4)
    s = gpu_lib.Solver(p.levels)
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.vcycle(p.rhs)
    assert e.value.status == -7
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.setup(depth=0)
    assert e.value.status == -1
    bad = fd.lognormal2d(16, nrhs=1, n_stop=4)
    A = bad.levels[0].A.tolil()
    A[3, 3] = -1.0
    bad.levels[0].A = A.tocsr()
    sb = gpu_lib.Solver(bad.levels)      # the diagonal is checked by the prescaling at setup
    with pytest.raises(gpu_lib.CascadeError) as e:
        sb.setup(depth=2)
    assert e.value.status == -1 and "positive diagonal" in str(e.value)
    s.setup(depth=2)
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.vcycle(np.zeros((p.n, 3)))
    assert e.value.status == -1
    x, info = s.solve(p.rhs, rtol=1e-14, maxit=1, raise_on_noconv=False)
    assert info["status"] == -6 and info["iterations"] == 1


def test_nan_rhs_reports_enan(gpu_lib):
    p = fd.lognormal2d(16, nrhs=1, n_stop=4)
    s = gpu_solver(gpu_lib, p, depth=2)
    b = p.rhs.copy()
    b[5, 0] = np.nan
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.solve(b)
    assert e.value.status == -8


def test_save_load_roundtrip(gpu_lib, tmp_path):
    p = fd.interface3d(16, nrhs=2)
    s = gpu_solver(gpu_lib, p, depth=3)
    ref = s.vcycle(p.rhs).cpu().numpy()
    path = str(tmp_path / "setup.bin")
    s.save(path)
    t = gpu_lib.Solver(p.levels)
    t.load(path)
    np.testing.assert_array_equal(t.vcycle(p.rhs).cpu().numpy(), ref)


def test_injected_smoother_vcycle(gpu_lib):
    """set_smoother: a V-cycle with smoothers computed elsewhere (damped block
    Jacobi, different weight per cascade level) matches the oracle."""
    p = fd.interface3d(16, nrhs=2)
    depth = 3
    s = gpu_solver(gpu_lib, p, depth=depth)
    sm = []
    for l, lv in enumerate(p.levels[:-1]):
        base = O.jacobi_smoother(lv.A, lv.block_size, 1)["lam"][0]
        lams = [w * base for w in (0.6, 0.75, 0.9)]
        for ell in range(depth):
            s.set_smoother(l, ell + 1, lams[ell])
        sm.append(dict(lam=lams, colours=None))
    g = s.vcycle(p.rhs).cpu().numpy()
    check_vec(g, O.vcycle(p.levels, sm, p.rhs), APPLY_TOL, "injected damped block-Jacobi V-cycle")


@pytest.mark.parametrize("mode", ["additive", "multiplicative"])
def test_autotuned_schedules_give_identical_results(gpu_lib, mode):
    """Sweep schedules change only the launch shape: solves are bit-identical."""
    p = fd.interface3d(24, nrhs=4) if mode == "additive" else fd.poisson2d(128, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, mode=mode, precision="fp32")
    x0, i0 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    x0 = x0.cpu().numpy()
    sched = s.autotune(4)
    assert len(sched) == len(p.levels)
    for l, (w, g, ms) in enumerate(sched[:-1]):
        assert w in (64, 256) and g in (0, 1024, 2048, 4096) and ms > 0, (l, w, g, ms)
    assert sched[-1][0] == 0
    x1, i1 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    assert i1["iterations"] == i0["iterations"]
    np.testing.assert_array_equal(x1.cpu().numpy(), x0)


@pytest.mark.parametrize("case,ridge", [("poisson32_points", 0.25), ("interface16_blocks8", 1e-3)])
def test_ridge_fit_parity(gpu_lib, case, ridge):
    """The Tikhonov-regularised fit (point blocks: the scalar kernel; 8x8
    blocks: the blocked normal equations) against the oracle's, and its
    V-cycle with the GPU's own setup."""
    p = fd.poisson2d(32) if case == "poisson32_points" else fd.interface3d(16, nrhs=2)
    sm = O.setup_hierarchy(p.levels, 3, ridge=ridge)
    s = gpu_solver(gpu_lib, p, depth=3, ridge=ridge)
    check_smoothers(s, sm, p, 3, f"{p.name} ridge {ridge:g}")
    check_patterns(s, sm, p)
    o = O.vcycle(p.levels, sm, p.rhs, "RF")
    check_vec(s.vcycle(p.rhs).cpu().numpy(), o, VCYCLE_TOL, f"{p.name} ridge {ridge:g} RF V-cycle, own setup")


def test_ridge_is_refused_where_it_does_not_apply(gpu_lib):
    p = fd.poisson2d(16)
    s = gpu_lib.Solver(p.levels)
    with pytest.raises(gpu_lib.CascadeError) as e:
        s.setup(depth=2, ridge=-1.0)
    assert e.value.status == -1
    import ctypes

    import torch
    S = torch.ones((sum(lv.n for lv in p.levels[:-1]), 8), dtype=torch.float64, device="cuda")
    o = gpu_lib.cs_options(2, 0, 1, 1, 1, 0, 0, 1e-3)
    st = s._lib.cs_setup_sketched(s._h, ctypes.byref(o), 8, ctypes.c_void_p(S.data_ptr()))
    assert st == -1 and "exact fit only" in s._lib.cs_last_error(s._h).decode()
