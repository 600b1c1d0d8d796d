"""Flexible CG around the V-cycle (cs_solve_cg) against the oracle's FCG.

FP64 with the oracle's smoothers injected: the two runs differ only in
summation order (about 1e-13 per V-cycle), which CG carries forward without
amplification over the few iterations used here, so residual histories agree
to 1e-6 relative and the iterates to 1e-8.
"""
import numpy as np
import pytest

import oracle as O
from parity import check_vec
from synth import fd
from synth.batch import concatenate
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu


def inject(s, sm):
    for l, d in enumerate(sm):
        for ell, L in enumerate(d["lam"]):
            s.set_smoother(l, ell + 1, L)


CASES = [("poisson64", lambda: fd.poisson2d(64, nrhs=2), 3, 2),
         ("interface24", lambda: fd.interface3d(24, nrhs=4), 3, 1),
         ("lognormal48", lambda: fd.lognormal2d(48, 2.0, 2), 3, 1)]


@pytest.mark.parametrize("name,make,depth,nv", CASES)
def test_cg_matches_oracle_fcg(gpu_lib, name, make, depth, nv):
    p = make()
    sm = O.setup_hierarchy(p.levels, depth)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=depth, n_pre=nv, n_post=nv)
    inject(s, sm)
    pre = lambda r: O.vcycle(p.levels, sm, r, "RF", nv, nv)
    xo, ho = O.fcg(p.levels[0].A, pre, p.rhs, rtol=1e-10, maxit=100)
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    assert info["iterations"] == len(ho) - 1
    np.testing.assert_allclose(info["history"], ho, rtol=1e-6)
    check_vec(x.cpu().numpy(), xo, 1e-8, "FCG iterate vs oracle")


def test_cg_beats_refinement_and_fp32_converges(gpu_lib):
    p = fd.interface3d(32, nrhs=8)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=4)
    _, ir = s.solve(p.rhs, rtol=1e-10, maxit=200)
    _, cg = s.solve(p.rhs, rtol=1e-10, maxit=200, method="cg")
    assert cg["iterations"] < ir["iterations"] and cg["rel_res"] <= 1e-10
    s.set_precision("fp32")
    x, c32 = s.solve(p.rhs, rtol=1e-10, maxit=200, method="cg")
    assert c32["rel_res"] <= 1e-10 and c32["iterations"] <= cg["iterations"] + 2
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-10


def test_batched_cg_runs_every_system_as_if_alone(gpu_lib):
    sizes = [48, 64, 80, 16, 112, 32, 8, 20, 12]
    probs = fd.lognormal_batch(len(sizes), nrhs=2, sizes=sizes, config_id=16)
    bt = concatenate(probs)
    sms = [O.setup_hierarchy(p.levels, 3) for p in probs]
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3)
    s.set_systems(bt.sys_ptr)
    rtol = 1e-10
    x, info = s.solve(bt.rhs, rtol=rtol, maxit=200, method="cg")
    its, rels = s.system_stats()
    xs = bt.split(x.cpu().numpy())
    for q, si in enumerate(bt.order):
        p = probs[si]
        r = p.rhs - p.levels[0].A @ xs[si]
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= rtol
        _, h = O.fcg(p.levels[0].A, lambda v: O.vcycle(p.levels, sms[si], v), p.rhs, rtol=rtol, maxit=200)
        k = len(h) - 1
        if abs(np.log(h[k] / rtol)) > 1e-3 and (k == 0 or abs(np.log(h[k - 1] / rtol)) > 1e-3):
            assert its[q] == k, (q, its[q], k)
    assert info["iterations"] == its.max()


# ---------------------------------------------------------------------------
# GMRES (cs_solve_gmres) against the oracle's GMRES: FP64, injected smoothers,
# short restarts so that several cycles run.  Classical Gram-Schmidt applied
# twice (GPU) and modified Gram-Schmidt (oracle) agree to rounding; histories
# to 1e-6 relative (1e-13 absolute for the explicitly recomputed residuals),
# iterates to 1e-8.
# ---------------------------------------------------------------------------

GM_CASES = [("poisson64", lambda: fd.poisson2d(64, nrhs=2), 3, "FF", 4),
            ("interface24", lambda: fd.interface3d(24, nrhs=4), 3, "RF", 3),
            ("lognormal48", lambda: fd.lognormal2d(48, 2.0, 1), 2, "FF", 30)]


@pytest.mark.parametrize("flexible", [False, True])
@pytest.mark.parametrize("name,make,depth,order,restart", GM_CASES)
def test_gmres_matches_oracle(gpu_lib, name, make, depth, order, restart, flexible):
    p = make()
    sm = O.setup_hierarchy(p.levels, depth)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=depth, order=order)
    inject(s, sm)
    pre = lambda r: O.vcycle(p.levels, sm, r, order)
    xo, ho = O.gmres(p.levels[0].A, pre, p.rhs, restart=restart, rtol=1e-10, maxit=100, flexible=flexible)
    x, info = s.solve(p.rhs, rtol=1e-10, maxit=100, method="fgmres" if flexible else "gmres", restart=restart)
    assert info["iterations"] == len(ho) - 1, (info["iterations"], len(ho) - 1)
    # a residual recomputed at a restart carries rounding of order u ||A|| ||x|| / ||b||
    # (absolute, in the history's relative units; the 1e4 contrast makes ||A|| ||x||
    # large), and the next cycle starts from it: 1e-13 absolute beside 1e-6 relative
    np.testing.assert_allclose(info["history"], ho, rtol=1e-6, atol=1e-13)
    check_vec(x.cpu().numpy(), xo, 1e-8, f"GMRES {name} restart={restart} flexible={flexible} iterate vs oracle")
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    true = np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0))
    assert true <= (1e-10 if flexible else 1e-7)


def test_gmres_fp32_vcycle_reaches_fp64_accuracy(gpu_lib):
    p = fd.interface3d(32, nrhs=8)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=4, order="FF")
    _, g64 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="fgmres")
    s.set_precision("fp32")
    for method in ("gmres", "fgmres"):
        x, g = s.solve(p.rhs, rtol=1e-10, maxit=100, method=method)
        assert g["precision"] == "fp32" and g["rel_res"] <= 1e-10, (method, g["rel_res"])
        assert g["iterations"] <= g64["iterations"] + 5, (method, g["iterations"], g64["iterations"])
        r = p.rhs - p.levels[0].A @ x.cpu().numpy()
        true = np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0))
        assert true <= (1e-10 if method == "fgmres" else 1e-8), (method, true)


def test_gmres_maxit_and_restart_limits(gpu_lib):
    p = fd.poisson2d(32, nrhs=1)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=1)
    x, info = s.solve(p.rhs, rtol=1e-14, maxit=3, method="gmres", restart=2, raise_on_noconv=False)
    assert info["status"] == -6 and info["iterations"] == 3 and len(info["history"]) == 4
    with pytest.raises(gpu_lib.CascadeError):
        s.solve(p.rhs, method="gmres", restart=32)


def test_batched_gmres_runs_every_system_as_if_alone(gpu_lib):
    sizes = [48, 64, 80, 16, 112, 32, 8, 20, 12]
    probs = fd.lognormal_batch(len(sizes), nrhs=2, sizes=sizes, config_id=16)
    bt = concatenate(probs)
    sms = [O.setup_hierarchy(p.levels, 3) for p in probs]
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3, order="FF")
    s.set_systems(bt.sys_ptr)
    rtol = 1e-10
    for flexible in (False, True):
        x, info = s.solve(bt.rhs, rtol=rtol, maxit=200, method="fgmres" if flexible else "gmres", restart=30)
        its, rels = s.system_stats()
        xs = bt.split(x.cpu().numpy())
        for q, si in enumerate(bt.order):
            p = probs[si]
            pre = lambda v: O.vcycle(p.levels, sms[si], v, "FF")
            xo, h = O.gmres(p.levels[0].A, pre, p.rhs, restart=30, rtol=rtol, maxit=200, flexible=flexible)
            check_vec(xs[si], xo, 1e-7, f"krylov batch system {q} flexible={flexible} iterate")
            k = next(i for i, v in enumerate(h) if v <= rtol)
            if abs(np.log(h[k] / rtol)) > 1e-3 and (k == 0 or abs(np.log(h[k - 1] / rtol)) > 1e-3):
                assert its[q] == k, (q, flexible, its[q], k)
        assert info["iterations"] == its.max()


@pytest.mark.parametrize("nrhs", [1, 2, 8])
def test_gmres_rhs_counts_and_ragged_batch(gpu_lib, nrhs):
    """Every RHS count, and a batch with odd sizes whose systems end on
    different levels (ragged direct segments)."""
    sizes = [20, 12, 36, 10, 6, 20]
    probs = fd.lognormal_batch(len(sizes), nrhs=nrhs, sizes=sizes, config_id=18)
    bt = concatenate(probs)
    sms = [O.setup_hierarchy(p.levels, 2) for p in probs]
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=2, order="FF")
    s.set_systems(bt.sys_ptr)
    for flexible in (False, True):
        x, info = s.solve(bt.rhs, rtol=1e-10, maxit=200, method="fgmres" if flexible else "gmres", restart=7)
        xs = bt.split(x.cpu().numpy())
        for si, p in enumerate(probs):
            pre = lambda v: O.vcycle(p.levels, sms[si], v, "FF")
            xo, _ = O.gmres(p.levels[0].A, pre, p.rhs, restart=7, rtol=1e-10, maxit=200, flexible=flexible)
            check_vec(xs[si], xo, 1e-7, f"krylov batch system {si} flexible={flexible} iterate")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vcycle_after_cg_is_unaffected(gpu_lib, precision):
    """CG issues the next V-cycle's first sweep before it reads the convergence
    norms; once a solve ends (converged or at maxit) that sweep must not leak into
    a later V-cycle: the V-cycle equals that of a fresh solver bit for bit."""
    p = fd.interface3d(32, nrhs=8)
    rng = stream(9, TEST, 1)
    v = rng.uniform(-1, 1, size=p.rhs.shape)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=4, precision=precision)
    ref = gpu_lib.Solver(p.levels)
    ref.setup(depth=4, precision=precision)
    expect = ref.vcycle(v).cpu().numpy()
    s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    np.testing.assert_array_equal(s.vcycle(v).cpu().numpy(), expect)
    s.solve(p.rhs, rtol=1e-30, maxit=3, method="cg", raise_on_noconv=False)
    np.testing.assert_array_equal(s.vcycle(v).cpu().numpy(), expect)
    # and CG itself is unchanged by a V-cycle in between
    x1, i1 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    x2, i2 = ref.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    assert i1["iterations"] == i2["iterations"]
    np.testing.assert_array_equal(x1.cpu().numpy(), x2.cpu().numpy())
