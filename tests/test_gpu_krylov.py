"""Flexible CG around the V-cycle (cs_solve_cg) against the oracle's FCG.

FP64 with the oracle's smoothers injected: the two runs differ only in
summation order (about 1e-13 per V-cycle), which CG carries forward without
amplification over the few iterations used here, so residual histories agree
to 1e-6 relative and the iterates to 1e-8.
"""
import numpy as np
import pytest

import oracle as O
from synth import fd
from synth.batch import concatenate
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


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
    assert rel(x.cpu().numpy(), xo) <= 1e-8


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
