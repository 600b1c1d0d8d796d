"""Batched V-cycle over many independent systems of uneven depth (GPU <-> oracle).

The batch is one block-diagonal hierarchy (synth.batch): systems that end on
a level are solved there directly while deeper ones continue.  Every system
must behave exactly as if it were solved alone, so each expected value is the
FP64 oracle run on that system by itself.  Tolerances as in the single-system
parity tests (the arithmetic per system is the same; bounds in tests/parity.py):
smoother blocks per block from the oracle's condition numbers of that system,
FP64 V-cycles 1e-12 per system in the 2-norm and per entry.
"""
import numpy as np
import pytest

import oracle as O
from parity import VCYCLE_TOL, check_blocks, check_vec, level_bounds
from synth import fd
from synth.batch import concatenate
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu

APPLY_TOL = VCYCLE_TOL
FP32_TOL = 1e-5

# 2D log-normal (sigma = 2) FD systems with 3, 4, 5 and 2 levels (coarsest
# 6^2 .. 8^2), plus a one-level system (all direct on the finest level)
SIZES = [48, 64, 80, 16, 112, 32, 80, 8]


@pytest.fixture(scope="module")
def small_batch():
    probs = fd.lognormal_batch(len(SIZES), nrhs=4, sizes=SIZES, config_id=14)
    bt = concatenate(probs)
    sms = [O.setup_hierarchy(p.levels, 3) for p in probs]
    return probs, bt, sms


# systems whose row counts are not multiples of 64 (slices straddle systems;
# the 36-row one sits inside a single slice)
ODD_SIZES = [20, 12, 36, 10, 6, 20]


@pytest.fixture(scope="module")
def odd_batch():
    probs = fd.lognormal_batch(len(ODD_SIZES), nrhs=2, sizes=ODD_SIZES, config_id=15)
    bt = concatenate(probs)
    sms = [O.setup_hierarchy(p.levels, 3) for p in probs]
    return probs, bt, sms


def batch_smoother(bt, sms, l, ell, bounds=False):
    """Oracle smoothers of every system present on batch level l, stacked in
    the batch order (zeros for the blocks of direct segments); bounds=True
    stacks the per-block parity bounds of each system's own fit instead."""
    out = []
    for s in bt.order:
        p = bt.problems[s]
        if len(p.levels) <= l:
            continue
        lv = p.levels[l]
        if l + 1 < len(p.levels):
            out.append(level_bounds(sms[s][l]["gram_cond"], ell) if bounds else sms[s][l]["lam"][ell - 1])
        else:
            out.append(np.ones(lv.n_blocks) if bounds else np.zeros((lv.n_blocks, lv.block_size, lv.block_size)))
    return np.concatenate(out)


def inject_batch(s, bt, sms, depth=3):
    for l in range(len(bt.levels) - 1):
        for ell in range(1, depth + 1):
            s.set_smoother(l, ell, batch_smoother(bt, sms, l, ell))


def test_batch_layout_is_depth_sorted(small_batch):
    probs, bt, _ = small_batch
    depths = [len(probs[s].levels) for s in bt.order]
    assert depths == sorted(depths, reverse=True)
    assert 1 in depths


def test_batch_smoother_parity(gpu_lib, small_batch):
    probs, bt, sms = small_batch
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3)
    for l in range(len(bt.levels) - 1):
        seg = bt.levels[l].direct_seg
        n_act = bt.levels[l].n if seg is None else int(seg[0])
        for ell in range(1, 4):
            g = s.get_smoother(l, ell)
            o = batch_smoother(bt, sms, l, ell)
            bnd = batch_smoother(bt, sms, l, ell, bounds=True)
            check_blocks(g[:n_act], o[:n_act], bnd[:n_act], f"batch level {l} Lambda_{ell}")


@pytest.mark.parametrize("which,precision", [("small_batch", "fp64"), ("small_batch", "fp32"),
                                             ("odd_batch", "fp64")])
def test_batch_vcycle_matches_separate_oracle_vcycles(gpu_lib, which, precision, request):
    probs, bt, sms = request.getfixturevalue(which)
    nr = probs[0].nrhs
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3, precision=precision)
    rng = stream(14, TEST, 1)
    bs = [rng.uniform(-1, 1, size=(p.n, nr)) for p in probs]
    expect = [O.vcycle(p.levels, sm, b, "RF", 1, 1) for p, sm, b in zip(probs, sms, bs)]
    tol = APPLY_TOL if precision == "fp64" else FP32_TOL
    g = bt.split(s.vcycle(bt.stack(bs)).cpu().numpy())
    for q in range(len(probs)):
        check_vec(g[q], expect[q], tol, f"{which} {precision} V-cycle system {q}, own setup")
    inject_batch(s, bt, sms)
    g = bt.split(s.vcycle(bt.stack(bs)).cpu().numpy())
    for q in range(len(probs)):
        check_vec(g[q], expect[q], tol, f"{which} {precision} V-cycle system {q}, oracle smoothers")


def test_batch_smooth_keeps_direct_rows(gpu_lib, small_batch):
    probs, bt, sms = small_batch
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3)
    inject_batch(s, bt, sms)
    l = 1
    lv = bt.levels[l]
    rng = stream(14, TEST, 2)
    b = rng.uniform(-1, 1, size=(lv.n, 2))
    x0 = rng.uniform(-1, 1, size=(lv.n, 2))
    g = s.smooth(l, b, x0, reverse=True).cpu().numpy()
    n_act = int(lv.direct_seg[0])
    np.testing.assert_array_equal(g[n_act:], x0[n_act:])
    # active rows: the oracle smoother of each system on its own slice
    off = 0
    for q in bt.order:
        p = probs[q]
        if len(p.levels) <= l + 1:
            continue
        m = p.levels[l].n
        o = O.smooth(p.levels[l].A, sms[q][l], x0[off:off + m], b[off:off + m], reverse=True)
        check_vec(g[off:off + m], o, APPLY_TOL, f"batch level {l} cascade apply, system {q}")
        off += m
    assert off == n_act


@pytest.mark.parametrize("which", ["small_batch", "odd_batch"])
def test_batch_solve_converges_per_system(gpu_lib, which, request):
    probs, bt, sms = request.getfixturevalue(which)
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3)
    s.set_systems(bt.sys_ptr)
    rtol = 1e-10
    x, info = s.solve(bt.rhs, rtol=rtol, maxit=200)
    its, rels = s.system_stats()
    xs = bt.split(x.cpu().numpy())
    for q, s_in in enumerate(bt.order):
        p = probs[s_in]
        r = p.rhs - p.levels[0].A @ xs[s_in]
        true_rel = float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)))
        assert true_rel <= rtol
        # the two residuals differ by the rounding of b - A x: a few ulps of |A||x|
        floor = 64 * np.finfo(float).eps * float(np.max(
            np.linalg.norm(abs(p.levels[0].A) @ abs(xs[s_in]), axis=0) / np.linalg.norm(p.rhs, axis=0)))
        assert abs(rels[q] - true_rel) <= 1e-6 * true_rel + floor
        # the V-cycles this system needed on its own (oracle, FP64)
        _, hist = O.solve(p.levels, sms[s_in], p.rhs, rtol=rtol, maxit=200)
        k = len(hist) - 1
        margin = abs(np.log(hist[k] / rtol)) > 1e-6 and (k == 0 or abs(np.log(hist[k - 1] / rtol)) > 1e-6)
        if margin:
            assert its[q] == k, (q, its[q], k)
    assert info["iterations"] == its.max()
    assert info["rel_res"] == pytest.approx(rels.max(), rel=1e-12)


def test_batch_fp32_solve(gpu_lib, small_batch):
    probs, bt, _ = small_batch
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3, precision="fp32")
    s.set_systems(bt.sys_ptr)
    x, info = s.solve(bt.rhs, rtol=1e-10, maxit=200)
    its, rels = s.system_stats()
    assert (rels <= 1e-10).all() and its.max() == info["iterations"]
    xs = bt.split(x.cpu().numpy())
    for p, xq in zip(probs, xs):
        r = p.rhs - p.levels[0].A @ xq
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-10


def test_set_systems_validation(gpu_lib, small_batch):
    _, bt, _ = small_batch
    s = gpu_lib.Solver(bt.levels)
    with pytest.raises(gpu_lib.CascadeError):
        s.set_systems(np.array([0, 5, 3, bt.levels[0].n]))
    with pytest.raises(gpu_lib.CascadeError):
        s.set_systems(np.array([0, bt.levels[0].n - 1]))
    with pytest.raises(gpu_lib.CascadeError):
        s.system_stats()          # no solve has run
    s.set_systems(None)


def _bad(levels, l, **kw):
    out = list(levels)
    lv = levels[l]
    out[l] = type(lv)(**{**lv.__dict__, **kw})
    return out


def test_direct_segment_validation(gpu_lib, small_batch):
    _, bt, _ = small_batch
    lv = bt.levels
    l = next(i for i, v in enumerate(lv[:-1]) if v.direct_seg is not None)
    seg = lv[l].direct_seg
    # a segment that does not end at n
    with pytest.raises(gpu_lib.CascadeError):
        gpu_lib.Solver(_bad(lv, l, direct_seg=np.concatenate([seg[:-1], [seg[-1] - 1]])))
    # a segment boundary that cuts a system (rows couple across it)
    cut = seg.copy()
    cut[-2] += 1
    with pytest.raises(gpu_lib.CascadeError):
        gpu_lib.Solver(_bad(lv, l, direct_seg=cut))
    # the last level must be solved directly in full
    last = lv[-1].direct_seg
    assert len(last) > 2
    with pytest.raises(gpu_lib.CascadeError):
        gpu_lib.Solver(_bad(lv, len(lv) - 1, direct_seg=last[1:]))
    # P with entries in a direct row
    P = lv[l].P.tolil()
    P[lv[l].n - 1, 0] = 1.0
    with pytest.raises(gpu_lib.CascadeError):
        gpu_lib.Solver(_bad(lv, l, P=P.tocsr()))


def test_batch_save_load_roundtrip(gpu_lib, small_batch, tmp_path):
    _, bt, _ = small_batch
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3)
    b = bt.rhs[:, :2].copy()
    y = s.vcycle(b).cpu().numpy()
    path = str(tmp_path / "batch.cs")
    s.save(path)
    t = gpu_lib.Solver(bt.levels)
    t.setup(depth=1)
    t.load(path)
    np.testing.assert_array_equal(t.vcycle(b).cpu().numpy(), y)
