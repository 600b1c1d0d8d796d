"""Sketched cascade construction (cs_setup_sketched) against the oracle's
fit_sketched on the same sketch.

Tolerances: the sketched normal equations are formed from the same products
as the exact ones, so the Lambda blocks agree to the exact fit's per-block
bound 16384 u cond(G_i) (cond from the oracle, worst up to the cascade level;
tests/parity.py), relative to the block's norm or, for blocks of rounding
size, to 1e-6 of the level's largest block.  With S = [I 0] the sketch is the
exact fit.
"""
import numpy as np
import pytest

import oracle as O
from parity import level_bounds, record
from synth import fd
from synth.batch import concatenate

pytestmark = pytest.mark.gpu


# A sketch of s <= 8 columns can leave a block's residual rows almost
# cancelled after the first cascade level (few columns, each nearly fitted), so
# the next level's blocks are ratios of cancelled quantities: their relative
# accuracy is set by that cancellation, which cond(G) does not measure.  Such
# narrow sketches get an absolute floor of 1e-9 beside the conditioning bound.
NARROW_FLOOR = 1e-9


def check_levels(s, sm_list, sizes, depth, width=64):
    floor = NARROW_FLOOR if width <= 8 else 0.0
    for l, sm in enumerate(sm_list):
        for ell in range(1, depth + 1):
            g, o = s.get_smoother(l, ell), sm["lam"][ell - 1]
            num = np.linalg.norm((g - o).reshape(len(g), -1), axis=1)
            # blocks whose sketch residual vanishes (a narrow sketch fitted exactly at
            # an earlier level) have Lambda of rounding size: measure those against
            # the level's scale
            no = np.linalg.norm(o.reshape(len(o), -1), axis=1)
            den = np.maximum(no, 1e-6 * max(no.max(), 1e-300))
            bound = level_bounds(sm["gram_cond"], ell) + floor
            k = int(np.argmax(num / den / bound))
            ratio = record(f"sketched level {l} Lambda_{ell}", num[k] / den[k], bound[k])
            assert ratio <= 1.0, (l, ell, ratio)


def oracle_sketched(levels, S, width, depth, mode="additive"):
    out, off = [], 0
    for lv in levels[:-1]:
        Sl = S[off:off + lv.A.shape[0]]
        off += lv.A.shape[0]
        out.append(O.fit_sketched(lv.A, lv.block_size, depth, Sl, mode=mode, colours=lv.colour))
    return out


@pytest.mark.parametrize("case", ["interface16_blocks8", "poisson64_points", "lognormal32_red_black"])
def test_sketched_setup_matches_oracle(gpu_lib, case):
    if case == "interface16_blocks8":
        p, mode, width, depth = fd.interface3d(16, nrhs=1), "additive", 24, 3
    elif case == "poisson64_points":
        p, mode, width, depth = fd.poisson2d(64), "additive", 16, 3
    else:
        p, mode, width, depth = fd.lognormal2d(32, nrhs=1, n_stop=4), "multiplicative", 16, 2
        for lv in p.levels:
            lv.colour = fd.parity_colour(int(round(np.sqrt(lv.n))), 2, 1, lv.cells)
    s = gpu_lib.Solver(p.levels)
    S = s.setup_sketched(width=width, seed=5, depth=depth, mode=mode).cpu().numpy()
    assert set(np.unique(S)) <= {-1.0, 1.0}
    check_levels(s, oracle_sketched(p.levels, S, width, depth, mode), None, depth, width)


def test_identity_sketch_is_the_exact_fit(gpu_lib):
    p = fd.poisson2d(8)
    width = 64
    blocks = []
    for lv in p.levels[:-1]:
        n = lv.A.shape[0]
        blocks.append(np.hstack([np.eye(n), np.zeros((n, width - n))]))
    S = np.vstack(blocks)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3)
    exact = [[s.get_smoother(l, ell) for ell in (1, 2, 3)] for l in range(len(p.levels) - 1)]
    s.setup_sketched(width=width, sketch=S, depth=3)
    for l in range(len(p.levels) - 1):
        for ell in (1, 2, 3):
            np.testing.assert_allclose(s.get_smoother(l, ell), exact[l][ell - 1], rtol=1e-9, atol=1e-13)


def test_sketched_cascade_solves(gpu_lib):
    p = fd.interface3d(32, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision="fp32")
    _, ex = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    s.setup_sketched(width=32, seed=1, depth=3, precision="fp32")
    x, sk = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    r = p.rhs - p.levels[0].A @ x.cpu().numpy()
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-10
    print(f"rho exact {ex['rho']:.4f} ({ex['iterations']} it), sketched s=32 {sk['rho']:.4f} ({sk['iterations']} it)")
    assert sk["iterations"] <= 3 * ex["iterations"]


def test_sketched_setup_on_a_batch(gpu_lib):
    sizes = [48, 64, 16, 32, 8]
    probs = fd.lognormal_batch(len(sizes), nrhs=2, sizes=sizes, config_id=16)
    bt = concatenate(probs)
    s = gpu_lib.Solver(bt.levels)
    s.set_systems(bt.sys_ptr)
    S = s.setup_sketched(width=16, seed=2, depth=3).cpu().numpy()
    x, info = s.solve(bt.rhs, rtol=1e-10, maxit=300, method="cg")
    assert info["rel_res"] <= 1e-10
    # the smoothed rows of every level match the oracle on the stacked operator
    sm = oracle_sketched(bt.levels, S, 16, 3)
    for l, lv in enumerate(bt.levels[:-1]):
        act = int(lv.direct_seg[0]) if lv.direct_seg is not None else lv.A.shape[0]
        for ell in (1, 2, 3):
            g, o = s.get_smoother(l, ell), sm[l]["lam"][ell - 1]
            nb = lv.block_size
            ab = act // nb
            np.testing.assert_allclose(g[:ab], o[:ab], rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("width,depth", [(1, 1), (4, 2), (8, 3), (64, 2)])
def test_sketch_width_limits(gpu_lib, width, depth):
    """Widths 1..64; a single column is fitted exactly by a point block, so a
    deeper cascade needs s > n (rejected otherwise).  Very narrow sketches
    (s = 2, n = 1) leave whole neighbourhoods with a vanishing residual, whose
    next-level blocks are ratios of rounding noise: not compared."""
    p = fd.poisson2d(32)
    s = gpu_lib.Solver(p.levels)
    S = s.setup_sketched(width=width, seed=9, depth=depth).cpu().numpy()
    check_levels(s, oracle_sketched(p.levels, S, width, depth), None, depth, width)
    with pytest.raises(gpu_lib.CascadeError):
        s.setup_sketched(width=65, seed=9, depth=2)
    with pytest.raises(gpu_lib.CascadeError):
        s.setup_sketched(width=1, seed=9, depth=2)
