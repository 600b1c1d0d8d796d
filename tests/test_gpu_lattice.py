"""Stencil-repetition setup cache (Sec. 4) on the GPU, through the C ABI.

With lattice points declared for the smoothed levels, the exact additive setup
fits one block per translation class and copies the rest.  Checked here:
  * the class representatives at every radius equal the oracle's brute-force
    classes, bit-exactly, and the fitted counts are the class counts;
  * the cached smoothers equal the oracle's plain fit to the bounds of the
    uncached setup parity (per block from the oracle's condition numbers,
    tests/parity.py), the residual patterns bit-exactly, the FP64 V-cycle to
    1e-12 (2-norm and per entry);
  * cached against uncached on the GPU: the same patterns and singular counts,
    smoothers within the same per-block bounds (1e-10 for the 32^3 case,
    which has no oracle fit), the same iteration counts;
  * settings the cache does not serve (multiplicative, truncation) fit every
    block and give the uncached results; argument and state errors.
"""
import numpy as np
import pytest

import oracle as O
from parity import VCYCLE_TOL, check_blocks, check_level_smoothers, check_vec, level_bounds, rel2
from synth import fd
from synth.problem import Problem
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu


def rel(a, b):
    return rel2(a, b)


def disk2d(n=48, bs=2):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    mu = np.where((X - 0.45) ** 2 + (Y - 0.55) ** 2 < 0.2 ** 2, 100.0, 1.0)
    levels = fd.fv_hierarchy(mu, bs=bs, n_stop=6, order="lex")
    rhs = stream(5, TEST, n).uniform(-1, 1, size=(n * n, 2))
    return Problem(f"disk2d_{n}", levels, rhs, meta=dict(d=2, n=n))


CASES = {
    "poisson2d_32_point": lambda: fd.poisson2d(32),
    "disk2d_48_lex_2x2": disk2d,
    "interface3d_16_morton_2x2x2": lambda: fd.interface3d(16, nrhs=2),
}


def with_lattice(cascade, prob):
    s = cascade.Solver(prob.levels)
    for l, lv in enumerate(prob.levels[:-1]):
        s.set_lattice(l, lv.block_lattice())
    return s


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    p = CASES[request.param]()
    print(f"[lattice] case {request.param}: {p.n} unknowns, {len(p.levels)} levels", flush=True)
    depth = 3
    sm = O.setup_hierarchy(p.levels, depth, "additive")
    reps = []
    for lv in p.levels[:-1]:
        coords = lv.block_lattice()
        reps.append([O.lattice_classes(lv.A, lv.block_size, coords, r) for r in range(depth)])
    return request.param, p, depth, sm, reps


def test_classes_match_oracle(gpu_lib, case):
    name, p, depth, sm, reps = case
    s = with_lattice(gpu_lib, p)
    s.setup(depth=depth)
    for l in range(len(p.levels) - 1):
        fitted, rep = s.lattice_stats(l, classes=True)
        for r in range(depth):
            np.testing.assert_array_equal(rep[r], reps[l][r], err_msg=f"{name} level {l} radius {r}")
            assert fitted[r] == len(np.unique(reps[l][r])), (name, l, r)
    # classes refine with the radius; the first step always shares work here
    fitted = s.lattice_stats(0)
    assert fitted[0] < p.levels[0].n_blocks and np.all(np.diff(fitted) >= 0), fitted


def test_cached_setup_matches_oracle(gpu_lib, case):
    name, p, depth, sm, _ = case
    s = with_lattice(gpu_lib, p)
    s.setup(depth=depth, order="FF")
    for l in range(len(p.levels) - 1):
        check_level_smoothers(s, sm[l], l, depth, f"lattice-cached {name}")
        for step, pat in enumerate(sm[l]["patterns"]):
            ptr, col = s.get_pattern(l, step)
            pat = pat.tocsr()
            pat.sort_indices()
            np.testing.assert_array_equal(ptr, pat.indptr.astype(np.int64))
            np.testing.assert_array_equal(col, pat.indices.astype(np.int32))
    o = O.vcycle(p.levels, sm, p.rhs, "FF", 1, 1)
    g = s.vcycle(p.rhs).cpu().numpy()
    check_vec(g, o, VCYCLE_TOL, f"lattice-cached {name} FF V-cycle, own setup")


def test_cached_against_uncached(gpu_lib, case):
    name, p, depth, sm, _ = case
    plain = gpu_lib.Solver(p.levels)
    plain.setup(depth=depth)
    s = with_lattice(gpu_lib, p)
    s.setup(depth=depth)
    for l in range(len(p.levels) - 1):
        for ell in range(1, depth + 1):
            check_blocks(s.get_smoother(l, ell), plain.get_smoother(l, ell), level_bounds(sm[l]["gram_cond"], ell),
                         f"lattice-cached vs uncached {name} level {l} Lambda_{ell}")
        for step in range(depth):
            a, b = s.get_pattern(l, step), plain.get_pattern(l, step)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
    x1, i1 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    x0, i0 = plain.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    assert i1["iterations"] == i0["iterations"]
    assert i1["singular_blocks"] == i0["singular_blocks"]
    assert rel(x1.cpu().numpy(), x0.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("opts", [dict(mode="multiplicative"), dict(alpha=3)])
def test_settings_without_cache_fit_every_block(gpu_lib, opts):
    p = fd.poisson2d(32)
    plain = gpu_lib.Solver(p.levels)
    plain.setup(depth=2, **opts)
    s = with_lattice(gpu_lib, p)
    s.setup(depth=2, **opts)
    for l in range(len(p.levels) - 1):
        fitted, rep = s.lattice_stats(l, classes=True)
        B = p.levels[l].n_blocks
        assert np.all(fitted == B)
        np.testing.assert_array_equal(rep, np.tile(np.arange(B, dtype=np.int32), (2, 1)))
        for ell in (1, 2):
            np.testing.assert_array_equal(s.get_smoother(l, ell), plain.get_smoother(l, ell))


def test_lattice_with_deeper_cascade_and_fp32(gpu_lib):
    """Depth 4 on the 3D interface problem (32^3), FP32 V-cycle in CG."""
    p = fd.interface3d(32, nrhs=4)
    plain = gpu_lib.Solver(p.levels)
    plain.setup(depth=4, precision="fp32")
    s = with_lattice(gpu_lib, p)
    s.setup(depth=4, precision="fp32")
    fitted = s.lattice_stats(0)
    print(f"[lattice] 32^3 fitted per step {fitted.tolist()} of {p.levels[0].n_blocks}", flush=True)
    for ell in range(1, 5):
        check_blocks(s.get_smoother(0, ell), plain.get_smoother(0, ell), 1e-10,
                     f"lattice-cached vs uncached interface3d_32 Lambda_{ell}")
    _, i1 = s.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    _, i0 = plain.solve(p.rhs, rtol=1e-10, maxit=100, method="cg")
    assert i1["rel_res"] <= 1e-10 and i1["iterations"] == i0["iterations"]


def test_lattice_errors(gpu_lib):
    p = fd.poisson2d(16)
    s = gpu_lib.Solver(p.levels)
    c = p.levels[0].block_lattice()
    bad = c.copy()
    bad[1] = bad[0]
    with pytest.raises(RuntimeError, match="distinct"):
        s.set_lattice(0, bad)
    with pytest.raises(RuntimeError, match="no smoother"):
        s.set_lattice(len(p.levels) - 1, p.levels[-1].block_lattice())
    with pytest.raises(RuntimeError, match="must lie in"):
        s.set_lattice(0, c.astype(np.int64) * (1 << 28))
    with pytest.raises(RuntimeError, match="box"):
        far = c.copy()
        far[:, 0] *= 1 << 23
        s.set_lattice(0, far)
    with pytest.raises(RuntimeError, match="dimension"):
        s.set_lattice(0, np.zeros((p.levels[0].n_blocks, 4), dtype=np.int32))
    with pytest.raises(RuntimeError, match="no setup"):
        s.lattice_stats(0)
    s.set_lattice(0, c)
    s.setup_sketched(width=8, depth=2)
    with pytest.raises(RuntimeError, match="not an exact block fit"):
        s.lattice_stats(0)
    s.setup(depth=2)
    assert s.lattice_stats(0)[0] < p.levels[0].n_blocks
    s.set_lattice(0, None)
    s.setup(depth=2)
    assert s.lattice_stats(0)[0] == p.levels[0].n_blocks
