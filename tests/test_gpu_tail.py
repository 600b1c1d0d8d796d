"""Single-workgroup tail V-cycle (cs_set_tail): the coarse levels of at most a
few thousand rows run Alg. 1 as one launch with workgroup barriers between the
steps.  Each row's arithmetic is the per-level kernels' own, in the same
order, so V-cycles and whole solves must be bit-identical with the tail on and
off - for point and block levels, every right-hand-side count, both working
precisions, a batch whose systems end on different levels (direct segments on
intermediate levels), graph replay, and the allocation-free entry point (which
always runs the per-level launches)."""
import numpy as np
import pytest

from synth import fd
from synth.batch import concatenate

pytestmark = pytest.mark.gpu


def _vcycle(s, b, tail):
    s.set_tail(tail)
    return s.vcycle(b).cpu().numpy()


def _check_vcycle(s, b, label):
    s.set_tail(4096)
    m, first = s.tail()
    assert m == 4096 and first >= 0, (label, first)   # the tail is in use
    x0 = _vcycle(s, b, 0)
    x1 = _vcycle(s, b, 4096)
    x2 = _vcycle(s, b, 4096)   # the table is reused
    print(f"[tail] {label}: tail from level {first} of {len(s.sizes)}, |x| {np.linalg.norm(x0):.6e}")
    np.testing.assert_array_equal(x1, x0)
    np.testing.assert_array_equal(x2, x0)
    return first


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nrhs", [1, 2, 4, 8])
def test_tail_vcycle_blocks8_3d(gpu_lib, precision, nrhs):
    p = fd.interface3d(32, nrhs=nrhs)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision=precision)
    _check_vcycle(s, p.rhs, f"interface3d_32 nb=8 {precision} nrhs={nrhs}")
    s.setup(depth=2, order="FF", n_pre=2, n_post=1, precision=precision)
    _check_vcycle(s, p.rhs, f"interface3d_32 FF V(2,1) {precision} nrhs={nrhs}")
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tail_vcycle_points_2d(gpu_lib, precision):
    p = fd.poisson2d(64, nrhs=2)   # levels of 4096, 1024, 256, 64 and 16 rows
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision=precision)
    assert _check_vcycle(s, p.rhs, f"poisson2d_64 {precision}") == 0   # the whole V-cycle in one launch
    s.set_tail(1024)
    assert s.tail()[1] == 1
    x0 = _vcycle(s, p.rhs, 0)
    np.testing.assert_array_equal(_vcycle(s, p.rhs, 1024), x0)
    for method in ("ir", "cg"):   # with the tail from level 0 the refinement issues no early sweep
        s.set_tail(0)
        xa, ia = s.solve(p.rhs, rtol=1e-10, maxit=100, method=method)
        s.set_tail(4096)
        xb, ib = s.solve(p.rhs, rtol=1e-10, maxit=100, method=method)
        assert ib["iterations"] == ia["iterations"]
        np.testing.assert_array_equal(xb.cpu().numpy(), xa.cpu().numpy())
        np.testing.assert_array_equal(ib["history"], ia["history"])
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tail_vcycle_2d_blocks4(gpu_lib, precision):
    rng = np.random.default_rng(7)
    levels = fd.fv_hierarchy(np.exp(rng.standard_normal((64, 64))), bs=2, n_stop=4)
    b = rng.standard_normal((64 * 64, 2))
    s = gpu_lib.Solver(levels)
    s.setup(depth=2, precision=precision)
    _check_vcycle(s, b, f"lognormal 64^2 blocks 2x2 {precision}")
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tail_solves_identical(gpu_lib, precision):
    p = fd.interface3d(32, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision=precision)
    for method in ("ir", "cg"):
        s.set_tail(0)
        x0, i0 = s.solve(p.rhs, rtol=1e-10, maxit=200, method=method)
        s.set_tail(4096)
        x1, i1 = s.solve(p.rhs, rtol=1e-10, maxit=200, method=method)
        assert i1["iterations"] == i0["iterations"]
        np.testing.assert_array_equal(x1.cpu().numpy(), x0.cpu().numpy())
        np.testing.assert_array_equal(i1["history"], i0["history"])
        print(f"[tail] solve {precision} {method}: {i0['iterations']} it, "
              f"{i0['solve_ms']:.2f} ms per-level, {i1['solve_ms']:.2f} ms tail")
    s.close()


def test_tail_batch_with_direct_segments(gpu_lib):
    sizes = [48, 64, 80, 16, 112, 32, 80, 8]
    bt = concatenate(fd.lognormal_batch(len(sizes), nrhs=4, sizes=sizes, config_id=14))
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3, precision="fp32")
    s.set_systems(bt.sys_ptr)
    _check_vcycle(s, bt.rhs, "batch of 8 lognormal2d")
    s.set_tail(0)
    x0, i0 = s.solve(bt.rhs, rtol=1e-10, maxit=300, method="ir")
    st0 = s.system_stats()
    s.set_tail(4096)
    x1, i1 = s.solve(bt.rhs, rtol=1e-10, maxit=300, method="ir")
    st1 = s.system_stats()
    np.testing.assert_array_equal(x1.cpu().numpy(), x0.cpu().numpy())
    np.testing.assert_array_equal(st1[0], st0[0])
    np.testing.assert_array_equal(st1[1], st0[1])
    s.close()


def test_tail_with_graphs_and_noalloc(gpu_lib):
    p = fd.interface3d(32, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision="fp32")
    s.set_tail(4096)
    import torch
    b = torch.as_tensor(p.rhs, device="cuda").contiguous()
    x0 = s.vcycle(b).cpu().numpy()
    xn = s.vcycle_noalloc(b, torch.empty_like(b)).cpu().numpy()   # per-level launches on the static array
    np.testing.assert_array_equal(xn, x0)
    x1 = s.vcycle(b).cpu().numpy()               # back on the context's buffers: table rebuilt
    np.testing.assert_array_equal(x1, x0)
    s.set_tail(0)
    s.set_graphs(False)
    xe, ie = s.solve(p.rhs, rtol=1e-10, maxit=200, method="ir")
    s.set_tail(4096)
    s.set_graphs(True)
    for _ in range(2):
        xg, ig = s.solve(p.rhs, rtol=1e-10, maxit=200, method="ir")
        assert ig["iterations"] == ie["iterations"]
        np.testing.assert_array_equal(xg.cpu().numpy(), xe.cpu().numpy())
    s.set_graphs(False)
    s.close()


def test_tail_settings(gpu_lib):
    p = fd.interface3d(32, nrhs=1)              # levels of 32768, 4096, 512 and 64 rows
    s = gpu_lib.Solver(p.levels)
    assert s.tail() == (0, -1)                 # off by default; no setup yet
    s.setup(depth=2)
    assert s.tail()[1] == -1
    s.set_tail(4096)
    assert s.tail()[1] == 1
    s.set_tail(1000)
    assert s.tail()[1] == 2
    s.set_tail(100)                             # only the bottom level is that small
    assert s.tail()[1] == -1
    s.set_tail(0)
    assert s.tail() == (0, -1)
    with pytest.raises(Exception, match="tail max_rows"):
        s.set_tail(-1)
    with pytest.raises(Exception, match="tail max_rows"):
        s.set_tail(1 << 20)
    s.close()


def test_autotune_picks_the_fastest_tail(gpu_lib):
    p = fd.poisson2d(64, nrhs=1)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, n_pre=2, n_post=2, precision="fp64")
    x0, i0 = s.solve(p.rhs, rtol=1e-10, maxit=100)
    s.autotune(1)
    cand = s.tail_candidates()
    rows, first = s.tail()
    print(f"[tail] autotune 64^2 V(2,2): {[(r, round(t, 4)) for r, t in cand]} -> max_rows {rows}, level {first}")
    assert cand[0][0] == 0 and len(cand) >= 2 and all(t > 0 for _, t in cand)
    assert rows == min(cand, key=lambda c: c[1])[0]
    x1, i1 = s.solve(p.rhs, rtol=1e-10, maxit=100)
    assert i1["iterations"] == i0["iterations"]
    np.testing.assert_array_equal(x1.cpu().numpy(), x0.cpu().numpy())
    s.close()
