"""Graph replay of the outer iterations (cs_set_graphs): every refinement / CG
iteration after the first is one launch of a captured HIP graph.  Replays
issue exactly the captured kernels, so solutions, residual histories and
per-system statistics must be bit-identical to eager launches - for a batch
of independent systems and a single system, and still after the graph has to
be recaptured (another precision, another setup, another method)."""
import numpy as np
import pytest

from synth import fd
from synth.batch import concatenate

pytestmark = pytest.mark.gpu

SIZES = [48, 64, 80, 16, 112, 32, 80, 8]


def _solve(s, b, method, maxit=300):
    x, info = s.solve(b, rtol=1e-10, maxit=maxit, method=method, raise_on_noconv=False)
    return x.cpu().numpy(), info


def _same(s, b, method, maxit=300, systems=False):
    s.set_graphs(False)
    x0, i0 = _solve(s, b, method, maxit)
    st0 = s.system_stats() if systems else None
    s.set_graphs(True)
    for _ in range(2):   # capture, then pure replay
        x1, i1 = _solve(s, b, method, maxit)
        assert i1["iterations"] == i0["iterations"], (method, i1["iterations"], i0["iterations"])
        np.testing.assert_array_equal(x1, x0)
        np.testing.assert_array_equal(i1["history"], i0["history"])
        if systems:
            st1 = s.system_stats()
            np.testing.assert_array_equal(st1[0], st0[0])
            np.testing.assert_array_equal(st1[1], st0[1])
    s.set_graphs(False)
    return i0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_graph_replay_is_bit_identical(gpu_lib, precision):
    bt = concatenate(fd.lognormal_batch(len(SIZES), nrhs=4, sizes=SIZES, config_id=14))
    s = gpu_lib.Solver(bt.levels)
    s.setup(depth=3, precision=precision)
    s.set_systems(bt.sys_ptr)
    for method in ("cg", "ir"):
        info = _same(s, bt.rhs, method, maxit=400, systems=True)
        print(f"[graphs] batch {precision} {method}: {info['iterations']} it, {info['solve_ms']:.2f} ms eager")
    s.close()


def test_single_system_graph_replay_after_precision_and_setup_changes(gpu_lib):
    p = fd.interface3d(24, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision="fp32")
    for method in ("ir", "cg", "ir"):          # the method switch recaptures
        _same(s, p.rhs, method)
    s.set_precision("fp64")                     # other kernels and buffers
    _same(s, p.rhs, "cg")
    s.setup(depth=2, precision="fp32")          # a second setup replaces the smoothers
    _same(s, p.rhs, "ir")
    s.close()


def test_autotune_decides_graph_replay(gpu_lib):
    p = fd.interface3d(24, nrhs=4)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision="fp32")
    x0, i0 = _solve(s, p.rhs, "cg")
    s.autotune(4)
    on, eager, graph = s.graphs()
    print(f"[graphs] V-cycle eager {eager:.3f} ms, replayed {graph:.3f} ms -> replay {'on' if on else 'off'}")
    assert eager > 0 and graph > 0 and on == (graph < eager)
    x1, i1 = _solve(s, p.rhs, "cg")
    assert i1["iterations"] == i0["iterations"]
    np.testing.assert_array_equal(x1, x0)
    s.close()
