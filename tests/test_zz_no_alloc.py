"""cs_vcycle_noalloc (the V-cycle whose workspace is the library's static
device array, for callers that cannot allocate) against cs_vcycle.

The two entry points run the same kernels in the same order on the same
setup, so their results must be bit-identical.  Checked on two calls in a
row, the second with a smaller input (fewer right-hand sides), in FP64 and
FP32, and with regular calls before and after (the context's own workspace
must be restored); sizes beyond the array are refused with CS_EINVAL.
"""
import ctypes

import numpy as np
import pytest

from synth import fd

pytestmark = pytest.mark.gpu


def _noalloc(s, b, x):
    """cs_vcycle_noalloc through the C ABI; x receives V b."""
    st = s._lib.cs_vcycle_noalloc(s._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), b.shape[1])
    s._torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_vcycle_equals_vcycle(gpu_lib, precision):
    import torch
    p = fd.interface3d(24, nrhs=8)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, precision=precision)
    dev = torch.device("cuda", 0)
    for nrhs in (8, 2):                       # the second call with a smaller input
        b = torch.as_tensor(np.ascontiguousarray(p.rhs[:, :nrhs]), device=dev)
        ref = s.vcycle(b).cpu().numpy()       # regular call: the context's own workspace
        x = torch.full_like(b, np.nan)
        assert _noalloc(s, b, x) == 0, s._lib.cs_last_error(s._h).decode()
        got = x.cpu().numpy()
        print(f"[noalloc] {precision} nrhs={nrhs}: max |noalloc - vcycle| = {np.max(np.abs(got - ref)):.1e}")
        np.testing.assert_array_equal(got, ref)
        # a regular call after the static-scratch call gives the same result again
        np.testing.assert_array_equal(s.vcycle(b).cpu().numpy(), ref)
    s.close()


def test_noalloc_refuses_oversize_and_bad_arguments(gpu_lib):
    import torch
    p = fd.interface3d(64, nrhs=8)            # FP64, 8 RHS: ~76 MB of workspace > 64 MiB
    s = gpu_lib.Solver(p.levels)
    b = torch.as_tensor(p.rhs, device="cuda")
    x = torch.empty_like(b)
    assert _noalloc(s, b, x) == -7            # before setup: CS_ESTATE
    s.setup(depth=2, precision="fp64")
    assert _noalloc(s, b, x) == -1            # CS_EINVAL: beyond the static array
    assert "static scratch" in s._lib.cs_last_error(s._h).decode()
    b1 = b[:, :1].contiguous()
    x1 = torch.empty_like(b1)
    assert _noalloc(s, b1, x1) == 0           # one RHS fits
    np.testing.assert_array_equal(x1.cpu().numpy(), s.vcycle(b1).cpu().numpy())
    b3 = b[:, :3].contiguous()
    assert _noalloc(s, b3, torch.empty_like(b3)) == -1   # nrhs must be 1, 2, 4 or 8
    s.close()
