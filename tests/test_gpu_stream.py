"""cs_stream_bandwidth: the streaming reference reported beside the roofline
figures (plain kernels that only move arrays through HBM)."""
import pytest

from synth import fd

pytestmark = pytest.mark.gpu


def test_stream_reference_rates(gpu_lib):
    p = fd.poisson2d(32, nrhs=1)
    s = gpu_lib.Solver(p.levels)
    rates = {}
    for nr, nw in ((1, 0), (0, 1), (1, 1), (4, 1)):
        g, us = s.stream_bandwidth(nr, nw, 64 << 20, reps=3)
        rates[(nr, nw)] = g
        assert g > 0 and us > 0
        # bytes moved over the launch time
        assert abs(g - (64 << 20) * (nr + nw) / (us * 1e-6) / 1e9) < 1e-6 * g
    print(f"[stream] 64 MiB arrays: {rates}")
    for bad in ((0, 0), (5, 0), (1, 2), (-1, 1)):
        with pytest.raises(Exception, match="stream probe"):
            s.stream_bandwidth(bad[0], bad[1], 1 << 20, reps=1)
    with pytest.raises(Exception, match="multiple of 16"):
        s.stream_bandwidth(1, 0, 1000, reps=1)
    with pytest.raises(Exception, match="reps"):
        s.stream_bandwidth(1, 0, 1 << 20, reps=0)
    s.close()
