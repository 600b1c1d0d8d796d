"""Seed streams.

Every random draw is made from ``numpy.random.Generator(PCG64(SeedSequence(
[2606, config_id, stream_id, *extra])))``.  Streams: 0 = right-hand sides,
1 = geometry / coefficients, 2 = training data, 3 = network initialisation,
4 = test-only perturbations (smoother injection, random small matrices).
"""
import numpy as np

RHS, GEOMETRY, TRAINING, NET_INIT, TEST = 0, 1, 2, 3, 4


def stream(config_id: int, stream_id: int, *extra: int) -> np.random.Generator:
    seq = np.random.SeedSequence([2606, int(config_id), int(stream_id), *[int(e) for e in extra]])
    return np.random.Generator(np.random.PCG64(seq))


def uniform_rhs(config_id: int, n: int, nrhs: int, *extra: int) -> np.ndarray:
    """i.i.d. U[-1, 1] right-hand sides, shape (n, nrhs), RHS index fastest."""
    return stream(config_id, RHS, *extra).uniform(-1.0, 1.0, size=(n, nrhs))
