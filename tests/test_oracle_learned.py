"""Pins of the learned-setup oracle (CPU): central differences for the
gradient, closed forms for SiLU, Adam's first step and the block features."""
import numpy as np
import pytest

from oracle import learned as OL
from synth.rng import TEST, stream


def small_net(n_in=7, width=5, n_out=3, seed=0):
    rng = stream(50, TEST, seed)
    sz = sum(int(np.prod(s)) for s in OL.shapes(n_in, width, n_out))
    return rng.normal(0, 0.5, size=sz), rng


def test_silu_derivative_closed_form():
    z = np.linspace(-8, 8, 41)
    h = 1e-6
    fd = (OL.silu(z + h) - OL.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(OL.dsilu(z), fd, rtol=1e-8, atol=1e-10)
    assert OL.silu(0.0) == 0.0 and OL.dsilu(0.0) == 0.5
    np.testing.assert_allclose(OL.silu(np.array([40.0, -40.0])), [40.0, 0.0], atol=1e-15)


def test_gradient_matches_central_differences():
    n_in, width, n_out = 7, 5, 3
    flat, rng = small_net(n_in, width, n_out)
    X = rng.normal(size=(11, n_in))
    T = rng.normal(size=(11, n_out)) * 3 + 1
    mean, std = OL.output_scaling(T)
    _, grads = OL.loss_and_grad(OL.unpack(flat, n_in, width, n_out), X, T, mean, std)
    g = np.concatenate([a.ravel() for a in grads])
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(len(flat)):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = OL.loss_and_grad(OL.unpack(flat + e, n_in, width, n_out), X, T, mean, std)
        lm, _ = OL.loss_and_grad(OL.unpack(flat - e, n_in, width, n_out), X, T, mean, std)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_loss_is_zero_at_the_fitted_output_and_scaling_inverts():
    n_in, width, n_out = 4, 6, 2
    flat, rng = small_net(n_in, width, n_out, seed=1)
    p = OL.unpack(flat, n_in, width, n_out)
    X = rng.normal(size=(9, n_in))
    mean, std = np.array([2.0, -1.0]), np.array([0.5, 4.0])
    T = OL.predict(p, X, mean, std)
    loss, grads = OL.loss_and_grad(p, X, T, mean, std)
    assert loss < 1e-28 and max(np.abs(g).max() for g in grads) < 1e-14
    m, s = OL.output_scaling(np.array([[1.0, 5.0], [3.0, 5.0]]))
    np.testing.assert_array_equal(m, [2.0, 5.0])
    np.testing.assert_array_equal(s, [1.0, 1.0])      # zero deviation replaced by 1


def test_adam_first_step_closed_form():
    rng = stream(50, TEST, 2)
    p, g = rng.normal(size=20), rng.normal(size=20)
    q, m, v = OL.adam_step(p, g, np.zeros(20), np.zeros(20), 1, lr=1e-3)
    # bias correction makes m^ = g and v^ = g^2 after the first step
    np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_decreases_the_loss():
    n_in, width, n_out = 6, 16, 2
    flat, rng = small_net(n_in, width, n_out, seed=3)
    flat = flat * 0.3
    X = rng.normal(size=(64, n_in))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1], X[:, 2] * X[:, 3]], axis=1)
    mean, std = OL.output_scaling(T)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    l0, _ = OL.loss_and_grad(OL.unpack(flat, n_in, width, n_out), X, T, mean, std)
    for t in range(1, 201):
        _, gr = OL.loss_and_grad(OL.unpack(flat, n_in, width, n_out), X, T, mean, std)
        flat, m, v = OL.adam_step(flat, np.concatenate([a.ravel() for a in gr]), m, v, t, 1e-2)
    l1, _ = OL.loss_and_grad(OL.unpack(flat, n_in, width, n_out), X, T, mean, std)
    assert l1 < 0.2 * l0


def test_feature_closed_forms():
    n = 12
    nb = n // 2
    F = OL.block_features(np.full((n, n, n), 2.5))
    assert F.shape == (nb ** 3, 1464)
    assert np.all(F[:, :729] == 0.0)                 # constant field: no contrast
    masks = F[:, 729:1458].sum(axis=1).reshape(nb, nb, nb)
    assert masks[0, 0, 0] == 5 ** 3                   # hexes -4..4 around node 0: 5 inside per axis
    assert masks[-1, -1, -1] == 6 ** 3                # 2(nb-1)-4 .. n-1: 6 inside per axis
    assert masks[2, 2, 2] == 9 ** 3
    assert masks[0, 2, 2] == 5 * 81                   # z = 0 face
    d = F[:, 1458:].reshape(nb, nb, nb, 6)            # [K, J, I, face]
    np.testing.assert_array_equal(d[0, 0, 0], [0, 1, 0, 1, 0, 1])          # distance 5 clipped to 4
    np.testing.assert_array_equal(d[2, 1, 5], [1, 0, 0.25, 1, 0.5, 0.75])  # I=5, J=1, K=2


def test_feature_single_hex_contrast():
    n = 12
    lm = np.zeros((n, n, n))
    lm[5, 6, 7] = 3.0                                 # hex (i, j, k) = (7, 6, 5)
    F = OL.block_features(lm)
    nb = n // 2
    I, J, K = 3, 3, 2                                 # block whose patch holds it (interior: 729 hexes)
    b = I + nb * (J + nb * K)
    u, v, w = 7 - (2 * I - 4), 6 - (2 * J - 4), 5 - (2 * K - 4)
    vals = F[b, :729]
    mean = 3.0 / 729
    assert vals[u + 9 * v + 81 * w] == pytest.approx((3.0 - mean) / 3.0, rel=1e-15)
    others = np.delete(vals, u + 9 * v + 81 * w)
    np.testing.assert_allclose(others, -mean / 3.0, rtol=1e-15)
    # a block whose patch misses it has no contrast
    assert np.all(F[0, :729] == 0.0)
