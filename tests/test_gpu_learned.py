"""Learned setup on the GPU against the FP64 oracle (oracle.learned).

Tolerances (FP32 kernels vs FP64 oracle):
  * network output: normwise relative 1e-5 (three FP32 GEMMs with sums of at
    most ~1.5e3 products; FP32 unit round-off 6e-8);
  * gradient: normwise relative 1e-4 per parameter tensor (the backward pass
    chains three more products and the SiLU derivative);
  * features: absolute 1e-6 (FP64 patch mean, one FP32 rounding of values of
    magnitude <= 2);
  * scaling statistics: relative 1e-5.
"""
import numpy as np
import pytest

from oracle import learned as OL
from synth import fe
from synth.rng import TEST, stream

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=float) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def L():
    from paper_2606_12577_amd import learned
    return learned


def random_case(n_in, width, n_out, n, seed):
    rng = stream(51, TEST, seed)
    X = rng.normal(size=(n, n_in)).astype(np.float32)
    T = (rng.normal(size=(n, n_out)) * rng.uniform(0.5, 3, size=n_out) + rng.normal(size=n_out)).astype(np.float32)
    return X, T, rng


# ragged sizes: none of n_in, width, n_out, rows is a multiple of the 64x64x16 tile
SHAPES = [(37, 24, 10, 200), (1464, 128, 128, 300), (5, 70, 3, 1)]


@pytest.mark.parametrize("n_in,width,n_out,n", SHAPES)
def test_forward_matches_oracle(gpu_lib, L, n_in, width, n_out, n):
    X, T, rng = random_case(n_in, width, n_out, n, 0)
    net = L.Mlp(n_in, width, n_out)
    net.init_params(seed=7)
    mean = rng.normal(size=n_out).astype(np.float32)
    std = rng.uniform(0.5, 2, size=n_out).astype(np.float32)
    net.set_scaling(mean, std)
    p = OL.unpack(net.get_params().astype(np.float64), n_in, width, n_out)
    y = net.forward(X).cpu().numpy()
    o = OL.predict(p, X.astype(np.float64), mean.astype(np.float64), std.astype(np.float64))
    assert rel(y, o) <= 1e-5


@pytest.mark.parametrize("n_in,width,n_out,n", SHAPES)
def test_gradient_matches_oracle(gpu_lib, L, n_in, width, n_out, n):
    X, T, rng = random_case(n_in, width, n_out, n + 13, 1)
    rows = rng.permutation(n + 13)[:n].astype(np.int32)          # gathered rows
    net = L.Mlp(n_in, width, n_out)
    net.init_params(seed=8)
    net.fit_scaling(T, rows)
    mean, std = net.get_scaling()
    om, os_ = OL.output_scaling(T[rows].astype(np.float64))
    np.testing.assert_allclose(mean, om, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(std, os_, rtol=1e-5)
    g, loss = net.gradient(X, T, rows)
    p = OL.unpack(net.get_params().astype(np.float64), n_in, width, n_out)
    ol, og = OL.loss_and_grad(p, X[rows].astype(np.float64), T[rows].astype(np.float64),
                              mean.astype(np.float64), std.astype(np.float64))
    assert loss == pytest.approx(ol, rel=1e-5)
    gg = OL.unpack(g.astype(np.float64), n_in, width, n_out)
    for k, (a, b) in enumerate(zip(gg, og)):
        assert rel(a, b) <= 1e-4, (k, rel(a, b))
    assert net.loss(X, T, rows) == pytest.approx(ol, rel=1e-5)


def test_adam_training_matches_oracle_loop(gpu_lib, L):
    """Two epochs of mini-batch Adam with the cosine rate (ragged last batch)
    against the same loop in FP64.  The first Adam steps move every weight by
    about lr * sign(g), so the comparison is in units of the step."""
    n_in, width, n_out, n = 12, 20, 4, 150
    X, T, rng = random_case(n_in, width, n_out, n, 2)
    net = L.Mlp(n_in, width, n_out)
    net.init_params(seed=9)
    net.fit_scaling(T)
    mean, std = (a.astype(np.float64) for a in net.get_scaling())
    p0 = net.get_params().astype(np.float64)
    epochs, batch, lr0 = 2, 64, 1e-3
    order = np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    net.train(X, T, order, batch=batch, lr0=lr0, lr_min=1e-4)
    steps = -(-n // batch)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    k = 0
    for ep in range(epochs):
        for st in range(steps):
            r = order[ep, st * batch:(st + 1) * batch]
            _, gr = OL.loss_and_grad(OL.unpack(p, n_in, width, n_out), X[r].astype(np.float64),
                                     T[r].astype(np.float64), mean, std)
            lr = OL.cosine_lr(k, epochs * steps, lr0, 1e-4)
            p, m, v = OL.adam_step(p, np.concatenate([a.ravel() for a in gr]), m, v, k + 1, lr)
            k += 1
    d = np.abs(net.get_params().astype(np.float64) - p)
    assert np.quantile(d, 0.999) <= 0.02 * lr0, np.quantile(d, 0.999)
    assert d.max() <= 2 * lr0 * k                    # no update of the wrong size anywhere


def test_training_reduces_validation_loss(gpu_lib, L):
    n_in, width, n_out, n = 16, 32, 6, 2048
    rng = stream(51, TEST, 3)
    X = rng.normal(size=(n, n_in)).astype(np.float32)
    W = rng.normal(size=(n_in, n_out))
    T = (np.tanh(X @ W) + 0.1 * X[:, :n_out] ** 2).astype(np.float32)
    net = L.Mlp(n_in, width, n_out)
    net.init_params(seed=10)
    tr, val = np.arange(1800, dtype=np.int32), np.arange(1800, n, dtype=np.int32)
    net.fit_scaling(T, tr)
    before = net.loss(X, T, val)
    order = np.stack([rng.permutation(tr) for _ in range(30)]).astype(np.int32)
    hist = net.train(X, T, order, batch=128, lr0=3e-3)
    after = net.loss(X, T, val)
    assert hist[-1] < 0.2 * hist[0] and after < 0.2 * before and after < 1.0   # beats the mean predictor


def test_features_match_oracle(gpu_lib, L):
    n = 12
    lm = np.log10(fe.grf_phases(n, seed_extra=3, corr_cells=2.0, config_id=51))
    g = L.fe_block_features(lm).cpu().numpy()
    o = OL.block_features(lm)
    assert g.shape == o.shape
    np.testing.assert_allclose(g, o, rtol=0, atol=1e-6)
    np.testing.assert_array_equal(g[:, 729:1458], o[:, 729:1458])         # mask bits exact


def test_prescaled_blocks_match_oracle(gpu_lib, L):
    """cs_get_prescaled_blocks returns W^-1 Lambda W^-1 of the Frobenius fit."""
    import oracle as O
    from paper_2606_12577_amd import cascade
    p = fe.multiphase3d(8, seed_extra=4, config_id=51)
    s = cascade.Solver(p.levels)
    s.setup(depth=2)
    got = s.get_prescaled_blocks(0).cpu().numpy()
    fit = O.fit(p.levels[0].A, 8, 2)
    d = np.sqrt(p.levels[0].A.diagonal()).reshape(-1, 8)
    for ell in range(2):
        lt = d[:, :, None] * fit["lam"][ell] * d[:, None, :]
        assert rel(got[:, ell], lt) <= 1e-6


def test_setup_learned_uses_the_network_blocks(gpu_lib, L):
    """A network with zero weights predicts its output shift for every block:
    with the shift set to one block's Frobenius Lambda~, every block must get
    that Lambda~ unscaled by its own W; coarser levels keep the Frobenius fit."""
    from paper_2606_12577_amd import cascade
    p = fe.multiphase3d(16, seed_extra=5, config_id=51)
    s = cascade.Solver(p.levels)
    s.setup(depth=2)
    T = s.get_prescaled_blocks(0).reshape(512, -1).cpu().numpy()
    X = L.fe_block_features(p.meta["log10mu"])
    net = L.Mlp(1464, 16, 128)
    net.set_params(np.zeros(net.n_params))
    net.set_scaling(T[5], np.ones(128))                # y = 0 -> prediction = T[5] for every block
    s.setup_learned(net, X, depth=2)
    w = 1.0 / np.sqrt(p.levels[0].A.diagonal()).reshape(-1, 8)
    for ell in range(2):
        lam = s.get_smoother(0, ell + 1)
        expect = w[:, :, None] * T[5].reshape(2, 8, 8)[ell][None] * w[:, None, :]
        assert rel(lam, expect) <= 1e-6
    # coarser levels keep the Frobenius fit
    s2 = cascade.Solver(p.levels)
    s2.setup(depth=2)
    np.testing.assert_array_equal(s.get_smoother(1, 1), s2.get_smoother(1, 1))


def test_setup_learned_validation(gpu_lib, L):
    from paper_2606_12577_amd import cascade
    p = fe.multiphase3d(8, seed_extra=5, config_id=51)
    s = cascade.Solver(p.levels)
    X = L.fe_block_features(p.meta["log10mu"])
    with pytest.raises(cascade.CascadeError):
        s.setup_learned(L.Mlp(1464, 16, 100), X, depth=2)      # outputs != depth * 64
    with pytest.raises(cascade.CascadeError):
        s.setup_learned(L.Mlp(1464, 16, 128), X, depth=3)
    net = L.Mlp(5, 4, 2)
    with pytest.raises(cascade.CascadeError):
        net.set_scaling(np.zeros(2), np.array([1.0, 0.0]))      # std must be positive
    with pytest.raises(cascade.CascadeError):
        net.set_params(np.full(net.n_params, np.nan))
