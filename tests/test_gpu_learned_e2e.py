"""End-to-end learned setup on Q1 multiphase diffusion (3 phases, coefficients
1 / 1e3 / 1e6): Frobenius setups of training samples -> features -> GPU
training -> learned finest-level cascade judged by measured convergence
factors against the Frobenius setup of an unseen sample.

What is asserted (parity of the learned blocks themselves is not defined:
the network approximates the Frobenius fit):
  * training lowers the validation loss below the untrained network's and
    below 1 (the loss of predicting the mean, on standardised targets);
  * the trained network passes the judge (rho within 5% of Frobenius);
  * a freshly initialised network fails it, so the gain comes from training;
  * the learned setup is cheaper than the Frobenius setup it replaces;
  * after a failed judgement the solver holds the Frobenius setup again.
"""
import numpy as np
import pytest

from synth import fe

pytestmark = pytest.mark.gpu


def pipeline(n, epochs, method, samples=200000, batch=1024):
    from paper_2606_12577_amd import cascade, learned as L
    train = [fe.multiphase3d(n, seed_extra=s) for s in (1, 2)]
    test = fe.multiphase3d(n, seed_extra=0)
    X, T = L.build_training_set(train, depth=2)
    net, rep = L.train_network(X, T, n_samples=samples, epochs=epochs, batch=batch, lr0=1e-3)
    s = cascade.Solver(test.levels)
    Xt = L.fe_block_features(test.meta["log10mu"])
    v = L.judge(s, net, Xt, test.rhs, depth=2, method=method, maxit=300)
    fresh = L.Mlp(1464, 128, 128)
    fresh.init_params(seed=99)
    u = L.judge(s, fresh, Xt, test.rhs, depth=2, method=method, maxit=300)
    # after the failed judgement the Frobenius setup is back in place
    _, again = s.solve(test.rhs, rtol=1e-10, maxit=300, method=method, raise_on_noconv=False)
    return rep, v, u, again


@pytest.mark.parametrize("n,epochs,batch,method", [(24, 30, 128, "ir"), (96, 40, 1024, "cg")])
def test_learned_setup_end_to_end(gpu_lib, n, epochs, batch, method):
    rep, v, u, again = pipeline(n, epochs, method, batch=batch)
    print(f"n={n} {method}: val {rep.val_loss:.4f} (untrained {rep.val_loss_untrained:.4f}); "
          f"rho learned {v.rho_learned:.4f} vs Frobenius {v.rho_frobenius:.4f}; "
          f"setup {v.setup_ms_learned:.1f} ms vs {v.setup_ms_frobenius:.1f} ms; fresh rho {u.rho_learned}")
    assert rep.val_loss < 0.5 * rep.val_loss_untrained and rep.val_loss < 1.0
    assert v.use_learned and v.rho_learned <= 1.05 * v.rho_frobenius
    assert not u.use_learned
    assert v.setup_ms_learned < v.setup_ms_frobenius
    assert again["rho"] == pytest.approx(v.rho_frobenius, rel=1e-9)
