"""FP64 CPU oracle of the learned setup: block features, the multilayer
perceptron, its gradient and the Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper has no learned
component; this part follows the extension it motivates: the Frobenius setup
(Sec. 2.1, Alg. 2) is costly, so a network is trained to map the local
coefficient field around a block to that block's prescaled cascade blocks
Lambda~_1..Lambda~_nu, which are then unscaled as in Sec. 2.3.

Parity unpinned by the paper: no value here appears in it.  The pins are
mathematical: central differences of the loss for the gradient, the closed
form of Adam's first step, and closed-form feature values on constant and
corner configurations.

Definitions
-----------
Features of the 2x2x2 node block (I, J, K) of a Q1 mesh with n^3 hexes and
coefficient mu per hex (array [k, j, i]): the 9^3 hexes (2I-4+u, 2J-4+v,
2K-4+w), u, v, w = 0..8, index u + 9 v + 81 w (x fastest):
  * value[u,v,w] = (log10 mu(hex) - m) / 3 for hexes inside the mesh, 0
    outside, m the mean of log10 mu over the inside hexes of the patch;
  * mask[u,v,w] = 1 inside, 0 outside;
  * six face distances in blocks, min(d, 4) / 4, for the faces x=0, x=1, y=0,
    y=1, z=0, z=1 (d = I, nb-1-I, J, nb-1-J, K, nb-1-K with nb = n/2).
Vector: [value (729), mask (729), distances (6)] = 1464 entries.

Network: h_1 = silu(W_1 x + b_1), h_2 = silu(W_2 h_1 + b_2), y = W_3 h_2 + b_3
with silu(z) = z / (1 + exp(-z)); weights W_l are (out, in) row-major.
Loss on a batch of B rows with targets standardised per output
(t' = (t - mean) / std): L = sum (y - t')^2 / (B * n_out).
Prediction in target units: y * std + mean.
Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from typing import Dict, List, Sequence, Tuple

import numpy as np

PATCH = 9
N_FEATURES = 2 * PATCH ** 3 + 6


def block_features(log10mu: np.ndarray) -> np.ndarray:
    """Features of every 2x2x2 node block, blocks lexicographic (x fastest)."""
    n = log10mu.shape[0]
    nb = n // 2
    out = np.zeros((nb ** 3, N_FEATURES))
    off = np.arange(PATCH) - 4
    for K in range(nb):
        for J in range(nb):
            for I in range(nb):
                b = I + nb * (J + nb * K)
                hk, hj, hi = 2 * K + off, 2 * J + off, 2 * I + off
                ink = (hk >= 0) & (hk < n)
                inj = (hj >= 0) & (hj < n)
                ini = (hi >= 0) & (hi < n)
                mask = ink[:, None, None] & inj[None, :, None] & ini[None, None, :]   # [w, v, u]
                vals = np.zeros((PATCH,) * 3)
                sub = log10mu[np.ix_(hk[ink], hj[inj], hi[ini])]
                vals[np.ix_(ink, inj, ini)] = (sub - sub.mean()) / 3.0
                d = np.array([I, nb - 1 - I, J, nb - 1 - J, K, nb - 1 - K], dtype=float)
                out[b, :PATCH ** 3] = vals.ravel()            # [w, v, u] ravel = u + 9v + 81w
                out[b, PATCH ** 3:2 * PATCH ** 3] = mask.ravel()
                out[b, 2 * PATCH ** 3:] = np.minimum(d, 4.0) / 4.0
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def shapes(n_in: int, width: int, n_out: int) -> List[Tuple[int, ...]]:
    """Parameter tensors in storage order: W1, b1, W2, b2, W3, b3."""
    return [(width, n_in), (width,), (width, width), (width,), (n_out, width), (n_out,)]


def unpack(flat: np.ndarray, n_in: int, width: int, n_out: int) -> List[np.ndarray]:
    out, o = [], 0
    for s in shapes(n_in, width, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    if o != len(flat):
        raise ValueError("parameter vector has the wrong length")
    return out


def forward(params: Sequence[np.ndarray], X: np.ndarray) -> Dict[str, np.ndarray]:
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return dict(x=X, z1=z1, h1=h1, z2=z2, h2=h2, y=y)


def loss_and_grad(params, X, T, mean=None, std=None):
    """MSE on standardised targets and its gradient by reverse-mode chain rule."""
    W1, b1, W2, b2, W3, b3 = params
    mean = 0.0 if mean is None else mean
    std = 1.0 if std is None else std
    t = (T - mean) / std
    f = forward(params, X)
    B, n_out = f["y"].shape
    diff = f["y"] - t
    loss = float((diff ** 2).sum() / (B * n_out))
    dy = 2.0 * diff / (B * n_out)
    gW3 = dy.T @ f["h2"]
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * dsilu(f["z2"])
    gW2 = dz2.T @ f["h1"]
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * dsilu(f["z1"])
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def predict(params, X, mean=0.0, std=1.0):
    return forward(params, X)["y"] * std + mean


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def output_scaling(T: np.ndarray):
    """Per-output mean and standard deviation (population) of the targets; a
    zero deviation is replaced by 1."""
    mean = T.mean(axis=0)
    std = T.std(axis=0)
    return mean, np.where(std > 0, std, 1.0)


def cosine_lr(step: int, total: int, lr0: float, lr_min: float = 0.0) -> float:
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * step / max(total, 1)))
