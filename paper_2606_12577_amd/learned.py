"""Python binding of the learned setup (include/cascade_learned.h).

Argument marshalling around the C ABI plus the host-side policy that uses it:
building a training set from Frobenius setups, training, and the judge that
keeps the learned finest-level cascade only when its measured convergence
factor is within a slack of the Frobenius one (Sec. 3.1 measures rho the same
way).  All arithmetic runs in the library's kernels.
"""
import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import cascade as C

N_FEATURES = 1464


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Mlp:
    """n_in -> width -> width -> n_out network with SiLU, FP32, on one GPU."""

    def __init__(self, n_in: int = N_FEATURES, width: int = 128, n_out: int = 128, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the network needs a HIP GPU")
        self._torch = torch
        self.device = torch.device("cuda", device)
        self._lib = C.load_library()
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self._lib.cs_mlp_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream.cuda_stream),
                                     n_in, width, n_out)
        if st != 0:
            raise C.CascadeError(st, self._lib.cs_mlp_last_error(None).decode())
        self._h = h
        self.n_in, self.width, self.n_out = n_in, width, n_out
        n = ctypes.c_int64()
        self._check(self._lib.cs_mlp_param_count(self._h, ctypes.byref(n)))
        self.n_params = n.value

    def _check(self, st):
        if st != 0:
            raise C.CascadeError(st, self._lib.cs_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cs_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters ------------------------------------------------------------
    def init_params(self, seed: int):
        """Kaiming-uniform weights (bound sqrt(6 / fan_in)) and uniform biases
        (bound 1 / sqrt(fan_in)) from a seeded generator."""
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2606, 5, 3, int(seed)])))
        parts = []
        for fan_in, fan_out in ((self.n_in, self.width), (self.width, self.width), (self.width, self.n_out)):
            parts.append(rng.uniform(-1, 1, size=fan_out * fan_in) * np.sqrt(6.0 / fan_in))
            parts.append(rng.uniform(-1, 1, size=fan_out) / np.sqrt(fan_in))
        self.set_params(np.concatenate(parts))

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        self._check(self._lib.cs_mlp_set_params(self._h, _f32p(p)))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.cs_mlp_get_params(self._h, _f32p(out)))
        return out

    def set_scaling(self, mean, std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        self._check(self._lib.cs_mlp_set_scaling(self._h, _f32p(m), _f32p(s)))

    def get_scaling(self):
        m = np.empty(self.n_out, dtype=np.float32)
        s = np.empty(self.n_out, dtype=np.float32)
        self._check(self._lib.cs_mlp_get_scaling(self._h, _f32p(m), _f32p(s)))
        return m, s

    # -- device data -------------------------------------------------------------
    def _mat(self, a, cols):
        t = self._torch
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(np.asarray(a, dtype=np.float32))
        a = a.to(device=self.device, dtype=t.float32).contiguous()
        if a.dim() != 2 or a.shape[1] != cols:
            raise ValueError(f"expected a matrix with {cols} columns")
        return a

    def _rows(self, r):
        if r is None:
            return None
        t = self._torch
        if not isinstance(r, t.Tensor):
            r = t.as_tensor(np.asarray(r, dtype=np.int32))
        return r.to(device=self.device, dtype=t.int32).contiguous()

    def fit_scaling(self, T, rows=None):
        T = self._mat(T, self.n_out)
        r = self._rows(rows)
        n = T.shape[0] if r is None else r.numel()
        self._check(self._lib.cs_mlp_fit_scaling(self._h, _dev(T), _dev(r), n))

    def gradient(self, X, T, rows=None):
        X, T, r = self._mat(X, self.n_in), self._mat(T, self.n_out), self._rows(rows)
        n = X.shape[0] if r is None else r.numel()
        g = np.empty(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self._lib.cs_mlp_gradient(self._h, _dev(X), _dev(T), _dev(r), n, _f32p(g), ctypes.byref(loss)))
        return g, loss.value

    def loss(self, X, T, rows=None) -> float:
        X, T, r = self._mat(X, self.n_in), self._mat(T, self.n_out), self._rows(rows)
        n = X.shape[0] if r is None else r.numel()
        loss = ctypes.c_double()
        self._check(self._lib.cs_mlp_loss(self._h, _dev(X), _dev(T), _dev(r), n, ctypes.byref(loss)))
        return loss.value

    def train(self, X, T, order, batch: int = 1024, lr0: float = 1e-3, lr_min: float = 0.0) -> np.ndarray:
        """order: [epochs, n_train] row visits (the caller's shuffles)."""
        X, T = self._mat(X, self.n_in), self._mat(T, self.n_out)
        o = self._rows(np.asarray(order) if not isinstance(order, self._torch.Tensor) else order)
        epochs, n_train = o.shape
        hist = np.zeros(epochs)
        self._check(self._lib.cs_mlp_train(self._h, _dev(X), _dev(T), _dev(o), n_train, epochs, batch, lr0, lr_min,
                                           hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return hist

    def forward(self, X):
        X = self._mat(X, self.n_in)
        Y = self._torch.empty((X.shape[0], self.n_out), dtype=self._torch.float32, device=self.device)
        self._check(self._lib.cs_mlp_forward(self._h, _dev(X), X.shape[0], _dev(Y)))
        return Y


def fe_block_features(log10mu, device: int = 0):
    """Q1 block features [(n/2)^3, 1464] (device FP32) of a hex coefficient field."""
    import torch
    lib = C.load_library()
    dev = torch.device("cuda", device)
    lm = torch.as_tensor(np.ascontiguousarray(log10mu, dtype=np.float64)).to(dev)
    n = lm.shape[0]
    X = torch.empty(((n // 2) ** 3, N_FEATURES), dtype=torch.float32, device=dev)
    st = lib.cs_fe_block_features(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream), _dev(lm), n, _dev(X))
    if st != 0:
        raise C.CascadeError(st, "cs_fe_block_features failed")
    return X


@dataclass
class TrainReport:
    epoch_loss: np.ndarray
    val_loss: float
    val_loss_untrained: float
    n_train: int
    n_val: int


def build_training_set(problems: Sequence, depth: int = 2, order: str = "RF"):
    """Features and Frobenius targets (prescaled Lambda~ of the finest level)
    of every block of the given problems (objects with .levels and
    .meta['log10mu'])."""
    import torch
    X, T = [], []
    for p in problems:
        s = C.Solver(p.levels)
        s.setup(depth=depth, order=order)
        X.append(fe_block_features(p.meta["log10mu"]))
        T.append(s.get_prescaled_blocks(0).reshape(X[-1].shape[0], -1))
        s.close()
    return torch.cat(X), torch.cat(T)


def regular_blocks(T, factor: float = 4.0) -> np.ndarray:
    """Rows of T whose largest entry stays within `factor` times the median
    of that statistic.  The few blocks outside are those whose normal
    equations were (nearly) singular; their minimum-norm fits are isolated,
    large and not a function of the local features, so they are left out of
    training (the judge still measures the whole cascade)."""
    big = T.abs().amax(dim=1).cpu().numpy()
    return np.where(big <= factor * np.median(big))[0].astype(np.int32)


def train_network(X, T, n_samples: int, epochs: int = 40, batch: int = 1024, lr0: float = 1e-3,
                  val_fraction: float = 0.1, seed: int = 0, width: int = 128,
                  outlier_factor: float = 4.0) -> (Mlp, TrainReport):
    """Sample n_samples regular blocks, split train/validation, fit the output
    scaling on the training rows and train with Adam and a cosine rate."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2606, 5, 2, int(seed)])))
    ok = regular_blocks(T, outlier_factor) if outlier_factor else np.arange(X.shape[0], dtype=np.int32)
    pick = ok[rng.choice(len(ok), size=min(n_samples, len(ok)), replace=False)].astype(np.int32)
    n_val = max(1, int(round(val_fraction * len(pick))))
    val, tr = pick[:n_val], pick[n_val:]
    net = Mlp(X.shape[1], width, T.shape[1])
    net.init_params(seed)
    net.fit_scaling(T, tr)
    val_untrained = net.loss(X, T, val)
    order = np.stack([tr[rng.permutation(len(tr))] for _ in range(epochs)])
    hist = net.train(X, T, order, batch=batch, lr0=lr0, lr_min=0.0)
    return net, TrainReport(hist, net.loss(X, T, val), val_untrained, len(tr), n_val)


@dataclass
class Verdict:
    use_learned: bool
    rho_learned: float
    rho_frobenius: float
    setup_ms_learned: float
    setup_ms_frobenius: float
    iterations_learned: int
    iterations_frobenius: int


def judge(solver, net, features, b, depth: int = 2, slack: float = 1.05, rtol: float = 1e-10, maxit: int = 200,
          order: str = "RF", precision: str = "fp64", method: str = "ir") -> Verdict:
    """Measure rho with the learned and with the Frobenius finest-level
    cascade and keep the learned one iff rho_learned <= slack * rho_frobenius.
    method selects the solve that measures rho ("ir": the stationary V-cycle
    iteration, "cg": the V-cycle as CG preconditioner).  The solver is left
    with the chosen setup."""
    solver.setup(depth=depth, order=order, precision=precision)
    _, fr = solver.solve(b, rtol=rtol, maxit=maxit, raise_on_noconv=False, method=method)
    solver.setup_learned(net, features, depth=depth, order=order, precision=precision)
    try:
        _, le = solver.solve(b, rtol=rtol, maxit=maxit, raise_on_noconv=False, method=method)
        rho_l = le["rho"] if np.isfinite(le["rho"]) else np.inf
    except C.CascadeError:          # a divergent learned cascade (non-finite residual)
        le = dict(setup_ms=float("nan"), iterations=-1)
        rho_l = np.inf
    ok = bool(rho_l <= slack * fr["rho"])
    if not ok:
        solver.setup(depth=depth, order=order, precision=precision)
    return Verdict(ok, float(rho_l), float(fr["rho"]), le["setup_ms"], fr["setup_ms"], le["iterations"],
                   fr["iterations"])
