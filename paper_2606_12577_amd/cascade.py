"""Python binding of libcascade.so (the C ABI declared in include/cascade.h).

Argument marshalling only: every step of the setup and of the solve runs in the
library's HIP kernels.  torch supplies device memory and the stream.  The
binding refuses to work without the built library.
"""
import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcascade.so")

ADDITIVE, MULTIPLICATIVE = 0, 1
FF, RF = 0, 1
FP64, FP32, BF16 = 0, 1, 2
_MODES = {"additive": ADDITIVE, "multiplicative": MULTIPLICATIVE}
_ORDERS = {"FF": FF, "RF": RF}
_PRECS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
_SOURCES = {"frobenius": 0, "jacobi": 1}   # cs_source

STATUS = {0: "CS_OK", -1: "CS_EINVAL", -2: "CS_ENOMEM", -3: "CS_EDEVICE", -4: "CS_ESINGULAR",
          -5: "CS_ECOLOR", -6: "CS_ENOCONV", -7: "CS_ESTATE", -8: "CS_ENAN", -9: "CS_EVERSION",
          -10: "CS_EIO"}


class CascadeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_p = ctypes.POINTER


class cs_level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("block_size", ctypes.c_int32),
                ("a_row_ptr", _p(ctypes.c_int64)), ("a_col", _p(ctypes.c_int32)), ("a_val", _p(ctypes.c_double)),
                ("n_coarse", ctypes.c_int64),
                ("p_row_ptr", _p(ctypes.c_int64)), ("p_col", _p(ctypes.c_int32)), ("p_val", _p(ctypes.c_double)),
                ("r_scale", ctypes.c_double), ("colour", _p(ctypes.c_int32)),
                ("n_direct_seg", ctypes.c_int32), ("direct_seg_ptr", _p(ctypes.c_int64))]


class cs_options(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("mode", ctypes.c_int32), ("order", ctypes.c_int32),
                ("n_pre", ctypes.c_int32), ("n_post", ctypes.c_int32), ("trunc_alpha", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("ridge", ctypes.c_double),
                ("source", ctypes.c_int32), ("jacobi_omega", ctypes.c_double)]


class cs_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_res", ctypes.c_double), ("rho", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("singular_blocks", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rho_geo", ctypes.c_double), ("eta", ctypes.c_double)]


# every symbol declared in include/cascade.h, with its ctypes signature
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
SIGNATURES = {
    "cs_abi_version": (_I32, []),
    "cs_status_string": (ctypes.c_char_p, [_I32]),
    "cs_create": (_I32, [_p(_VP), _I32, _VP]),
    "cs_destroy": (None, [_VP]),
    "cs_last_error": (ctypes.c_char_p, [_VP]),
    "cs_set_hierarchy": (_I32, [_VP, _I32, _p(cs_level)]),
    "cs_setup": (_I32, [_VP, _p(cs_options)]),
    "cs_set_precision": (_I32, [_VP, _I32]),
    "cs_get_smoother": (_I32, [_VP, _I32, _I32, _p(_D)]),
    "cs_set_smoother": (_I32, [_VP, _I32, _I32, _p(_D)]),
    "cs_get_pattern_size": (_I32, [_VP, _I32, _I32, _p(_I64)]),
    "cs_get_pattern": (_I32, [_VP, _I32, _I32, _p(_I64), _p(_I32)]),
    "cs_get_colours": (_I32, [_VP, _I32, _p(_I32)]),
    "cs_smooth": (_I32, [_VP, _I32, _I32, _VP, _VP, _I32]),
    "cs_vcycle": (_I32, [_VP, _VP, _VP, _I32]),
    "cs_vcycle_noalloc": (_I32, [_VP, _VP, _VP, _I32]),
    "cs_set_graphs": (_I32, [_VP, _I32]),
    "cs_get_graphs": (_I32, [_VP, _p(_I32), _p(_D), _p(_D)]),
    "cs_set_tail": (_I32, [_VP, _I64]),
    "cs_get_tail": (_I32, [_VP, _p(_I64), _p(_I32), _I32, _p(_I64), _p(_D), _p(_I32)]),
    "cs_stream_bandwidth": (_I32, [_VP, _I32, _I32, _I64, _I32, _p(_D), _p(_D)]),
    "cs_solve": (_I32, [_VP, _VP, _VP, _I32, _D, _I32, _p(cs_info), _p(_D)]),
    "cs_solve_cg": (_I32, [_VP, _VP, _VP, _I32, _D, _I32, _p(cs_info), _p(_D)]),
    "cs_solve_gmres": (_I32, [_VP, _VP, _VP, _I32, _D, _I32, _I32, _I32, _p(cs_info), _p(_D)]),
    "cs_autotune": (_I32, [_VP, _I32, _p(_I32), _p(_I64), _p(_D)]),
    "cs_setup_sketched": (_I32, [_VP, _p(cs_options), _I32, _VP]),
    "cs_set_saddle_point": (_I32, [_VP, _I32, _p(_I32), _I32]),
    "cs_set_lattice": (_I32, [_VP, _I32, _I32, _p(_I32)]),
    "cs_get_lattice_stats": (_I32, [_VP, _I32, _p(_I64), _p(_I32)]),
    "cs_set_overlapping_blocks": (_I32, [_VP, _I32, _I64, _I32, _p(_I32)]),
    "cs_trace": (_I32, [_VP, _I32, _I32]),
    "cs_trace_read": (_I32, [_VP, _I32, _p(_D), _p(_I64), _p(_D)]),
    "cs_set_systems": (_I32, [_VP, _I32, _p(_I64)]),
    "cs_get_system_stats": (_I32, [_VP, _p(_I32), _p(_D)]),
    # learned setup (cascade_learned.h)
    "cs_mlp_create": (_I32, [_p(_VP), _I32, _VP, _I32, _I32, _I32]),
    "cs_mlp_destroy": (None, [_VP]),
    "cs_mlp_last_error": (ctypes.c_char_p, [_VP]),
    "cs_mlp_param_count": (_I32, [_VP, _p(_I64)]),
    "cs_mlp_set_params": (_I32, [_VP, _p(ctypes.c_float)]),
    "cs_mlp_get_params": (_I32, [_VP, _p(ctypes.c_float)]),
    "cs_mlp_set_scaling": (_I32, [_VP, _p(ctypes.c_float), _p(ctypes.c_float)]),
    "cs_mlp_get_scaling": (_I32, [_VP, _p(ctypes.c_float), _p(ctypes.c_float)]),
    "cs_mlp_fit_scaling": (_I32, [_VP, _VP, _VP, _I64]),
    "cs_mlp_gradient": (_I32, [_VP, _VP, _VP, _VP, _I64, _p(ctypes.c_float), _p(_D)]),
    "cs_mlp_loss": (_I32, [_VP, _VP, _VP, _VP, _I64, _p(_D)]),
    "cs_mlp_train": (_I32, [_VP, _VP, _VP, _VP, _I64, _I32, _I32, _D, _D, _p(_D)]),
    "cs_mlp_forward": (_I32, [_VP, _VP, _I64, _VP]),
    "cs_fe_block_features": (_I32, [_VP, _VP, _I32, _VP]),
    "cs_get_prescaled_blocks": (_I32, [_VP, _I32, _VP]),
    "cs_setup_learned": (_I32, [_VP, _p(cs_options), _VP, _VP]),
    "cs_save_setup": (_I32, [_VP, ctypes.c_char_p]),
    "cs_load_setup": (_I32, [_VP, ctypes.c_char_p]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcascade.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_2606_12577_amd.build`")
    # load torch's HIP runtime first, so that the library binds to the same one
    # (a second runtime loaded ahead of torch cannot see the device afterwards)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, ctype):
    return a.ctypes.data_as(_p(ctype))


def _tensor_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One hierarchy on one GPU.

    levels: sequence of objects with attributes A (scipy CSR, float64),
    block_size, P (CSR interpolation from the next coarser level or None),
    r_scale, colour (int array per block or None) and optionally direct_seg
    (row offsets of trailing segments solved directly); level 0 is the finest.
    """

    def __init__(self, levels: Sequence, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the cascade solver needs a HIP GPU")
        self._torch = torch
        self.device = torch.device("cuda", device)
        self._lib = load_library()
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self._lib.cs_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream.cuda_stream))
        if st != 0:
            raise CascadeError(st, self._lib.cs_last_error(None).decode())
        self._h = h
        self.n_levels = 0
        self.sizes = []
        self.set_hierarchy(levels)

    # -- plumbing --------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise CascadeError(st, self._lib.cs_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hierarchy and setup ----------------------------------------------
    def set_hierarchy(self, levels: Sequence):
        keep = []
        arr = (cs_level * len(levels))()
        for i, lv in enumerate(levels):
            A = lv.A.tocsr()
            A.sort_indices()
            ap = _arr(A.indptr, np.int64)
            ac = _arr(A.indices, np.int32)
            av = _arr(A.data, np.float64)
            keep += [ap, ac, av]
            s = arr[i]
            s.n = A.shape[0]
            s.block_size = int(lv.block_size)
            s.a_row_ptr, s.a_col, s.a_val = _ptr(ap, ctypes.c_int64), _ptr(ac, ctypes.c_int32), _ptr(av, ctypes.c_double)
            if getattr(lv, "P", None) is not None and i + 1 < len(levels):
                P = lv.P.tocsr()
                pp, pc, pv = _arr(P.indptr, np.int64), _arr(P.indices, np.int32), _arr(P.data, np.float64)
                keep += [pp, pc, pv]
                s.n_coarse = P.shape[1]
                s.p_row_ptr, s.p_col, s.p_val = (_ptr(pp, ctypes.c_int64), _ptr(pc, ctypes.c_int32),
                                                 _ptr(pv, ctypes.c_double))
                s.r_scale = float(lv.r_scale)
            col = getattr(lv, "colour", None)
            if col is not None:
                c = _arr(col, np.int32)
                keep.append(c)
                s.colour = _ptr(c, ctypes.c_int32)
            seg = getattr(lv, "direct_seg", None)
            if seg is not None and len(seg) > 1:
                sp = _arr(seg, np.int64)
                keep.append(sp)
                s.n_direct_seg = len(sp) - 1
                s.direct_seg_ptr = _ptr(sp, ctypes.c_int64)
        self._check(self._lib.cs_set_hierarchy(self._h, len(levels), arr))
        self.n_levels = len(levels)
        self.n_systems = 1
        self.sizes = [(int(lv.A.shape[0]), int(lv.block_size)) for lv in levels]
        self.ovl = {}
        # saddle-point levels (a `kind` array: 0 velocity, 1 pressure, 2 inert)
        for i, lv in enumerate(levels):
            kind = getattr(lv, "kind", None)
            if kind is not None:
                self.set_saddle_point(i, kind, l1=True)

    def set_overlapping_blocks(self, level: int, nodes=None):
        """Overlapping blocks for a level (Sec. 3.6.2): nodes[i][s] is the
        unknown of slot s of block i (-1 unused); None restores the partition.
        Such levels are fitted by setup_sketched (additive, FF)."""
        if nodes is None:
            self._check(self._lib.cs_set_overlapping_blocks(self._h, level, 0, 0, None))
            self.ovl.pop(level, None)
            return
        nd = _arr(nodes, np.int32)
        self._check(self._lib.cs_set_overlapping_blocks(self._h, level, nd.shape[0], nd.shape[1], _ptr(nd, _I32)))
        self.ovl[level] = (int(nd.shape[0]), int(nd.shape[1]))

    def _lam_shape(self, level: int):
        if level in self.ovl:
            nblk, m = self.ovl[level]
            return (nblk, m, m)
        n, nb = self.sizes[level]
        return (n // nb, nb, nb)

    def set_saddle_point(self, level: int, kind=None, l1: bool = True):
        """Stokes prescaling for a level (Sec. 2.3.2): kind per unknown, 0
        velocity, 1 pressure, 2 inert; constraint rows normalised by the 1-norm
        (l1, the staggered-grid choice) or the max-norm.  None: elliptic."""
        if kind is None:
            self._check(self._lib.cs_set_saddle_point(self._h, level, None, 0))
            return
        k = _arr(kind, np.int32)
        self._check(self._lib.cs_set_saddle_point(self._h, level, _ptr(k, _I32), int(bool(l1))))

    def set_lattice(self, level: int, coords=None):
        """Stencil-repetition cache for a level (Sec. 4): coords (n_blocks x
        dim integer lattice points, distinct) lets the exact additive setup fit
        one block per class of translation-equivalent neighbourhoods and copy
        the rest.  None removes it."""
        if coords is None:
            self._check(self._lib.cs_set_lattice(self._h, level, 0, None))
            return
        c = _arr(np.asarray(coords).reshape(self.sizes[level][0] // self.sizes[level][1], -1), np.int32)
        self._check(self._lib.cs_set_lattice(self._h, level, c.shape[1], _ptr(c, _I32)))

    def lattice_stats(self, level: int, classes: bool = False):
        """Blocks fitted per cascade step by the last exact setup of a level
        and, with classes=True, the class representatives (depth x n_blocks,
        radius l - 1 for step l)."""
        depth = getattr(self, "depth", 1)   # before any setup the library reports the state error
        fitted = np.zeros(depth, dtype=np.int64)
        rep = np.zeros((depth, self.sizes[level][0] // self.sizes[level][1]), dtype=np.int32) if classes else None
        self._check(self._lib.cs_get_lattice_stats(self._h, level, _ptr(fitted, _I64),
                                                   _ptr(rep, _I32) if classes else None))
        return (fitted, rep) if classes else fitted

    def setup(self, depth: int = 3, mode: str = "additive", order: str = "RF", n_pre: int = 1,
              n_post: int = 1, alpha: int = 0, precision: str = "fp64", ridge: float = 0.0,
              source: str = "frobenius", omega: float = 1.0):
        """source "frobenius": the cascade fit; "jacobi": every cascade level
        omega * blockdiag(A)^-1 (the reference smoother)."""
        o = cs_options(depth, _MODES[mode], _ORDERS[order], n_pre, n_post, alpha, _PRECS[precision], ridge,
                       _SOURCES[source], omega)
        self.depth = depth
        self._check(self._lib.cs_setup(self._h, ctypes.byref(o)))

    def setup_sketched(self, width: int = 32, seed: int = 0, sketch=None, depth: int = 3, mode: str = "additive",
                       order: str = "RF", n_pre: int = 1, n_post: int = 1, precision: str = "fp64"):
        """Sketched cascade construction: every level is fitted against `width`
        random error modes.  `sketch` (device or host, (sum of the smoothed
        levels' sizes) x width) gives them; otherwise Rademacher +-1 modes are
        drawn on the device from `seed`.  Returns the sketch used."""
        total = sum(n for n, _ in self.sizes[:-1])
        if sketch is None:
            g = self._torch.Generator(device=self.device)
            g.manual_seed(int(seed))
            sketch = self._torch.randint(0, 2, (total, width), generator=g, device=self.device)
            sketch = (2.0 * sketch - 1.0).to(self._torch.float64)
        S = self._torch.as_tensor(sketch, dtype=self._torch.float64, device=self.device).contiguous()
        if tuple(S.shape) != (total, width):
            raise ValueError(f"sketch must be {total} x {width}")
        o = cs_options(depth, _MODES[mode], _ORDERS[order], n_pre, n_post, 0, _PRECS[precision])
        self.depth = depth
        self._check(self._lib.cs_setup_sketched(self._h, ctypes.byref(o), width, _tensor_ptr(S)))
        return S

    def set_precision(self, precision: str):
        self._check(self._lib.cs_set_precision(self._h, _PRECS[precision]))

    def get_smoother(self, level: int, ell: int) -> np.ndarray:
        out = np.empty(self._lam_shape(level), dtype=np.float64)
        self._check(self._lib.cs_get_smoother(self._h, level, ell, _ptr(out, ctypes.c_double)))
        return out

    def set_smoother(self, level: int, ell: int, blocks: np.ndarray):
        b = _arr(blocks, np.float64)
        if b.size != int(np.prod(self._lam_shape(level))):
            raise ValueError("smoother has the wrong size")
        self._check(self._lib.cs_set_smoother(self._h, level, ell, _ptr(b, ctypes.c_double)))

    def get_pattern(self, level: int, step: int):
        nnz = ctypes.c_int64()
        self._check(self._lib.cs_get_pattern_size(self._h, level, step, ctypes.byref(nnz)))
        n, nb = self.sizes[level]
        ptr = np.empty(n // nb + 1, dtype=np.int64)
        col = np.empty(max(nnz.value, 1), dtype=np.int32)
        self._check(self._lib.cs_get_pattern(self._h, level, step, _ptr(ptr, ctypes.c_int64),
                                             _ptr(col, ctypes.c_int32)))
        return ptr, col[:nnz.value]

    def get_colours(self, level: int) -> np.ndarray:
        n, nb = self.sizes[level]
        out = np.empty(n // nb, dtype=np.int32)
        self._check(self._lib.cs_get_colours(self._h, level, _ptr(out, ctypes.c_int32)))
        return out

    # -- application ----------------------------------------------------------
    def _vec(self, b):
        t = self._torch
        if not isinstance(b, t.Tensor):
            b = t.as_tensor(np.asarray(b, dtype=np.float64))
        b = b.to(device=self.device, dtype=t.float64)
        if b.dim() == 1:
            b = b[:, None]
        b = b.contiguous()
        if b.data_ptr() % 64:
            b = b.clone()       # the kernels load whole rows as 16-byte vectors
        return b

    def smooth(self, level: int, b, x, reverse: bool = False):
        b = self._vec(b)
        x = self._vec(x).clone()
        self._check(self._lib.cs_smooth(self._h, level, int(reverse), _tensor_ptr(b), _tensor_ptr(x), b.shape[1]))
        return x

    def vcycle(self, b):
        b = self._vec(b)
        x = self._torch.empty_like(b)
        self._check(self._lib.cs_vcycle(self._h, _tensor_ptr(b), _tensor_ptr(x), b.shape[1]))
        return x

    def vcycle_noalloc(self, b, x):
        """cs_vcycle_noalloc: x = V b into the caller's tensor x, the workspace
        in the library's static device array; waits for the result."""
        b = self._vec(b)
        if x.shape != b.shape or x.dtype != b.dtype or not x.is_contiguous() or x.device != b.device:
            raise ValueError("x must be a contiguous tensor shaped like b on the same device")
        self._check(self._lib.cs_vcycle_noalloc(self._h, _tensor_ptr(b), _tensor_ptr(x), b.shape[1]))
        self._torch.cuda.synchronize(b.device)
        return x

    def solve(self, b, rtol: float = 1e-10, maxit: int = 100, x=None, raise_on_noconv: bool = True,
              method: str = "ir", restart: int = 30):
        """method "ir": FP64 iterative refinement around the V-cycle (stationary);
        "cg": flexible conjugate gradients preconditioned by the V-cycle;
        "gmres": restarted GMRES with the V-cycle as left preconditioner (the
        history is ||V(b - Ax)|| / ||Vb||); "fgmres": flexible (right) GMRES."""
        b = self._vec(b)
        if x is None:
            x = self._torch.empty_like(b)
        info = cs_info()
        hist = np.full(maxit + 1, np.nan)
        args = (self._h, _tensor_ptr(b), _tensor_ptr(x), b.shape[1], rtol, maxit)
        tail = (ctypes.byref(info), _ptr(hist, ctypes.c_double))
        if method in ("gmres", "fgmres"):
            st = self._lib.cs_solve_gmres(*args, restart, int(method == "fgmres"), *tail)
        else:
            fn = {"ir": self._lib.cs_solve, "cg": self._lib.cs_solve_cg}[method]
            st = fn(*args, *tail)
        if st != 0 and not (st == -6 and not raise_on_noconv):
            self._check(st)
        k = info.iterations
        return x, dict(iterations=k, rel_res=info.rel_res, rho=info.rho, rho_geo=info.rho_geo, eta=info.eta,
                       setup_ms=info.setup_ms,
                       solve_ms=info.solve_ms, singular_blocks=info.singular_blocks,
                       precision={v: k for k, v in _PRECS.items()}.get(info.precision),
                       history=hist[:k + 1].copy(), status=st)

    def get_prescaled_blocks(self, level: int = 0):
        """Lambda~ of a level as a device tensor [n_blocks, depth, nb, nb] (FP32)."""
        n, nb = self.sizes[level]
        out = self._torch.empty((n // nb, self.depth, nb, nb), dtype=self._torch.float32, device=self.device)
        self._check(self._lib.cs_get_prescaled_blocks(self._h, level, _tensor_ptr(out)))
        return out

    def setup_learned(self, net, features, depth: int = 2, order: str = "RF", n_pre: int = 1, n_post: int = 1,
                      precision: str = "fp64"):
        """Finest-level cascade from the network's prediction for `features`
        (device FP32 [n_blocks, n_in]); Frobenius fit on coarser levels."""
        X = features.contiguous()
        o = cs_options(depth, _MODES["additive"], _ORDERS[order], n_pre, n_post, 0, _PRECS[precision])
        self.depth = depth
        self._check(self._lib.cs_setup_learned(self._h, ctypes.byref(o), net._h, _tensor_ptr(X)))

    def set_systems(self, row_ptr=None):
        """Declare the finest level a batch of independent systems with row
        ranges [row_ptr[s], row_ptr[s+1]); None restores one system."""
        if row_ptr is None:
            self._check(self._lib.cs_set_systems(self._h, 1, None))
            self.n_systems = 1
            return
        rp = _arr(row_ptr, np.int64)
        self._check(self._lib.cs_set_systems(self._h, len(rp) - 1, _ptr(rp, ctypes.c_int64)))
        self.n_systems = len(rp) - 1

    def system_stats(self):
        """Per system of the last solve: V-cycles to convergence and final
        max relative residual."""
        ns = getattr(self, "n_systems", 1)
        it = np.empty(ns, dtype=np.int32)
        rel = np.empty(ns, dtype=np.float64)
        self._check(self._lib.cs_get_system_stats(self._h, _ptr(it, ctypes.c_int32), _ptr(rel, ctypes.c_double)))
        return it, rel

    TRACE_CLASSES = ("sweep", "sweep_zero", "residual", "prolong", "bottom", "refine", "sweep_prolong",
                     "sweep_small", "tail")

    def autotune(self, nrhs: int):
        """Time the candidate sweep schedules of every level (current precision,
        nrhs right-hand sides) and keep the fastest; returns per level
        (rows per workgroup, workgroup cap, best ms per cascade application)."""
        L = len(self.sizes)
        wgs, grid, ms = np.zeros(L, np.int32), np.zeros(L, np.int64), np.zeros(L)
        self._check(self._lib.cs_autotune(self._h, nrhs, _ptr(wgs, _I32), _ptr(grid, _I64), _ptr(ms, _D)))
        return [(int(w), int(g), float(t)) for w, g, t in zip(wgs, grid, ms)]

    def set_graphs(self, on: bool):
        """Replay the outer iterations of refinement / CG solves from a graph."""
        self._check(self._lib.cs_set_graphs(self._h, int(bool(on))))

    def graphs(self):
        """(replay on?, V-cycle ms eager, V-cycle ms replayed) - the times of the last autotune."""
        on, e, g = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.cs_get_graphs(self._h, ctypes.byref(on), ctypes.byref(e), ctypes.byref(g)))
        return bool(on.value), e.value, g.value

    def set_tail(self, max_rows: int):
        """Run the V-cycle on the coarse levels of at most max_rows rows as one
        single-workgroup launch (0: per-level launches)."""
        self._check(self._lib.cs_set_tail(self._h, int(max_rows)))

    def tail(self):
        """(max_rows, first level the tail covers or -1)."""
        m, f = ctypes.c_int64(), ctypes.c_int32()
        self._check(self._lib.cs_get_tail(self._h, ctypes.byref(m), ctypes.byref(f), 0, None, None, None))
        return m.value, f.value

    def tail_candidates(self):
        """The last autotune's tail candidates: [(max_rows, V-cycle ms)], 0 = off."""
        cap = len(self.sizes) + 1
        m, f, n = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        rows, ms = np.zeros(cap, np.int64), np.zeros(cap)
        self._check(self._lib.cs_get_tail(self._h, ctypes.byref(m), ctypes.byref(f), cap, _ptr(rows, _I64),
                                          _ptr(ms, _D), ctypes.byref(n)))
        return [(int(r), float(t)) for r, t in zip(rows[:n.value], ms[:n.value])]

    def stream_bandwidth(self, n_read: int, n_write: int, nbytes: int, reps: int = 20):
        """Streaming reference: (GB/s, us per launch) of plain kernels that read
        n_read and write n_write arrays of nbytes each on this device."""
        g, u = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.cs_stream_bandwidth(self._h, n_read, n_write, int(nbytes), reps, ctypes.byref(g),
                                                  ctypes.byref(u)))
        return g.value, u.value

    def trace(self, classes=("sweep",), period: int = 1):
        """Start (clearing the counters) event timing of every period-th launch
        of the given kernel classes; an empty sequence stops it."""
        mask = 0
        for name in classes:
            mask |= 1 << self.TRACE_CLASSES.index(name)
        self._check(self._lib.cs_trace(self._h, mask, period))

    def trace_read(self):
        out = {}
        for k, name in enumerate(self.TRACE_CLASSES):
            ms, cnt, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
            self._check(self._lib.cs_trace_read(self._h, k, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by)))
            out[name] = dict(ms=ms.value, launches=cnt.value, bytes=by.value)
        return out

    def save(self, path: str):
        self._check(self._lib.cs_save_setup(self._h, path.encode()))

    def load(self, path: str):
        self._check(self._lib.cs_load_setup(self._h, path.encode()))
