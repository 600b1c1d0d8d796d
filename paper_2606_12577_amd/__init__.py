"""Cascading-smoother geometric multigrid on MI355X (gfx950).

The compute path is the HIP library libcascade.so (C ABI in include/cascade.h);
`paper_2606_12577_amd.cascade` is its Python binding.
"""
from .cascade import Solver, load_library, CascadeError  # noqa: F401
