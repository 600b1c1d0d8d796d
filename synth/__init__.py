"""Seeded synthetic inputs for cascading-smoother multigrid.

This package only builds *inputs*: discretised operators for every level of a
geometric hierarchy, interpolation matrices, block sizes, colourings and
right-hand sides.  It contains none of the smoother construction or V-cycle
arithmetic, so both the CPU oracle and the HIP library can consume it without
sharing any of the method's code.

Every generator returns a :class:`synth.problem.Problem`.
"""
from .problem import Level, Problem  # noqa: F401
from .rng import stream  # noqa: F401
