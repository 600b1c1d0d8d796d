"""Containers for a multigrid hierarchy handed to the solver."""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class Level:
    """One level of the geometric hierarchy; level 0 is the finest.

    A          scalar CSR (float64), n x n, with unknowns ordered so that block i
               owns the contiguous scalar range [i*block_size, (i+1)*block_size)
    block_size uniform block size n_b (1 = point blocks)
    P          interpolation from the next coarser level (CSR, n x n_coarse);
               None on the coarsest level
    r_scale    restriction is r_scale * P^T
    colour     optional int32 colour per block (multiplicative smoothers)
    cells      optional array giving the unknown number of every grid cell
    """
    A: sp.csr_matrix
    block_size: int = 1
    P: Optional[sp.csr_matrix] = None
    r_scale: float = 1.0
    colour: Optional[np.ndarray] = None
    cells: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def n_blocks(self) -> int:
        return self.A.shape[0] // self.block_size


@dataclass
class Problem:
    name: str
    levels: List[Level]
    rhs: np.ndarray                     # (n_fine, nrhs), RHS index fastest
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.levels[0].n

    @property
    def nrhs(self) -> int:
        return self.rhs.shape[1]
