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

    def block_lattice(self) -> np.ndarray:
        """Integer lattice point of every block, (n_blocks, d): the grid
        coordinates of its cells divided by the block edge (cells must be set
        and every block must be a cube of cells)."""
        if self.cells is None:
            raise ValueError("level has no cell numbering")
        d = self.cells.ndim
        edge = int(round(self.block_size ** (1.0 / d)))
        if edge ** d != self.block_size:
            raise ValueError("blocks are not cubes of cells")
        coords = np.indices(self.cells.shape).reshape(d, -1).T
        blk = self.cells.ravel() // self.block_size
        out = np.empty((self.n_blocks, d), dtype=np.int32)
        out[blk] = coords // edge
        return out


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
