"""Many independent systems as one block-diagonal hierarchy.

Systems are reordered by their number of levels (deepest first, ties kept in
input order).  Level l of the batch stacks, in that order, level l of every
system that has one; the systems whose last level is l come last on it and
form its direct segments (solved exactly, one dense inverse each).  P of level
l is block diagonal over the systems that continue below l and has empty rows
for the direct segments.  This is pure data layout: the method itself runs on
the stacked hierarchy unchanged, system by system.
"""
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

from .problem import Level, Problem


@dataclass
class BatchLevel(Level):
    direct_seg: np.ndarray = None      # row offsets of the direct segments (None: none)


@dataclass
class Batch:
    levels: List[BatchLevel]
    order: np.ndarray                  # order[q] = input index of the q-th stacked system
    sys_ptr: np.ndarray                # finest-level row offsets of the stacked systems
    rhs: np.ndarray                    # stacked right-hand sides
    problems: List[Problem]

    def split(self, x) -> List[np.ndarray]:
        """Per-system slices of a finest-level vector, in input order."""
        x = np.asarray(x)
        out = [None] * len(self.problems)
        for q, s in enumerate(self.order):
            out[s] = x[self.sys_ptr[q]:self.sys_ptr[q + 1]]
        return out

    def stack(self, xs: Sequence[np.ndarray]) -> np.ndarray:
        """Stack per-system vectors (input order) into the batch layout."""
        return np.concatenate([np.asarray(xs[s]) for s in self.order], axis=0)


def concatenate(problems: Sequence[Problem]) -> Batch:
    nlev = np.array([len(p.levels) for p in problems])
    order = np.argsort(-nlev, kind="stable")
    levels = []
    for l in range(int(nlev.max())):
        present = [s for s in order if nlev[s] > l]
        active = [s for s in present if nlev[s] > l + 1]
        sizes = [problems[s].levels[l].n for s in present]
        bsz = {problems[s].levels[l].block_size for s in present}
        if len(bsz) != 1:
            raise ValueError(f"level {l}: systems disagree on the block size {sorted(bsz)}")
        A = sp.block_diag([problems[s].levels[l].A for s in present], format="csr")
        A.sort_indices()
        off = np.concatenate([[0], np.cumsum(sizes)])
        n_act = int(off[len(active)])
        seg = off[len(active):].astype(np.int64) if len(active) < len(present) else None
        P = None
        r_scale = 1.0
        if active:
            scales = {problems[s].levels[l].r_scale for s in active}
            if len(scales) != 1:
                raise ValueError(f"level {l}: systems disagree on the restriction scale")
            r_scale = scales.pop()
            blocks = [problems[s].levels[l].P for s in active]
            Pa = sp.block_diag(blocks, format="csr")
            P = sp.vstack([Pa, sp.csr_matrix((int(off[-1]) - n_act, Pa.shape[1]))], format="csr")
            P.sort_indices()
        cols = [problems[s].levels[l].colour for s in present]
        colour = np.concatenate(cols).astype(np.int32) if all(c is not None for c in cols) else None
        levels.append(BatchLevel(A=A, block_size=bsz.pop(), P=P, r_scale=r_scale, colour=colour,
                                 direct_seg=seg))
    sys_ptr = np.concatenate([[0], np.cumsum([problems[s].n for s in order])]).astype(np.int64)
    rhs = np.concatenate([problems[s].rhs for s in order], axis=0)
    return Batch(levels, order, sys_ptr, rhs, list(problems))
