"""2D Stokes on a MAC staggered grid (Sec. 3.6.1 setting), closed unit box.

Unknowns per cell (i, j) (cell index c = i + n j, block of 4, scalar 4c + s):
  s = 0  u at the cell's right face  (x = (i+1) h, y = (j+1/2) h)
  s = 1  v at the cell's top face    (x = (i+1/2) h, y = (j+1) h)
  s = 2  p at the cell centre
  s = 3  an inert slot (identity row, no coupling) that makes the block size 4
Faces on the walls (x = 1 for u, y = 1 for v) carry no unknown: their slots are
inert too, and so is p in cell (0, 0), pinned to 0 so that the enclosed flow
has a unique pressure.  Viscous operator: 5-point -Laplacian / h^2 (mu = 1)
with no-slip walls (ghost values mirrored); gradient (p_E - p_W) / h; the
constraint rows are the transpose (negative divergence), so A is symmetric
indefinite.  This is the cell-wise non-overlapping blocking of the paper
(central pressure with the right-facing velocities), padded to 4.

Hierarchy: Galerkin A_c = P^T A P with bilinear interpolation of each velocity
component on its staggered grid (no-slip ghosts at the walls) and piecewise
constant pressure; R = P^T.  Inert slots have zero rows/columns in P and unit
diagonals on every level.
"""
from typing import List

import numpy as np
import scipy.sparse as sp

from .problem import Level, Problem
from .rng import stream, RHS


def kinds(n: int) -> np.ndarray:
    """0 velocity, 1 pressure, 2 inert, per scalar unknown."""
    k = np.zeros((n * n, 4), dtype=np.int32)
    k[:, 2] = 1
    k[:, 3] = 2
    i = np.arange(n * n) % n
    j = np.arange(n * n) // n
    k[i == n - 1, 0] = 2
    k[j == n - 1, 1] = 2
    k[0, 2] = 2
    return k.ravel()


def operator(n: int) -> sp.csr_matrix:
    h = 1.0 / n
    N = 4 * n * n
    kind = kinds(n)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r), cols.append(c), vals.append(v)

    def U(i, j):   # u at face x = (i+1) h of cell (i, j); None on a wall
        return 4 * (i + n * j) + 0 if 0 <= i < n - 1 and 0 <= j < n else None

    def V(i, j):
        return 4 * (i + n * j) + 1 if 0 <= i < n and 0 <= j < n - 1 else None

    def Pr(i, j):
        return 4 * (i + n * j) + 2 if 0 <= i < n and 0 <= j < n and (i, j) != (0, 0) else None

    inv2 = 1.0 / (h * h)
    for j in range(n):
        for i in range(n):
            # u-momentum at face (i+1, j)
            r = U(i, j)
            if r is not None:
                diag = 4.0
                for (a, b) in ((i + 1, j), (i - 1, j)):        # east / west faces (walls: u = 0)
                    c = U(a, b) if a >= 0 else None
                    if c is not None:
                        add(r, c, -inv2)
                for b in (j + 1, j - 1):                        # north / south (walls: ghost -u)
                    if 0 <= b < n:
                        add(r, U(i, b), -inv2)
                    else:
                        diag += 1.0
                add(r, r, diag * inv2)
                for (pc, s) in ((Pr(i + 1, j), 1.0), (Pr(i, j), -1.0)):
                    if pc is not None:
                        add(r, pc, s / h)
            r = V(i, j)
            if r is not None:
                diag = 4.0
                for (a, b) in ((i, j + 1), (i, j - 1)):
                    c = V(a, b) if b >= 0 else None
                    if c is not None:
                        add(r, c, -inv2)
                for a in (i + 1, i - 1):
                    if 0 <= a < n:
                        add(r, V(a, j), -inv2)
                    else:
                        diag += 1.0
                add(r, r, diag * inv2)
                for (pc, s) in ((Pr(i, j + 1), 1.0), (Pr(i, j), -1.0)):
                    if pc is not None:
                        add(r, pc, s / h)
    # constraint rows: the transpose of the gradient entries (negative divergence)
    r0, c0, v0 = np.array(rows), np.array(cols), np.array(vals)
    g = kind[c0] == 1
    rows = np.concatenate([r0, c0[g], np.flatnonzero(kind == 2)])
    cols = np.concatenate([c0, r0[g], np.flatnonzero(kind == 2)])
    vals = np.concatenate([v0, v0[g], np.ones(int((kind == 2).sum()))])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    return A


def _interp_cc(nc: int) -> np.ndarray:
    """Cell-centred linear interpolation weights (fine cell -> coarse cells) along
    one axis with no-slip (odd) ghosts: dense (2 nc, nc)."""
    W = np.zeros((2 * nc, nc))
    for f in range(2 * nc):
        J = f // 2
        other = J - 1 if f % 2 == 0 else J + 1
        if 0 <= other < nc:
            W[f, J] += 0.75
            W[f, other] += 0.25
        else:
            W[f, J] += 0.5          # ghost = -u_J
    return W


def _interp_face(nc: int) -> np.ndarray:
    """Face interpolation along the staggered axis: fine interior faces 1..2nc-1
    from coarse interior faces 1..nc-1 (wall faces are zero): dense (2nc-1, nc-1),
    row f-1 for fine face f, column K-1 for coarse face K."""
    W = np.zeros((2 * nc - 1, nc - 1))
    for f in range(1, 2 * nc):
        if f % 2 == 0:
            W[f - 1, f // 2 - 1] = 1.0
        else:
            for K in ((f - 1) // 2, (f + 1) // 2):
                if 1 <= K <= nc - 1:
                    W[f - 1, K - 1] += 0.5
    return W


def prolongation(n: int) -> sp.csr_matrix:
    nc = n // 2
    Wc = _interp_cc(nc)
    Wf = _interp_face(nc)
    kf, kc = kinds(n), kinds(nc)
    rows, cols, vals = [], [], []
    for j in range(n):
        for i in range(n):
            base = 4 * (i + n * j)
            # u at face (i+1, j): face index i+1 along x, cell j along y
            if kf[base] == 0:
                for K in range(1, nc):
                    wx = Wf[i, K - 1]
                    if wx == 0.0:
                        continue
                    for J in range(nc):
                        wy = Wc[j, J]
                        if wy != 0.0:
                            c = 4 * ((K - 1) + nc * J)
                            rows.append(base), cols.append(c), vals.append(wx * wy)
            if kf[base + 1] == 0:
                for K in range(1, nc):
                    wy = Wf[j, K - 1]
                    if wy == 0.0:
                        continue
                    for I in range(nc):
                        wx = Wc[i, I]
                        if wx != 0.0:
                            c = 4 * (I + nc * (K - 1)) + 1
                            rows.append(base + 1), cols.append(c), vals.append(wx * wy)
            if kf[base + 2] == 1:
                c = 4 * ((i // 2) + nc * (j // 2)) + 2
                if kc[c] == 1:
                    rows.append(base + 2), cols.append(c), vals.append(1.0)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(4 * n * n, 4 * nc * nc))
    P.sum_duplicates()
    P.sort_indices()
    return P


def hierarchy(n: int, n_stop: int = 4) -> List[Level]:
    A = operator(n)
    levels = []
    m = n
    while True:
        lv = Level(A=A, block_size=4)
        lv.kind = kinds(m)
        if m <= n_stop or m % 2:
            levels.append(lv)
            break
        P = prolongation(m)
        lv.P, lv.r_scale = P, 1.0
        levels.append(lv)
        Ac = (P.T @ (A @ P)).tolil()
        for s in np.flatnonzero(kinds(m // 2) == 2):
            Ac[s, s] = 1.0
        A = Ac.tocsr()
        A.eliminate_zeros()
        A.sum_duplicates()
        A.sort_indices()
        m //= 2
    return levels


def vanka_nodes(n: int) -> np.ndarray:
    """Overlapping cell patches (the Vanka layout): every cell's pressure with
    its four face velocities, [u_left, u_right, v_bottom, v_top, p] (-1 where a
    face is a wall or the pressure is pinned), then one single-slot block for
    every inert unknown so that every unknown lies in some block."""
    kind = kinds(n)
    blocks = []
    for j in range(n):
        for i in range(n):
            c = i + n * j
            uL = 4 * (c - 1) if i > 0 else -1
            uR = 4 * c if kind[4 * c] == 0 else -1
            vB = 4 * (c - n) + 1 if j > 0 else -1
            vT = 4 * c + 1 if kind[4 * c + 1] == 0 else -1
            p = 4 * c + 2 if kind[4 * c + 2] == 1 else -1
            blocks.append([uL, uR, vB, vT, p])
    for s in np.flatnonzero(kind == 2):
        blocks.append([int(s), -1, -1, -1, -1])
    return np.array(blocks, dtype=np.int32)


def mac2d(n: int = 64, nrhs: int = 1, config_id: int = 6) -> Problem:
    """Enclosed 2D Stokes flow on n x n cells; RHS U[-1,1] on the momentum and
    constraint rows, zero on inert slots."""
    levels = hierarchy(n)
    b = stream(config_id, RHS).uniform(-1.0, 1.0, size=(levels[0].n, nrhs))
    b[kinds(n) == 2] = 0.0
    return Problem(f"mac2d_{n}", levels, b, meta=dict(d=2, n=n, bs=4))
