"""Cell-centred finite-volume (finite-difference) Poisson problems.

Discretisation (the cell-centred scheme of the supplementary Poisson-FD
section: piecewise-constant interpolation, restriction 2^-d P^T, rediscretised
coarse operators):

* n^d cells of width h = 1/n on the unit square/cube; one unknown per cell.
* -div(mu grad u) = f with homogeneous Dirichlet data imposed through a ghost
  cell: a boundary face has transmissibility 2 mu_cell / h^2, an interior face
  mu_face / h^2 with mu_face the harmonic mean of the two cell coefficients.
* A coarse face coefficient is the arithmetic mean of the 2^(d-1) fine face
  coefficients it covers (boundary faces included), and the coarse operator is
  rebuilt from those faces with h_c = 2h.
* Unknowns are ordered block by block: blocks of bs^d cells, block index
  lexicographic over the block grid (x fastest), local index lexicographic
  inside the block (x fastest).  bs = 1 gives plain lexicographic order.
"""
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

from .problem import Level, Problem
from .rng import GEOMETRY, stream, uniform_rhs


def morton_order(n: int, d: int, L: int) -> np.ndarray:
    """Recursive order for a grid that coarsens L more times: cells are
    numbered lexicographically by their ancestor on the grid n / 2^L and, inside
    it, in Z-order (Morton) of their offset.  The 2^d children of coarse cell I
    are then the fine unknowns 2^d I .. 2^d I + 2^d - 1 on every level, and 2^d
    siblings form a contiguous block."""
    if n % (1 << L):
        raise ValueError("grid size must be divisible by 2^L")
    c = n >> L
    coords = np.indices((n,) * d)
    lex = np.zeros((n,) * d, dtype=np.int64)
    m = 1
    for a in range(d):
        lex += (coords[a] >> L) * m
        m *= c
    mort = np.zeros((n,) * d, dtype=np.int64)
    for bit in range(L):
        for a in range(d):
            mort |= ((coords[a] >> bit) & 1).astype(np.int64) << (bit * d + a)
    return lex * (1 << (d * L)) + mort


def cell_order(n: int, d: int, bs: int) -> np.ndarray:
    """Unknown number of every cell, as an array indexed [i0, i1(, i2)]."""
    if n % bs:
        raise ValueError("block size must divide the grid size")
    nb = n // bs
    coords = np.indices((n,) * d)
    blk = np.zeros((n,) * d, dtype=np.int64)
    loc = np.zeros((n,) * d, dtype=np.int64)
    mb = ml = 1
    for a in range(d):
        blk += (coords[a] // bs) * mb
        loc += (coords[a] % bs) * ml
        mb *= nb
        ml *= bs
    return blk * bs ** d + loc


def block_coords(n: int, d: int, bs: int) -> np.ndarray:
    """(n_blocks, d) integer coordinates of every block in block-index order."""
    nb = n // bs
    c = np.indices((nb,) * d).reshape(d, -1).T      # row-major: last axis fastest
    return c[:, ::-1].copy() if d > 1 else c          # reorder so axis 0 is fastest


def parity_colour(n: int, d: int, bs: int, idx: Optional[np.ndarray] = None) -> np.ndarray:
    """Red-black colouring of the block grid: (sum of block coordinates) mod 2,
    listed in block-index order of the numbering idx (default: cell_order)."""
    if idx is None:
        idx = cell_order(n, d, bs)
    coords = np.indices((n,) * d)
    par = (sum(c // bs for c in coords) % 2).ravel()
    out = np.empty(n ** d // bs ** d, dtype=np.int32)
    out[idx.ravel() // bs ** d] = par
    return out


def face_coefficients(mu: np.ndarray) -> List[np.ndarray]:
    """Per-direction face coefficients; faces[a] has n+1 entries along axis a.

    Interior faces take the harmonic mean of their two cells, boundary faces
    the coefficient of the single adjacent cell."""
    n = mu.shape[0]
    faces = []
    for a in range(mu.ndim):
        lo = np.take(mu, range(0, n - 1), axis=a)
        hi = np.take(mu, range(1, n), axis=a)
        inner = 2.0 * lo * hi / (lo + hi)
        faces.append(np.concatenate(
            [np.take(mu, [0], axis=a), inner, np.take(mu, [n - 1], axis=a)], axis=a))
    return faces


def coarsen_faces(faces: Sequence[np.ndarray]) -> List[np.ndarray]:
    out = []
    for a, f in enumerate(faces):
        g = np.take(f, range(0, f.shape[a], 2), axis=a)
        for b in range(f.ndim):
            if b != a:
                g = 0.5 * (np.take(g, range(0, g.shape[b], 2), axis=b)
                           + np.take(g, range(1, g.shape[b], 2), axis=b))
        out.append(g)
    return out


def assemble(faces: Sequence[np.ndarray], idx: np.ndarray) -> sp.csr_matrix:
    """Operator of the faces, unknowns numbered by idx[cell]."""
    d = len(faces)
    n = faces[0].shape[0] - 1
    h = 1.0 / n
    diag = np.zeros((n,) * d)
    rows, cols, vals = [], [], []
    for a, f in enumerate(faces):
        t = f / h ** 2
        tb = t.copy()
        sl0 = [slice(None)] * d
        sl0[a] = 0
        tb[tuple(sl0)] *= 2.0
        sl0[a] = n
        tb[tuple(sl0)] *= 2.0
        diag += np.take(tb, range(0, n), axis=a) + np.take(tb, range(1, n + 1), axis=a)
        tin = np.take(t, range(1, n), axis=a)
        lo = np.take(idx, range(0, n - 1), axis=a)
        hi = np.take(idx, range(1, n), axis=a)
        for p, q in ((lo, hi), (hi, lo)):
            rows.append(p.ravel())
            cols.append(q.ravel())
            vals.append(-tin.ravel())
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    N = n ** d
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def piecewise_constant_P(n: int, d: int, bs_f: int, bs_c: int, idx_f: Optional[np.ndarray] = None,
                         idx_c: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """Injection of each coarse cell value into its 2^d fine sub-cells."""
    if idx_f is None:
        idx_f = cell_order(n, d, bs_f)
    if idx_c is None:
        idx_c = cell_order(n // 2, d, bs_c)
    coords = np.indices((n,) * d)
    parent = idx_c[tuple(c // 2 for c in coords)]
    N = n ** d
    P = sp.csr_matrix((np.ones(N), (idx_f.ravel(), parent.ravel())), shape=(N, (n // 2) ** d))
    P.sort_indices()
    return P


def fv_hierarchy(mu: np.ndarray, bs: int = 1, n_stop: int = 4, colour: bool = False,
                 order: str = "morton") -> List[Level]:
    """Levels n, n/2, ... while the size is even and above n_stop.

    order="morton" numbers cells recursively (see morton_order) when bs <= 2,
    so that blocks and coarse-cell children are contiguous on every level;
    order="lex" uses cell_order (lexicographic blocks)."""
    d = mu.ndim
    n = mu.shape[0]
    faces = face_coefficients(mu)
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] > n_stop:
        sizes.append(sizes[-1] // 2)
    L = len(sizes) - 1
    use_morton = order == "morton" and bs <= 2
    blocks = [bs if m % bs == 0 else 1 for m in sizes]
    if use_morton:
        idxs = [morton_order(m, d, L - li) for li, m in enumerate(sizes)]
        # a level's 2x2x2 blocks are sibling groups: they exist while the level
        # still coarsens
        blocks = [bs if li < L else 1 for li in range(len(sizes))]
    else:
        idxs = [cell_order(m, d, b) for m, b in zip(sizes, blocks)]
    levels = []
    for li, m in enumerate(sizes):
        b = blocks[li]
        lv = Level(A=assemble(faces, idxs[li]), block_size=b ** d, cells=idxs[li])
        if colour:
            lv.colour = parity_colour(m, d, b, idxs[li])
        if li + 1 < len(sizes):
            lv.P = piecewise_constant_P(m, d, b, blocks[li + 1], idxs[li], idxs[li + 1])
            lv.r_scale = 2.0 ** (-d)
            faces = coarsen_faces(faces)
        levels.append(lv)
    return levels


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def poisson2d(n: int = 64, nrhs: int = 1, n_stop: int = 4, config_id: int = 1) -> Problem:
    """Constant-coefficient 2D 5-point Poisson, point blocks (64^2 down to 4^2)."""
    levels = fv_hierarchy(np.ones((n, n)), bs=1, n_stop=n_stop)
    return Problem(f"poisson2d_{n}", levels, uniform_rhs(config_id, n * n, nrhs),
                   meta=dict(d=2, n=n, bs=1))


def sphere_mu(n: int, centre: np.ndarray, radius: float, contrast: float) -> np.ndarray:
    x = (np.arange(n) + 0.5) / n
    X = np.meshgrid(x, x, x, indexing="ij")
    r2 = sum((X[a] - centre[a]) ** 2 for a in range(3))
    return np.where(r2 < radius ** 2, contrast, 1.0)


def interface3d(n: int = 128, nrhs: int = 8, contrast: float = 1e4, radius: float = 0.3,
                bs: int = 2, n_stop: int = 4, config_id: int = 2) -> Problem:
    """3D 7-point variable-coefficient interface problem: mu = contrast inside a
    sphere of the given radius whose centre is drawn U[0.3, 0.7]^3, 1 outside."""
    centre = stream(config_id, GEOMETRY).uniform(0.3, 0.7, size=3)
    mu = sphere_mu(n, centre, radius, contrast)
    levels = fv_hierarchy(mu, bs=bs, n_stop=n_stop)
    return Problem(f"interface3d_{n}", levels, uniform_rhs(config_id, n ** 3, nrhs),
                   meta=dict(d=3, n=n, bs=bs, centre=centre.tolist(), contrast=contrast))


def lognormal2d(n: int, sigma: float = 2.0, nrhs: int = 4, n_stop: int = 8,
                config_id: int = 4, system: int = 0) -> Problem:
    """2D 5-point problem with i.i.d. log-normal cell coefficients exp(sigma Z)."""
    z = stream(config_id, GEOMETRY, system).standard_normal((n, n))
    levels = fv_hierarchy(np.exp(sigma * z), bs=1, n_stop=n_stop)
    return Problem(f"lognormal2d_{n}_{system}", levels,
                   uniform_rhs(config_id, n * n, nrhs, system), meta=dict(d=2, n=n, bs=1))


def batch_sizes(n_sys: int = 64, lo: float = 6.0, hi: float = 9.0, config_id: int = 4) -> np.ndarray:
    """Sizes 16*round(2^u/16), u ~ U[lo, hi] (log-uniform between 64 and 512)."""
    u = stream(config_id, GEOMETRY).uniform(lo, hi, size=n_sys)
    return (16 * np.maximum(1, np.round(2.0 ** u / 16))).astype(int)


def lognormal_batch(n_sys: int = 64, nrhs: int = 4, sigma: float = 2.0,
                    sizes: Optional[Sequence[int]] = None, config_id: int = 4) -> List[Problem]:
    if sizes is None:
        sizes = batch_sizes(n_sys, config_id=config_id)
    return [lognormal2d(int(n), sigma, nrhs, config_id=config_id, system=s)
            for s, n in enumerate(sizes)]


def periodic_laplacian(N: int, d: int) -> sp.csr_matrix:
    """Unit-spacing periodic 5-point (d=2) / 7-point (d=3) negative Laplacian,
    diagonal 2d, lexicographic order."""
    idx = np.arange(N ** d).reshape((N,) * d)
    rows, cols = [idx.ravel()], [idx.ravel()]
    vals = [np.full(N ** d, 2.0 * d)]
    for a in range(d):
        for s in (1, -1):
            rows.append(idx.ravel())
            cols.append(np.roll(idx, s, axis=a).ravel())
            vals.append(-np.ones(N ** d))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N ** d, N ** d)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def periodic_parity(N: int, d: int) -> np.ndarray:
    c = np.indices((N,) * d).reshape(d, -1)
    return (c.sum(axis=0) % 2).astype(np.int32)
