"""Trilinear (Q1) finite-element diffusion on the unit cube with a multiphase
coefficient, and its Galerkin hierarchy.

* n^3 hexahedra of width h = 1/n; nodes (i, j, k), 0 <= i, j, k <= n.
  Homogeneous Dirichlet data on the faces x = 1, y = 1, z = 1 (those nodes are
  eliminated) and natural (Neumann) conditions on x = 0, y = 0, z = 0, so the
  unknown nodes are 0 <= i, j, k < n: n^3 unknowns.
* Element matrix of hex e: mu_e * h * K, K the exact trilinear stiffness of
  the unit cube, K = S x M x M + M x S x M + M x M x S with the 1D linear
  element stiffness S and mass M.
* Unknowns come in 2x2x2 node blocks: block (I, J, K) holds nodes
  (2I + a, 2J + b, 2K + c), blocks lexicographic (x fastest), local index
  a + 2b + 4c.
* Coarse level: the nodes (2I, 2J, 2K) of the fine grid; P is trilinear
  interpolation (1D: even fine node = coarse node, odd = mean of its two
  coarse neighbours, a Dirichlet neighbour contributing 0); A_c = P^T A P,
  restriction P^T (r_scale 1).
* Coefficient: a Gaussian random field with squared-exponential covariance
  exp(-r^2 / (2 l^2)), l = 8h, sampled spectrally on a periodic (2n)^3 grid of
  hex centres and cropped to n^3; thresholds at its empirical 1/3 and 2/3
  quantiles give three phases with mu = 1, 1e3, 1e6 (low to high).
"""
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .problem import Level, Problem
from .rng import GEOMETRY, stream, uniform_rhs

S1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0


def q1_stiffness() -> np.ndarray:
    """8x8 stiffness of the unit cube, local node a + 2b + 4c (x fastest)."""
    # np.kron(Z, np.kron(Y, X)) indexes (c, b, a) -> a + 2b + 4c
    return (np.kron(M1, np.kron(M1, S1)) + np.kron(M1, np.kron(S1, M1)) + np.kron(S1, np.kron(M1, M1)))


def node_order(n: int) -> np.ndarray:
    """Unknown number of node (i, j, k), array indexed [k, j, i]; n even."""
    k, j, i = np.indices((n, n, n))
    nb = n // 2
    blk = (i // 2) + nb * ((j // 2) + nb * (k // 2))
    loc = (i % 2) + 2 * (j % 2) + 4 * (k % 2)
    return 8 * blk + loc


def grf_phases(n: int, seed_extra: int = 0, corr_cells: float = 8.0, config_id: int = 5,
               values=(1.0, 1e3, 1e6)) -> np.ndarray:
    """Three-phase coefficient per hex, array indexed [k, j, i]."""
    m = 2 * n
    w = stream(config_id, GEOMETRY, seed_extra).standard_normal((m, m, m))
    f = 2.0 * np.pi * np.fft.fftfreq(m)          # angular wavenumbers per cell
    kk = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    spec = np.exp(-0.5 * corr_cells ** 2 * kk)   # SE spectrum up to a constant
    g = np.fft.ifftn(np.fft.fftn(w) * np.sqrt(spec)).real[:n, :n, :n]
    t1, t2 = np.quantile(g, [1.0 / 3.0, 2.0 / 3.0])
    mu = np.full(g.shape, values[0])
    mu[g > t1] = values[1]
    mu[g > t2] = values[2]
    return mu


def assemble(mu: np.ndarray) -> sp.csr_matrix:
    """Global stiffness on the unknown nodes, in block order."""
    n = mu.shape[0]
    h = 1.0 / n
    K = q1_stiffness()
    order = node_order(n)
    ez, ey, ex = np.indices((n, n, n))
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    scale = (mu * h).ravel()
    gid, ok = [], []
    for loc in range(8):
        a, b, c = loc & 1, (loc >> 1) & 1, (loc >> 2) & 1
        i, j, k = ex + a, ey + b, ez + c
        inside = (i < n) & (j < n) & (k < n)
        gid.append(np.where(inside, order[np.minimum(k, n - 1), np.minimum(j, n - 1), np.minimum(i, n - 1)], -1))
        ok.append(inside)
    rows, cols, vals = [], [], []
    for p in range(8):
        for q in range(8):
            m = ok[p] & ok[q]
            rows.append(gid[p][m])
            cols.append(gid[q][m])
            vals.append(scale[m] * K[p, q])
    N = n ** 3
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    return A


def interp1d(n: int) -> sp.csr_matrix:
    """Linear interpolation from the n/2 coarse to the n fine unknown nodes of
    one axis (the node at n / n/2 is Dirichlet)."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        if i % 2 == 0:
            rows.append(i), cols.append(i // 2), vals.append(1.0)
        else:
            for c in ((i - 1) // 2, (i + 1) // 2):
                if c < nc:
                    rows.append(i), cols.append(c), vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def trilinear_P(n: int) -> sp.csr_matrix:
    """Trilinear interpolation, fine block order <- coarse block order."""
    P1 = interp1d(n)
    P = sp.kron(P1, sp.kron(P1, P1, format="csr"), format="csr")   # lexicographic, x fastest
    of = node_order(n).ravel()          # lexicographic -> block order
    oc = node_order(n // 2).ravel()
    P = P.tocoo()
    P = sp.csr_matrix((P.data, (of[P.row], oc[P.col])), shape=P.shape)
    P.sort_indices()
    return P


def galerkin_hierarchy(A: sp.csr_matrix, n: int, n_stop: int = 6) -> List[Level]:
    levels = []
    while True:
        lv = Level(A=A, block_size=8)
        if n <= n_stop or n % 4:
            levels.append(lv)
            break
        P = trilinear_P(n)
        lv.P, lv.r_scale = P, 1.0
        levels.append(lv)
        A = (P.T @ (A @ P)).tocsr()
        A.sum_duplicates()
        A.sort_indices()
        n //= 2
    return levels


def multiphase3d(n: int = 96, nrhs: int = 1, seed_extra: int = 0, config_id: int = 5) -> Problem:
    """Q1 multiphase diffusion; seed_extra selects the coefficient sample
    (training samples and the test sample use different values)."""
    mu = grf_phases(n, seed_extra, config_id=config_id)
    levels = galerkin_hierarchy(assemble(mu), n)
    return Problem(f"multiphase3d_{n}_{seed_extra}", levels,
                   uniform_rhs(config_id, n ** 3, nrhs, seed_extra),
                   meta=dict(d=3, n=n, bs=2, log10mu=np.log10(mu)))
