"""Symmetric interior-penalty DG (SIPG) for -Laplace(u) = f on (0, 1)^2 with a
tensor Q3 orthonormal Legendre basis on a jittered quadrilateral mesh, and its
Galerkin hierarchy.

* n^2 quadrilaterals; interior vertices of the uniform grid are moved by i.i.d.
  U[-0.2h, 0.2h] per coordinate, boundary vertices stay; bilinear element maps
  from the reference square [-1, 1]^2.
* Basis on the reference square: phi_{a+4b}(xi, eta) = L_a(xi) L_b(eta),
  L_a = sqrt((2a+1)/2) P_a (Legendre), a, b = 0..3: 16 modes per element.
  Element (I, J) -> block I + nJ; unknown 16 (I + nJ) + a + 4b.
* 6x6 Gauss quadrature on elements, 6 Gauss points per face.
* a(u, v) = sum_K int_K grad u . grad v
            - sum_F int_F ({grad u . n}[v] + {grad v . n}[u])
            + sum_F sigma_F int_F [u][v],
  [u] = u^- - u^+ across an interior face (n from K^- to K^+), {.} the average;
  on a boundary face [u] = u, {grad u . n} = grad u . n (outward): homogeneous
  Dirichlet data imposed weakly.  sigma_F = (p+1)(p+2) max(|F|/|K^-|, |F|/|K^+|)
  = 20 max(...) (boundary: 20 |F|/|K|).
* Coarsening: coarse element (I, J) owns the fine elements (2I+c_x, 2J+c_y);
  P maps coarse Legendre coefficients to each child's by the exact L^2
  projection on the logical reference square (4 fixed 16x16 matrices); A_c =
  P^T A P (Galerkin), restriction P^T.  Down to 4 x 4 elements.
* Colours (I mod 2) + 2 (J mod 2): a proper 4-colouring of the 5-point block
  graph.
"""
from typing import List

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npl

from .problem import Level, Problem
from .rng import GEOMETRY, stream, uniform_rhs

P_DEG = 3
NM = (P_DEG + 1) ** 2     # 16 modes per element


def leg1d(t):
    """Orthonormal Legendre values and derivatives, each [len(t), 4]."""
    t = np.asarray(t, dtype=float)
    V = np.empty((t.size, P_DEG + 1))
    D = np.empty((t.size, P_DEG + 1))
    for a in range(P_DEG + 1):
        c = np.zeros(a + 1)
        c[a] = np.sqrt((2 * a + 1) / 2.0)
        V[:, a] = npl.legval(t, c)
        D[:, a] = npl.legval(t, npl.legder(c))
    return V, D


def basis2d(xi, eta):
    """Values [q, 16] and reference gradients [q, 16, 2] at points (xi, eta)."""
    Vx, Dx = leg1d(xi)
    Vy, Dy = leg1d(eta)
    val = (Vy[:, :, None] * Vx[:, None, :]).reshape(len(xi), NM)                 # index a + 4b
    gx = (Vy[:, :, None] * Dx[:, None, :]).reshape(len(xi), NM)
    gy = (Dy[:, :, None] * Vx[:, None, :]).reshape(len(xi), NM)
    return val, np.stack([gx, gy], axis=-1)


def jittered_vertices(n: int, jitter: float = 0.2, config_id: int = 3, seed_extra: int = 0) -> np.ndarray:
    """Vertex coordinates [n+1, n+1, 2] indexed [i, j] (x index first)."""
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    v = np.stack([i * h, j * h], axis=-1).astype(float)
    d = stream(config_id, GEOMETRY, seed_extra).uniform(-jitter * h, jitter * h, size=v.shape)
    inner = (i > 0) & (i < n) & (j > 0) & (j < n)
    v[inner] += d[inner]
    return v


def _corners(v, n):
    """Element corner coordinates [E, 4, 2] (order (-1,-1), (1,-1), (-1,1), (1,1)), E = I + nJ."""
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")          # [J, I]
    I, J = I.ravel(), J.ravel()                                             # element e = I + n J
    return np.stack([v[I, J], v[I + 1, J], v[I, J + 1], v[I + 1, J + 1]], axis=1)


def _geometry(C, xi, eta):
    """Physical points [E, q, 2], Jacobians [E, q, 2, 2] of the bilinear maps."""
    N = np.stack([(1 - xi) * (1 - eta), (1 + xi) * (1 - eta), (1 - xi) * (1 + eta), (1 + xi) * (1 + eta)],
                 axis=1) / 4.0                                              # [q, 4]
    dNx = np.stack([-(1 - eta), (1 - eta), -(1 + eta), (1 + eta)], axis=1) / 4.0
    dNy = np.stack([-(1 - xi), -(1 + xi), (1 - xi), (1 + xi)], axis=1) / 4.0
    X = np.einsum("qc,ecd->eqd", N, C)
    J = np.stack([np.einsum("qc,ecd->eqd", dNx, C), np.einsum("qc,ecd->eqd", dNy, C)], axis=-1)   # [E,q,d,ref]
    return X, J


def _phys_grad(J, g):
    """grad phi = J^{-T} ghat: J [E, q, 2, 2], g [q, 16, 2] -> [E, q, 16, 2]."""
    Jinv = np.linalg.inv(J)                                                 # [E, q, ref, d]
    return np.einsum("eqrd,qmr->eqmd", Jinv, g)


def assemble(v: np.ndarray, sigma0: float = (P_DEG + 1) * (P_DEG + 2), rhs_fn=None):
    """Block matrix (scipy BSR, 16x16 blocks) and optional load vector."""
    n = v.shape[0] - 1
    E = n * n
    C = _corners(v, n)
    gq, gw = npl.leggauss(6)
    xi, eta = np.meshgrid(gq, gq, indexing="xy")
    xi, eta, w2 = xi.ravel(), eta.ravel(), np.outer(gw, gw).ravel()
    X, J = _geometry(C, xi, eta)
    det = np.linalg.det(J)                                                  # [E, q]
    area = (det * w2).sum(axis=1)
    val, g = basis2d(xi, eta)
    G = _phys_grad(J, g)                                                    # [E, q, 16, 2]
    Gt = G.transpose(0, 2, 1, 3).reshape(E, NM, -1)                       # [E, 16, q*2]
    Gw = (G * (det * w2)[:, :, None, None]).transpose(0, 2, 1, 3).reshape(E, NM, -1)
    Kvol = np.matmul(Gt, Gw.transpose(0, 2, 1))
    rows_d = np.arange(E)
    diag = Kvol.copy()
    offd_r, offd_c, offd_B = [], [], []

    def face_side(ref_xi, ref_eta, elems):
        """Trace values [F, q, 16], physical gradients [F, q, 16, 2] and
        geometry of elements `elems` at reference face points."""
        Xf, Jf = _geometry(C[elems], ref_xi, ref_eta)
        vf, gf = basis2d(ref_xi, ref_eta)
        return np.broadcast_to(vf[None], (len(elems),) + vf.shape), _phys_grad(Jf, gf), Xf

    t = gq
    one = np.ones_like(t)
    # vertical faces x-direction: K- = (I, J) right edge, K+ = (I+1, J) left edge
    # horizontal faces: K- = (I, J) top edge, K+ = (I, J+1) bottom edge
    for direction in (0, 1):
        for I0 in range(-1, n):
            # faces between column/row I0 and I0+1, all J at once
            Js = np.arange(n)
            if direction == 0:
                em = I0 + n * Js
                ep = I0 + 1 + n * Js
                vm = (v[I0 + 1, Js], v[I0 + 1, Js + 1])                    # edge endpoints (bottom, top)
            else:
                em = Js + n * I0
                ep = Js + n * (I0 + 1)
                vm = (v[Js, I0 + 1], v[Js + 1, I0 + 1])                    # (left, right)
            a0, a1 = vm
            L = np.linalg.norm(a1 - a0, axis=1)                            # |F|
            tau = (a1 - a0) / L[:, None]
            nrm = np.stack([tau[:, 1], -tau[:, 0]], axis=1) if direction == 0 else \
                np.stack([-tau[:, 1], tau[:, 0]], axis=1)                  # from K- to K+
            ds = (L / 2.0)[:, None] * gw[None, :]                          # [F, q]
            sides = []
            if I0 >= 0:
                rx, ry = (one, t) if direction == 0 else (t, one)
                vf, gf, _ = face_side(rx, ry, em)
                sides.append((em, +1.0, vf, np.einsum("fqmd,fd->fqm", gf, nrm)))
            if I0 + 1 <= n - 1:
                rx, ry = (-one, t) if direction == 0 else (t, -one)
                vf, gf, _ = face_side(rx, ry, ep)
                sides.append((ep, -1.0, vf, np.einsum("fqmd,fd->fqm", gf, nrm)))
            interior = len(sides) == 2
            if interior:
                sig = sigma0 * np.maximum(L / area[em], L / area[ep])
                avg = 0.5
            else:
                # boundary face: the outward normal is c * nrm, and the same form
                # with average weight 1 gives -(grad u.n) v - (grad v.n) u + sigma u v
                sig = sigma0 * L / area[sides[0][0]]
                avg = 1.0
            for k1, (e1, c1, v1, g1) in enumerate(sides):
                for k2, (e2, c2, v2, g2) in enumerate(sides):
                    w1 = (ds[:, :, None] * v1).transpose(0, 2, 1)           # [F, 16, q]
                    gw1 = (ds[:, :, None] * g1).transpose(0, 2, 1)
                    B = (-avg * c1 * np.matmul(w1, g2) - avg * c2 * np.matmul(gw1, v2)
                         + (c1 * c2) * sig[:, None, None] * np.matmul(w1, v2))
                    if k1 == k2:
                        np.add.at(diag, e1, B)
                    else:
                        offd_r.append(e1)
                        offd_c.append(e2)
                        offd_B.append(B)
    rows = np.concatenate([rows_d] + offd_r)
    cols = np.concatenate([rows_d] + offd_c)
    data = np.concatenate([diag] + offd_B)
    order = np.lexsort((cols, rows))
    rows, cols, data = rows[order], cols[order], data[order]
    indptr = np.searchsorted(rows, np.arange(E + 1))
    A = sp.bsr_matrix((data, cols, indptr), shape=(E * NM, E * NM))
    b = None
    if rhs_fn is not None:
        fq = rhs_fn(X[..., 0], X[..., 1])                                   # [E, q]
        b = np.einsum("eq,eq,qi->ei", fq, det * w2, val).ravel()
    return A, b


def child_matrices() -> np.ndarray:
    """[4, 16, 16]: child c = cx + 2 cy, fine coefficients = M_c @ coarse."""
    gq, gw = npl.leggauss(8)
    out = []
    for cy in (0, 1):
        for cx in (0, 1):
            Ms = []
            for c in (cx, cy):
                s = (gq + (2 * c - 1)) / 2.0                # parent coordinate of child point t
                Vf, _ = leg1d(gq)
                Vc, _ = leg1d(s)
                Ms.append(np.einsum("q,qa,qb->ab", gw, Vf, Vc))
            out.append(np.kron(Ms[1], Ms[0]))
    return np.stack(out)


def prolongation(n: int) -> sp.bsr_matrix:
    """Fine n x n elements <- coarse n/2 x n/2, block rows per fine element."""
    M = child_matrices()
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    I, J = I.ravel(), J.ravel()
    parent = (I // 2) + (n // 2) * (J // 2)
    child = (I % 2) + 2 * (J % 2)
    indptr = np.arange(n * n + 1)
    return sp.bsr_matrix((M[child], parent, indptr), shape=(n * n * NM, (n // 2) ** 2 * NM))


def galerkin(A: sp.bsr_matrix, n: int) -> sp.bsr_matrix:
    """P^T A P block by block: coarse (F, G) += M_f^T A_fg M_g."""
    M = child_matrices()
    E = n * n
    rows = np.repeat(np.arange(E), np.diff(A.indptr))
    cols = A.indices
    nc = n // 2

    def parent(e):
        return (e % n) // 2 + nc * ((e // n) // 2)

    def child(e):
        return (e % n) % 2 + 2 * ((e // n) % 2)

    Bc = np.matmul(np.matmul(np.transpose(M[child(rows)], (0, 2, 1)), A.data), M[child(cols)])
    key = parent(rows) * (nc * nc) + parent(cols)
    uk, inv = np.unique(key, return_inverse=True)
    data = np.zeros((len(uk), NM, NM))
    np.add.at(data, inv, Bc)
    r, c = uk // (nc * nc), uk % (nc * nc)
    indptr = np.searchsorted(r, np.arange(nc * nc + 1))
    return sp.bsr_matrix((data, c, indptr), shape=(nc * nc * NM, nc * nc * NM))


def colours(n: int) -> np.ndarray:
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    return ((I % 2) + 2 * (J % 2)).ravel().astype(np.int32)


def hierarchy(A: sp.bsr_matrix, n: int, n_stop: int = 4) -> List[Level]:
    levels = []
    while True:
        lv = Level(A=A.tocsr(), block_size=NM, colour=colours(n))
        lv.A.sort_indices()
        if n <= n_stop or n % 2:
            levels.append(lv)
            break
        lv.P = prolongation(n).tocsr()
        lv.r_scale = 1.0
        levels.append(lv)
        A = galerkin(A, n)
        n //= 2
    return levels


def sipg_q3(n: int = 256, nrhs: int = 1, jitter: float = 0.2, config_id: int = 3, seed_extra: int = 0) -> Problem:
    v = jittered_vertices(n, jitter, config_id, seed_extra)
    A, _ = assemble(v)
    levels = hierarchy(A, n)
    return Problem(f"sipg_q3_{n}", levels, uniform_rhs(config_id, n * n * NM, nrhs, seed_extra),
                   meta=dict(d=2, n=n, p=P_DEG, vertices=v))
