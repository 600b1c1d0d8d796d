"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here is CPU-only.  None of them re-calls the oracle routine it
checks to produce the expected value: expectations come from the paper's
Table 1, closed forms (Fourier symbols, first-level least squares), textbook
iterations written as explicit loops, dense brute-force least squares over the
whole Frobenius objective, or invariances of the definitions.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from synth import fd
from synth.rng import TEST, stream

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers (independent of the oracle)
# ---------------------------------------------------------------------------

def random_block_matrix(B, n, seed, extra_edges=2, symmetric=False):
    """Block-sparse matrix with a positive diagonal: ring + random couplings,
    dense random blocks, diagonally dominant diagonal blocks."""
    rng = stream(0, TEST, seed)
    edges = {(i, (i + 1) % B) for i in range(B)}
    for _ in range(extra_edges * B // 2):
        i, j = rng.integers(0, B, size=2)
        if i != j:
            edges.add((int(i), int(j)))
    N = B * n
    A = np.zeros((N, N))
    for (i, j) in edges:
        blk = rng.uniform(-1.0, 0.2, size=(n, n))
        A[i * n:(i + 1) * n, j * n:(j + 1) * n] += blk
        A[j * n:(j + 1) * n, i * n:(i + 1) * n] += blk.T if symmetric else rng.uniform(-1.0, 0.2, size=(n, n))
    for i in range(B):
        D = rng.uniform(-0.3, 0.3, size=(n, n))
        if symmetric:
            D = D + D.T
        A[i * n:(i + 1) * n, i * n:(i + 1) * n] += D
    rowsum = np.abs(A).sum(axis=1)
    A[np.arange(N), np.arange(N)] = rowsum + 1.0
    return A


def brute_force_cascade(A, n, depth, colours=None, ridge=0.0):
    """Solve every Frobenius problem of the cascade as ONE dense least-squares
    problem over all block-diagonal unknowns at once (SVD lstsq), without any
    per-block decoupling, normal equations or sparse products.  ridge > 0 adds
    the Tikhonov term tau_i ||Lambda_i||_F^2, tau_i = ridge * (squared norm of
    block i's rows of M) / n, as extra rows sqrt(tau_i) e_(i,r,s) with target 0."""
    N = A.shape[0]
    B = N // n
    w = 1.0 / np.sqrt(np.diag(A))
    At = w[:, None] * A * w[None, :]
    E = np.eye(N)
    chi = 1 if colours is None else int(np.max(colours)) + 1
    lams = [np.zeros((B, n, n)) for _ in range(depth)]
    for l in range(depth):
        for k in range(chi):
            blocks = np.arange(B) if colours is None else np.flatnonzero(colours == k)
            M = At @ E
            cols = []
            for i in blocks:
                for r in range(n):
                    for s in range(n):
                        Z = np.zeros((N, N))
                        Z[i * n + r, :] = M[i * n + s, :]
                        cols.append(Z.ravel())
            D = np.stack(cols, axis=1)
            rhs = E.ravel()
            if ridge:
                tau = np.repeat([ridge * np.sum(M[i * n:(i + 1) * n] ** 2) / n for i in blocks], n * n)
                D = np.vstack([D, np.diag(np.sqrt(tau))])
                rhs = np.concatenate([rhs, np.zeros(len(tau))])
            sol = np.linalg.lstsq(D, rhs, rcond=None)[0]
            Lfull = np.zeros((N, N))
            t = 0
            for i in blocks:
                for r in range(n):
                    for s in range(n):
                        lams[l][i, r, s] = sol[t]
                        Lfull[i * n + r, i * n + s] = sol[t]
                        t += 1
            E = E - Lfull @ M
    return lams


def load_table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows[(parts[0], int(parts[1]))] = [float(v) for v in parts[2:]]
    return rows


# ---------------------------------------------------------------------------
# Table 1 and Fourier closed forms
# ---------------------------------------------------------------------------

# N > 2 x (fill radius) so that no fill wraps round the torus.
TABLE1_N = {2: 20, 3: 16}


@pytest.mark.parametrize("d", [2, 3])
def test_table1_additive(d):
    want = load_table1()[("additive", d)]
    A = fd.periodic_laplacian(TABLE1_N[d], d)
    res = O.fit_additive(A, 1, 4)
    for l, L in enumerate(res["lam"]):
        lam = L[:, 0, 0] * 2 * d                     # Lambda_l = lambda_l diag(A)^-1
        assert np.ptp(lam) < 1e-12                   # scaled identity on a periodic grid
        assert abs(lam[0] - want[l]) <= 0.005 + 1e-12, (d, l, lam[0], want[l])


@pytest.mark.parametrize("d", [2, 3])
def test_table1_red_black(d):
    want = load_table1()[("multiplicative", d)]
    N = TABLE1_N[d]
    A = fd.periodic_laplacian(N, d)
    c = fd.periodic_parity(N, d)
    res = O.fit_multiplicative(A, 1, 4, c)
    for l, L in enumerate(res["lam"]):
        for k in range(2):
            lam = L[c == k, 0, 0] * 2 * d
            assert np.ptp(lam) < 1e-12
            assert abs(lam[0] - want[2 * l + k]) <= 0.005 + 1e-12, (d, l, k, lam[0])


def fourier_lambdas(N, d, depth):
    """lambda_l from the discrete Fourier symbol of the periodic Laplacian:
    sigma(theta) = 1 - mean_k cos(theta_k) is the symbol of the prescaled
    operator; by Parseval the Frobenius objective of level l is
    sum_theta (1 - lambda sigma)^2 prod_{m<l} (1 - lambda_m sigma)^2."""
    th = 2 * np.pi * np.arange(N) / N
    grids = np.meshgrid(*([th] * d), indexing="ij")
    sigma = 1.0 - sum(np.cos(g) for g in grids) / d
    P = np.ones_like(sigma)
    out = []
    for _ in range(depth):
        lam = float((sigma * P ** 2).sum() / (sigma ** 2 * P ** 2).sum())
        out.append(lam)
        P = P * (1.0 - lam * sigma)
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_additive_matches_fourier_symbol(d):
    N = TABLE1_N[d]
    res = O.fit_additive(fd.periodic_laplacian(N, d), 1, 4)
    want = fourier_lambdas(N, d, 4)
    got = [L[0, 0, 0] * 2 * d for L in res["lam"]]
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_exact_rationals():
    # Infinite-grid moments: 2D lambda_1 = 4/5, lambda_2 = 6/7;
    # 3D lambda_1 = 6/7 (optimal Jacobi damping, Sec. 3.4.1), lambda_2 = 15/17.
    r2 = O.fit_additive(fd.periodic_laplacian(12, 2), 1, 2)["lam"]
    r3 = O.fit_additive(fd.periodic_laplacian(8, 3), 1, 2)["lam"]
    assert abs(r2[0][0, 0, 0] * 4 - 4 / 5) < 1e-13
    assert abs(r2[1][0, 0, 0] * 4 - 6 / 7) < 1e-13
    assert abs(r3[0][0, 0, 0] * 6 - 6 / 7) < 1e-13
    assert abs(r3[1][0, 0, 0] * 6 - 15 / 17) < 1e-13


@pytest.mark.parametrize("d,mu_exact", [(2, 3 / 5), (3, 5 / 7)])
def test_one_level_is_optimally_damped_jacobi(d, mu_exact):
    """A depth-1 point cascade is damped Jacobi with the classical optimal
    weight; its local Fourier smoothing factor over the high frequencies is
    3/5 (2D) / 5/7 (3D)."""
    lam = O.fit_additive(fd.periodic_laplacian(8, d), 1, 1)["lam"][0][0, 0, 0] * 2 * d
    th = np.linspace(-np.pi, np.pi, 257)
    grids = np.meshgrid(*([th] * d), indexing="ij")
    high = np.zeros_like(grids[0], dtype=bool)
    for g in grids:
        high |= np.abs(g) >= np.pi / 2
    sigma = 1.0 - sum(np.cos(g) for g in grids) / d
    mu = np.abs(1.0 - lam * sigma)[high].max()
    assert abs(mu - mu_exact) < 1e-12


# ---------------------------------------------------------------------------
# First-level closed form on a bounded problem (every row, boundary included)
# ---------------------------------------------------------------------------

def test_first_level_closed_form_dirichlet():
    """With E_0 = I and point blocks, the level-1 least-squares problem has the
    solution lambda~_i = a~_ii / sum_j a~_ij^2 on the prescaled matrix."""
    p = fd.poisson2d(64)
    A = p.levels[0].A
    res = O.fit_additive(A, 1, 3)
    C = sp.coo_matrix(A)
    dg = A.diagonal()
    at = C.data / np.sqrt(dg[C.row] * dg[C.col])
    s2 = np.bincount(C.row, weights=at ** 2, minlength=A.shape[0])
    lam = (1.0 / s2) / dg
    np.testing.assert_allclose(res["lam"][0][:, 0, 0], lam, rtol=1e-14)
    # interior rows: optimal Jacobi damping 4/5 of 1/diag
    inner = np.flatnonzero(np.isclose(s2, 1.25))
    assert len(inner) == 60 * 60        # rows whose neighbours are all interior too
    np.testing.assert_allclose(res["lam"][0][inner, 0, 0] * dg[inner], 0.8, rtol=1e-14)


@pytest.mark.parametrize("nu", [1, 2])
def test_depth_one_vcycle_is_the_weighted_jacobi_textbook_vcycle(nu):
    """Alg. 1 with a depth-1 point cascade is the textbook V-cycle with the
    weighted Jacobi smoother x <- x + w_i (b - A x)_i, w_i = 1 / sum_j
    (a_ij^2 / a_jj) (the level-1 closed form above, unscaled; 4/5 of 1/a_ii on
    interior rows of the 5-point Laplacian, Sec. 3.2): written here in the
    error-correction form,
    with dense matrices, restriction r_scale P^T of the residual b - A x,
    correction x + P e_c and an exact bottom solve, independently of the
    oracle's setup and of its sign convention."""
    p = fd.poisson2d(32)
    lv = p.levels

    def weights(A):
        C = sp.coo_matrix(A)
        return 1.0 / np.bincount(C.row, weights=C.data ** 2 / A.diagonal()[C.col], minlength=A.shape[0])

    def textbook(l, b):
        A = lv[l].A.toarray()
        if l == len(lv) - 1:
            return np.linalg.solve(A, b)
        w = weights(lv[l].A)[:, None]
        x = np.zeros_like(b)
        for _ in range(nu):
            x = x + w * (b - A @ x)
        P = lv[l].P.toarray()
        e = textbook(l + 1, lv[l].r_scale * (P.T @ (b - A @ x)))
        x = x + P @ e
        for _ in range(nu):
            x = x + w * (b - A @ x)
        return x

    b = stream(0, TEST, 19).uniform(-1, 1, size=(p.n, 2))
    sm = O.setup_hierarchy(lv, 1)
    want = textbook(0, b)
    for order in ("RF", "FF"):   # a single point level: forward and reverse coincide
        got = O.vcycle(lv, sm, b, order, nu, nu)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), order


def test_jacobi_reference_smoother():
    """The reference smoother of Sec. 3.2: every level omega A_ii^-1.  Its blocks
    times the diagonal blocks of a non-symmetric A give omega I (a transposed or
    undamped inverse fails), and with point blocks on the periodic 5-point
    Laplacian and omega = 4/5 it is the depth-1 cascade fit (Table 1), reached by
    the least-squares route instead of the inverse."""
    n, B = 3, 7
    A = random_block_matrix(B, n, 5, symmetric=False)
    sm = O.jacobi_smoother(sp.csr_matrix(A), n, 2, omega=0.7)
    assert len(sm["lam"]) == 2 and sm["colours"] is None
    for L in sm["lam"]:
        for i in range(B):
            Aii = A[i * n:(i + 1) * n, i * n:(i + 1) * n]
            np.testing.assert_allclose(L[i] @ Aii, 0.7 * np.eye(n), atol=1e-13)
    P = fd.periodic_laplacian(12, 2)
    fit = O.fit_additive(P, 1, 1)["lam"][0]
    jac = O.jacobi_smoother(P, 1, 1, omega=0.8)["lam"][0]
    np.testing.assert_allclose(jac, fit, rtol=1e-13)


# ---------------------------------------------------------------------------
# Brute-force Frobenius minimisation on tiny matrices
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("B,n,depth,seed", [(12, 1, 3, 0), (8, 2, 3, 1), (6, 3, 2, 2), (6, 4, 2, 3)])
def test_additive_vs_brute_force(B, n, depth, seed):
    A = random_block_matrix(B, n, seed)
    want = brute_force_cascade(A, n, depth)
    got = O.fit_additive(sp.csr_matrix(A), n, depth)["lam_tilde"]
    for l in range(depth):
        np.testing.assert_allclose(got[l], want[l], rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("B,n,depth,chi,seed", [(12, 1, 3, 2, 4), (9, 2, 2, 3, 5), (8, 3, 2, 2, 6)])
def test_multiplicative_vs_brute_force(B, n, depth, chi, seed):
    A = random_block_matrix(B, n, seed)
    colours = np.arange(B) % chi
    want = brute_force_cascade(A, n, depth, colours)
    got = O.fit_multiplicative(sp.csr_matrix(A), n, depth, colours)["lam_tilde"]
    for l in range(depth):
        np.testing.assert_allclose(got[l], want[l], rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("mode,B,n,depth,seed", [("additive", 10, 1, 3, 21), ("additive", 6, 3, 2, 22),
                                                  ("multiplicative", 8, 2, 2, 23)])
def test_ridge_fit_vs_brute_force(mode, B, n, depth, seed):
    """The Tikhonov-regularised fit against the whole regularised objective as
    one dense least-squares problem (augmented rows)."""
    A = random_block_matrix(B, n, seed)
    colours = None if mode == "additive" else np.arange(B) % 2
    for ridge in (1e-3, 0.5):
        want = brute_force_cascade(A, n, depth, colours, ridge=ridge)
        got = O.fit(sp.csr_matrix(A), n, depth, mode, colours, ridge=ridge)["lam_tilde"]
        for l in range(depth):
            np.testing.assert_allclose(got[l], want[l], rtol=1e-9, atol=1e-11)


def test_ridge_first_level_closed_form():
    """Point blocks, E_0 = I: lambda~_i = a~_ii / ((1 + ridge) sum_j a~_ij^2)."""
    p = fd.poisson2d(32)
    A = p.levels[0].A
    C = sp.coo_matrix(A)
    dg = A.diagonal()
    at = C.data / np.sqrt(dg[C.row] * dg[C.col])
    s2 = np.bincount(C.row, weights=at ** 2, minlength=A.shape[0])
    for ridge in (1e-3, 0.25):
        res = O.fit_additive(A, 1, 2, ridge=ridge)
        np.testing.assert_allclose(res["lam_tilde"][0][:, 0, 0], 1.0 / ((1.0 + ridge) * s2), rtol=1e-14)


def test_first_order_optimality():
    """[(E - Lambda M) M^T]_ii = 0 for every block at every level."""
    A = random_block_matrix(10, 3, 7)
    n, depth = 3, 3
    res = O.fit_additive(sp.csr_matrix(A), n, depth)
    w = 1.0 / np.sqrt(np.diag(A))
    At = w[:, None] * A * w[None, :]
    E = np.eye(A.shape[0])
    for l in range(depth):
        M = At @ E
        L = np.zeros_like(A)
        for i in range(10):
            L[i * n:(i + 1) * n, i * n:(i + 1) * n] = res["lam_tilde"][l][i]
        R = (E - L @ M) @ M.T
        for i in range(10):
            blk = R[i * n:(i + 1) * n, i * n:(i + 1) * n]
            assert np.abs(blk).max() < 1e-12 * np.abs(M).max() ** 2 * A.shape[0]
        E = E - L @ M


def test_one_colour_collapses_to_additive():
    A = sp.csr_matrix(random_block_matrix(10, 2, 8))
    a = O.fit_additive(A, 2, 3)
    m = O.fit_multiplicative(A, 2, 3, np.zeros(10, dtype=np.int32))
    for l in range(3):
        np.testing.assert_array_equal(a["lam"][l], m["lam"][l])


# ---------------------------------------------------------------------------
# Application: block Jacobi / block Gauss-Seidel as written in textbooks
# ---------------------------------------------------------------------------

def test_inverse_diagonal_gives_block_jacobi_and_gauss_seidel():
    n, B = 2, 9
    A = random_block_matrix(B, n, 9, symmetric=True)
    rng = stream(0, TEST, 10)
    b = rng.uniform(-1, 1, size=(B * n, 2))
    x0 = rng.uniform(-1, 1, size=(B * n, 2))
    Ainv = [np.linalg.inv(A[i * n:(i + 1) * n, i * n:(i + 1) * n]) for i in range(B)]
    lam = np.stack(Ainv)
    # block Jacobi, two sweeps: x_i <- A_ii^-1 (b_i - sum_{j != i} A_ij x_j)
    x = x0.copy()
    for _ in range(2):
        xn = x.copy()
        for i in range(B):
            s = b[i * n:(i + 1) * n].copy()
            for j in range(B):
                if j != i:
                    s -= A[i * n:(i + 1) * n, j * n:(j + 1) * n] @ x[j * n:(j + 1) * n]
            xn[i * n:(i + 1) * n] = Ainv[i] @ s
        x = xn
    got = O.smooth(sp.csr_matrix(A), dict(lam=[lam, lam], colours=None), x0, b)
    np.testing.assert_allclose(got, x, rtol=1e-13, atol=1e-14)
    # multicoloured block Gauss-Seidel (in place, colours 0,1,2 in order)
    colours = np.arange(B) % 3
    x = x0.copy()
    for _ in range(2):
        for k in range(3):
            for i in np.flatnonzero(colours == k):
                s = b[i * n:(i + 1) * n].copy()
                for j in range(B):
                    if j != i:
                        s -= A[i * n:(i + 1) * n, j * n:(j + 1) * n] @ x[j * n:(j + 1) * n]
                x[i * n:(i + 1) * n] = Ainv[i] @ s
    # the in-place sweep equals the colour-restricted smoother only when no two
    # blocks of one colour are coupled; check that first
    Apat = O.block_pattern(sp.csr_matrix(A), n)
    if O.is_proper_colouring(Apat, colours):
        got = O.smooth(sp.csr_matrix(A), dict(lam=[lam, lam], colours=colours), x0, b)
        np.testing.assert_allclose(got, x, rtol=1e-13, atol=1e-14)


def test_gauss_seidel_proper_colouring_grid():
    """Red-black block GS on a 5-point grid, textbook in-place loops."""
    n_grid = 6
    lv0 = fd.poisson2d(n_grid).levels[0]
    A = lv0.A.toarray()
    N = A.shape[0]
    colours = fd.parity_colour(n_grid, 2, 1, lv0.cells)
    rng = stream(0, TEST, 11)
    b = rng.uniform(-1, 1, size=(N, 1))
    x = np.zeros((N, 1))
    for _ in range(3):
        for k in (0, 1):
            for i in np.flatnonzero(colours == k):
                x[i] = (b[i] - A[i] @ x + A[i, i] * x[i]) / A[i, i]
    lam = (1.0 / np.diag(A)).reshape(N, 1, 1)
    got = O.smooth(sp.csr_matrix(A), dict(lam=[lam] * 3, colours=colours), np.zeros((N, 1)), b)
    np.testing.assert_allclose(got, x, rtol=1e-13, atol=1e-15)


def test_forward_and_reverse_closed_forms():
    """Supplementary V-cycle symmetry section: forward application maps
    x0 -> (I-L_nu A)...(I-L_1 A) x0 + A^-1 [I - (I-A L_nu)...(I-A L_1)] b and
    reverse uses L_l^T in the opposite order."""
    n, B, depth = 2, 6, 3
    A = random_block_matrix(B, n, 12)
    N = A.shape[0]
    rng = stream(0, TEST, 13)
    lam = [rng.uniform(-0.3, 0.3, size=(B, n, n)) for _ in range(depth)]
    Ls = []
    for L in lam:
        F = np.zeros((N, N))
        for i in range(B):
            F[i * n:(i + 1) * n, i * n:(i + 1) * n] = L[i]
        Ls.append(F)
    x0 = rng.uniform(-1, 1, size=(N, 1))
    b = rng.uniform(-1, 1, size=(N, 1))
    I = np.eye(N)
    Ainv = np.linalg.inv(A)
    # forward
    T = I.copy()
    S = I.copy()
    for F in Ls:
        T = (I - F @ A) @ T
        S = (I - A @ F) @ S
    want = T @ x0 + Ainv @ (I - S) @ b
    got = O.smooth(sp.csr_matrix(A), dict(lam=lam, colours=None), x0, b)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12)
    # reverse
    T = I.copy()
    S = I.copy()
    for F in reversed(Ls):
        T = (I - F.T @ A) @ T
        S = (I - A @ F.T) @ S
    want = T @ x0 + Ainv @ (I - S) @ b
    got = O.smooth(sp.csr_matrix(A), dict(lam=lam, colours=None), x0, b, reverse=True)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# Invariances of the setup
# ---------------------------------------------------------------------------

def test_diagonal_scaling_invariance():
    """Lambda(D A D) = D^-1 Lambda(A) D^-1 for positive diagonal D, and
    Lambda(c A) = Lambda(A) / c (prescaling, Sec. 2.3)."""
    n, B = 2, 8
    A = random_block_matrix(B, n, 14)
    dvec = stream(0, TEST, 15).uniform(0.1, 10.0, size=B * n)
    base = O.fit_additive(sp.csr_matrix(A), n, 3)["lam"]
    scaled = O.fit_additive(sp.csr_matrix(dvec[:, None] * A * dvec[None, :]), n, 3)["lam"]
    times = O.fit_additive(sp.csr_matrix(7.5 * A), n, 3)["lam"]
    db = dvec.reshape(B, n)
    for l in range(3):
        want = base[l] / db[:, :, None] / db[:, None, :]
        np.testing.assert_allclose(scaled[l], want, rtol=1e-10)
        np.testing.assert_allclose(times[l], base[l] / 7.5, rtol=1e-12)


def test_permutation_equivariance():
    n, B = 2, 10
    A = random_block_matrix(B, n, 16)
    perm = stream(0, TEST, 17).permutation(B)          # new block p holds old block perm[p]
    sidx = (perm[:, None] * n + np.arange(n)[None, :]).ravel()
    Ap = A[np.ix_(sidx, sidx)]
    base = O.fit_additive(sp.csr_matrix(A), n, 3)["lam"]
    got = O.fit_additive(sp.csr_matrix(Ap), n, 3)["lam"]
    for l in range(3):
        np.testing.assert_allclose(got[l], base[l][perm], rtol=1e-12, atol=1e-15)


def test_additive_pattern_is_power_of_A():
    p = fd.lognormal2d(12, n_stop=12)
    A = p.levels[0].A
    res = O.fit_additive(A, 1, 4)
    S = (A.toarray() != 0).astype(np.int64)
    Pw = np.eye(A.shape[0], dtype=np.int64)
    for l, pat in enumerate(res["patterns"]):
        np.testing.assert_array_equal(pat.toarray(), Pw > 0)
        Pw = np.minimum(S @ Pw, 1)


# ---------------------------------------------------------------------------
# V-cycle properties
# ---------------------------------------------------------------------------

def test_periodic_ff_equals_rf():
    """Every Lambda_l is a scaled identity on a periodic grid, so forward and
    reverse applications coincide (footnote of Sec. 3.4.1)."""
    N = 12
    A = fd.periodic_laplacian(N, 2)
    sm = O.fit_additive(A, 1, 3)
    b = stream(0, TEST, 18).uniform(-1, 1, size=(N * N, 1))
    f = O.smooth(A, sm, np.zeros_like(b), b)
    r = O.smooth(A, sm, np.zeros_like(b), b, reverse=True)
    np.testing.assert_allclose(f, r, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("mode", ["additive", "multiplicative"])
def test_rf_vcycle_is_symmetric(mode):
    p = fd.lognormal2d(16, n_stop=4)
    for lv in p.levels:
        lv.colour = fd.parity_colour(int(round(np.sqrt(lv.n))), 2, 1, lv.cells)
    sm = O.setup_hierarchy(p.levels, 2, mode)
    I = np.eye(p.n)
    V = O.vcycle(p.levels, sm, I, order="RF")
    assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    Vf = O.vcycle(p.levels, sm, I, order="FF")
    assert np.abs(Vf - Vf.T).max() > 1e-6 * np.abs(Vf).max()


def test_poisson64_convergence():
    """64^2 Dirichlet Poisson, depth-3 additive, V(2,2): monotone residual decay,
    rho < 1, eta < 3 (the 'effective' threshold of Sec. 3.3)."""
    p = fd.poisson2d(64)
    sm = O.setup_hierarchy(p.levels, 3)
    x, hist = O.solve(p.levels, sm, p.rhs, npre=2, npost=2)
    assert hist[-1] <= 1e-10
    assert all(b < a for a, b in zip(hist, hist[1:]))
    rho = O.rho_regression(hist)
    assert rho < 0.1 and O.eta(rho) < 3
    r = p.rhs - p.levels[0].A @ x
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(p.rhs)


def test_rho_regression_geometric():
    h = [3.0 * 0.37 ** i for i in range(9)]
    assert abs(O.rho_regression(h) - 0.37) < 1e-12
    assert abs(O.eta(0.1) - 1.0) < 1e-15
    # C_d(nu=1, eta=1) in 2D: 1 + 3/(3/4) = 5
    assert abs(O.cost_model(1, 1.0, 2) - 5.0) < 1e-15


# ---------------------------------------------------------------------------
# Colouring, truncation and the local evaluation used at large sizes
# ---------------------------------------------------------------------------

def test_greedy_colouring_of_grid_is_red_black():
    n = 9
    A = fd.poisson2d(n, n_stop=n).levels[0].A
    c = O.greedy_colour(O.block_pattern(A, 1))
    np.testing.assert_array_equal(c, fd.parity_colour(n, 2, 1))
    rnd = sp.csr_matrix(random_block_matrix(30, 1, 19, extra_edges=4))
    pat = O.block_pattern(rnd, 1)
    cc = O.greedy_colour(pat)
    assert O.is_proper_colouring(pat, cc)
    assert not O.is_proper_colouring(pat, np.zeros(30, dtype=np.int32))


def test_truncation():
    A = sp.csr_matrix(random_block_matrix(10, 2, 20, extra_edges=3))
    full = O.fit_additive(A, 2, 3)
    big = O.fit_additive(A, 2, 3, alpha=10)          # alpha >= row length: no change
    for l in range(3):
        np.testing.assert_allclose(full["lam"][l], big["lam"][l], rtol=1e-12, atol=1e-15)
    one = O.fit_additive(A, 2, 2, alpha=1)
    # with alpha = 1 each row of E_1 keeps exactly its largest block; the next
    # fit sees that truncated E (brute force on the truncated E_1)
    w = 1.0 / np.sqrt(A.diagonal())
    At = (w[:, None] * A.toarray() * w[None, :])
    lt1 = one["lam_tilde"][0]
    L1 = np.zeros_like(At)
    for i in range(10):
        L1[2 * i:2 * i + 2, 2 * i:2 * i + 2] = lt1[i]
    E1 = np.eye(20) - L1 @ At
    Et = np.zeros_like(E1)
    for i in range(10):
        norms = [np.linalg.norm(E1[2 * i:2 * i + 2, 2 * j:2 * j + 2]) for j in range(10)]
        j = int(np.argmax(norms))
        Et[2 * i:2 * i + 2, 2 * j:2 * j + 2] = E1[2 * i:2 * i + 2, 2 * j:2 * j + 2]
    assert one["patterns"][1].sum(axis=1).max() == 1
    M = At @ Et
    for i in range(10):
        Mi, Ei = M[2 * i:2 * i + 2], Et[2 * i:2 * i + 2]
        want = np.linalg.lstsq(Mi.T, Ei.T, rcond=None)[0].T
        np.testing.assert_allclose(one["lam_tilde"][1][i], want, rtol=1e-9, atol=1e-12)


def test_local_patch_fit_reproduces_full_fit():
    p = fd.interface3d(16, nrhs=1, n_stop=16)
    A = p.levels[0].A
    full = O.fit_additive(A, 8, 3)["lam"]
    centres = [0, 27, 100, 219, 511]
    loc = O.fit_local(A, 8, 3, centres)
    for c in centres:
        for l in range(3):
            np.testing.assert_allclose(loc[c][l], full[l][c], rtol=1e-11, atol=1e-14)
    # one layer less is not enough (negative control)
    short = O.fit_local(A, 8, 3, [219], radius=2)
    assert np.abs(short[219][2] - full[2][219]).max() > 1e-10 * np.abs(full[2][219]).max()


def test_local_patch_fit_multiplicative():
    p = fd.lognormal2d(16, n_stop=16)
    A = p.levels[0].A
    c = fd.parity_colour(16, 2, 1)
    full = O.fit_multiplicative(A, 1, 2, c)["lam"]
    loc = O.fit_local(A, 1, 2, [0, 77, 136, 255], mode="multiplicative", colours=c)
    for i, v in loc.items():
        for l in range(2):
            np.testing.assert_allclose(v[l], full[l][i], rtol=1e-11)


# ---------------------------------------------------------------------------
# Flexible CG (Krylov acceleration of the V-cycle)
# ---------------------------------------------------------------------------

def _textbook_pcg(A, Minv, b, iters):
    """Preconditioned CG in its textbook form (Hestenes-Stiefel with
    beta = (r_new, z_new) / (r_old, z_old)), one column."""
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    out = [x.copy()]
    for _ in range(iters):
        q = A @ p
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        z = Minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        out.append(x.copy())
    return out


def test_fcg_equals_textbook_pcg_for_fixed_spd_preconditioner():
    p = fd.poisson2d(16)
    A = p.levels[0].A
    d = A.diagonal()
    rng = stream(1, TEST, 40)
    b = rng.uniform(-1, 1, size=(A.shape[0], 1))
    ref = _textbook_pcg(A, lambda r: r / d, b[:, 0], 12)
    for k in (3, 7, 12):
        x, _ = O.fcg(A, lambda r: r / d[:, None], b, rtol=0.0, maxit=k)
        np.testing.assert_allclose(x[:, 0], ref[k], rtol=1e-9, atol=1e-12)


def test_fcg_exact_preconditioner_converges_in_one_step_and_cg_terminates():
    p = fd.poisson2d(8)
    A = p.levels[0].A
    Ad = A.toarray()
    rng = stream(1, TEST, 41)
    b = rng.uniform(-1, 1, size=(A.shape[0], 3))
    x, hist = O.fcg(A, lambda r: np.linalg.solve(Ad, r), b, rtol=1e-12, maxit=5)
    assert len(hist) == 2 and hist[-1] <= 1e-12
    np.testing.assert_allclose(x, np.linalg.solve(Ad, b), rtol=1e-10)
    # unpreconditioned CG terminates within the number of distinct eigenvalues
    _, h = O.fcg(A, lambda r: r, b, rtol=1e-10, maxit=64)
    ev = np.unique(np.round(np.linalg.eigvalsh(Ad), 9))
    assert len(h) - 1 <= len(ev)


def test_fcg_with_vcycle_beats_stationary_iteration():
    p = fd.interface3d(16, nrhs=2)
    sm = O.setup_hierarchy(p.levels, 3)
    _, h_ir = O.solve(p.levels, sm, p.rhs, rtol=1e-10, maxit=200)
    _, h_cg = O.fcg(p.levels[0].A, lambda r: O.vcycle(p.levels, sm, r), p.rhs, rtol=1e-10, maxit=200)
    assert h_cg[-1] <= 1e-10 and len(h_cg) < len(h_ir)


def test_gram_condition_closed_form():
    G = np.stack([np.diag([4.0, 2.0, 1.0]), np.diag([5.0, 1e-20, 0.5]),
                  np.zeros((3, 3))])
    Q, _ = np.linalg.qr(stream(1, TEST, 42).normal(size=(3, 3)))
    G[0] = Q @ G[0] @ Q.T
    c = O.gram_condition(G)
    np.testing.assert_allclose(c[:2], [4.0, 10.0], rtol=1e-12)   # 1e-20 is below the cut-off
    assert c[2] == 1.0


# ---------------------------------------------------------------------------
# GMRES (Sec. 3.1 driver): pinned to the minimisation property by brute force
# over an explicit Krylov basis, to closed forms and to finite termination.
# ---------------------------------------------------------------------------

def _convdiff(n, peclet=0.7):
    """Nonsymmetric tridiagonal test matrix (upwinded convection-diffusion)."""
    return sp.diags([np.full(n - 1, -1.0 - peclet), np.full(n, 2.0 + peclet), np.full(n - 1, -1.0)],
                    [-1, 0, 1]).tocsr()


def _krylov(Op, v, k):
    K = [v]
    for _ in range(k - 1):
        K.append(Op @ K[-1])
    return np.stack(K, axis=1)


def test_gmres_left_minimises_preconditioned_residual():
    n = 14
    A = _convdiff(n)
    rng = stream(1, TEST, 60)
    M = np.linalg.inv(A.toarray() + np.diag(rng.uniform(0.5, 1.5, n)))   # fixed, nonsymmetric
    b = rng.uniform(-1, 1, size=(n, 1))
    MA = M @ A.toarray()
    Mb = M @ b[:, 0]
    for k in range(1, 6):
        x, hist = O.gmres(A, lambda r: M @ r, b, restart=20, rtol=0.0, maxit=k)
        K = _krylov(MA, Mb, k)
        y = np.linalg.lstsq(MA @ K, Mb, rcond=None)[0]
        best = np.linalg.norm(Mb - MA @ K @ y)
        assert len(hist) == k + 1
        np.testing.assert_allclose(hist[-1] * np.linalg.norm(Mb), best, rtol=1e-8)
        np.testing.assert_allclose(x[:, 0], K @ y, rtol=1e-8, atol=1e-12)


def test_gmres_flexible_with_fixed_preconditioner_is_right_preconditioned_gmres():
    n = 14
    A = _convdiff(n, 1.3)
    rng = stream(1, TEST, 61)
    M = np.linalg.inv(A.toarray() + np.diag(rng.uniform(0.5, 1.5, n)))
    b = rng.uniform(-1, 1, size=(n, 1))
    AM = A.toarray() @ M
    for k in range(1, 6):
        x, hist = O.gmres(A, lambda r: M @ r, b, restart=20, rtol=0.0, maxit=k, flexible=True)
        K = _krylov(AM, b[:, 0], k)
        y = np.linalg.lstsq(AM @ K, b[:, 0], rcond=None)[0]
        best = np.linalg.norm(b[:, 0] - AM @ K @ y)
        np.testing.assert_allclose(hist[-1] * np.linalg.norm(b), best, rtol=1e-8)
        np.testing.assert_allclose(x[:, 0], M @ K @ y, rtol=1e-8, atol=1e-12)


def test_gmres_restart_one_is_the_minimal_residual_iteration():
    n = 12
    A = _convdiff(n)
    rng = stream(1, TEST, 62)
    b = rng.uniform(-1, 1, size=(n, 2))
    x, hist = O.gmres(A, lambda r: r, b, restart=1, rtol=0.0, maxit=5)
    xr = np.zeros_like(b)
    for _ in range(5):
        r = b - A @ xr
        Ar = A @ r
        xr = xr + np.sum(r * Ar, axis=0) / np.sum(Ar * Ar, axis=0) * r
    np.testing.assert_allclose(x, xr, rtol=1e-10)
    rn = np.linalg.norm(b - A @ xr, axis=0) / np.linalg.norm(b, axis=0)
    np.testing.assert_allclose(hist[-1], np.max(rn), rtol=1e-10)


def test_gmres_terminates_within_n_steps_and_columns_are_independent():
    n = 10
    A = _convdiff(n, 2.0)
    rng = stream(1, TEST, 63)
    b = rng.uniform(-1, 1, size=(n, 3))
    b[:, 2] = A @ np.ones(n)   # another right-hand side
    x, hist = O.gmres(A, lambda r: r, b, restart=30, rtol=1e-12, maxit=30)
    assert len(hist) - 1 <= n and hist[-1] <= 1e-12
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-9)
    # without a restart every column follows its own Krylov space
    for c in range(3):
        xc, _ = O.gmres(A, lambda r: r, b[:, c:c + 1], restart=30, rtol=0.0, maxit=4)
        xa, _ = O.gmres(A, lambda r: r, b, restart=30, rtol=0.0, maxit=4)
        np.testing.assert_allclose(xa[:, c], xc[:, 0], rtol=1e-12, atol=1e-15)


def test_gmres_with_vcycle_left_and_flexible():
    p = fd.interface3d(16, nrhs=2)
    sm = O.setup_hierarchy(p.levels, 3)
    pre = lambda r: O.vcycle(p.levels, sm, r, "FF")
    A = p.levels[0].A
    x, h = O.gmres(A, pre, p.rhs, rtol=1e-10, maxit=60)
    assert h[-1] <= 1e-10
    # the left residual is ||V(b - A x)||: the true residual follows within the V-cycle's conditioning
    r = p.rhs - A @ x
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)) <= 1e-8
    xf, hf = O.gmres(A, pre, p.rhs, rtol=1e-10, maxit=60, flexible=True)
    r = p.rhs - A @ xf
    np.testing.assert_allclose(hf[-1], np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(p.rhs, axis=0)), rtol=1e-9)
    assert hf[-1] <= 1e-10 and abs(len(hf) - len(h)) <= 2


# ---------------------------------------------------------------------------
# Sketched construction (Sec. 4): pinned to the exact fit (S = I), to brute-force
# least squares per block and to the invariances of the sketch.
# ---------------------------------------------------------------------------

def _small_interface():
    p = fd.interface3d(8, nrhs=1)
    return p.levels[0].A, p.levels[0].block_size


@pytest.mark.parametrize("mode", ["additive", "multiplicative"])
def test_sketch_with_identity_is_the_exact_fit(mode):
    if mode == "additive":
        A, n = _small_interface()
        colours = None
        exact = O.fit_additive(A, n, 3)
    else:
        A = fd.poisson2d(12).levels[0].A
        n = 1
        colours = O.greedy_colour(O.block_pattern(A, 1))
        exact = O.fit_multiplicative(A, n, 3, colours)
    sk = O.fit_sketched(A, n, 3, np.eye(A.shape[0]), mode=mode, colours=colours)
    for L1, L2 in zip(sk["lam"], exact["lam"]):
        np.testing.assert_allclose(L1, L2, rtol=1e-10, atol=1e-14)


def test_sketch_first_level_is_blockwise_least_squares():
    A, n = _small_interface()
    rng = stream(1, TEST, 70)
    S = rng.choice([-1.0, 1.0], size=(A.shape[0], 24))
    sk = O.fit_sketched(A, n, 1, S)
    w, At = O.prescale(A)
    M = At @ S
    for i in range(0, A.shape[0] // n, 7):
        r = slice(i * n, (i + 1) * n)
        # Lambda_i = argmin ||S_i - Lambda M_i||_F  <=>  M_i^T Lambda^T = S_i^T
        Lt = np.linalg.lstsq(M[r].T, S[r].T, rcond=None)[0].T
        np.testing.assert_allclose(sk["lam_tilde"][0][i], Lt, rtol=1e-9, atol=1e-12)


def test_sketch_is_invariant_to_scaling_sign_flips_and_column_order():
    A, n = _small_interface()
    rng = stream(1, TEST, 71)
    S = rng.choice([-1.0, 1.0], size=(A.shape[0], 16))
    ref = O.fit_sketched(A, n, 3, S)
    signs = rng.choice([-1.0, 1.0], size=16)
    perm = rng.permutation(16)
    for S2 in (3.7 * S, S * signs, S[:, perm]):
        got = O.fit_sketched(A, n, 3, S2)
        for L1, L2 in zip(got["lam"], ref["lam"]):
            np.testing.assert_allclose(L1, L2, rtol=1e-9, atol=1e-13)


def test_wider_sketch_approaches_the_exact_fit():
    A, n = _small_interface()
    exact = O.fit_additive(A, n, 2)
    rng = stream(1, TEST, 72)
    errs = []
    for s in (16, 64, 256):
        S = rng.choice([-1.0, 1.0], size=(A.shape[0], s))
        sk = O.fit_sketched(A, n, 2, S)
        errs.append(np.linalg.norm(sk["lam"][0] - exact["lam"][0]) / np.linalg.norm(exact["lam"][0]))
    assert errs[0] > errs[1] > errs[2], errs


# ---------------------------------------------------------------------------
# Stokes prescaling (Sec. 2.3.2) on the MAC grid: closed-form weights, the
# invariance that motivates it, inert slots, and convergence of the cascade.
# ---------------------------------------------------------------------------

from synth import stokes as _stokes


def test_stokes_prescaling_closed_form_on_the_mac_grid():
    n = 8
    h = 1.0 / n
    A = _stokes.operator(n)
    kind = _stokes.kinds(n)
    for norm, wp_int in (("l1", 1.0 / (2.0 * np.sqrt(2.0))), ("max", np.sqrt(2.0))):
        w, _ = O.prescale(A, kind, norm)
        # u at the face between cells (3, 4) and (4, 4): away from every wall
        u_int = 4 * (3 + n * 4) + 0
        np.testing.assert_allclose(w[u_int], h / np.sqrt(2.0), rtol=1e-14)
        # u next to the bottom wall (ghost mirror: diagonal 5/h^2, |row| 8/h^2)
        u_wall = 4 * (3 + n * 0) + 0
        np.testing.assert_allclose(w[u_wall], 2.0 * np.sqrt(2.0) * h / 5.0, rtol=1e-14)
        # pressure of a cell whose four faces are interior faces
        p_int = 4 * (4 + n * 4) + 2
        np.testing.assert_allclose(w[p_int], wp_int, rtol=1e-14)
        assert np.all(w[kind == 2] == 1.0)


def test_stokes_prescaling_is_invariant_to_viscosity_and_constraint_scale():
    A = _stokes.operator(8)
    kind = _stokes.kinds(8)
    vel = (kind != 1).astype(float)
    pre = (kind == 1).astype(float)
    Dv, Dp = sp.diags(vel), sp.diags(pre)
    V = Dv @ A @ Dv
    G = Dv @ A @ Dp
    Dm = Dp @ A @ Dv
    _, ref = O.prescale(A, kind, "l1")
    for c, a in ((1e-3, 1.0), (37.0, 1.0), (1.0, 1e2), (5.0, 1e-2)):
        # inert slots keep their unit diagonal
        Vc = c * V + (1.0 - c) * sp.diags((kind == 2).astype(float))
        A2 = (Vc + a * G + a * Dm).tocsr()
        _, got = O.prescale(A2, kind, "l1")
        np.testing.assert_allclose(got.toarray(), ref.toarray(), rtol=1e-12, atol=1e-14)


def test_inert_slots_decouple_in_the_fit():
    p = _stokes.mac2d(8)
    lv = p.levels[0]
    sm = O.fit_additive(lv.A, 4, 3, kind=lv.kind, norm="l1")
    L1 = sm["lam"][0]
    inert = np.flatnonzero(lv.kind == 2)
    for s in inert:
        b, r = divmod(int(s), 4)
        e = np.zeros(4)
        e[r] = 1.0
        np.testing.assert_allclose(L1[b][r], e, atol=1e-14)
        np.testing.assert_allclose(L1[b][:, r], e, atol=1e-14)


def test_stokes_cascade_converges_under_gmres():
    p = _stokes.mac2d(16)
    sm = O.setup_hierarchy(p.levels, 4, norm="l1")
    pre = lambda r: O.vcycle(p.levels, sm, r, "FF")
    x, h = O.gmres(p.levels[0].A, pre, p.rhs, restart=30, rtol=1e-10, maxit=60)
    assert h[-1] <= 1e-10 and O.rho_regression(h) < 0.2
    r = p.rhs - p.levels[0].A @ x
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.rhs)


# ---------------------------------------------------------------------------
# Overlapping-block cascades (Sec. 3.6.2)
# ---------------------------------------------------------------------------

def test_overlapping_with_a_partition_is_the_additive_cascade():
    p = fd.interface3d(8, nrhs=1)
    A, n = p.levels[0].A, 8
    nodes = np.arange(A.shape[0]).reshape(-1, n)
    a = O.fit_additive(A, n, 3)
    o = O.fit_overlapping(A, nodes, 3)
    for L1, L2 in zip(o["lam"], a["lam"]):
        np.testing.assert_allclose(L1, L2, rtol=1e-12, atol=1e-15)
    x0 = stream(1, TEST, 80).uniform(-1, 1, size=(A.shape[0], 2))
    b = stream(1, TEST, 81).uniform(-1, 1, size=(A.shape[0], 2))
    ya, yo = O.smooth(A, a, x0, b), O.smooth_overlapping(A, o, x0, b)
    assert np.linalg.norm(yo - ya) <= 1e-13 * np.linalg.norm(ya)


def test_overlapping_levels_are_blockwise_least_squares():
    """Vanka patches on a small MAC grid: every level's blocks against dense
    least squares on the explicitly formed replicated residual."""
    n = 4
    p = _stokes.mac2d(n)
    lv = p.levels[0]
    nodes = _stokes.vanka_nodes(n)
    sm = O.fit_overlapping(lv.A, nodes, 2, kind=lv.kind, norm="l1")
    w, At = O.prescale(lv.A, lv.kind, "l1")
    N = lv.A.shape[0]
    At = At.toarray()
    nblk, m = nodes.shape
    Th = np.zeros((nblk * m, N))
    for i in range(nblk):
        for s_ in range(m):
            if nodes[i, s_] >= 0:
                Th[i * m + s_, nodes[i, s_]] = 1.0
    theta = Th.sum(axis=0)
    E = np.eye(N)
    for ell in range(2):
        M, T = Th @ At @ E, Th @ E
        L = np.zeros((nblk, m, m))
        for i in range(nblk):
            r = slice(i * m, (i + 1) * m)
            # min ||T_i - Lambda M_i||_F  <=>  M_i^T Lambda^T = T_i^T (minimum norm)
            L[i] = np.linalg.lstsq(M[r].T, T[r].T, rcond=1e-13)[0].T
        np.testing.assert_allclose(sm["lam_tilde"][ell], L, rtol=1e-8, atol=1e-11)
        Lbig = np.zeros((nblk * m, nblk * m))
        for i in range(nblk):
            Lbig[i * m:(i + 1) * m, i * m:(i + 1) * m] = L[i]
        E = np.diag(1.0 / theta) @ Th.T @ (T - Lbig @ M)


def test_overlapping_identity_sketch_and_convergence():
    p = _stokes.mac2d(8)
    lv = p.levels[0]
    nodes = _stokes.vanka_nodes(8)
    ex = O.fit_overlapping(lv.A, nodes, 2, kind=lv.kind, norm="l1")
    sk = O.fit_overlapping(lv.A, nodes, 2, S=np.eye(lv.n), kind=lv.kind, norm="l1")
    for L1, L2 in zip(sk["lam"], ex["lam"]):
        np.testing.assert_allclose(L1, L2, rtol=1e-10, atol=1e-12)
    p = _stokes.mac2d(16)
    sm, m = [], 16
    for lv in p.levels[:-1]:
        sm.append(O.fit_overlapping(lv.A, _stokes.vanka_nodes(m), 2, kind=lv.kind, norm="l1"))
        m //= 2
    x, h = O.gmres(p.levels[0].A, lambda r: O.vcycle(p.levels, sm, r, "FF"), p.rhs, restart=30, rtol=1e-10,
                   maxit=60)
    assert h[-1] <= 1e-10 and O.rho_regression(h) < 0.15


# ---------------------------------------------------------------------------
# Stencil repetition (Sec. 4): translation classes of block neighbourhoods
# ---------------------------------------------------------------------------

def _disk_problem(n=48, bs=2, contrast=100.0):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    mu = np.where((X - 0.45) ** 2 + (Y - 0.55) ** 2 < 0.2 ** 2, contrast, 1.0)
    return fd.fv_hierarchy(mu, bs=bs, n_stop=n, order="lex")[0]


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_lattice_classes_constant_poisson_closed_forms(r):
    """5-point Dirichlet Poisson on a 16^2 grid: a cell's row differs from the
    bulk when it or a neighbour touches the boundary (cells 0, 1, n-2, n-1 of
    an axis), so the class of a cell at radius r is fixed by its distance to
    each side capped at r + 2: (2r + 5)^2 classes, and the bulk class is the
    (n - 4 - 2r)^2 cells with both coordinates in [2 + r, n - 3 - r]."""
    n = 16
    L = fd.poisson2d(n, n_stop=n).levels[0]
    coords = L.block_lattice()
    rep = O.lattice_classes(L.A, 1, coords, r)
    assert len(np.unique(rep)) == (2 * r + 5) ** 2
    inner = np.all((coords >= 2 + r) & (coords <= n - 3 - r), axis=1)
    assert inner.sum() == (n - 4 - 2 * r) ** 2
    assert len(np.unique(rep[inner])) == 1
    assert not np.any(rep[~inner] == rep[inner][0])
    # every representative is the smallest index of its class
    assert np.all(rep <= np.arange(len(rep))) and np.all(rep[rep] == rep)


def test_lattice_classes_fix_the_cascade_fit():
    """Blocks in one class at radius l - 1 get the same Lambda_l from the plain
    fit (the fit of a block reads the rows within l - 1 block layers, as the
    local-patch pin above fixes); classes at radius l - 2 do not suffice."""
    L = _disk_problem()
    coords = L.block_lattice()
    res = O.fit_additive(L.A, 4, 3)
    for ell in (1, 2, 3):
        lam = res["lam_tilde"][ell - 1]
        rep = O.lattice_classes(L.A, 4, coords, ell - 1)
        members = np.nonzero(rep != np.arange(len(rep)))[0]
        assert len(members) > 100
        scale = np.abs(lam).max()
        assert np.abs(lam[members] - lam[rep[members]]).max() <= 1e-12 * scale
        if ell > 1:
            short = O.lattice_classes(L.A, 4, coords, ell - 2)
            m2 = np.nonzero(short != np.arange(len(short)))[0]
            assert np.abs(lam[m2] - lam[short[m2]]).max() > 1e-8 * scale


def test_lattice_classes_independent_of_block_order():
    """Renumbering the blocks (with their lattice points) renumbers the classes."""
    L = fd.poisson2d(16, n_stop=16).levels[0]
    coords = L.block_lattice()
    B = coords.shape[0]
    perm = stream(0, TEST, 71).permutation(B)      # new index of old block i is perm[i]
    Pm = sp.csr_matrix((np.ones(B), (perm, np.arange(B))), shape=(B, B))
    A2 = (Pm @ L.A @ Pm.T).tocsr()
    c2 = np.empty_like(coords)
    c2[perm] = coords
    for r in (1, 3):
        rep = O.lattice_classes(L.A, 1, coords, r)
        rep2 = O.lattice_classes(A2, 1, c2, r)
        same = rep[:, None] == rep[None, :]
        same2 = rep2[perm][:, None] == rep2[perm][None, :]
        assert np.array_equal(same, same2)
