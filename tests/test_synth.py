"""Checks of the synthetic input generators (no solver arithmetic involved)."""
import pytest
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import fd


def test_fd_symmetric_and_row_sums():
    p = fd.poisson2d(16)
    for lv in p.levels:
        A = lv.A
        assert abs(A - A.T).max() == 0
        rs = np.asarray(A.sum(axis=1)).ravel()[lv.cells]     # indexed by cell coordinates
        assert np.abs(rs[1:-1, 1:-1]).max() < 1e-9 * A.max()   # interior rows sum to zero
        assert rs[0, 0] > 0                                      # Dirichlet boundary rows do not


def test_fd_second_order():
    errs = []
    for n in (16, 32, 64):
        lv = fd.poisson2d(n, n_stop=n).levels[0]
        x = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(x, x, indexing="ij")
        u = np.sin(np.pi * X) * np.sin(np.pi * Y)
        f = 2 * np.pi ** 2 * u
        idx = lv.cells
        rhs = np.empty(n * n)
        rhs[idx.ravel()] = f.ravel()
        uh = spla.spsolve(lv.A.tocsc(), rhs)
        ue = np.empty(n * n)
        ue[idx.ravel()] = u.ravel()
        errs.append(np.abs(uh - ue).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


def test_block_ordering_and_transfer():
    n, bs = 8, 2
    idx = fd.cell_order(n, 3, bs)
    assert sorted(idx.ravel().tolist()) == list(range(n ** 3))
    # cells of one block are contiguous
    assert set(idx[:2, :2, :2].ravel().tolist()) == set(range(8))
    P = fd.piecewise_constant_P(n, 3, bs, bs)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0)          # P 1 = 1
    assert np.all(np.asarray((P != 0).sum(axis=1)).ravel() == 1)
    assert np.all(np.asarray(P.sum(axis=0)).ravel() == 8)


def test_interface_problem():
    p = fd.interface3d(32, nrhs=3)
    c = np.array(p.meta["centre"])
    assert np.all((c >= 0.3) & (c <= 0.7))
    A = p.levels[0].A
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    assert A.diagonal().max() / A.diagonal().min() > 1e3       # high contrast present
    assert [lv.n for lv in p.levels] == [32 ** 3, 16 ** 3, 8 ** 3, 4 ** 3]
    assert p.rhs.shape == (32 ** 3, 3) and np.abs(p.rhs).max() <= 1


def test_batch_sizes():
    s = fd.batch_sizes(64)
    assert np.all(s % 16 == 0) and s.min() >= 64 and s.max() <= 512
    probs = fd.lognormal_batch(sizes=[64, 80])
    assert probs[1].levels[-1].n == 5 * 5            # 80 -> 40 -> 20 -> 10 -> 5 (odd)
    assert probs[0].levels[-1].n == 8 * 8            # 64 -> ... -> 8


def test_block_size_counts_unknowns_per_block():
    p = fd.interface3d(16, nrhs=1, bs=2)
    assert [lv.block_size for lv in p.levels] == [8, 8, 1]      # bottom level: no smoother
    z = np.ones((8, 8))
    assert [lv.block_size for lv in fd.fv_hierarchy(z, bs=2, n_stop=2, order="lex")] == [4, 4, 4]


def test_morton_numbering_makes_children_contiguous():
    for d, n in ((2, 32), (3, 16)):
        levels = fd.fv_hierarchy(np.ones((n,) * d), bs=2, n_stop=4)
        for lv in levels[:-1]:
            P = lv.P.tocsr()
            k = 2 ** d
            assert np.all(np.diff(P.indptr) == 1)
            np.testing.assert_array_equal(P.indices, np.arange(P.shape[0]) // k)
            assert lv.block_size == k
        # numbering is a permutation and the operator is the lexicographic one permuted
        lex = fd.fv_hierarchy(np.ones((n,) * d), bs=1, n_stop=n, order="lex")[0].A
        mor = levels[0]
        perm = np.empty(n ** d, dtype=np.int64)
        perm[mor.cells.ravel()] = fd.cell_order(n, d, 1).ravel()
        Pm = lex[perm][:, perm]
        assert abs(Pm - mor.A).max() == 0


def test_batch_concatenation_layout():
    """Stacked levels are block diagonal over the present systems (deepest
    first); systems that end on a level are its trailing direct segments; P
    is block diagonal over the continuing systems with empty direct rows."""
    import scipy.sparse as sp
    from synth.batch import concatenate
    sizes = [16, 32, 8, 24]
    probs = fd.lognormal_batch(len(sizes), nrhs=2, sizes=sizes, config_id=14)
    bt = concatenate(probs)
    nlev = [len(p.levels) for p in probs]
    assert [nlev[s] for s in bt.order] == sorted(nlev, reverse=True)
    for l, lv in enumerate(bt.levels):
        present = [s for s in bt.order if nlev[s] > l]
        ref = sp.block_diag([probs[s].levels[l].A for s in present], format="csr")
        assert (lv.A != ref).nnz == 0
        ends = [s for s in present if nlev[s] == l + 1]
        if ends:
            seg = np.asarray(lv.direct_seg)
            assert seg[-1] == lv.n and np.array_equal(np.diff(seg), [probs[s].levels[l].n for s in ends])
        else:
            assert lv.direct_seg is None
        if lv.P is not None:
            n_act = lv.n if lv.direct_seg is None else lv.direct_seg[0]
            assert lv.P.shape == (lv.n, bt.levels[l + 1].n)
            assert lv.P[n_act:].nnz == 0
    assert bt.levels[-1].direct_seg[0] == 0
    xs = [np.arange(p.n * 2, dtype=float).reshape(p.n, 2) + 1000 * i for i, p in enumerate(probs)]
    back = bt.split(bt.stack(xs))
    for a, b in zip(xs, back):
        np.testing.assert_array_equal(a, b)
    assert bt.sys_ptr[-1] == bt.levels[0].n and np.array_equal(bt.split(bt.rhs)[1], probs[1].rhs)


def test_q1_multiphase_generator():
    """Q1 FE: exact element stiffness, symmetric positive definite global
    matrix, zero row sums away from the Dirichlet faces, Galerkin coarse
    operator equal to the rediscretisation on the coarse mesh, phases at the
    1/3 and 2/3 quantiles."""
    from synth import fe
    K = fe.q1_stiffness()
    np.testing.assert_allclose(K.sum(axis=1), 0, atol=1e-15)
    assert K[0, 0] == pytest.approx(1.0 / 3.0)       # diagonal of the unit-cube Q1 Laplacian
    n = 8
    mu = fe.grf_phases(n, config_id=99)
    assert sorted(np.unique(mu)) == [1.0, 1e3, 1e6]
    assert all(abs(np.mean(mu == v) - 1 / 3) < 0.01 for v in (1.0, 1e3, 1e6))
    A = fe.assemble(mu)
    assert abs(A - A.T).max() < 1e-9 * abs(A).max()
    order = fe.node_order(n)
    kk, jj, ii = np.indices((n, n, n))
    interior = (ii < n - 1) & (jj < n - 1) & (kk < n - 1)     # no Dirichlet neighbour
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.all(np.abs(rs[order[interior]]) <= 1e-9 * abs(A).max())
    assert np.all(rs[order[~interior]] > 0)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    for m in (8, 12):
        P = fe.trilinear_P(m)
        Ac = P.T @ fe.assemble(np.ones((m,) * 3)) @ P
        assert abs(Ac - fe.assemble(np.ones((m // 2,) * 3))).max() < 1e-14
    lv = fe.galerkin_hierarchy(A, n, n_stop=2)
    assert [l.n for l in lv] == [512, 64, 8] and all(l.block_size == 8 for l in lv)


def test_sipg_q3_generator():
    """SIPG Q3 on the jittered mesh: symmetric, O(h^4) L2 convergence for a
    manufactured solution, exact child projections (sum of M_c^T M_c = 4 I,
    constants map to constants), proper 4-colouring of the block graph."""
    import scipy.sparse.linalg as spla
    from numpy.polynomial import legendre as npl
    from synth import dg
    f = lambda x, y: 2 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y)
    u = lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y)
    errs = []
    for n in (4, 8, 16):
        v = dg.jittered_vertices(n)
        A, b = dg.assemble(v, rhs_fn=f)
        A = A.tocsr()
        assert abs(A - A.T).max() < 1e-12 * abs(A).max()
        x = spla.spsolve(A.tocsc(), b)
        gq, gw = npl.leggauss(6)
        xi, eta = np.meshgrid(gq, gq, indexing="xy")
        X, J = dg._geometry(dg._corners(v, n), xi.ravel(), eta.ravel())
        wdet = np.linalg.det(J) * np.outer(gw, gw).ravel()
        val, _ = dg.basis2d(xi.ravel(), eta.ravel())
        uh = x.reshape(-1, 16) @ val.T
        errs.append(np.sqrt((wdet * (uh - u(X[..., 0], X[..., 1])) ** 2).sum()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.7), rates
    M = dg.child_matrices()
    np.testing.assert_allclose(sum(m.T @ m for m in M), 4 * np.eye(16), atol=1e-13)
    np.testing.assert_allclose(M[:, 0, 0], 1.0, rtol=1e-14)
    np.testing.assert_allclose(M[:, 1:, 0], 0.0, atol=1e-14)
    p = dg.sipg_q3(8)
    assert [l.n for l in p.levels] == [1024, 256] and p.levels[0].block_size == 16
    Ab = abs(p.levels[0].A).tocsr()
    B = sp.csr_matrix((np.ones(Ab.nnz), Ab.indices // 16, Ab.indptr), shape=(1024, 64))
    col = p.levels[0].colour
    for i in range(64):
        nbrs = np.unique(B[i * 16:(i + 1) * 16].indices)
        assert all(col[j] != col[i] for j in nbrs if j != i)


def test_mac_stokes_operator_and_hierarchy():
    from synth import stokes
    p = stokes.mac2d(16)
    for lv in p.levels:
        A = lv.A
        assert abs(A - A.T).max() == 0.0
        assert lv.block_size == 4 and len(lv.kind) == A.shape[0]
        # inert slots: unit diagonal, nothing else in their row
        for s in np.flatnonzero(lv.kind == 2):
            row = A.getrow(s)
            assert row.nnz == 1 and row.indices[0] == s and row.data[0] == 1.0
        # constraint rows have a zero diagonal and couple to velocities only
        for s in np.flatnonzero(lv.kind == 1)[:20]:
            row = A.getrow(s)
            assert A[s, s] == 0.0 and np.all(lv.kind[row.indices] == 0)
    d = np.linalg.eigvalsh(p.levels[-1].A.toarray())
    assert np.min(np.abs(d)) > 1e-8 and (d < 0).sum() == (p.levels[-1].kind == 1).sum()
    # the interpolation reproduces a constant pressure away from the pinned cell
    lv = p.levels[0]
    pc = np.where(p.levels[1].kind == 1, 1.0, 0.0)
    pf = lv.P @ pc
    fine_p = np.flatnonzero(lv.kind == 1)
    assert np.mean(pf[fine_p] == 1.0) > 0.9
