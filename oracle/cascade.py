"""Plain FP64 CPU oracle for cascading-smoother multigrid (Saye, "Cascading
Smoothers for Multigrid", arXiv 2606.12577).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the HIP library.

Every function writes out the definition it implements, in the paper's
notation, with dense or scipy.sparse library products as the only building
blocks.  Nothing is blocked, fused or reordered beyond the definitions.

Conventions
-----------
* A is a scalar CSR matrix; block i owns scalar rows [i*n, (i+1)*n).
* A block-diagonal Lambda is stored as an array of shape (B, n, n).
* Vectors are (N, R) arrays: R right-hand sides side by side.
* Structural block patterns (which blocks of E may be non-zero) are kept as
  boolean B x B CSR matrices; numerical cancellation never removes a block
  from a structural pattern.

Readings taken where the paper leaves a choice open
---------------------------------------------------
* Least squares per block (Sec. 2.1, Alg. 2): the normal equations
  Lambda_i G_i = H_i with G_i = M_i M_i^T, H_i = E_i M_i^T, M = A E, solved
  as the minimum-norm least-squares solution (pseudo-inverse of G_i with a
  relative cut-off of 1e-13; identical to H_i G_i^{-1} whenever G_i is SPD).
* Prescaling (Sec. 2.3, elliptic): W = diag(a_kk^{-1/2}) over the scalar
  diagonal of A.
* Multiplicative construction (Sec. 2.2): every block of colour k is fitted
  from the same E (the state before the colour-k update), then the colour-k
  rows are updated; colours are swept in ascending id.
* Reverse application (Sec. 2.4): the cascade is applied in the order
  Lambda_nu^T, ..., Lambda_1^T (the index printed in the reverse formulas is
  off by two; the supplementary symmetry section fixes this order).
* Truncation (Alg. 2, optional step): keep the alpha blocks of largest
  Frobenius norm in each updated block row of E; ties go to the lower block
  column.
* Regularised fit (an extension, not in the paper; ridge = 0 is the paper's
  fit): Lambda_i (G_i + ridge tr(G_i)/n I) = H_i, the Tikhonov-regularised
  least squares, used to fit cascades that are applied in reduced precision.
"""
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

PINV_RCOND = 1e-13


# ---------------------------------------------------------------------------
# Block helpers (pure bookkeeping)
# ---------------------------------------------------------------------------

def aggregator(N: int, n: int) -> sp.csr_matrix:
    """B x N 0/1 matrix summing the n scalar rows of each block."""
    return sp.csr_matrix((np.ones(N), (np.arange(N) // n, np.arange(N))), shape=(N // n, N))


def block_pattern(X: sp.spmatrix, n: int) -> sp.csr_matrix:
    """Structural block pattern of X (every stored entry counts)."""
    Xs = sp.csr_matrix(X, copy=True)
    Xs.data[:] = 1.0
    Q = aggregator(X.shape[0], n)
    P = (Q @ Xs @ Q.T).tocsr()
    P.data[:] = 1.0
    P.sort_indices()
    return P.astype(bool)


def pattern_product(P1: sp.csr_matrix, P2: sp.csr_matrix) -> sp.csr_matrix:
    """Structural pattern of a product of two block-sparse matrices."""
    R = (P1.astype(np.float64) @ P2.astype(np.float64)).tocsr()
    R.data[:] = 1.0
    R.sort_indices()
    return R.astype(bool)


def blockdiag(blocks: np.ndarray) -> sp.csr_matrix:
    B, n, _ = blocks.shape
    return sp.bsr_matrix((blocks, np.arange(B), np.arange(B + 1)), shape=(B * n, B * n)).tocsr()


def blockdiag_of_product(X: sp.spmatrix, Y: sp.spmatrix, n: int) -> np.ndarray:
    """Z[i] = X_i Y_i^T, X_i being the n x N block row i of X."""
    X = sp.csr_matrix(X)
    Y = sp.csr_matrix(Y)
    B = X.shape[0] // n
    Z = np.empty((B, n, n))
    for r in range(n):
        Xr = X[r::n]
        for s in range(n):
            Z[:, r, s] = np.asarray(Xr.multiply(Y[s::n]).sum(axis=1)).ravel()
    return Z


def block_rows(blocks: Sequence[int], n: int) -> np.ndarray:
    b = np.asarray(blocks, dtype=np.int64)
    return (b[:, None] * n + np.arange(n)[None, :]).ravel()


# ---------------------------------------------------------------------------
# Setup (Sec. 2.1-2.3, Alg. 2, supplementary multicoloured algorithm)
# ---------------------------------------------------------------------------

def prescale(A: sp.spmatrix, kind: Optional[np.ndarray] = None, norm: str = "max"):
    """Symmetric diagonal prescaling W, returns (w, W A W) (Sec. 2.3).

    kind None (elliptic, Sec. 2.3.1): W = diag(A_kk^{-1/2}).
    kind given (Stokes, Sec. 2.3.2): per unknown 0 velocity, 1 pressure (2: an
    inert unknown, scaled as a velocity).  With the viscous block V = A[vel, vel]
    and the constraint block D = A[pres, vel]:
      velocity: w_i chosen so that (W V W)_ii = ||V_i,:||_1 / V_ii, i.e.
                w_i = sqrt(||V_i,:||_1) / V_ii;
      pressure: every row of diag(w_p) D diag(w_u) has unit max-norm
                (norm "max") or unit 1-norm (norm "l1", the MAC variant)."""
    A = sp.csr_matrix(A)
    if kind is None:
        d = A.diagonal()
        if np.any(d <= 0):
            raise ValueError("elliptic prescaling needs a positive diagonal")
        w = 1.0 / np.sqrt(d)
    else:
        kind = np.asarray(kind)
        vel = kind != 1
        pre = kind == 1
        V = A[vel][:, vel]
        dv = V.diagonal()
        if np.any(dv <= 0):
            raise ValueError("Stokes prescaling needs a positive viscous diagonal")
        l1 = np.asarray(abs(V).sum(axis=1)).ravel()
        w = np.empty(A.shape[0])
        w[vel] = np.sqrt(l1) / dv
        D = sp.csr_matrix(A[pre][:, vel] @ sp.diags(w[vel]))
        if norm == "max":
            m = np.asarray(abs(D).max(axis=1).todense()).ravel()
        elif norm == "l1":
            m = np.asarray(abs(D).sum(axis=1)).ravel()
        else:
            raise ValueError(norm)
        if np.any(m <= 0):
            raise ValueError("a constraint row couples to no velocity")
        w[pre] = 1.0 / m
    W = sp.diags(w)
    return w, (W @ A @ W).tocsr()


def regularised_gram(G: np.ndarray, ridge: float) -> np.ndarray:
    """G_i + tau_i I with tau_i = ridge * trace(G_i) / n: the normal-equation
    matrices of the Tikhonov-regularised fit (ridge = 0: G itself)."""
    if not ridge:
        return G
    n = G.shape[1]
    tau = ridge * np.trace(G, axis1=1, axis2=2) / n
    return G + tau[:, None, None] * np.eye(n)[None, :, :]


def least_squares_blocks(H: np.ndarray, G: np.ndarray, ridge: float = 0.0) -> np.ndarray:
    """Minimum-norm solution Lambda_i of Lambda_i M_i = E_i via its normal
    equations Lambda_i G_i = H_i (Alg. 2, least-squares step).

    ridge > 0 (a precision-aware reading, not in the paper): minimise
    ||E_i - Lambda_i M_i||_F^2 + tau_i ||Lambda_i||_F^2, tau_i = ridge tr(G_i)/n,
    i.e. Lambda_i (G_i + tau_i I) = H_i.  It bounds the blocks whose fit
    amplifies the nearly dependent directions of M_i, which a reduced-precision
    application would otherwise turn into large errors."""
    Gr = regularised_gram(G, ridge)
    out = np.empty_like(H)
    for i in range(G.shape[0]):
        out[i] = H[i] @ np.linalg.pinv(Gr[i], rcond=PINV_RCOND, hermitian=True)
    return out


def gram_condition(G: np.ndarray) -> np.ndarray:
    """Spectral condition number of every G_i restricted to the eigenvalues the
    least-squares step keeps (those above PINV_RCOND times the largest).  The
    solve of Lambda_i G_i = H_i loses about that factor of relative accuracy,
    which bounds how closely two implementations can agree on Lambda_i."""
    out = np.empty(G.shape[0])
    for i in range(G.shape[0]):
        ev = np.linalg.eigvalsh(G[i])
        top = ev[-1]
        kept = ev[ev > PINV_RCOND * top]
        out[i] = top / kept[0] if top > 0 else 1.0
    return out


def truncate_rows(E: sp.csr_matrix, Epat: sp.csr_matrix, n: int, alpha: int,
                  rows: np.ndarray):
    """Keep the alpha blocks of largest Frobenius norm in the given block rows of
    E (ties -> lower block column); other rows are left as they are."""
    Q = aggregator(E.shape[0], n)
    S = (Q @ E.multiply(E) @ Q.T).tocsr()
    Epat = Epat.tocsr()
    keep_r, keep_c = [], []
    rowset = np.zeros(Epat.shape[0], dtype=bool)
    rowset[rows] = True
    for i in range(Epat.shape[0]):
        cols = Epat.indices[Epat.indptr[i]:Epat.indptr[i + 1]]
        if rowset[i] and len(cols) > alpha:
            norms = np.sqrt(np.asarray(S[i, cols].todense()).ravel())
            order = sorted(range(len(cols)), key=lambda t: (-norms[t], cols[t]))
            cols = np.sort(cols[order[:alpha]])
        keep_r.append(np.full(len(cols), i))
        keep_c.append(cols)
    r = np.concatenate(keep_r)
    c = np.concatenate(keep_c)
    K = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=Epat.shape)
    K.sort_indices()
    mask = (Q.T @ K @ Q).tocsr()
    return E.multiply(mask).tocsr(), K.astype(bool)


def unscale(lam_t: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Lambda <- W Lambda W (Alg. 2, final step)."""
    B, n, _ = lam_t.shape
    wb = w.reshape(B, n)
    return wb[:, :, None] * lam_t * wb[:, None, :]


def fit_additive(A: sp.spmatrix, n: int, depth: int, alpha: Optional[int] = None,
                 kind: Optional[np.ndarray] = None, norm: str = "max", ridge: float = 0.0) -> Dict:
    """Depth-nu additive cascade (Sec. 2.1, Alg. 2).

    Lambda_l = argmin_{Lambda block-diagonal} ||(I - Lambda A~) E_{l-1}||_F,
    E_l = (I - Lambda_l A~) E_{l-1}, E_0 = I, on the prescaled A~ = W A W.
    Returns lam (unscaled, list over l), lam_tilde, w, and the structural block
    patterns of E_0 .. E_{nu-1}."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    B = N // n
    w, At = prescale(A, kind, norm)
    Apat = block_pattern(At, n)
    E = sp.identity(N, format="csr")
    Epat = sp.identity(B, format="csr", dtype=bool)
    lam_t, pats = [], [Epat]
    cond = []
    for ell in range(1, depth + 1):
        M = (At @ E).tocsr()
        G = blockdiag_of_product(M, M, n)
        H = blockdiag_of_product(E, M, n)
        Lt = least_squares_blocks(H, G, ridge)
        cond.append(gram_condition(regularised_gram(G, ridge)))
        lam_t.append(Lt)
        if ell < depth:
            E = (E - blockdiag(Lt) @ M).tocsr()
            Epat = pattern_product(Apat, Epat)
            if alpha:
                E, Epat = truncate_rows(E, Epat, n, alpha, np.arange(B))
            pats.append(Epat)
    return dict(lam=[unscale(L, w) for L in lam_t], lam_tilde=lam_t, w=w, patterns=pats,
                colours=None, gram_cond=cond)


def fit_multiplicative(A: sp.spmatrix, n: int, depth: int, colours: np.ndarray,
                       alpha: Optional[int] = None, kind: Optional[np.ndarray] = None, norm: str = "max",
                       ridge: float = 0.0) -> Dict:
    """Depth-nu multicoloured cascade (Sec. 2.2).

    For l = 1..nu and colours k in ascending order,
    Lambda_{l,k} = argmin_{Lambda in D_k} ||(I - Lambda A~) E_{l,k-1}||_F and
    E_{l,k} = (I - Lambda_{l,k} A~) E_{l,k-1}, continuing E across levels.
    lam[l][i] holds the block of Lambda_{l, colour(i)}.  The returned
    patterns are those of E after every colour step, in sweep order."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    B = N // n
    colours = np.asarray(colours, dtype=np.int64)
    chi = int(colours.max()) + 1
    w, At = prescale(A, kind, norm)
    Apat = block_pattern(At, n)
    E = sp.identity(N, format="csr")
    Epat = sp.identity(B, format="csr", dtype=bool)
    lam_t = [np.zeros((B, n, n)) for _ in range(depth)]
    cond = [np.ones(B) for _ in range(depth)]
    pats = [Epat]
    for ell in range(1, depth + 1):
        for k in range(chi):
            blocks = np.flatnonzero(colours == k)
            if len(blocks) == 0:
                continue
            sel = block_rows(blocks, n)
            M = (At @ E).tocsr()
            Mk, Ek = M[sel], E[sel]
            G = blockdiag_of_product(Mk, Mk, n)
            H = blockdiag_of_product(Ek, Mk, n)
            Lt = least_squares_blocks(H, G, ridge)
            lam_t[ell - 1][blocks] = Lt
            cond[ell - 1][blocks] = gram_condition(regularised_gram(G, ridge))
            if ell < depth or k < chi - 1:
                D = np.zeros((B, n, n))
                D[blocks] = Lt
                E = (E - blockdiag(D) @ M).tocsr()
                grown = pattern_product(Apat, Epat)
                mask = sp.diags((colours == k).astype(np.float64))
                keep = sp.diags((colours != k).astype(np.float64))
                Epat = (keep @ Epat.astype(np.float64) + mask @ grown.astype(np.float64)).tocsr()
                Epat.eliminate_zeros()
                Epat.data[:] = 1.0
                Epat.sort_indices()
                Epat = Epat.astype(bool)
                if alpha:
                    E, Epat = truncate_rows(E, Epat, n, alpha, blocks)
                pats.append(Epat)
    return dict(lam=[unscale(L, w) for L in lam_t], lam_tilde=lam_t, w=w, patterns=pats,
                colours=colours.astype(np.int32), gram_cond=cond)


def fit_sketched(A: sp.spmatrix, n: int, depth: int, S: np.ndarray, mode: str = "additive",
                 colours: Optional[np.ndarray] = None, kind: Optional[np.ndarray] = None,
                 norm: str = "max") -> Dict:
    """Sketched cascade construction (Sec. 4, Concluding Remarks, proposed there as
    future work).

    The square residual E_{l-1} is replaced by the tall-and-narrow sketch
    T_{l-1} = E_{l-1} S, S an N x s matrix of random error modes (given):
        Lambda_l = argmin_{Lambda block-diagonal} ||(I - Lambda A~) T_{l-1}||_F,
        T_l = (I - Lambda_l A~) T_{l-1},  T_0 = S,
    on the prescaled A~ = W A W, block by block through the normal equations
    Lambda_i G_i = H_i with M = A~ T, G_i = M_i M_i^T, H_i = T_i M_i^T (the
    same minimum-norm solve as the exact fit).  With S = I it is the exact fit.
    Multiplicative: the blocks of colour k are fitted from the current T, then
    their rows of T are updated, colours ascending (Sec. 2.2)."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    B = N // n
    w, At = prescale(A, kind, norm)
    T = np.array(S, dtype=np.float64, copy=True)
    s = T.shape[1]
    if mode == "additive":
        groups = [np.arange(B)]
    elif mode == "multiplicative":
        colours = np.asarray(colours, dtype=np.int64)
        groups = [np.flatnonzero(colours == k) for k in range(int(colours.max()) + 1)]
    else:
        raise ValueError(mode)
    lam_t = [np.zeros((B, n, n)) for _ in range(depth)]
    cond = [np.ones(B) for _ in range(depth)]
    for ell in range(1, depth + 1):
        for blocks in groups:
            if len(blocks) == 0:
                continue
            M = At @ T
            rows = block_rows(blocks, n)
            Mb = M[rows].reshape(len(blocks), n, s)
            Tb = T[rows].reshape(len(blocks), n, s)
            G = Mb @ Mb.transpose(0, 2, 1)
            H = Tb @ Mb.transpose(0, 2, 1)
            Lt = least_squares_blocks(H, G)
            lam_t[ell - 1][blocks] = Lt
            cond[ell - 1][blocks] = gram_condition(G)
            T[rows] = (Tb - Lt @ Mb).reshape(-1, s)
    return dict(lam=[unscale(L, w) for L in lam_t], lam_tilde=lam_t, w=w,
                colours=None if mode == "additive" else colours.astype(np.int32), gram_cond=cond)


def replication(nodes: np.ndarray, N: int):
    """Theta (Sec. 3.6.2): the tall binary matrix that copies nodal values into
    the slots of overlapping blocks (nodes[i][s] = node of slot s of block i,
    -1 for an unused slot, which gets a zero row), and theta = its column sums,
    the multiplicity of every node."""
    nodes = np.asarray(nodes)
    nblk, m = nodes.shape
    r = np.flatnonzero(nodes.ravel() >= 0)
    Th = sp.csr_matrix((np.ones(len(r)), (r, nodes.ravel()[r])), shape=(nblk * m, N))
    theta = np.asarray(Th.sum(axis=0)).ravel()
    return Th, theta


def fit_overlapping(A: sp.spmatrix, nodes: np.ndarray, depth: int, S: Optional[np.ndarray] = None,
                    kind: Optional[np.ndarray] = None, norm: str = "max") -> Dict:
    """Overlapping-block additive cascade (Sec. 3.6.2), on the prescaled A~:
        Lambda_l = argmin_{Lambda block-diagonal over the slots}
                   ||(Theta - Lambda Theta A~) E_{l-1}||_F,
        E_l = diag(theta)^{-1} Theta^T (Theta - Lambda_l Theta A~) E_{l-1},
    E_0 = I, or E_0 = S for the sketched form (Sec. 4).  Blockwise through the
    normal equations Lambda_i G_i = H_i, G_i = M_i M_i^T, H_i = T_i M_i^T with
    M = Theta A~ E and T = Theta E (unused slots: zero rows, and the
    minimum-norm solution leaves their rows and columns zero).  Every node must
    lie in some block.  Unscaled: Lambda_i <- W_i Lambda~_i W_i with W_i the
    weights of the block's nodes.  Returns lam[l] of shape (nblk, m, m)."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    nodes = np.asarray(nodes)
    nblk, m = nodes.shape
    w, At = prescale(A, kind, norm)
    Th, theta = replication(nodes, N)
    if np.any(theta == 0):
        raise ValueError("every node must belong to a block")
    Dinv = sp.diags(1.0 / theta)
    E = sp.identity(N, format="csr") if S is None else np.array(S, dtype=np.float64)
    lam_t, cond = [], []
    for ell in range(1, depth + 1):
        M = Th @ (At @ E)
        T = Th @ E
        if sp.issparse(M):
            G = blockdiag_of_product(M, M, m)
            H = blockdiag_of_product(T, M, m)
        else:
            Mb = M.reshape(nblk, m, -1)
            Tb = T.reshape(nblk, m, -1)
            G = Mb @ Mb.transpose(0, 2, 1)
            H = Tb @ Mb.transpose(0, 2, 1)
        Lt = least_squares_blocks(H, G)
        lam_t.append(Lt)
        cond.append(gram_condition(G))
        if ell < depth:
            E = Dinv @ (Th.T @ (T - blockdiag(Lt) @ M))
            if sp.issparse(E):
                E = sp.csr_matrix(E)
    wr = (Th @ w).reshape(nblk, m)
    lam = [wr[:, :, None] * L * wr[:, None, :] for L in lam_t]
    return dict(lam=lam, lam_tilde=lam_t, w=w, nodes=nodes, theta=theta, gram_cond=cond)


def smooth_overlapping(A: sp.spmatrix, sm: Dict, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One forward application of an overlapping-block additive cascade
    (Sec. 3.6.2): x <- x - diag(theta)^{-1} Theta^T Lambda_l Theta (A x - b),
    l = 1..nu."""
    Th, theta = replication(sm["nodes"], A.shape[0])
    Dinv = sp.diags(1.0 / theta)
    for L in sm["lam"]:
        x = x - Dinv @ (Th.T @ (blockdiag(L) @ (Th @ (A @ x - b))))
    return x


def fit(A, n, depth, mode="additive", colours=None, alpha=None, kind=None, norm="max", ridge=0.0) -> Dict:
    if mode == "additive":
        return fit_additive(A, n, depth, alpha, kind, norm, ridge)
    if mode == "multiplicative":
        return fit_multiplicative(A, n, depth, colours, alpha, kind, norm, ridge)
    raise ValueError(mode)


def jacobi_smoother(A: sp.spmatrix, n: int, depth: int, omega: float = 1.0) -> Dict:
    """Reference smoother: every Lambda_l = omega * blockdiag(A)^{-1} (Sec. 2.1:
    nu steps of damped block Jacobi / block Gauss-Seidel)."""
    A = sp.csr_matrix(A)
    B = A.shape[0] // n
    D = np.empty((B, n, n))
    for i in range(B):
        D[i] = np.linalg.inv(A[i * n:(i + 1) * n, i * n:(i + 1) * n].toarray())
    return dict(lam=[omega * D for _ in range(depth)], colours=None)


def greedy_colour(Apat: sp.csr_matrix) -> np.ndarray:
    """Colour blocks in index order, each with the smallest colour not used by
    an already-coloured neighbour (a proper colouring of the block graph)."""
    Apat = sp.csr_matrix(Apat)
    B = Apat.shape[0]
    c = np.full(B, -1, dtype=np.int64)
    for i in range(B):
        used = {c[j] for j in Apat.indices[Apat.indptr[i]:Apat.indptr[i + 1]] if j < i}
        k = 0
        while k in used:
            k += 1
        c[i] = k
    return c.astype(np.int32)


def is_proper_colouring(Apat: sp.csr_matrix, colours: np.ndarray) -> bool:
    C = sp.coo_matrix(Apat)
    off = C.row != C.col
    return bool(np.all(colours[C.row[off]] != colours[C.col[off]]))


# ---------------------------------------------------------------------------
# Application (Sec. 2.1 / 2.2 forward, Sec. 2.4 reverse)
# ---------------------------------------------------------------------------

def smooth(A: sp.spmatrix, sm: Dict, x: np.ndarray, b: np.ndarray, reverse: bool = False) -> np.ndarray:
    """One application of a cascading smoother.

    additive forward:  x <- x - Lambda_l (A x - b),    l = 1..nu
    additive reverse:  x <- x - Lambda_l^T (A x - b),  l = nu..1
    multiplicative: the same over the flattened sequence (l, k), k = 1..chi,
    with Lambda_{l,k} zero outside colour k; reverse runs it backwards."""
    lam = sm["lam"]
    colours = sm.get("colours")
    depth = len(lam)
    if colours is None:
        seq = [(l, None) for l in range(depth)]
    else:
        chi = int(np.max(colours)) + 1
        seq = [(l, k) for l in range(depth) for k in range(chi)]
    if reverse:
        seq = seq[::-1]
    for l, k in seq:
        blocks = lam[l] if k is None else lam[l] * (colours == k)[:, None, None]
        L = blockdiag(blocks)
        if reverse:
            L = L.T
        x = x - L @ (A @ x - b)
    return x


def setup_hierarchy(levels, depth: int, mode: str = "additive", alpha=None, norm: str = "max",
                    ridge: float = 0.0) -> List[Dict]:
    """Fit a cascade on every level except the coarsest (Sec. 2.5); a level
    with a `kind` array (velocity / pressure per unknown) is prescaled as a
    Stokes problem (Sec. 2.3.2) with the given constraint-row norm."""
    out = []
    for lv in levels[:-1]:
        colours = lv.colour
        if mode == "multiplicative" and colours is None:
            colours = greedy_colour(block_pattern(lv.A, lv.block_size))
        out.append(fit(lv.A, lv.block_size, depth, mode, colours, alpha, getattr(lv, "kind", None), norm, ridge))
    return out


def vcycle(levels, smoothers: List[Dict], b: np.ndarray, order: str = "RF",
           npre: int = 1, npost: int = 1, lvl: int = 0) -> np.ndarray:
    """Alg. 1 applied to right-hand side b with a zero initial guess.

    Pre-smoother: reverse application for RF, forward for FF; post-smoother:
    forward.  Restriction r_scale * P^T, correction x <- x - P x_c, and a dense
    direct solve on the bottom level."""
    lv = levels[lvl]
    if lvl == len(levels) - 1:
        return np.linalg.solve(lv.A.toarray(), b)
    x = np.zeros_like(b)
    sm = smoothers[lvl]
    if "nodes" in sm:        # overlapping blocks: forward applications only (FF)
        if order != "FF":
            raise ValueError("overlapping-block cascades are applied forward (FF)")
        for _ in range(npre):
            x = smooth_overlapping(lv.A, sm, x, b)
        rc = lv.r_scale * (lv.P.T @ (lv.A @ x - b))
        xc = vcycle(levels, smoothers, rc, order, npre, npost, lvl + 1)
        x = x - lv.P @ xc
        for _ in range(npost):
            x = smooth_overlapping(lv.A, sm, x, b)
        return x
    for _ in range(npre):
        x = smooth(lv.A, smoothers[lvl], x, b, reverse=(order == "RF"))
    rc = lv.r_scale * (lv.P.T @ (lv.A @ x - b))
    xc = vcycle(levels, smoothers, rc, order, npre, npost, lvl + 1)
    x = x - lv.P @ xc
    for _ in range(npost):
        x = smooth(lv.A, smoothers[lvl], x, b, reverse=False)
    return x


def solve(levels, smoothers, b: np.ndarray, rtol: float = 1e-10, maxit: int = 100,
          order: str = "RF", npre: int = 1, npost: int = 1):
    """Stationary V-cycle iteration (defect correction) in FP64:
    x_0 = 0; r = b - A x; stop when max_j ||r_j|| <= rtol ||b_j||; x += V r.
    Returns x and the history of max_j ||r_j|| / ||b_j||."""
    A = levels[0].A
    x = np.zeros_like(b)
    bn = np.linalg.norm(b, axis=0)
    hist = []
    for it in range(maxit + 1):
        r = b - A @ x
        rel = float(np.max(np.linalg.norm(r, axis=0) / bn))
        hist.append(rel)
        if rel <= rtol or it == maxit:
            break
        x = x + vcycle(levels, smoothers, r, order, npre, npost)
    return x, hist


def fcg(A, precond, b: np.ndarray, rtol: float = 1e-10, maxit: int = 100):
    """Flexible conjugate gradients with one-vector truncation (FCG(1)): the
    new direction is the preconditioned residual minus its A-projection on
    the previous direction.  Independent scalars per column of b.
        x = 0, r = b;  z = M(r);  p = z - (z, A p_old)/(p_old, A p_old) p_old;
        alpha = (p, r)/(p, A p);  x += alpha p;  r -= alpha A p.
    With a fixed symmetric positive definite M this is preconditioned CG.
    Returns x and the history of max_j ||r_j|| / ||b_j||."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b, axis=0)
    hist = [float(np.max(np.linalg.norm(r, axis=0) / bn))]
    p_old = q_old = None
    for it in range(maxit):
        if hist[-1] <= rtol:
            break
        z = precond(r)
        if p_old is None:
            p = z
        else:
            beta = -np.sum(z * q_old, axis=0) / np.sum(p_old * q_old, axis=0)
            p = z + beta * p_old
        q = A @ p
        alpha = np.sum(p * r, axis=0) / np.sum(p * q, axis=0)
        x = x + alpha * p
        r = r - alpha * q
        p_old, q_old = p, q
        hist.append(float(np.max(np.linalg.norm(r, axis=0) / bn)))
    return x, hist


def gmres(A, precond, b: np.ndarray, restart: int = 30, rtol: float = 1e-10, maxit: int = 200,
          flexible: bool = False, inner: float = 0.0):
    """Restarted GMRES(m) around a preconditioner M (Sec. 3.1 uses the V-cycle
    as a left preconditioner).  Independent Krylov spaces per column of b.

    left (flexible=False): minimise ||M(b - A x)|| over x in
        x_0 + K_k(M A, M r_0); the monitored residual is ||M(b - A x_k)||, the
        norm Sec. 3.1 regresses rho on.
    flexible (right): z_j = M(v_j), w = A z_j, x = x_0 + Z y; the monitored
        residual is ||b - A x_k|| (M may change from step to step).

    Arnoldi with modified Gram-Schmidt; y minimises ||beta e_1 - Hbar y||
    (dense least squares).  The columns advance in lockstep: a column whose
    estimate reaches rtol ||u_0|| (or inner times the cycle's starting norm,
    inner > 0) or breaks down stops growing its basis, and the cycle ends when
    every column has stopped or after `restart` steps.  Then x is updated,
    the monitored residual is recomputed explicitly (it replaces the estimate
    of the last step), and columns still above rtol start a new cycle.
    Returns x and the history of max_j u_j(x_k) / u_j(x_0)."""
    n, R = b.shape
    x = np.zeros_like(b)

    def monitored(xx):
        r = b - A @ xx
        return r if flexible else precond(r)

    u = monitored(x)
    res = np.linalg.norm(u, axis=0)
    beta0 = np.where(res > 0, res, 1.0)
    hist = [float(np.max(res / beta0))]
    done = res <= rtol * beta0
    it = 0
    while not np.all(done) and it < maxit:
        start = res.copy()
        V = [np.where(start > 0, u / np.where(start > 0, start, 1.0), 0.0)]
        Z = []
        H = np.zeros((restart + 1, restart, R))
        steps = np.zeros(R, dtype=int)
        est = res.copy()
        growing = ~done
        for j in range(restart):
            if it == maxit:
                break
            if flexible:
                z = precond(V[j])
                Z.append(z)
                w = A @ z
            else:
                w = precond(A @ V[j])
            for i in range(j + 1):
                h = np.sum(w * V[i], axis=0)
                H[i, j] = h
                w = w - h * V[i]
            hn = np.linalg.norm(w, axis=0)
            H[j + 1, j] = hn
            V.append(np.where(hn > 0, w / np.where(hn > 0, hn, 1.0), 0.0))
            it += 1
            for c in np.flatnonzero(growing):
                Hb = H[: j + 2, : j + 1, c]
                g = np.zeros(j + 2)
                g[0] = start[c]
                y = np.linalg.lstsq(Hb, g, rcond=None)[0]
                steps[c] = j + 1
                est[c] = np.linalg.norm(g - Hb @ y)
                if est[c] <= max(rtol * beta0[c], inner * start[c]) or hn[c] == 0:
                    growing[c] = False
            hist.append(float(np.max(est / beta0)))
            if not np.any(growing):
                break
        basis = Z if flexible else V
        for c in np.flatnonzero(~done):
            k = steps[c]
            if k == 0:
                continue
            g = np.zeros(k + 1)
            g[0] = start[c]
            y = np.linalg.lstsq(H[: k + 1, :k, c], g, rcond=None)[0]
            for i in range(k):
                x[:, c] += y[i] * basis[i][:, c]
        u = monitored(x)
        res = np.linalg.norm(u, axis=0)
        done = res <= rtol * beta0
        hist[-1] = float(np.max(res / beta0))
    return x, hist


def rho_regression(hist: Sequence[float]) -> float:
    """Convergence rate from a least-squares line through (i, log r_i),
    i = 1..K (Sec. 3.1); r_0 is left out."""
    h = np.asarray(hist[1:], dtype=np.float64)
    if len(h) < 2:
        return float(h[0] / hist[0]) if len(h) else float("nan")
    i = np.arange(1, len(h) + 1, dtype=np.float64)
    slope = np.polyfit(i, np.log(h), 1)[0]
    return float(np.exp(slope))


def eta(rho: float) -> float:
    """Iterations per decade of residual reduction: log 0.1 / log rho (Sec. 3.1)."""
    return float(np.log(0.1) / np.log(rho))


def cost_model(nu: int, eta_: float, d: int) -> float:
    """C_d(nu, eta) = eta (1 + (2 nu + 1) / (1 - 2^-d)) (Sec. 3.1)."""
    return eta_ * (1.0 + (2 * nu + 1) / (1.0 - 2.0 ** (-d)))


# ---------------------------------------------------------------------------
# Local (patch) evaluation for large problems
# ---------------------------------------------------------------------------

def block_ball(Apat: sp.csr_matrix, centre: int, radius: int) -> np.ndarray:
    seen = {centre}
    front = [centre]
    for _ in range(radius):
        nxt = []
        for i in front:
            for j in Apat.indices[Apat.indptr[i]:Apat.indptr[i + 1]]:
                if j not in seen:
                    seen.add(j)
                    nxt.append(j)
        front = nxt
    return np.array(sorted(seen), dtype=np.int64)


def fit_local(A: sp.spmatrix, n: int, depth: int, centres: Sequence[int], mode: str = "additive",
              colours: Optional[np.ndarray] = None, radius: Optional[int] = None,
              with_cond: bool = False, ridge: float = 0.0):
    """Lambda_{l,i} for selected blocks i, each fitted on the sub-matrix of A
    over the blocks within block-graph distance `radius` of i.

    Lambda_{l,i} depends on A only through E_{l-1} on the neighbours of i,
    which in turn reaches at most l block layers out, so radius = nu
    (additive) or nu * chi (multiplicative) reproduces the full fit.
    with_cond: also return, per centre, the largest condition number of the
    normal equations met in its patch at each cascade level."""
    A = sp.csr_matrix(A)
    Apat = block_pattern(A, n)
    if radius is None:
        radius = depth if mode == "additive" else depth * (int(np.max(colours)) + 1)
    out, conds = {}, {}
    for c in centres:
        S = block_ball(Apat, int(c), radius)
        sel = block_rows(S, n)
        sub = A[sel][:, sel]
        pos = int(np.searchsorted(S, c))
        res = fit(sub, n, depth, mode, None if colours is None else np.asarray(colours)[S], ridge=ridge)
        out[int(c)] = [L[pos] for L in res["lam"]]
        conds[int(c)] = [float(np.max(g)) for g in res["gram_cond"]]
    return (out, conds) if with_cond else out


# ---------------------------------------------------------------------------
# Stencil repetition (Sec. 4, caching repeated local setups on structured meshes)
# ---------------------------------------------------------------------------

def lattice_row_signatures(A: sp.spmatrix, n: int, coords: np.ndarray) -> List[bytes]:
    """Byte signature of every block row of A seen from its own lattice point:
    for each block column c of row k (in order of the offset coords[c] -
    coords[k]), the offset, the n x n block A_kc and the n diagonal entries of
    A_cc.  Two rows with equal signatures have equal prescaled rows
    W A W (W = diag(A)^{-1/2}) under the translation of their lattice points."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    coords = np.asarray(coords, dtype=np.int64)
    B = A.shape[0] // n
    Apat = block_pattern(A, n)
    diag = A.diagonal()
    sig = []
    for k in range(B):
        cols = Apat.indices[Apat.indptr[k]:Apat.indptr[k + 1]]
        parts = []
        for c in cols:
            blk = A[k * n:(k + 1) * n, c * n:(c + 1) * n].toarray()
            off = tuple(int(v) for v in coords[c] - coords[k])
            parts.append((off, blk.tobytes() + diag[c * n:(c + 1) * n].tobytes()))
        parts.sort(key=lambda p: p[0])
        sig.append(repr([p[0] for p in parts]).encode() + b"|" + b"".join(p[1] for p in parts))
    return sig


def lattice_classes(A: sp.spmatrix, n: int, coords: np.ndarray, radius: int) -> np.ndarray:
    """rep[i] = the smallest block j such that translating the lattice by
    t = coords[j] - coords[i] maps every block k within block-graph distance
    `radius` of i onto a block k' (coords[k'] = coords[k] + t) whose row
    signature equals that of k.  By the dependence stated in fit_local, the
    cascade step l (Lambda_l and the residual row E_l) of every block equals
    that of its representative at radius l - 1, up to the rounding order of
    the sums (the columns are relabelled by the translation)."""
    A = sp.csr_matrix(A)
    coords = np.asarray(coords, dtype=np.int64)
    B = A.shape[0] // n
    Apat = block_pattern(A, n)
    sig = lattice_row_signatures(A, n, coords)
    at = {tuple(int(v) for v in coords[k]): k for k in range(B)}
    if len(at) != B:
        raise ValueError("lattice points must be distinct")
    balls = [block_ball(Apat, i, radius) for i in range(B)]
    rep = np.arange(B, dtype=np.int64)
    for i in range(B):
        for j in range(i):
            if rep[j] != j:
                continue
            t = coords[j] - coords[i]
            ok = True
            for k in balls[i]:
                kk = at.get(tuple(int(v) for v in coords[k] + t))
                if kk is None or sig[kk] != sig[k]:
                    ok = False
                    break
            if ok:
                rep[i] = j
                break
    return rep
