"""The reference smoother of Sec. 2.1 through the C ABI (cs_options.source =
CS_SRC_JACOBI): every cascade level Lambda_l = omega * A_ii^{-1}, the damped
block Jacobi (additive) and block Gauss-Seidel / SOR (multiplicative) steps the
cascade is measured against, against the oracle's `jacobi_smoother`, and the
convergence figures of cs_info (rho, rho_geo, eta; Sec. 3.1) against their
definitions on the returned residual history.

Bounds: a block inverse by Gauss-Jordan with partial pivoting differs from
LAPACK's in rounding only, by at most a modest multiple of u cond(A_ii)
(per block: the least-squares constant of tests/parity.py, 16384 u cond);
V-cycles 1e-12 relative as for the fitted cascade.
"""
import numpy as np
import pytest

import oracle as O
from parity import VCYCLE_TOL, block_errors, check_vec, record, scalar_bound
from paper_2606_12577_amd.cascade import CascadeError
from synth import fd
from synth.problem import Problem
from synth.rng import stream

pytestmark = pytest.mark.gpu

OMEGA = 0.8


def jacobi_oracle(prob, depth, omega, colours=None):
    out = []
    for lv in prob.levels[:-1]:
        sm = O.jacobi_smoother(lv.A, lv.block_size, depth, omega)
        if colours is not None:
            sm["colours"] = colours(lv)
        out.append(sm)
    return out


def check_blocks(s, prob, sm, depth, label):
    for l, lv in enumerate(prob.levels[:-1]):
        nb = lv.block_size
        A = lv.A.tocsr()
        cond = np.array([np.linalg.cond(A[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb].toarray())
                         for i in range(lv.n // nb)])
        for ell in range(1, depth + 1):
            g = s.get_smoother(l, ell).reshape(-1, nb, nb)
            e = block_errors(g, sm[l]["lam"][ell - 1])
            ratio = max(record(f"{label} level {l} Lambda_{ell} block {i}", e[i], scalar_bound([cond[i]]))
                        for i in range(len(e)))
            assert ratio <= 1.0, (l, ell, float(e.max()))


@pytest.mark.parametrize("case", ["interface3d_16", "ln2d_2x2", "ln2d_4x4"])
def test_block_jacobi_additive(gpu_lib, case):
    if case == "interface3d_16":
        p = fd.interface3d(16, nrhs=2)
    else:
        bs = int(case[-1])
        z = stream(7, 1).standard_normal((32, 32))
        p = Problem(case, fd.fv_hierarchy(np.exp(2.0 * z), bs=bs, n_stop=4),
                    stream(7, 0).uniform(-1, 1, size=(32 * 32, 4)))
    depth = 2
    sm = jacobi_oracle(p, depth, OMEGA)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=depth, source="jacobi", omega=OMEGA)
    check_blocks(s, p, sm, depth, f"block Jacobi {p.name}")
    for order in ("RF", "FF"):
        s.setup(depth=depth, order=order, source="jacobi", omega=OMEGA)
        o = O.vcycle(p.levels, sm, p.rhs, order)
        check_vec(s.vcycle(p.rhs).cpu().numpy(), o, VCYCLE_TOL, f"block Jacobi {p.name} {order} V-cycle")
    s.close()


def test_block_gauss_seidel_red_black(gpu_lib):
    """Multiplicative mode: omega A_ii^{-1} applied colour by colour (SOR over
    the red-black colouring of a 2D log-normal problem)."""
    p = fd.lognormal2d(32, nrhs=2, n_stop=4)
    for lv in p.levels:
        lv.colour = fd.parity_colour(int(round(np.sqrt(lv.n))), 2, 1, lv.cells)
    depth = 2
    sm = jacobi_oracle(p, depth, 1.2, colours=lambda lv: lv.colour)
    s = gpu_lib.Solver(p.levels)
    for order in ("FF", "RF"):
        s.setup(depth=depth, mode="multiplicative", order=order, source="jacobi", omega=1.2)
        check_blocks(s, p, sm, depth, "block Gauss-Seidel red-black")
        o = O.vcycle(p.levels, sm, p.rhs, order)
        check_vec(s.vcycle(p.rhs).cpu().numpy(), o, VCYCLE_TOL, f"block Gauss-Seidel red-black {order} V-cycle")
    s.close()


def test_solve_rates_and_cascade_beats_jacobi(gpu_lib):
    """cs_info's rho (regression), rho_geo and eta against their definitions on
    the returned history; the solve with the Jacobi source takes the oracle's
    iteration count; a depth-3 cascade converges faster than three damped
    Jacobi steps (Sec. 3.2)."""
    p = fd.poisson2d(64)
    s = gpu_lib.Solver(p.levels)
    s.setup(depth=3, source="jacobi", omega=OMEGA, n_pre=1, n_post=1)
    _, info = s.solve(p.rhs, rtol=1e-10, maxit=200)
    h = info["history"]
    K = info["iterations"]
    assert h[-1] <= 1e-10 and len(h) == K + 1
    rho = O.rho_regression(h)
    assert abs(info["rho"] - rho) <= 1e-12 * rho
    assert abs(info["rho_geo"] - (h[-1] / h[0]) ** (1.0 / K)) <= 1e-12
    assert abs(info["eta"] - O.eta(rho)) <= 1e-10 * O.eta(rho)
    sm = jacobi_oracle(p, 3, OMEGA)
    _, ho = O.solve(p.levels, sm, p.rhs)
    assert abs(K - (len(ho) - 1)) <= 1, (K, len(ho) - 1)
    s.setup(depth=3)
    _, fit = s.solve(p.rhs, rtol=1e-10, maxit=200)
    print(f"[jacobi] 64^2 Poisson V(1,1) depth 3: damped Jacobi rho {info['rho']:.4f} eta {info['eta']:.2f}, "
          f"cascade rho {fit['rho']:.4f} eta {fit['eta']:.2f}", flush=True)
    assert fit["rho"] < info["rho"] and fit["eta"] < info["eta"]
    s.close()


def test_bad_omega_is_rejected(gpu_lib):
    p = fd.poisson2d(16)
    s = gpu_lib.Solver(p.levels)
    for w in (0.0, -1.0, 2.5):
        with pytest.raises(CascadeError):
            s.setup(depth=2, source="jacobi", omega=w)
    with pytest.raises(CascadeError):
        s.setup(depth=2, source="jacobi", omega=1.0, ridge=1e-3)
    s.close()
