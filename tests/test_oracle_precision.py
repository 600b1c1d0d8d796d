"""Which reduced-precision operand breaks the depth-3 multicoloured DG cascade,
and what makes BF16 block applies usable (CPU, FP64 emulation of rounding).

The SIPG Q3 hierarchy (16^2 elements, 16x16 element blocks, four-colour
multiplicative FF cascade of depth 3, V(1,1)) is solved by FP64 iterative
refinement around a V-cycle whose operands are rounded to FP32 or BF16
(round to nearest even) before use:
  * the paper's fit (plain least squares): FP32 everywhere leaves the
    convergence factor unchanged, but BF16 A, BF16 Lambda or BF16 sweeps
    diverge.  The fitted Lambda_2 and Lambda_3 are 10-100x larger than
    Lambda_1 (normal equations with condition numbers ~1e7): they cancel
    nearly dependent directions, and BF16 rounding (2^-9) of either factor
    destroys that cancellation;
  * the Tikhonov-regularised fit (ridge 1e-3 of the mean diagonal of G_i)
    keeps every block small; its FP64 V-cycle converges slightly faster than
    the plain fit's, and BF16 sweeps (A and Lambda in BF16, FP32 vectors)
    converge within 5% of it, provided the residual that is restricted to the
    coarse level is formed in FP32 (a BF16 residual corrupts the smooth error
    components the coarse grid must see).
This is the split the BF16 matrix-core path implements.
"""
import numpy as np
import pytest

import oracle as O
from synth import dg


def bf16(a):
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def fp32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def same(a):
    return np.asarray(a, dtype=np.float64)


class Emulated:
    """FF V(1,1) of Alg. 1 with the multiplicative cascade of Sec. 2.2; the
    sweeps use A rounded by `sweep_a`, Lambda rounded by `lam`, every vector
    result rounded by `vec`, and the residual that is restricted uses A rounded
    by `res_a`.  The bottom level is solved exactly."""

    def __init__(self, levels, sms, sweep_a, lam, vec, res_a):
        self.levels, self.vec = levels, vec
        self.per = []
        for lv, sm in zip(levels[:-1], sms):
            As, Ar = lv.A.copy().tocsr(), lv.A.copy().tocsr()
            As.data, Ar.data = sweep_a(As.data), res_a(Ar.data)
            chi = int(np.max(sm["colours"])) + 1
            steps = [O.blockdiag(lam(L) * (sm["colours"] == k)[:, None, None])
                     for L in sm["lam"] for k in range(chi)]
            self.per.append((As, Ar, steps))
        self.bottom = np.linalg.inv(levels[-1].A.toarray())

    def __call__(self, b, l=0):
        if l == len(self.levels) - 1:
            return self.vec(self.bottom @ b)
        lv, (As, Ar, steps), v = self.levels[l], self.per[l], self.vec
        x = np.zeros_like(b)
        for S in steps:
            x = v(x - S @ v(As @ x - b))
        xc = self(v(lv.r_scale * (lv.P.T @ v(Ar @ x - b))), l + 1)
        x = v(x - lv.P @ xc)
        for S in steps:
            x = v(x - S @ v(As @ x - b))
        return x


def refinement_rho(levels, V, b, maxit=40):
    """FP64 defect correction x += V(b - A x); rho by the regression of Sec. 3.1."""
    A = levels[0].A
    x = np.zeros_like(b)
    hist = []
    for _ in range(maxit + 1):
        r = b - A @ x
        hist.append(float(np.linalg.norm(r) / np.linalg.norm(b)))
        if hist[-1] <= 1e-10 or not np.isfinite(hist[-1]) or hist[-1] > 1e6:
            break
        x = x + V(r)
    return O.rho_regression(hist) if len(hist) > 2 else hist[-1] / hist[0], hist


@pytest.fixture(scope="module")
def dg16():
    p = dg.sipg_q3(16)
    return p, p.rhs[:, :1].copy()


def test_plain_fit_diverges_in_bf16_but_not_in_fp32(dg16):
    p, b = dg16
    sms = O.setup_hierarchy(p.levels, 3, "multiplicative")
    lam_max = [float(np.abs(L).max()) for L in sms[0]["lam"]]
    assert lam_max[1] > 10 * lam_max[0] and lam_max[2] > 10 * lam_max[0], lam_max
    rho64, h64 = refinement_rho(p.levels, Emulated(p.levels, sms, same, same, same, same), b)
    assert h64[-1] <= 1e-10 and rho64 < 0.2
    rho32, _ = refinement_rho(p.levels, Emulated(p.levels, sms, fp32, fp32, fp32, fp32), b)
    assert abs(rho32 - rho64) <= 0.01 * rho64, (rho32, rho64)
    for name, ops in (("A", (bf16, same, same, bf16)), ("Lambda", (same, bf16, same, same)),
                      ("sweeps", (bf16, bf16, fp32, fp32))):
        rho, hist = refinement_rho(p.levels, Emulated(p.levels, sms, *ops), b)
        assert rho > 1.0 or not np.isfinite(hist[-1]) or hist[-1] > 1.0, (name, rho)


def test_ridge_fit_makes_bf16_sweeps_converge(dg16):
    p, b = dg16
    plain = O.setup_hierarchy(p.levels, 3, "multiplicative")
    sms = O.setup_hierarchy(p.levels, 3, "multiplicative", ridge=1e-3)
    # the regularised blocks stay at the scale of the first level's
    lam_max = [float(np.abs(L).max()) for L in sms[0]["lam"]]
    assert max(lam_max) < 5 * lam_max[0], lam_max
    rho_plain, _ = refinement_rho(p.levels, Emulated(p.levels, plain, same, same, same, same), b)
    rho64, h64 = refinement_rho(p.levels, Emulated(p.levels, sms, same, same, same, same), b)
    assert h64[-1] <= 1e-10 and rho64 <= rho_plain
    rho16, h16 = refinement_rho(p.levels, Emulated(p.levels, sms, bf16, bf16, fp32, fp32), b)
    assert h16[-1] <= 1e-10 and rho16 <= 1.05 * rho64, (rho16, rho64)
    # a BF16 residual for the restriction costs much of the coarse-grid correction
    rho_bad, _ = refinement_rho(p.levels, Emulated(p.levels, sms, bf16, bf16, fp32, bf16), b)
    assert rho_bad > 1.5 * rho64, (rho_bad, rho64)
