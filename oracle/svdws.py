"""SVD with warm start (Sec. 5, Alg. 2 and Appendix A), in FP64.

TEST INFRASTRUCTURE.  Same rule as ``tilt_oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
import or run it.

Given the decomposition (U, Sigma, V) of the previous matrix and the next
matrix M, one step searches the curve

    U(t) = (I + t/2 P_U)^{-1} (I - t/2 P_U) U,
    Sigma(t) = Sigma - t P_Sigma,
    V(t) = (I + t/2 P_V)^{-1} (I - t/2 P_V) V

(Cayley transforms keep U and V orthonormal) along the projected gradients
of F = 1/2 ||M - U Sigma V^T||_F^2 (Eqs. projected_gradient1-3), and takes
t* = -f'(0)/f''(0) from the second-order model of f(t) = F(U(t), Sigma(t),
V(t)) (Eq. ft), with f'(0) and f''(0) from Appendix A.  Alg. 2 uses the
step only when ||M_k - M_{k-1}|| < eps_svd and otherwise computes a full
SVD.

Readings (the paper leaves these open): the norm in the switch test is the
Frobenius norm; eps_svd is relative, eps_svd * ||M_k||_F; a step with
f''(0) <= 0 (the quadratic model has no minimum) falls back to the full
SVD; Sigma may carry signs (the paper allows negated columns), so the
shrinkage soft-thresholds the signed diagonal.  The m x m inverse is taken
directly here (the oracle favours the plain definition); P_U has rank at
most 2 n, which a fast implementation would exploit with the
Sherman-Morrison-Woodbury identity.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


def projected_gradients(U, S, V, M):
    """P_U, P_Sigma (as a vector) and P_V at (U, S, V) for matrix M."""
    X = (U * S) @ V.T
    PU = X @ M.T - M @ X.T                      # Eq. projected_gradient1
    PV = X.T @ M - M.T @ X                      # Eq. projected_gradient2
    PS = S - np.einsum("ij,ij->j", U, M @ V)    # Eq. projected_gradient3: diag(Sigma - U^T M V)
    return PU, PS, PV


def cayley(P, t, Q):
    """(I + t/2 P)^{-1} (I - t/2 P) Q."""
    I = np.eye(P.shape[0])
    return np.linalg.solve(I + 0.5 * t * P, (I - 0.5 * t * P) @ Q)


def curve(U, S, V, PU, PS, PV, t):
    return cayley(PU, t, U), S - t * PS, cayley(PV, t, V)


def f_of_t(U, S, V, M, PU, PS, PV, t):
    """f(t) = 1/2 ||M - U(t) Sigma(t) V(t)^T||_F^2 (Eq. solve_t)."""
    Ut, St, Vt = curve(U, S, V, PU, PS, PV, t)
    return 0.5 * float(np.sum((M - (Ut * St) @ Vt.T) ** 2))


def derivatives(U, S, V, M, PU, PS, PV):
    """f'(0) and f''(0) from Appendix A:
       h(0) = M - X, h'(0) = P_U X + U P_Sigma V^T - X P_V,
       h''(0) = -P_U Z + Z P_V with Z = h'(0) + U P_Sigma V^T,
       f'(0) = tr(h(0)^T h'(0)), f''(0) = tr(h'(0)^T h'(0) + h(0)^T h''(0))."""
    X = (U * S) @ V.T
    UPV = (U * PS) @ V.T
    h0 = M - X
    h1 = PU @ X + UPV - X @ PV
    Z = h1 + UPV
    h2 = -PU @ Z + Z @ PV
    f1 = float(np.sum(h0 * h1))
    f2 = float(np.sum(h1 * h1) + np.sum(h0 * h2))
    return f1, f2


@dataclasses.dataclass
class WarmSVD:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    M: np.ndarray


@dataclasses.dataclass
class StepInfo:
    warm: bool        # the Cayley step was used (else a full SVD)
    t: float
    f0: float
    ft: float


def svd_full(M) -> WarmSVD:
    U, S, Vt = np.linalg.svd(M, full_matrices=False)
    return WarmSVD(U, S, Vt.T, M.copy())


def svdws(prev: Optional[WarmSVD], M, eps_svd: float):
    """Alg. 2: warm-started decomposition of M from the previous one, or a
    full SVD when there is none, when ||M - M_prev||_F >= eps_svd ||M||_F or
    when f''(0) <= 0."""
    if prev is None or np.linalg.norm(M - prev.M) >= eps_svd * np.linalg.norm(M):
        return svd_full(M), StepInfo(False, 0.0, 0.0, 0.0)
    PU, PS, PV = projected_gradients(prev.U, prev.S, prev.V, M)
    f1, f2 = derivatives(prev.U, prev.S, prev.V, M, PU, PS, PV)
    if not f2 > 0.0:
        return svd_full(M), StepInfo(False, 0.0, 0.0, 0.0)
    t = -f1 / f2
    U, S, V = curve(prev.U, prev.S, prev.V, PU, PS, PV, t)
    f0 = 0.5 * float(np.sum((M - (prev.U * prev.S) @ prev.V.T) ** 2))
    ft = 0.5 * float(np.sum((M - (U * S) @ V.T) ** 2))
    return WarmSVD(U, S, V, M.copy()), StepInfo(True, t, f0, ft)


def shrink(dec: WarmSVD, eps: float):
    """U T_eps(Sigma) V^T with the signed soft threshold."""
    T = np.sign(dec.S) * np.maximum(np.abs(dec.S) - eps, 0.0)
    return (dec.U * T) @ dec.V.T


class SvdwsSvt:
    """Alg. 2 as the SVT of the LADMAP inner loop (``ladmap_inner``'s
    ``svt_op``): the decomposition of the previous call is kept, and each
    call either takes the Cayley step from it or computes a full SVD, then
    shrinks the result with the signed soft threshold.  The switch is
    Alg. 2's, ||M - M_prev||_F < eps_svd ||M||_F, or, with every > 0, a
    fixed schedule: a full SVD at iterations 0, every, 2 every, ... and the
    step at the others.  A step with f''(0) <= 0 falls back to the full SVD.
    ``steps`` counts the calls done by a step."""

    def __init__(self, eps_svd: float = 1e-3, every: int = 0):
        self.eps_svd = eps_svd
        self.every = every
        self.prev: Optional[WarmSVD] = None
        self.steps = 0

    def __call__(self, M, eps, k):
        use = self.prev is not None and (
            (k % self.every != 0) if self.every > 0
            else np.linalg.norm(M - self.prev.M) < self.eps_svd * np.linalg.norm(M))
        dec = None
        if use:
            U, S, V = self.prev.U, self.prev.S, self.prev.V
            PU, PS, PV = projected_gradients(U, S, V, M)
            f1, f2 = derivatives(U, S, V, M, PU, PS, PV)
            if f2 > 0.0:
                Ut, St, Vt = curve(U, S, V, PU, PS, PV, -f1 / f2)
                dec = WarmSVD(Ut, St, Vt, M.copy())
                self.steps += 1
        if dec is None:
            dec = svd_full(M)
        self.prev = dec
        return shrink(dec, eps), np.sort(np.abs(dec.S))[::-1]

